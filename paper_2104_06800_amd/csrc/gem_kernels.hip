// GEM kernels for gfx950: initial depth, per-level fused E-step / M-step on the alternately
// directed 1D chains, pose normal equations with an on-device FP64 solve, and the final
// confidence / statistics pass (VOLDOR+SLAM sec. III-A, Eqs. 1-6).
#include "device.h"
#include "kernels.h"

namespace vd {

// ----------------------------------------------------------------------------------
// pose conversion (FP64 6-vectors -> FP32 R|t for frames and priors)
// ----------------------------------------------------------------------------------
__device__ __forceinline__ void pose_prep_body(const double* __restrict__ pose, int N, const double* __restrict__ prior_pose,
                                               int P, PoseF* __restrict__ out, PoseD* __restrict__ outd) {
    const int i = threadIdx.x;
    if (i < N) {
        pose_tables_from_vec(pose + 6 * i, out + i, outd + i);
    } else if (i < N + P) {
        pose_to_f(prior_pose + 6 * (i - N), out + i);
    }
}

__global__ void k_pose_prep(const double* __restrict__ pose, int N, const double* __restrict__ prior_pose, int P,
                            PoseF* __restrict__ out, PoseD* __restrict__ outd) {
    pose_prep_body(pose, N, prior_pose, P, out, outd);
}

// ----------------------------------------------------------------------------------
// initial inverse depth: random, or read off the first depth prior
// ----------------------------------------------------------------------------------
// The inverse depth of pixel j whose transfer into prior 0's camera meets the prior at the
// pixel l it lands on (sec. III-A, priors bootstrap the estimate): R x~ / rho + t has depth
// a / rho + t_z with a = r_3 . x~, so 1 / phi_z = rho^(l) gives rho = rho^(l) a / (1 - rho^(l) t_z).
// l depends on rho: two fixed-point rounds from the prior's value at j (the first is exact
// for an identity pose).  FP64 throughout so that the nearest-pixel choices are the exact
// arithmetic's.  False where a round leaves the image, lands behind the camera, or meets a
// hole or a non-positive solution.
__device__ inline bool prior_boot(const Win& w, InitSrc s, int j, double& out) {
    double R[9];
    exp_so3(s.pose, R);
    const int x = j % w.W, y = j / w.W;
    const double fx = w.fx, fy = w.fy, cx = w.cx, cy = w.cy;
    const double rx = ((double)x - cx) / fx, ry = ((double)y - cy) / fy;
    const double a = R[6] * rx + R[7] * ry + R[8];
    double rho = s.prior[j];
    if (!(rho > 0.0) || !isfinite(rho)) return false;
    for (int r = 0; r < 2; ++r) {
        const double ir = 1.0 / rho;
        const double qx = (R[0] * rx + R[1] * ry + R[2]) * ir + s.pose[3];
        const double qy = (R[3] * rx + R[4] * ry + R[5]) * ir + s.pose[4];
        const double qz = a * ir + s.pose[5];
        if (!(qz > 0.0)) return false;
        const double lx = floor(fx * qx / qz + cx + 0.5), ly = floor(fy * qy / qz + cy + 0.5);
        if (!(lx >= 0.0 && lx <= (double)(w.W - 1) && ly >= 0.0 && ly <= (double)(w.H - 1))) return false;
        const double rh = s.prior[(int)ly * w.W + (int)lx];
        const double den = 1.0 - rh * s.pose[5];
        if (!(rh > 0.0) || !isfinite(rh) || !(den > 0.0) || !(a > 0.0)) return false;
        rho = rh * a / den;
    }
    out = rho;
    return true;
}

__device__ __forceinline__ void init_body(const Win& w, float* __restrict__ idepth, InitSrc s, int blk) {
    const int j = blk * VD_BLOCK + threadIdx.x;
    if (j >= w.H * w.W) return;
    double b;
    if (s.prior && prior_boot(w, s, j, b)) {
        idepth[j] = (float)fmin(fmax(b, (double)w.rmin), (double)w.rmax);
        return;
    }
    const uint4 r = philox10(make_uint4((uint32_t)j, 0u, philox_word2(0, 1, PURPOSE_INIT), w.window_id),
                             w.key0, w.key1);
    idepth[j] = fmaf(unit24(r.x), w.rmax - w.rmin, w.rmin);
}

__global__ void __launch_bounds__(VD_BLOCK) k_init_idepth(Win w, float* __restrict__ idepth, InitSrc s) {
    init_body(w, idepth, s, blockIdx.x);
}

// the start where a learned start raised its fallback flag (always without a flag); the flag
// is copied out
__global__ void __launch_bounds__(VD_BLOCK)
k_init_idepth_if(Win w, float* __restrict__ idepth, InitSrc s, const int* __restrict__ flag, int32_t* __restrict__ out) {
    const int f = flag ? *flag : 1;
    if (out && blockIdx.x == 0 && threadIdx.x == 0) *out = f;
    if (f) init_body(w, idepth, s, blockIdx.x);
}

// ----------------------------------------------------------------------------------
// row-pair flow layout for the bilinear samples of frames t >= 2:
// F2[t][y][x] = (X_t(x, y), X_t(x, y + 1)), y <= H - 2
// ----------------------------------------------------------------------------------
__device__ __forceinline__ void flow_pairs_body(const float2* __restrict__ flow, float4* __restrict__ f2, int N, int H,
                                                int W, int blk) {
    const size_t per = (size_t)(H - 1) * W;
    const size_t i = (size_t)blk * VD_BLOCK + threadIdx.x;
    if (i >= per * (N - 1)) return;
    const size_t t = 1 + i / per, r = i - (t - 1) * per;
    const size_t o = t * (size_t)H * W + r;
    const float2 a = flow[o], b = flow[o + W];
    f2[o] = make_float4(a.x, a.y, b.x, b.y);
}

__global__ void __launch_bounds__(VD_BLOCK) k_flow_pairs(const float2* __restrict__ flow, float4* __restrict__ f2, int N,
                                                         int H, int W) {
    flow_pairs_body(flow, f2, N, H, W, blockIdx.x);
}

// ----------------------------------------------------------------------------------
// fused level kernel
//
// A block owns C chain segments of length <= seg of one level (coarse lattice rows /
// columns, or rows / columns of the local tiles).  Block-local arrays live in LDS with a
// padded row stride seg + 1:
//   E-step : per-frame emission ratios L1/L0, forward messages, then posteriors q
//   M-step : phase A   each pixel's best over slots {0, 2, 3..K-1} (energy, value, slot)
//            phase A2  each pixel's energy at its predecessor's phase-A winner
//            phase B   one lane per chain walks it in direction d: slot 1 (the
//                      predecessor's updated value) replaces the phase-A winner iff its
//                      energy is lower, or equal with the winner's slot > 1.  When the
//                      predecessor took its own phase-A winner the energy from A2 is
//                      used; otherwise it is evaluated on the spot.
// ----------------------------------------------------------------------------------
struct BlockPix {
    int c, i;      // chain within block, node along the chain (storage order)
    int li;        // level-grid index
    int u, v;      // full-resolution pixel
    bool valid;
};

__device__ __forceinline__ BlockPix block_pix(const LevelGeom& g, int b, int k) {
    BlockPix p;
    const int sidx = b % g.nseg, lb = b / g.nseg;
    int c, i;
    if (g.horizontal) { c = k / g.seg; i = k - c * g.seg; }
    else { i = k / g.C; c = k - i * g.C; }
    p.c = c; p.i = i;
    const int line = lb * g.C + c, pos = sidx * g.seg + i;
    int lx, ly;
    if (g.horizontal) { ly = line; lx = pos; } else { lx = line; ly = pos; }
    p.valid = (c < g.C) && (i < g.seg) && (lx < g.w) && (ly < g.h);
    p.li = ly * g.w + lx;
    p.u = g.s * lx + g.off;
    p.v = g.s * ly + g.off;
    return p;
}

// number of valid nodes of chain c of this block
__device__ __forceinline__ int chain_len(const LevelGeom& g, int b, int c) {
    const int sidx = b % g.nseg, lb = b / g.nseg;
    const int line = lb * g.C + c;
    const int nlines = g.horizontal ? g.h : g.w;
    const int axis = g.horizontal ? g.w : g.h;
    if (line >= nlines) return 0;
    return min(g.seg, axis - sidx * g.seg);
}

// ----------------------------------------------------------------------------------
// Forward-backward on long chains as a segmented scan (sec. III-A, the two-state chain
// of the rigidness maps).  Both recursions are linear in the unnormalised state
// (alpha, 1 - alpha): the forward step of node i is diag(r_i, 1) T and the backward
// step into node i - 1 is T diag(r_i, 1), with T = [[g, 1 - g], [1 - g, g]] the
// transition matrix.  A group of G lanes splits a chain into G segments; each lane
// composes its segment's 2x2 matrices, the group scans them (prefix for the forward
// pass, suffix for the backward), and each lane then runs the ordinary normalised
// recursion over its own nodes from the state that enters the segment.  The result
// equals the serial recursion up to rounding; the serial path per chain drops from 2L
// steps to about 4L/G + 2 log2 G.
// ----------------------------------------------------------------------------------
struct Mat2 {
    float a, b, c, d;  // [[a b] [c d]]
};

// x y scaled to unit entry sum (all entries are non-negative, the sum is positive)
__device__ __forceinline__ Mat2 mat2_mul(const Mat2& x, const Mat2& y) {
    Mat2 z;
    z.a = fmaf(x.a, y.a, x.b * y.c);
    z.b = fmaf(x.a, y.b, x.b * y.d);
    z.c = fmaf(x.c, y.a, x.d * y.c);
    z.d = fmaf(x.c, y.b, x.d * y.d);
    const float s = rcp((z.a + z.b) + (z.c + z.d));
    z.a *= s; z.b *= s; z.c *= s; z.d *= s;
    return z;
}

__device__ __forceinline__ Mat2 mat2_shfl_up(const Mat2& x, int d, int G) {
    return {__shfl_up(x.a, d, G), __shfl_up(x.b, d, G), __shfl_up(x.c, d, G), __shfl_up(x.d, d, G)};
}

__device__ __forceinline__ Mat2 mat2_shfl_down(const Mat2& x, int d, int G) {
    return {__shfl_down(x.a, d, G), __shfl_down(x.b, d, G), __shfl_down(x.c, d, G), __shfl_down(x.d, d, G)};
}

// chain (c, t) of the block: emission ratios r_s in, posteriors q_s out ([N][C][stride]);
// returns this lane's share of the chain log-likelihood.  Every lane of a group takes the
// same branches up to the shuffles (G is a power of two, groups never straddle a wave).
__device__ __forceinline__ double chain_fb_scan(const Win& w, const LevelGeom& g, int blk, const float* r_s,
                                                float* q_s, int nodes, int stride) {
    const int nch = g.C * w.N;
    int G = 64;
    while (G > 1 && G * nch > VD_BLOCK) G >>= 1;
    const int tid = threadIdx.x;
    if (tid >= G * nch) return 0.0;
    const int j = tid / G, lane = tid & (G - 1);
    const int c = j % g.C, t = j / g.C;
    const int L = chain_len(g, blk, c);
    if (L <= 0) return 0.0;
    const int sl = (L + G - 1) / G;
    const int s0 = min(L, lane * sl), s1 = min(L, s0 + sl);
    const float* r = r_s + t * nodes + c * stride;
    float* a = q_s + t * nodes + c * stride;
    const float gm = w.gamma, gc = 1.f - w.gamma, h = 2.f * w.gamma - 1.f;

    // forward: the segment's map, then the prefix over the group
    Mat2 F = {1.f, 0.f, 0.f, 1.f};
    for (int i = s0; i < s1; ++i) {
        const float ri = r[i];
        const Mat2 M = {ri * gm, ri * gc, gc, gm};
        F = mat2_mul(M, F);
    }
    for (int d = 1; d < G; d <<= 1) {
        const Mat2 X = mat2_shfl_up(F, d, G);
        if (lane >= d) F = mat2_mul(F, X);
    }
    const Mat2 Fin = mat2_shfl_up(F, 1, G);
    float a1 = 0.5f;  // the state before node 0 gives the prior 1/2
    if (lane > 0) {
        const float v1 = Fin.a + Fin.b, v0 = Fin.c + Fin.d;
        a1 = v1 * rcp(v1 + v0);
    }
    float logc = 0.f;
    for (int i = s0; i < s1; ++i) {
        const float p1 = (i == 0) ? 0.5f : fmaf(h, a1, gc);
        const float x1 = p1 * r[i];
        const float cc = (1.f - p1) + x1;
        a1 = x1 * rcp(cc);
        a[i] = a1;
        logc += log2f_fast(cc);
    }

    // backward: the segment's map (its nodes' ratios, last node first), then the suffix
    Mat2 Bk = {1.f, 0.f, 0.f, 1.f};
    for (int i = s1 - 1; i >= s0; --i) {
        const float ri = r[i];
        const Mat2 M = {gm * ri, gc, gc * ri, gm};
        Bk = mat2_mul(M, Bk);
    }
    for (int d = 1; d < G; d <<= 1) {
        const Mat2 X = mat2_shfl_down(Bk, d, G);
        if (lane + d < G) Bk = mat2_mul(Bk, X);
    }
    const Mat2 Bin = mat2_shfl_down(Bk, 1, G);
    float b1 = 0.5f;  // the last node's backward message
    if (lane < G - 1) {
        const float v1 = Bin.a + Bin.b, v0 = Bin.c + Bin.d;
        b1 = v1 * rcp(v1 + v0);
    }
    for (int i = s1 - 1; i >= s0; --i) {
        if (i < s1 - 1) {
            const float m0 = 1.f - b1, m1 = r[i + 1] * b1;
            const float y1 = fmaf(gm, m1, gc * m0);
            const float y0 = fmaf(gm, m0, gc * m1);
            b1 = y1 * rcp(y0 + y1);
        }
        const float ai = a[i];
        const float num = ai * b1;
        a[i] = num * rcp(fmaf(1.f - ai, 1.f - b1, num));
    }
    return (double)(logc * VD_LN2) + (double)(s1 - s0) * (double)w.ln_L0;
}

template <bool B2, bool PR, bool LC = false>
__device__ __forceinline__ void level_body(const Win& w, const LevelGeom& g, const LevelBufs& B, int do_e, int do_m,
                                           int blk, float* lds) {
    const int stride = g.seg + 1;
    const int nodes = g.C * stride;
    const int nf = g.nf;
    energy_t* bestE = (energy_t*)lds;       // [C][stride]
    energy_t* specE = bestE + nodes;        // [spec][C][stride]
    float* q_s = (float*)(specE + g.spec * nodes);   // [N][C][stride] emission ratios -> alpha -> q
    float* r_s = q_s + nf * nodes;          // [N][C][stride] emission ratios (E-step)
    float* bestV = r_s + nf * nodes;
    float* rcur = bestV + nodes;
    float* newV = rcur + nodes;
    int* bestS = (int*)(newV + nodes);
    float* cost_s = (float*)(bestS + nodes);  // [ncost][C][stride] E-step frame costs at rho
    __shared__ double ll_red[VD_BLOCK / 64];
    // a fused pass keeps the E-step's frame costs at the current value: the M-step's slot-0
    // energy is then their q-weighted sum, with no flow gathers
    const bool keep_cost = do_e && do_m == 1 && g.ncost > 0;
    // per-chain log-likelihood terms of an E-only pass, over the M-step arrays (unused there)
    double* llc = bestE;

    const int tid = threadIdx.x;
    const int npix = g.C * g.seg;
    const size_t lplane = (size_t)g.h * g.w;       // level plane
    const float* rho_full = B.idepth;
    double ll = 0.0;

    // -------------------------------- E-step ------------------------------------
    if (do_e) {
        for (int k = tid; k < npix; k += VD_BLOCK) {
            const BlockPix p = block_pix(g, blk, k);
            if (!p.valid) continue;
            Pix c;
            pix_geometry<PR>(w, B.P, B.flow, p.u, p.v, c);
            const float rho = rho_full[p.v * w.W + p.u];
            const int o = p.c * stride + p.i;
            if (w.chain_axis == 0) {
                emissions<B2>(w, B.P, B.flow2, c, rho, [&](int t, float ratio, bool ok, float r2) {
                    r_s[t * nodes + o] = ratio;
                    if (keep_cost) cost_s[t * nodes + o] = ok ? flow_cost2<B2>(w, r2) : 1.0f;
                });
            } else {
                // temporal chain over the frame window, in registers
                float rr[VD_NMAX], al[VD_NMAX];
                emissions<B2>(w, B.P, B.flow2, c, rho, [&](int t, float ratio, bool ok, float r2) {
                    rr[t] = ratio;
                    if (keep_cost) cost_s[t * nodes + o] = ok ? flow_cost2<B2>(w, r2) : 1.0f;
                });
                float logc = 0.f;
                float a1 = 0.f;
#pragma unroll
                for (int t = 0; t < VD_NMAX; ++t) {
                    if (t < w.N) {
                        const float p1 = (t == 0) ? 0.5f : fmaf(2.f * w.gamma - 1.f, a1, 1.f - w.gamma);
                        const float x1 = p1 * rr[t];
                        const float cc = (1.f - p1) + x1;
                        a1 = x1 * rcp(cc);
                        al[t] = a1;
                        logc += log2f_fast(cc);
                    }
                }
                float b1 = 0.5f;
#pragma unroll
                for (int t = VD_NMAX - 1; t >= 0; --t) {
                    if (t < w.N) {
                        if (t < w.N - 1) {
                            const float m0 = 1.f - b1, m1 = rr[t + 1] * b1;
                            const float y1 = fmaf(w.gamma, m1, (1.f - w.gamma) * m0);
                            const float y0 = fmaf(w.gamma, m0, (1.f - w.gamma) * m1);
                            b1 = y1 * rcp(y0 + y1);
                        }
                        const float num = al[t] * b1;
                        q_s[t * nodes + o] = num * rcp(fmaf(1.f - al[t], 1.f - b1, num));
                    }
                }
                const double llv = (double)(logc * VD_LN2) + (double)w.N * (double)w.ln_L0;
                if constexpr (LC) ll += llv;
                else if (B.ll_partial) llc[o] = llv;
            }
        }
        __syncthreads();
        if constexpr (LC) {
            if (w.chain_axis == 0) ll += chain_fb_scan(w, g, blk, r_s, q_s, nodes, stride);
        } else if (w.chain_axis == 0 && tid < g.C * w.N) {
            const int c = tid % g.C, t = tid / g.C;
            const int L = chain_len(g, blk, c);
            if (L > 0) {
                const float* r = r_s + t * nodes + c * stride;
                float* a = q_s + t * nodes + c * stride;
                const float gm = w.gamma, h = 2.f * w.gamma - 1.f;
                float logc = 0.f;
                float a1 = 0.f;
                for (int i = 0; i < L; ++i) {
                    const float p1 = (i == 0) ? 0.5f : fmaf(h, a1, 1.f - gm);
                    const float x1 = p1 * r[i];
                    const float cc = (1.f - p1) + x1;
                    a1 = x1 * rcp(cc);
                    a[i] = a1;
                    logc += log2f_fast(cc);
                }
                float b1 = 0.5f;
                for (int i = L - 1; i >= 0; --i) {
                    if (i < L - 1) {
                        const float m0 = 1.f - b1, m1 = r[i + 1] * b1;
                        const float y1 = fmaf(gm, m1, (1.f - gm) * m0);
                        const float y0 = fmaf(gm, m0, (1.f - gm) * m1);
                        b1 = y1 * rcp(y0 + y1);
                    }
                    const float ai = a[i];
                    const float num = ai * b1;
                    a[i] = num * rcp(fmaf(1.f - ai, 1.f - b1, num));
                }
                if (B.ll_partial) llc[c * VD_NMAX + t] = (double)(logc * VD_LN2) + (double)L * (double)w.ln_L0;
            }
        }
        __syncthreads();
        // posteriors out (coalesced along the level grid rows)
        for (int k = tid; k < npix; k += VD_BLOCK) {
            const BlockPix p = block_pix(g, blk, k);
            if (!p.valid) continue;
            const int o = p.c * stride + p.i;
            for (int t = 0; t < w.N; ++t) B.q_out[t * lplane + p.li] = q_s[t * nodes + o];
        }
        if (B.ll_partial) {
            if constexpr (LC) {
                // block sum of chain log-likelihoods, fixed order
                for (int off = 32; off > 0; off >>= 1) ll += __shfl_xor(ll, off);
                if ((tid & 63) == 0) ll_red[tid >> 6] = ll;
                __syncthreads();
                if (tid == 0) {
                    double s = 0.0;
                    for (int i = 0; i < VD_BLOCK / 64; ++i) s += ll_red[i];
                    B.ll_partial[blk] = s;
                }
            } else if (tid < g.C) {
                // one entry per chain, at the chain's place on the level grid: the frames (or the
                // nodes of a temporal-axis chain) summed in order, so the sums do not depend on
                // how many chains a block holds
                const int c = tid, L = chain_len(g, blk, c);
                if (L > 0) {
                    double sum = 0.0;
                    if (w.chain_axis == 0) {
                        for (int t = 0; t < w.N; ++t) sum += llc[c * VD_NMAX + t];
                    } else {
                        for (int i = 0; i < L; ++i) sum += llc[c * stride + i];
                    }
                    const int sidx = blk % g.nseg, lb = blk / g.nseg;
                    B.ll_partial[(size_t)(lb * g.C + c) * g.nseg + sidx] = sum;
                }
            }
        }
    }
    if (!do_m) return;

    // -------------------------------- M-step ------------------------------------
    if (!do_e) {
        for (int k = tid; k < npix; k += VD_BLOCK) {
            const BlockPix p = block_pix(g, blk, k);
            if (!p.valid) continue;
            const int o = p.c * stride + p.i;
            for (int t = 0; t < w.N; ++t) q_s[t * nodes + o] = B.q_in[t * lplane + p.li];
        }
        __syncthreads();
    }
    const uint32_t word2 = philox_word2(w.it, w.level, PURPOSE_CAND);
    const bool local = (w.level == 1);

    // phase A: parallel over pixels and slots {0, 2, 3..K-1} (or precomputed by k_phase_a)
    if (do_m == 2) {
        for (int k = tid; k < npix; k += VD_BLOCK) {
            const BlockPix p = block_pix(g, blk, k);
            if (!p.valid) continue;
            const int o = p.c * stride + p.i;
            bestE[o] = B.pa_E[p.li];
            bestV[o] = B.pa_V[p.li];
            bestS[o] = B.pa_S[p.li];
            rcur[o] = rho_full[p.v * w.W + p.u];
            for (int d = 0; d < g.spec; ++d) specE[d * nodes + o] = B.pa_spec[d * lplane + p.li];
        }
    }
    for (int k = tid; k < npix && do_m == 1; k += VD_BLOCK) {
        const BlockPix p = block_pix(g, blk, k);
        if (!p.valid) continue;
        const int o = p.c * stride + p.i;
        Pix c;
        pix_geometry<PR>(w, B.P, B.flow, p.u, p.v, c);
#pragma unroll
        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) c.q[t] = q_s[t * nodes + o];
        const int fpix = p.v * w.W + p.u;
        const float r0 = rho_full[fpix];
        prior_posteriors<PR>(w, B.P, B.prior, B.prior_weight, fpix, c, r0);
        energy_t bE = keep_cost ? energy2_costs<PR>(w, B.P, B.prior, c, r0, cost_s + o, nodes)
                                : energy2<B2, PR>(w, B.P, B.flow2, B.prior, c, r0);
        float bV = r0;
        int bS = 0;
        // the candidates are evaluated in groups of PG against the best before the group,
        // then merged in slot order: the same winner and energy as one at a time.  A group's
        // flow gathers of a frame are issued together.  Group h holds slots 4h + 2 .. 4h + 5:
        // slot 2 (the coarse value, local level only) rides with the first three draws of
        // Philox group 0, and each later group starts with the previous Philox group's last
        // draw.  Groups of 4 (pairs with priors, whose per-pixel context is larger) at 4
        // waves per SIMD.
        float rc = 0.f;
        if (local) {
            const int U = min(p.u / w.s, w.wc - 1), V = min(p.v / w.s, w.hc - 1);
            rc = B.idepth_coarse[V * w.wc + U];
        }
        constexpr int PG = PR ? 2 : 4;
        const int NH = (w.K - 2 + 3) / 4;
        uint32_t carry = 0u;
        for (int h = 0; h < NH; ++h) {
            uint4 r = make_uint4(0u, 0u, 0u, 0u);
            if (4 * h + 3 < w.K)
                r = philox10(make_uint4((uint32_t)p.li, (uint32_t)h, word2, w.window_id), w.key0, w.key1);
            const uint32_t words[4] = {carry, r.x, r.y, r.z};
            carry = r.w;
            float cand[4];
            energy_t e[4];
            unsigned live = 0u;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int slot = 4 * h + 2 + m;
                const float uu = unit24(words[m]);
                cand[m] = (slot & 1) ? fminf(fmaxf(r0 * fmaf(w.sigma_it, fmaf(2.f, uu, -1.f), 1.f), w.rmin), w.rmax)
                                     : fmaf(uu, w.rmax - w.rmin, w.rmin);
                if (slot < w.K) live |= 1u << m;
            }
            if (h == 0) {
                cand[0] = rc;
                if (!local) live &= ~1u;
            }
#pragma unroll
            for (int q = 0; q < 4; q += PG) {
                energy2_bounded_m<B2, PR, PG>(w, B.P, B.flow2, B.prior, c, cand + q,
                                              (live >> q) & ((1u << PG) - 1u), bE, e + q);
#pragma unroll
                for (int m = q; m < q + PG; ++m)
                    if (((live >> m) & 1u) && e[m] < bE) { bE = e[m]; bV = cand[m]; bS = 4 * h + 2 + m; }
            }
        }
        bestE[o] = bE; bestV[o] = bV; bestS[o] = bS; rcur[o] = r0;
    }
    __syncthreads();

    // phase A2: energies at the phase-A winners of the g.spec previous nodes of the chain
    const bool fwd = (w.dir < 2);
    const int di = fwd ? 1 : -1;
    for (int k = tid; k < npix && do_m == 1; k += VD_BLOCK) {
        const BlockPix p = block_pix(g, blk, k);
        if (!p.valid) continue;
        const int L = chain_len(g, blk, p.c);
        const int o = p.c * stride + p.i;
        Pix c;
        pix_geometry<PR>(w, B.P, B.flow, p.u, p.v, c);
#pragma unroll
        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) c.q[t] = q_s[t * nodes + o];
        prior_posteriors<PR>(w, B.P, B.prior, B.prior_weight, p.v * w.W + p.u, c, rcur[o]);
        // the speculative energies in lockstep pairs (one strict bound, no merging): each is
        // the value of its own bounded evaluation, their gathers in flight together
        for (int d0 = 0; d0 < g.spec; d0 += 2) {
            float cand[2];
            unsigned live = 0u;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int ip = p.i - (d0 + m + 1) * di;
                const bool in = d0 + m < g.spec && ip >= 0 && ip < L;
                cand[m] = in ? bestV[p.c * stride + ip] : 0.f;
                if (in) live |= 1u << m;
            }
            if (live == 0u) break;
            energy_t e[2];
            energy2_bounded_m<B2, PR, 2, true>(w, B.P, B.flow2, B.prior, c, cand, live, bestE[o], e);
#pragma unroll
            for (int m = 0; m < 2; ++m)
                if ((live >> m) & 1u) specE[(d0 + m) * nodes + o] = e[m];
        }
    }
    __syncthreads();

    // phase B: serial scan per chain, a group of 32 lanes per chain.  A speculation miss
    // evaluates E_i(carried) with the frame terms on separate lanes of the group
    // (energy2_lanes), which equals the sequential evaluation bit for bit.  Without priors a
    // miss evaluates the carried value at this node and the next LA - 1 nodes of the chain
    // at once, one lane per (node, frame), each energy summed in frame order as energy2_lanes
    // does; the next nodes use them while the same value is carried.
    {
        const int grp = tid >> 5, hl = tid & 31, hbase = tid & 32;
        const int LA = 32 / w.N;                            // nodes per lookahead
        if constexpr (LC) {
            // Long chains: the serial path visits only the nodes whose phase-A result replaces
            // the carried value.  Every node first finds, from the speculative energies and in
            // parallel, the next node that would replace its phase-A result within the
            // speculation depth (-1: none there, -2: none up to the chain end).  A walk per
            // chain then hops from replacement to replacement; a value that outlives the
            // speculation depth is evaluated at the following nodes as in the scan below.
            // The decisions are those of the node-by-node scan, bit for bit.
            // [C][stride] (next replacement, phase-A value) per node, one 8-byte LDS read per hop;
            // the E-step ratios are dead here
            int2* hop = (int2*)r_s;
            int* mark = (int*)(hop + nodes);                // [C][stride] replacement nodes of the walk
            for (int k = tid; k < npix; k += VD_BLOCK) {
                const BlockPix p = block_pix(g, blk, k);
                if (!p.valid) continue;
                const int L = chain_len(g, blk, p.c);
                const int base = p.c * stride;
                const int pos = fwd ? p.i : L - 1 - p.i;    // steps from the chain start
                int nx = -1;
                for (int d = 1; d <= g.spec; ++d) {
                    if (pos + d >= L) { nx = -2; break; }
                    const int j = p.i + d * di;
                    const energy_t e1 = specE[(d - 1) * nodes + base + j], eA = bestE[base + j];
                    if (!((e1 < eA) || (e1 == eA && bestS[base + j] > 1))) { nx = j; break; }
                }
                hop[base + p.i] = make_int2(nx, __float_as_int(bestV[base + p.i]));
                mark[base + p.i] = 0;
            }
            __syncthreads();
            if constexpr (!PR) {
                // one wave per chain: the walk's state is uniform over the wave and kept in
                // scalar registers, so a hop costs one LDS round trip, one mark and a few
                // scalar instructions; a value that outlives the speculation depth is
                // evaluated at the next 64 / N nodes at once, one lane per (node, frame).
                // The nodes between two marks are filled afterwards by a prefix pass.
                const int wl = tid & 63;
                const int LW = 64 / w.N;
                for (int c = __builtin_amdgcn_readfirstlane(tid >> 6); c < g.C; c += VD_BLOCK / 64) {
                    const int L = chain_len(g, blk, c);
                    if (L <= 0) continue;
                    const int base = c * stride;
                    const int iend = fwd ? L : -1;
                    for (int i = fwd ? 0 : L - 1; i != iend;) {
                        mark[base + i] = 1;                         // the same address on every lane
                        const int2 h = hop[base + i];
                        const float carried = __int_as_float(h.y);
                        int ni = __builtin_amdgcn_readfirstlane(h.x);
                        if (ni == -1) {
                            ni = iend;
                            for (int j0 = i + (g.spec + 1) * di; (fwd ? j0 < L : j0 >= 0) && ni == iend; j0 += LW * di) {
                                const int m = wl / w.N, t = wl - m * w.N;
                                const int jm = j0 + m * di;
                                float mine = 0.f;
                                if (m < LW && jm >= 0 && jm < L) {
                                    const int kk = g.horizontal ? (c * g.seg + jm) : (jm * g.C + c);
                                    const BlockPix p = block_pix(g, blk, kk);
                                    Pix cx;
                                    pix_geometry<false>(w, B.P, B.flow, p.u, p.v, cx);
                                    mine = frame_cost<B2>(w, B.P, B.flow2, cx, carried, t);
                                }
                                const int mm = min(wl, LW - 1), jmm = j0 + mm * di;
                                const bool mine_node = wl < LW && jmm >= 0 && jmm < L;
                                energy_t la_e = 0.0;
#pragma unroll
                                for (int tt = 0; tt < VD_NMAX; ++tt) {
                                    if (tt < w.N) {
                                        const float ct = __shfl(mine, mm * w.N + tt);
                                        if (mine_node) la_e = eacc(q_s[tt * nodes + base + jmm], ct, la_e);
                                    }
                                }
                                // lane m < LW decides node j0 + m di; the first replacing
                                // node in sweep order is the lowest such lane
                                bool rep = false;
                                if (mine_node) {
                                    const energy_t eA = bestE[base + jmm];
                                    rep = !((la_e < eA) || (la_e == eA && bestS[base + jmm] > 1));
                                }
                                const unsigned long long rm = __ballot(rep);
                                if (rm) ni = j0 + (__ffsll((long long)rm) - 1) * di;
                            }
                        } else if (ni == -2) {
                            ni = iend;
                        }
                        i = ni;
                    }
                    // every node takes the phase-A value of the last mark at or before it along
                    // the sweep: 64-node chunks, the marks of a chunk by ballot, the last mark
                    // of the chunks before carried along (the chain head is always marked)
                    int last = 0;
                    for (int cb = 0; cb < L; cb += 64) {
                        const int pos = cb + wl;
                        const int ii = fwd ? pos : L - 1 - pos;
                        const unsigned long long mk = __ballot(pos < L && mark[base + ii] != 0);
                        const unsigned long long below = wl == 63 ? mk : mk & ((2ull << wl) - 1ull);
                        const int src = below ? cb + 63 - __clzll(below) : last;
                        if (pos < L) newV[base + ii] = bestV[base + (fwd ? src : L - 1 - src)];
                        if (mk) last = cb + 63 - __clzll(mk);
                    }
                }
            } else {
                // with priors: a group of 32 lanes per chain; a value that outlives the
                // speculation depth is evaluated at the next 32 / N nodes at once, with each
                // node's prior terms on its own lane; marks and the fill pass as above
                for (int c = grp; c < g.C; c += VD_BLOCK / 32) {
                    const int L = chain_len(g, blk, c);
                    if (L <= 0) continue;
                    const int base = c * stride;
                    const int iend = fwd ? L : -1;
                    for (int i = fwd ? 0 : L - 1; i != iend;) {
                        mark[base + i] = 1;
                        const int2 h = hop[base + i];
                        const float carried = __int_as_float(h.y);
                        int ni = h.x;
                        if (ni == -1) {
                            ni = iend;
                            for (int j0 = i + (g.spec + 1) * di; (fwd ? j0 < L : j0 >= 0) && ni == iend; j0 += LA * di) {
                                // lane m * N + t: frame t at node j0 + m di; lane m < LA sums node
                                // m's frame terms in frame order, then adds its prior terms, as
                                // energy2_lanes does for one node
                                const int m = hl / w.N, t = hl - m * w.N;
                                const int jm = j0 + m * di;
                                float mine = 0.f;
                                if (m < LA && jm >= 0 && jm < L) {
                                    const int kk = g.horizontal ? (c * g.seg + jm) : (jm * g.C + c);
                                    const BlockPix p = block_pix(g, blk, kk);
                                    Pix cx;
                                    pix_geometry<PR>(w, B.P, B.flow, p.u, p.v, cx);
                                    mine = frame_cost<B2>(w, B.P, B.flow2, cx, carried, t);
                                }
                                const int mm = min(hl, LA - 1), jmm = j0 + mm * di;
                                const bool mine_node = hl < LA && jmm >= 0 && jmm < L;
                                const int on = base + (mine_node ? jmm : 0);
                                Pix cn;
                                if (mine_node) {
                                    const int kk = g.horizontal ? (c * g.seg + jmm) : (jmm * g.C + c);
                                    const BlockPix p = block_pix(g, blk, kk);
                                    pix_geometry<PR>(w, B.P, B.flow, p.u, p.v, cn);
#pragma unroll
                                    for (int tt = 0; tt < VD_NMAX; ++tt) if (tt < w.N) cn.q[tt] = q_s[tt * nodes + on];
                                    prior_posteriors<PR>(w, B.P, B.prior, B.prior_weight, p.v * w.W + p.u, cn, rcur[on]);
                                }
                                energy_t e1 = 0.0;
#pragma unroll
                                for (int tt = 0; tt < VD_NMAX; ++tt) {
                                    if (tt < w.N) {
                                        const float ct = __shfl(mine, hbase + mm * w.N + tt);
                                        if (mine_node) e1 = eacc(cn.q[tt], ct, e1);
                                    }
                                }
                                bool rep = false;
                                if (mine_node) {
                                    e1 = prior_terms<PR>(w, B.P, B.prior, cn, carried, e1);
                                    const energy_t eA = bestE[on];
                                    rep = !((e1 < eA) || (e1 == eA && bestS[on] > 1));
                                }
                                // the first replacing node in sweep order: this group's lowest lane
                                const unsigned rm = (unsigned)(__ballot(rep) >> hbase);
                                if (rm) ni = j0 + (__ffs(rm) - 1) * di;
                            }
                        } else if (ni == -2) {
                            ni = iend;
                        }
                        i = ni;
                    }
                    // the fill pass as above, 32-node chunks (this group's half of the ballot)
                    int last = 0;
                    for (int cb = 0; cb < L; cb += 32) {
                        const int pos = cb + hl;
                        const int ii = fwd ? pos : L - 1 - pos;
                        const unsigned mk = (unsigned)(__ballot(pos < L && mark[base + ii] != 0) >> hbase);
                        const unsigned below = hl == 31 ? mk : mk & ((2u << hl) - 1u);
                        const int src = below ? cb + 31 - __clz(below) : last;
                        if (pos < L) newV[base + ii] = bestV[base + (fwd ? src : L - 1 - src)];
                        if (mk) last = cb + 31 - __clz(mk);
                    }
                }
            }
        } else {
            for (int c = grp; c < g.C; c += VD_BLOCK / 32) {
                const int L = chain_len(g, blk, c);
                if (L <= 0) continue;
                const int i0 = fwd ? 0 : L - 1;
                const int base = c * stride;
                float carried = bestV[base + i0];
                int src = i0;
                int la_src = -1, la_i = 0;                      // lookahead: source node, first node
                energy_t la_e = 0.0;                            // lane m < LA: energy at node la_i + m*di
                if (hl == 0) newV[base + i0] = carried;
                for (int n = 1, i = i0 + di; n < L; ++n, i += di) {
                    const int o = base + i;
                    energy_t e1;
                    const int dist = (i - src) * di;            // steps back to the carried value's node
                    if (dist <= g.spec) {
                        e1 = specE[(dist - 1) * nodes + o];
                    } else if constexpr (!PR) {
                        if (la_src != src || (i - la_i) * di >= LA) {
                            la_src = src;
                            la_i = i;
                            const int m = hl / w.N, t = hl - m * w.N;
                            const int im = i + m * di;
                            float mine = 0.f;
                            if (m < LA && im >= 0 && im < L) {
                                const int kk = g.horizontal ? (c * g.seg + im) : (im * g.C + c);
                                const BlockPix p = block_pix(g, blk, kk);
                                Pix cx;
                                pix_geometry<false>(w, B.P, B.flow, p.u, p.v, cx);
                                mine = frame_cost<B2>(w, B.P, B.flow2, cx, carried, t);
                            }
                            const int mm = min(hl, LA - 1), imm = i + mm * di;
                            const bool mine_node = hl < LA && imm >= 0 && imm < L;
                            la_e = 0.0;
#pragma unroll
                            for (int tt = 0; tt < VD_NMAX; ++tt) {
                                if (tt < w.N) {
                                    const float ct = __shfl(mine, hbase + mm * w.N + tt);
                                    if (mine_node) la_e = eacc(q_s[tt * nodes + base + imm], ct, la_e);
                                }
                            }
                        }
                        e1 = __shfl(la_e, hbase + (i - la_i) * di);
                    } else {
                        // storage-order node i of chain c -> block linear index
                        const int kk = g.horizontal ? (c * g.seg + i) : (i * g.C + c);
                        const BlockPix p = block_pix(g, blk, kk);
                        Pix cx;
                        pix_geometry<PR>(w, B.P, B.flow, p.u, p.v, cx);
#pragma unroll
                        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) cx.q[t] = q_s[t * nodes + o];
                        prior_posteriors<PR>(w, B.P, B.prior, B.prior_weight, p.v * w.W + p.u, cx, rcur[o]);
                        e1 = energy2_lanes<B2, PR>(w, B.P, B.flow2, B.prior, cx, carried, hl, hbase);
                    }
                    const energy_t eA = bestE[o];
                    const bool keep = (e1 < eA) || (e1 == eA && bestS[o] > 1);
                    if (!keep) { carried = bestV[o]; src = i; }
                    if (hl == 0) newV[o] = carried;
                }
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < npix; k += VD_BLOCK) {
        const BlockPix p = block_pix(g, blk, k);
        if (!p.valid) continue;
        B.rho_out[local ? (p.v * w.W + p.u) : p.li] = newV[p.c * stride + p.i];
    }
}

// LC: the E-only and scan-only launches of a level with few long chains (the coarse
// lattice): forward-backward as a segmented scan, and the streamlined serial scan
// 4 waves per SIMD (up to 128 VGPRs): the candidate groups' gathers need the registers
template <bool B2, bool PR, bool LC>
__global__ void __launch_bounds__(VD_BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_level(Win w, LevelGeom g, LevelBufs B, int do_e, int do_m) {
    extern __shared__ __align__(16) float lds[];
    const int xb = xcd_block(blockIdx.x, gridDim.x);
    level_body<B2, PR, LC>(w, g, B, do_e, do_m, B.blk_order ? B.blk_order[xb] : xb, lds);
}

// ----------------------------------------------------------------------------------
// phase A as a separate grid: LANES lanes per level pixel (4, 8 or 16).  Lane 0 takes slot
// 0; with up to 8 lanes, lane l takes the Philox groups g = l, l + LANES, ... (slots
// 3 + 4g .. 6 + 4g); with 16, lanes 2h and 2h + 1 share the groups of h, each taking two of
// a group's four slots.  On the local level lane 1 takes slot 2 first.  Each lane scans its
// slots in increasing order with strict improvement and pruning at its own best, then the
// lanes merge by (energy, slot): the result equals the argmin over all slots with ties to
// the lowest slot, whatever LANES is.
// ----------------------------------------------------------------------------------
template <bool B2, bool PR, int LANES = VD_PA_LANES>
__device__ __forceinline__ void phase_a_body(const Win& w, const LevelGeom& g, const LevelBufs& B, int blk) {
    constexpr int SUB = LANES > 8 ? LANES / 8 : 1;        // lanes per Philox group
    constexpr int GSTRIDE = LANES / SUB;                  // groups advance by this much
    constexpr int MPER = 4 / SUB;                         // slots of a group per lane
    const int gid = blk * VD_BLOCK + threadIdx.x;
    const int li = gid / LANES, lane = gid % LANES;
    const int gl = lane / SUB, part = lane - gl * SUB;
    const size_t lplane = (size_t)g.h * g.w;
    const bool valid = li < (int)lplane;
    energy_t bE = __builtin_huge_val();
    float bV = 0.f, r0 = 0.f;
    int bS = 1 << 30;
    if (valid) {
        const int ly = li / g.w, lx = li - ly * g.w;
        const int u = g.s * lx + g.off, v = g.s * ly + g.off;
        Pix c;
        pix_geometry<PR>(w, B.P, B.flow, u, v, c);
#pragma unroll
        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) c.q[t] = B.q_in[t * lplane + li];
        const int fpix = v * w.W + u;
        r0 = B.idepth[fpix];
        prior_posteriors<PR>(w, B.P, B.prior, B.prior_weight, fpix, c, r0);
        if (lane == 0) {
            bE = energy2<B2, PR>(w, B.P, B.flow2, B.prior, c, r0); bV = r0; bS = 0;
        }
        if (lane == 1 && w.level == 1) {
            const int U = min(u / w.s, w.wc - 1), V = min(v / w.s, w.hc - 1);
            const float rc = B.idepth_coarse[V * w.wc + U];
            const energy_t e = energy2_bounded<B2, PR, false>(w, B.P, B.flow2, B.prior, c, rc, bE);
            if (e < bE) { bE = e; bV = rc; bS = 2; }
        }
        const int G = (w.K - 3 + 3) / 4;
        const uint32_t word2 = philox_word2(w.it, w.level, PURPOSE_CAND);
        for (int gi = gl; gi < G; gi += GSTRIDE) {
            const uint4 r = philox10(make_uint4((uint32_t)li, (uint32_t)gi, word2, w.window_id), w.key0, w.key1);
            const uint32_t words[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int m = part * MPER; m < (part + 1) * MPER; ++m) {
                const int slot = 3 + 4 * gi + m;
                if (slot < w.K) {
                    const float uu = unit24(words[m]);
                    const float cand = (slot & 1)
                        ? fminf(fmaxf(r0 * fmaf(w.sigma_it, fmaf(2.f, uu, -1.f), 1.f), w.rmin), w.rmax)
                        : fmaf(uu, w.rmax - w.rmin, w.rmin);
                    const energy_t e = energy2_bounded<B2, PR, false>(w, B.P, B.flow2, B.prior, c, cand, bE);
                    if (e < bE) { bE = e; bV = cand; bS = slot; }
                }
            }
        }
    }
#pragma unroll
    for (int off = 1; off < LANES; off <<= 1) {
        const energy_t oE = __shfl_xor(bE, off);
        const float oV = __shfl_xor(bV, off);
        const int oS = __shfl_xor(bS, off);
        if (oE < bE || (oE == bE && oS < bS)) { bE = oE; bV = oV; bS = oS; }
    }
    if (valid && lane == 0) {
        B.pa_E[li] = bE;
        B.pa_V[li] = bV;
        B.pa_S[li] = bS;
    }
}

template <bool B2, bool PR, int LANES>
__global__ void __launch_bounds__(VD_BLOCK) k_phase_a(Win w, LevelGeom g, LevelBufs B) {
    phase_a_body<B2, PR, LANES>(w, g, B, xcd_block(blockIdx.x, gridDim.x));
}

// ----------------------------------------------------------------------------------
// phase A2 as a separate grid (level with few long chains): one lane per (level pixel,
// depth d), E_i at the phase-A winner of the node d + 1 steps back along the chain,
// bounded (strict) by the pixel's phase-A energy.
// ----------------------------------------------------------------------------------
template <bool B2, bool PR>
__device__ __forceinline__ void phase_a2_body(const Win& w, const LevelGeom& g, const LevelBufs& B, int blk) {
    const int gid = blk * VD_BLOCK + threadIdx.x;
    const int li = gid / g.spec, d = gid - li * g.spec;
    const size_t lplane = (size_t)g.h * g.w;
    if (li >= (int)lplane) return;
    const int ly = li / g.w, lx = li - ly * g.w;
    const int pos = g.horizontal ? lx : ly;
    const int axis = g.horizontal ? g.w : g.h;
    const int start = (pos / g.seg) * g.seg, end = min(start + g.seg, axis);
    const int step = (w.dir < 2) ? 1 : -1;
    const int pp = pos - (d + 1) * step;
    if (pp < start || pp >= end) return;
    const int lp = g.horizontal ? (ly * g.w + pp) : (pp * g.w + lx);
    const int u = g.s * lx + g.off, v = g.s * ly + g.off;
    Pix c;
    pix_geometry<PR>(w, B.P, B.flow, u, v, c);
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) c.q[t] = B.q_in[t * lplane + li];
    const int fpix = v * w.W + u;
    prior_posteriors<PR>(w, B.P, B.prior, B.prior_weight, fpix, c, B.idepth[fpix]);
    B.pa_spec[d * lplane + li] =
        energy2_bounded<B2, PR, true>(w, B.P, B.flow2, B.prior, c, B.pa_V[lp], B.pa_E[li]);
}

template <bool B2, bool PR>
__global__ void __launch_bounds__(VD_BLOCK) k_phase_a2(Win w, LevelGeom g, LevelBufs B) {
    phase_a2_body<B2, PR>(w, g, B, xcd_block(blockIdx.x, gridDim.x));
}

// ----------------------------------------------------------------------------------
// pose normal equations for frame t at candidate poses; optional FP64 solve + update
// ----------------------------------------------------------------------------------
// Pose-step terms exist only where the reprojection lands inside frame t's image: a flow
// end point is observed nowhere else, and points passing just in front of camera t
// (Q_z -> 0+, far outside the image) would otherwise dominate the normal equations with
// weight ~ 1/Q_z^2.  NaN coordinates fail the test.
__device__ __forceinline__ bool in_frame(const Win& w, float px, float py) {
    return px >= 0.f && px <= (float)(w.W - 1) && py >= 0.f && py <= (float)(w.H - 1);
}

template <bool B2>
__device__ __forceinline__ void pose_pixel(const Win& w, const PoseBufs& B, const PoseF& Tc, int t, int j,
                                           float* acc) {
    const size_t plane = (size_t)w.H * w.W;
    const float2* flow_t = B.flow + (t - 1) * plane;
    const float4* flow2_t = B.flow2 + (t - 1) * plane;
    const int v = j / w.W, u = j - v * w.W;
    const float rho = B.idepth[j];
    const float q = B.rigid[(t - 1) * plane + j];
    const float x0 = ((float)u - w.cx) * w.ifx, x1 = ((float)v - w.cy) * w.ify;
    // displacement form (see frame_residuals): d = p - j from D = (R - I) x~ + rho t
    float dpx = 0.f, dpy = 0.f, fx, fy;
    bool zprev = true, fok;
    if (t == 1) {
        const float2 f = flow_t[j];
        fx = f.x; fy = f.y;
        fok = isfinite(fx) && isfinite(fy);
    } else {
        const PoseF& Tp = B.P[t - 2];
        const float Dx = fmaf(rho, Tp.t[0], fmaf(Tp.d[0], x0, fmaf(Tp.d[1], x1, Tp.d[2])));
        const float Dy = fmaf(rho, Tp.t[1], fmaf(Tp.d[3], x0, fmaf(Tp.d[4], x1, Tp.d[5])));
        const float Dz = fmaf(rho, Tp.t[2], fmaf(Tp.d[6], x0, fmaf(Tp.d[7], x1, Tp.d[8])));
        zprev = 1.f + Dz > 0.f;
        const float iz = rcp(1.f + Dz);
        dpx = w.fx * fmaf(-x0, Dz, Dx) * iz;
        dpy = w.fy * fmaf(-x1, Dz, Dy) * iz;
        fok = sample_flow2(flow2_t, w.H, w.W, (float)u + dpx, (float)v + dpy, fx, fy);
    }
    const float Dx = fmaf(rho, Tc.t[0], fmaf(Tc.d[0], x0, fmaf(Tc.d[1], x1, Tc.d[2])));
    const float Dy = fmaf(rho, Tc.t[1], fmaf(Tc.d[3], x0, fmaf(Tc.d[4], x1, Tc.d[5])));
    const float Dz = fmaf(rho, Tc.t[2], fmaf(Tc.d[6], x0, fmaf(Tc.d[7], x1, Tc.d[8])));
    const float Qx = x0 + Dx, Qy = x1 + Dy, Qz = 1.f + Dz;
    const bool zok = Qz > 0.f;
    const float iz = rcp(Qz);
    const float dx = w.fx * fmaf(-x0, Dz, Dx) * iz, dy = w.fy * fmaf(-x1, Dz, Dy) * iz;
    const bool ok = zprev && zok && fok && in_frame(w, (float)u + dx, (float)v + dy);
    const float ex = (dx - dpx) - fx, ey = (dy - dpy) - fy;
    const float r2 = fmaf(ex, ex, ey * ey);
    acc[0] = fmaf(q, ok ? flow_cost2<B2>(w, r2) : 1.0f, acc[0]);
    if (ok) {
        const float wt = q * flow_dcost<B2>(w, r2);
        // J rows of p = pi(Q), Q = R x~ + rho t, left update (dw, dv): dQ = [-[Q]x | rho I]
        const float a = w.fx * iz, b = -w.fx * Qx * iz * iz;
        const float c = w.fy * iz, d = -w.fy * Qy * iz * iz;
        const float jx[6] = {b * Qy, a * Qz - b * Qx, -a * Qy, a * rho, 0.f, b * rho};
        const float jy[6] = {d * Qy - c * Qz, -d * Qx, c * Qx, 0.f, c * rho, d * rho};
        int k = 1;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const float wxi = wt * jx[i], wyi = wt * jy[i];
#pragma unroll
            for (int l = i; l < 6; ++l) {
                acc[k] = fmaf(wxi, jx[l], fmaf(wyi, jy[l], acc[k]));
                ++k;
            }
            acc[22 + i] = fmaf(wxi, ex, fmaf(wyi, ey, acc[22 + i]));
        }
        acc[28] += 1.f;
    }
}

// Normal equations of frame t at candidate poses: two pixels per thread summed in FP32,
// then FP64 across threads and blocks.  One record per block, value-major.
template <bool B2>
__global__ void __launch_bounds__(VD_BLOCK)
k_pose(Win w, PoseBufs B, int t, const double* __restrict__ cand) {
    __shared__ double red[(VD_BLOCK / 64) * 29];
    __shared__ PoseF candF;
    const int tid = threadIdx.x;
    const int ci = blockIdx.y;
    if (tid == 0) {
        if (cand) pose_to_f(cand + 6 * ci, &candF);
        else candF = B.P[t - 1];
    }
    __syncthreads();
    const PoseF Tc = candF;
    const int plane = w.H * w.W;
    double acc[29];
#pragma unroll
    for (int k = 0; k < 29; ++k) acc[k] = 0.0;
    const int stride = gridDim.x * VD_BLOCK;
    for (int j = xcd_block(blockIdx.x, gridDim.x) * VD_BLOCK + tid; j < plane; j += 2 * stride) {
        float a32[29];
#pragma unroll
        for (int k = 0; k < 29; ++k) a32[k] = 0.f;
        pose_pixel<B2>(w, B, Tc, t, j, a32);
        if (j + stride < plane) pose_pixel<B2>(w, B, Tc, t, j + stride, a32);
#pragma unroll
        for (int k = 0; k < 29; ++k) acc[k] += (double)a32[k];
    }
    block_reduce<29>(acc, red);
    // energy was summed in log2 units
    if (tid < 29) B.partials[((size_t)ci * 29 + tid) * gridDim.x + blockIdx.x] = red[tid] * (tid == 0 ? (double)VD_LN2 : 1.0);
}

// Sum of candidate ci's block records (fixed order); optional FP64 solve and pose update.
// One block per candidate; launched after k_pose on the same stream.
__global__ void __launch_bounds__(VD_BLOCK)
k_pose_finish(PoseBufs B, int t, unsigned nb, int solve) {
    __shared__ double red[(VD_BLOCK / 64) * 29];
    const int ci = blockIdx.x;
    reduce_partials<29>(B.partials + (size_t)ci * nb * 29, nb, red);
    if (threadIdx.x != 0) return;
    if (B.out) for (int k = 0; k < 29; ++k) B.out[ci * 29 + k] = red[k];
    if (!solve) return;
    double H[36], gv[6], x[6];
    int k = 1;
    for (int i = 0; i < 6; ++i)
        for (int l = i; l < 6; ++l) { H[6 * i + l] = H[6 * l + i] = red[k++]; }
    double tr = 0.0;
    for (int i = 0; i < 6; ++i) { gv[i] = -red[22 + i]; tr += H[7 * i]; }
    const double lam = 1e-9 * tr / 6.0;
    for (int i = 0; i < 6; ++i) H[7 * i] += lam;
    if (chol6_solve(H, gv, x)) {
        left_update_d(B.PD + (t - 1), x);
        posef_from_d(B.PD[t - 1], B.P + (t - 1));
    }
}

// ----------------------------------------------------------------------------------
// pose step, one launch per Gauss-Newton step s = 0 .. N*G-1 (frame t = s/G + 1, GN index
// k = s mod G).  Prologue: every block sums the previous step's block records (fixed
// order, so all blocks agree bit for bit), solves (H + 1e-9 tr(H)/6 I) delta = -g in FP64
// and applies it to that frame's pose; block 0 persists the result in hist[s-1] (no other
// block reads it during this launch).  Pass: normal equations of frame t at its current
// pose; the observation o_t = p_{t-1} + X_t(p_{t-1}) is formed at k = 0 and stored as a
// displacement from the pixel (NaN when invalid) for the frame's later steps.
// ----------------------------------------------------------------------------------
// A Gauss-Newton record holds the normal equations only: H (upper triangle, 21 values)
// then g (6 values); the energy and term count of the pose score are not needed here.
constexpr int kGnRec = 27;

__device__ inline void pose_gn_solve(const double* red, PoseD& P) {
    double H[36], gv[6], x[6];
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int l = i; l < 6; ++l) { H[6 * i + l] = H[6 * l + i] = red[k++]; }
    double tr = 0.0;
    for (int i = 0; i < 6; ++i) { gv[i] = -red[21 + i]; tr += H[7 * i]; }
    const double lam = 1e-9 * tr / 6.0;
    for (int i = 0; i < 6; ++i) H[7 * i] += lam;
    if (chol6_solve(H, gv, x)) left_update_d(&P, x);      // singular: pose unchanged
}

// SPLIT (batched launches): no prologue solve; the pose of step s-1 is read from hist[s-1],
// stored there by the one-block solve launch that follows each pass (pose_gn_solve_body).
// Many windows' blocks share the chip there, and re-reducing every window's records in each
// of its blocks would cost more than the extra launch.
template <bool B2, bool SPLIT = false>
__device__ __forceinline__ void pose_gn_body(const Win& w, const PoseBufs& B, int s, int G, int blk, unsigned nb) {
    __shared__ double red[(VD_GN_BLOCK / 64) * 29];
    __shared__ PoseF curF, prevF;
    const int tid = threadIdx.x;
    const int t = s / G + 1, k = s - (t - 1) * G;
    const int plane = w.H * w.W;
    const float2* __restrict__ flow_t = B.flow + (size_t)(t - 1) * plane;
    const float4* __restrict__ flow2_t = B.flow2 + (size_t)(t - 1) * plane;
    const float* __restrict__ idepth = B.idepth;
    const float* __restrict__ rig = B.rigid + (size_t)(t - 1) * plane;
    float2* __restrict__ obs = B.obs;
    const int stride = (int)nb * VD_GN_BLOCK;
    // pixels per thread and batch, loads issued together: all of a thread's pixels for one
    // window (one block per CU, registers to spare); two in the batched pass, whose many
    // blocks per CU need the occupancy.  The pixel order, and so every sum, is the same.
    constexpr int UB = SPLIT ? VD_GN_PIX : VD_GN_UB;
    float rho[UB], q[UB], ox[UB], oy[UB];
    int jj[UB];
    auto load = [&](int j0) {
#pragma unroll
        for (int b = 0; b < UB; ++b) {
            const int j = j0 + b * stride;
            jj[b] = j < plane ? j : -1;
            const int jc = j < plane ? j : 0;
            rho[b] = idepth[jc];
            q[b] = rig[jc];
            if (k > 0) { const float2 o = obs[jc]; ox[b] = o.x; oy[b] = o.y; }
            else if (t == 1) { const float2 f = flow_t[jc]; ox[b] = f.x; oy[b] = f.y; }
        }
    };
    int j0 = blk * VD_GN_BLOCK + tid;
    if (j0 < plane) load(j0);              // the first batch is in flight during the prologue
    if constexpr (SPLIT) {
        if (tid == 0) {
            if (k > 0) {
                posef_from_d(B.hist[s - 1], &curF);
            } else {
                curF = B.P[t - 1];
                if (t > 1) posef_from_d(B.hist[s - 1], &prevF);
            }
        }
    } else if (s > 0) {
        reduce_partials<kGnRec, VD_GN_BLOCK>(B.partials + (size_t)((s - 1) & 1) * kGnRec * nb, nb, red);
        if (tid == 0) {
            const int sp = s - 1, tp = sp / G + 1, kp = sp - (tp - 1) * G;
            PoseD P = (kp == 0) ? B.PD[tp - 1] : B.hist[sp - 1];
            pose_gn_solve(red, P);
            PoseF F;
            posef_from_d(P, &F);
            if (blk == 0) B.hist[sp] = P;
            if (k == 0) { prevF = F; curF = B.P[t - 1]; }
            else curF = F;
        }
    } else if (tid == 0) {
        curF = B.P[t - 1];
    }
    __syncthreads();
    const PoseF Tc = curF;
    // per-thread sums in FP32 (a thread covers a few pixels), FP64 across threads and blocks
    float a32[kGnRec];
#pragma unroll
    for (int i = 0; i < kGnRec; ++i) a32[i] = 0.f;
    while (j0 < plane) {
        if (k == 0 && t > 1) {
            const PoseF& Tp = prevF;
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                const int jc = jj[b] >= 0 ? jj[b] : 0;
                const int v = jc / w.W, u = jc - v * w.W;
                const float x0 = ((float)u - w.cx) * w.ifx, x1 = ((float)v - w.cy) * w.ify;
                const float Dx = fmaf(rho[b], Tp.t[0], fmaf(Tp.d[0], x0, fmaf(Tp.d[1], x1, Tp.d[2])));
                const float Dy = fmaf(rho[b], Tp.t[1], fmaf(Tp.d[3], x0, fmaf(Tp.d[4], x1, Tp.d[5])));
                const float Dz = fmaf(rho[b], Tp.t[2], fmaf(Tp.d[6], x0, fmaf(Tp.d[7], x1, Tp.d[8])));
                const bool zprev = 1.f + Dz > 0.f;
                const float iz = rcp(1.f + Dz);
                const float dpx = w.fx * fmaf(-x0, Dz, Dx) * iz;
                const float dpy = w.fy * fmaf(-x1, Dz, Dy) * iz;
                float fx, fy;
                const bool fok = sample_flow2(flow2_t, w.H, w.W, (float)u + dpx, (float)v + dpy, fx, fy);
                ox[b] = (zprev && fok) ? dpx + fx : __builtin_nanf("");
                oy[b] = (zprev && fok) ? dpy + fy : __builtin_nanf("");
            }
        }
        if (k == 0 && G > 1) {
#pragma unroll
            for (int b = 0; b < UB; ++b) if (jj[b] >= 0) obs[jj[b]] = make_float2(ox[b], oy[b]);
        }
#pragma unroll
        for (int b = 0; b < UB; ++b) {
            if (jj[b] < 0) continue;
            const int v = jj[b] / w.W, u = jj[b] - v * w.W;
            const float x0 = ((float)u - w.cx) * w.ifx, x1 = ((float)v - w.cy) * w.ify;
            const float r = rho[b];
            const float Dx = fmaf(r, Tc.t[0], fmaf(Tc.d[0], x0, fmaf(Tc.d[1], x1, Tc.d[2])));
            const float Dy = fmaf(r, Tc.t[1], fmaf(Tc.d[3], x0, fmaf(Tc.d[4], x1, Tc.d[5])));
            const float Dz = fmaf(r, Tc.t[2], fmaf(Tc.d[6], x0, fmaf(Tc.d[7], x1, Tc.d[8])));
            const float Qx = x0 + Dx, Qy = x1 + Dy, Qz = 1.f + Dz;
            const bool zok = Qz > 0.f;
            const float iz = rcp(Qz);
            const float dx = w.fx * fmaf(-x0, Dz, Dx) * iz, dy = w.fy * fmaf(-x1, Dz, Dy) * iz;
            const bool ok = zok && isfinite(ox[b]) && isfinite(oy[b]) && in_frame(w, (float)u + dx, (float)v + dy);
            const float ex = dx - ox[b], ey = dy - oy[b];
            const float r2 = fmaf(ex, ex, ey * ey);
            if (ok) {
                const float wt = q[b] * flow_dcost<B2>(w, r2);
                const float a = w.fx * iz, bb = -w.fx * Qx * iz * iz;
                const float c = w.fy * iz, d = -w.fy * Qy * iz * iz;
                const float jx[6] = {bb * Qy, a * Qz - bb * Qx, -a * Qy, a * r, 0.f, bb * r};
                const float jy[6] = {d * Qy - c * Qz, -d * Qx, c * Qx, 0.f, c * r, d * r};
                int m = 0;
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    const float wxi = wt * jx[i], wyi = wt * jy[i];
#pragma unroll
                    for (int l = i; l < 6; ++l) { a32[m] = fmaf(wxi, jx[l], fmaf(wyi, jy[l], a32[m])); ++m; }
                    a32[21 + i] = fmaf(wxi, ex, fmaf(wyi, ey, a32[21 + i]));
                }
            }
        }
        j0 += UB * stride;
        if (j0 < plane) load(j0);
    }
    block_sum_transposed<kGnRec, VD_GN_BLOCK>(a32, [&](int v, double sum) {
        B.partials[((size_t)(s & 1) * kGnRec + v) * nb + blk] = sum;
    });
}

template <bool B2>
__global__ void __launch_bounds__(VD_GN_BLOCK) k_pose_gn(Win w, PoseBufs B, int s, int G) {
    pose_gn_body<B2>(w, B, s, G, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
}

// frame i's final pose: the caller's 6-vector, then the FP32 / FP64 tables built from that
// 6-vector with the same function as the pose-table preparation at the start of a step, so
// the next iteration needs no separate preparation
__device__ __forceinline__ void final_pose(const PoseBufs& B, int G, int i) {
    const PoseD P = B.hist[(i + 1) * G - 1];
    double v[6];
    log_so3(P.R, v);
    v[3] = P.t[0];
    v[4] = P.t[1];
    v[5] = P.t[2];
    for (int k = 0; k < 6; ++k) B.pose[6 * i + k] = v[k];
    pose_tables_from_vec(v, B.P + i, B.PD + i);
}

// Step s's solve (one block, the same fixed-order reduction and solve as the prologue of the
// unsplit pass); after the window's last step, every frame's final pose into the FP32 /
// FP64 tables and the caller's 6-vectors.
__device__ __forceinline__ void pose_gn_solve_body(const PoseBufs& B, int N, int G, int s, unsigned nb) {
    __shared__ double red[kGnRec];
    reduce_partials<kGnRec, VD_GN_BLOCK>(B.partials + (size_t)(s & 1) * kGnRec * nb, nb, red);
    const int t = s / G + 1, k = s - (t - 1) * G;
    if (threadIdx.x == 0) {
        PoseD P = k == 0 ? B.PD[t - 1] : B.hist[s - 1];
        pose_gn_solve(red, P);
        B.hist[s] = P;
    }
    if (s < N * G - 1) return;
    __syncthreads();
    if (threadIdx.x < N) final_pose(B, G, threadIdx.x);
}

// Last step's solve, then every frame's final pose into the FP32 / FP64 copies and the
// caller's 6-vectors.
__device__ __forceinline__ void pose_gn_finish_body(const PoseBufs& B, int N, int G, unsigned nb) {
    __shared__ double red[kGnRec];
    const int S = N * G;
    reduce_partials<kGnRec, VD_GN_BLOCK>(B.partials + (size_t)((S - 1) & 1) * kGnRec * nb, nb, red);
    if (threadIdx.x == 0) {
        const int sp = S - 1, tp = sp / G + 1, kp = sp - (tp - 1) * G;
        PoseD P = (kp == 0) ? B.PD[tp - 1] : B.hist[sp - 1];
        pose_gn_solve(red, P);
        B.hist[sp] = P;
    }
    __syncthreads();
    if (threadIdx.x < N) final_pose(B, G, threadIdx.x);
}

__global__ void __launch_bounds__(VD_GN_BLOCK) k_pose_gn_finish(PoseBufs B, int N, int G, unsigned nb) {
    pose_gn_finish_body(B, N, G, nb);
}

// ----------------------------------------------------------------------------------
// final confidence and statistics
// ----------------------------------------------------------------------------------
template <bool B2, bool PR>
__device__ __forceinline__ void finalize_body(const Win& w, const FinalBufs& B, int blk, int nb) {
    __shared__ double red[(VD_BLOCK / 64) * 5];
    const int tid = threadIdx.x;
    const size_t plane = (size_t)w.H * w.W;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // energy, valid, invalid, prior terms, sum C
    const int j = blk * VD_BLOCK + tid;
    if (j < (int)plane) {
        const int v = j / w.W, u = j - v * w.W;
        Pix c;
        pix_geometry<PR>(w, B.P, B.flow, u, v, c);
        float qs = 0.f;
#pragma unroll
        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) { c.q[t] = B.rigid[t * plane + j]; qs += c.q[t]; }
        const float rho = B.idepth[j];
        const int pmask = prior_posteriors<PR>(w, B.P, B.prior, B.prior_weight, j, c, rho);
        const int npr = __popc(pmask);
#pragma unroll
        for (int k = 0; k < VD_PMAX; ++k) if (k < w.P) qs += c.qh[k];
        const float C = qs / (float)(w.N + w.P);
        B.conf[j] = C;
        int nv = 0;
        emissions<B2>(w, B.P, B.flow2, c, rho, [&](int, float, bool ok, float) { nv += ok; });
        acc[0] = energy2<B2, PR>(w, B.P, B.flow2, B.prior, c, rho) * (double)VD_LN2;
        acc[1] = nv;
        acc[2] = w.N - nv;
        acc[3] = npr;
        acc[4] = C;
    }
    block_reduce<5>(acc, red);
    if (tid < 5) B.partials[(size_t)tid * nb + blk] = red[tid];
}

template <bool B2, bool PR>
__global__ void __launch_bounds__(VD_BLOCK) k_finalize(Win w, FinalBufs B) {
    finalize_body<B2, PR>(w, B, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void finalize_finish_body(const FinalBufs& B, unsigned nb, int n_ll) {
    __shared__ double red[(VD_BLOCK / 64) * 5];
    reduce_partials<5>(B.partials, nb, red);
    const double s0 = red[0], s1 = red[1], s2 = red[2], s3 = red[3], s4 = red[4];
    reduce_partials<1>(B.ll_partial, (unsigned)n_ll, red);
    if (threadIdx.x == 0) {
        B.stats[0] = red[0];
        B.stats[1] = s0;
        B.stats[2] = s1;
        B.stats[3] = s2;
        B.stats[4] = s3;
        B.stats[5] = s4;
        B.stats[6] = 0.0;
        B.stats[7] = 0.0;
    }
}

__global__ void __launch_bounds__(VD_BLOCK) k_finalize_finish(FinalBufs B, unsigned nb, int n_ll) {
    finalize_finish_body(B, nb, n_ll);
}

// ----------------------------------------------------------------------------------
// batched kernels: one launch serves many windows
// ----------------------------------------------------------------------------------
// pose tables of every window: one block per window
__global__ void k_prep_batch(const PrepItem* __restrict__ items) {
    const PrepItem& it = items[blockIdx.x];
    pose_prep_body(it.pose, it.N, it.prior_pose, it.P, it.out, it.outd);
}

// initial depth (when asked) and the row-pair flow layout of every window
__global__ void __launch_bounds__(VD_BLOCK) k_setup_batch(const PrepItem* __restrict__ items,
                                                          const int* __restrict__ blk2item) {
    const int gb = xcd_block(blockIdx.x, gridDim.x);
    const PrepItem& it = items[blk2item[gb]];
    const int blk = gb - it.begin;
    if (it.init) init_body(it.w, it.idepth, it.boot, blk);
    flow_pairs_body(it.flow, it.flow2, it.N, it.w.H, it.w.W, blk);
}

// mode 0: fused level pass (do_e / do_m of the item); 1: phase A; 2: phase A2; 3: E-only or
// scan-only pass of the coarse level (long chains)
template <bool B2, bool PR, int MODE>
__global__ void __launch_bounds__(VD_BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
k_level_batch(const LevelItem* __restrict__ items, const int* __restrict__ blk2item) {
    extern __shared__ __align__(16) float lds[];
    const int gb = xcd_block(blockIdx.x, gridDim.x);
    const LevelItem& it = items[blk2item[gb]];
    const int lb = gb - it.begin;
    const int blk = MODE == 0 && it.b.blk_order ? it.b.blk_order[lb] : lb;
    if (MODE == 0) level_body<B2, PR>(it.w, it.g, it.b, it.do_e, it.do_m, blk, lds);
    else if (MODE == 3) level_body<B2, PR, true>(it.w, it.g, it.b, it.do_e, it.do_m, blk, lds);
    else if (MODE == 1) phase_a_body<B2, PR>(it.w, it.g, it.b, blk);
    else phase_a2_body<B2, PR>(it.w, it.g, it.b, blk);
}

// Gauss-Newton step s of every window that has one (windows with fewer steps idle)
template <bool B2>
__global__ void __launch_bounds__(VD_GN_BLOCK) k_pose_gn_batch(const PoseItem* __restrict__ items,
                                                            const int* __restrict__ blk2item, int s) {
    const int gb = xcd_block(blockIdx.x, gridDim.x);
    const PoseItem& it = items[blk2item[gb]];
    if (s >= it.S) return;
    pose_gn_body<B2, true>(it.w, it.b, s, it.G, gb - it.begin, (unsigned)it.nblocks);
}

// step s's solve of every window that has the step, one block per window
__global__ void __launch_bounds__(VD_GN_BLOCK) k_pose_gn_solve_batch(const PoseItem* __restrict__ items, int s) {
    const PoseItem& it = items[blockIdx.x];
    if (s < it.S) pose_gn_solve_body(it.b, it.w.N, it.G, s, (unsigned)it.nblocks);
}

template <bool B2, bool PR>
__global__ void __launch_bounds__(VD_BLOCK) k_finalize_batch(const FinalItem* __restrict__ items,
                                                             const int* __restrict__ blk2item) {
    const int gb = xcd_block(blockIdx.x, gridDim.x);
    const FinalItem& it = items[blk2item[gb]];
    finalize_body<B2, PR>(it.w, it.b, gb - it.begin, it.nblocks);
}

__global__ void __launch_bounds__(VD_BLOCK) k_finalize_finish_batch(const FinalItem* __restrict__ items) {
    const FinalItem& it = items[blockIdx.x];
    finalize_finish_body(it.b, (unsigned)it.nblocks, it.n_ll);
}

}  // namespace vd

// ----------------------------------------------------------------------------------
// host launch wrappers
// ----------------------------------------------------------------------------------
namespace vd {

size_t level_lds_bytes(const LevelGeom& g) {
    const size_t nodes = (size_t)g.C * (g.seg + 1);
    return (1 + (size_t)g.spec) * nodes * sizeof(energy_t) +
           (2 * (size_t)g.nf * nodes + 3 * nodes + (size_t)g.ncost * nodes) * sizeof(float) +
           nodes * sizeof(int);
}

hipError_t set_level_lds_limit(size_t bytes) {
    const void* fns[16] = {(const void*)k_level<false, false, false>, (const void*)k_level<false, true, false>,
                           (const void*)k_level<true, false, false>, (const void*)k_level<true, true, false>,
                           (const void*)k_level<false, false, true>, (const void*)k_level<false, true, true>,
                           (const void*)k_level<true, false, true>, (const void*)k_level<true, true, true>,
                           (const void*)k_level_batch<false, false, 0>, (const void*)k_level_batch<false, true, 0>,
                           (const void*)k_level_batch<true, false, 0>, (const void*)k_level_batch<true, true, 0>,
                           (const void*)k_level_batch<false, false, 3>, (const void*)k_level_batch<false, true, 3>,
                           (const void*)k_level_batch<true, false, 3>, (const void*)k_level_batch<true, true, 3>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pose_prep(const double* pose, int N, const double* prior_pose, int P, PoseF* out, PoseD* outd,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_pose_prep, dim3(1), dim3(64), 0, st, pose, N, prior_pose, P, out, outd);
    return hipGetLastError();
}

hipError_t launch_flow_pairs(const float2* flow, float4* f2, int N, int H, int W, hipStream_t st) {
    if (N < 2) return hipSuccess;
    const size_t n = (size_t)(H - 1) * W * (N - 1);
    hipLaunchKernelGGL(k_flow_pairs, dim3((unsigned)((n + VD_BLOCK - 1) / VD_BLOCK)), dim3(VD_BLOCK), 0, st, flow, f2, N, H, W);
    return hipGetLastError();
}

hipError_t launch_init(const Win& w, float* idepth, InitSrc boot, hipStream_t st) {
    const int n = w.H * w.W;
    hipLaunchKernelGGL(k_init_idepth, dim3((n + VD_BLOCK - 1) / VD_BLOCK), dim3(VD_BLOCK), 0, st, w, idepth, boot);
    return hipGetLastError();
}

hipError_t launch_init_if(const Win& w, float* idepth, InitSrc boot, const int* flag, int32_t* out, hipStream_t st) {
    const int n = w.H * w.W;
    hipLaunchKernelGGL(k_init_idepth_if, dim3((n + VD_BLOCK - 1) / VD_BLOCK), dim3(VD_BLOCK), 0, st, w, idepth, boot,
                       flag, out);
    return hipGetLastError();
}

hipError_t launch_level(const Win& w, const LevelGeom& g, const LevelBufs& b, int do_e, int do_m, hipStream_t st) {
    const size_t lds = level_lds_bytes(g);
    const bool lc = do_m == 2 || (w.level == 0 && do_m == 0);
    if (w.beta2) {
        if (lc) {
            if (w.P > 0) hipLaunchKernelGGL((k_level<true, true, true>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
            else hipLaunchKernelGGL((k_level<true, false, true>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
        } else if (w.P > 0) hipLaunchKernelGGL((k_level<true, true, false>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
        else hipLaunchKernelGGL((k_level<true, false, false>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
    } else {
        if (lc) {
            if (w.P > 0) hipLaunchKernelGGL((k_level<false, true, true>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
            else hipLaunchKernelGGL((k_level<false, false, true>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
        } else if (w.P > 0) hipLaunchKernelGGL((k_level<false, true, false>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
        else hipLaunchKernelGGL((k_level<false, false, false>), dim3(g.nblocks), dim3(VD_BLOCK), lds, st, w, g, b, do_e, do_m);
    }
    return hipGetLastError();
}

template <int LANES>
hipError_t launch_phase_a_lanes(const Win& w, const LevelGeom& g, const LevelBufs& b, hipStream_t st) {
    const dim3 grid((unsigned)(((size_t)g.h * g.w * LANES + VD_BLOCK - 1) / VD_BLOCK));
    if (w.beta2) {
        if (w.P > 0) hipLaunchKernelGGL((k_phase_a<true, true, LANES>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
        else hipLaunchKernelGGL((k_phase_a<true, false, LANES>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
    } else {
        if (w.P > 0) hipLaunchKernelGGL((k_phase_a<false, true, LANES>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
        else hipLaunchKernelGGL((k_phase_a<false, false, LANES>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
    }
    return hipGetLastError();
}

hipError_t launch_phase_a(const Win& w, const LevelGeom& g, const LevelBufs& b, hipStream_t st) {
    if (g.pa_lanes == 4) return launch_phase_a_lanes<4>(w, g, b, st);
    if (g.pa_lanes == 16) return launch_phase_a_lanes<16>(w, g, b, st);
    return launch_phase_a_lanes<8>(w, g, b, st);
}

hipError_t launch_phase_a2(const Win& w, const LevelGeom& g, const LevelBufs& b, hipStream_t st) {
    const dim3 grid((unsigned)(((size_t)g.h * g.w * g.spec + VD_BLOCK - 1) / VD_BLOCK));
    if (w.beta2) {
        if (w.P > 0) hipLaunchKernelGGL((k_phase_a2<true, true>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
        else hipLaunchKernelGGL((k_phase_a2<true, false>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
    } else {
        if (w.P > 0) hipLaunchKernelGGL((k_phase_a2<false, true>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
        else hipLaunchKernelGGL((k_phase_a2<false, false>), grid, dim3(VD_BLOCK), 0, st, w, g, b);
    }
    return hipGetLastError();
}

hipError_t launch_pose_gn(const Win& w, const PoseBufs& b, int s, int G, int nblocks, hipStream_t st) {
    if (w.beta2) hipLaunchKernelGGL((k_pose_gn<true>), dim3(nblocks), dim3(VD_GN_BLOCK), 0, st, w, b, s, G);
    else hipLaunchKernelGGL((k_pose_gn<false>), dim3(nblocks), dim3(VD_GN_BLOCK), 0, st, w, b, s, G);
    return hipGetLastError();
}

hipError_t launch_pose_gn_finish(const PoseBufs& b, int N, int G, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_pose_gn_finish, dim3(1), dim3(VD_GN_BLOCK), 0, st, b, N, G, (unsigned)nblocks);
    return hipGetLastError();
}

hipError_t launch_pose(const Win& w, const PoseBufs& b, int t, const double* cand, int n_cand, int solve,
                       int nblocks, hipStream_t st) {
    if (w.beta2) hipLaunchKernelGGL((k_pose<true>), dim3(nblocks, n_cand), dim3(VD_BLOCK), 0, st, w, b, t, cand);
    else hipLaunchKernelGGL((k_pose<false>), dim3(nblocks, n_cand), dim3(VD_BLOCK), 0, st, w, b, t, cand);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pose_finish, dim3(n_cand), dim3(VD_BLOCK), 0, st, b, t, (unsigned)nblocks, solve);
    return hipGetLastError();
}

hipError_t launch_finalize(const Win& w, const FinalBufs& b, int n_ll, hipStream_t st) {
    const int n = w.H * w.W;
    const dim3 grid((n + VD_BLOCK - 1) / VD_BLOCK);
    if (w.beta2) {
        if (w.P > 0) hipLaunchKernelGGL((k_finalize<true, true>), grid, dim3(VD_BLOCK), 0, st, w, b);
        else hipLaunchKernelGGL((k_finalize<true, false>), grid, dim3(VD_BLOCK), 0, st, w, b);
    } else {
        if (w.P > 0) hipLaunchKernelGGL((k_finalize<false, true>), grid, dim3(VD_BLOCK), 0, st, w, b);
        else hipLaunchKernelGGL((k_finalize<false, false>), grid, dim3(VD_BLOCK), 0, st, w, b);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize_finish, dim3(1), dim3(VD_BLOCK), 0, st, b, grid.x, n_ll);
    return hipGetLastError();
}

hipError_t launch_prep_batch(const PrepItem* items, int n_items, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_batch, dim3((unsigned)n_items), dim3(64), 0, st, items);
    return hipGetLastError();
}

hipError_t launch_setup_batch(const PrepItem* items, const int* blk2item, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_setup_batch, dim3((unsigned)nblocks), dim3(VD_BLOCK), 0, st, items, blk2item);
    return hipGetLastError();
}

template <int MODE>
static void level_batch_mode(const LevelItem* items, const int* b2i, int nb, size_t lds, bool b2, bool pr,
                             hipStream_t st) {
    if (b2) {
        if (pr) hipLaunchKernelGGL((k_level_batch<true, true, MODE>), dim3(nb), dim3(VD_BLOCK), lds, st, items, b2i);
        else hipLaunchKernelGGL((k_level_batch<true, false, MODE>), dim3(nb), dim3(VD_BLOCK), lds, st, items, b2i);
    } else {
        if (pr) hipLaunchKernelGGL((k_level_batch<false, true, MODE>), dim3(nb), dim3(VD_BLOCK), lds, st, items, b2i);
        else hipLaunchKernelGGL((k_level_batch<false, false, MODE>), dim3(nb), dim3(VD_BLOCK), lds, st, items, b2i);
    }
}

hipError_t launch_level_batch(const LevelItem* items, const int* blk2item, int nblocks, size_t lds, int mode,
                              bool b2, bool pr, hipStream_t st) {
    if (mode == 0) level_batch_mode<0>(items, blk2item, nblocks, lds, b2, pr, st);
    else if (mode == 3) level_batch_mode<3>(items, blk2item, nblocks, lds, b2, pr, st);
    else if (mode == 1) level_batch_mode<1>(items, blk2item, nblocks, 0, b2, pr, st);
    else level_batch_mode<2>(items, blk2item, nblocks, 0, b2, pr, st);
    return hipGetLastError();
}

hipError_t launch_pose_gn_batch(const PoseItem* items, const int* blk2item, int nblocks, int s, bool b2,
                                hipStream_t st) {
    if (b2) hipLaunchKernelGGL((k_pose_gn_batch<true>), dim3(nblocks), dim3(VD_GN_BLOCK), 0, st, items, blk2item, s);
    else hipLaunchKernelGGL((k_pose_gn_batch<false>), dim3(nblocks), dim3(VD_GN_BLOCK), 0, st, items, blk2item, s);
    return hipGetLastError();
}

hipError_t launch_pose_gn_solve_batch(const PoseItem* items, int n_items, int s, hipStream_t st) {
    hipLaunchKernelGGL(k_pose_gn_solve_batch, dim3((unsigned)n_items), dim3(VD_GN_BLOCK), 0, st, items, s);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const FinalItem* items, const int* blk2item, int nblocks, bool b2, bool pr,
                                 hipStream_t st) {
    if (b2) {
        if (pr) hipLaunchKernelGGL((k_finalize_batch<true, true>), dim3(nblocks), dim3(VD_BLOCK), 0, st, items, blk2item);
        else hipLaunchKernelGGL((k_finalize_batch<true, false>), dim3(nblocks), dim3(VD_BLOCK), 0, st, items, blk2item);
    } else {
        if (pr) hipLaunchKernelGGL((k_finalize_batch<false, true>), dim3(nblocks), dim3(VD_BLOCK), 0, st, items, blk2item);
        else hipLaunchKernelGGL((k_finalize_batch<false, false>), dim3(nblocks), dim3(VD_BLOCK), 0, st, items, blk2item);
    }
    return hipGetLastError();
}

hipError_t launch_finalize_finish_batch(const FinalItem* items, int n_items, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_finish_batch, dim3((unsigned)n_items), dim3(VD_BLOCK), 0, st, items);
    return hipGetLastError();
}

}  // namespace vd
