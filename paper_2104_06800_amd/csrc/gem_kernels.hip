// GEM kernels for gfx950: initial depth, per-level fused E-step / M-step on the alternately
// directed 1D chains, pose normal equations with an on-device FP64 solve, and the final
// confidence / statistics pass (VOLDOR+SLAM sec. III-A, Eqs. 1-6).
#include "device.h"
#include "kernels.h"

namespace vd {

// ----------------------------------------------------------------------------------
// pose conversion (FP64 6-vectors -> FP32 R|t for frames and priors)
// ----------------------------------------------------------------------------------
__global__ void k_pose_prep(const double* __restrict__ pose, int N, const double* __restrict__ prior_pose, int P,
                            PoseF* __restrict__ out) {
    const int i = threadIdx.x;
    if (i < N) pose_to_f(pose + 6 * i, out + i);
    else if (i < N + P) pose_to_f(prior_pose + 6 * (i - N), out + i);
}

// ----------------------------------------------------------------------------------
// random initial inverse depth
// ----------------------------------------------------------------------------------
__global__ void k_init_idepth(Win w, float* __restrict__ idepth) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= w.H * w.W) return;
    const uint4 r = philox10(make_uint4((uint32_t)j, 0u, philox_word2(0, 1, PURPOSE_INIT), w.window_id),
                             w.key0, w.key1);
    idepth[j] = fmaf(unit24(r.x), w.rmax - w.rmin, w.rmin);
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

__device__ __forceinline__ BlockPix block_pix(const LevelGeom& g, int k) {
    BlockPix p;
    const int b = blockIdx.x;
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
__device__ __forceinline__ int chain_len(const LevelGeom& g, int c) {
    const int b = blockIdx.x;
    const int sidx = b % g.nseg, lb = b / g.nseg;
    const int line = lb * g.C + c;
    const int nlines = g.horizontal ? g.h : g.w;
    const int axis = g.horizontal ? g.w : g.h;
    if (line >= nlines) return 0;
    return min(g.seg, axis - sidx * g.seg);
}

__global__ void __launch_bounds__(VD_BLOCK)
k_level(Win w, LevelGeom g, LevelBufs B, int do_e, int do_m) {
    extern __shared__ float lds[];
    const int stride = g.seg + 1;
    const int nodes = g.C * stride;
    float* q_s = lds;                       // [N][C][stride] emission ratios -> alpha -> q
    float* r_s = q_s + VD_NMAX * nodes;     // [N][C][stride] emission ratios (E-step)
    float* bestE = r_s + VD_NMAX * nodes;   // [C][stride]
    float* bestV = bestE + nodes;
    float* specE = bestV + nodes;
    float* rcur = specE + nodes;
    float* newV = rcur + nodes;
    int* bestS = (int*)(newV + nodes);
    __shared__ double ll_red[VD_BLOCK / 64];

    const int tid = threadIdx.x;
    const int npix = g.C * g.seg;
    const size_t lplane = (size_t)g.h * g.w;       // level plane
    const float* rho_full = B.idepth;
    double ll = 0.0;

    // -------------------------------- E-step ------------------------------------
    if (do_e) {
        for (int k = tid; k < npix; k += VD_BLOCK) {
            const BlockPix p = block_pix(g, k);
            if (!p.valid) continue;
            Pix c;
            pix_geometry(w, B.P, B.flow, p.u, p.v, c);
            const float rho = rho_full[p.v * w.W + p.u];
            const int o = p.c * stride + p.i;
            if (w.chain_axis == 0) {
                emissions(w, B.P, B.flow, c, rho, [&](int t, float ratio, bool) { r_s[t * nodes + o] = ratio; });
            } else {
                // temporal chain over the frame window, in registers
                float rr[VD_NMAX], al[VD_NMAX];
                emissions(w, B.P, B.flow, c, rho, [&](int t, float ratio, bool) { rr[t] = ratio; });
                float logc = 0.f;
                float a1 = 0.f;
#pragma unroll
                for (int t = 0; t < VD_NMAX; ++t) {
                    if (t < w.N) {
                        const float p1 = (t == 0) ? 0.5f : fmaf(2.f * w.gamma - 1.f, a1, 1.f - w.gamma);
                        const float x1 = p1 * rr[t];
                        const float cc = (1.f - p1) + x1;
                        a1 = x1 / cc;
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
                            b1 = y1 / (y0 + y1);
                        }
                        const float num = al[t] * b1;
                        q_s[t * nodes + o] = num / fmaf(1.f - al[t], 1.f - b1, num);
                    }
                }
                ll += (double)(logc * VD_LN2) + (double)w.N * (double)w.ln_L0;
            }
        }
        __syncthreads();
        if (w.chain_axis == 0 && tid < g.C * w.N) {
            const int c = tid % g.C, t = tid / g.C;
            const int L = chain_len(g, c);
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
                    a1 = x1 / cc;
                    a[i] = a1;
                    logc += log2f_fast(cc);
                }
                float b1 = 0.5f;
                for (int i = L - 1; i >= 0; --i) {
                    if (i < L - 1) {
                        const float m0 = 1.f - b1, m1 = r[i + 1] * b1;
                        const float y1 = fmaf(gm, m1, (1.f - gm) * m0);
                        const float y0 = fmaf(gm, m0, (1.f - gm) * m1);
                        b1 = y1 / (y0 + y1);
                    }
                    const float ai = a[i];
                    const float num = ai * b1;
                    a[i] = num / fmaf(1.f - ai, 1.f - b1, num);
                }
                ll += (double)(logc * VD_LN2) + (double)L * (double)w.ln_L0;
            }
        }
        __syncthreads();
        // posteriors out (coalesced along the level grid rows)
        for (int k = tid; k < npix; k += VD_BLOCK) {
            const BlockPix p = block_pix(g, k);
            if (!p.valid) continue;
            const int o = p.c * stride + p.i;
            for (int t = 0; t < w.N; ++t) B.q_out[t * lplane + p.li] = q_s[t * nodes + o];
        }
        if (B.ll_partial) {
            // block sum of chain log-likelihoods, fixed order
            for (int off = 32; off > 0; off >>= 1) ll += __shfl_xor(ll, off);
            if ((tid & 63) == 0) ll_red[tid >> 6] = ll;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int i = 0; i < VD_BLOCK / 64; ++i) s += ll_red[i];
                B.ll_partial[blockIdx.x] = s;
            }
        }
    }
    if (!do_m) return;

    // -------------------------------- M-step ------------------------------------
    if (!do_e) {
        for (int k = tid; k < npix; k += VD_BLOCK) {
            const BlockPix p = block_pix(g, k);
            if (!p.valid) continue;
            const int o = p.c * stride + p.i;
            for (int t = 0; t < w.N; ++t) q_s[t * nodes + o] = B.q_in[t * lplane + p.li];
        }
        __syncthreads();
    }
    const int G = (w.K - 3 + 3) / 4;
    const uint32_t word2 = philox_word2(w.it, w.level, PURPOSE_CAND);
    const bool local = (w.level == 1);

    // phase A: parallel over pixels and slots {0, 2, 3..K-1}
    for (int k = tid; k < npix; k += VD_BLOCK) {
        const BlockPix p = block_pix(g, k);
        if (!p.valid) continue;
        const int o = p.c * stride + p.i;
        Pix c;
        pix_geometry(w, B.P, B.flow, p.u, p.v, c);
#pragma unroll
        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) c.q[t] = q_s[t * nodes + o];
        const int fpix = p.v * w.W + p.u;
        const float r0 = rho_full[fpix];
        prior_posteriors(w, B.P, B.prior, B.prior_weight, fpix, c, r0);
        float bE = energy2(w, B.P, B.flow, B.prior, c, r0), bV = r0;
        int bS = 0;
        if (local) {
            const int U = min(p.u / w.s, w.wc - 1), V = min(p.v / w.s, w.hc - 1);
            const float rc = B.idepth_coarse[V * w.wc + U];
            const float e = energy2(w, B.P, B.flow, B.prior, c, rc);
            if (e < bE) { bE = e; bV = rc; bS = 2; }
        }
        for (int gi = 0; gi < G; ++gi) {
            const uint4 r = philox10(make_uint4((uint32_t)p.li, (uint32_t)gi, word2, w.window_id), w.key0, w.key1);
            const uint32_t words[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int slot = 3 + 4 * gi + m;
                if (slot < w.K) {
                    const float uu = unit24(words[m]);
                    const float cand = (slot & 1)
                        ? fminf(fmaxf(r0 * fmaf(w.sigma_it, fmaf(2.f, uu, -1.f), 1.f), w.rmin), w.rmax)
                        : fmaf(uu, w.rmax - w.rmin, w.rmin);
                    const float e = energy2(w, B.P, B.flow, B.prior, c, cand);
                    if (e < bE) { bE = e; bV = cand; bS = slot; }
                }
            }
        }
        bestE[o] = bE; bestV[o] = bV; bestS[o] = bS; rcur[o] = r0;
    }
    __syncthreads();

    // phase A2: energy at the predecessor's phase-A winner
    const bool fwd = (w.dir < 2);
    for (int k = tid; k < npix; k += VD_BLOCK) {
        const BlockPix p = block_pix(g, k);
        if (!p.valid) continue;
        const int L = chain_len(g, p.c);
        const int ip = fwd ? p.i - 1 : p.i + 1;
        if (ip < 0 || ip >= L) continue;
        const int o = p.c * stride + p.i;
        Pix c;
        pix_geometry(w, B.P, B.flow, p.u, p.v, c);
#pragma unroll
        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) c.q[t] = q_s[t * nodes + o];
        prior_posteriors(w, B.P, B.prior, B.prior_weight, p.v * w.W + p.u, c, rcur[o]);
        specE[o] = energy2(w, B.P, B.flow, B.prior, c, bestV[p.c * stride + ip]);
    }
    __syncthreads();

    // phase B: serial scan per chain
    if (tid < g.C) {
        const int c = tid;
        const int L = chain_len(g, c);
        if (L > 0) {
            const int i0 = fwd ? 0 : L - 1, di = fwd ? 1 : -1;
            const int base = c * stride;
            float carried = bestV[base + i0];
            int src = i0;
            newV[base + i0] = carried;
            for (int n = 1, i = i0 + di; n < L; ++n, i += di) {
                const int o = base + i;
                float e1;
                if (src == i - di) {
                    e1 = specE[o];
                } else {
                    // storage-order node i of chain c -> block linear index
                    const int kk = g.horizontal ? (c * g.seg + i) : (i * g.C + c);
                    const BlockPix p = block_pix(g, kk);
                    Pix cx;
                    pix_geometry(w, B.P, B.flow, p.u, p.v, cx);
#pragma unroll
                    for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) cx.q[t] = q_s[t * nodes + o];
                    prior_posteriors(w, B.P, B.prior, B.prior_weight, p.v * w.W + p.u, cx, rcur[o]);
                    e1 = energy2(w, B.P, B.flow, B.prior, cx, carried);
                }
                const float eA = bestE[o];
                const bool keep = (e1 < eA) || (e1 == eA && bestS[o] > 1);
                if (!keep) { carried = bestV[o]; src = i; }
                newV[o] = carried;
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < npix; k += VD_BLOCK) {
        const BlockPix p = block_pix(g, k);
        if (!p.valid) continue;
        B.rho_out[local ? (p.v * w.W + p.u) : p.li] = newV[p.c * stride + p.i];
    }
}

// ----------------------------------------------------------------------------------
// pose normal equations for frame t at candidate poses; optional FP64 solve + update
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(VD_BLOCK)
k_pose(Win w, PoseBufs B, int t, const double* __restrict__ cand, int solve) {
    __shared__ double red[(VD_BLOCK / 64) * 29];
    __shared__ PoseF candF;
    __shared__ int flag;
    const int tid = threadIdx.x;
    const int ci = blockIdx.y;
    if (tid == 0) {
        if (cand) pose_to_f(cand + 6 * ci, &candF);
        else candF = B.P[t - 1];
    }
    __syncthreads();
    const PoseF Tc = candF;
    const size_t plane = (size_t)w.H * w.W;
    const float2* flow_t = B.flow + (t - 1) * plane;
    double acc[29];
#pragma unroll
    for (int k = 0; k < 29; ++k) acc[k] = 0.0;
    for (int j = blockIdx.x * VD_BLOCK + tid; j < (int)plane; j += gridDim.x * VD_BLOCK) {
        const int v = j / w.W, u = j - v * w.W;
        const float rho = B.idepth[j];
        const float q = B.rigid[(t - 1) * plane + j];
        const float x0 = ((float)u - w.cx) * w.ifx, x1 = ((float)v - w.cy) * w.ify;
        float ppx, ppy, fx, fy;
        bool zprev = true, fok;
        if (t == 1) {
            ppx = (float)u; ppy = (float)v;
            const float2 f = flow_t[j];
            fx = f.x; fy = f.y;
            fok = isfinite(fx) && isfinite(fy);
        } else {
            const PoseF& Tp = B.P[t - 2];
            const float Qx = fmaf(rho, Tp.t[0], fmaf(Tp.r[0], x0, fmaf(Tp.r[1], x1, Tp.r[2])));
            const float Qy = fmaf(rho, Tp.t[1], fmaf(Tp.r[3], x0, fmaf(Tp.r[4], x1, Tp.r[5])));
            const float Qz = fmaf(rho, Tp.t[2], fmaf(Tp.r[6], x0, fmaf(Tp.r[7], x1, Tp.r[8])));
            zprev = Qz > 0.f;
            const float iz = rcp(Qz);
            ppx = fmaf(w.fx, Qx * iz, w.cx);
            ppy = fmaf(w.fy, Qy * iz, w.cy);
            fok = sample_flow(flow_t, w.H, w.W, ppx, ppy, fx, fy);
        }
        const float ox = ppx + fx, oy = ppy + fy;
        const float Qx = fmaf(rho, Tc.t[0], fmaf(Tc.r[0], x0, fmaf(Tc.r[1], x1, Tc.r[2])));
        const float Qy = fmaf(rho, Tc.t[1], fmaf(Tc.r[3], x0, fmaf(Tc.r[4], x1, Tc.r[5])));
        const float Qz = fmaf(rho, Tc.t[2], fmaf(Tc.r[6], x0, fmaf(Tc.r[7], x1, Tc.r[8])));
        const bool zok = Qz > 0.f;
        const float iz = rcp(Qz);
        const float px = fmaf(w.fx, Qx * iz, w.cx), py = fmaf(w.fy, Qy * iz, w.cy);
        const bool ok = zprev && zok && fok;
        const float ex = px - ox, ey = py - oy;
        const float r2 = fmaf(ex, ex, ey * ey);
        acc[0] += (double)(q * (ok ? flow_cost2(w, r2) : 1.0f) * VD_LN2);
        if (ok) {
            const float wt = q * flow_dcost(w, r2);
            // J rows of p = pi(Q), Q = R x~ + rho t, left update (dw, dv): dQ = [-[Q]x | rho I]
            const float a = w.fx * iz, b = -w.fx * Qx * iz * iz;
            const float c = w.fy * iz, d = -w.fy * Qy * iz * iz;
            const float jx[6] = {b * Qy, a * Qz - b * Qx, -a * Qy, a * rho, 0.f, b * rho};
            const float jy[6] = {d * Qy - c * Qz, -d * Qx, c * Qx, 0.f, c * rho, d * rho};
            int k = 1;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
#pragma unroll
                for (int l = i; l < 6; ++l) {
                    acc[k++] += (double)(wt * fmaf(jx[i], jx[l], jy[i] * jy[l]));
                }
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) acc[22 + i] += (double)(wt * fmaf(jx[i], ex, jy[i] * ey));
            acc[28] += 1.0;
        }
    }
    block_reduce<29>(acc, red);
    double* part = B.partials + ((size_t)ci * gridDim.x + blockIdx.x) * 29;
    if (tid < 29) part[tid] = red[tid];
    if (!last_block(B.counters + ci, gridDim.x, &flag)) return;
    if (tid < 29) {
        const double* pc = B.partials + (size_t)ci * gridDim.x * 29;
        double s = 0.0;
        for (unsigned bi = 0; bi < gridDim.x; ++bi) s += __builtin_nontemporal_load(pc + (size_t)bi * 29 + tid);
        red[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        B.counters[ci] = 0u;
        if (B.out) for (int k = 0; k < 29; ++k) B.out[ci * 29 + k] = red[k];
        if (solve) {
            double H[36], gv[6], x[6];
            int k = 1;
            for (int i = 0; i < 6; ++i)
                for (int l = i; l < 6; ++l) { H[6 * i + l] = H[6 * l + i] = red[k++]; }
            double tr = 0.0;
            for (int i = 0; i < 6; ++i) { gv[i] = -red[22 + i]; tr += H[7 * i]; }
            const double lam = 1e-9 * tr / 6.0;
            for (int i = 0; i < 6; ++i) H[7 * i] += lam;
            if (chol6_solve(H, gv, x)) {
                double* p = B.pose + 6 * (t - 1);
                left_update(p, x);
                pose_to_f(p, B.P + (t - 1));
            }
        }
    }
}

// ----------------------------------------------------------------------------------
// final confidence and statistics
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(VD_BLOCK)
k_finalize(Win w, FinalBufs B, int n_ll) {
    __shared__ double red[(VD_BLOCK / 64) * 5];
    __shared__ int flag;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)w.H * w.W;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // energy, valid, invalid, prior terms, sum C
    const int j = blockIdx.x * VD_BLOCK + tid;
    if (j < (int)plane) {
        const int v = j / w.W, u = j - v * w.W;
        Pix c;
        pix_geometry(w, B.P, B.flow, u, v, c);
        float qs = 0.f;
#pragma unroll
        for (int t = 0; t < VD_NMAX; ++t) if (t < w.N) { c.q[t] = B.rigid[t * plane + j]; qs += c.q[t]; }
        const float rho = B.idepth[j];
        prior_posteriors(w, B.P, B.prior, B.prior_weight, j, c, rho);
        int npr = 0;
#pragma unroll
        for (int k = 0; k < VD_PMAX; ++k) if (k < w.P) { qs += c.qh[k]; npr += c.qh[k] > 0.f; }
        const float C = qs / (float)(w.N + w.P);
        B.conf[j] = C;
        int nv = 0;
        emissions(w, B.P, B.flow, c, rho, [&](int, float, bool ok) { nv += ok; });
        acc[0] = (double)energy2(w, B.P, B.flow, B.prior, c, rho) * (double)VD_LN2;
        acc[1] = nv;
        acc[2] = w.N - nv;
        acc[3] = npr;
        acc[4] = C;
    }
    block_reduce<5>(acc, red);
    if (tid < 5) B.partials[(size_t)blockIdx.x * 5 + tid] = red[tid];
    if (!last_block(B.counter, gridDim.x, &flag)) return;
    if (tid < 5) {
        double s = 0.0;
        for (unsigned bi = 0; bi < gridDim.x; ++bi) s += __builtin_nontemporal_load(B.partials + (size_t)bi * 5 + tid);
        red[tid] = s;
    }
    if (tid == 5) {
        double s = 0.0;
        for (int bi = 0; bi < n_ll; ++bi) s += __builtin_nontemporal_load(B.ll_partial + bi);
        red[5] = s;
    }
    __syncthreads();
    if (tid == 0) {
        *B.counter = 0u;
        B.stats[0] = red[5];
        B.stats[1] = red[0];
        B.stats[2] = red[1];
        B.stats[3] = red[2];
        B.stats[4] = red[3];
        B.stats[5] = red[4];
        B.stats[6] = 0.0;
        B.stats[7] = 0.0;
    }
}

}  // namespace vd

// ----------------------------------------------------------------------------------
// host launch wrappers
// ----------------------------------------------------------------------------------
namespace vd {

size_t level_lds_bytes(const LevelGeom& g) {
    const size_t nodes = (size_t)g.C * (g.seg + 1);
    return (2 * VD_NMAX * nodes + 5 * nodes) * sizeof(float) + nodes * sizeof(int);
}

hipError_t set_level_lds_limit(size_t bytes) {
    return hipFuncSetAttribute((const void*)k_level, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_pose_prep(const double* pose, int N, const double* prior_pose, int P, PoseF* out, hipStream_t st) {
    hipLaunchKernelGGL(k_pose_prep, dim3(1), dim3(64), 0, st, pose, N, prior_pose, P, out);
    return hipGetLastError();
}

hipError_t launch_init(const Win& w, float* idepth, hipStream_t st) {
    const int n = w.H * w.W;
    hipLaunchKernelGGL(k_init_idepth, dim3((n + VD_BLOCK - 1) / VD_BLOCK), dim3(VD_BLOCK), 0, st, w, idepth);
    return hipGetLastError();
}

hipError_t launch_level(const Win& w, const LevelGeom& g, const LevelBufs& b, int do_e, int do_m, hipStream_t st) {
    hipLaunchKernelGGL(k_level, dim3(g.nblocks), dim3(VD_BLOCK), level_lds_bytes(g), st, w, g, b, do_e, do_m);
    return hipGetLastError();
}

hipError_t launch_pose(const Win& w, const PoseBufs& b, int t, const double* cand, int n_cand, int solve,
                       int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_pose, dim3(nblocks, n_cand), dim3(VD_BLOCK), 0, st, w, b, t, cand, solve);
    return hipGetLastError();
}

hipError_t launch_finalize(const Win& w, const FinalBufs& b, int n_ll, hipStream_t st) {
    const int n = w.H * w.W;
    hipLaunchKernelGGL(k_finalize, dim3((n + VD_BLOCK - 1) / VD_BLOCK), dim3(VD_BLOCK), 0, st, w, b, n_ll);
    return hipGetLastError();
}

}  // namespace vd
