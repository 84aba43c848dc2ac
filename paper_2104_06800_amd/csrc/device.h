// Device-side building blocks of the gfx950 GEM kernels: window constants, Philox draws,
// pose conversion, bilinear flow sampling and the per-pixel maximum-inlier energy.
//
// Precision: per-pixel likelihoods, reprojection and energies in FP32 (energies kept in
// log2 units inside the kernels; the argmin is scale invariant); pose algebra, normal
// equations and their reductions in FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define VD_NMAX 8
#define VD_PMAX 4
#define VD_BLOCK 256
#define VD_LN2 0.69314718055994530942f
#define VD_LOG2E 1.44269504088896340736f

namespace vd {

// ----------------------------------------------------------------------------------
// constants of one launch
// ----------------------------------------------------------------------------------
struct PoseF {          // rotation (row-major) and translation, FP32 copy of a 6-vector
    float r[9];
    float t[3];
    int ident;          // the 6-vector is exactly zero (identity transfer)
    int pad[3];
};

struct Win {
    int H, W, N, P;
    float fx, fy, cx, cy, ifx, ify;
    float inv_a2;        // 1 / alpha^2
    float fl_c;          // shape 2: c = L0 pi alpha^2; other shapes: log2(L0 2 pi alpha^2 / beta)
    float beta;
    int beta2;           // shape == 2 (fast path)
    float zfloor;        // shape < 2: floor of r / alpha
    float ln_L0;         // natural log of L0 (log-likelihood in px^-2 densities)
    float gamma;
    float rmin, rmax;
    float sigma_it;      // relative perturbation width of this iteration
    float csig;          // prior sigma relative to rho^
    float log2kappa;     // log2(sqrt(2 pi) csig / cu)
    float pi_default;
    int K;               // candidate slots
    int s, hc, wc;       // coarse stride and lattice shape
    int it, level, dir;  // iteration, level, direction (0 right, 1 down, 2 left, 3 up)
    int chain_axis;
    uint32_t key0, key1, window_id;
    int has_prior_weight;
};

// ----------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 multiplies
// ----------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ float unit24(uint32_t x) {          // exact (x >> 8) / 2^24
    return (float)(x >> 8) * (1.0f / 16777216.0f);
}

enum { PURPOSE_INIT = 0, PURPOSE_CAND = 1 };

__device__ __forceinline__ uint32_t philox_word2(int it, int level, int purpose) {
    return ((uint32_t)it << 8) | ((uint32_t)level << 4) | (uint32_t)purpose;
}

// ----------------------------------------------------------------------------------
// FP64 rotation algebra (pose solve and conversion)
// ----------------------------------------------------------------------------------
__device__ inline void exp_so3(const double w[3], double R[9]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double a, b;
    if (th2 < 1e-8) {
        a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    } else {
        const double th = sqrt(th2);
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
    }
    // R = I + a K + b K^2, K = [w]x, K^2 = w w^T - th2 I
    R[0] = 1.0 + b * (w[0] * w[0] - th2);
    R[4] = 1.0 + b * (w[1] * w[1] - th2);
    R[8] = 1.0 + b * (w[2] * w[2] - th2);
    R[1] = -a * w[2] + b * w[0] * w[1];
    R[3] = a * w[2] + b * w[0] * w[1];
    R[2] = a * w[1] + b * w[0] * w[2];
    R[6] = -a * w[1] + b * w[0] * w[2];
    R[5] = -a * w[0] + b * w[1] * w[2];
    R[7] = a * w[0] + b * w[1] * w[2];
}

__device__ inline void log_so3(const double R[9], double w[3]) {
    const double v0 = R[7] - R[5], v1 = R[2] - R[6], v2 = R[3] - R[1];   // 2 sin(th) axis
    const double s = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const double c = R[0] + R[4] + R[8] - 1.0;                            // 2 cos(th)
    const double th = atan2(s, c);
    if (c > -1.9) {
        const double f = (th < 1e-4) ? (0.5 + th * th / 12.0) : th / s;
        w[0] = f * v0; w[1] = f * v1; w[2] = f * v2;
        return;
    }
    // near pi: symmetric part gives the axis
    const double ct = cos(th), d = 1.0 - ct;
    double B[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            B[3 * i + j] = (0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? ct : 0.0)) / d;
    int k = 0;
    if (B[4] > B[3 * k + k]) k = 1;
    if (B[8] > B[3 * k + k]) k = 2;
    const double n = sqrt(B[3 * k + k]);
    double a0 = B[0 * 3 + k] / n, a1 = B[1 * 3 + k] / n, a2 = B[2 * 3 + k] / n;
    if (a0 * v0 + a1 * v1 + a2 * v2 < 0) { a0 = -a0; a1 = -a1; a2 = -a2; }
    w[0] = a0 * th; w[1] = a1 * th; w[2] = a2 * th;
}

__device__ inline void pose_to_f(const double* p, PoseF* out) {
    double R[9];
    exp_so3(p, R);
    for (int i = 0; i < 9; ++i) out->r[i] = (float)R[i];
    for (int i = 0; i < 3; ++i) out->t[i] = (float)p[3 + i];
    out->ident = (p[0] == 0.0 && p[1] == 0.0 && p[2] == 0.0 && p[3] == 0.0 && p[4] == 0.0 && p[5] == 0.0);
}

// p <- (exp([dw]x) R, exp([dw]x) t + dv)
__device__ inline void left_update(double* p, const double* d) {
    double R[9], E[9], R2[9];
    exp_so3(p, R);
    exp_so3(d, E);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            R2[3 * i + j] = E[3 * i + 0] * R[0 + j] + E[3 * i + 1] * R[3 + j] + E[3 * i + 2] * R[6 + j];
    double t2[3];
    for (int i = 0; i < 3; ++i)
        t2[i] = E[3 * i + 0] * p[3] + E[3 * i + 1] * p[4] + E[3 * i + 2] * p[5] + d[3 + i];
    log_so3(R2, p);
    p[3] = t2[0]; p[4] = t2[1]; p[5] = t2[2];
}

// Solve A x = b (6x6 SPD, row-major) by Cholesky; false when a pivot is not finite or not
// above 1e-12 times the largest diagonal entry.
__device__ inline bool chol6_solve(const double* A, const double* b, double* x) {
    double L[36];
    double dmax = 0.0;
    for (int i = 0; i < 6; ++i) dmax = fmax(dmax, A[7 * i]);
    const double tol = 1e-12 * dmax;
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[6 * i + j];
            for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
            if (i == j) {
                if (!(s > tol) || !isfinite(s)) return false;
                L[6 * i + i] = sqrt(s);
            } else {
                L[6 * i + j] = s / L[6 * j + j];
            }
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
        y[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * x[k];
        x[i] = s / L[6 * i + i];
    }
    return true;
}

// ----------------------------------------------------------------------------------
// fast FP32 transcendentals (v_rcp_f32, v_log_f32 = log2, v_exp_f32 = 2^x)
// ----------------------------------------------------------------------------------
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float log2f_fast(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float exp2f_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// log2(1 + 2^y)
__device__ __forceinline__ float softplus2(float y) {
    return y > 24.f ? y : log2f_fast(1.f + exp2f_fast(y));
}

// log2(L0 / L1(r)) of the log-logistic planar density, r^2 given
__device__ __forceinline__ float log2_ratio(const Win& w, float r2) {
    if (w.beta2) {
        const float s = fmaf(r2, w.inv_a2, 1.f);
        return log2f_fast(w.fl_c * s * s);
    }
    const float z2 = fmaxf(r2 * w.inv_a2, w.zfloor * w.zfloor);
    const float lz = 0.5f * log2f_fast(z2);                            // log2(r/alpha)
    const float y = exp2f_fast(w.beta * lz);                           // (r/alpha)^beta
    return w.fl_c + 2.f * log2f_fast(1.f + y) + (2.f - w.beta) * lz;
}

// MIE cost of a valid flow term, log2(1 + L0/L1), in log2 units
__device__ __forceinline__ float flow_cost2(const Win& w, float r2) {
    if (w.beta2) {
        const float s = fmaf(r2, w.inv_a2, 1.f);
        return log2f_fast(fmaf(w.fl_c * s, s, 1.f));
    }
    return softplus2(log2_ratio(w, r2));
}

// d cost / d r^2 in natural-log units (IRLS weight without q)
__device__ __forceinline__ float flow_dcost(const Win& w, float r2) {
    if (w.beta2) {
        const float s = fmaf(r2, w.inv_a2, 1.f);
        const float cs = w.fl_c * s;
        return 2.f * cs * w.inv_a2 / fmaf(cs, s, 1.f);
    }
    const float z2 = fmaxf(r2 * w.inv_a2, w.zfloor * w.zfloor);
    const float x = z2 / w.inv_a2;                                     // floored r^2
    const float lz = 0.5f * log2f_fast(z2);
    const float y = exp2f_fast(w.beta * lz);
    const float dlog = w.beta * w.inv_a2 * exp2f_fast((w.beta - 2.f) * lz) / (1.f + y)
                     + (2.f - w.beta) / (2.f * x);
    const float g = exp2f_fast(log2_ratio(w, r2));
    return g / (1.f + g) * dlog;
}

// ----------------------------------------------------------------------------------
// bilinear flow sample on [0, W-1] x [0, H-1]; invalid outside or on non-finite taps
// ----------------------------------------------------------------------------------
__device__ __forceinline__ bool sample_flow(const float2* __restrict__ F, int H, int W, float x, float y,
                                            float& fx, float& fy) {
    const bool inside = (x >= 0.f) && (x <= (float)(W - 1)) && (y >= 0.f) && (y <= (float)(H - 1));
    const float xs = inside ? x : 0.f, ys = inside ? y : 0.f;
    const int x0 = (int)xs, y0 = (int)ys;
    const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
    const float ax = xs - (float)x0, ay = ys - (float)y0;
    const float2 a = F[y0 * W + x0], b = F[y0 * W + x1];
    const float2 c = F[y1 * W + x0], d = F[y1 * W + x1];
    const float tx = fmaf(ax, b.x - a.x, a.x), ty = fmaf(ax, b.y - a.y, a.y);
    const float bx = fmaf(ax, d.x - c.x, c.x), by = fmaf(ax, d.y - c.y, c.y);
    fx = fmaf(ay, bx - tx, tx);
    fy = fmaf(ay, by - ty, ty);
    return inside && isfinite(fx) && isfinite(fy);
}

// ----------------------------------------------------------------------------------
// per-pixel context of the energy E_j(rho) and its evaluation
// ----------------------------------------------------------------------------------
struct Pix {
    float u, v;
    float ax[VD_NMAX], ay[VD_NMAX], az[VD_NMAX];   // R_t x~
    float q[VD_NMAX];                              // rigidness posteriors
    float o1x, o1y;                                // first observation j + X_1(j)
    bool ok1;
    float qh[VD_PMAX];                             // prior posteriors at the current value
    float rh[VD_PMAX];                             // identity-pose priors: rho^ at the pixel
    float px[VD_PMAX], py[VD_PMAX], pz[VD_PMAX];   // other priors: R^_k x~
};

__device__ __forceinline__ void pix_geometry(const Win& w, const PoseF* __restrict__ P, const float2* __restrict__ flow,
                                             int u, int v, Pix& c) {
    c.u = (float)u;
    c.v = (float)v;
    const float x0 = ((float)u - w.cx) * w.ifx, x1 = ((float)v - w.cy) * w.ify;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t) {
        if (t < w.N) {
            const PoseF& T = P[t];
            c.ax[t] = fmaf(T.r[0], x0, fmaf(T.r[1], x1, T.r[2]));
            c.ay[t] = fmaf(T.r[3], x0, fmaf(T.r[4], x1, T.r[5]));
            c.az[t] = fmaf(T.r[6], x0, fmaf(T.r[7], x1, T.r[8]));
        }
    }
    const float2 f = flow[v * w.W + u];
    c.o1x = (float)u + f.x;
    c.o1y = (float)v + f.y;
    c.ok1 = isfinite(f.x) && isfinite(f.y);
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        if (k < w.P && !P[w.N + k].ident) {
            const PoseF& T = P[w.N + k];
            c.px[k] = fmaf(T.r[0], x0, fmaf(T.r[1], x1, T.r[2]));
            c.py[k] = fmaf(T.r[3], x0, fmaf(T.r[4], x1, T.r[5]));
            c.pz[k] = fmaf(T.r[6], x0, fmaf(T.r[7], x1, T.r[8]));
        }
    }
}

// Normalised prior difference z for candidate rho: false when the transfer is invalid or
// lands on a hole.
__device__ __forceinline__ bool prior_z(const Win& w, const PoseF* __restrict__ P, const float* __restrict__ prior,
                                        const Pix& c, int k, float rho, float& z) {
    float rh, inv_phi;
    if (P[w.N + k].ident) {
        rh = c.rh[k];
        inv_phi = rho;
    } else {
        const PoseF& T = P[w.N + k];
        const float Qx = fmaf(rho, T.t[0], c.px[k]);
        const float Qy = fmaf(rho, T.t[1], c.py[k]);
        const float Qz = fmaf(rho, T.t[2], c.pz[k]);
        if (!(Qz > 0.f)) return false;
        const float iz = rcp(Qz);
        const float lx = floorf(fmaf(w.fx, Qx * iz, w.cx) + 0.5f);
        const float ly = floorf(fmaf(w.fy, Qy * iz, w.cy) + 0.5f);
        if (!(lx >= 0.f && lx <= (float)(w.W - 1) && ly >= 0.f && ly <= (float)(w.H - 1))) return false;
        rh = prior[(size_t)k * w.H * w.W + (int)ly * w.W + (int)lx];
        inv_phi = rho * iz;
    }
    if (!(rh > 0.f) || !isfinite(rh)) return false;
    z = (rh - inv_phi) / (w.csig * rh);
    return true;
}

// E_j(rho) in log2 units: sum_t q_t cost_t + sum_k q^_k cost^_k.
__device__ __forceinline__ float energy2(const Win& w, const PoseF* __restrict__ P, const float2* __restrict__ flow,
                                         const float* __restrict__ prior, const Pix& c, float rho) {
    float E = 0.f;
    float ppx = c.u, ppy = c.v;
    bool zprev = true;
    const size_t plane = (size_t)w.H * w.W;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t) {
        if (t < w.N) {
            const PoseF& T = P[t];
            const float Qx = fmaf(rho, T.t[0], c.ax[t]);
            const float Qy = fmaf(rho, T.t[1], c.ay[t]);
            const float Qz = fmaf(rho, T.t[2], c.az[t]);
            const bool zok = Qz > 0.f;
            const float iz = rcp(Qz);
            const float px = fmaf(w.fx, Qx * iz, w.cx);
            const float py = fmaf(w.fy, Qy * iz, w.cy);
            float ox, oy;
            bool fok;
            if (t == 0) {
                ox = c.o1x; oy = c.o1y; fok = c.ok1;
            } else {
                float fx, fy;
                fok = sample_flow(flow + t * plane, w.H, w.W, ppx, ppy, fx, fy);
                ox = ppx + fx;
                oy = ppy + fy;
            }
            const bool ok = zprev && zok && fok;
            const float ex = px - ox, ey = py - oy;
            const float cost = ok ? flow_cost2(w, fmaf(ex, ex, ey * ey)) : 1.0f;
            E = fmaf(c.q[t], cost, E);
            ppx = px; ppy = py; zprev = zok;
        }
    }
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        if (k < w.P && c.qh[k] > 0.f) {
            float z;
            const float cost = prior_z(w, P, prior, c, k, rho, z)
                             ? softplus2(fmaf(0.5f * VD_LOG2E * z, z, w.log2kappa)) : 1.0f;
            E = fmaf(c.qh[k], cost, E);
        }
    }
    return E;
}

// Prior posteriors q^_k at the current value (Eq. 3 mixture): pi N / (pi N + (1 - pi) U).
__device__ __forceinline__ void prior_posteriors(const Win& w, const PoseF* __restrict__ P,
                                                 const float* __restrict__ prior, const float* __restrict__ pweight,
                                                 int pix, Pix& c, float rho_cur) {
    const size_t plane = (size_t)w.H * w.W;
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        c.qh[k] = 0.f;
        if (k < w.P) {
            if (P[w.N + k].ident) c.rh[k] = prior[k * plane + pix];
            float z;
            if (prior_z(w, P, prior, c, k, rho_cur, z)) {
                const float pw = w.has_prior_weight ? pweight[k * plane + pix] : w.pi_default;
                if (pw > 0.f) {
                    const float odds = (1.f - pw) / pw;
                    c.qh[k] = 1.f / fmaf(odds, exp2f_fast(fmaf(0.5f * VD_LOG2E * z, z, w.log2kappa)), 1.f);
                }
            }
        }
    }
}

// Emission ratio L1/L0 of one frame term at rho (1 for an invalid term); frames in order.
template <typename F>
__device__ __forceinline__ void emissions(const Win& w, const PoseF* __restrict__ P, const float2* __restrict__ flow,
                                          const Pix& c, float rho, F&& out) {
    float ppx = c.u, ppy = c.v;
    bool zprev = true;
    const size_t plane = (size_t)w.H * w.W;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t) {
        if (t < w.N) {
            const PoseF& T = P[t];
            const float Qx = fmaf(rho, T.t[0], c.ax[t]);
            const float Qy = fmaf(rho, T.t[1], c.ay[t]);
            const float Qz = fmaf(rho, T.t[2], c.az[t]);
            const bool zok = Qz > 0.f;
            const float iz = rcp(Qz);
            const float px = fmaf(w.fx, Qx * iz, w.cx);
            const float py = fmaf(w.fy, Qy * iz, w.cy);
            float ox, oy;
            bool fok;
            if (t == 0) {
                ox = c.o1x; oy = c.o1y; fok = c.ok1;
            } else {
                float fx, fy;
                fok = sample_flow(flow + t * plane, w.H, w.W, ppx, ppy, fx, fy);
                ox = ppx + fx;
                oy = ppy + fy;
            }
            const bool ok = zprev && zok && fok;
            const float ex = px - ox, ey = py - oy;
            const float ratio = ok ? exp2f_fast(-log2_ratio(w, fmaf(ex, ex, ey * ey))) : 1.0f;
            out(t, ratio, ok);
            ppx = px; ppy = py; zprev = zok;
        }
    }
}

// ----------------------------------------------------------------------------------
// block-level FP64 reduction of NR values held per thread (fixed order)
// ----------------------------------------------------------------------------------
template <int NR>
__device__ __forceinline__ void block_reduce(double* acc, double* red /* [4][NR] in LDS */) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        double v = acc[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        acc[k] = v;
    }
    if ((tid & 63) == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) red[(tid >> 6) * NR + k] = acc[k];
    }
    __syncthreads();
    if (tid < NR) {
        double s = 0.0;
        for (int wv = 0; wv < VD_BLOCK / 64; ++wv) s += red[wv * NR + tid];
        red[tid] = s;      // wave 0's slots: safe, each tid < NR reads all waves before writing its own
    }
}

// Last-block detection; returns true in every thread of the block that arrives last.
__device__ __forceinline__ bool last_block(unsigned* counter, unsigned nblocks, int* flag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned ticket = atomicAdd(counter, 1u);
        *flag = (ticket == nblocks - 1);
    }
    __syncthreads();
    const bool last = *flag;
    if (last) __threadfence();
    return last;
}

}  // namespace vd
