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
// pose Gauss-Newton launches: threads per block and pixels per thread and load batch
#ifndef VD_GN_BLOCK
#define VD_GN_BLOCK 512
#endif
#ifndef VD_GN_PIX
#define VD_GN_PIX 2
#endif
// pixels per thread whose loads are issued together (the grid is sized by VD_GN_PIX)
#ifndef VD_GN_UB
#define VD_GN_UB 4
#endif
#define VD_SPEC 8       // maximum speculation depth of the chain scan
// lanes per lattice node in the separate phase-A grid (a power of two; one Philox group of
// four candidates per lane at K = 32)
#ifndef VD_PA_LANES
#define VD_PA_LANES 8
#endif
#define VD_LN2 0.69314718055994530942f
#define VD_LOG2E 1.44269504088896340736f

namespace vd {

// ----------------------------------------------------------------------------------
// constants of one launch
// ----------------------------------------------------------------------------------
struct PoseF {          // rotation (row-major) and translation, FP32 copy of a 6-vector
    float r[9];
    float t[3];
    float d[9];         // R - I, rounded from FP64 (keeps small rotations at full precision)
    int ident;          // the 6-vector is exactly zero (identity transfer)
    int pad[2];
};

// The frame pose tables are not written by the kernels that evaluate energies: their reads
// go through the constant address space, so a wave-uniform read is a scalar load (scalar
// cache, SGPR operands) rather than three vector loads per pixel and frame
struct PoseTD {
    float t[3];
    float d[9];
};
__device__ __forceinline__ PoseTD pose_td(const PoseF* P, int t) {
    typedef const PoseF __attribute__((address_space(4))) CPoseF;
    const CPoseF* p = (const CPoseF*)(P) + t;
    PoseTD r;
#pragma unroll
    for (int i = 0; i < 3; ++i) r.t[i] = p->t[i];
#pragma unroll
    for (int i = 0; i < 9; ++i) r.d[i] = p->d[i];
    return r;
}
__device__ __forceinline__ bool pose_ident(const PoseF* P, int t) {
    typedef const PoseF __attribute__((address_space(4))) CPoseF;
    return ((const CPoseF*)(P) + t)->ident != 0;
}

struct PoseD {          // FP64 rotation matrix (row-major) and translation of a frame
    double R[9];
    double t[3];
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
    // empirical disparity model of the priors (prior_model 1): residual r = fb (rho^ - 1/phi_z)
    int prior_disp;
    float disp_fb;        // focal length times baseline
    float disp_inv_alpha; // 1 / log-logistic scale (px)
    float disp_beta;      // log-logistic shape, in (0, 1]
    int disp_beta1;       // shape 1 (fast path)
    float disp_zfloor;    // floor of |r| / alpha (shape < 1: the density diverges at 0)
    float disp_c;         // log2(2 alpha / (beta D)), D the outlier disparity range
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
    for (int i = 0; i < 9; ++i) {
        out->r[i] = (float)R[i];
        out->d[i] = (float)(R[i] - ((i & 3) == 0 ? 1.0 : 0.0));
    }
    for (int i = 0; i < 3; ++i) out->t[i] = (float)p[3 + i];
    out->ident = (p[0] == 0.0 && p[1] == 0.0 && p[2] == 0.0 && p[3] == 0.0 && p[4] == 0.0 && p[5] == 0.0);
}

// exp([w]x) for the small increments of a Gauss-Newton step: Rodrigues coefficients by their
// Taylor series (exact to double rounding for |w| < 0.1), sin/cos beyond.
__device__ inline void exp_so3_small(const double w[3], double R[9]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    if (th2 >= 1e-2) { exp_so3(w, R); return; }
    const double a = 1.0 + th2 * (-1.0 / 6 + th2 * (1.0 / 120 + th2 * (-1.0 / 5040 + th2 * (1.0 / 362880 - th2 / 39916800))));
    const double b = 0.5 + th2 * (-1.0 / 24 + th2 * (1.0 / 720 + th2 * (-1.0 / 40320 + th2 * (1.0 / 3628800 - th2 / 479001600))));
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

// both pose tables of one 6-vector from one rotation: the FP32 table exactly as pose_to_f
// builds it, and the FP64 rotation and translation
__device__ inline void pose_tables_from_vec(const double* p, PoseF* f, PoseD* d) {
    double R[9];
    exp_so3(p, R);
    for (int i = 0; i < 9; ++i) {
        d->R[i] = R[i];
        f->r[i] = (float)R[i];
        f->d[i] = (float)(R[i] - ((i & 3) == 0 ? 1.0 : 0.0));
    }
    for (int i = 0; i < 3; ++i) {
        d->t[i] = p[3 + i];
        f->t[i] = (float)p[3 + i];
    }
    f->ident = (p[0] == 0.0 && p[1] == 0.0 && p[2] == 0.0 && p[3] == 0.0 && p[4] == 0.0 && p[5] == 0.0);
}

__device__ inline void posef_from_d(const PoseD& D, PoseF* out) {
    for (int i = 0; i < 9; ++i) {
        out->r[i] = (float)D.R[i];
        out->d[i] = (float)(D.R[i] - ((i & 3) == 0 ? 1.0 : 0.0));
    }
    for (int i = 0; i < 3; ++i) out->t[i] = (float)D.t[i];
    out->ident = 0;
}

// (R, t) <- (exp([dw]x) R, exp([dw]x) t + dv) on the FP64 matrix form
__device__ inline void left_update_d(PoseD* P, const double* d) {
    double E[9], R2[9], t2[3];
    exp_so3_small(d, E);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            R2[3 * i + j] = E[3 * i] * P->R[j] + E[3 * i + 1] * P->R[3 + j] + E[3 * i + 2] * P->R[6 + j];
        t2[i] = E[3 * i] * P->t[0] + E[3 * i + 1] * P->t[1] + E[3 * i + 2] * P->t[2] + d[3 + i];
    }
    for (int i = 0; i < 9; ++i) P->R[i] = R2[i];
    for (int i = 0; i < 3; ++i) P->t[i] = t2[i];
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
// above 1e-12 times the largest diagonal entry.  One division per pivot (its reciprocal).
__device__ inline bool chol6_solve(const double* A, const double* b, double* x) {
    double L[36], inv[6];
    double dmax = 0.0;
    for (int i = 0; i < 6; ++i) dmax = fmax(dmax, A[7 * i]);
    const double tol = 1e-12 * dmax;
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[6 * i + j];
            for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
            if (i == j) {
                if (!(s > tol) || !isfinite(s)) return false;
                // 1 / sqrt(s): the hardware estimate and two Newton steps (full FP64
                // accuracy, a short dependent chain instead of sqrt and a division)
                const double hs = 0.5 * s;
                double r = __builtin_amdgcn_rsq(s);
                r = r * fma(-hs * r, r, 1.5);
                r = r * fma(-hs * r, r, 1.5);
                L[6 * i + i] = s * r;
                inv[i] = r;
            } else {
                L[6 * i + j] = s * inv[j];
            }
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
        y[i] = s * inv[i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * x[k];
        x[i] = s * inv[i];
    }
    return true;
}

// ----------------------------------------------------------------------------------
// fast FP32 transcendentals (v_rcp_f32, v_log_f32 = log2, v_exp_f32 = 2^x)
// ----------------------------------------------------------------------------------
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float log2f_fast(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float exp2f_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// log2(1 + x) for x >= 0 with the rounding of 1 + x compensated (u - 1 is exact for
// u in [1, 2]), so small arguments keep full relative precision
__device__ __forceinline__ float log2_1p(float x) {
    const float u = 1.f + x;
    const float d = u - 1.f;
    return d == 0.f ? x * VD_LOG2E : log2f_fast(u) * (x * rcp(d));
}

// log2(1 + 2^y)
__device__ __forceinline__ float softplus2(float y) {
    return y > 24.f ? y : log2_1p(exp2f_fast(y));
}

// log2(L0 / L1(r)) of the log-logistic planar density, r^2 given.  B2: shape == 2.
template <bool B2>
__device__ __forceinline__ float log2_ratio(const Win& w, float r2) {
    if (B2) {
        const float s = fmaf(r2, w.inv_a2, 1.f);
        return log2f_fast(w.fl_c * s * s);
    }
    const float z2 = fmaxf(r2 * w.inv_a2, w.zfloor * w.zfloor);
    const float lz = 0.5f * log2f_fast(z2);                            // log2(r/alpha)
    const float y = exp2f_fast(w.beta * lz);                           // (r/alpha)^beta
    return w.fl_c + 2.f * log2f_fast(1.f + y) + (2.f - w.beta) * lz;
}

// MIE cost of a valid flow term, log2(1 + L0/L1), in log2 units.  Shape 2: L0/L1 = c s^2 >= c,
// and 1 + c s^2 is rounded once before the log: the absolute error stays at the log's FP32
// resolution, which is what a sum of such terms needs
template <bool B2>
__device__ __forceinline__ float flow_cost2(const Win& w, float r2) {
    if (B2) {
        const float s = fmaf(r2, w.inv_a2, 1.f);
        return log2f_fast(fmaf(w.fl_c * s, s, 1.f));
    }
    return softplus2(log2_ratio<false>(w, r2));
}

// d cost / d r^2 in natural-log units (IRLS weight without q)
template <bool B2>
__device__ __forceinline__ float flow_dcost(const Win& w, float r2) {
    if (B2) {
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
    const float g = exp2f_fast(log2_ratio<false>(w, r2));
    return g / (1.f + g) * dlog;
}

// ----------------------------------------------------------------------------------
// bilinear flow sample on [0, W-1] x [0, H-1]; invalid outside or on non-finite taps.
// Each image row contributes one 16-byte load of two horizontally adjacent taps; at the
// right / lower border the pair is taken one pixel earlier with weight 1 on its second
// element (needs W, H >= 2).  Offsets are 32-bit from the frame's base pointer.
// ----------------------------------------------------------------------------------
struct __attribute__((aligned(8))) TapPair { float ax, ay, bx, by; };

__device__ __forceinline__ bool sample_flow(const float2* __restrict__ F, int H, int W, float x, float y,
                                            float& fx, float& fy) {
    const bool inside = (x >= 0.f) && (x <= (float)(W - 1)) && (y >= 0.f) && (y <= (float)(H - 1));
    float xs = inside ? x : 0.f, ys = inside ? y : 0.f;
    int x0 = (int)xs, y0 = (int)ys;
    x0 = min(x0, W - 2);
    y0 = min(y0, H - 2);
    const float ax = xs - (float)x0, ay = ys - (float)y0;
    const unsigned o = (unsigned)y0 * (unsigned)W + (unsigned)x0;
    TapPair r0, r1;
    __builtin_memcpy(&r0, F + o, sizeof(TapPair));
    __builtin_memcpy(&r1, F + o + (unsigned)W, sizeof(TapPair));
    const float tx = fmaf(ax, r0.bx - r0.ax, r0.ax), ty = fmaf(ax, r0.by - r0.ay, r0.ay);
    const float bx = fmaf(ax, r1.bx - r1.ax, r1.ax), by = fmaf(ax, r1.by - r1.ay, r1.ay);
    fx = fmaf(ay, bx - tx, tx);
    fy = fmaf(ay, by - ty, ty);
    return inside && isfinite(fx) && isfinite(fy);
}

// Same sample from the row-pair layout F2[y][x] = (X(x, y), X(x, y + 1)) (rows 0..H-2): the
// four taps are 32 contiguous bytes.  Arithmetic identical to sample_flow.
// In two parts, so that callers can issue several gathers before the first blend: the
// fetch (position, weights, the two 16-byte loads) and the blend.
struct FlowTap {
    float4 l, r;
    float ax, ay;
    bool inside;
};
__device__ __forceinline__ FlowTap fetch_flow2(const float4* __restrict__ F2, int H, int W, float x, float y) {
    FlowTap f;
    f.inside = (x >= 0.f) && (x <= (float)(W - 1)) && (y >= 0.f) && (y <= (float)(H - 1));
    float xs = f.inside ? x : 0.f, ys = f.inside ? y : 0.f;
    int x0 = (int)xs, y0 = (int)ys;
    x0 = min(x0, W - 2);
    y0 = min(y0, H - 2);
    f.ax = xs - (float)x0;
    f.ay = ys - (float)y0;
    const unsigned o = __umul24((unsigned)y0, (unsigned)W) + (unsigned)x0;
    const float4* q = (const float4*)((const char*)F2 + (o << 4));
    f.l = q[0];
    f.r = q[1];
    return f;
}
__device__ __forceinline__ bool blend_flow2(const FlowTap& f, float& fx, float& fy) {
    const float4 l = f.l, r = f.r;
    const float ax = f.ax, ay = f.ay;
    const float tx = fmaf(ax, r.x - l.x, l.x), ty = fmaf(ax, r.y - l.y, l.y);
    const float bx = fmaf(ax, r.z - l.z, l.z), by = fmaf(ax, r.w - l.w, l.w);
    fx = fmaf(ay, bx - tx, tx);
    fy = fmaf(ay, by - ty, ty);
    return f.inside && isfinite(fx) && isfinite(fy);
}
__device__ __forceinline__ bool sample_flow2(const float4* __restrict__ F2, int H, int W, float x, float y,
                                             float& fx, float& fy) {
    return blend_flow2(fetch_flow2(F2, H, W, x, y), fx, fy);
}

// Block index remapped so that each of the 8 XCDs (own L2; workgroups are dispatched to
// them round-robin) works on a contiguous range of logical blocks.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, i = b >> 3, per = nb >> 3, rem = nb & 7;
    return x * per + min(x, rem) + i;
}

// ----------------------------------------------------------------------------------
// per-pixel context of the energy E_j(rho) and its evaluation.  (R_t - I) x~ is recomputed
// per frame from x~ (6 FMAs) rather than cached in 3N registers.
// ----------------------------------------------------------------------------------
struct Pix {
    float u, v;
    float x0, x1;                                  // x~ = ((u - cx)/fx, (v - cy)/fy, 1)
    float q[VD_NMAX];                              // rigidness posteriors
    float f1x, f1y;                                // first flow X_1(j)
    bool ok1;
    float qh[VD_PMAX];                             // prior posteriors at the current value
    float rh[VD_PMAX];                             // identity-pose priors: rho^ at the pixel
    float px[VD_PMAX], py[VD_PMAX], pz[VD_PMAX];   // other priors: R^_k x~
};

template <bool PR>
__device__ __forceinline__ void pix_geometry(const Win& w, const PoseF* __restrict__ P, const float2* __restrict__ flow,
                                             int u, int v, Pix& c) {
    c.u = (float)u;
    c.v = (float)v;
    const float x0 = ((float)u - w.cx) * w.ifx, x1 = ((float)v - w.cy) * w.ify;
    c.x0 = x0;
    c.x1 = x1;
    const float2 f = flow[v * w.W + u];
    c.f1x = f.x;
    c.f1y = f.y;
    c.ok1 = isfinite(f.x) && isfinite(f.y);
    if (!PR) return;
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
    if (pose_ident(P, w.N + k)) {
        rh = c.rh[k];
        inv_phi = rho;
    } else {
        const PoseTD T = pose_td(P, w.N + k);
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
    z = w.prior_disp ? w.disp_fb * (rh - inv_phi) : (rh - inv_phi) * rcp(w.csig * rh);
    return true;
}

// log2(p0 / p1) of a prior term with a valid transfer: Eq. 3's Gaussian-uniform mixture (z the
// inverse-depth difference in units of sigma), or the empirical log-logistic law of the
// disparity residual (z = fb (rho^ - 1/phi_z) px): p1 = f_Fisk(|z|) / 2, p0 = 1 / D
__device__ __forceinline__ float prior_log2_ratio(const Win& w, float z) {
    if (!w.prior_disp) return fmaf(0.5f * VD_LOG2E * z, z, w.log2kappa);
    const float a = fmaxf(fabsf(z) * w.disp_inv_alpha, w.disp_zfloor);
    if (w.disp_beta1) return fmaf(2.f, log2f_fast(1.f + a), w.disp_c);
    const float la = log2f_fast(a);
    return fmaf(2.f, log2f_fast(1.f + exp2f_fast(w.disp_beta * la)), fmaf(1.f - w.disp_beta, la, w.disp_c));
}

// Per-frame flow residuals of candidate rho, frames in order: f(t, r^2, valid).
// Reprojection in displacement form: with D = (R_t - I) x~ + rho t_t the rigid image
// displacement of frame t is d_t = (fx (D_x - x0 D_z), fy (D_y - x1 D_z)) / (1 + D_z), so
// p_t = j + d_t and the residual p_t - (p_{t-1} + X_t(p_{t-1})) = d_t - d_{t-1} - X_t is
// formed from small numbers (no cancellation of image coordinates).
template <typename F>
__device__ __forceinline__ void frame_residuals(const Win& w, const PoseF* __restrict__ P,
                                                const float4* __restrict__ flow2, const Pix& c, float rho, F&& f) {
    float dpx = 0.f, dpy = 0.f;
    bool zprev = true;
    const size_t plane = (size_t)w.H * w.W;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t) {
        if (t < w.N) {
            const PoseTD T = pose_td(P, t);
            const float Dx = fmaf(rho, T.t[0], fmaf(T.d[0], c.x0, fmaf(T.d[1], c.x1, T.d[2])));
            const float Dy = fmaf(rho, T.t[1], fmaf(T.d[3], c.x0, fmaf(T.d[4], c.x1, T.d[5])));
            const float Dz = fmaf(rho, T.t[2], fmaf(T.d[6], c.x0, fmaf(T.d[7], c.x1, T.d[8])));
            const float Qz = 1.f + Dz;
            const bool zok = Qz > 0.f;
            const float iz = rcp(Qz);
            const float dx = w.fx * fmaf(-c.x0, Dz, Dx) * iz;
            const float dy = w.fy * fmaf(-c.x1, Dz, Dy) * iz;
            float fx, fy;
            bool fok;
            if (t == 0) {
                fx = c.f1x; fy = c.f1y; fok = c.ok1;
            } else {
                fok = sample_flow2(flow2 + t * plane, w.H, w.W, c.u + dpx, c.v + dpy, fx, fy);
            }
            const bool ok = zprev && zok && fok;
            const float ex = (dx - dpx) - fx, ey = (dy - dpy) - fy;
            f(t, fmaf(ex, ex, ey * ey), ok);
            dpx = dx; dpy = dy; zprev = zok;
        }
    }
}

// Energies are sums of FP32 terms (weight times cost factor) accumulated in FP64: with an
// FP32 sum, candidates whose energies differ by less than the sum's rounding tie, and ties go
// to the lowest slot (the current value), which holds values in place that an exact sum
// would move.  The product of two FP32 numbers is exact in FP64, so each step is one FP64
// FMA, the same in every phase (phase A, the speculative energies, the scan), bit for bit.
typedef double energy_t;

__device__ __forceinline__ energy_t eacc(float q, float cost, energy_t E) {
    return fma((double)q, (double)cost, E);
}

// E_j(rho) in log2 units: sum_t q_t cost_t + sum_k q^_k cost^_k.  PR: window has priors.
template <bool B2, bool PR>
__device__ __forceinline__ energy_t energy2(const Win& w, const PoseF* __restrict__ P, const float4* __restrict__ flow2,
                                            const float* __restrict__ prior, const Pix& c, float rho) {
    energy_t E = 0.0;
    frame_residuals(w, P, flow2, c, rho, [&](int t, float r2, bool ok) {
        E = eacc(c.q[t], ok ? flow_cost2<B2>(w, r2) : 1.0f, E);
    });
    if (!PR) return E;
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        if (k < w.P && c.qh[k] > 0.f) {
            float z;
            const float cost = prior_z(w, P, prior, c, k, rho, z)
                             ? softplus2(prior_log2_ratio(w, z)) : 1.0f;
            E = eacc(c.qh[k], cost, E);
        }
    }
    return E;
}

// E_j(rho) from frame cost factors already evaluated at rho (cost[t * step], as energy2
// forms them): the same FMAs in the same order as energy2, so the same value bit for bit.
template <bool PR>
__device__ __forceinline__ energy_t energy2_costs(const Win& w, const PoseF* __restrict__ P,
                                                  const float* __restrict__ prior, const Pix& c, float rho,
                                                  const float* cost, int step) {
    energy_t E = 0.0;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t)
        if (t < w.N) E = eacc(c.q[t], cost[t * step], E);
    if (!PR) return E;
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        if (k < w.P && c.qh[k] > 0.f) {
            float z;
            const float cost_k = prior_z(w, P, prior, c, k, rho, z)
                               ? softplus2(prior_log2_ratio(w, z)) : 1.0f;
            E = eacc(c.qh[k], cost_k, E);
        }
    }
    return E;
}

// E_j(rho) with the frame terms on separate lanes of a 32-lane group: lane hl < N computes
// frame hl's cost factor (its own reprojections into frames hl-1 and hl, as the sequential
// loop does), so the frames' flow gathers are in flight together; the terms are then summed
// in frame order with the sequential loop's FMAs, so the result equals energy2's bit for bit.
// Every lane of the group must call it (hbase = the group's first lane in the wave).
template <bool B2>
__device__ __forceinline__ float frame_cost(const Win& w, const PoseF* __restrict__ P, const float4* __restrict__ flow2,
                                            const Pix& c, float rho, int t) {
    const PoseTD T = pose_td(P, t);
    const float Dx = fmaf(rho, T.t[0], fmaf(T.d[0], c.x0, fmaf(T.d[1], c.x1, T.d[2])));
    const float Dy = fmaf(rho, T.t[1], fmaf(T.d[3], c.x0, fmaf(T.d[4], c.x1, T.d[5])));
    const float Dz = fmaf(rho, T.t[2], fmaf(T.d[6], c.x0, fmaf(T.d[7], c.x1, T.d[8])));
    const float Qz = 1.f + Dz;
    const bool zok = Qz > 0.f;
    const float iz = rcp(Qz);
    const float dx = w.fx * fmaf(-c.x0, Dz, Dx) * iz;
    const float dy = w.fy * fmaf(-c.x1, Dz, Dy) * iz;
    float dpx = 0.f, dpy = 0.f, fx, fy;
    bool zprev = true, fok;
    if (t == 0) {
        fx = c.f1x; fy = c.f1y; fok = c.ok1;
    } else {
        const PoseTD Tp = pose_td(P, t - 1);
        const float Ex = fmaf(rho, Tp.t[0], fmaf(Tp.d[0], c.x0, fmaf(Tp.d[1], c.x1, Tp.d[2])));
        const float Ey = fmaf(rho, Tp.t[1], fmaf(Tp.d[3], c.x0, fmaf(Tp.d[4], c.x1, Tp.d[5])));
        const float Ez = fmaf(rho, Tp.t[2], fmaf(Tp.d[6], c.x0, fmaf(Tp.d[7], c.x1, Tp.d[8])));
        const float Pz = 1.f + Ez;
        zprev = Pz > 0.f;
        const float ipz = rcp(Pz);
        dpx = w.fx * fmaf(-c.x0, Ez, Ex) * ipz;
        dpy = w.fy * fmaf(-c.x1, Ez, Ey) * ipz;
        fok = sample_flow2(flow2 + t * (size_t)w.H * w.W, w.H, w.W, c.u + dpx, c.v + dpy, fx, fy);
    }
    const bool ok = zprev && zok && fok;
    const float ex = (dx - dpx) - fx, ey = (dy - dpy) - fy;
    return ok ? flow_cost2<B2>(w, fmaf(ex, ex, ey * ey)) : 1.0f;
}

// E plus the prior terms of E_j(rho) in prior order (the tail of energy2 / energy2_lanes)
template <bool PR>
__device__ __forceinline__ energy_t prior_terms(const Win& w, const PoseF* __restrict__ P,
                                                const float* __restrict__ prior, const Pix& c, float rho, energy_t E) {
    if (!PR) return E;
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        if (k < w.P && c.qh[k] > 0.f) {
            float z;
            const float cost = prior_z(w, P, prior, c, k, rho, z)
                             ? softplus2(prior_log2_ratio(w, z)) : 1.0f;
            E = eacc(c.qh[k], cost, E);
        }
    }
    return E;
}

template <bool B2, bool PR>
__device__ __forceinline__ energy_t energy2_lanes(const Win& w, const PoseF* __restrict__ P,
                                                  const float4* __restrict__ flow2, const float* __restrict__ prior,
                                                  const Pix& c, float rho, int hl, int hbase) {
    const float mine = hl < w.N ? frame_cost<B2>(w, P, flow2, c, rho, hl) : 0.f;
    energy_t E = 0.0;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t)
        if (t < w.N) E = eacc(c.q[t], __shfl(mine, hbase + t), E);
    return prior_terms<PR>(w, P, prior, c, rho, E);
}

// E_j(rho) with pruning: all terms are non-negative and the FP64 running sum only grows, so
// once it passes `bound` the candidate cannot win and the remaining frames (and their flow
// gathers) are skipped.  STRICT: stop when E > bound (callers that keep ties), otherwise
// when E >= bound.  A pruned result is a partial sum on the losing side of the bound, so
// every comparison against the bound is decided exactly as with the full sum.
template <bool B2, bool PR, bool STRICT>
__device__ __forceinline__ energy_t energy2_bounded(const Win& w, const PoseF* __restrict__ P,
                                                    const float4* __restrict__ flow2, const float* __restrict__ prior,
                                                    const Pix& c, float rho, energy_t bound) {
    energy_t E = 0.0;
    float dpx = 0.f, dpy = 0.f;
    bool zprev = true;
    const size_t plane = (size_t)w.H * w.W;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t) {
        if (t >= w.N) break;
        const PoseTD T = pose_td(P, t);
        const float Dx = fmaf(rho, T.t[0], fmaf(T.d[0], c.x0, fmaf(T.d[1], c.x1, T.d[2])));
        const float Dy = fmaf(rho, T.t[1], fmaf(T.d[3], c.x0, fmaf(T.d[4], c.x1, T.d[5])));
        const float Dz = fmaf(rho, T.t[2], fmaf(T.d[6], c.x0, fmaf(T.d[7], c.x1, T.d[8])));
        const float Qz = 1.f + Dz;
        const bool zok = Qz > 0.f;
        const float iz = rcp(Qz);
        const float dx = w.fx * fmaf(-c.x0, Dz, Dx) * iz;
        const float dy = w.fy * fmaf(-c.x1, Dz, Dy) * iz;
        float fx, fy;
        bool fok;
        if (t == 0) {
            fx = c.f1x; fy = c.f1y; fok = c.ok1;
        } else {
            fok = sample_flow2(flow2 + t * plane, w.H, w.W, c.u + dpx, c.v + dpy, fx, fy);
        }
        const bool ok = zprev && zok && fok;
        const float ex = (dx - dpx) - fx, ey = (dy - dpy) - fy;
        E = eacc(c.q[t], ok ? flow_cost2<B2>(w, fmaf(ex, ex, ey * ey)) : 1.0f, E);
        if (STRICT ? (E > bound) : (E >= bound)) return E;
        dpx = dx; dpy = dy; zprev = zok;
    }
    if (!PR) return E;
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        if (k < w.P && c.qh[k] > 0.f) {
            float z;
            const float cost = prior_z(w, P, prior, c, k, rho, z)
                             ? softplus2(prior_log2_ratio(w, z)) : 1.0f;
            E = eacc(c.qh[k], cost, E);
        }
    }
    return E;
}

// M candidates against one bound with their frames in lockstep.  Each candidate keeps the
// running sum and stop test of energy2_bounded (STRICT as there), so every returned value
// is exactly what energy2_bounded returns for that candidate and bound; the flow gathers of
// the candidates of a frame are in flight together.  Bit m of live selects
// candidate m; an unselected candidate's value is meaningless.
template <bool B2, bool PR, int M, bool STRICT = false>
__device__ __forceinline__ void energy2_bounded_m(const Win& w, const PoseF* __restrict__ P,
                                                  const float4* __restrict__ flow2, const float* __restrict__ prior,
                                                  const Pix& c, const float* rho, unsigned live, energy_t bound,
                                                  energy_t* E) {
    float dpx[M], dpy[M];
    bool zprev[M];
#pragma unroll
    for (int m = 0; m < M; ++m) { E[m] = 0.0; dpx[m] = 0.f; dpy[m] = 0.f; zprev[m] = true; }
    const size_t plane = (size_t)w.H * w.W;
#pragma unroll
    for (int t = 0; t < VD_NMAX; ++t) {
        if (t >= w.N || live == 0u) break;
        // the gathers first, without branches: their positions are the previous frame's
        // reprojections, so the loads are in flight together during this frame's
        // reprojection; a pruned candidate fetches the in-range tap at (0, 0), unused
        FlowTap tap[M];
        if (t > 0) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const bool lv = (live >> m) & 1u;
                tap[m] = fetch_flow2(flow2 + t * plane, w.H, w.W, lv ? c.u + dpx[m] : -1.f, lv ? c.v + dpy[m] : -1.f);
            }
        }
        const PoseTD T = pose_td(P, t);
        float dx[M], dy[M], fx[M], fy[M];
        bool zok[M], fok[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float r = rho[m];
            const float Dx = fmaf(r, T.t[0], fmaf(T.d[0], c.x0, fmaf(T.d[1], c.x1, T.d[2])));
            const float Dy = fmaf(r, T.t[1], fmaf(T.d[3], c.x0, fmaf(T.d[4], c.x1, T.d[5])));
            const float Dz = fmaf(r, T.t[2], fmaf(T.d[6], c.x0, fmaf(T.d[7], c.x1, T.d[8])));
            const float Qz = 1.f + Dz;
            zok[m] = Qz > 0.f;
            const float iz = rcp(Qz);
            dx[m] = w.fx * fmaf(-c.x0, Dz, Dx) * iz;
            dy[m] = w.fy * fmaf(-c.x1, Dz, Dy) * iz;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            fx[m] = 0.f; fy[m] = 0.f; fok[m] = false;
            if (t == 0) {
                fx[m] = c.f1x; fy[m] = c.f1y; fok[m] = c.ok1;
            } else if ((live >> m) & 1u) {
                fok[m] = blend_flow2(tap[m], fx[m], fy[m]);
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if ((live >> m) & 1u) {
                const bool ok = zprev[m] && zok[m] && fok[m];
                const float ex = (dx[m] - dpx[m]) - fx[m], ey = (dy[m] - dpy[m]) - fy[m];
                E[m] = eacc(c.q[t], ok ? flow_cost2<B2>(w, fmaf(ex, ex, ey * ey)) : 1.0f, E[m]);
                if (STRICT ? (E[m] > bound) : (E[m] >= bound)) live &= ~(1u << m);
            }
            dpx[m] = dx[m]; dpy[m] = dy[m]; zprev[m] = zok[m];
        }
    }
    if (!PR) return;
    // candidates below the bound after every frame take the prior terms
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (!((live >> m) & 1u)) continue;
#pragma unroll
        for (int k = 0; k < VD_PMAX; ++k) {
            if (k < w.P && c.qh[k] > 0.f) {
                float z;
                const float cost = prior_z(w, P, prior, c, k, rho[m], z)
                                 ? softplus2(prior_log2_ratio(w, z)) : 1.0f;
                E[m] = eacc(c.qh[k], cost, E[m]);
            }
        }
    }
}

// Prior posteriors q^_k at the current value (Eq. 3 mixture): pi N / (pi N + (1 - pi) U).
// Returns a bit mask of the priors whose transfer is valid (no hole) at rho_cur.
template <bool PR>
__device__ __forceinline__ int prior_posteriors(const Win& w, const PoseF* __restrict__ P,
                                                const float* __restrict__ prior, const float* __restrict__ pweight,
                                                int pix, Pix& c, float rho_cur) {
    const size_t plane = (size_t)w.H * w.W;
    int mask = 0;
    if (!PR) return 0;
#pragma unroll
    for (int k = 0; k < VD_PMAX; ++k) {
        c.qh[k] = 0.f;
        if (k < w.P) {
            if (P[w.N + k].ident) c.rh[k] = prior[k * plane + pix];
            float z;
            if (prior_z(w, P, prior, c, k, rho_cur, z)) {
                mask |= 1 << k;
                const float pw = w.has_prior_weight ? pweight[k * plane + pix] : w.pi_default;
                if (pw > 0.f) {
                    const float odds = (1.f - pw) / pw;
                    c.qh[k] = rcp(fmaf(odds, exp2f_fast(prior_log2_ratio(w, z)), 1.f));
                }
            }
        }
    }
    return mask;
}

// Emission ratio L1/L0 of one frame term at rho (1 for an invalid term); frames in order.
template <bool B2, typename F>
__device__ __forceinline__ void emissions(const Win& w, const PoseF* __restrict__ P, const float4* __restrict__ flow2,
                                          const Pix& c, float rho, F&& out) {
    frame_residuals(w, P, flow2, c, rho, [&](int t, float r2, bool ok) {
        float ratio = 1.0f;
        if (ok) {
            if (B2) {
                const float s = fmaf(r2, w.inv_a2, 1.f);
                ratio = rcp(w.fl_c * s * s);                    // L1 / L0 = 1 / (c s^2)
            } else {
                ratio = exp2f_fast(-log2_ratio<false>(w, r2));
            }
        }
        out(t, ratio, ok, r2);
    });
}

// ----------------------------------------------------------------------------------
// block-level FP64 reduction of NR values held per thread (fixed order)
// ----------------------------------------------------------------------------------
template <int NR, int NT = VD_BLOCK>
__device__ __forceinline__ void block_reduce(double* acc, double* red /* [NT/64][NR] in LDS */) {
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
        for (int wv = 0; wv < NT / 64; ++wv) s += red[wv * NR + tid];
        red[tid] = s;      // wave 0's slots: safe, each tid < NR reads all waves before writing its own
    }
}

// Deterministic sum of per-block records stored value-major, part[k * nb + b], b < nb:
// value k is summed by SL consecutive lanes, lane l taking the blocks l, l + SL, ... in
// order, then an xor tree over the SL lanes: few levels of shuffles per value and many
// independent loads in flight per lane.  SL is the largest power of two up to 64 with
// NR * SL <= NT: every kernel that reduces one kind of record uses the same NT, so they
// all sum in the same order.  The NR sums are in red[0..NR-1] after the call (all threads
// synchronised).
template <int NR, int NT>
constexpr int partial_slices() {
    int sl = 64;
    while (sl > 1 && NR * sl > NT) sl >>= 1;
    return sl;
}

// Block sum of NR per-thread FP32 values, transposed through LDS: the values go to
// tr[v][thread] (the row stride keeps both the writes and the reads free of bank conflicts),
// then value v is summed in FP64 by SL lanes in thread order and an xor tree over the SL
// lanes; out(v, sum) is called once per value.  A fixed order, so every block sums alike.
template <int NR, int NT, class F>
__device__ __forceinline__ void block_sum_transposed(const float* a32, F&& out) {
    constexpr int SL = partial_slices<NR, NT>();
    constexpr int TS = NT + (SL < 32 ? SL : 0);
    __shared__ float tr[NR * TS];
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NR; ++i) tr[i * TS + tid] = a32[i];
    __syncthreads();
    const int v = tid / SL, l = tid % SL;
    double acc = 0.0;
    if (v < NR) {
#pragma unroll 8
        for (int i = l; i < NT; i += SL) acc += (double)tr[v * TS + i];
    }
#pragma unroll
    for (int off = SL / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (v < NR && l == 0) out(v, acc);
}

template <int NR, int NT = VD_BLOCK>
__device__ __forceinline__ void reduce_partials(const double* part, unsigned nb, double* red) {
    constexpr int SL = partial_slices<NR, NT>();
    const int tid = threadIdx.x;
    const int k = tid / SL, l = tid % SL;
    double acc = 0.0;
    if (k < NR) {
        const double* pk = part + (size_t)k * nb;
#pragma unroll 8
        for (unsigned b = l; b < nb; b += SL) acc += pk[b];
    }
#pragma unroll
    for (int off = SL / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __syncthreads();
    if (k < NR && l == 0) red[k] = acc;
    __syncthreads();
}

}  // namespace vd
