// Robust point-to-plane inverse-depth keyframe alignment on gfx950 (VOLDOR+SLAM sec.
// III-B, Eq. 10 with the criterion of Eq. 12, no photometric term).
//
//   prepare : per map-1 pixel l, the plane (A, b) = (rho1 n, n . x~_l) from central
//             differences of map 1 (NaN where the normal is invalid), so that for a
//             map-2 point Q~ = rho2 Q the residual is r = (rho2 b - A . Q~) / (s Q~_z)
//   step    : per map-2 pixel the residual, its Jacobian w.r.t. a left pose update and the
//             robust weight, reduced per block in FP64 to H (21), g (6), cost, count;
//   finish  : one block per pair sums the block records, solves H delta = -g by Cholesky
//             and updates the pose, or (final pass) inverts H into the covariance.
//   sim(3)  : the same terms with the relative depth scale as a seventh unknown, under
//             Levenberg-Marquardt (a trial step per evaluation, kept when its cost is lower).
#include "device.h"
#include "kernels.h"

namespace vd {

__global__ void __launch_bounds__(VD_BLOCK)
k_align_prepare(AlignArgs a, AlignBufs B) {
    const size_t plane = (size_t)a.H * a.W;
    const size_t j = (size_t)blockIdx.x * VD_BLOCK + threadIdx.x;
    if (j < (size_t)a.n_pairs) {            // per-pair bookkeeping
        B.status[j] = 0;
        for (int k = 0; k < 4; ++k) B.stats[4 * j + k] = 0.0;
    }
    if (j >= plane * a.n_pairs) return;
    const int pair = (int)(j / plane);
    const int l = (int)(j - (size_t)pair * plane);
    const int v = l / a.W, u = l - v * a.W;
    const float* R = B.idepth1 + (size_t)pair * plane;
    float4 out = make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""));
    if (u >= 1 && u <= a.W - 2 && v >= 1 && v <= a.H - 2) {
        const float r0 = R[l];
        const float rr = R[l + 1], rl = R[l - 1], rd = R[l + a.W], ru = R[l - a.W];
        const float lim = a.disc * r0;
        bool ok = r0 > 0.f && isfinite(r0);
        ok = ok && rr > 0.f && isfinite(rr) && fabsf(rr - r0) <= lim;
        ok = ok && rl > 0.f && isfinite(rl) && fabsf(rl - r0) <= lim;
        ok = ok && rd > 0.f && isfinite(rd) && fabsf(rd - r0) <= lim;
        ok = ok && ru > 0.f && isfinite(ru) && fabsf(ru - r0) <= lim;
        if (ok) {
            // P(l) = x~_l / rho;  dx = P(l+x) - P(l-x),  dy = P(l+y) - P(l-y)
            const float xr = ((float)(u + 1) - a.cx) * a.ifx, xl = ((float)(u - 1) - a.cx) * a.ifx;
            const float xc = ((float)u - a.cx) * a.ifx;
            const float yd = ((float)(v + 1) - a.cy) * a.ify, yu = ((float)(v - 1) - a.cy) * a.ify;
            const float yc = ((float)v - a.cy) * a.ify;
            const float irr = 1.f / rr, irl = 1.f / rl, ird = 1.f / rd, iru = 1.f / ru;
            const float dx0 = xr * irr - xl * irl, dx1 = yc * irr - yc * irl, dx2 = irr - irl;
            const float dy0 = xc * ird - xc * iru, dy1 = yd * ird - yu * iru, dy2 = ird - iru;
            float n0 = dx1 * dy2 - dx2 * dy1;
            float n1 = dx2 * dy0 - dx0 * dy2;
            float n2 = dx0 * dy1 - dx1 * dy0;
            const float nn = sqrtf(n0 * n0 + n1 * n1 + n2 * n2);
            if (nn > 0.f && isfinite(nn)) {
                n0 /= nn; n1 /= nn; n2 /= nn;
                const float b = n0 * xc + n1 * yc + n2;          // n . x~_l (sign of n . P)
                if (b > 0.f) { n0 = -n0; n1 = -n1; n2 = -n2; }
                out = make_float4(r0 * n0, r0 * n1, r0 * n2, b > 0.f ? -b : b);
            }
        }
    }
    B.normals[j] = out;
}

__device__ __forceinline__ void robust(int kind, float scale, float r, float& psi, float& w) {
    const float ar = fabsf(r);
    if (kind == 0) {
        if (ar <= scale) { psi = 0.5f * r * r; w = 1.f; }
        else { psi = scale * (ar - 0.5f * scale); w = scale / ar; }
    } else {
        const float z = r / scale;
        psi = 0.5f * scale * scale * log1pf(z * z);
        w = 1.f / fmaf(z, z, 1.f);
    }
}

__global__ void __launch_bounds__(VD_BLOCK)
k_align_step(AlignArgs a, AlignBufs B) {
    __shared__ PoseF Tsh;
    const int tid = threadIdx.x;
    const int pair = blockIdx.y;
    if (B.status[pair] != 0) return;          // frozen after a singular step (uniform per pair)
    if (tid == 0) pose_to_f(B.pose + 6 * pair, &Tsh);
    __syncthreads();
    const PoseF T = Tsh;
    const size_t plane = (size_t)a.H * a.W;
    const float* R2 = B.idepth2 + (size_t)pair * plane;
    const float* C2 = B.conf2 + (size_t)pair * plane;
    const float4* NB = B.normals + (size_t)pair * plane;
    const float is = 1.f / a.s;
    // per-thread sums in FP32 (a thread covers a few pixels), FP64 across threads and blocks
    float acc[29];
#pragma unroll
    for (int k = 0; k < 29; ++k) acc[k] = 0.f;
    for (int j = blockIdx.x * VD_BLOCK + tid; j < (int)plane; j += gridDim.x * VD_BLOCK) {
        const float rho2 = R2[j], c2 = C2[j];
        if (!(rho2 > 0.f) || !isfinite(rho2) || !isfinite(c2)) continue;
        const int v = j / a.W, u = j - v * a.W;
        const float x0 = ((float)u - a.cx) * a.ifx, x1 = ((float)v - a.cy) * a.ify;
        // Q~ = rho2 (R X2 + t) = R x~ + rho2 t
        const float Qx = fmaf(rho2, T.t[0], fmaf(T.r[0], x0, fmaf(T.r[1], x1, T.r[2])));
        const float Qy = fmaf(rho2, T.t[1], fmaf(T.r[3], x0, fmaf(T.r[4], x1, T.r[5])));
        const float Qz = fmaf(rho2, T.t[2], fmaf(T.r[6], x0, fmaf(T.r[7], x1, T.r[8])));
        if (!(Qz > 0.f)) continue;
        const float iz = 1.f / Qz;
        const float lx = floorf(fmaf(a.fx, Qx * iz, a.cx) + 0.5f);
        const float ly = floorf(fmaf(a.fy, Qy * iz, a.cy) + 0.5f);
        if (!(lx >= 1.f && lx <= (float)(a.W - 2) && ly >= 1.f && ly <= (float)(a.H - 2))) continue;
        const float4 nb = NB[(int)ly * a.W + (int)lx];
        if (!isfinite(nb.x)) continue;
        const float r = (rho2 * nb.w - (nb.x * Qx + nb.y * Qy + nb.z * Qz)) * is * iz;
        // d = -(A/s + r e_z) / Q~_z ;  J_w = d (-[Q~]x),  J_v = rho2 d
        const float d0 = -nb.x * is * iz, d1 = -nb.y * is * iz, d2 = -(nb.z * is + r) * iz;
        const float J[6] = {-d1 * Qz + d2 * Qy, d0 * Qz - d2 * Qx, -d0 * Qy + d1 * Qx,
                            rho2 * d0, rho2 * d1, rho2 * d2};
        float psi, wr;
        robust(a.robust, a.scale, r, psi, wr);
        const float W = c2 * wr;
        int k = 1;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
#pragma unroll
            for (int l = i; l < 6; ++l) acc[k++] += W * J[i] * J[l];
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[22 + i] += W * J[i] * r;
        acc[0] += c2 * psi;
        acc[28] += 1.f;
    }
    block_sum_transposed<29, VD_BLOCK>(acc, [&](int v, double sum) {
        B.partials[((size_t)pair * 29 + v) * gridDim.x + blockIdx.x] = sum;
    });
}

// One block per pair: sum the pair's block records (fixed order), then the FP64 solve and
// pose update, or (final pass) the covariance.
__global__ void __launch_bounds__(VD_BLOCK)
k_align_finish(AlignBufs B, unsigned nb, int final_pass) {
    __shared__ double red[(VD_BLOCK / 64) * 29];
    const int pair = blockIdx.x;
    if (B.status[pair] != 0) return;
    reduce_partials<29>(B.partials + (size_t)pair * nb * 29, nb, red);
    if (threadIdx.x != 0) return;
    double H[36], g[6], x[6];
    int k = 1;
    for (int i = 0; i < 6; ++i)
        for (int l = i; l < 6; ++l) { H[6 * i + l] = H[6 * l + i] = red[k++]; }
    for (int i = 0; i < 6; ++i) g[i] = -red[22 + i];
    double* st = B.stats + 4 * pair;
    if (!final_pass) {
        if (st[3] == 0.0) st[0] = red[0];
        if (chol6_solve(H, g, x)) {
            left_update(B.pose + 6 * pair, x);
            st[3] += 1.0;
        } else {
            // ESINGULAR: the pose keeps the completed steps; cost and count at that pose
            B.status[pair] = 4;
            st[1] = red[0];
            st[2] = red[28];
            for (int i = 0; i < 36; ++i) B.cov[36 * pair + i] = __builtin_nan("");
        }
        return;
    }
    if (st[3] == 0.0) st[0] = red[0];
    st[1] = red[0];
    st[2] = red[28];
    double* cov = B.cov + 36 * pair;
    bool ok = true;
    for (int c = 0; c < 6 && ok; ++c) {
        double e[6] = {0, 0, 0, 0, 0, 0};
        e[c] = 1.0;
        ok = chol6_solve(H, e, x);
        for (int i = 0; i < 6; ++i) cov[6 * i + c] = x[i];
    }
    if (!ok) {
        for (int i = 0; i < 36; ++i) cov[i] = __builtin_nan("");
        B.status[pair] = 4;
    }
}

// ----------------------------------------------------------------------------------
// 7-DoF alignment (relative motion and depth scale) by Levenberg-Marquardt.  Map 1's plane
// of pixel l passes through s P1(l): for Q~ = rho2 Q the residual is
// r = (rho2 b - A . Q~ / s) / Q~_z, with d r / d log s = (A . Q~) / (s Q~_z).  Each step
// evaluates the cost and normal equations at a trial state; the finish kernel keeps the
// trial when its cost is lower than the accepted state's (damping / 10), otherwise keeps the
// accepted state (damping * 10), and solves (H + lambda diag H) d = -g for the next trial.
// Per-pair state in scratch: [trial pose 6 | trial s | lambda | accepted records 37 |
// accepted steps | evaluated]
// ----------------------------------------------------------------------------------
constexpr int kSimRec = 37;        // H upper (28), g (7), cost, count
constexpr int kSimState = 6 + 1 + 1 + kSimRec + 2;

__global__ void __launch_bounds__(VD_BLOCK)
k_sim3_step(AlignArgs a, AlignBufs B, const double* __restrict__ state) {
    __shared__ PoseF Tsh;
    __shared__ float s_sh;
    const int tid = threadIdx.x;
    const int pair = blockIdx.y;
    if (B.status[pair] != 0) return;
    const double* S = state + (size_t)pair * kSimState;
    if (tid == 0) {
        pose_to_f(S, &Tsh);
        s_sh = (float)S[6];
    }
    __syncthreads();
    const PoseF T = Tsh;
    const float is = 1.f / s_sh;
    const size_t plane = (size_t)a.H * a.W;
    const float* R2 = B.idepth2 + (size_t)pair * plane;
    const float* C2 = B.conf2 + (size_t)pair * plane;
    const float4* NB = B.normals + (size_t)pair * plane;
    float acc[kSimRec];
#pragma unroll
    for (int k = 0; k < kSimRec; ++k) acc[k] = 0.f;
    for (int j = blockIdx.x * VD_BLOCK + tid; j < (int)plane; j += gridDim.x * VD_BLOCK) {
        const float rho2 = R2[j], c2 = C2[j];
        if (!(rho2 > 0.f) || !isfinite(rho2) || !isfinite(c2)) continue;
        const int v = j / a.W, u = j - v * a.W;
        const float x0 = ((float)u - a.cx) * a.ifx, x1 = ((float)v - a.cy) * a.ify;
        const float Qx = fmaf(rho2, T.t[0], fmaf(T.r[0], x0, fmaf(T.r[1], x1, T.r[2])));
        const float Qy = fmaf(rho2, T.t[1], fmaf(T.r[3], x0, fmaf(T.r[4], x1, T.r[5])));
        const float Qz = fmaf(rho2, T.t[2], fmaf(T.r[6], x0, fmaf(T.r[7], x1, T.r[8])));
        if (!(Qz > 0.f)) continue;
        const float iz = 1.f / Qz;
        const float lx = floorf(fmaf(a.fx, Qx * iz, a.cx) + 0.5f);
        const float ly = floorf(fmaf(a.fy, Qy * iz, a.cy) + 0.5f);
        if (!(lx >= 1.f && lx <= (float)(a.W - 2) && ly >= 1.f && ly <= (float)(a.H - 2))) continue;
        const float4 nb = NB[(int)ly * a.W + (int)lx];
        if (!isfinite(nb.x)) continue;
        const float aq = nb.x * Qx + nb.y * Qy + nb.z * Qz;
        const float r = (rho2 * nb.w - aq * is) * iz;
        const float d0 = -nb.x * is * iz, d1 = -nb.y * is * iz, d2 = -(nb.z * is + r) * iz;
        const float J[7] = {-d1 * Qz + d2 * Qy, d0 * Qz - d2 * Qx, -d0 * Qy + d1 * Qx,
                            rho2 * d0, rho2 * d1, rho2 * d2, aq * is * iz};
        float psi, wr;
        robust(a.robust, a.scale, r, psi, wr);
        const float W = c2 * wr;
        int k = 0;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
#pragma unroll
            for (int l = i; l < 7; ++l) acc[k++] += W * J[i] * J[l];
        }
#pragma unroll
        for (int i = 0; i < 7; ++i) acc[28 + i] += W * J[i] * r;
        acc[35] += c2 * psi;
        acc[36] += 1.f;
    }
    block_sum_transposed<kSimRec, VD_BLOCK>(acc, [&](int v, double sum) {
        B.partials[((size_t)pair * kSimRec + v) * gridDim.x + blockIdx.x] = sum;
    });
}

// Solve A x = b (7x7 SPD, row-major) by Cholesky; false when a pivot is not finite or not
// above 1e-12 times the largest diagonal entry.
__device__ inline bool chol7_solve(const double* A, const double* b, double* x) {
    double L[49];
    double dmax = 0.0;
    for (int i = 0; i < 7; ++i) dmax = fmax(dmax, A[8 * i]);
    const double tol = 1e-12 * dmax;
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[7 * i + j];
            for (int k = 0; k < j; ++k) s -= L[7 * i + k] * L[7 * j + k];
            if (i == j) {
                if (!(s > tol) || !isfinite(s)) return false;
                L[7 * i + i] = sqrt(s);
            } else {
                L[7 * i + j] = s / L[7 * j + j];
            }
        }
    }
    double y[7];
    for (int i = 0; i < 7; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[7 * i + k] * y[k];
        y[i] = s / L[7 * i + i];
    }
    for (int i = 6; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 7; ++k) s -= L[7 * k + i] * x[k];
        x[i] = s / L[7 * i + i];
    }
    return true;
}

// One block per pair: the evaluation's records (fixed order), then LM's accept / reject and
// the next trial, or (last) the covariance of the accepted state.  phase 0: the evaluation is
// of the initial state.
__global__ void __launch_bounds__(VD_BLOCK)
k_sim3_finish(AlignBufs B, double* __restrict__ state, double* __restrict__ scale, unsigned nb, int phase,
              int last) {
    __shared__ double red[(VD_BLOCK / 64) * kSimRec];
    const int pair = blockIdx.x;
    if (B.status[pair] != 0) return;
    reduce_partials<kSimRec>(B.partials + (size_t)pair * nb * kSimRec, nb, red);
    if (threadIdx.x != 0) return;
    double* S = state + (size_t)pair * kSimState;
    double* acc = S + 8;
    double* st = B.stats + 4 * pair;
    double* pose = B.pose + 6 * pair;
    if (phase == 0) {
        for (int i = 0; i < kSimRec; ++i) acc[i] = red[i];
        st[0] = red[35];
        S[7] = 1e-4;                       // lambda
        S[8 + kSimRec] = 0.0;              // accepted steps
    } else if (red[35] < acc[35]) {
        for (int i = 0; i < 6; ++i) pose[i] = S[i];
        scale[pair] = S[6];
        for (int i = 0; i < kSimRec; ++i) acc[i] = red[i];
        S[7] = fmax(S[7] / 10.0, 1e-12);
        S[8 + kSimRec] += 1.0;
    } else {
        S[7] = fmin(S[7] * 10.0, 1e12);
    }
    st[1] = acc[35];
    st[2] = acc[36];
    st[3] = S[8 + kSimRec];
    double H[49], g[7], x[7];
    int k = 0;
    for (int i = 0; i < 7; ++i)
        for (int l = i; l < 7; ++l) { H[7 * i + l] = H[7 * l + i] = acc[k++]; }
    for (int i = 0; i < 7; ++i) g[i] = -acc[28 + i];
    double* cov = B.cov + 49 * pair;
    if (!last) {
        double A[49];
        for (int i = 0; i < 49; ++i) A[i] = H[i];
        for (int i = 0; i < 7; ++i) A[8 * i] += S[7] * H[8 * i];
        if (!chol7_solve(A, g, x)) {
            B.status[pair] = 4;
            for (int i = 0; i < 49; ++i) cov[i] = __builtin_nan("");
            return;
        }
        for (int i = 0; i < 6; ++i) S[i] = pose[i];
        left_update(S, x);
        S[6] = scale[pair] * exp(x[6]);
        return;
    }
    bool ok = true;
    for (int c = 0; c < 7 && ok; ++c) {
        double e[7] = {0, 0, 0, 0, 0, 0, 0};
        e[c] = 1.0;
        ok = chol7_solve(H, e, x);
        for (int i = 0; i < 7; ++i) cov[7 * i + c] = x[i];
    }
    if (!ok) {
        for (int i = 0; i < 49; ++i) cov[i] = __builtin_nan("");
        B.status[pair] = 4;
    }
}

__global__ void k_sim3_init(const double* __restrict__ pose, const double* __restrict__ scale, double* __restrict__ state,
                            int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double* S = state + (size_t)p * kSimState;
    for (int i = 0; i < 6; ++i) S[i] = pose[6 * p + i];
    S[6] = scale[p];
}

size_t sim3_state_doubles(int n_pairs) { return (size_t)n_pairs * kSimState; }

hipError_t launch_align_sim3(const AlignArgs& a, const AlignBufs& b, double* scale, double* state, int steps, int nblocks,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_sim3_init, dim3((a.n_pairs + 63) / 64), dim3(64), 0, st, b.pose, scale, state, a.n_pairs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int k = 0; k <= steps; ++k) {
        hipLaunchKernelGGL(k_sim3_step, dim3(nblocks, a.n_pairs), dim3(VD_BLOCK), 0, st, a, b, (const double*)state);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_sim3_finish, dim3(a.n_pairs), dim3(VD_BLOCK), 0, st, b, state, scale, (unsigned)nblocks,
                           k == 0 ? 0 : 1, k == steps ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_align_prepare(const AlignArgs& a, const AlignBufs& b, hipStream_t st) {
    const size_t n = (size_t)a.H * a.W * a.n_pairs;
    hipLaunchKernelGGL(k_align_prepare, dim3((unsigned)((n + VD_BLOCK - 1) / VD_BLOCK)), dim3(VD_BLOCK), 0, st, a, b);
    return hipGetLastError();
}

hipError_t launch_align_step(const AlignArgs& a, const AlignBufs& b, int final_pass, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_align_step, dim3(nblocks, a.n_pairs), dim3(VD_BLOCK), 0, st, a, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_align_finish, dim3(a.n_pairs), dim3(VD_BLOCK), 0, st, b, (unsigned)nblocks, final_pass);
    return hipGetLastError();
}

}  // namespace vd
