// Visibility-coverage (VC) scores for VO stride and keyframe selection on gfx950
// (VOLDOR+SLAM sec. III-A "VO Stride and Keyframe Selection" and its VC equation).
//
//   prep   : FP64 rotation and translation of every pose; clears the counters and the
//            per-pose coverage bitmaps (one bit per cell x cell block of frame 2)
//   pass   : one thread per frame-1 pixel, looping over the poses so that the depth map is
//            read once: depth-pixel test, FP64 projection into frame 2, inside test on the
//            nearest pixel, the covered cell's bit set in that pose's bitmap (only when it
//            reads as clear, so most pixels of an already covered cell issue no atomic);
//            counts by wave ballot into LDS, then one global add per block and pose
//   finish : one block: covered cells per pose by popcount, visibility, coverage, their
//            harmonic mean, and the first pose whose VC is below tau
// Counts are integers added atomically (exact in any order) and the bitmaps are ORs, so the
// results do not depend on scheduling.
#include <algorithm>

#include "device.h"
#include "kernels.h"

namespace vd {

__global__ void __launch_bounds__(VD_BLOCK)
k_vc_prep(VcArgs a, VcBufs B) {
    const size_t i = (size_t)blockIdx.x * VD_BLOCK + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * VD_BLOCK;
    for (size_t k = i; k < (size_t)a.n; k += stride) {
        const double* p = B.pose + 6 * k;
        const double w[3] = {p[0], p[1], p[2]};
        double R[9];
        exp_so3(w, R);
        double* T = B.RT + 12 * k;
        for (int e = 0; e < 9; ++e) T[e] = R[e];
        T[9] = p[3]; T[10] = p[4]; T[11] = p[5];
    }
    for (size_t k = i; k <= (size_t)a.n; k += stride) B.count[k] = 0u;
    const size_t nw = (size_t)a.n * a.words;
    for (size_t k = i; k < nw; k += stride) B.bits[k] = 0u;
}

__global__ void __launch_bounds__(VD_BLOCK)
k_vc_pass(VcArgs a, VcBufs B) {
    extern __shared__ uint32_t cnt[];          // [n] visible counts, [n] depth pixels
    // with lds_bits, the block's coverage bits go to an LDS copy of the n bitmaps first and
    // only its nonzero words reach the global bitmaps: one atomic per word per block instead
    // of one per pixel and pose that lands in a not yet covered cell
    uint32_t* lbits = cnt + ((a.n + 2) & ~1);
    const int nwords = a.n * a.words;
    for (int k = threadIdx.x; k <= a.n; k += VD_BLOCK) cnt[k] = 0u;
    if (a.lds_bits)
        for (int k = threadIdx.x; k < nwords; k += VD_BLOCK) lbits[k] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int j = blk * VD_BLOCK + threadIdx.x;
    bool depth = false;
    double rho = 0.0, x0 = 0.0, x1 = 0.0;
    if (j < a.H * a.W) {
        const float r = B.idepth[j];
        depth = isfinite(r) && r > 0.f;
        if (depth && B.conf) depth = B.conf[j] >= a.conf_min;
        const int v = j / a.W, u = j - v * a.W;
        rho = (double)r;
        x0 = ((double)u - a.cx) / a.fx;
        x1 = ((double)v - a.cy) / a.fy;
    }
    const unsigned long long dm = __ballot(depth);
    if (lane == 0 && dm) atomicAdd(&cnt[a.n], (uint32_t)__popcll(dm));
    for (int k = 0; k < a.n; ++k) {
        bool in = false;
        if (depth) {
            const double* T = B.RT + 12 * k;
            // rho (R X + t) with X = x~ / rho: the projection does not need 1/rho
            const double qx = T[0] * x0 + T[1] * x1 + T[2] + rho * T[9];
            const double qy = T[3] * x0 + T[4] * x1 + T[5] + rho * T[10];
            const double qz = T[6] * x0 + T[7] * x1 + T[8] + rho * T[11];
            if (qz > 0.0) {
                const double x = a.fx * qx / qz + a.cx;
                const double y = a.fy * qy / qz + a.cy;
                const double xn = floor(x + 0.5), yn = floor(y + 0.5);
                in = xn >= 0.0 && xn <= (double)(a.W - 1) && yn >= 0.0 && yn <= (double)(a.H - 1);
                if (in) {
                    const int c = ((int)yn / a.cell) * a.wc + (int)xn / a.cell;
                    const uint32_t bit = 1u << (c & 31);
                    if (a.lds_bits) {
                        atomicOr(lbits + k * a.words + (c >> 5), bit);
                    } else {
                        uint32_t* word = B.bits + (size_t)k * a.words + (c >> 5);
                        if (!(*word & bit)) atomicOr(word, bit);
                    }
                }
            }
        }
        const unsigned long long m = __ballot(in);
        if (lane == 0 && m) atomicAdd(&cnt[k], (uint32_t)__popcll(m));
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= a.n; k += VD_BLOCK) {
        const uint32_t c = cnt[k];
        if (c) atomicAdd(&B.count[k == a.n ? 0 : k + 1], c);
    }
    if (a.lds_bits)
        for (int k = threadIdx.x; k < nwords; k += VD_BLOCK) {
            const uint32_t v = lbits[k];
            if (v) atomicOr(B.bits + k, v);
        }
}

__global__ void __launch_bounds__(VD_BLOCK)
k_vc_finish(VcArgs a, VcBufs B) {
    __shared__ uint32_t part[VD_BLOCK / 64];
    __shared__ int first;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) first = a.n;
    const uint32_t n_depth = B.count[0];
    const double cells = (double)a.hc * (double)a.wc;
    for (int k = 0; k < a.n; ++k) {
        uint32_t c = 0u;
        const uint32_t* w = B.bits + (size_t)k * a.words;
        for (int i = threadIdx.x; i < a.words; i += VD_BLOCK) c += (uint32_t)__popc(w[i]);
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
        if (lane == 0) part[wid] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t hit = 0u;
            for (int q = 0; q < VD_BLOCK / 64; ++q) hit += part[q];
            const uint32_t vis_n = B.count[k + 1];
            const double vis = n_depth ? (double)vis_n / (double)n_depth : 0.0;
            const double cov = (double)hit / cells;
            const double vc = (vis > 0.0 && cov > 0.0) ? 2.0 / (1.0 / vis + 1.0 / cov) : 0.0;
            double* o = B.out + 5 * (size_t)k;
            o[0] = vis; o[1] = cov; o[2] = vc; o[3] = (double)vis_n; o[4] = (double)hit;
            if (first == a.n && vc < a.tau) first = k;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && B.first_below) *B.first_below = first;
}

hipError_t launch_vc(const VcArgs& a, const VcBufs& b, hipStream_t st) {
    const size_t prep_items = std::max<size_t>((size_t)a.n * a.words, (size_t)a.n + 1);
    const int prep_blocks = (int)std::min<size_t>((prep_items + VD_BLOCK - 1) / VD_BLOCK, 2048);
    hipLaunchKernelGGL(k_vc_prep, dim3(prep_blocks), dim3(VD_BLOCK), 0, st, a, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nb = (a.H * a.W + VD_BLOCK - 1) / VD_BLOCK;
    const size_t lds = sizeof(uint32_t) * (((size_t)a.n + 2) & ~(size_t)1) +
                       (a.lds_bits ? sizeof(uint32_t) * (size_t)a.n * a.words : 0);
    hipLaunchKernelGGL(k_vc_pass, dim3(nb), dim3(VD_BLOCK), lds, st, a, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_vc_finish, dim3(1), dim3(VD_BLOCK), 0, st, a, b);
    return hipGetLastError();
}

}  // namespace vd
