// Learned depth / rigidness proposal on gfx950: BF16 3x3 convolutions as implicit GEMMs on
// the matrix cores (v_mfma_f32_32x32x16_bf16), FP32 accumulation, NHWC activations.
//
//   k_conv_halo       the fast path: a block stages the halo of its output tile and the
//                     weights of a chunk of input channels in LDS with buffer loads.
//                     MODE 0: y = act(conv3x3(x) + b [+ skip]), stride 1 (optional 2x
//                     nearest upsampling of the input) or 2, optionally with the heads fused;
//                     MODE 1: data gradient dx = conv3x3^T(dy) with the transposed weights
//                     [Cin][3][3][Cout], optional "+ add" and "* (mask > 0)" epilogue; stride-2
//                     layers by sub-pixel classes, upsampling layers pooled 2x2 in registers
//   k_conv2           the general LDS-staged kernel for every other shape (same arithmetic
//                     roles; Cin a multiple of 16, Cout of 16)
//   k_wgrad2          dW[co][tap][ci] = sum_m dy[m][co] x_tap(m)[ci] per pixel chunk (FP32
//                     partials), dy and the 9 im2col slices staged pixel-contiguous in LDS;
//                     k_sum_chunks reduces the partials in a fixed order; k_bgrad the bias
//                     gradient (16-byte aligned BF16 arrays throughout)
//   k_features, k_loss (+ finish), k_adam: the element-wise rest.
//
// MFMA operand layout (32x32x16, wave64): lane l supplies A[i = l%32][k = 8(l/32) .. +7] and
// B[k = 8(l/32) .. +7][j = l%32]; the 16 accumulators of lane l hold D[i][j = l%32] for
// i = 8(a/4) + 4(l/32) + a%4, a = 0..15.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "proposal.h"

namespace vp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}


// heads of the last layer: rho = clip(softplus(o_0) / |t_1|, rho_min, rho_max), q_t = sigmoid(o_t)
__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoidf(float z) { return 0.5f * (1.f + tanhf(0.5f * z)); }

// ---------------------------------------------------------------------------------------
// input features: channel 2(t-1) + c = X_t[c] / FLOW_SCALE (non-finite -> 0), 16 channels
// ---------------------------------------------------------------------------------------
__global__ void k_features(const float2* __restrict__ flow, int N, int HW, uint16_t* __restrict__ x) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= HW) return;
    uint16_t v[VP_C_IN];
#pragma unroll
    for (int c = 0; c < VP_C_IN; ++c) v[c] = 0;
    for (int t = 0; t < N; ++t) {
        const float2 f = flow[(size_t)t * HW + j];
        v[2 * t] = isfinite(f.x) ? f2bf(f.x * (1.0f / VP_FLOW_SCALE)) : (uint16_t)0;
        v[2 * t + 1] = isfinite(f.y) ? f2bf(f.y * (1.0f / VP_FLOW_SCALE)) : (uint16_t)0;
    }
    u32x4* out = reinterpret_cast<u32x4*>(x + (size_t)j * VP_C_IN);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        u32x4 w;
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = (uint32_t)v[8 * q + 2 * e] | ((uint32_t)v[8 * q + 2 * e + 1] << 16);
        out[q] = w;
    }
}

// ---------------------------------------------------------------------------------------
// LDS-staged implicit-GEMM convolution (the fast path; same arithmetic roles as k_conv).
// Block tile BM pixels x BN output channels with 4 waves arranged WAVES_M x (4 / WAVES_M);
// a wave owns (32 WM) x (32 WN) (WM * WN accumulators).  K is walked in chunks of KC
// channels of one tap; the A chunk (BM x KC) and the B chunk (BN x KC) are staged in LDS
// with 16-byte loads, double buffered: the next chunk's global loads are in flight while
// the matrix cores work on the current one.
// ---------------------------------------------------------------------------------------
template <int WAVES_M, int WM, int WN, int KC, int MODE>
__global__ void __launch_bounds__(256) k_conv2(ConvArgs a) {
    constexpr int WAVES_N = 4 / WAVES_M;
    constexpr int BM = WAVES_M * 32 * WM, BN = WAVES_N * 32 * WN;
    constexpr int LD = KC + 8;                         // padded LDS row (bf16 elements)
    constexpr int QA = KC / 8;                         // 16-byte units per row
    constexpr int UA = (BM * QA + 255) / 256, UB = (BN * QA + 255) / 256;
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WAVES_M) * 32 * WM, wn0 = (wave / WAVES_M) * 32 * WN;
    const int Mpix = a.Ho * a.Wo;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kchunks = a.Cin / KC, nchunks = 9 * kchunks;

    // the rows (pixels / output channels) this thread stages
    int a_oy[UA], a_ox[UA];
    bool a_pv[UA];
#pragma unroll
    for (int i = 0; i < UA; ++i) {
        const int u = tid + 256 * i, r = u / QA;
        const int m = m0 + r;
        a_pv[i] = (u < BM * QA) && (m < Mpix);
        a_oy[i] = a_pv[i] ? m / a.Wo : 0;
        a_ox[i] = a_pv[i] ? m - a_oy[i] * a.Wo : 0;
    }
    u32x4 ra[UA], rb[UB];
    auto load_chunk = [&](int c) {
        const int tap = c / kchunks, c0 = (c - tap * kchunks) * KC;
        const int ky = tap / 3, kx = tap - 3 * ky;
#pragma unroll
        for (int i = 0; i < UA; ++i) {
            const int u = tid + 256 * i, q = u % QA;
            int sy, sx;
            bool ok = a_pv[i];
            if (MODE == 0) {
                sy = a_oy[i] * a.stride + ky - 1;
                sx = a_ox[i] * a.stride + kx - 1;
                ok = ok && sy >= 0 && sy < a.Hs && sx >= 0 && sx < a.Ws;
                if (a.up) { sy >>= 1; sx >>= 1; }
            } else {
                sy = a_oy[i] + 1 - ky;
                sx = a_ox[i] + 1 - kx;
                if (a.stride == 2) {
                    ok = ok && !(sy & 1) && !(sx & 1);
                    sy >>= 1;
                    sx >>= 1;
                }
                ok = ok && sy >= 0 && sy < a.Hs && sx >= 0 && sx < a.Ws;
            }
            ra[i] = ok ? *reinterpret_cast<const u32x4*>(a.x + ((size_t)sy * a.Wx + sx) * a.Cin + c0 + 8 * q)
                       : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int i = 0; i < UB; ++i) {
            const int u = tid + 256 * i, r = u / QA, q = u % QA;
            const int n = n0 + r;
            const bool ok = (u < BN * QA) && (n < a.Cout);
            rb[i] = ok ? *reinterpret_cast<const u32x4*>(a.w + ((size_t)n * 9 + tap) * a.Cin + c0 + 8 * q)
                       : u32x4{0u, 0u, 0u, 0u};
        }
    };
    auto store_chunk = [&](int st) {
#pragma unroll
        for (int i = 0; i < UA; ++i) {
            const int u = tid + 256 * i;
            if (u < BM * QA) *reinterpret_cast<u32x4*>(&As[st][(u / QA) * LD + 8 * (u % QA)]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < UB; ++i) {
            const int u = tid + 256 * i;
            if (u < BN * QA) *reinterpret_cast<u32x4*>(&Bs[st][(u / QA) * LD + 8 * (u % QA)]) = rb[i];
        }
    };

    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int st = c & 1;
        if (c + 1 < nchunks) load_chunk(c + 1);
#pragma unroll
        for (int kk = 0; kk < KC / 16; ++kk) {
            const int col = 16 * kk + 8 * (lane >> 5);
            bf16x8 A[WM], B[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i)
                A[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(
                                                      &As[st][(wm0 + 32 * i + (lane & 31)) * LD + col]));
#pragma unroll
            for (int j = 0; j < WN; ++j)
                B[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(
                                                      &Bs[st][(wn0 + 32 * j + (lane & 31)) * LD + col]));
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i], B[j], acc[i][j], 0, 0, 0);
        }
        if (c + 1 < nchunks) store_chunk(st ^ 1);
        __syncthreads();
    }

    // epilogue: lane holds D[i][j = lane%32] for rows i = 8(e/4) + 4(lane/32) + e%4
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int n = n0 + wn0 + 32 * j + (lane & 31);
        if (n >= a.Cout) continue;
        const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int mm = m0 + wm0 + 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                if (mm >= Mpix) continue;
                const size_t o = (size_t)mm * a.Cout + n;
                float v = acc[i][j][e] + bias;
                if (a.skip) v += bf2f(a.skip[o]);
                if (a.addf) v += a.addf[o];
                if (a.relu) v = fmaxf(v, 0.f);
                if (a.mask && !(bf2f(a.mask[o]) > 0.f)) v = 0.f;
                if (a.y) a.y[o] = f2bf(v);
                if (a.yf) a.yf[o] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Stride-1 convolution from an LDS halo tile (the fast path of stride-1 layers).  A block
// owns TH output rows x 32 output columns x BN output channels; a wave owns WM of those rows
// (each an MFMA M tile of 32 pixels: lane % 32 is the column) and WN tiles of 32 channels.
// Per chunk of KC input channels the block stages the (TH + 2) x 34 input halo and the
// weights of all 9 taps in LDS once, and every tap's A operand is read from the halo
// shifted by the tap: 9 x KC/16 MFMA steps per wave per chunk instead of KC/16, and each
// input pixel is fetched about 1.3 times instead of 9.  MODE 0: forward; with UP the source
// is read through a 2x nearest upsampling, and the halo holds the (TH/2 + 2) x 18 source
// pixels under the tile, each tap reading the pixel its upsampled position falls on;
// MODE 1: data gradient (taps flipped, transposed weights).  The next chunk's global
// loads are in flight while the matrix cores work.
// ---------------------------------------------------------------------------------------
template <int WAVES_M, int WM, int WN, int KC, int MODE, bool UP, int S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_conv_halo(ConvArgs a) {
    constexpr int WAVES_N = 4 / WAVES_M;
    constexpr int TW = 32, TH = WAVES_M * WM, BN = WAVES_N * 32 * WN;
    static_assert(!UP || (MODE == 0 && TH % 2 == 0 && S == 1), "upsampling: forward, even tile rows");
    static_assert(S == 1 || S == 2, "stride 1 or 2");
    // SUB: data gradient of a stride-2 layer by sub-pixel classes.  Output (2y' + py, 2x' + px)
    // takes tap (ky, kx) only where py + 1 - ky and px + 1 - kx are even, from gradient pixel
    // (y' + (py + 1 - ky) / 2, x' + (px + 1 - kx) / 2): per class (blockIdx.z = 2 py + px) a
    // stride-1 problem with 1, 2, 2 or 4 taps on tiles of the class's sub-grid.
    constexpr bool SUB = MODE == 1 && S == 2;
    // halo columns, rows: a tile of TW outputs at stride S reads S (TW - 1) + 3 source columns;
    // a SUB tile reads TW + 1
    constexpr int HX = SUB ? TW + 1 : (UP ? TW / 2 + 2 : S * (TW - 1) + 3);
    constexpr int HY = SUB ? TH + 1 : (UP ? TH / 2 + 2 : S * (TH - 1) + 3);
    constexpr int LD = KC + 8;                         // padded LDS pixel / weight row (bf16)
    constexpr int QA = KC / 8;                         // 16-byte units per pixel / weight row
    constexpr int NA = HY * HX * QA, NB = 9 * BN * QA; // 16-byte units of one chunk
    constexpr int UA = (NA + 255) / 256, UB = (NB + 255) / 256;
    constexpr unsigned kOut = 0x7ffffff0u;             // beyond any buffer: the load returns zeros
    // the halo and the weights of a chunk; after the last chunk the same LDS holds the tile's
    // skip input, staged with 16-byte loads, or its FP32 outputs for the heads
    // heads: stride-1 forward blocks of 32 output channels
    constexpr bool HEADS = MODE == 0 && !UP && S == 1 && BN == 32;
    constexpr int NHS = HY * HX * LD, NBS = 9 * BN * LD, NSK = TH * TW * BN, NHD = HEADS ? TH * TW * (BN + 1) * 2 : 0;
    constexpr int NLDS = (NHS + NBS) > NSK ? ((NHS + NBS) > NHD ? NHS + NBS : NHD) : (NSK > NHD ? NSK : NHD);
    __shared__ __attribute__((aligned(16))) uint16_t lds_u16[NLDS];
    uint16_t* const Hs = lds_u16;
    uint16_t* const Bs = lds_u16 + NHS;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr0 = (wave % WAVES_M) * WM, wn0 = (wave / WAVES_M) * 32 * WN;
    const int ntx = ((SUB ? (a.Wo + 1) / 2 : a.Wo) + TW - 1) / TW;
    const int ox0 = (int)(blockIdx.x % (unsigned)ntx) * TW, oy0 = (int)(blockIdx.x / (unsigned)ntx) * TH;
    const int py = SUB ? (int)(blockIdx.z >> 1) : 0, px = SUB ? (int)(blockIdx.z & 1) : 0;
    const int n0 = blockIdx.y * BN;
    const int nchunks = a.Cin / KC;

    // The units a thread stages do not depend on the chunk: byte offsets into the source and
    // weight arrays (kOut where the halo leaves the source grid or the channel tile leaves
    // Cout: buffer loads out of range return zeros) and LDS positions, computed once.  A
    // chunk moves the two buffer bases by KC channels.
    unsigned offA[UA], offB[UB];
    int ldsA[UA], ldsB[UB];
#pragma unroll
    for (int i = 0; i < UA; ++i) {
        const int u = tid + 256 * i;
        const int pix = u / QA, q = u - pix * QA;
        const int hy = pix / HX, hx = pix - hy * HX;
        // halo origin: the source pixel left of and above the tile's first tap (with UP, on
        // the stored grid, whose pixel covers upsampled positions 2s and 2s + 1)
        const int sy = SUB ? oy0 + hy : (UP ? oy0 / 2 + hy - 1 : S * oy0 + hy - 1);
        const int sx = SUB ? ox0 + hx : (UP ? ox0 / 2 + hx - 1 : S * ox0 + hx - 1);
        const bool ok = u < NA && sy >= 0 && sy < (UP ? a.Hx : a.Hs) && sx >= 0 && sx < (UP ? a.Wx : a.Ws);
        offA[i] = ok ? (unsigned)((((size_t)sy * a.Wx + sx) * a.Cin + 8 * q) * 2) : kOut;
        ldsA[i] = u < NA ? pix * LD + 8 * q : -1;
    }
#pragma unroll
    for (int i = 0; i < UB; ++i) {
        const int u = tid + 256 * i;
        const int row = u / QA, q = u - row * QA;       // row = tap * BN + local channel
        const int tap = row / BN, n = n0 + (row - tap * BN);
        // SUB: only the class's taps are used
        const bool in_class = !SUB || (!((py + 1 - tap / 3) & 1) && !((px + 1 - tap % 3) & 1));
        const bool ok = u < NB && n < a.Cout && in_class;
        offB[i] = ok ? (unsigned)((((size_t)n * 9 + tap) * a.Cin + 8 * q) * 2) : kOut;
        ldsB[i] = u < NB ? row * LD + 8 * q : -1;
    }
    const int bytesX = (int)min((size_t)0x7fffffff, (size_t)a.Hx * a.Wx * a.Cin * 2);
    const int bytesW = (int)min((size_t)0x7fffffff, (size_t)a.Cout * 9 * a.Cin * 2);

    u32x4 ra[UA], rb[UB];
    auto load_chunk = [&](int c) {
        const int cb = c * KC * 2;                      // chunk's byte shift within a pixel / row
        const __amdgpu_buffer_rsrc_t rx =
            __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)a.x + cb), (short)0, bytesX - cb, 0x00020000);
        const __amdgpu_buffer_rsrc_t rw =
            __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)a.w + cb), (short)0, bytesW - cb, 0x00020000);
#pragma unroll
        for (int i = 0; i < UA; ++i) ra[i] = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)offA[i], 0, 0);
#pragma unroll
        for (int i = 0; i < UB; ++i) rb[i] = __builtin_amdgcn_raw_buffer_load_b128(rw, (int)offB[i], 0, 0);
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int i = 0; i < UA; ++i)
            if (ldsA[i] >= 0) *reinterpret_cast<u32x4*>(&Hs[ldsA[i]]) = ra[i];
#pragma unroll
        for (int i = 0; i < UB; ++i)
            if (ldsB[i] >= 0) *reinterpret_cast<u32x4*>(&Bs[ldsB[i]]) = rb[i];
    };

    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

    const int col_lane = lane & 31, khalf = 8 * (lane >> 5);
    load_chunk(0);
    for (int c = 0; c < nchunks; ++c) {
        __syncthreads();                                // the previous chunk's reads are done
        store_chunk();
        __syncthreads();
        if (c + 1 < nchunks) load_chunk(c + 1);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int ky = tap / 3, kx = tap - 3 * (tap / 3);
            // forward: output (y, x) reads source (y + ky - 1, x + kx - 1) = halo (r + ky, col + kx);
            // data gradient: source (y + 1 - ky, x + 1 - kx) = halo (r + 2 - ky, col + 2 - kx);
            // UP: upsampled position (y + ky - 1) lies on stored row floor((y + ky - 1) / 2), halo
            // row floor((r + ky - 1) / 2) + 1 = (r + ky + 1) >> 1 (tile origin even), likewise columns
            if (SUB && (((py + 1 - ky) & 1) || ((px + 1 - kx) & 1))) continue;
            const int dy = SUB ? (py + 1 - ky) >> 1 : (MODE == 0 ? ky : 2 - ky);
            const int dx = SUB ? (px + 1 - kx) >> 1 : (MODE == 0 ? kx : 2 - kx);
            const int hcol = SUB ? col_lane + dx : (UP ? (col_lane + dx + 1) >> 1 : S * col_lane + dx);
#pragma unroll
            for (int kk = 0; kk < KC / 16; ++kk) {
                const int col = 16 * kk + khalf;
                bf16x8 A[WM], B[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i) {
                    const int hrow = SUB ? wr0 + i + dy : (UP ? (wr0 + i + dy + 1) >> 1 : S * (wr0 + i) + dy);
                    A[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&Hs[(hrow * HX + hcol) * LD + col]));
                }
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    B[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(
                                                          &Bs[(tap * BN + wn0 + 32 * j + col_lane) * LD + col]));
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[i], B[j], acc[i][j], 0, 0, 0);
            }
        }
    }

    // epilogue: lane holds D[i][j = lane % 32] of M tile (row) wr0 + t for columns
    // i = 8(e/4) + 4(lane/32) + e%4; the element offsets of the 16 columns are multiples of
    // Cout shared by every row and channel tile
    const bool full = !SUB && ox0 + TW <= a.Wo;
    // heads (first channel block, no skip input): the tile's FP32 outputs go to LDS as
    // [pixel][BN + 1] (padded against bank conflicts on the pixel reads)
    const bool heads = HEADS && a.hN > 0 && n0 == 0;
    float* const hv = reinterpret_cast<float*>(lds_u16);
    if (heads) __syncthreads();                         // every wave is done with the last chunk
    const bool plain = !a.addf && !a.mask && !a.yf && a.y && !heads;
    const int xb = ox0 + 4 * (lane >> 5);
    // skip input of the tile into LDS as [row][column][BN channels]: rows of BN channels are
    // contiguous in the source, so one 16-byte load per 8 channels (out of range: zeros)
    const bool skip_lds = MODE == 0 && a.skip;
    if (skip_lds) {
        __syncthreads();                                // every wave is done with the last chunk
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)a.skip, (short)0, (int)min((size_t)0x7fffffff, (size_t)a.Ho * a.Wo * a.Cout * 2), 0x00020000);
        constexpr int QS = BN / 8, NSU = TH * TW * QS;
#pragma unroll
        for (int i = 0; i < (NSU + 255) / 256; ++i) {
            const int u = tid + 256 * i;
            if (u >= NSU) break;
            const int px = u / QS, q = u - px * QS;
            const int r = px / TW, x = px - r * TW;
            const int oy = oy0 + r, ox = ox0 + x;
            const unsigned off = (oy < a.Ho && ox < a.Wo && n0 + 8 * q < a.Cout)
                                     ? (unsigned)((((size_t)oy * a.Wo + ox) * a.Cout + n0 + 8 * q) * 2) : kOut;
            *reinterpret_cast<u32x4*>(&lds_u16[px * BN + 8 * q]) = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
        }
        __syncthreads();
    }
    if constexpr (MODE == 1 && S == 1 && WM == 2) {
        if (a.pool) {
            // the data gradient of an upsampling layer: sums over 2 x 2 output blocks, which lie
            // in one lane (rows t = 0, 1 of an even tile row; columns e, e + 1 for e % 4 = 0, 2),
            // in the order (row 0 pair) + (row 1 pair); mask, y and yf on the half grid
            const int Hp = a.Ho / 2, Wp = a.Wo / 2, Y = (oy0 + wr0) / 2;
            // every mask value is read before the first store (the compiler cannot tell the
            // output from the mask, so a store would hold back every later load)
            uint32_t keep[WN];
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                const int n = n0 + wn0 + 32 * j + col_lane;
                keep[j] = 0xffffu;
                if (!a.mask || n >= a.Cout || Y >= Hp) continue;
#pragma unroll
                for (int e = 0; e < 16; e += 2) {
                    const int X = (xb + 8 * (e >> 2) + (e & 3)) / 2;
                    if (X < Wp && !(bf2f(a.mask[((size_t)Y * Wp + X) * a.Cout + n]) > 0.f)) keep[j] &= ~(1u << e);
                }
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                const int n = n0 + wn0 + 32 * j + col_lane;
                if (n >= a.Cout || Y >= Hp) continue;
                const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
                for (int e = 0; e < 16; e += 2) {
                    const int X = (xb + 8 * (e >> 2) + (e & 3)) / 2;
                    if (X >= Wp) continue;
                    const size_t o = ((size_t)Y * Wp + X) * a.Cout + n;
                    float v = ((acc[0][j][e] + bias) + (acc[0][j][e + 1] + bias)) +
                              ((acc[1][j][e] + bias) + (acc[1][j][e + 1] + bias));
                    if (!((keep[j] >> e) & 1u)) v = 0.f;
                    if (a.y) a.y[o] = __builtin_bit_cast(uint16_t, (__bf16)v);
                    if (a.yf) a.yf[o] = v;
                }
            }
            return;
        }
    }
    // data gradient: the mask and skip tiles go through LDS ([pixel][BN channels], 16-byte
    // loads; a SUB tile's outputs are every other pixel), the mask kept as one bit per element
    uint32_t keepbits[WM * WN];
#pragma unroll
    for (int i = 0; i < WM * WN; ++i) keepbits[i] = 0xffffu;
    if constexpr (MODE == 1) {
        const int bytesO = (int)min((size_t)0x7fffffff, (size_t)a.Ho * a.Wo * a.Cout * 2);
        auto stage = [&](const uint16_t* src) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, bytesO, 0x00020000);
            constexpr int QS = BN / 8, NSU = TH * TW * QS;
#pragma unroll
            for (int i = 0; i < (NSU + 255) / 256; ++i) {
                const int u = tid + 256 * i;
                if (u >= NSU) break;
                const int pix = u / QS, q = u - pix * QS;
                const int r = pix / TW, x = pix - r * TW;
                const int oy = SUB ? 2 * (oy0 + r) + py : oy0 + r, ox = SUB ? 2 * (ox0 + x) + px : ox0 + x;
                const unsigned off = (oy < a.Ho && ox < a.Wo && n0 + 8 * q < a.Cout)
                                         ? (unsigned)((((size_t)oy * a.Wo + ox) * a.Cout + n0 + 8 * q) * 2) : kOut;
                *reinterpret_cast<u32x4*>(&lds_u16[pix * BN + 8 * q]) = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
            }
        };
        if (a.mask) {
            __syncthreads();                            // every wave is done with the last chunk
            stage(a.mask);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int t = 0; t < WM; ++t) {
                    uint32_t b = 0;
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int dxe = 8 * (e >> 2) + (e & 3);
                        const uint16_t m = lds_u16[((wr0 + t) * TW + 4 * (lane >> 5) + dxe) * BN + wn0 + 32 * j + col_lane];
                        b |= (bf2f(m) > 0.f ? 1u : 0u) << e;
                    }
                    keepbits[j * WM + t] = b;
                }
        }
        if (a.skip) {
            __syncthreads();
            stage(a.skip);
            __syncthreads();
        }
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int nl = wn0 + 32 * j + col_lane, n = n0 + nl;
        if (n >= a.Cout) continue;
        const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
        for (int t = 0; t < WM; ++t) {
            const int oy = SUB ? 2 * (oy0 + wr0 + t) + py : oy0 + wr0 + t;
            if (oy >= a.Ho) continue;
            const size_t o0 = ((size_t)oy * a.Wo + xb) * a.Cout + n;
            if (plain && full) {
                uint16_t* yp = a.y + o0;
                const int sk0 = ((wr0 + t) * TW + 4 * (lane >> 5)) * BN + nl;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    float v = acc[t][j][e] + bias;
                    if (skip_lds) v += bf2f(lds_u16[sk0 + (8 * (e >> 2) + (e & 3)) * BN]);
                    if (a.relu) v = fmaxf(v, 0.f);
                    yp[(size_t)(8 * (e >> 2) + (e & 3)) * a.Cout] = __builtin_bit_cast(uint16_t, (__bf16)v);
                }
                continue;
            }
            if constexpr (MODE == 1) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int dxe = 8 * (e >> 2) + (e & 3);
                    const int ox = SUB ? 2 * (xb + dxe) + px : xb + dxe;
                    if (ox >= a.Wo) continue;
                    const size_t o = ((size_t)oy * a.Wo + ox) * a.Cout + n;
                    float v = acc[t][j][e] + bias;
                    if (a.skip) v += bf2f(lds_u16[((wr0 + t) * TW + 4 * (lane >> 5) + dxe) * BN + nl]);
                    if (a.addf) v += a.addf[o];
                    if (a.relu) v = fmaxf(v, 0.f);
                    if (!((keepbits[j * WM + t] >> e) & 1u)) v = 0.f;
                    if (a.y) a.y[o] = __builtin_bit_cast(uint16_t, (__bf16)v);
                    if (a.yf) a.yf[o] = v;
                }
                continue;
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int dxe = 8 * (e >> 2) + (e & 3);
                const int ox = xb + dxe;
                if (ox >= a.Wo) continue;
                const size_t o = ((size_t)oy * a.Wo + ox) * a.Cout + n;
                float v = acc[t][j][e] + bias;
                if (skip_lds) v += bf2f(lds_u16[((wr0 + t) * TW + 4 * (lane >> 5) + dxe) * BN + nl]);
                if (a.addf) v += a.addf[o];
                if (a.relu) v = fmaxf(v, 0.f);
                if (a.mask && !(bf2f(a.mask[o]) > 0.f)) v = 0.f;
                if (a.y) a.y[o] = __builtin_bit_cast(uint16_t, (__bf16)v);
                if (a.yf) a.yf[o] = v;
                if (heads) hv[((wr0 + t) * TW + 4 * (lane >> 5) + dxe) * (BN + 1) + nl] = v;
            }
        }
    }
    if (heads) {
        // one thread per pixel of the tile: rho from channel 0, q_t from channel 1 + t
        __syncthreads();
        float tn = a.htnorm;
        if (a.hpose) {
            const double t0 = a.hpose[3], t1 = a.hpose[4], t2 = a.hpose[5];
            tn = (float)sqrt(t0 * t0 + t1 * t1 + t2 * t2);
        }
        for (int p = tid; p < TH * TW; p += 256) {
            const int oy = oy0 + p / TW, ox = ox0 + p % TW;
            if (oy >= a.Ho || ox >= a.Wo) continue;
            const size_t px = (size_t)oy * a.Wo + ox;
            const float* hp = hv + p * (BN + 1);
            if (a.hrho) {
                // the learned start checks the scale and the logit; the plain forward clips
                // whatever comes
                const float v = hp[0];
                const bool ok = !a.hpose || (isfinite(tn) && tn > 0.f && isfinite(v));
                if (!ok && a.hflag) atomicOr(a.hflag, 1);
                a.hrho[px] = ok ? fminf(fmaxf(softplusf(v) / tn, a.hrmin), a.hrmax) : a.hrmin;
            }
            if (a.hq)
                for (int t = 0; t < a.hN; ++t) a.hq[(size_t)t * a.Ho * a.Wo + px] = sigmoidf(hp[1 + t]);
        }
    }
}

// ---------------------------------------------------------------------------------------
// weight gradient, LDS-staged: block = (CO_T output channels) x (32 input channels) x all 9
// taps x a chunk of output pixels.  D[co][ci] (one 32 x 32 tile per tap and 32 output
// channels) = sum over pixels m of dy[m][co] x_tap(m)[ci]: the contraction runs over pixels,
// so both operands are staged pixel-contiguous.  Per step of KP = 32 pixels a thread loads
// one unit, 8 pixels x 8 channels (eight 16-byte loads: dy rows, or the source pixels of one
// tap), transposes it in registers and writes 8 channel rows of 8 pixels to LDS:
// dy^T [CO_T][KP] and the im2col slices [9][32][KP].  The next step's loads are in flight
// while the matrix cores work.  The 9 CO_T / 32 output tiles are split evenly over the 4 waves.
// ---------------------------------------------------------------------------------------
template <int CO_T>
__global__ void __launch_bounds__(256) k_wgrad2(WgradArgs a) {
    constexpr int CI_T = 32, KP = 32, LDP = KP + 8;     // padded LDS row (bf16): 80 bytes
    constexpr int NT = 9 * (CO_T / 32), MAXT = (NT + 3) / 4;
    constexpr int NA = (CO_T / 8) * (KP / 8), NB = 9 * (CI_T / 8) * (KP / 8);
    static_assert(NA + NB <= 256, "one staging unit per thread");
    __shared__ __attribute__((aligned(16))) uint16_t As[CO_T * LDP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[9 * CI_T * LDP];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int co0 = blockIdx.x * CO_T, ci0 = blockIdx.y * CI_T;
    const int Wo = a.Wo, Hs = a.Hs, Ws = a.Ws, Wx = a.Wx, Cin = a.Cin, Cout = a.Cout;
    const int stride = a.stride, up = a.up;
    const int Mpix = a.Ho * Wo;
    const int chunk = (Mpix + gridDim.z - 1) / gridDim.z;
    const int mbeg = blockIdx.z * chunk, mend = min(Mpix, mbeg + chunk);

    // this thread's staging unit: an A unit (8 output channels g, 8 pixels p8) or a B unit
    // (tap, 8 input channels g, 8 pixels p8)
    const bool isA = tid < NA, isB = !isA && tid < NA + NB;
    const int ub = isA ? tid : tid - NA;
    const int tap = isA ? 0 : ub / ((CI_T / 8) * (KP / 8));
    const int ur = isA ? ub : ub - tap * ((CI_T / 8) * (KP / 8));
    const int g = isA ? ur % (CO_T / 8) : ur % (CI_T / 8);
    const int p8 = isA ? ur / (CO_T / 8) : ur / (CI_T / 8);
    const int ky = tap / 3, kx = tap - 3 * ky;
    const bool active = isA || (isB && ci0 + 8 * g < Cin);
    const int dst = isA ? (8 * g) * LDP + 8 * p8 : (tap * CI_T + 8 * g) * LDP + 8 * p8;
    uint16_t* const dstp = isA ? As + dst : Bs + dst;
    const uint16_t* const dyb = a.dy + co0 + 8 * g;
    const uint16_t* const xb = a.x + ci0 + 8 * g;

    u32x4 r[8];
    const int t0 = (wave * NT) / 4, t1 = ((wave + 1) * NT) / 4;
    f32x16 acc[MAXT];
#pragma unroll
    for (int i = 0; i < MAXT; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][e] = 0.f;
    const int col_lane = lane & 31, khalf = 8 * (lane >> 5);

    for (int m0 = mbeg - KP; m0 < mend; m0 += KP) {
        if (m0 >= mbeg) {
            // r[e] holds channels 0..7 of pixel e; row c of the unit: pixels 0..7 of channel c
            __syncthreads();                            // the previous step's reads are done
            if (isA || isB) {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    u32x4 w;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t lo = r[2 * q][c >> 1], hi = r[2 * q + 1][c >> 1];
                        w[q] = (c & 1) ? ((lo >> 16) | (hi & 0xffff0000u)) : ((lo & 0xffffu) | (hi << 16));
                    }
                    *reinterpret_cast<u32x4*>(dstp + c * LDP) = w;
                }
            }
            __syncthreads();
        }
        // the next step's unit: eight 16-byte loads (zeros off the chunk, the grid or Cin)
        const int mn = m0 + KP;
        if (mn < mend) {
            const int mf = mn + 8 * p8;
            int oy = mf / Wo, ox = mf - oy * Wo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int m = mf + e;
                int sy = oy * stride + ky - 1, sx = ox * stride + kx - 1;
                const bool ok = active && m < mend && (isA || (sy >= 0 && sy < Hs && sx >= 0 && sx < Ws));
                if (up) { sy >>= 1; sx >>= 1; }
                const size_t off = isA ? (size_t)m * Cout : ((size_t)sy * Wx + sx) * Cin;
                r[e] = ok ? *reinterpret_cast<const u32x4*>((isA ? dyb : xb) + off) : u32x4{0u, 0u, 0u, 0u};
                if (++ox == Wo) { ox = 0; ++oy; }
            }
        }
        if (m0 < mbeg) continue;
#pragma unroll
        for (int kk = 0; kk < KP / 16; ++kk) {
            const int col = 16 * kk + khalf;
#pragma unroll
            for (int i = 0; i < MAXT; ++i) {
                const int t = t0 + i;
                if (t >= t1) break;
                const int c = t / 9, tp = t - 9 * c;
                const bf16x8 A = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(
                                                            &As[(32 * c + col_lane) * LDP + col]));
                const bf16x8 B = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(
                                                            &Bs[(tp * CI_T + col_lane) * LDP + col]));
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[i], 0, 0, 0);
            }
        }
    }

    // lane holds D[co = 32 c + 8(e/4) + 4(lane/32) + e%4][ci = lane % 32]
    float* const part = a.part + (size_t)blockIdx.z * a.nparam;
#pragma unroll
    for (int i = 0; i < MAXT; ++i) {
        const int t = t0 + i;
        if (t >= t1) break;
        const int c = t / 9, tp = t - 9 * c;
        const int ci = ci0 + col_lane;
        if (ci >= Cin) continue;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int co = co0 + 32 * c + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
            part[((size_t)co * 9 + tp) * Cin + ci] = acc[i][e];
        }
    }
}

// bias gradient partials: block b sums the pixels [b chunk, (b + 1) chunk) of dy [Mpix][C].
// Thread t takes the 8 channels of group g = t % G (G = C / 8; one 16-byte load per pixel)
// on the pixels mbeg + p, mbeg + p + P, ... (p = t / G, P = 256 / G); the P sums of a
// channel are added in LDS in a fixed order.
__global__ void __launch_bounds__(256) k_bgrad(const uint16_t* __restrict__ dy, int Mpix, int C, int nchunks,
                                               float* __restrict__ part) {
    extern __shared__ float red_b[];                    // [P][C]
    const int G = C / 8, P = 256 / G;
    const int t = threadIdx.x, g = t % G, pl = t / G;
    const int chunk = (Mpix + nchunks - 1) / nchunks;
    const int mbeg = blockIdx.x * chunk, mend = min(Mpix, mbeg + chunk);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (pl < P) {
        for (int m = mbeg + pl; m < mend; m += P) {
            const u32x4 v = *reinterpret_cast<const u32x4*>(dy + (size_t)m * C + 8 * g);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[2 * e] += __uint_as_float(v[e] << 16);
                acc[2 * e + 1] += __uint_as_float(v[e] & 0xffff0000u);
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) red_b[pl * C + 8 * g + e] = acc[e];
    }
    __syncthreads();
    for (int c = t; c < C; c += 256) {
        float s = 0.f;
        for (int q = 0; q < P; ++q) s += red_b[q * C + c];
        part[(size_t)blockIdx.x * C + c] = s;
    }
}

// out[i] = sum over chunks of part[chunk][i] in a fixed order: block = 64 outputs x 16 rows,
// row r sums the chunks r, r + 16, ..., then the 16 row sums are added in order
__global__ void __launch_bounds__(1024) k_sum_chunks(const float* __restrict__ part, int n, int nchunks,
                                                     float* __restrict__ out) {
    __shared__ float red[16][64];
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + x;
    float s = 0.f;
    if (i < n)
        for (int c = y; c < nchunks; c += 16) s += part[(size_t)c * n + i];
    red[y][x] = s;
    __syncthreads();
    if (y == 0 && i < n) {
        float t = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) t += red[r][x];
        out[i] = t;
    }
}

// ---------------------------------------------------------------------------------------
// learned start of a GEM window: the heads fused into the last layer take tnorm = |t| of
// frame 1's pose (FP64, on the device); a non-finite depth logit or an unusable tnorm raises
// the window's fallback flag (cleared here beforehand), in which case the caller's random
// start replaces every pixel
// ---------------------------------------------------------------------------------------
__global__ void k_flag_clear(int* __restrict__ flag) { *flag = 0; }

hipError_t launch_flag_clear(int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(1), 0, st, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// loss: L = mean_mask |softplus(o_0) - rho_t tnorm| + lam mean BCE(sigmoid(o_t), q_t); its
// gradient w.r.t. o (BF16, zero on unused channels) and per-block FP64 partial sums
// [L1 sum, mask count, BCE sum]
// ---------------------------------------------------------------------------------------
// number of masked pixels in each 4096-byte span of the mask (one block per span, 16 bytes per
// thread); integer partial counts, so their sum is exact in any order
__global__ void __launch_bounds__(256) k_mask_count(const uint8_t* __restrict__ mask, int HW, int* __restrict__ cnt) {
    __shared__ int red[4];
    const int j0 = (blockIdx.x * 256 + threadIdx.x) * 16;
    int c = 0;
    if (j0 + 16 <= HW && (reinterpret_cast<uintptr_t>(mask) & 15) == 0) {
        const u32x4 v = *reinterpret_cast<const u32x4*>(mask + j0);
        // a byte b is non-zero iff the top bit of ((b & 0x7f) + 0x7f) | b is set (no carry
        // leaves the byte)
#pragma unroll
        for (int e = 0; e < 4; ++e) c += __popc((((v[e] & 0x7f7f7f7fu) + 0x7f7f7f7fu) | v[e]) & 0x80808080u);
    } else {
        for (int j = j0; j < min(HW, j0 + 16); ++j) c += mask[j] != 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_loss(const float* __restrict__ o, int HW, int N, float tnorm, const float* __restrict__ rho_t,
                       const float* __restrict__ q_t, const uint8_t* __restrict__ mask, float lam,
                       const int* __restrict__ mcnt, int ncnt, uint16_t* __restrict__ dout, double* __restrict__ part) {
    __shared__ double red[3][4];
    __shared__ float inv_s;
    if (threadIdx.x < 64) {                             // 1 / max(1, masked pixels)
        int c = 0;
        for (int i = threadIdx.x; i < ncnt; i += 64) c += mcnt[i];
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
        if (threadIdx.x == 0) inv_s = 1.0f / (float)max(c, 1);
    }
    __syncthreads();
    const float inv_cnt = inv_s;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double l1 = 0.0, cnt = 0.0, bce = 0.0;
    if (j < HW) {
        // logits 0 .. N (N <= 8) as three 16-byte loads; the gradient row (32 BF16, zero past
        // channel N) as four 16-byte stores
        const float4* o4 = reinterpret_cast<const float4*>(o + (size_t)j * VP_C_HEAD);
        const float4 l0 = o4[0], l1v = o4[1], l2 = o4[2];
        const float z[9] = {l0.x, l0.y, l0.z, l0.w, l1v.x, l1v.y, l1v.z, l1v.w, l2.x};
        uint32_t wd[VP_C_HEAD / 2];
#pragma unroll
        for (int k = 0; k < VP_C_HEAD / 2; ++k) wd[k] = 0u;
        const float s = softplusf(z[0]);
        const float d = s - rho_t[j] * tnorm;
        const bool mk = mask[j] != 0;
        float g0 = 0.f;
        if (mk) {
            l1 = fabs((double)d);
            cnt = 1.0;
            g0 = (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) * sigmoidf(z[0]) * inv_cnt;
        }
        wd[0] = f2bf(g0);
        const float inv_q = lam / (float)((size_t)N * HW);
#pragma unroll
        for (int c = 1; c <= 8; ++c) {
            if (c > N) break;
            const float zc = z[c], qt = q_t[(size_t)(c - 1) * HW + j];
            bce += (double)(softplusf(zc) - qt * zc);
            const uint32_t h = f2bf((sigmoidf(zc) - qt) * inv_q);
            wd[c >> 1] |= (c & 1) ? (h << 16) : h;
        }
        u32x4* dq = reinterpret_cast<u32x4*>(dout + (size_t)j * VP_C_HEAD);
#pragma unroll
        for (int q = 0; q < VP_C_HEAD / 8; ++q) dq[q] = u32x4{wd[4 * q], wd[4 * q + 1], wd[4 * q + 2], wd[4 * q + 3]};
    }
    double v[3] = {l1, cnt, bce};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    }
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 3; ++k) red[k][threadIdx.x >> 6] = v[k];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        part[(size_t)k * gridDim.x + blockIdx.x] = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
    }
}

// loss[0] = L, loss[1] = L1 part, loss[2] = BCE part: one block of 256 threads, thread t sums
// the partials t, t + 256, ... and the 256 sums are added pairwise in LDS (a fixed order)
__global__ void __launch_bounds__(256) k_loss_finish(const double* __restrict__ part, int nb, int N, int HW,
                                                     float lam, double* __restrict__ loss) {
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    for (int k = 0; k < 3; ++k) {
        double a = 0.0;
        for (int b = t; b < nb; b += 256) a += part[(size_t)k * nb + b];
        red[k][t] = a;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int k = 0; k < 3; ++k) red[k][t] += red[k][t + h];
        __syncthreads();
    }
    if (t != 0) return;
    const double s[3] = {red[0][0], red[1][0], red[2][0]};
    const double l1 = s[0] / fmax(s[1], 1.0), bce = s[2] / ((double)N * HW);
    loss[0] = l1 + (double)lam * bce;
    loss[1] = l1;
    loss[2] = bce;
}

// ---------------------------------------------------------------------------------------
// Adam on the FP32 master parameters; refreshes the BF16 weights and their transposed copy
// ---------------------------------------------------------------------------------------
__global__ void k_adam(AdamArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= VP_NPARAM) return;
    float p = a.params[i];
    if (a.grads) {
        const float g = a.grads[i];
        const float m = fmaf(a.b1, a.m[i], (1.f - a.b1) * g);
        const float v = fmaf(a.b2, a.v[i], (1.f - a.b2) * g * g);
        a.m[i] = m;
        a.v[i] = v;
        p -= a.lr * (m * a.inv_bc1) / (sqrtf(v * a.inv_bc2) + a.eps);
        a.params[i] = p;
    }
    const uint16_t h = f2bf(p);
    a.wbf[i] = h;
    // transposed copy of a weight: [co][tap][ci] -> [ci][tap][co] within its layer
    int L = 0;
    while (L + 1 < VP_NLAYERS && i >= c_layer_off[L + 1]) ++L;
    const int r = i - c_layer_off[L];
    const int ci_n = c_layer_cin[L], co_n = c_layer_cout[L];
    if (r < co_n * 9 * ci_n && a.wt) {
        const int co = r / (9 * ci_n), rr = r - co * 9 * ci_n, tap = rr / ci_n, ci = rr - tap * ci_n;
        a.wt[c_layer_off[L] + ((size_t)ci * 9 + tap) * co_n + co] = h;
    }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------

hipError_t launch_features(const float* flow, int N, int HW, uint16_t* x, hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3((HW + 255) / 256), dim3(256), 0, st, (const float2*)flow, N, HW, x);
    return hipGetLastError();
}

template <int WAVES_M, int WM, int WN, int KC>
static void conv2_launch(const ConvArgs& a, int mode, hipStream_t st) {
    constexpr int BM = WAVES_M * 32 * WM, BN = (4 / WAVES_M) * 32 * WN;
    const int Mpix = a.Ho * a.Wo;
    const dim3 grid((unsigned)((Mpix + BM - 1) / BM), (unsigned)((a.Cout + BN - 1) / BN));
    if (mode == 0) hipLaunchKernelGGL((k_conv2<WAVES_M, WM, WN, KC, 0>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_conv2<WAVES_M, WM, WN, KC, 1>), grid, dim3(256), 0, st, a);
}

// S = 1: stride 1 (forward, upsampling forward or data gradient); 2: stride-2 forward;
// -2: data gradient of a stride-2 layer by sub-pixel classes
template <int WAVES_M, int WM, int WN, int KC, int S>
static void halo_launch(const ConvArgs& a, int mode, hipStream_t st) {
    constexpr int TH = WAVES_M * WM, BN = (4 / WAVES_M) * 32 * WN;
    const dim3 grid((unsigned)(((a.Wo + 31) / 32) * ((a.Ho + TH - 1) / TH)), (unsigned)((a.Cout + BN - 1) / BN));
    if constexpr (S == 2) {
        hipLaunchKernelGGL((k_conv_halo<WAVES_M, WM, WN, KC, 0, false, 2>), grid, dim3(256), 0, st, a);
    } else if constexpr (S == -2) {
        // sub-pixel data gradient: tiles of the largest class's grid, one z slice per class
        const int Hq = (a.Ho + 1) / 2, Wq = (a.Wo + 1) / 2;
        const dim3 gq((unsigned)(((Wq + 31) / 32) * ((Hq + TH - 1) / TH)), (unsigned)((a.Cout + BN - 1) / BN), 4u);
        hipLaunchKernelGGL((k_conv_halo<WAVES_M, WM, WN, KC, 1, false, 2>), gq, dim3(256), 0, st, a);
    } else {
        if (mode == 1) hipLaunchKernelGGL((k_conv_halo<WAVES_M, WM, WN, KC, 1, false, 1>), grid, dim3(256), 0, st, a);
        else if (a.up) hipLaunchKernelGGL((k_conv_halo<WAVES_M, WM, WN, KC, 0, true, 1>), grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_conv_halo<WAVES_M, WM, WN, KC, 0, false, 1>), grid, dim3(256), 0, st, a);
    }
}

// Stride-1 layers (forward with or without upsampling; data gradient without): the halo
// kernel, blocks of 8 rows x 32 columns x 64 channels (chunks of 16 input channels; 128
// output channels take two such blocks per tile, which keeps 3 blocks per CU) or x 32
// channels (chunks of 32).
static bool launch_halo(const ConvArgs& a, int mode, hipStream_t st) {
    if ((mode == 1 && a.up) || (a.up && (a.stride != 1 || a.Hs != 2 * a.Hx || a.Ws != 2 * a.Wx))) return false;
    // heads: stride-1 forward, 32 output channels (one 32-channel block), no skip input
    if (a.hN > 0 && (mode != 0 || a.up || a.stride != 1 || a.skip || a.Cout != 32 || a.hN >= a.Cout)) return false;
    // pooled data gradient: stride 1, even output grid, no skip / addend / activation
    if (a.pool && (mode != 1 || a.up || a.stride != 1 || (a.Ho & 1) || (a.Wo & 1) || a.skip || a.addf || a.relu))
        return false;
    if (a.stride == 2) {
        if (a.Cout % 64 != 0) return false;
        if (mode == 1) halo_launch<4, 2, 2, 16, -2>(a, mode, st);   // sub-pixel classes
        else halo_launch<4, 1, 2, 16, 2>(a, mode, st);              // 4-row tiles: 2 x 32 + 1 halo columns
        return true;
    }
    if (a.Cout % 64 == 0) halo_launch<4, 2, 2, 16, 1>(a, mode, st);
    else if (a.Cin % 32 == 0) halo_launch<4, 2, 1, 32, 1>(a, mode, st);
    else halo_launch<4, 2, 1, 16, 1>(a, mode, st);
    return true;
}

// LDS-staged kernel: block 128 x 128 (Cout multiple of 128), 256 x 64 (Cout multiple of 64)
// or 256 x 32; chunks of 32 channels (16 when Cin is not a multiple of 32)
static void launch_conv2(const ConvArgs& a, int mode, hipStream_t st) {
    const bool k32 = (a.Cin % 32) == 0;
    if (a.Cout % 128 == 0) {
        if (k32) conv2_launch<2, 2, 2, 32>(a, mode, st); else conv2_launch<2, 2, 2, 16>(a, mode, st);
    } else if (a.Cout % 64 == 0) {
        if (k32) conv2_launch<4, 2, 2, 32>(a, mode, st); else conv2_launch<4, 2, 2, 16>(a, mode, st);
    } else {
        if (k32) conv2_launch<4, 2, 1, 32>(a, mode, st); else conv2_launch<4, 2, 1, 16>(a, mode, st);
    }
}

hipError_t launch_conv(const ConvArgs& a, int mode, hipStream_t st) {
    if (launch_halo(a, mode, st)) return hipGetLastError();
    if (a.hN > 0 || a.pool) return hipErrorInvalidValue;  // fused heads, pooling: the halo kernel only
    launch_conv2(a, mode, st);
    return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& a, int nchunks, hipStream_t st) {
    // 16-byte channel groups: both arrays 16-byte aligned, Cin a multiple of 8
    if (((reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.dy)) & 15) != 0 || a.Cin % 8 != 0)
        return hipErrorInvalidValue;
    const int cot = wgrad_co_tile(a.Cout);
    const dim3 grid((unsigned)(a.Cout / cot), (unsigned)((a.Cin + 31) / 32), (unsigned)nchunks);
    if (cot == 128) hipLaunchKernelGGL(k_wgrad2<128>, grid, dim3(256), 0, st, a);
    else if (cot == 64) hipLaunchKernelGGL(k_wgrad2<64>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_wgrad2<32>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_bgrad(const uint16_t* dy, int Mpix, int C, int nchunks, float* part, hipStream_t st) {
    if (C % 8 != 0 || C > 2048 || (reinterpret_cast<uintptr_t>(dy) & 15) != 0) return hipErrorInvalidValue;
    const int P = 256 / (C / 8);
    hipLaunchKernelGGL(k_bgrad, dim3((unsigned)nchunks), dim3(256), (size_t)P * C * sizeof(float), st, dy, Mpix, C,
                       nchunks, part);
    return hipGetLastError();
}

hipError_t launch_sum_chunks(const float* part, int n, int nchunks, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((n + 63) / 64)), dim3(1024), 0, st, part, n, nchunks, out);
    return hipGetLastError();
}

hipError_t launch_loss(const float* o, int HW, int N, float tnorm, const float* rho_t, const float* q_t,
                       const uint8_t* mask, float lam, int* cnt, uint16_t* dout, double* part, double* loss,
                       hipStream_t st) {
    const int nb = (HW + 255) / 256, ncnt = mask_count_blocks(HW);
    hipLaunchKernelGGL(k_mask_count, dim3(ncnt), dim3(256), 0, st, mask, HW, cnt);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, st, o, HW, N, tnorm, rho_t, q_t, mask, lam,
                       (const int*)cnt, ncnt, dout, part);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, st, part, nb, N, HW, lam, loss);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((VP_NPARAM + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace vp
