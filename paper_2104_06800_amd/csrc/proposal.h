// Internal interface of the proposal-network kernels (architecture constants, kernel
// arguments and launchers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define VP_C_IN 16          // input feature channels (2N real, N <= 8)
#define VP_C_HEAD 32        // output channels (1 + N real)
#define VP_NLAYERS 6
#define VP_FLOW_SCALE 16.0f
#define VP_NPARAM 470560    // FP32 parameters of c1..c6: w [Cout][3][3][Cin] then b [Cout]

namespace vp {

// layer table: c1 16->64, c2 64->128 (stride 2), c3 128->128, c4 128->128,
// c5 128->64 (input upsampled 2x, + a1 before the ReLU), c6 64->32 (linear)
constexpr int kLayerCin[VP_NLAYERS] = {16, 64, 128, 128, 128, 64};
constexpr int kLayerCout[VP_NLAYERS] = {64, 128, 128, 128, 64, 32};
constexpr int kLayerStride[VP_NLAYERS] = {1, 2, 1, 1, 1, 1};
constexpr int kLayerUp[VP_NLAYERS] = {0, 0, 0, 0, 1, 0};
constexpr int kLayerRelu[VP_NLAYERS] = {1, 1, 1, 1, 1, 0};

constexpr int layer_size(int L) { return kLayerCout[L] * 9 * kLayerCin[L] + kLayerCout[L]; }
constexpr int layer_off(int L) { return L == 0 ? 0 : layer_off(L - 1) + layer_size(L - 1); }
static_assert(layer_off(VP_NLAYERS - 1) + layer_size(VP_NLAYERS - 1) == VP_NPARAM, "parameter count");

__constant__ static const int c_layer_off[VP_NLAYERS] = {layer_off(0), layer_off(1), layer_off(2),
                                                         layer_off(3), layer_off(4), layer_off(5)};
__constant__ static const int c_layer_cin[VP_NLAYERS] = {16, 64, 128, 128, 128, 64};
__constant__ static const int c_layer_cout[VP_NLAYERS] = {64, 128, 128, 128, 64, 32};

struct ConvArgs {
    int Hs, Ws;              // source grid read by the kernel (MODE 0 with up: the 2x grid)
    int Hx, Wx;              // stored source array dims (row pitch Wx)
    int Cin;                 // source channels (multiple of 16)
    int Ho, Wo, Cout;        // output grid and channels (Cout multiple of 32)
    int stride, up, relu;
    const uint16_t* x;       // [Hx][Wx][Cin] BF16
    const uint16_t* w;       // [Cout][3][3][Cin] BF16
    const float* bias;       // [Cout] or null
    const uint16_t* skip;    // [Ho][Wo][Cout] BF16 added before the activation, or null
    const float* addf;       // [Ho][Wo][Cout] FP32 added before the activation, or null
    const uint16_t* mask;    // [Ho][Wo][Cout] BF16: output zeroed where mask <= 0, or null
    uint16_t* y;             // BF16 output or null
    float* yf;               // FP32 output or null
    // heads fused into the last layer (stride-1 forward, hN > 0): rho [Ho][Wo] from channel 0,
    // q [hN][Ho][Wo] from channels 1 .. hN (either may be null); the depth scale is |t| of
    // hpose (FP64 pose; a non-finite scale or logit sets *hflag, when given, and gives hrmin)
    // or htnorm when hpose is null
    int hN;
    float htnorm, hrmin, hrmax;
    // data gradient of an upsampling layer (MODE 1, stride 1, even Ho and Wo): the result
    // summed over 2 x 2 blocks onto the (Ho / 2) x (Wo / 2) grid, where mask, y and yf live
    int pool;
    float* hrho;
    float* hq;
    const double* hpose;
    int* hflag;
};

struct WgradArgs {
    int Hs, Ws, Hx, Wx, Cin; // forward source (as in ConvArgs MODE 0)
    int Ho, Wo, Cout;        // forward output grid
    int stride, up;
    const uint16_t* x;       // forward input [Hx][Wx][Cin]
    const uint16_t* dy;      // gradient of the forward output (pre-activation) [Ho][Wo][Cout]
    float* part;             // [chunks][nparam] partials, weight part [Cout][9][Cin]
    int nparam;              // stride of a chunk in part (= Cout * 9 * Cin)
};

struct AdamArgs {
    float* params;           // [VP_NPARAM] FP32 master
    const float* grads;      // [VP_NPARAM] or null (then only the BF16 copies are refreshed)
    float* m;
    float* v;
    uint16_t* wbf;           // [VP_NPARAM] BF16 copy ([Cout][3][3][Cin] per layer)
    uint16_t* wt;            // [VP_NPARAM] BF16 transposed weights ([Cin][3][3][Cout] per layer) or null
    float lr, b1, b2, eps, inv_bc1, inv_bc2;
};

hipError_t launch_features(const float* flow, int N, int HW, uint16_t* x, hipStream_t st);
hipError_t launch_conv(const ConvArgs& a, int mode, hipStream_t st);
// output channels per block of the staged weight-gradient kernel (32 input channels, 9 taps)
inline int wgrad_co_tile(int Cout) { return Cout % 128 == 0 ? 128 : (Cout % 64 == 0 ? 64 : 32); }
hipError_t launch_wgrad(const WgradArgs& a, int nchunks, hipStream_t st);
hipError_t launch_bgrad(const uint16_t* dy, int Mpix, int C, int nchunks, float* part, hipStream_t st);
hipError_t launch_sum_chunks(const float* part, int n, int nchunks, float* out, hipStream_t st);
hipError_t launch_flag_clear(int* flag, hipStream_t st);
// blocks of the mask count (4096 mask bytes each): the loss's count buffer holds that many ints
inline int mask_count_blocks(int HW) { return (HW + 4095) / 4096; }
hipError_t launch_loss(const float* o, int HW, int N, float tnorm, const float* rho_t, const float* q_t,
                       const uint8_t* mask, float lam, int* cnt, uint16_t* dout, double* part, double* loss,
                       hipStream_t st);
hipError_t launch_adam(const AdamArgs& a, hipStream_t st);


}  // namespace vp
