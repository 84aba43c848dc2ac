// C ABI of the learned proposal network: argument checks, workspace layout and the launch
// sequences of inference, of one training step (forward, loss, backward, Adam) and of the
// single-layer entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/voldor.h"
#include "ctx.h"
#include "proposal.h"

using vdc::fail;

namespace {

inline size_t al(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxWgradChunks = 64;
constexpr int kMaxBgradChunks = 256;

// blocks of the bias-gradient sum: about 1024 pixels each, at most kMaxBgradChunks
int bgrad_chunks(int Mpix) { return std::max(1, std::min(kMaxBgradChunks, (Mpix + 1023) / 1024)); }
constexpr int kMaxLayerWeights = 128 * 9 * 128;

// pixel chunks of a weight-gradient launch: about 512 blocks, at least 256 pixels per chunk,
// and at most kMaxWgradChunks x kMaxLayerWeights partial sums (chunks x parameters)
int wgrad_chunks(int Cout, int Cin, int Mpix) {
    const int tiles = (Cout / vp::wgrad_co_tile(Cout)) * ((Cin + 31) / 32);
    const int nparam = Cout * 9 * Cin;
    const int cap = std::min(kMaxWgradChunks * kMaxLayerWeights / nparam, (Mpix + 255) / 256);
    return std::max(1, std::min((512 + tiles - 1) / tiles, cap));
}

struct Acts {
    uint16_t *x, *a1, *a2, *a3, *a4, *a5;
    float* o;
    int* flag;          // learned start: fallback flag
    // training
    uint16_t *go, *g5, *g4, *g3, *g2, *g1;
    float* wpart;
    float* bpart;
    double* lpart;
    int* mask_cnt;
};

int check_net_shape(voldor_ctx ctx, int H, int W, int N) {
    if (H < 2 || W < 2 || (H & 1) || (W & 1) || (int64_t)H * W > (1 << 26))
        return fail(ctx, VOLDOR_EINVAL, "network input must be even-sized, got %dx%d", W, H);
    if (N < 1 || N > 8) return fail(ctx, VOLDOR_EINVAL, "N=%d outside 1..8", N);
    return VOLDOR_OK;
}

int layout(voldor_ctx ctx, int H, int W, bool train, hipStream_t st, Acts& A, int lane = -1) {
    const size_t HW = (size_t)H * W, HW2 = (size_t)(H / 2) * (W / 2);
    const size_t b16 = sizeof(uint16_t);
    size_t sz[24];
    int k = 0;
    sz[k++] = al(HW * 16 * b16);     // x
    sz[k++] = al(HW * 64 * b16);     // a1
    sz[k++] = al(HW2 * 128 * b16);   // a2
    sz[k++] = al(HW2 * 128 * b16);   // a3
    sz[k++] = al(HW2 * 128 * b16);   // a4
    sz[k++] = al(HW * 64 * b16);     // a5
    sz[k++] = al(HW * 32 * sizeof(float));   // o
    sz[k++] = al(sizeof(int));                // flag
    const int nfwd = k;
    sz[k++] = al(HW * 32 * b16);     // go
    sz[k++] = al(HW * 64 * b16);     // g5
    sz[k++] = al(HW2 * 128 * b16);   // g4
    sz[k++] = al(HW2 * 128 * b16);   // g3
    sz[k++] = al(HW2 * 128 * b16);   // g2
    sz[k++] = al(HW * 64 * b16);     // g1
    sz[k++] = al((size_t)kMaxWgradChunks * kMaxLayerWeights * sizeof(float));
    sz[k++] = al((size_t)kMaxBgradChunks * 128 * sizeof(float));
    sz[k++] = al((size_t)3 * ((HW + 255) / 256) * sizeof(double));
    sz[k++] = al(sizeof(int) * (size_t)vp::mask_count_blocks(HW));   // masked-pixel counts per span
    const int n = train ? k : nfwd;
    size_t total = 0;
    for (int i = 0; i < n; ++i) total += sz[i];
    void** ws = lane < 0 ? &ctx->net_ws : &ctx->lane_ws[lane];
    int rc = vdc::ensure_buffer(ctx, ws, lane < 0 ? &ctx->net_ws_bytes : &ctx->lane_ws_bytes[lane], total, st);
    if (rc) return rc;
    char* p = (char*)*ws;
    void** slots[18] = {(void**)&A.x, (void**)&A.a1, (void**)&A.a2, (void**)&A.a3, (void**)&A.a4, (void**)&A.a5,
                        (void**)&A.o, (void**)&A.flag, (void**)&A.go, (void**)&A.g5, (void**)&A.g4, (void**)&A.g3, (void**)&A.g2,
                        (void**)&A.g1, (void**)&A.wpart, (void**)&A.bpart, (void**)&A.lpart,
                        (void**)&A.mask_cnt};
    std::memset(&A, 0, sizeof(A));
    for (int i = 0; i < n; ++i) {
        *slots[i] = p;
        p += sz[i];
    }
    return VOLDOR_OK;
}

// forward arguments of layer L for an H x W network input
vp::ConvArgs layer_args(int L, int H, int W, const voldor_net* net, const Acts& A) {
    const int H2 = H / 2, W2 = W / 2;
    vp::ConvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Cin = vp::kLayerCin[L];
    a.Cout = vp::kLayerCout[L];
    a.stride = vp::kLayerStride[L];
    a.up = vp::kLayerUp[L];
    a.relu = vp::kLayerRelu[L];
    a.w = net->wbf16 + vp::layer_off(L);
    a.bias = net->params + vp::layer_off(L) + a.Cout * 9 * a.Cin;
    const uint16_t* src[6] = {A.x, A.a1, A.a2, A.a3, A.a4, A.a5};
    a.x = src[L];
    const bool half_in = (L == 2 || L == 3 || L == 4);
    a.Hx = half_in ? H2 : H;
    a.Wx = half_in ? W2 : W;
    a.Hs = a.up ? 2 * a.Hx : a.Hx;
    a.Ws = a.up ? 2 * a.Wx : a.Wx;
    a.Ho = (a.Hs - 1) / a.stride + 1;
    a.Wo = (a.Ws - 1) / a.stride + 1;
    uint16_t* dst[6] = {A.a1, A.a2, A.a3, A.a4, A.a5, nullptr};
    a.y = dst[L];
    a.yf = (L == 5) ? A.o : nullptr;
    a.skip = (L == 4) ? A.a1 : nullptr;
    return a;
}

// heads of a forward pass, fused into the last layer's epilogue; logits (FP32 [H][W][32]) are
// written only where asked for
struct Heads {
    float* rho;
    float* q;
    float tnorm, rmin, rmax;
    const double* pose;
    int* flag;
    float* logits;
};

// the forward pass; without heads the last layer writes its FP32 output to A.o (training)
int run_forward(voldor_ctx ctx, const voldor_net* net, int H, int W, int N, const float* flow, const Acts& A,
                hipStream_t st, const Heads* h = nullptr) {
    VD_CHECK(vp::launch_features(flow, N, H * W, A.x, st), "feature launch");
    for (int L = 0; L < VP_NLAYERS; ++L) {
        vp::ConvArgs a = layer_args(L, H, W, net, A);
        if (h && L == VP_NLAYERS - 1) {
            a.yf = h->logits;
            a.hN = N;
            a.htnorm = h->tnorm;
            a.hrmin = h->rmin;
            a.hrmax = h->rmax;
            a.hrho = h->rho;
            a.hq = h->q;
            a.hpose = h->pose;
            a.hflag = h->flag;
        }
        VD_CHECK(vp::launch_conv(a, 0, st), "conv launch");
    }
    return VOLDOR_OK;
}

// weight + bias gradients of layer L (forward args f, pre-activation gradient dy) into
// grads at the layer's offset
int layer_param_grads(voldor_ctx ctx, const vp::ConvArgs& f, const uint16_t* dy, float* grads, const Acts& A,
                      hipStream_t st) {
    vp::WgradArgs g;
    g.Hs = f.Hs; g.Ws = f.Ws; g.Hx = f.Hx; g.Wx = f.Wx; g.Cin = f.Cin;
    g.Ho = f.Ho; g.Wo = f.Wo; g.Cout = f.Cout;
    g.stride = f.stride; g.up = f.up;
    g.x = f.x; g.dy = dy;
    g.part = A.wpart;
    g.nparam = f.Cout * 9 * f.Cin;
    const int Mpix = f.Ho * f.Wo;
    const int nch = wgrad_chunks(f.Cout, f.Cin, Mpix);
    VD_CHECK(vp::launch_wgrad(g, nch, st), "wgrad launch");
    if (grads) VD_CHECK(vp::launch_sum_chunks(A.wpart, g.nparam, nch, grads, st), "wgrad reduce launch");
    const int nb = bgrad_chunks(Mpix);
    VD_CHECK(vp::launch_bgrad(dy, Mpix, f.Cout, nb, A.bpart, st), "bgrad launch");
    if (grads) VD_CHECK(vp::launch_sum_chunks(A.bpart, f.Cout, nb, grads + g.nparam, st), "bgrad reduce launch");
    return VOLDOR_OK;
}

// data-gradient arguments of layer L: transposed weights, source dy on the forward output grid
vp::ConvArgs dgrad_args(const vp::ConvArgs& f, const uint16_t* wt, const uint16_t* dy) {
    vp::ConvArgs d;
    std::memset(&d, 0, sizeof(d));
    d.Hs = f.Ho; d.Ws = f.Wo; d.Hx = f.Ho; d.Wx = f.Wo;
    d.Cin = f.Cout;
    d.Ho = f.Hs; d.Wo = f.Ws;        // on the (upsampled) forward input grid
    d.Cout = f.Cin;
    d.stride = f.stride;
    d.x = dy;
    d.w = wt;
    return d;
}

// the convolution kernels read and write BF16 arrays as 16-byte vectors (null passes)
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int check_conv(voldor_ctx ctx, int H, int W, int Cin, int Cout, int stride, int up) {
    if (H < 1 || W < 1 || (int64_t)H * W > (1 << 26)) return fail(ctx, VOLDOR_EINVAL, "bad conv input size");
    if (Cin < 16 || Cin % 16 || Cin > 1024 || Cout < 32 || Cout % 32 || Cout > 1024)
        return fail(ctx, VOLDOR_EINVAL, "conv channels: Cin multiple of 16, Cout multiple of 32");
    if (!(stride == 1 || stride == 2) || (up != 0 && up != 1) || (up && stride == 2))
        return fail(ctx, VOLDOR_EINVAL, "conv stride 1 or 2, no stride with upsampling");
    if ((int64_t)Cout * 9 * Cin > kMaxLayerWeights) return fail(ctx, VOLDOR_EINVAL, "layer too large");
    return VOLDOR_OK;
}

}  // namespace

namespace vdc {

int net_workspace(voldor_ctx ctx, int H, int W, hipStream_t st, int lane) {
    Acts A;
    return layout(ctx, H, W, false, st, A, lane);
}

int proposal_start(voldor_ctx ctx, const voldor_net* net, int H, int W, int N, const float* flow, const double* pose,
                   float rmin, float rmax, float* idepth, float* rigid, int** flag, hipStream_t st, int lane) {
    int rc;
    if ((rc = check_net_shape(ctx, H, W, N))) return rc;
    if (!net || !net->params || !net->wbf16) return fail(ctx, VOLDOR_EINVAL, "null network pointer");
    if (!aligned16(net->wbf16)) return fail(ctx, VOLDOR_EINVAL, "network BF16 weights must be 16-byte aligned");
    Acts A;
    if ((rc = layout(ctx, H, W, false, st, A, lane))) return rc;
    VD_CHECK(vp::launch_flag_clear(A.flag, st), "flag clear launch");
    const Heads h = {idepth, rigid, 0.f, rmin, rmax, pose, A.flag, nullptr};
    if ((rc = run_forward(ctx, net, H, W, N, flow, A, st, &h))) return rc;
    *flag = A.flag;
    return VOLDOR_OK;
}

}  // namespace vdc

extern "C" {

int voldor_net_refresh(voldor_ctx ctx, const voldor_net* net, void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    if (!net || !net->params || !net->wbf16) return fail(ctx, VOLDOR_EINVAL, "null network pointer");
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    vp::AdamArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = net->params;
    a.wbf = net->wbf16;
    a.wt = net->wt_bf16;
    VD_CHECK(vp::launch_adam(a, (hipStream_t)stream), "refresh launch");
    return VOLDOR_OK;
}

int voldor_proposal_forward(voldor_ctx ctx, const voldor_net* net, int32_t H, int32_t W, int32_t N,
                            const float* flow, float tnorm, float idepth_min, float idepth_max, float* idepth_out,
                            float* rigid_out, float* logits_out, void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    int rc;
    if ((rc = check_net_shape(ctx, H, W, N))) return rc;
    if (!net || !net->params || !net->wbf16 || !flow) return fail(ctx, VOLDOR_EINVAL, "null pointer");
    if (!aligned16(net->wbf16)) return fail(ctx, VOLDOR_EINVAL, "network BF16 weights must be 16-byte aligned");
    if (!(tnorm > 0.f) || !std::isfinite(tnorm)) return fail(ctx, VOLDOR_EINVAL, "tnorm must be > 0");
    if (!(idepth_min > 0.f) || !(idepth_max > idepth_min)) return fail(ctx, VOLDOR_EINVAL, "bad idepth range");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    Acts A;
    if ((rc = layout(ctx, H, W, false, st, A))) return rc;
    const Heads h = {idepth_out, rigid_out, tnorm, idepth_min, idepth_max, nullptr, nullptr, logits_out};
    if ((rc = run_forward(ctx, net, H, W, N, flow, A, st, &h))) return rc;
    return VOLDOR_OK;
}

int voldor_proposal_train_step(voldor_ctx ctx, const voldor_net* net, int32_t H, int32_t W, int32_t N,
                               const float* flow, float tnorm, const float* idepth_target, const float* rigid_target,
                               const uint8_t* mask, float lam, float lr, int32_t step, double* loss_out,
                               void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    int rc;
    if ((rc = check_net_shape(ctx, H, W, N))) return rc;
    if (!net || !net->params || !net->wbf16 || !net->wt_bf16 || !net->adam_m || !net->adam_v || !net->grads)
        return fail(ctx, VOLDOR_EINVAL, "training needs every network buffer");
    if (!aligned16(net->wbf16) || !aligned16(net->wt_bf16))
        return fail(ctx, VOLDOR_EINVAL, "network BF16 weights must be 16-byte aligned");
    if (!flow || !idepth_target || !rigid_target || !mask || !loss_out)
        return fail(ctx, VOLDOR_EINVAL, "null training input");
    if (!(tnorm > 0.f) || !std::isfinite(tnorm) || !(lam >= 0.f) || !(lr > 0.f) || step < 1)
        return fail(ctx, VOLDOR_EINVAL, "bad training constants");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    Acts A;
    if ((rc = layout(ctx, H, W, true, st, A))) return rc;
    if ((rc = run_forward(ctx, net, H, W, N, flow, A, st))) return rc;
    const int HW = H * W;
    VD_CHECK(vp::launch_loss(A.o, HW, N, tnorm, idepth_target, rigid_target, mask, lam, A.mask_cnt, A.go, A.lpart,
                             loss_out, st), "loss launch");

    vp::ConvArgs f[VP_NLAYERS];
    for (int L = 0; L < VP_NLAYERS; ++L) f[L] = layer_args(L, H, W, net, A);
    auto wt = [&](int L) { return (const uint16_t*)(net->wt_bf16 + vp::layer_off(L)); };
    float* grads = net->grads;
    // c6: dy = go
    if ((rc = layer_param_grads(ctx, f[5], A.go, grads + vp::layer_off(5), A, st))) return rc;
    vp::ConvArgs d = dgrad_args(f[5], wt(5), A.go);
    d.y = A.g5;
    d.mask = A.a5;                       // c5's ReLU
    VD_CHECK(vp::launch_conv(d, 1, st), "dgrad launch");
    // c5: dy = g5 (also the gradient reaching a1 through the skip)
    if ((rc = layer_param_grads(ctx, f[4], A.g5, grads + vp::layer_off(4), A, st))) return rc;
    d = dgrad_args(f[4], wt(4), A.g5);
    d.pool = 1;                          // summed back onto the half grid, then c4's ReLU
    d.mask = A.a4;
    d.y = A.g4;
    VD_CHECK(vp::launch_conv(d, 1, st), "dgrad launch");
    // c4, c3
    if ((rc = layer_param_grads(ctx, f[3], A.g4, grads + vp::layer_off(3), A, st))) return rc;
    d = dgrad_args(f[3], wt(3), A.g4);
    d.y = A.g3;
    d.mask = A.a3;
    VD_CHECK(vp::launch_conv(d, 1, st), "dgrad launch");
    if ((rc = layer_param_grads(ctx, f[2], A.g3, grads + vp::layer_off(2), A, st))) return rc;
    d = dgrad_args(f[2], wt(2), A.g3);
    d.y = A.g2;
    d.mask = A.a2;
    VD_CHECK(vp::launch_conv(d, 1, st), "dgrad launch");
    // c2 (stride 2): a1's gradient adds the skip path, then c1's ReLU
    if ((rc = layer_param_grads(ctx, f[1], A.g2, grads + vp::layer_off(1), A, st))) return rc;
    d = dgrad_args(f[1], wt(1), A.g2);
    d.skip = A.g5;
    d.y = A.g1;
    d.mask = A.a1;
    VD_CHECK(vp::launch_conv(d, 1, st), "dgrad launch");
    // c1
    if ((rc = layer_param_grads(ctx, f[0], A.g1, grads + vp::layer_off(0), A, st))) return rc;

    vp::AdamArgs ad;
    ad.params = net->params;
    ad.grads = grads;
    ad.m = net->adam_m;
    ad.v = net->adam_v;
    ad.wbf = net->wbf16;
    ad.wt = net->wt_bf16;
    ad.lr = lr;
    ad.b1 = 0.9f;
    ad.b2 = 0.999f;
    ad.eps = 1e-8f;
    ad.inv_bc1 = (float)(1.0 / (1.0 - std::pow(0.9, step)));
    ad.inv_bc2 = (float)(1.0 / (1.0 - std::pow(0.999, step)));
    VD_CHECK(vp::launch_adam(ad, st), "adam launch");
    return VOLDOR_OK;
}

int voldor_conv3x3_bf16(voldor_ctx ctx, int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t stride, int32_t up,
                        int32_t relu, const uint16_t* x, const uint16_t* w, const float* bias, const uint16_t* skip,
                        uint16_t* y, float* yf, void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    int rc;
    if ((rc = check_conv(ctx, H, W, Cin, Cout, stride, up))) return rc;
    if (!x || !w || (!y && !yf)) return fail(ctx, VOLDOR_EINVAL, "null conv pointer");
    if (!aligned16(x) || !aligned16(w) || !aligned16(skip) || !aligned16(y))
        return fail(ctx, VOLDOR_EINVAL, "conv BF16 arrays must be 16-byte aligned");
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    vp::ConvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Hx = H; a.Wx = W; a.Cin = Cin; a.Cout = Cout;
    a.Hs = up ? 2 * H : H;
    a.Ws = up ? 2 * W : W;
    a.Ho = (a.Hs - 1) / stride + 1;
    a.Wo = (a.Ws - 1) / stride + 1;
    a.stride = stride; a.up = up; a.relu = relu ? 1 : 0;
    a.x = x; a.w = w; a.bias = bias; a.skip = skip; a.y = y; a.yf = yf;
    VD_CHECK(vp::launch_conv(a, 0, (hipStream_t)stream), "conv launch");
    return VOLDOR_OK;
}

int voldor_conv3x3_bf16_backward(voldor_ctx ctx, int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t stride,
                                 int32_t up, const uint16_t* x, const uint16_t* w_t, const uint16_t* dy, float* dx,
                                 float* dw, float* db, void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    int rc;
    if ((rc = check_conv(ctx, H, W, Cin, Cout, stride, up))) return rc;
    if (!x || !dy || (dx && !w_t)) return fail(ctx, VOLDOR_EINVAL, "null conv pointer");
    if (!aligned16(x) || !aligned16(dy) || !aligned16(w_t))
        return fail(ctx, VOLDOR_EINVAL, "conv BF16 arrays must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    vp::ConvArgs f;
    std::memset(&f, 0, sizeof(f));
    f.Hx = H; f.Wx = W; f.Cin = Cin; f.Cout = Cout;
    f.Hs = up ? 2 * H : H;
    f.Ws = up ? 2 * W : W;
    f.Ho = (f.Hs - 1) / stride + 1;
    f.Wo = (f.Ws - 1) / stride + 1;
    f.stride = stride; f.up = up;
    f.x = x;
    // workspace: weight-gradient partials, bias partials
    const int Mpix0 = f.Ho * f.Wo;
    const int nch = wgrad_chunks(Cout, Cin, Mpix0);
    const int nbb = bgrad_chunks(Mpix0);
    const size_t wbytes = al(sizeof(float) * (size_t)nch * Cout * 9 * Cin);
    const size_t bbytes = al(sizeof(float) * (size_t)nbb * Cout);
    if ((rc = vdc::ensure_buffer(ctx, &ctx->net_ws, &ctx->net_ws_bytes, wbytes + bbytes, st))) return rc;
    Acts A;
    std::memset(&A, 0, sizeof(A));
    A.wpart = (float*)ctx->net_ws;
    A.bpart = (float*)((char*)ctx->net_ws + wbytes);
    if (dw || db) {
        vp::WgradArgs g;
        g.Hs = f.Hs; g.Ws = f.Ws; g.Hx = f.Hx; g.Wx = f.Wx; g.Cin = f.Cin;
        g.Ho = f.Ho; g.Wo = f.Wo; g.Cout = f.Cout; g.stride = f.stride; g.up = f.up;
        g.x = x; g.dy = dy; g.part = A.wpart; g.nparam = Cout * 9 * Cin;
        if (dw) {
            VD_CHECK(vp::launch_wgrad(g, nch, st), "wgrad launch");
            VD_CHECK(vp::launch_sum_chunks(A.wpart, g.nparam, nch, dw, st), "wgrad reduce launch");
        }
        if (db) {
            VD_CHECK(vp::launch_bgrad(dy, Mpix0, Cout, nbb, A.bpart, st), "bgrad launch");
            VD_CHECK(vp::launch_sum_chunks(A.bpart, Cout, nbb, db, st), "bgrad reduce launch");
        }
    }
    if (dx) {
        vp::ConvArgs d = dgrad_args(f, w_t, dy);
        d.pool = up ? 1 : 0;             // upsampling: summed back onto the stored grid
        d.yf = dx;
        VD_CHECK(vp::launch_conv(d, 1, st), "dgrad launch");
    }
    return VOLDOR_OK;
}

}  // extern "C"
