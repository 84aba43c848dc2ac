// C ABI of the library: context and scratch management, argument validation, and the
// launch sequences of the GEM entry points and of keyframe alignment.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/voldor.h"
#include "ctx.h"
#include "device.h"
#include "kernels.h"

using vdc::fail;
using vdc::hip_fail;

// Scratch of voldor_run_noalloc: one copy per device, loaded with the code object and held
// until the process ends.  Host code never passes this name to a kernel (on the host it is
// a stand-in, not a device address); it uses the per-device address that
// hipGetSymbolAddress returns at context creation.
static __device__ __align__(256) unsigned char scratch[VOLDOR_NOALLOC_SCRATCH_BYTES];

namespace {

// device address of `scratch` per device ordinal, looked up once with that device current
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};
hipError_t g_noalloc_err[kMaxDevices] = {};

// Looks up the address of the static scratch on the current device (ordinal dev), once.
void noalloc_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[dev]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        g_noalloc_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        return;
    }
    g_noalloc_ptr[dev] = p;
    g_noalloc_err[dev] = hipSuccess;
}

void* noalloc_base(int dev, hipError_t* err) {
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    *err = g_noalloc_err[dev];
    return g_noalloc_ptr[dev];
}

constexpr size_t kMaxBatch = 4096;         // candidates per pose_score call / pairs per align call
constexpr size_t kLevelLdsMax = 150 * 1024;
constexpr size_t kMaxBlockOrders = 1024;   // cached local-level block orders per context

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ---- launch timers: an event pair per bracketed launch, recycled through a pool
hipError_t take_event(voldor_ctx ctx, hipEvent_t* e) {
    if (!ctx->ev_pool.empty()) {
        *e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Start of a bracket: *a stays null when timing is off.
hipError_t timer_start(voldor_ctx ctx, int which, hipStream_t st, hipEvent_t* a) {
    *a = nullptr;
    if (!(ctx->timing & (1u << which))) return hipSuccess;
    hipError_t e = take_event(ctx, a);
    if (e == hipSuccess) e = hipEventRecord(*a, st);
    return e;
}

hipError_t timer_stop(voldor_ctx ctx, int which, hipStream_t st, hipEvent_t a) {
    if (!a) return hipSuccess;
    hipEvent_t b = nullptr;
    hipError_t e = take_event(ctx, &b);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e != hipSuccess) {
        ctx->ev_pool.push_back(a);
        if (b) ctx->ev_pool.push_back(b);
        return e;
    }
    ctx->ev_rec[which].emplace_back(a, b);
    return hipSuccess;
}

void timers_discard(voldor_ctx ctx) {
    for (auto& r : ctx->ev_rec) {
        for (auto& p : r) {
            ctx->ev_pool.push_back(p.first);
            ctx->ev_pool.push_back(p.second);
        }
        r.clear();
    }
}

// Per-window scratch: [FP32 poses | FP64 poses | flow layout | pose history | observations |
// log-likelihood partials | reduction partials | phase-A arrays].
struct Scratch {
    vd::PoseF* poses;
    vd::PoseD* posed;
    char* a;
};

int lattice(int H, int W, int s, int* hc, int* wc) {
    const int o = s / 2;
    if (s < 1 || H <= o || W <= o) return 0;
    *hc = (H - o + s - 1) / s;
    *wc = (W - o + s - 1) / s;
    return 1;
}

int check_window(voldor_ctx ctx, const voldor_window* w, const voldor_buffers* b) {
    if (!ctx) return VOLDOR_EINVAL;
    if (!w || !b) return fail(ctx, VOLDOR_EINVAL, "null window or buffer struct");
    if (w->H < 2 || w->W < 2 || (int64_t)w->H * w->W > (1 << 28))
        return fail(ctx, VOLDOR_EINVAL, "bad image size %dx%d", w->W, w->H);
    if (w->N < 1 || w->N > VD_NMAX) return fail(ctx, VOLDOR_EINVAL, "N=%d outside 1..%d", w->N, VD_NMAX);
    if (w->P < 0 || w->P > VD_PMAX) return fail(ctx, VOLDOR_EINVAL, "P=%d outside 0..%d", w->P, VD_PMAX);
    if (!(w->fx > 0) || !(w->fy > 0) || !std::isfinite(w->cx) || !std::isfinite(w->cy))
        return fail(ctx, VOLDOR_EINVAL, "bad intrinsics");
    if (!(w->fisk_alpha > 0) || !(w->fisk_beta >= 1.0f && w->fisk_beta <= 4.0f))
        return fail(ctx, VOLDOR_EINVAL, "bad log-logistic parameters (alpha > 0, beta in [1, 4])");
    if (!(w->outlier_density > 0)) return fail(ctx, VOLDOR_EINVAL, "outlier_density must be > 0");
    if (!(w->hmm_gamma > 0.5f && w->hmm_gamma <= 1.0f)) return fail(ctx, VOLDOR_EINVAL, "hmm_gamma must be in (0.5, 1]");
    if (!(w->idepth_min > 0) || !(w->idepth_max > w->idepth_min))
        return fail(ctx, VOLDOR_EINVAL, "need 0 < idepth_min < idepth_max");
    if (!(w->perturb_sigma0 >= 0)) return fail(ctx, VOLDOR_EINVAL, "perturb_sigma0 must be >= 0");
    if (w->P > 0 && (!(w->prior_sigma_rel > 0) || !(w->prior_uniform_rel > 0) ||
                     !(w->prior_inlier_default >= 0 && w->prior_inlier_default <= 1)))
        return fail(ctx, VOLDOR_EINVAL, "bad prior constants");
    if (w->prior_model != 0 && w->prior_model != 1) return fail(ctx, VOLDOR_EINVAL, "prior_model must be 0 or 1");
    if (w->init_random > 1) return fail(ctx, VOLDOR_EINVAL, "init_random must be 0 or 1");
    if (w->P > 0 && w->prior_model == 1 &&
        (!(w->prior_disp_scale > 0) || !(w->prior_fisk_beta > 0 && w->prior_fisk_beta <= 1)))
        return fail(ctx, VOLDOR_EINVAL, "disparity prior model: need prior_disp_scale > 0 and prior_fisk_beta in (0, 1]");
    if (w->n_candidates < 3 || w->n_candidates > 64) return fail(ctx, VOLDOR_EINVAL, "n_candidates outside 3..64");
    int hc, wc;
    if (!lattice(w->H, w->W, w->coarse_stride, &hc, &wc)) return fail(ctx, VOLDOR_EINVAL, "bad coarse_stride");
    if (hc > 2048 || wc > 2048) return fail(ctx, VOLDOR_EINVAL, "coarse lattice longer than 2048 along an axis");
    const int T = w->tile;
    if (!(T == 8 || T == 16 || T == 32 || T == 64 || T == 128 || T == 256))
        return fail(ctx, VOLDOR_EINVAL, "tile must be 8, 16, 32, 64, 128 or 256");
    if (w->pose_gn_steps < 0 || w->pose_gn_steps > 100) return fail(ctx, VOLDOR_EINVAL, "pose_gn_steps outside 0..100");
    if (w->chain_axis != 0 && w->chain_axis != 1) return fail(ctx, VOLDOR_EINVAL, "chain_axis must be 0 or 1");
    if (!b->flow || !b->pose || !b->idepth || !b->rigid || !b->idepth_coarse || !b->rigid_coarse)
        return fail(ctx, VOLDOR_EINVAL, "null buffer pointer");
    if (w->P > 0 && (!b->prior_idepth || !b->prior_pose)) return fail(ctx, VOLDOR_EINVAL, "null prior pointer");
    return VOLDOR_OK;
}

// the first depth prior, which the initial inverse depth starts from, or none
vd::InitSrc boot_src(const voldor_window* v, const voldor_buffers* b) {
    vd::InitSrc s{nullptr, nullptr};
    if (v->P > 0 && !v->init_random) {
        s.prior = b->prior_idepth;
        s.pose = b->prior_pose;
    }
    return s;
}

vd::Win make_win(const voldor_window* v, int it, int level, const voldor_buffers* b = nullptr) {
    vd::Win w;
    std::memset(&w, 0, sizeof(w));
    w.H = v->H; w.W = v->W; w.N = v->N; w.P = v->P;
    w.fx = v->fx; w.fy = v->fy; w.cx = v->cx; w.cy = v->cy;
    w.ifx = (float)(1.0 / (double)v->fx);
    w.ify = (float)(1.0 / (double)v->fy);
    const double al = v->fisk_alpha, be = v->fisk_beta, L0 = v->outlier_density;
    w.inv_a2 = (float)(1.0 / (al * al));
    w.beta = (float)be;
    w.beta2 = (v->fisk_beta == 2.0f);
    w.fl_c = w.beta2 ? (float)(L0 * M_PI * al * al) : (float)std::log2(L0 * 2.0 * M_PI * al * al / be);
    w.zfloor = be < 2.0 ? 1e-3f : 0.0f;
    w.ln_L0 = (float)std::log(L0);
    w.gamma = v->hmm_gamma;
    w.rmin = v->idepth_min; w.rmax = v->idepth_max;
    w.sigma_it = (float)std::fmax(v->perturb_sigma0 * std::ldexp(1.0, -(it / 2)), 0.005);
    w.csig = v->prior_sigma_rel;
    w.log2kappa = v->P > 0 ? (float)std::log2(std::sqrt(2.0 * M_PI) * v->prior_sigma_rel / v->prior_uniform_rel) : 0.f;
    w.pi_default = v->prior_inlier_default;
    w.K = v->n_candidates;
    w.s = v->coarse_stride;
    lattice(v->H, v->W, v->coarse_stride, &w.hc, &w.wc);
    w.it = it; w.level = level; w.dir = it & 3;
    w.chain_axis = v->chain_axis;
    w.key0 = (uint32_t)(v->seed & 0xffffffffu);
    w.key1 = (uint32_t)(v->seed >> 32);
    w.window_id = v->window_id;
    w.has_prior_weight = (b && v->P > 0 && b->prior_weight) ? 1 : 0;
    w.prior_disp = (v->P > 0 && v->prior_model == 1) ? 1 : 0;
    if (w.prior_disp) {
        const double al = v->prior_sigma_rel, be = v->prior_fisk_beta, D = v->prior_uniform_rel;
        w.disp_fb = v->prior_disp_scale;
        w.disp_inv_alpha = (float)(1.0 / al);
        w.disp_beta = (float)be;
        w.disp_beta1 = be == 1.0;
        w.disp_zfloor = be < 1.0 ? 1e-3f : 0.0f;
        w.disp_c = (float)std::log2(2.0 * al / (be * D));
    }
    return w;
}

// Effective launch knobs of a window: the context's entry for its (H, W, N, K, prior)
// bucket, else the defaults (all zero).
voldor_knobs knobs_for(voldor_ctx ctx, const voldor_window* v) {
    voldor_knobs k;
    std::memset(&k, 0, sizeof(k));
    if (!ctx) return k;
    for (const auto& e : ctx->knobs)
        if (e.H == v->H && e.W == v->W && e.N == v->N && e.K == v->n_candidates && e.prior == (v->P > 0))
            return e.k;
    return k;
}

vd::LevelGeom make_geom(const voldor_window* v, const vd::Win& w, int level, int it, const voldor_knobs& kn) {
    vd::LevelGeom g;
    g.horizontal = ((it & 3) % 2 == 0);
    if (level == VOLDOR_LEVEL_COARSE) {
        g.h = w.hc; g.w = w.wc; g.s = w.s; g.off = w.s / 2;
        g.seg = g.horizontal ? g.w : g.h;
    } else {
        g.h = v->H; g.w = v->W; g.s = 1; g.off = 0;
        g.seg = v->tile;
    }
    // one lane per (chain, frame) in the forward-backward phase: C * N <= block size
    g.C = std::max(1, std::min(VD_BLOCK / g.seg, VD_BLOCK / v->N));
    if (level == VOLDOR_LEVEL_LOCAL && kn.local_chains > 0) g.C = std::min(g.C, kn.local_chains);
    const int axis = g.horizontal ? g.w : g.h;
    const int lines = g.horizontal ? g.h : g.w;
    g.nseg = (axis + g.seg - 1) / g.seg;
    g.nblocks = g.nseg * ((lines + g.C - 1) / g.C);
    g.nchains = g.nseg * lines;
    // speculation depth of the chain scan: the coarse level's long chains carry a value over
    // many nodes, so it speculates deeper (phase A2 cost grows with the depth, misses shrink)
    g.spec = level == VOLDOR_LEVEL_COARSE ? (kn.coarse_spec > 0 ? kn.coarse_spec : VD_SPEC)
                                          : (kn.local_spec > 0 ? kn.local_spec : 2);
    g.pa_lanes = kn.coarse_lanes > 0 ? kn.coarse_lanes : VD_PA_LANES;
    g.nf = std::max(v->N, 3);
    g.ncost = 0;
    // a long chain (coarse stride 1 on a wide image) speculates less deep if its block would
    // not fit the LDS; the speculation depth never changes a result
    while (g.spec > 1 && vd::level_lds_bytes(g) > kLevelLdsMax) --g.spec;
    // a fused local pass keeps its E-step frame costs when there are no priors and the
    // block still fits 5 per CU (32 KB of the 160 KB LDS)
    g.ncost = 0;
    if (level == VOLDOR_LEVEL_LOCAL && v->P == 0) {
        g.ncost = v->N;
        if (vd::level_lds_bytes(g) > 32 * 1024) g.ncost = 0;
    }
    return g;
}

struct GemLaunch {
    voldor_ctx ctx;
    const voldor_window* v;
    const voldor_buffers* b;
    hipStream_t st;
    Scratch s;
    double* ll_partial;
    double* pose_partials;
    double* pa_E;         // coarse-level phase-A results [Hc*Wc]
    float* pa_V;
    int* pa_S;
    double* pa_spec;      // [VD_SPEC][Hc*Wc]
    float4* flow2;        // [N][H][W] row-pair layout of the flows
    vd::PoseD* hist;      // pose history of a pose step
    float2* obs;          // [H][W] observed displacements
    int gn_blocks;
    int pose_blocks;
    int max_level_blocks;
    bool timers = true;   // bracket launches with the context's timers (when enabled)
    bool may_alloc = true; // may create context-owned buffers (not in the no-allocation entry)
    voldor_knobs kn;      // launch knobs of the window (results do not depend on them)
    struct { size_t head, f2, hist, obs, ll, red, pa; } sz;
};

// Launch dimensions of one window and the byte size of its scratch.
size_t gem_layout(const voldor_window* v, int n_cand, GemLaunch& L) {
    L.kn = knobs_for(L.ctx, v);
    vd::Win w0 = make_win(v, 0, 1);
    int mx = 0;
    for (int lvl = 0; lvl < 2; ++lvl)
        for (int d = 0; d < 2; ++d) {
            const vd::LevelGeom g = make_geom(v, w0, lvl, d, L.kn);
            mx = std::max(mx, std::max(g.nblocks, g.nchains));
        }
    L.max_level_blocks = mx;
    const int64_t npix = (int64_t)v->H * v->W;
    // ~4 pixels per thread: enough blocks to fill the chip, few partial records
    L.pose_blocks = (int)std::min<int64_t>(std::max<int64_t>(1, (npix + 2 * VD_BLOCK - 1) / (2 * VD_BLOCK)), 2048);
    // pose step: one block per 1024 pixels keeps the per-block prologue cheap
    L.gn_blocks = (int)std::min<int64_t>(
        std::max<int64_t>(1, (npix + VD_GN_PIX * VD_GN_BLOCK - 1) / (VD_GN_PIX * VD_GN_BLOCK)), 256);
    const int fin_blocks = (int)((npix + VD_BLOCK - 1) / VD_BLOCK);
    L.sz.head = align_up((VD_NMAX + VD_PMAX) * sizeof(vd::PoseF)) + align_up(VD_NMAX * sizeof(vd::PoseD));
    L.sz.ll = align_up(sizeof(double) * mx);
    const size_t pp_bytes = align_up(sizeof(double) * 29 * (size_t)L.pose_blocks * n_cand);
    const size_t fin_bytes = align_up(sizeof(double) * 5 * (size_t)fin_blocks);
    const size_t gnp_bytes = align_up(sizeof(double) * 29 * 2 * (size_t)L.gn_blocks);
    L.sz.red = std::max(std::max(pp_bytes, fin_bytes), gnp_bytes);
    L.sz.pa = align_up(sizeof(double) * (size_t)w0.hc * w0.wc);
    L.sz.f2 = align_up(sizeof(float4) * (size_t)npix * v->N);
    L.sz.hist = align_up(sizeof(vd::PoseD) * (size_t)v->N * std::max(1, v->pose_gn_steps));
    L.sz.obs = align_up(sizeof(float2) * (size_t)npix);
    return L.sz.head + L.sz.f2 + L.sz.hist + L.sz.obs + L.sz.ll + L.sz.red + (3 + VD_SPEC) * L.sz.pa;
}

// Points L's scratch arrays into the region at base (sized by gem_layout).
void gem_carve(char* base, GemLaunch& L) {
    L.s.poses = (vd::PoseF*)base;
    L.s.posed = (vd::PoseD*)(base + align_up((VD_NMAX + VD_PMAX) * sizeof(vd::PoseF)));
    char* p = base + L.sz.head;
    L.s.a = p;
    L.flow2 = (float4*)p;
    p += L.sz.f2;
    L.hist = (vd::PoseD*)p;
    p += L.sz.hist;
    L.obs = (float2*)p;
    p += L.sz.obs;
    L.ll_partial = (double*)p;
    p += L.sz.ll;
    L.pose_partials = (double*)p;
    p += L.sz.red;
    L.pa_E = (double*)p;
    L.pa_V = (float*)(p + L.sz.pa);
    L.pa_S = (int*)(p + 2 * L.sz.pa);
    L.pa_spec = (double*)(p + 3 * L.sz.pa);
}

int gem_prepare(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, hipStream_t st, GemLaunch& L,
                int n_cand = 1) {
    L.ctx = ctx; L.v = v; L.b = b; L.st = st;
    const size_t bytes = gem_layout(v, n_cand, L);
    int rc = vdc::ensure_buffer(ctx, &ctx->scratch, &ctx->scratch_bytes, bytes, st);
    if (rc) return rc;
    gem_carve((char*)ctx->scratch, L);
    return VOLDOR_OK;
}

vd::LevelBufs level_bufs(const GemLaunch& L, int level, bool want_ll) {
    vd::LevelBufs B;
    B.P = L.s.poses;
    B.flow = (const float2*)L.b->flow;
    B.flow2 = L.flow2;
    B.idepth = L.b->idepth;
    B.idepth_coarse = L.b->idepth_coarse;
    B.blk_order = nullptr;
    B.prior = L.b->prior_idepth;
    B.prior_weight = L.b->prior_weight;
    float* q = level == VOLDOR_LEVEL_COARSE ? L.b->rigid_coarse : L.b->rigid;
    B.q_out = q;
    B.q_in = q;
    B.rho_out = level == VOLDOR_LEVEL_COARSE ? L.b->idepth_coarse : L.b->idepth;
    B.ll_partial = want_ll ? L.ll_partial : nullptr;
    B.pa_E = L.pa_E;
    B.pa_V = L.pa_V;
    B.pa_S = L.pa_S;
    B.pa_spec = L.pa_spec;
    return B;
}

vd::PoseBufs pose_bufs(const GemLaunch& L) {
    vd::PoseBufs B;
    B.P = L.s.poses;
    B.PD = L.s.posed;
    B.flow = (const float2*)L.b->flow;
    B.flow2 = L.flow2;
    B.idepth = L.b->idepth;
    B.rigid = L.b->rigid;
    B.pose = L.b->pose;
    B.partials = L.pose_partials;
    B.out = nullptr;
    B.hist = L.hist;
    B.obs = L.obs;
    return B;
}

vd::FinalBufs final_bufs(const GemLaunch& L) {
    vd::FinalBufs B;
    B.P = L.s.poses;
    B.flow = (const float2*)L.b->flow;
    B.flow2 = L.flow2;
    B.idepth = L.b->idepth;
    B.rigid = L.b->rigid;
    B.prior = L.b->prior_idepth;
    B.prior_weight = L.b->prior_weight;
    B.conf = L.b->conf;
    B.stats = L.b->stats;
    B.partials = L.pose_partials;
    B.ll_partial = L.ll_partial;
    return B;
}

// Block order of the local level: the level's blocks sorted by the angle of their centre
// around the principal point.  Each XCD takes a contiguous range of logical blocks
// (xcd_block), so it then works on an angular sector of the image.  For a camera moving
// forward the epipolar lines radiate from near the principal point, so the flow samples of
// a sector's candidates stay in that sector's part of the flows and the XCD's L2 holds more
// of them.  Only the schedule changes: every block computes what it computes in order.
// Created once per context and geometry (up to kMaxBlockOrders of them), outside stream
// capture; null (blocks in row order) under the local_order knob 2, in the no-allocation
// entry, and where it cannot be created.
const int* block_order(const GemLaunch& L, const vd::LevelGeom& g, const vd::Win& w) {
    voldor_ctx ctx = L.ctx;
    if (L.kn.local_order == 2 || !L.may_alloc) return nullptr;
    int cxb, cyb;
    std::memcpy(&cxb, &w.cx, sizeof(int));
    std::memcpy(&cyb, &w.cy, sizeof(int));
    const std::array<int, 10> key = {g.h, g.w, g.s, g.off, g.seg, g.horizontal, g.C, g.nseg, cxb, cyb};
    for (const auto& e : ctx->block_orders)
        if (e.key == key) return e.d;
    if (ctx->block_orders.size() >= kMaxBlockOrders) return nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(L.st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    const int nb = g.nblocks;
    std::vector<std::pair<double, int>> a((size_t)nb);
    for (int b = 0; b < nb; ++b) {
        const int sidx = b % g.nseg, lb = b / g.nseg;
        const double line = lb * g.C + 0.5 * g.C, pos = sidx * g.seg + 0.5 * g.seg;
        const double lx = g.horizontal ? pos : line, ly = g.horizontal ? line : pos;
        a[(size_t)b] = {std::atan2(g.s * ly + g.off - w.cy, g.s * lx + g.off - w.cx), b};
    }
    std::sort(a.begin(), a.end());
    std::vector<int> order((size_t)nb);
    for (int i = 0; i < nb; ++i) order[(size_t)i] = a[(size_t)i].second;
    int* d = nullptr;
    if (hipMalloc(&d, sizeof(int) * (size_t)nb) != hipSuccess) return nullptr;
    // on the launch stream, waited for before the host copy goes away (as the batch tables)
    if (hipMemcpyAsync(d, order.data(), sizeof(int) * (size_t)nb, hipMemcpyHostToDevice, L.st) != hipSuccess ||
        hipStreamSynchronize(L.st) != hipSuccess) {
        (void)hipFree(d);
        return nullptr;
    }
    ctx->block_orders.push_back({key, d});
    return d;
}

int run_level(GemLaunch& L, int it, int level, int do_e, int do_m, bool want_ll) {
    voldor_ctx ctx = L.ctx;
    const vd::Win w = make_win(L.v, it, level, L.b);
    const vd::LevelGeom g = make_geom(L.v, w, level, it, L.kn);
    const size_t lds = vd::level_lds_bytes(g);
    if (lds > kLevelLdsMax) return fail(ctx, VOLDOR_EINVAL, "chain segment too long for LDS (%zu bytes)", lds);
    vd::LevelBufs B = level_bufs(L, level, want_ll);
    if (level == VOLDOR_LEVEL_LOCAL) B.blk_order = block_order(L, g, w);
    hipEvent_t t0 = nullptr;
    const int timer = level == VOLDOR_LEVEL_COARSE ? VOLDOR_TIMER_COARSE : VOLDOR_TIMER_LOCAL;
    const bool timed = L.timers && (level == VOLDOR_LEVEL_COARSE || (do_e && do_m));
    if (timed) VD_CHECK(timer_start(ctx, timer, L.st, &t0), "timer event");
    if (level == VOLDOR_LEVEL_COARSE && do_m) {
        // few long chains: E-step per chain, phase A over the whole lattice, then the
        // per-chain speculation + scan from the stored phase-A results
        if (do_e) VD_CHECK(vd::launch_level(w, g, B, 1, 0, L.st), "level kernel launch");
        VD_CHECK(vd::launch_phase_a(w, g, B, L.st), "phase A launch");
        VD_CHECK(vd::launch_phase_a2(w, g, B, L.st), "phase A2 launch");
        VD_CHECK(vd::launch_level(w, g, B, 0, 2, L.st), "level kernel launch");
    } else {
        VD_CHECK(vd::launch_level(w, g, B, do_e, do_m, L.st), "level kernel launch");
    }
    if (timed) VD_CHECK(timer_stop(ctx, timer, L.st, t0), "timer event");
    return VOLDOR_OK;
}

int run_pose_step(GemLaunch& L) {
    voldor_ctx ctx = L.ctx;
    vd::Win w = make_win(L.v, 0, 1);
    const vd::PoseBufs B = pose_bufs(L);
    const int G = L.v->pose_gn_steps;
    if (G == 0) return VOLDOR_OK;
    hipEvent_t t0 = nullptr;
    if (L.timers) VD_CHECK(timer_start(ctx, VOLDOR_TIMER_POSE, L.st, &t0), "timer event");
    for (int s = 0; s < L.v->N * G; ++s)
        VD_CHECK(vd::launch_pose_gn(w, B, s, G, L.gn_blocks, L.st), "pose step launch");
    VD_CHECK(vd::launch_pose_gn_finish(B, L.v->N, G, L.gn_blocks, L.st), "pose finish launch");
    VD_CHECK(timer_stop(ctx, VOLDOR_TIMER_POSE, L.st, t0), "timer event");
    return VOLDOR_OK;
}

// FP32/FP64 pose tables from the caller's 6-vectors; with layout, also the row-pair flow
// layout (needed once per window: the flows do not change within it).
int prep_poses(GemLaunch& L, bool layout = true) {
    voldor_ctx ctx = L.ctx;
    VD_CHECK(vd::launch_pose_prep(L.b->pose, L.v->N, L.b->prior_pose, L.v->P, L.s.poses, L.s.posed, L.st),
             "pose prep launch");
    if (layout)
        VD_CHECK(vd::launch_flow_pairs((const float2*)L.b->flow, L.flow2, L.v->N, L.v->H, L.v->W, L.st),
                 "flow layout launch");
    return VOLDOR_OK;
}

// Final local E-step + confidence and statistics (poses already prepared).
int run_finalize(GemLaunch& L, int iter) {
    voldor_ctx ctx = L.ctx;
    int rc;
    if ((rc = run_level(L, iter, VOLDOR_LEVEL_LOCAL, 1, 0, true))) return rc;
    const vd::Win w = make_win(L.v, iter, 1, L.b);
    const vd::LevelGeom g = make_geom(L.v, w, 1, iter, L.kn);
    const vd::FinalBufs B = final_bufs(L);
    VD_CHECK(vd::launch_finalize(w, B, g.nchains, L.st), "finalize launch");
    return VOLDOR_OK;
}

// One GEM iteration on a prepared launch.  The first iteration of a call builds the pose
// tables (and the flow layout) from the caller's 6-vectors; later ones find them already
// built from the updated 6-vectors by the previous pose step's finish, with the same
// functions, so the tables are those a separate voldor_gem_step call would build.
int run_iteration(GemLaunch& L, int it, bool first) {
    int rc;
    if (first && (rc = prep_poses(L, true))) return rc;
    if ((rc = run_level(L, it, VOLDOR_LEVEL_COARSE, 1, 1, false))) return rc;
    if ((rc = run_level(L, it, VOLDOR_LEVEL_LOCAL, 1, 1, false))) return rc;
    return run_pose_step(L);
}

// A whole window on a prepared launch: iterations first .. first + n_iters - 1.
int run_window(GemLaunch& L, int first, int n_iters, int flags) {
    voldor_ctx ctx = L.ctx;
    int rc;
    if (flags & VOLDOR_RUN_INIT)
        VD_CHECK(vd::launch_init(make_win(L.v, 0, 1), L.b->idepth, boot_src(L.v, L.b), L.st), "init launch");
    for (int it = first; it < first + n_iters; ++it)
        if ((rc = run_iteration(L, it, it == first))) return rc;
    return run_finalize(L, first + n_iters - 1);
}

// ---- batched run: every window's scratch lives at once; each step of the launch sequence
// is one launch per (shape class) over all windows, driven by item tables in device memory

enum BKind { BK_PREP, BK_SETUP, BK_LEVEL, BK_POSE, BK_POSE_SOLVE, BK_FINAL, BK_FINAL_FINISH };

struct BLaunch {
    int kind;
    size_t items, b2i;         // byte offsets into the table region
    int n_items, nblocks;
    size_t lds;
    int mode, s;
    bool b2, pr;
};

struct BPlan {
    std::vector<char> host;
    std::vector<BLaunch> launches;
    template <class T>
    size_t put(const std::vector<T>& v) {
        const size_t off = align_up(host.size());
        host.resize(off + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
    void add(int kind, size_t items, size_t b2i, int n_items, int nblocks, size_t lds = 0, int mode = 0, int s = 0,
             bool b2 = true, bool pr = false) {
        launches.push_back(BLaunch{kind, items, b2i, n_items, nblocks, lds, mode, s, b2, pr});
    }
};

struct BWin {
    GemLaunch L;
    bool b2, pr;
};

// block -> item table of a launch whose items have the given block counts
std::vector<int> blocks_to_items(const std::vector<int>& counts, std::vector<int>& begins) {
    std::vector<int> b2i;
    begins.clear();
    for (size_t i = 0; i < counts.size(); ++i) {
        begins.push_back((int)b2i.size());
        b2i.insert(b2i.end(), (size_t)counts[i], (int)i);
    }
    return b2i;
}

// one level launch per shape class over the windows; geometry per window from make(L)
template <class MakeItem>
void plan_level(BPlan& P, const std::vector<BWin>& W, int mode, MakeItem make) {
    for (int cls = 0; cls < 4; ++cls) {
        const bool b2 = cls & 1, pr = cls & 2;
        std::vector<vd::LevelItem> items;
        std::vector<int> counts;
        size_t lds = 0;
        for (const BWin& bw : W) {
            if (bw.b2 != b2 || bw.pr != pr) continue;
            vd::LevelItem it = make(bw.L);
            int nb = it.g.nblocks;
            const size_t lat = (size_t)it.g.h * it.g.w;
            if (mode == 1) nb = (int)((lat * VD_PA_LANES + VD_BLOCK - 1) / VD_BLOCK);
            if (mode == 2) nb = (int)((lat * it.g.spec + VD_BLOCK - 1) / VD_BLOCK);
            if (mode == 0 || mode == 3) lds = std::max(lds, vd::level_lds_bytes(it.g));
            items.push_back(it);
            counts.push_back(nb);
        }
        if (items.empty()) continue;
        std::vector<int> begins;
        const std::vector<int> b2i = blocks_to_items(counts, begins);
        for (size_t i = 0; i < items.size(); ++i) items[i].begin = begins[i];
        const size_t io = P.put(items), bo = P.put(b2i);
        P.add(BK_LEVEL, io, bo, (int)items.size(), (int)b2i.size(), lds, mode, 0, b2, pr);
    }
}

int build_plan(voldor_ctx ctx, std::vector<BWin>& W, int n_iters, int flags, BPlan& P) {
    // setup: initial depth (when asked) and the flow layout, once per window
    {
        std::vector<vd::PrepItem> items;
        std::vector<int> counts;
        for (BWin& bw : W) {
            const GemLaunch& L = bw.L;
            vd::PrepItem it;
            std::memset(&it, 0, sizeof(it));
            it.w = make_win(L.v, 0, 1);
            it.idepth = L.b->idepth;
            it.flow = (const float2*)L.b->flow;
            it.flow2 = L.flow2;
            it.N = L.v->N;
            it.init = (flags & VOLDOR_RUN_INIT) ? 1 : 0;
            it.boot = boot_src(L.v, L.b);
            const int64_t npix = (int64_t)L.v->H * L.v->W;
            const int64_t pairs = (int64_t)(L.v->H - 1) * L.v->W * (L.v->N - 1);
            it.nblocks = (int)((std::max(npix, pairs) + VD_BLOCK - 1) / VD_BLOCK);
            items.push_back(it);
            counts.push_back(std::max(1, it.nblocks));
        }
        std::vector<int> begins;
        const std::vector<int> b2i = blocks_to_items(counts, begins);
        for (size_t i = 0; i < items.size(); ++i) items[i].begin = begins[i];
        const size_t io = P.put(items), bo = P.put(b2i);
        P.add(BK_SETUP, io, bo, (int)items.size(), (int)b2i.size());
    }
    // pose tables per window class (as every later per-iteration launch), so that the classes'
    // iteration chains need no common step until the statistics
    size_t prep_off[4] = {0, 0, 0, 0};
    int prep_n[4] = {0, 0, 0, 0};
    for (int cls = 0; cls < 4; ++cls) {
        std::vector<vd::PrepItem> prep;
        for (BWin& bw : W) {
            if ((bw.b2 ? 1 : 0) + (bw.pr ? 2 : 0) != cls) continue;
            const GemLaunch& L = bw.L;
            vd::PrepItem it;
            std::memset(&it, 0, sizeof(it));
            it.pose = L.b->pose;
            it.prior_pose = L.b->prior_pose;
            it.N = L.v->N;
            it.P = L.v->P;
            it.out = L.s.poses;
            it.outd = L.s.posed;
            prep.push_back(it);
        }
        prep_n[cls] = (int)prep.size();
        if (!prep.empty()) prep_off[cls] = P.put(prep);
    }
    auto add_prep = [&]() {
        for (int cls = 0; cls < 4; ++cls)
            if (prep_n[cls]) P.add(BK_PREP, prep_off[cls], 0, prep_n[cls], prep_n[cls], 0, 0, 0, cls & 1, cls & 2);
    };
    int maxS = 0;
    for (BWin& bw : W) maxS = std::max(maxS, bw.L.v->N * bw.L.v->pose_gn_steps);
    for (int it = 0; it < n_iters; ++it) {
        add_prep();
        auto item = [&](const GemLaunch& L, int level, int do_e, int do_m, bool want_ll) {
            vd::LevelItem x;
            std::memset(&x, 0, sizeof(x));
            x.w = make_win(L.v, it, level, L.b);
            x.g = make_geom(L.v, x.w, level, it, L.kn);
            x.g.pa_lanes = VD_PA_LANES;             // the batched phase-A grid keeps 8 lanes
            x.b = level_bufs(L, level, want_ll);
            if (level == VOLDOR_LEVEL_LOCAL) x.b.blk_order = block_order(L, x.g, x.w);
            x.do_e = do_e;
            x.do_m = do_m;
            return x;
        };
        plan_level(P, W, 3, [&](const GemLaunch& L) { return item(L, VOLDOR_LEVEL_COARSE, 1, 0, false); });
        plan_level(P, W, 1, [&](const GemLaunch& L) { return item(L, VOLDOR_LEVEL_COARSE, 0, 1, false); });
        plan_level(P, W, 2, [&](const GemLaunch& L) { return item(L, VOLDOR_LEVEL_COARSE, 0, 1, false); });
        plan_level(P, W, 3, [&](const GemLaunch& L) { return item(L, VOLDOR_LEVEL_COARSE, 0, 2, false); });
        plan_level(P, W, 0, [&](const GemLaunch& L) { return item(L, VOLDOR_LEVEL_LOCAL, 1, 1, false); });
        // pose step: Gauss-Newton step s of the windows that have one
        std::vector<vd::PoseItem> all;
        for (BWin& bw : W) {
            const GemLaunch& L = bw.L;
            vd::PoseItem x;
            std::memset(&x, 0, sizeof(x));
            x.w = make_win(L.v, 0, 1);
            x.b = pose_bufs(L);
            x.G = L.v->pose_gn_steps;
            x.S = L.v->N * L.v->pose_gn_steps;
            x.nblocks = L.gn_blocks;
            all.push_back(x);
        }
        // per window class (as the level launches), so that the classes' step chains run
        // side by side
        for (int s = 0; s < maxS; ++s) {
            for (int cls = 0; cls < 4; ++cls) {
                const bool b2 = cls & 1, pr = cls & 2;
                std::vector<vd::PoseItem> items;
                std::vector<int> counts;
                for (size_t i = 0; i < W.size(); ++i)
                    if (W[i].b2 == b2 && W[i].pr == pr && s < all[i].S) {
                        items.push_back(all[i]);
                        counts.push_back(all[i].nblocks);
                    }
                if (items.empty()) continue;
                std::vector<int> begins;
                const std::vector<int> b2i = blocks_to_items(counts, begins);
                for (size_t i = 0; i < items.size(); ++i) items[i].begin = begins[i];
                const size_t io = P.put(items), bo = P.put(b2i);
                P.add(BK_POSE, io, bo, (int)items.size(), (int)b2i.size(), 0, 0, s, b2, pr);
                // step s's solve, one block per window of the class that has the step
                P.add(BK_POSE_SOLVE, P.put(items), 0, (int)items.size(), (int)items.size(), 0, 0, s, b2, pr);
            }
        }
    }
    // final E-step, confidence and statistics
    add_prep();
    const int last = n_iters - 1;
    plan_level(P, W, 0, [&](const GemLaunch& L) {
        vd::LevelItem x;
        std::memset(&x, 0, sizeof(x));
        x.w = make_win(L.v, last, VOLDOR_LEVEL_LOCAL, L.b);
        x.g = make_geom(L.v, x.w, VOLDOR_LEVEL_LOCAL, last, L.kn);
        x.b = level_bufs(L, VOLDOR_LEVEL_LOCAL, true);
        x.b.blk_order = block_order(L, x.g, x.w);
        x.do_e = 1;
        x.do_m = 0;
        return x;
    });
    std::vector<vd::FinalItem> fin_all;
    for (BWin& bw : W) {
        const GemLaunch& L = bw.L;
        vd::FinalItem x;
        std::memset(&x, 0, sizeof(x));
        x.w = make_win(L.v, last, VOLDOR_LEVEL_LOCAL, L.b);
        x.b = final_bufs(L);
        x.n_ll = make_geom(L.v, x.w, VOLDOR_LEVEL_LOCAL, last, L.kn).nchains;
        x.nblocks = (int)(((int64_t)L.v->H * L.v->W + VD_BLOCK - 1) / VD_BLOCK);
        fin_all.push_back(x);
    }
    for (int cls = 0; cls < 4; ++cls) {
        const bool b2 = cls & 1, pr = cls & 2;
        std::vector<vd::FinalItem> items;
        std::vector<int> counts;
        for (size_t i = 0; i < W.size(); ++i)
            if (W[i].b2 == b2 && W[i].pr == pr) {
                items.push_back(fin_all[i]);
                counts.push_back(fin_all[i].nblocks);
            }
        if (items.empty()) continue;
        std::vector<int> begins;
        const std::vector<int> b2i = blocks_to_items(counts, begins);
        for (size_t i = 0; i < items.size(); ++i) items[i].begin = begins[i];
        const size_t io = P.put(items), bo = P.put(b2i);
        P.add(BK_FINAL, io, bo, (int)items.size(), (int)b2i.size(), 0, 0, 0, b2, pr);
    }
    P.add(BK_FINAL_FINISH, P.put(fin_all), 0, (int)fin_all.size(), (int)fin_all.size());
    for (const BLaunch& l : P.launches)
        if (l.lds > kLevelLdsMax) return fail(ctx, VOLDOR_EINVAL, "chain segment too long for LDS (%zu bytes)", l.lds);
    return VOLDOR_OK;
}

// The streams of the window classes (shape-2 cost or not, priors or not) and their events.
int ensure_class_streams(voldor_ctx ctx) {
    for (int c = 0; c < 4; ++c)
        if (!ctx->class_streams[c])
            VD_CHECK(hipStreamCreateWithFlags(&ctx->class_streams[c], hipStreamNonBlocking), "stream create");
    for (int i = 0; i < 5; ++i)
        if (!ctx->class_events[i])
            VD_CHECK(hipEventCreateWithFlags(&ctx->class_events[i], hipEventDisableTiming), "event create");
    return VOLDOR_OK;
}

// Enqueues the plan on st.  Every launch of one window class (all but the setup and the
// statistics' finish, which serve every window) goes to the class's own stream, forked from
// st at the class's first launch and joined back into st before the next launch that serves
// every window: the windows of different classes share no buffer, so the classes' whole
// iteration chains (latency-bound coarse launches and pose steps above all) overlap.
int enqueue_plan(voldor_ctx ctx, const BPlan& P, const char* dev, hipStream_t st) {
    const bool par = ctx->class_streams[0] != nullptr;
    unsigned open = 0;                           // classes forked in the current run
    auto join = [&]() -> int {
        for (int c = 0; c < 4; ++c)
            if (open & (1u << c)) {
                VD_CHECK(hipEventRecord(ctx->class_events[1 + c], ctx->class_streams[c]), "join record");
                VD_CHECK(hipStreamWaitEvent(st, ctx->class_events[1 + c], 0), "join wait");
            }
        open = 0;
        return VOLDOR_OK;
    };
    for (const BLaunch& l : P.launches) {
        hipStream_t s = st;
        if (par && l.kind != BK_SETUP && l.kind != BK_FINAL_FINISH) {
            const int c = (l.b2 ? 1 : 0) + (l.pr ? 2 : 0);
            if (!open) VD_CHECK(hipEventRecord(ctx->class_events[0], st), "fork record");
            if (!(open & (1u << c))) {
                VD_CHECK(hipStreamWaitEvent(ctx->class_streams[c], ctx->class_events[0], 0), "fork wait");
                open |= 1u << c;
            }
            s = ctx->class_streams[c];
        } else if (open) {
            const int rc = join();
            if (rc) return rc;
        }
        const void* items = dev + l.items;
        const int* b2i = (const int*)(dev + l.b2i);
        hipError_t e = hipSuccess;
        switch (l.kind) {
        case BK_PREP: e = vd::launch_prep_batch((const vd::PrepItem*)items, l.n_items, s); break;
        case BK_SETUP: e = vd::launch_setup_batch((const vd::PrepItem*)items, b2i, l.nblocks, st); break;
        case BK_LEVEL:
            e = vd::launch_level_batch((const vd::LevelItem*)items, b2i, l.nblocks, l.lds, l.mode, l.b2, l.pr, s);
            break;
        case BK_POSE: e = vd::launch_pose_gn_batch((const vd::PoseItem*)items, b2i, l.nblocks, l.s, l.b2, s); break;
        case BK_POSE_SOLVE: e = vd::launch_pose_gn_solve_batch((const vd::PoseItem*)items, l.n_items, l.s, s); break;
        case BK_FINAL: e = vd::launch_finalize_batch((const vd::FinalItem*)items, b2i, l.nblocks, l.b2, l.pr, s); break;
        case BK_FINAL_FINISH: e = vd::launch_finalize_finish_batch((const vd::FinalItem*)items, l.n_items, st); break;
        }
        VD_CHECK(e, "batched launch");
    }
    return open ? join() : VOLDOR_OK;
}

void drop_graph(voldor_ctx ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->batch_key.clear();
}

}  // namespace

namespace vdc {

namespace {
thread_local std::string g_create_err;
}

const char* create_error() { return g_create_err.c_str(); }

int fail(voldor_ctx ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_err = buf;
    return code;
}

int hip_fail(voldor_ctx ctx, hipError_t e, const char* what) {
    return fail(ctx, VOLDOR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int ensure_buffer(voldor_ctx ctx, void** buf, size_t* cap, size_t need, hipStream_t st) {
    if (need <= *cap) return VOLDOR_OK;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    if (*buf) {
        VD_CHECK(hipStreamSynchronize(st), "hipStreamSynchronize");
        VD_CHECK(hipFree(*buf), "hipFree");
        *buf = nullptr;
        *cap = 0;
    }
    const size_t bytes = need + need / 4;
    if (hipMalloc(buf, bytes) != hipSuccess) {
        *buf = nullptr;
        return fail(ctx, VOLDOR_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
    }
    *cap = bytes;
    return VOLDOR_OK;
}

}  // namespace vdc

// ======================================================================================
extern "C" {

int voldor_ctx_create(voldor_ctx* out, int device_ordinal) {
    if (!out) return fail(nullptr, VOLDOR_EINVAL, "null output pointer");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device_ordinal < 0 || device_ordinal >= n)
        return fail(nullptr, VOLDOR_EINVAL, "device %d not available (%d devices)", device_ordinal, n);
    voldor_ctx c = new (std::nothrow) voldor_ctx_s;
    if (!c) return fail(nullptr, VOLDOR_ENOMEM, "context allocation failed");
    c->device = device_ordinal;
    if (hipSetDevice(device_ordinal) != hipSuccess) {
        delete c;
        return fail(nullptr, VOLDOR_EDEVICE, "hipSetDevice(%d) failed", device_ordinal);
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device_ordinal) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    if (vd::set_level_lds_limit(kLevelLdsMax) != hipSuccess) {
        delete c;
        return fail(nullptr, VOLDOR_EDEVICE, "cannot raise the LDS limit of the level kernel");
    }
    noalloc_setup(device_ordinal);
    *out = c;
    return VOLDOR_OK;
}

void voldor_ctx_destroy(voldor_ctx ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->net_ws) (void)hipFree(ctx->net_ws);
    for (void* p : ctx->lane_ws)
        if (p) (void)hipFree(p);
    drop_graph(ctx);
    if (ctx->batch_ws) (void)hipFree(ctx->batch_ws);
    if (ctx->batch_tab) (void)hipFree(ctx->batch_tab);
    for (const auto& e : ctx->block_orders) (void)hipFree(e.d);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (hipStream_t s : ctx->class_streams)
        if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t e : ctx->class_events)
        if (e) (void)hipEventDestroy(e);
    timers_discard(ctx);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

const char* voldor_last_error(voldor_ctx ctx) {
    return ctx ? ctx->err.c_str() : vdc::create_error();
}

int voldor_lattice_shape(int32_t H, int32_t W, int32_t stride, int32_t* Hc, int32_t* Wc) {
    int hc, wc;
    if (!Hc || !Wc || !lattice(H, W, stride, &hc, &wc)) return VOLDOR_EINVAL;
    *Hc = hc;
    *Wc = wc;
    return VOLDOR_OK;
}

int voldor_init_idepth(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    VD_CHECK(vd::launch_init(make_win(v, 0, 1), b->idepth, boot_src(v, b), st), "init launch");
    return VOLDOR_OK;
}

int voldor_rigidness_fb(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int iter, int level,
                        void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (iter < 0 || iter > 0xffffff || (level != 0 && level != 1)) return fail(ctx, VOLDOR_EINVAL, "bad iter/level");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L))) return rc;
    if ((rc = prep_poses(L))) return rc;
    return run_level(L, iter, level, 1, 0, false);
}

int voldor_depth_update(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int iter, int level,
                        void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (iter < 0 || iter > 0xffffff || (level != 0 && level != 1)) return fail(ctx, VOLDOR_EINVAL, "bad iter/level");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L))) return rc;
    if ((rc = prep_poses(L))) return rc;
    return run_level(L, iter, level, 0, 1, false);
}

int voldor_level_step(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int iter, int level,
                      void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (iter < 0 || iter > 0xffffff || (level != 0 && level != 1)) return fail(ctx, VOLDOR_EINVAL, "bad iter/level");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L))) return rc;
    if ((rc = prep_poses(L))) return rc;
    return run_level(L, iter, level, 1, 1, false);
}

int voldor_pose_score(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int t, int n_cand,
                      const double* cand_pose, double* out, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (t < 1 || t > v->N) return fail(ctx, VOLDOR_EINVAL, "t=%d outside 1..N", t);
    if (n_cand < 1 || n_cand > (int)kMaxBatch || !cand_pose || !out)
        return fail(ctx, VOLDOR_EINVAL, "bad candidate set");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L, n_cand))) return rc;
    if ((rc = prep_poses(L))) return rc;
    vd::PoseBufs B;
    B.P = L.s.poses;
    B.PD = L.s.posed;
    B.flow = (const float2*)b->flow;
    B.flow2 = L.flow2;
    B.idepth = b->idepth;
    B.rigid = b->rigid;
    B.pose = b->pose;
    B.partials = L.pose_partials;
    B.out = out;
    VD_CHECK(vd::launch_pose(make_win(v, 0, 1), B, t, cand_pose, n_cand, 0, L.pose_blocks, st), "pose score launch");
    return VOLDOR_OK;
}

int voldor_pose_step(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L))) return rc;
    if ((rc = prep_poses(L))) return rc;
    return run_pose_step(L);
}

int voldor_gem_step(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int iter, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (iter < 0 || iter > 0xffffff) return fail(ctx, VOLDOR_EINVAL, "bad iter");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L))) return rc;
    return run_iteration(L, iter, true);
}

int voldor_finalize(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int iter, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (!b->conf || !b->stats) return fail(ctx, VOLDOR_EINVAL, "null conf/stats pointer");
    if (iter < 0 || iter > 0xffffff) return fail(ctx, VOLDOR_EINVAL, "bad iter");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L))) return rc;
    if ((rc = prep_poses(L))) return rc;
    return run_finalize(L, iter);
}

int voldor_run(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int first_iter, int n_iters,
               int flags, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (!b->conf || !b->stats) return fail(ctx, VOLDOR_EINVAL, "null conf/stats pointer");
    if (n_iters < 1 || first_iter < 0 || (int64_t)first_iter + n_iters > 0xffffff)
        return fail(ctx, VOLDOR_EINVAL, "need n_iters >= 1 and first_iter >= 0");
    if (flags & ~VOLDOR_RUN_INIT) return fail(ctx, VOLDOR_EINVAL, "unknown flags 0x%x", flags);
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    GemLaunch L;
    if ((rc = gem_prepare(ctx, v, b, st, L))) return rc;
    return run_window(L, first_iter, n_iters, flags);
}

int voldor_run_noalloc(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int first_iter,
                       int n_iters, int flags, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (!b->conf || !b->stats) return fail(ctx, VOLDOR_EINVAL, "null conf/stats pointer");
    if (n_iters < 1 || first_iter < 0 || (int64_t)first_iter + n_iters > 0xffffff)
        return fail(ctx, VOLDOR_EINVAL, "need n_iters >= 1 and first_iter >= 0");
    if (flags & ~VOLDOR_RUN_INIT) return fail(ctx, VOLDOR_EINVAL, "unknown flags 0x%x", flags);
    GemLaunch L;
    L.ctx = ctx; L.v = v; L.b = b; L.st = (hipStream_t)stream;
    L.timers = false;
    L.may_alloc = false;
    const size_t need = gem_layout(v, 1, L);
    if (need > (size_t)VOLDOR_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, VOLDOR_EINVAL, "window %dx%d with N=%d needs %zu bytes of scratch; the static area holds %zu",
                    v->W, v->H, v->N, need, (size_t)VOLDOR_NOALLOC_SCRATCH_BYTES);
    hipError_t e = hipSuccess;
    void* base = noalloc_base(ctx->device, &e);
    if (!base) return hip_fail(ctx, e, "static scratch address of this device");
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    gem_carve((char*)base, L);
    return run_window(L, first_iter, n_iters, flags);
}

}  // extern "C"

namespace {

// The batched run, optionally with every window started by the proposal network (net set):
// windows the network can take (even H and W) get its start, with the random start where
// its output is unusable (fallback_out[i] = 1); the others take the random start.
int batch_run_impl(voldor_ctx ctx, const voldor_net* net, int n_windows, const voldor_window* wins,
                   const voldor_buffers* bufs, int n_iters, int flags, int32_t* fallback_out, hipStream_t st) {
    if (!ctx) return VOLDOR_EINVAL;
    if (n_windows < 1 || n_windows > (int)kMaxBatch || !wins || !bufs)
        return fail(ctx, VOLDOR_EINVAL, "bad window batch");
    if (n_iters < 1 || n_iters > 0xffffff) return fail(ctx, VOLDOR_EINVAL, "n_iters must be >= 1");
    if (flags & ~(VOLDOR_RUN_INIT | VOLDOR_RUN_NO_GRAPH)) return fail(ctx, VOLDOR_EINVAL, "unknown flags 0x%x", flags);
    if (net && (!net->params || !net->wbf16)) return fail(ctx, VOLDOR_EINVAL, "null network pointer");
    if (net) flags &= ~VOLDOR_RUN_INIT;        // the starts come from the network (or its fallback)
    int rc;
    for (int i = 0; i < n_windows; ++i) {
        if ((rc = check_window(ctx, &wins[i], &bufs[i]))) return rc;
        if (!bufs[i].conf || !bufs[i].stats) return fail(ctx, VOLDOR_EINVAL, "null conf/stats pointer (window %d)", i);
    }
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    const bool use_graph = !(flags & VOLDOR_RUN_NO_GRAPH);
    // the same windows, buffers and settings as the captured graph: replay it
    const voldor_net no_net = {};
    const voldor_net& nk = net ? *net : no_net;
    std::vector<char> key(sizeof(int) * 2 + sizeof(voldor_net) + sizeof(void*) +
                          n_windows * (sizeof(voldor_window) + sizeof(voldor_buffers)));
    {
        char* k = key.data();
        const int hdr[2] = {n_iters, flags & VOLDOR_RUN_INIT};
        std::memcpy(k, hdr, sizeof(hdr));
        k += sizeof(hdr);
        std::memcpy(k, &nk, sizeof(voldor_net));
        k += sizeof(voldor_net);
        std::memcpy(k, &fallback_out, sizeof(void*));
        k += sizeof(void*);
        std::memcpy(k, wins, n_windows * sizeof(voldor_window));
        std::memcpy(k + n_windows * sizeof(voldor_window), bufs, n_windows * sizeof(voldor_buffers));
    }
    if (use_graph && ctx->graph_exec && key == ctx->batch_key) {
        VD_CHECK(hipGraphLaunch(ctx->graph_exec, st), "hipGraphLaunch");
        return VOLDOR_OK;
    }
    // layout: every window's scratch, then the item tables
    std::vector<BWin> W((size_t)n_windows);
    size_t total = 0;
    std::vector<size_t> offs((size_t)n_windows);
    for (int i = 0; i < n_windows; ++i) {
        GemLaunch& L = W[i].L;
        L.ctx = ctx; L.v = &wins[i]; L.b = &bufs[i]; L.st = st;
        offs[i] = total;
        total += align_up(gem_layout(&wins[i], 1, L));
        W[i].b2 = wins[i].fisk_beta == 2.0f;
        W[i].pr = wins[i].P > 0;
    }
    // a new set of windows: the old graph goes before its buffers may be replaced
    drop_graph(ctx);
    if ((rc = vdc::ensure_buffer(ctx, &ctx->batch_ws, &ctx->batch_ws_bytes, total, st))) return rc;
    for (int i = 0; i < n_windows; ++i) gem_carve((char*)ctx->batch_ws + offs[i], W[i].L);
    auto net_ok = [&](const voldor_window& v) { return !(v.H & 1) && !(v.W & 1) && (int64_t)v.H * v.W <= (1 << 26); };
    auto lane_of = [&](int i) { return (W[i].b2 ? 1 : 0) + (W[i].pr ? 2 : 0); };
    if (net) {
        // a forward workspace per class stream for the largest window of the class, allocated
        // before any capture
        int64_t best[4] = {0, 0, 0, 0};
        int bi[4] = {-1, -1, -1, -1};
        for (int i = 0; i < n_windows; ++i) {
            const int c = lane_of(i);
            if (net_ok(wins[i]) && (int64_t)wins[i].H * wins[i].W > best[c]) {
                best[c] = (int64_t)wins[i].H * wins[i].W;
                bi[c] = i;
            }
        }
        for (int c = 0; c < 4; ++c)
            if (bi[c] >= 0 && (rc = vdc::net_workspace(ctx, wins[bi[c]].H, wins[bi[c]].W, st, c))) return rc;
    }
    BPlan plan;
    if ((rc = build_plan(ctx, W, n_iters, flags, plan))) return rc;
    if ((rc = vdc::ensure_buffer(ctx, &ctx->batch_tab, &ctx->batch_tab_bytes, plan.host.size(), st))) return rc;
    char* tables = (char*)ctx->batch_tab;
    ctx->batch_host = plan.host;
    VD_CHECK(hipMemcpyAsync(tables, ctx->batch_host.data(), ctx->batch_host.size(), hipMemcpyHostToDevice, st),
             "table upload");
    VD_CHECK(hipStreamSynchronize(st), "hipStreamSynchronize");
    if ((rc = ensure_class_streams(ctx))) return rc;
    auto enqueue = [&](hipStream_t s) -> int {
        if (net) {
            // each window's start on its class stream with that stream's workspace, so the
            // classes' network passes overlap; joined back into s before the plan
            unsigned open = 0;
            VD_CHECK(hipEventRecord(ctx->class_events[0], s), "fork record");
            for (int i = 0; i < n_windows; ++i) {
                const voldor_window& v = wins[i];
                const voldor_buffers& b = bufs[i];
                const int c = lane_of(i);
                hipStream_t cs = ctx->class_streams[c];
                if (!(open & (1u << c))) {
                    VD_CHECK(hipStreamWaitEvent(cs, ctx->class_events[0], 0), "fork wait");
                    open |= 1u << c;
                }
                int32_t* fo = fallback_out ? fallback_out + i : nullptr;
                int* flag = nullptr;
                if (net_ok(v)) {
                    int r = vdc::proposal_start(ctx, net, v.H, v.W, v.N, b.flow, b.pose, v.idepth_min, v.idepth_max,
                                                b.idepth, b.rigid, &flag, cs, c);
                    if (r) return r;
                }
                VD_CHECK(vd::launch_init_if(make_win(&v, 0, 1), b.idepth, boot_src(&v, &b), flag, fo, cs), "start launch");
            }
            for (int c = 0; c < 4; ++c)
                if (open & (1u << c)) {
                    VD_CHECK(hipEventRecord(ctx->class_events[1 + c], ctx->class_streams[c]), "join record");
                    VD_CHECK(hipStreamWaitEvent(s, ctx->class_events[1 + c], 0), "join wait");
                }
        }
        return enqueue_plan(ctx, plan, tables, s);
    };
    if (!use_graph) return enqueue(st);
    if (!ctx->cap_stream) VD_CHECK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "stream create");
    VD_CHECK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed), "begin capture");
    rc = enqueue(ctx->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    VD_CHECK(ec, "end capture");
    ctx->graph = g;
    VD_CHECK(hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0), "graph instantiate");
    ctx->batch_key = key;
    VD_CHECK(hipGraphLaunch(ctx->graph_exec, st), "hipGraphLaunch");
    return VOLDOR_OK;
}

}  // namespace

extern "C" {

int voldor_batch_run(voldor_ctx ctx, int n_windows, const voldor_window* wins, const voldor_buffers* bufs,
                     int n_iters, int flags, void* stream) {
    return batch_run_impl(ctx, nullptr, n_windows, wins, bufs, n_iters, flags, nullptr, (hipStream_t)stream);
}

int voldor_batch_run_learned(voldor_ctx ctx, const voldor_net* net, int n_windows, const voldor_window* wins,
                             const voldor_buffers* bufs, int n_iters, int flags, int32_t* fallback_out, void* stream) {
    if (ctx && !net) return fail(ctx, VOLDOR_EINVAL, "null network");
    return batch_run_impl(ctx, net, n_windows, wins, bufs, n_iters, flags, fallback_out, (hipStream_t)stream);
}

int voldor_proposal_start(voldor_ctx ctx, const voldor_net* net, const voldor_window* v, const voldor_buffers* b,
                          int32_t* fallback_out, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    int* flag = nullptr;
    if ((rc = vdc::proposal_start(ctx, net, v->H, v->W, v->N, b->flow, b->pose, v->idepth_min, v->idepth_max,
                                  b->idepth, b->rigid, &flag, st)))
        return rc;
    VD_CHECK(vd::launch_init_if(make_win(v, 0, 1), b->idepth, boot_src(v, b), flag, fallback_out, st), "fallback launch");
    return VOLDOR_OK;
}

int voldor_set_knobs(voldor_ctx ctx, const voldor_window* bucket, const voldor_knobs* knobs) {
    if (!ctx) return VOLDOR_EINVAL;
    if (!bucket) return fail(ctx, VOLDOR_EINVAL, "null bucket window");
    auto same = [&](const voldor_ctx_s::KnobEntry& e) {
        return e.H == bucket->H && e.W == bucket->W && e.N == bucket->N && e.K == bucket->n_candidates &&
               e.prior == (bucket->P > 0);
    };
    if (knobs) {
        const voldor_knobs& k = *knobs;
        if (k.local_chains < 0 || k.local_chains > VD_BLOCK) return fail(ctx, VOLDOR_EINVAL, "local_chains outside 0..%d", VD_BLOCK);
        if (k.local_spec < 0 || k.local_spec > VD_SPEC || k.coarse_spec < 0 || k.coarse_spec > VD_SPEC)
            return fail(ctx, VOLDOR_EINVAL, "speculation depths outside 0..%d", VD_SPEC);
        if (k.coarse_lanes != 0 && k.coarse_lanes != 4 && k.coarse_lanes != 8 && k.coarse_lanes != 16)
            return fail(ctx, VOLDOR_EINVAL, "coarse_lanes must be 0, 4, 8 or 16");
        if (k.local_order < 0 || k.local_order > 2) return fail(ctx, VOLDOR_EINVAL, "local_order must be 0, 1 or 2");
    }
    // a batch graph captured with the old knobs would no longer match the table
    drop_graph(ctx);
    for (auto& e : ctx->knobs)
        if (same(e)) {
            if (knobs) e.k = *knobs;
            else { e = ctx->knobs.back(); ctx->knobs.pop_back(); }
            return VOLDOR_OK;
        }
    if (knobs) ctx->knobs.push_back({bucket->H, bucket->W, bucket->N, bucket->n_candidates, bucket->P > 0, *knobs});
    return VOLDOR_OK;
}

int voldor_get_knobs(voldor_ctx ctx, const voldor_window* win, voldor_knobs* out) {
    if (!ctx) return VOLDOR_EINVAL;
    if (!win || !out) return fail(ctx, VOLDOR_EINVAL, "null pointer");
    *out = knobs_for(ctx, win);
    return VOLDOR_OK;
}

int voldor_timing(voldor_ctx ctx, int mask) {
    if (!ctx) return VOLDOR_EINVAL;
    if (mask < 0 || mask >= (1 << kTimers)) return fail(ctx, VOLDOR_EINVAL, "timer mask %d outside 0..%d", mask, (1 << kTimers) - 1);
    timers_discard(ctx);
    ctx->timing = (unsigned)mask;
    return VOLDOR_OK;
}

int voldor_timing_read(voldor_ctx ctx, int timer, double* total_ms, int64_t* launches) {
    if (!ctx) return VOLDOR_EINVAL;
    if (timer < 0 || timer >= kTimers || !total_ms || !launches) return fail(ctx, VOLDOR_EINVAL, "bad timer query");
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    double sum = 0.0;
    auto& rec = ctx->ev_rec[timer];
    for (auto& p : rec) {
        float ms = 0.f;
        VD_CHECK(hipEventSynchronize(p.second), "hipEventSynchronize");
        VD_CHECK(hipEventElapsedTime(&ms, p.first, p.second), "hipEventElapsedTime");
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)rec.size();
    for (auto& p : rec) {
        ctx->ev_pool.push_back(p.first);
        ctx->ev_pool.push_back(p.second);
    }
    rec.clear();
    return VOLDOR_OK;
}

int voldor_pose_sample(voldor_ctx ctx, const voldor_window* v, const voldor_buffers* b, int iter,
                       const voldor_sample_params* sp, double* cov_out, double* info_out, void* stream) {
    int rc = check_window(ctx, v, b);
    if (rc) return rc;
    if (!sp) return fail(ctx, VOLDOR_EINVAL, "null sampling parameters");
    if (iter < 0 || iter > 0xffffff) return fail(ctx, VOLDOR_EINVAL, "bad iter");
    if (sp->samples < 1 || sp->samples > VOLDOR_POSE_MAX_SAMPLES)
        return fail(ctx, VOLDOR_EINVAL, "samples outside 1..%d", VOLDOR_POSE_MAX_SAMPLES);
    if (sp->tries < 1 || sp->tries > 64) return fail(ctx, VOLDOR_EINVAL, "tries outside 1..64");
    if (!(sp->sigma_w > 0) || !(sp->sigma_t_rel > 0) || !(sp->eps > 0) || !std::isfinite(sp->sigma_w) ||
        !std::isfinite(sp->sigma_t_rel))
        return fail(ctx, VOLDOR_EINVAL, "kernel widths and eps must be > 0");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    rc = vdc::ensure_buffer(ctx, &ctx->scratch, &ctx->scratch_bytes, sizeof(double) * 12 * (size_t)sp->samples, st);
    if (rc) return rc;
    vd::PoseSampleArgs a;
    a.H = v->H; a.W = v->W; a.N = v->N;
    a.fx = v->fx; a.fy = v->fy; a.cx = v->cx; a.cy = v->cy;
    a.S = sp->samples; a.tries = sp->tries; a.it = iter;
    a.sigma_w = sp->sigma_w; a.sigma_t_rel = sp->sigma_t_rel; a.eps = sp->eps;
    a.key0 = (uint32_t)(v->seed & 0xffffffffu);
    a.key1 = (uint32_t)(v->seed >> 32);
    a.window_id = v->window_id;
    vd::PoseSampleBufs B;
    B.flow = (const float2*)b->flow;
    B.idepth = b->idepth;
    B.rigid = b->rigid;
    B.pose = b->pose;
    B.samples = (double*)ctx->scratch;
    B.cov = cov_out;
    B.info = info_out;
    VD_CHECK(vd::launch_pose_sample(a, B, st), "pose sampling launch");
    return VOLDOR_OK;
}

int voldor_vc_scores(voldor_ctx ctx, const voldor_vc_params* vp, const float* idepth, const float* conf,
                     int n_poses, const double* poses, double tau, double* out, int32_t* first_below,
                     void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    if (!vp) return fail(ctx, VOLDOR_EINVAL, "null params");
    if (vp->H < 1 || vp->W < 1 || (int64_t)vp->H * vp->W > (1 << 28)) return fail(ctx, VOLDOR_EINVAL, "bad image size");
    if (!(vp->fx > 0) || !(vp->fy > 0) || !std::isfinite(vp->cx) || !std::isfinite(vp->cy))
        return fail(ctx, VOLDOR_EINVAL, "bad intrinsics");
    if (vp->cell < 1 || vp->cell > 1024) return fail(ctx, VOLDOR_EINVAL, "cell outside 1..1024");
    if (n_poses < 1 || n_poses > VOLDOR_VC_MAX_POSES)
        return fail(ctx, VOLDOR_EINVAL, "n_poses outside 1..%d", VOLDOR_VC_MAX_POSES);
    if (!idepth || !poses || !out) return fail(ctx, VOLDOR_EINVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    vd::VcArgs a;
    a.H = vp->H; a.W = vp->W; a.cell = vp->cell;
    a.hc = (vp->H + vp->cell - 1) / vp->cell;
    a.wc = (vp->W + vp->cell - 1) / vp->cell;
    a.words = (int)(((int64_t)a.hc * a.wc + 31) / 32);
    a.n = n_poses;
    a.fx = vp->fx; a.fy = vp->fy; a.cx = vp->cx; a.cy = vp->cy;
    a.conf_min = vp->conf_min;
    a.tau = tau;
    a.lds_bits = (size_t)a.words * n_poses <= 8192;   // up to 32 KB of LDS bitmaps per block
    const size_t rt_bytes = align_up(sizeof(double) * 12 * (size_t)n_poses);
    const size_t cnt_bytes = align_up(sizeof(uint32_t) * (size_t)(n_poses + 1));
    const size_t bit_bytes = align_up(sizeof(uint32_t) * (size_t)a.words * n_poses);
    int rc = vdc::ensure_buffer(ctx, &ctx->scratch, &ctx->scratch_bytes, rt_bytes + cnt_bytes + bit_bytes, st);
    if (rc) return rc;
    char* base = (char*)ctx->scratch;
    vd::VcBufs B;
    B.idepth = idepth; B.conf = conf; B.pose = poses;
    B.RT = (double*)base;
    B.count = (uint32_t*)(base + rt_bytes);
    B.bits = (uint32_t*)(base + rt_bytes + cnt_bytes);
    B.out = out; B.first_below = first_below;
    VD_CHECK(vd::launch_vc(a, B, st), "visibility-coverage launch");
    return VOLDOR_OK;
}

int voldor_align_sim3(voldor_ctx ctx, const voldor_align_params* ap, int n_pairs, const float* idepth1,
                      const float* idepth2, const float* conf2, double* pose_inout, double* scale_inout,
                      double* cov_out, double* stats_out, int32_t* status_out, void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    if (!ap) return fail(ctx, VOLDOR_EINVAL, "null params");
    if (n_pairs < 0 || n_pairs > (int)kMaxBatch) return fail(ctx, VOLDOR_EINVAL, "n_pairs outside 0..%zu", kMaxBatch);
    if (n_pairs == 0) return VOLDOR_OK;
    if (ap->H < 3 || ap->W < 3 || (int64_t)ap->H * ap->W > (1 << 28)) return fail(ctx, VOLDOR_EINVAL, "bad image size");
    if (!(ap->fx > 0) || !(ap->fy > 0)) return fail(ctx, VOLDOR_EINVAL, "bad intrinsics");
    if (ap->robust != 0 && ap->robust != 1) return fail(ctx, VOLDOR_EINVAL, "robust must be 0 or 1");
    if (!(ap->robust_scale > 0) || !(ap->normal_disc_rel > 0))
        return fail(ctx, VOLDOR_EINVAL, "robust_scale and normal_disc_rel must be > 0");
    if (ap->gn_steps < 0 || ap->gn_steps > 1000) return fail(ctx, VOLDOR_EINVAL, "gn_steps outside 0..1000");
    if (!idepth1 || !idepth2 || !conf2 || !pose_inout || !scale_inout || !cov_out || !stats_out || !status_out)
        return fail(ctx, VOLDOR_EINVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t plane = (size_t)ap->H * ap->W;
    const int nblk = (int)std::min<size_t>(std::max<size_t>(1, (plane + VD_BLOCK * 4 - 1) / (VD_BLOCK * 4)), 512);
    const size_t nrm_bytes = align_up(sizeof(float4) * plane * n_pairs);
    const size_t part_bytes = align_up(sizeof(double) * 37 * nblk * (size_t)n_pairs);
    const size_t state_bytes = align_up(sizeof(double) * vd::sim3_state_doubles(n_pairs));
    int rc = vdc::ensure_buffer(ctx, &ctx->scratch, &ctx->scratch_bytes, nrm_bytes + part_bytes + state_bytes, st);
    if (rc) return rc;
    char* base = (char*)ctx->scratch;
    vd::AlignArgs a;
    a.H = ap->H; a.W = ap->W;
    a.fx = ap->fx; a.fy = ap->fy; a.cx = ap->cx; a.cy = ap->cy;
    a.ifx = (float)(1.0 / (double)ap->fx);
    a.ify = (float)(1.0 / (double)ap->fy);
    a.robust = ap->robust; a.scale = ap->robust_scale; a.disc = ap->normal_disc_rel; a.s = 1.0f;
    a.n_pairs = n_pairs;
    vd::AlignBufs B;
    B.idepth1 = idepth1; B.idepth2 = idepth2; B.conf2 = conf2;
    B.normals = (float4*)base;
    B.partials = (double*)(base + nrm_bytes);
    B.pose = pose_inout; B.cov = cov_out; B.stats = stats_out; B.status = status_out;
    double* state = (double*)(base + nrm_bytes + part_bytes);
    VD_CHECK(vd::launch_align_prepare(a, B, st), "align prepare launch");
    VD_CHECK(vd::launch_align_sim3(a, B, scale_inout, state, ap->gn_steps, nblk, st), "sim(3) alignment launch");
    return VOLDOR_OK;
}

int voldor_align_p2p(voldor_ctx ctx, const voldor_align_params* ap, int n_pairs, const float* idepth1,
                     const float* idepth2, const float* conf2, double* pose_inout, double* cov_out,
                     double* stats_out, int32_t* status_out, void* stream) {
    if (!ctx) return VOLDOR_EINVAL;
    if (!ap) return fail(ctx, VOLDOR_EINVAL, "null params");
    if (n_pairs < 0 || n_pairs > (int)kMaxBatch) return fail(ctx, VOLDOR_EINVAL, "n_pairs outside 0..%zu", kMaxBatch);
    if (n_pairs == 0) return VOLDOR_OK;
    if (ap->H < 3 || ap->W < 3 || (int64_t)ap->H * ap->W > (1 << 28)) return fail(ctx, VOLDOR_EINVAL, "bad image size");
    if (!(ap->fx > 0) || !(ap->fy > 0)) return fail(ctx, VOLDOR_EINVAL, "bad intrinsics");
    if (ap->robust != 0 && ap->robust != 1) return fail(ctx, VOLDOR_EINVAL, "robust must be 0 or 1");
    if (!(ap->robust_scale > 0) || !(ap->scale_s > 0) || !(ap->normal_disc_rel > 0))
        return fail(ctx, VOLDOR_EINVAL, "robust_scale, scale_s and normal_disc_rel must be > 0");
    if (ap->gn_steps < 0 || ap->gn_steps > 1000) return fail(ctx, VOLDOR_EINVAL, "gn_steps outside 0..1000");
    if (!idepth1 || !idepth2 || !conf2 || !pose_inout || !cov_out || !stats_out || !status_out)
        return fail(ctx, VOLDOR_EINVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    VD_CHECK(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t plane = (size_t)ap->H * ap->W;
    const int nblk = (int)std::min<size_t>(std::max<size_t>(1, (plane + VD_BLOCK * 4 - 1) / (VD_BLOCK * 4)), 512);
    const size_t nrm_bytes = align_up(sizeof(float4) * plane * n_pairs);
    const size_t part_bytes = align_up(sizeof(double) * 29 * nblk * (size_t)n_pairs);
    int rc = vdc::ensure_buffer(ctx, &ctx->scratch, &ctx->scratch_bytes, nrm_bytes + part_bytes, st);
    if (rc) return rc;
    char* base = (char*)ctx->scratch;
    vd::AlignArgs a;
    a.H = ap->H; a.W = ap->W;
    a.fx = ap->fx; a.fy = ap->fy; a.cx = ap->cx; a.cy = ap->cy;
    a.ifx = (float)(1.0 / (double)ap->fx);
    a.ify = (float)(1.0 / (double)ap->fy);
    a.robust = ap->robust; a.scale = ap->robust_scale; a.disc = ap->normal_disc_rel; a.s = ap->scale_s;
    a.n_pairs = n_pairs;
    vd::AlignBufs B;
    B.idepth1 = idepth1; B.idepth2 = idepth2; B.conf2 = conf2;
    B.normals = (float4*)base;
    B.partials = (double*)(base + nrm_bytes);
    B.pose = pose_inout; B.cov = cov_out; B.stats = stats_out; B.status = status_out;
    VD_CHECK(vd::launch_align_prepare(a, B, st), "align prepare launch");
    for (int k = 0; k < ap->gn_steps; ++k) VD_CHECK(vd::launch_align_step(a, B, 0, nblk, st), "align step launch");
    VD_CHECK(vd::launch_align_step(a, B, 1, nblk, st), "align final launch");
    return VOLDOR_OK;
}

}  // extern "C"
