// Library context shared by the C-ABI translation units: device, last error message,
// scratch / workspace buffers and launch timers.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <string>
#include <utility>
#include <vector>

#include "../../include/voldor.h"

constexpr int kTimers = 3;

struct voldor_ctx_s {
    int device = 0;
    std::string err;
    void* scratch = nullptr;          // GEM scratch (pose tables, flow layout, partials)
    size_t scratch_bytes = 0;
    void* net_ws = nullptr;           // proposal-network workspace (activations, gradients)
    size_t net_ws_bytes = 0;
    void* lane_ws[4] = {};            // batched learned start: forward workspace per class stream
    size_t lane_ws_bytes[4] = {};
    void* batch_ws = nullptr;         // batched run: every window's scratch
    size_t batch_ws_bytes = 0;
    void* batch_tab = nullptr;        // batched run: item tables of the launch sequence
    size_t batch_tab_bytes = 0;
    std::vector<char> batch_host;     // host copy of the item tables
    std::vector<char> batch_key;      // windows / buffers / settings of the captured graph
    hipStream_t cap_stream = nullptr; // capture stream (default priority, non-blocking)
    hipStream_t class_streams[4] = {};  // batched run: one stream per window class (same)
    hipEvent_t class_events[5] = {};    // their fork (0) and join (1 + class) events
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    struct KnobEntry {                // launch knobs per (H, W, N, K, prior) bucket
        int32_t H, W, N, K;
        bool prior;
        voldor_knobs k;
    };
    std::vector<KnobEntry> knobs;
    struct BlockOrder {               // local-level block order of one level geometry
        std::array<int, 10> key;      // geometry fields and the principal point's bits
        int* d;                       // device copy [nblocks]
    };
    std::vector<BlockOrder> block_orders;
    int n_cu = 256;
    unsigned timing = 0;              // enabled timer classes, bit (1 << timer)
    std::vector<hipEvent_t> ev_pool;                                   // idle events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_rec[kTimers];    // recorded brackets
};

namespace vdc {

// Records the message on ctx (or as the thread's context-creation error when ctx is null)
// and returns code.
int fail(voldor_ctx ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int hip_fail(voldor_ctx ctx, hipError_t e, const char* what);
const char* create_error();
// Grows *buf (device memory on ctx's device) to at least need bytes; the old contents are
// not kept.  Waits for st before freeing a smaller buffer.
int ensure_buffer(voldor_ctx ctx, void** buf, size_t* cap, size_t need, hipStream_t st);
// Proposal network (proposal_api.hip): sizes the context's network workspace for an H x W
// input; runs the network on a window's flows and writes its start (inverse depth, rigidness)
// with *flag (device) set where the output is unusable.
// lane >= 0: the forward workspace of that class stream of the batched run instead.
int net_workspace(voldor_ctx ctx, int H, int W, hipStream_t st, int lane = -1);
int proposal_start(voldor_ctx ctx, const voldor_net* net, int H, int W, int N, const float* flow, const double* pose,
                   float rmin, float rmax, float* idepth, float* rigid, int** flag, hipStream_t st, int lane = -1);

}  // namespace vdc

#define VD_CHECK(call, what)                                        \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return vdc::hip_fail(ctx, e_, what);  \
    } while (0)
