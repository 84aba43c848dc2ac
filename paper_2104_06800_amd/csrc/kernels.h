// Internal interface between the C-ABI layer (api.hip) and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vd {

struct PoseF;
struct PoseD;
struct Win;

// Chain geometry of one launch of the level kernel.
struct LevelGeom {
    int h, w;          // level grid (coarse lattice or full image)
    int s, off;        // full-resolution coordinate = s * index + off
    int seg;           // chain segment length (tile, or a whole lattice row / column)
    int horizontal;    // chains run along x
    int C;             // chain segments per block
    int nseg;          // segments per line
    int nblocks;
    int spec;          // speculation depth of the chain scan
    int ncost;         // frames of E-step costs kept for a fused pass's M-step (0: none)
    int pa_lanes;      // lanes per lattice node of the separate phase-A grid (4, 8 or 16)
    int nchains;       // chain segments of the level (one log-likelihood entry each)
    int nf;            // frames of the per-frame LDS arrays: max(N, 3) (the scan reuses them)
};

struct LevelBufs {
    const PoseF* P;
    const float2* flow;
    const float4* flow2;         // row-pair layout of frames t >= 2
    const float* idepth;         // full resolution, read
    const float* idepth_coarse;  // slot 2 source (local level)
    const int* blk_order;        // logical block of each launched block (null: in order)
    const float* prior;
    const float* prior_weight;
    float* q_out;                // E-step output (level grid)
    const float* q_in;           // M-step input when the E-step is not fused
    float* rho_out;              // M-step output (coarse lattice or full image)
    double* ll_partial;          // per-block log-likelihood, or null
    double* pa_E;                // phase-A results per level pixel (split M-step)
    float* pa_V;
    int* pa_S;
    double* pa_spec;             // [spec][level plane] speculative predecessor energies
};

struct PoseBufs {
    PoseF* P;
    PoseD* PD;
    const float2* flow;
    const float4* flow2;
    const float* idepth;
    const float* rigid;
    double* pose;
    double* partials;
    double* out;
    PoseD* hist;                 // per-step pose history of a pose step (N * G entries)
    float2* obs;                 // observed displacement of the current frame
};

struct FinalBufs {
    const PoseF* P;
    const float2* flow;
    const float4* flow2;
    const float* idepth;
    const float* rigid;
    const float* prior;
    const float* prior_weight;
    float* conf;
    double* stats;
    double* partials;
    const double* ll_partial;
};

struct AlignArgs {
    int H, W;
    float fx, fy, cx, cy, ifx, ify;
    int robust;
    float scale;
    float disc;
    float s;
    int n_pairs;
};

struct AlignBufs {
    const float* idepth1;
    const float* idepth2;
    const float* conf2;
    float4* normals;
    double* pose;
    double* cov;
    double* stats;
    int32_t* status;
    double* partials;
};

// Visibility-coverage scores: frame 1's inverse depth against n poses of frame 2.
struct VcArgs {
    int H, W;
    int cell, hc, wc;          // coverage cell size and the cell grid of frame 2
    int words;                 // 32-bit words of one pose's coverage bitmap
    int n;                     // poses
    double fx, fy, cx, cy;
    float conf_min;
    double tau;
    int lds_bits;              // the block gathers its coverage bits in LDS first
};

struct VcBufs {
    const float* idepth;       // [H][W]
    const float* conf;         // [H][W] or null
    const double* pose;        // [n][6]
    double* RT;                // [n][12] scratch: R row-major, t
    uint32_t* count;           // [1 + n] scratch: depth pixels, visible per pose
    uint32_t* bits;            // [n][words] scratch: coverage bitmaps
    double* out;               // [n][5]
    int32_t* first_below;      // [1] or null
};

// Sampled pose M-step (Monte-Carlo P3P, meanshift, covariance fit) of frames 1..N.
struct PoseSampleArgs {
    int H, W, N;
    double fx, fy, cx, cy;
    int S, tries, it;
    double sigma_w, sigma_t_rel, eps;
    uint32_t key0, key1, window_id;
};

struct PoseSampleBufs {
    const float2* flow;        // [N][H][W]
    const float* idepth;       // [H][W]
    const float* rigid;        // [N][H][W]
    double* pose;              // [N][6] in/out
    double* samples;           // [S][12] scratch: R (9), t (3), NaN when void
    double* cov;               // [N][36] or null
    double* info;              // [N][4] or null
};

// ---- batched launches over many windows: one item per window and launch; a block finds
// its item through blk2item[global block] and its block index within the window as
// (global block - begin).  Global blocks are XCD-remapped first.
struct LevelItem {
    Win w;
    LevelGeom g;
    LevelBufs b;
    int do_e, do_m;
    int begin;
};

struct PoseItem {
    Win w;
    PoseBufs b;
    int G, S;          // Gauss-Newton steps per frame, steps of the window (N * G)
    int begin, nblocks;
};

struct FinalItem {
    Win w;
    FinalBufs b;
    int n_ll;
    int begin, nblocks;
};

// first depth prior of a window, which the initial inverse depth starts from (null prior:
// random start everywhere)
struct InitSrc {
    const float* prior;          // prior 0's inverse depth [H][W]
    const double* pose;          // prior 0's pose 6-vector
};

struct PrepItem {
    const double* pose;
    const double* prior_pose;
    int N, P;
    PoseF* out;
    PoseD* outd;
    // initial depth and flow layout (done once per window)
    Win w;
    float* idepth;
    const float2* flow;
    float4* flow2;
    InitSrc boot;
    int init;
    int begin, nblocks;
};

size_t level_lds_bytes(const LevelGeom& g);
hipError_t launch_pose_prep(const double* pose, int N, const double* prior_pose, int P, PoseF* out, PoseD* outd,
                            hipStream_t st);
hipError_t launch_init(const Win& w, float* idepth, InitSrc boot, hipStream_t st);
hipError_t launch_init_if(const Win& w, float* idepth, InitSrc boot, const int* flag, int32_t* out, hipStream_t st);
hipError_t launch_flow_pairs(const float2* flow, float4* f2, int N, int H, int W, hipStream_t st);
hipError_t launch_level(const Win& w, const LevelGeom& g, const LevelBufs& b, int do_e, int do_m, hipStream_t st);
hipError_t launch_phase_a(const Win& w, const LevelGeom& g, const LevelBufs& b, hipStream_t st);
hipError_t launch_phase_a2(const Win& w, const LevelGeom& g, const LevelBufs& b, hipStream_t st);
hipError_t launch_pose_gn(const Win& w, const PoseBufs& b, int s, int G, int nblocks, hipStream_t st);
hipError_t launch_pose_gn_finish(const PoseBufs& b, int N, int G, int nblocks, hipStream_t st);
hipError_t launch_pose(const Win& w, const PoseBufs& b, int t, const double* cand, int n_cand, int solve,
                       int nblocks, hipStream_t st);
hipError_t launch_finalize(const Win& w, const FinalBufs& b, int n_ll, hipStream_t st);
hipError_t set_level_lds_limit(size_t bytes);

// batched launchers: items / blk2item in device memory, nblocks = total blocks; PR selects the
// prior path (all items of one launch share it and the log-logistic shape class B2)
hipError_t launch_prep_batch(const PrepItem* items, int n_items, hipStream_t st);
hipError_t launch_setup_batch(const PrepItem* items, const int* blk2item, int nblocks, hipStream_t st);
hipError_t launch_level_batch(const LevelItem* items, const int* blk2item, int nblocks, size_t lds, int mode,
                              bool b2, bool pr, hipStream_t st);
hipError_t launch_pose_gn_batch(const PoseItem* items, const int* blk2item, int nblocks, int s, bool b2,
                                hipStream_t st);
hipError_t launch_pose_gn_solve_batch(const PoseItem* items, int n_items, int s, hipStream_t st);
hipError_t launch_finalize_batch(const FinalItem* items, const int* blk2item, int nblocks, bool b2, bool pr,
                                 hipStream_t st);
hipError_t launch_finalize_finish_batch(const FinalItem* items, int n_items, hipStream_t st);

hipError_t launch_vc(const VcArgs& a, const VcBufs& b, hipStream_t st);
hipError_t launch_pose_sample(const PoseSampleArgs& a, const PoseSampleBufs& b, hipStream_t st);
hipError_t launch_align_prepare(const AlignArgs& a, const AlignBufs& b, hipStream_t st);
hipError_t launch_align_step(const AlignArgs& a, const AlignBufs& b, int final_pass, int nblocks, hipStream_t st);
size_t sim3_state_doubles(int n_pairs);
hipError_t launch_align_sim3(const AlignArgs& a, const AlignBufs& b, double* scale, double* state, int steps, int nblocks,
                             hipStream_t st);

}  // namespace vd
