/*
 * voldor.h -- C ABI of the MI355X (gfx950) library for the dense hot path of
 * VOLDOR+SLAM (Min & Dunn, arXiv 2104.06800): generalized-EM inference of
 * inverse depth, rigidness and camera poses over a window of N optical flows
 * (sec. III-A, Eqs. 1-6), and robust point-to-plane inverse-depth keyframe
 * alignment (sec. III-B, Eqs. 10 and 12).
 *
 * Conventions (all entry points)
 *   - Every array is caller-owned and lives in device memory of the context's
 *     GPU unless stated otherwise.  The library never frees caller memory and
 *     keeps no pointer after the work it enqueued has completed.  It allocates
 *     only its own scratch (grown on demand, freed by voldor_ctx_destroy).
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     default stream).  Buffers must stay valid until the stream reaches it.
 *   - Return value: VOLDOR_OK or an error code.  Shapes, parameters and null
 *     pointers are checked before anything is enqueued (VOLDOR_EINVAL, message
 *     in voldor_last_error).  A HIP failure returns VOLDOR_EDEVICE.  NaN or Inf
 *     inside the data are not errors: they make the affected terms invalid and
 *     are counted in the statistics.  No C++ exception crosses this boundary.
 *   - Images are row-major [H][W]; pixel (u, v) is at integer coordinates.
 *     A pose 6-vector (w, t) maps reference-camera points to camera t as
 *     X_t = exp([w]x) X_ref + t (Rodrigues rotation vector w), FP64.
 *   - The state is inverse depth rho = 1/theta (the paper's theta is depth).
 *   - Not thread-safe per context: calls on one context must not overlap
 *     across host threads; calls on different contexts may.
 */
#ifndef VOLDOR_H
#define VOLDOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VOLDOR_OK = 0,
    VOLDOR_EINVAL = 1,     /* bad shape / parameter / null pointer; nothing enqueued  */
    VOLDOR_ENOMEM = 2,     /* scratch allocation failed                               */
    VOLDOR_EDEVICE = 3,    /* HIP runtime error; see voldor_last_error                */
    VOLDOR_ESINGULAR = 4   /* per-pair status of voldor_align_p2p: 6x6 system not PD  */
};

enum { VOLDOR_LEVEL_COARSE = 0, VOLDOR_LEVEL_LOCAL = 1 };
enum { VOLDOR_ROBUST_HUBER = 0, VOLDOR_ROBUST_CAUCHY = 1 };

#define VOLDOR_MAX_FRAMES 8     /* N <= 8 flows per window              */
#define VOLDOR_MAX_PRIORS 4     /* P <= 4 depth priors per window       */
#define VOLDOR_SCORE_LEN 29     /* energy, H upper (21), g (6), count   */
#define VOLDOR_STATS_LEN 8

typedef struct voldor_ctx_s* voldor_ctx;

/* Window geometry and model constants (host struct, passed by pointer). */
typedef struct {
    int32_t H, W;              /* image size, both >= 2                                   */
    int32_t N;                 /* flows in the window, 1..8                               */
    int32_t P;                 /* depth priors, 0..4                                      */
    float fx, fy, cx, cy;      /* pinhole intrinsics                                      */
    float fisk_alpha;          /* log-logistic scale of the flow end-point error (px)     */
    float fisk_beta;           /* log-logistic shape, in [1, 4]; 2 takes a fast path      */
    float outlier_density;     /* planar outlier density L0 (px^-2), e.g. 1/(pi 8^2)      */
    float hmm_gamma;           /* rigidness-chain stay probability, in (0.5, 1]           */
    float idepth_min, idepth_max;  /* candidate inverse-depth range                       */
    float perturb_sigma0;      /* relative width of perturbation candidates at it 0,1     */
    float prior_sigma_rel;     /* Eq. 3: sigma(rho^) = prior_sigma_rel * rho^ (model 1:   */
                               /*   scale of the disparity residual law, px)              */
    float prior_uniform_rel;   /* Eq. 3: U(rho^) = 1 / (prior_uniform_rel * rho^) (model  */
                               /*   1: width of the outlier disparity range, px)          */
    float prior_inlier_default;/* prior weight where prior_weight is NULL                 */
    int32_t n_candidates;      /* K slots per pixel per pass, 3..64                       */
    int32_t coarse_stride;     /* s of the coarse lattice, >= 1                           */
    int32_t tile;              /* T of the local tiles: 8, 16, 32, 64, 128 or 256         */
    int32_t pose_gn_steps;     /* Gauss-Newton steps per frame in the pose step, >= 0     */
    int32_t chain_axis;        /* rigidness chains: 0 spatial (paper), 1 frame window     */
    int32_t prior_model;       /* 0: Eq. 3's Gaussian-uniform mixture on inverse depth;   */
                               /* 1: empirical residual model of external (stereo) priors */
                               /*    (sec. III-A, after Eq. 5): the disparity residual    */
                               /*    r = prior_disp_scale (rho^ - 1/phi_z) has inlier     */
                               /*    density f_Fisk(|r|; prior_sigma_rel,                 */
                               /*    prior_fisk_beta) / 2 and outlier density             */
                               /*    1 / prior_uniform_rel                                */
    uint64_t seed;             /* Philox key                                              */
    uint32_t window_id;        /* Philox counter word 3                                   */
    float prior_disp_scale;    /* model 1: focal length times baseline (disparity / rho)  */
    float prior_fisk_beta;     /* model 1: shape of the disparity residual law, in (0, 1] */
    uint32_t init_random;      /* 0: the initial inverse depth starts from depth prior 0  */
                               /*    wherever its transfer resolves (sec. III-A, priors   */
                               /*    bootstrap the estimate), random elsewhere; 1: random */
                               /*    everywhere.  Without priors the start is random.     */
} voldor_window;

/* Device buffers of one window.  Sizes: Hc x Wc from voldor_lattice_shape. */
typedef struct {
    const float*  flow;          /* [N][H][W][2] flow X_t (frame t-1 -> t) on frame t-1's grid  */
    double*       pose;          /* [N][6] T_t, reference -> camera t (in/out)                  */
    float*        idepth;        /* [H][W] inverse depth of the reference frame (in/out)        */
    float*        rigid;         /* [N][H][W] rigidness posteriors q_t (out of the E-step)      */
    float*        idepth_coarse; /* [Hc][Wc] coarse-lattice inverse depth (work buffer)         */
    float*        rigid_coarse;  /* [N][Hc][Wc] coarse-lattice rigidness (work buffer)          */
    const float*  prior_idepth;  /* [P][H][W] prior inverse depth, NaN = hole; NULL if P = 0    */
    const double* prior_pose;    /* [P][6] fixed pose T^_k of prior k (reference -> camera k)  */
    const float*  prior_weight;  /* [P][H][W] prior inlier weight pi^ in [0,1], or NULL         */
    float*        conf;          /* [H][W] confidence C (Eq. 6), written by voldor_finalize     */
    double*       stats;         /* [8] statistics, written by voldor_finalize                  */
} voldor_buffers;

/* Context bound to one device ordinal.  Owns scratch memory only. */
int  voldor_ctx_create(voldor_ctx* out, int device_ordinal);
void voldor_ctx_destroy(voldor_ctx ctx);
/* Message of the last non-zero status on this context (or of ctx creation when ctx is NULL). */
const char* voldor_last_error(voldor_ctx ctx);
/* Size of the coarse lattice {(s U + floor(s/2), s V + floor(s/2))} inside H x W (host). */
int voldor_lattice_shape(int32_t H, int32_t W, int32_t stride, int32_t* Hc, int32_t* Wc);

/* Random initial inverse depth, rho_min + u (rho_max - rho_min) with u from Philox
 * (counter: pixel index, 0, purpose INIT at iteration 0 / local level, window id).
 * Writes idepth. */
int voldor_init_idepth(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                       void* stream);

/* E-step of one level (sec. III-A "Hierarchical Propagation Scheme": HMM smoothing of the
 * rigidness maps by forward-backward on the alternately directed 1D chains), direction
 * iter mod 4.  Emissions use the current idepth and poses.  Level COARSE writes
 * rigid_coarse (chains = whole lattice rows/columns); level LOCAL writes rigid (chains =
 * rows/columns of tile x tile blocks).  With chain_axis = 1 each pixel's chain runs over
 * the frame window instead. */
int voldor_rigidness_fb(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                        int iter, int level, void* stream);

/* M-step of one level (sec. III-A, Eqs. 3-5): per pixel argmin of the maximum-inlier energy
 * over K candidate slots -- 0 current value, 1 predecessor's updated value along the chain,
 * 2 coarse result of the pixel's lattice cell (LOCAL only), 3..K-1 Philox draws -- ties to
 * the lowest slot, chains swept in direction iter mod 4.  Uses the level's rigidness from
 * its last E-step and the prior posteriors at the current value.  COARSE writes
 * idepth_coarse; LOCAL writes idepth. */
int voldor_depth_update(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                        int iter, int level, void* stream);

/* Scores candidate poses of frame t (1..N) (sec. III-A "Uncertainty-aware Pose Estimation":
 * the quantity its pose samples are scored by).  For each candidate: energy
 * sum_j q_t^j log1p(L0/L1(r)) (invalid terms cost q log 2), the Gauss-Newton normal
 * equations H = sum w J^T J (upper triangle, row-major, 21 values) and g = sum w J^T e of
 * the residual e = p_t - o_t with IRLS weight w = q d cost / d r^2 and J the derivative
 * w.r.t. a left update (dw, dv), and the count of valid terms.  o_t uses the current pose
 * of frame t-1.  A term is valid where the point is in front of cameras t-1 and t, the
 * flow sample at p_{t-1} exists and p_t lies inside frame t's image.
 * cand_pose: [n_cand][6] device FP64; out: [n_cand][29] device FP64. */
int voldor_pose_score(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                      int t, int n_cand, const double* cand_pose, double* out, void* stream);

/* Pose step: frames t = 1..N in order, pose_gn_steps FP64 Cholesky solves of
 * (H + 1e-9 tr(H)/6 I) delta = -g each, T_t <- (exp([dw]x) R, exp([dw]x) t + dv).
 * A numerically singular system leaves that frame's pose unchanged. */
int voldor_pose_step(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                     void* stream);

/* The paper's pose M-step (sec. III-A "Uncertainty-aware Pose Estimation", its sampling
 * equation), an alternative to voldor_pose_step: for frames t = 1..N in order (each frame's
 * observations use the already updated pose of frame t-1), S pose samples, each the P3P
 * solution (of those nearest the frame's current pose in the kernel metric) of three pixels
 * drawn with probability proportional to q_t -- a Philox draw picks a pixel, a second
 * accepts it when below q_t and the pixel has a depth and an observation
 * o_t = p_{t-1} + X_t(p_{t-1}), up to `tries` attempts per point; counter (sample,
 * point * tries + attempt, (iter << 8) | (t << 4) | 2, window id); the frame's pose becomes
 * the mode of the samples found by meanshift with the Gaussian kernel
 * diag(sigma_w^2 I, (sigma_t_rel |t|)^2 I) in the left-update chart of the pose step,
 * started at the current pose.  Its uncertainty Sigma_t (cov_out [N][36], FP64 device, or
 * NULL) is fitted to the samples from the mode by iterated 3-sigma inlier fits, each inlier
 * covariance divided by P(chi2_8 <= 9) / P(chi2_6 <= 9) so that a Gaussian's own covariance
 * is the fixed point, eigenvalues floored at eps.  info_out [N][4] (or NULL): valid
 * samples, inliers, meanshift steps, fit rounds.  A frame without valid samples keeps its
 * pose.  FP64 throughout. */
#define VOLDOR_POSE_MAX_SAMPLES 4096
typedef struct {
    int32_t samples;           /* S, 1..4096                                           */
    int32_t tries;             /* draw attempts per point, 1..64                       */
    double sigma_w;            /* kernel std of the rotation coordinates (rad)         */
    double sigma_t_rel;        /* kernel std of the translation coordinates / |t|      */
    double eps;                /* eigenvalue floor of Sigma_t                          */
} voldor_sample_params;
int voldor_pose_sample(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf, int iter,
                       const voldor_sample_params* sp, double* cov_out, double* info_out, void* stream);

/* One pass of one level: its E-step immediately followed by its M-step (same chains,
 * direction iter mod 4), fused in a single launch; equivalent to voldor_rigidness_fb then
 * voldor_depth_update on the same level. */
int voldor_level_step(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                      int iter, int level, void* stream);

/* One GEM iteration: coarse E+M, local E+M, pose step (each level fused in one launch). */
int voldor_gem_step(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                    int iter, void* stream);

/* Final local E-step (direction iter mod 4), confidence C^j = (sum_t q_t + sum_k q^_k)/(N+P)
 * (Eq. 6) and statistics: [0] log-likelihood (sum of chain log Z, densities in px^-2),
 * [1] MIE energy sum_j E_j(rho_j) (natural log), [2] valid flow terms, [3] invalid flow
 * terms, [4] prior terms with a valid transfer (not a hole), [5] sum of C, [6..7] 0. */
int voldor_finalize(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                    int iter, void* stream);

/* Flags of voldor_run / voldor_batch_run. */
#define VOLDOR_RUN_INIT 1          /* start from voldor_init_idepth's random inverse depth  */
#define VOLDOR_RUN_NO_GRAPH 2      /* voldor_batch_run: launch directly, no graph capture    */

/* A whole GEM window (sec. III-A, the iteration of Fig. 2's GEM block): optional random
 * initial depth (flags & VOLDOR_RUN_INIT), iterations first_iter .. first_iter + n_iters - 1
 * of voldor_gem_step and voldor_finalize at the last of them.  Same results, bit for bit,
 * as that sequence of calls; the flow layout the kernels read is built once per window
 * rather than once per call.  A start at first_iter > 0 continues from the caller's depth
 * with the later, narrower candidate perturbations (a warm start, e.g. from the learned
 * proposal).  n_iters >= 1, first_iter >= 0. */
int voldor_run(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
               int first_iter, int n_iters, int flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): voldor_run with the same arguments and
 * the same results bit for bit, whose scratch is a static device array of
 * VOLDOR_NOALLOC_SCRATCH_BYTES (64 MiB) per device instead of the context's grown buffer.
 * It calls no allocating routine and records no timer events.  The array is loaded with the
 * library's code object on each device it runs on and held until the process ends; its
 * address is looked up when a context is created on that device.  It holds windows up to
 * 1216x352 with N = 8; a window needing more scratch returns VOLDOR_EINVAL before anything is
 * enqueued.  Every call on one device shares that array and leaves its contents behind
 * (nothing in it needs clearing: each kernel writes what it later reads): calls that overlap
 * on one device, on any streams or contexts, race and must be serialised by the caller. */
#define VOLDOR_NOALLOC_SCRATCH_BYTES (64u << 20)
int voldor_run_noalloc(voldor_ctx ctx, const voldor_window* win, const voldor_buffers* buf,
                       int first_iter, int n_iters, int flags, void* stream);

/* n_windows independent windows (wins[i] with bufs[i]; shapes, N, K, priors may differ),
 * each as voldor_run from iteration 0 with the same n_iters and flags (VOLDOR_RUN_INIT),
 * bit for bit.  Each
 * step of the launch sequence is one launch over all windows per shape class (log-logistic
 * shape 2 or not, priors or not): a block finds its window in an item table.  Each class's
 * launches run on a stream of the context's own (forked from and joined back into
 * `stream`), so the classes overlap; the call's work is still ordered on `stream` as a whole.
 * The whole sequence is captured once into a HIP graph on the first call for a given set of windows,
 * buffers and settings and replayed by later identical calls (VOLDOR_RUN_NO_GRAPH launches
 * directly).  The context keeps every window's scratch (about 60 MB for 1216x352, N = 6) for
 * the graph's lifetime.  1 <= n_windows <= 4096; every window is validated before anything
 * is launched.  The first call for a set waits for the stream once (table upload). */
int voldor_batch_run(voldor_ctx ctx, int n_windows, const voldor_window* wins, const voldor_buffers* bufs,
                     int n_iters, int flags, void* stream);

/* Launch knobs (tuning).  Settings that change how the work is split over the chip and
 * never what is computed: every run gives the same results bit for bit whatever they are.
 * 0 keeps a knob's default.
 *   local_chains  local-level chain segments per block (default: as many as fit the block,
 *                 8 for 32x32 tiles); fewer means more, lighter blocks
 *   local_spec    speculation depth of the local scan, 1..8 (default 2): predecessor
 *                 energies evaluated ahead in the parallel phase
 *   coarse_spec   speculation depth of the coarse scan, 1..8 (default 8)
 *   coarse_lanes  lanes per lattice node of the coarse phase-A grid, 4, 8 or 16 (default 8;
 *                 the batched run keeps 8)
 *   local_order   order in which the local level's blocks are handed to the XCDs: 1 by the
 *                 angle of the block's centre around the principal point, so that each XCD
 *                 works on one angular sector (default; pays off when the camera moves
 *                 forward and the flows' epipolar lines radiate from near the principal
 *                 point), 2 row by row.  The no-allocation entry always takes row order. */
typedef struct {
    int32_t local_chains;
    int32_t local_spec;
    int32_t coarse_spec;
    int32_t coarse_lanes;
    int32_t local_order;
} voldor_knobs;

/* Sets (knobs != NULL) or removes (NULL) the knobs of every window with the same H, W, N,
 * n_candidates and presence of priors as `bucket` (host structs).  Drops a captured batch
 * graph. */
int voldor_set_knobs(voldor_ctx ctx, const voldor_window* bucket, const voldor_knobs* knobs);
/* The knobs that calls on `win` use (zeros: defaults). */
int voldor_get_knobs(voldor_ctx ctx, const voldor_window* win, voldor_knobs* out);

/* Launch timers (measurement).  The library brackets launches of each enabled timer class
 * with HIP events on the launch stream: VOLDOR_TIMER_LOCAL = the fused local-level E+M
 * kernel, VOLDOR_TIMER_COARSE = a coarse-level pass (its E-step and M-step launches),
 * VOLDOR_TIMER_POSE = a pose step (all its Gauss-Newton launches).  Each event record costs
 * the stream a few microseconds, so enable only the classes you read.
 * voldor_timing(ctx, mask) enables the classes whose bit (1 << timer) is set, starts afresh
 * and discards earlier records; mask 0 stops recording; a mask outside 0..7 is
 * VOLDOR_EINVAL.  voldor_timing_read waits for the recorded events of one class, returns
 * the summed duration (ms) and the number of bracketed launches, and clears that class. */
#define VOLDOR_TIMER_LOCAL  0
#define VOLDOR_TIMER_COARSE 1
#define VOLDOR_TIMER_POSE   2
int voldor_timing(voldor_ctx ctx, int mask);
int voldor_timing_read(voldor_ctx ctx, int timer, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------------
 * Learned depth / rigidness proposal.  The paper initialises depth at random (sec. III-A);
 * this project adds a small convolutional encoder-decoder that maps the flow stack of a
 * window to an initial inverse depth and initial rigidness maps, while plain GEM stays the
 * fallback and the reference for its error.  BF16 weights and activations, FP32 accumulation on
 * the matrix cores, FP32 master weights and Adam.
 *
 * Layers (3x3, zero padding 1, NHWC; stored channel counts):
 *   c1 16 -> 64, c2 64 -> 128 stride 2, c3 128 -> 128, c4 128 -> 128, all ReLU;
 *   c5 128 -> 64 on the 2x nearest upsampling of c4's output, + c1's output, ReLU;
 *   c6 64 -> 32 linear.
 * Input channel 2(t-1)+c = X_t[c] / 16 (non-finite -> 0; N <= 8, the rest 0).  Outputs:
 * idepth = clip(softplus(o_0) / tnorm, idepth_min, idepth_max), where tnorm = |t| of frame
 * 1's initial pose (flows fix depth only up to that scale); rigid_t = sigmoid(o_t).
 * H and W must be even (the stride-2 / upsampling pair).
 * ------------------------------------------------------------------------------- */
#define VOLDOR_NET_PARAMS 470560   /* FP32 parameters: per layer c1..c6, w [Cout][3][3][Cin], b [Cout] */

typedef struct {
    float*    params;        /* [VOLDOR_NET_PARAMS] FP32 master parameters                  */
    uint16_t* wbf16;         /* [VOLDOR_NET_PARAMS] BF16 copy of params (the kernels' weights;
                                this and wt_bf16 16-byte aligned, VOLDOR_EINVAL otherwise) */
    uint16_t* wt_bf16;       /* [VOLDOR_NET_PARAMS] BF16 weights transposed to [Cin][3][3][Cout]
                                per layer (training; NULL for inference)                    */
    float*    adam_m;        /* [VOLDOR_NET_PARAMS] Adam moments (training; else NULL)       */
    float*    adam_v;
    float*    grads;         /* [VOLDOR_NET_PARAMS] gradients of the last training step      */
} voldor_net;

/* Rewrites wbf16 (and wt_bf16 when set) from params; call after changing params. */
int voldor_net_refresh(voldor_ctx ctx, const voldor_net* net, void* stream);

/* Inference on one window: flow [N][H][W][2] FP32 -> idepth_out [H][W], rigid_out [N][H][W]
 * (either may be NULL) and, when logits_out is set, the linear output [H][W][32] FP32. */
int voldor_proposal_forward(voldor_ctx ctx, const voldor_net* net, int32_t H, int32_t W, int32_t N,
                            const float* flow, float tnorm, float idepth_min, float idepth_max,
                            float* idepth_out, float* rigid_out, float* logits_out, void* stream);

/* One training step on one window: forward, loss
 *   L = mean over mask of |softplus(o_0) - idepth_target * tnorm|
 *       + lam * mean over pixels and frames of BCE(sigmoid(o_t), rigid_target_t),
 * backward (gradients into net->grads) and an Adam step (lr, beta 0.9 / 0.999, eps 1e-8;
 * step counts from 1).  loss_out (device, FP64 [3]) receives L, its depth part and its BCE
 * part.  Needs every training pointer of net. */
int voldor_proposal_train_step(voldor_ctx ctx, const voldor_net* net, int32_t H, int32_t W, int32_t N,
                               const float* flow, float tnorm, const float* idepth_target,
                               const float* rigid_target, const uint8_t* mask, float lam, float lr,
                               int32_t step, double* loss_out, void* stream);

/* One 3x3 convolution layer (the network's building block): input x [H][W][Cin] BF16 (its 2x
 * nearest upsampling when up = 1), weights w [Cout][3][3][Cin] BF16, bias [Cout] FP32 (or
 * NULL), optional skip [Ho][Wo][Cout] BF16 added before the optional ReLU; output y BF16
 * and/or yf FP32, [Ho][Wo][Cout] with Ho = (H' - 1) / stride + 1 on the (upsampled) input
 * H'.  Cin a multiple of 16, Cout of 32; stride 1 or 2 (not with up).  The BF16 arrays (x,
 * w, skip, y) must be 16-byte aligned, as every hipMalloc allocation is: VOLDOR_EINVAL
 * otherwise, before any launch. */
int voldor_conv3x3_bf16(voldor_ctx ctx, int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t stride,
                        int32_t up, int32_t relu, const uint16_t* x, const uint16_t* w, const float* bias,
                        const uint16_t* skip, uint16_t* y, float* yf, void* stream);

/* Gradients of that layer (without its activation) for an upstream gradient dy
 * [Ho][Wo][Cout] BF16: dx [H][W][Cin], dw [Cout][3][3][Cin], db [Cout], all FP32 (each
 * may be NULL).  w_t is the BF16 weight transposed to [Cin][3][3][Cout].  x, w_t and dy
 * must be 16-byte aligned (VOLDOR_EINVAL otherwise). */
int voldor_conv3x3_bf16_backward(voldor_ctx ctx, int32_t H, int32_t W, int32_t Cin, int32_t Cout,
                                 int32_t stride, int32_t up, const uint16_t* x, const uint16_t* w_t,
                                 const uint16_t* dy, float* dx, float* dw, float* db, void* stream);

/* Learned start of one GEM window: the network on buf->flow writes buf->idepth and buf->rigid,
 * with tnorm = |t| of buf->pose's frame 1 read on the device.  Where its output is unusable
 * (a non-finite depth logit anywhere, or a non-finite or zero tnorm) the whole window takes
 * voldor_init_idepth's random start instead and *fallback_out (device int32, or NULL) is set
 * to 1, else 0.  voldor_run(first_iter 0, k iterations, flags 0) then runs GEM from it; after
 * a fallback, voldor_run(first_iter k, I - k iterations, flags 0) completes plain GEM's
 * I-iteration run bit for bit.  H and W even. */
int voldor_proposal_start(voldor_ctx ctx, const voldor_net* net, const voldor_window* win, const voldor_buffers* buf,
                          int32_t* fallback_out, void* stream);

/* voldor_batch_run with every window started by the proposal network as voldor_proposal_start
 * does (VOLDOR_RUN_INIT is ignored): windows with odd H or W, and windows whose network
 * output is unusable, take the random start (fallback_out[i] = 1, device int32 [n_windows],
 * or NULL).  The starts are part of the captured graph; each window class runs its
 * windows' network passes on its own stream with a forward workspace of its own (held by the
 * context, about 0.6 KB per pixel of the class's largest window). */
int voldor_batch_run_learned(voldor_ctx ctx, const voldor_net* net, int n_windows, const voldor_window* wins,
                             const voldor_buffers* bufs, int n_iters, int flags, int32_t* fallback_out, void* stream);

/* Keyframe-alignment parameters (sec. III-B, Eqs. 10, 12). */
typedef struct {
    int32_t H, W;
    float fx, fy, cx, cy;
    int32_t robust;            /* VOLDOR_ROBUST_HUBER or VOLDOR_ROBUST_CAUCHY          */
    float robust_scale;        /* Huber delta / Cauchy scale, inverse-depth units      */
    int32_t gn_steps;          /* Gauss-Newton steps, >= 0                             */
    float normal_disc_rel;     /* normal invalid if |rho_nb - rho| > this * rho        */
    float scale_s;             /* relative depth scale s (1 for absolute scale)        */
} voldor_align_params;

/* Robust point-to-plane inverse-depth alignment of n_pairs keyframe pairs (Eq. 10):
 * r_j = rho1(l) <n(l), P1(l) - Q_j> / (s Q_j,z), Q_j = T X2_j, l the nearest pixel of Q_j's
 * projection (fixed within a step), normals by central differences of idepth1; weight
 * conf2_j * psi'(r)/r; undamped Gauss-Newton with an FP64 Cholesky solve per step; then
 * cov = H^-1 at the final pose (Eq. 12's covariance).  Inputs [n][H][W] FP32 (NaN or <= 0
 * = missing); pose_inout [n][6] FP64 (T: camera 2 -> camera 1); cov_out [n][36];
 * stats_out [n][4] = initial cost, final cost, final valid count, steps taken;
 * status_out [n] int32: VOLDOR_OK or VOLDOR_ESINGULAR (the failing step is not applied and
 * cov is NaN).  All device memory. */
int voldor_align_p2p(voldor_ctx ctx, const voldor_align_params* ap, int n_pairs,
                     const float* idepth1, const float* idepth2, const float* conf2,
                     double* pose_inout, double* cov_out, double* stats_out, int32_t* status_out,
                     void* stream);

/* ---------------------------------------------------------------------------------
 * Visibility-coverage scores (sec. III-A "VO Stride and Keyframe Selection", its VC
 * equation): frame 1 carries an inverse-depth map, frame 2 only a pose.  A depth pixel is
 * a pixel of frame 1 with finite inverse depth > 0 (and conf >= conf_min when conf is
 * given).  visibility = share of depth pixels whose projection (FP64, in front of camera 2)
 * has its nearest pixel inside frame 2's H x W image; coverage = share of frame 2's
 * cell x cell blocks (ragged at the far edges) holding at least one such nearest pixel;
 * VC = 2 / (visibility^-1 + coverage^-1), 0 when either is 0.
 * ------------------------------------------------------------------------------- */
#define VOLDOR_VC_MAX_POSES 1024
#define VOLDOR_VC_OUT_LEN 5    /* visibility, coverage, VC, visible depth pixels, covered cells */

typedef struct {
    int32_t H, W;              /* image size of both frames                            */
    float fx, fy, cx, cy;      /* pinhole intrinsics of both frames                    */
    int32_t cell;              /* coverage cell size in pixels, 1..1024                */
    float conf_min;            /* depth-pixel confidence threshold (when conf is set)  */
} voldor_vc_params;

/* Scores of frame 1 (idepth [H][W] FP32, conf [H][W] FP32 or NULL) against n_poses poses of
 * frame 2 (poses [n][6] FP64, mapping frame-1 points to frame 2), 1 <= n_poses <= 1024:
 * out [n][5] FP64 as VOLDOR_VC_OUT_LEN lists; first_below (one int32, or NULL) receives the
 * index of the first pose whose VC is below tau, or n_poses when none is.  With the poses
 * of a batch's frames relative to its reference and tau = tau_stride, that index is the next
 * batch's reference; with the pose of the latest keyframe and tau = tau_keyframe, 0 makes
 * the reference a keyframe.  All device memory. */
int voldor_vc_scores(voldor_ctx ctx, const voldor_vc_params* vp, const float* idepth, const float* conf,
                     int n_poses, const double* poses, double tau, double* out, int32_t* first_below,
                     void* stream);

/* 7-DoF keyframe alignment (sec. III-B: "we estimate both their relative motion T and scale
 * factor s", optimised by Levenberg-Marquardt, Eq. 12): as voldor_align_p2p with the
 * relative depth scale unknown too.  Map 1's geometry is scaled by s, so the plane of pixel
 * l passes through s P1(l): r = rho1(l) <n(l), s P1(l) - Q_j> / (s Q_j,z), which is Eq. 9's
 * 1/(s theta1) - 1/phi_z for a fronto-parallel plane.  Unknowns (left pose update,
 * log s); ap->gn_steps evaluations, each of the trial step solving
 * (H + lambda diag(H)) d = -g at the accepted state (lambda from 1e-4): a trial with a lower
 * cost is accepted (lambda / 10), otherwise lambda * 10.  scale_inout [n] FP64 (start and
 * result, > 0); cov_out [n][49] = H^-1 of (w, v, log s) at the accepted state; stats_out
 * [n][4] = initial cost, final cost, final valid count, accepted steps; status_out as for
 * voldor_align_p2p (ESINGULAR: the accepted state is kept, cov is NaN).  ap->scale_s is
 * not used.  All device memory. */
int voldor_align_sim3(voldor_ctx ctx, const voldor_align_params* ap, int n_pairs, const float* idepth1,
                      const float* idepth2, const float* conf2, double* pose_inout, double* scale_inout,
                      double* cov_out, double* stats_out, int32_t* status_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* VOLDOR_H */
