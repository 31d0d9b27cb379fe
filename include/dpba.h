/*
 * dpba.h - C ABI of the MI355X (gfx950) bundle-adjustment library for Deep
 * Patch Visual Odometry (Teed, Lipson, Deng, arXiv 2208.04726).
 *
 * One call solves a batch of independent BA windows.  Each window is the
 * paper's sliding-window patch graph (Sec. 3 "Patch Graph"): N frames with
 * poses T in SE(3), M patches each anchored in a source frame with pixel
 * centre (x, y) and inverse depth d (Sec. 3 "Preliminaries", Eq. 1), and E
 * edges (k, j) joining patch k to frame j.  Every edge carries a target pixel
 * (the reprojected centre plus the flow revision, Sec. 3.1 "Factor Head") and
 * a per-coordinate confidence weight.  The library runs a fixed number of
 * damped Gauss-Newton iterations on the weighted reprojection objective
 * (Sec. 3.1 "Differentiable Bundle Adjustment", Eq. 6, with the projection of
 * Eq. 2-3), over the free poses and every patch's inverse depth, pixel
 * coordinates held constant, depths eliminated by the Schur complement
 * (Sec. 3.1), damping 1e-4 (Appendix "Bundle Adjustment Layer"), poses
 * outside the optimisation window held fixed (Sec. 3.3 "Optimization").
 *
 * Conventions (the paper fixes none of these):
 *   - pose 7-vector (tx, ty, tz, qx, qy, qz, qw): world->camera, unit Hamilton
 *     quaternion, scalar last.  T_j T_i^{-1} maps camera i to camera j (Eq. 2).
 *   - tangent (rho, phi), translation first; retraction T <- Exp(xi) T.
 *   - weights are diagonal information: the cost of an edge is
 *     w_x r_x^2 + w_y r_y^2 with r = projection - target.
 *   - an edge is active iff j != source frame of k and the homogeneous depth
 *     of the reprojected point exceeds z_min; inactive edges contribute nothing.
 *   - lambda is added to the diagonal of every free unknown.
 *   - poses [0, n_fixed) of a window are fixed; all inverse depths are free.
 *
 * Memory: the caller owns every input and output buffer.  "dev" pointers are
 * device (HBM) pointers on the current HIP device; "host" pointers are read
 * during the call only.  The handle owns only its workspace, allocated by
 * ba_create; ba_solve and ba_backward allocate nothing.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  Calls enqueue work and return without waiting for the device;
 * outputs are valid once the stream has reached that point.  One handle
 * serves one host thread and one stream at a time: calls on a handle run in
 * issue order on the stream they are given, and a caller that switches
 * streams must order them itself.
 *
 * Errors: functions return BA_OK or a negative BA_E_* code and never throw.
 * Host-side argument errors are reported before anything is enqueued.
 * Per-window numerical conditions are reported through ba_status; a window
 * that fails leaves poses_out / depth_out equal to its inputs.
 */
#ifndef DPBA_H
#define DPBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_handle ba_handle;

enum {
  BA_OK = 0,
  BA_E_INVAL = -1,     /* bad argument (null pointer, bad offsets, bad count) */
  BA_E_CAPACITY = -2,  /* batch exceeds the capacities given to ba_create      */
  BA_E_HIP = -3,       /* a HIP runtime call failed; see ba_last_error          */
  BA_E_STATE = -4      /* call not allowed in the handle's current state       */
};

enum {
  BA_PREC_FP64 = 0,    /* linearisation, assembly, Schur in FP64                */
  BA_PREC_FP32 = 1     /* linearisation, assembly, Schur in FP32 with FP32
                          accumulation; reduced-pose Cholesky, depth
                          back-substitution and retraction in FP64             */
};

enum {
  BA_SCHED_AUTO = 0,   /* the split schedule (on MI355X it measured faster than
                          the fused one at every batch size, 1 to 256 windows
                          of 22 frames x 96 patches)                            */
  BA_SCHED_SPLIT = 1,  /* one launch per stage, many workgroups per window      */
  BA_SCHED_FUSED = 2   /* one persistent launch, one workgroup per window runs
                          every stage of every iteration                        */
};

/* per-window status bits (ba_status) */
enum {
  BA_W_OK = 0,
  BA_W_NOT_SPD = 1,     /* reduced pose system not positive definite            */
  BA_W_NONFINITE = 2,   /* a non-finite input or intermediate value             */
  BA_W_BAD_INDEX = 4,   /* anchor / kk / jj outside the window                  */
  BA_W_DEGREE = 8       /* a patch has more than 64 edges                       */
};

typedef struct {
  int32_t precision;              /* BA_PREC_*                                   */
  int32_t iterations;             /* Gauss-Newton iterations per solve (paper: 2) */
  double lambda;                  /* damping (paper: 1e-4)                        */
  double z_min;                   /* active-edge threshold on homogeneous depth   */
  int32_t schedule;               /* BA_SCHED_*                                   */
  int32_t max_windows;            /* windows per call                             */
  int32_t max_frames_per_window;  /* 1..64 (1..24 for BA_PREC_FP64)               */
  int32_t chunk_frames;           /* split schedule: source frames per assembly
                                     workgroup.  0 = chosen per call from the
                                     batch size (about one workgroup per CU, at
                                     least two source frames each);
                                     > 0 = fixed, so that each window's result
                                     is bitwise independent of the other windows
                                     of the batch (the fused schedule always is) */
  int64_t max_frames;             /* total frames per call                        */
  int64_t max_patches;            /* total patches per call                       */
  int64_t max_edges;              /* total edges per call                         */
} ba_config;

typedef struct {
  int32_t n_windows;
  int32_t reserved;
  /* host [W+1] prefix offsets of each window's frames, patches and edges in
     the concatenated device arrays below; offsets[0] = 0                    */
  const int64_t* frame_off;
  const int64_t* patch_off;
  const int64_t* edge_off;
  const int32_t* n_fixed;      /* host [W]   poses [0, n_fixed) fixed              */
  const double* intrinsics;    /* host [W,4] fx, fy, cx, cy                        */
  const double* poses_in;      /* dev [F,7]  initial poses, f64                    */
  const double* patches_in;    /* dev [P,3]  x, y (source-frame pixel), inverse depth, f64 */
  const int32_t* anchor;       /* dev [P]    window-local source frame of each patch */
  const int32_t* kk;           /* dev [E]    window-local patch of each edge       */
  const int32_t* jj;           /* dev [E]    window-local target frame of each edge */
  const void* targets;         /* dev [E,2]  f32 (BA_PREC_FP32) or f64, pixels     */
  const void* weights;         /* dev [E,2]  same dtype as targets                 */
  double* poses_out;           /* dev [F,7]  solved poses (may alias poses_in)     */
  double* depth_out;           /* dev [P]    solved inverse depths                 */
} ba_problem;

/* Creates a handle and allocates its device workspace for the capacities in
 * *cfg.  Returns BA_E_INVAL for out-of-range fields, BA_E_HIP if allocation
 * fails.  *out is NULL on failure. */
int ba_create(const ba_config* cfg, ba_handle** out);

/* Solves every window of *p: `iterations` damped Gauss-Newton steps of the
 * Eq. 6 objective from the state (poses_in, patches_in[:,2]), writing the
 * result to poses_out / depth_out.  Edges may come in any order; duplicate
 * (k, j) edges are independent residuals; self-edges (j = anchor[k]) are
 * accepted and contribute nothing.  Host-side checks return BA_E_INVAL /
 * BA_E_CAPACITY before anything is enqueued. */
int ba_solve(ba_handle* h, const ba_problem* p, void* stream);

/* Vector-Jacobian product of the ba_solve map with respect to targets and
 * weights (the paper back-propagates through the Gauss-Newton iterations,
 * Sec. 3.1; the initial state is a constant, Sec. 3.2).  `p` must describe
 * the same inputs as the forward call; the iterates are recomputed, nothing is
 * kept between calls.  grad_poses: dev [F,7] f64 cotangent of poses_out;
 * grad_depth: dev [P] f64 cotangent of depth_out; grad_targets / grad_weights:
 * dev [E,2] outputs in the dtype of targets.  Entries of inactive edges and of
 * failed windows are zero. */
int ba_backward(ba_handle* h, const ba_problem* p, const double* grad_poses,
                const double* grad_depth, void* grad_targets, void* grad_weights,
                void* stream);

/* Two-phase form of ba_solve for callers that replay the device work as a
 * graph: batched serving of many odometry streams, each of which runs two
 * BA iterations after every update of its window (Sec. 3.3 "Optimization").
 *
 * ba_prepare runs the host-side checks and window / chunk bookkeeping of
 * ba_solve for *p and enqueues the upload of the resulting descriptor table
 * (and the window and chunk counts) on `stream`.  It keeps a copy of *p.
 *
 * ba_launch enqueues the solve of the last prepared problem on `stream`.  It
 * issues kernel launches only, sized for the handle's capacities rather than
 * for the prepared batch (workgroups beyond the batch exit at once), so the
 * launches may be captured into a HIP graph.  A captured graph holds the
 * device pointers of the problem prepared before the capture: before every
 * replay, call ba_prepare with a problem over the same device buffers (sizes
 * and contents may change within the capacities) on the replay stream.
 * The schedule is fixed per handle (BA_SCHED_AUTO is the split schedule).
 * Returns BA_E_STATE if nothing was prepared. */
int ba_prepare(ba_handle* h, const ba_problem* p, void* stream);
int ba_launch(ba_handle* h, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ba_solve
 * without a handle.  Same problem, same kernels and the same results as
 * ba_solve with a handle created from *cfg (bitwise, when the chunking below
 * is the same).  The capacity fields of *cfg (max_*) are ignored: the
 * workspace is sized for this batch and carved from a static device array of
 * 64 MiB that each GPU the library runs on holds until the process ends
 * (about 16 windows of 22 frames x 96 patches, or one of 64 frames x 256
 * patches).  A batch beyond it, more than 256 windows, more than 64 frames in
 * a window (24 in BA_PREC_FP64) or more than 4096 chunks returns
 * BA_E_CAPACITY before anything is enqueued; with chunk_frames = 0 the
 * chunking is that of ba_solve, coarsened until the chunk partials fit.
 * Nothing is allocated: no hipMalloc, hipFree, or host allocation.  Argument
 * errors return BA_E_INVAL as for ba_solve; there is no handle, so no
 * message is kept.
 * status_out: dev [W] int32, may be NULL: the per-window BA_W_* bits, written
 * on `stream` after the solve.
 * Every call on a GPU uses that GPU's one workspace, which keeps the last
 * call's contents: calls whose device work overlaps on one GPU (different
 * streams, or host threads) race and give undefined results; calls in
 * sequence on one stream are safe.  The host part of concurrent calls is
 * serialised per device. */
int ba_solve_noalloc(const ba_config* cfg, const ba_problem* p, int32_t* status_out, void* stream);

/* Kernel stages, for ba_kernel_times. */
enum {
  BA_STAGE_PREP = 0,      /* graph validation and ordering                       */
  BA_STAGE_ASSEMBLE = 1,  /* edge linearisation, block assembly, Schur complement */
  BA_STAGE_CHOL = 2,      /* reduced pose Cholesky, pose solve and retraction     */
  BA_STAGE_BACKSUB = 3,   /* depth back-substitution                              */
  BA_STAGE_FINALIZE = 4,  /* output poses                                         */
  BA_STAGE_FUSED = 5,     /* the persistent launch of the fused schedule          */
  BA_STAGE_COUNT = 6
};

#define BA_TIMING_ALL ((1 << BA_STAGE_COUNT) - 1)

/* Measurement aid: `enable` is a mask of stages (bit s for BA_STAGE s,
 * BA_TIMING_ALL for all, 0 to stop).  Every kernel of a timed stage that
 * ba_solve or ba_launch enqueues (not while the stream is being captured) is
 * bracketed by a pair of HIP events on its stream.  ba_kernel_times waits for the
 * bracketed launches, writes per stage the summed kernel time in ms
 * (ms_out[BA_STAGE_COUNT]) and the number of launches
 * (launches_out[BA_STAGE_COUNT]) since the previous ba_kernel_times, and
 * recycles the events.  Timing creates events on first use and keeps one pair
 * per launch until ba_kernel_times is called. */
int ba_set_timing(ba_handle* h, int32_t enable);
int ba_kernel_times(ba_handle* h, double* ms_out, int32_t* launches_out);

/* Waits for the last stream used with the handle and copies the per-window
 * BA_W_* bits of the last ba_solve / ba_prepare / ba_backward into
 * host_flags[W]. */
int ba_status(ba_handle* h, int32_t* host_flags);

/* Message of the last error on this handle ("" if none).  Valid until the
 * next call on the handle. */
const char* ba_last_error(const ba_handle* h);

/* Waits for outstanding work and frees the handle and its workspace. */
void ba_destroy(ba_handle* h);

/* Inspection entry point for tests: the depth-eliminated pose system of
 * window `window` at the input state, S (n x n, full symmetric, row-major)
 * and s (n), n = 6 (frames - n_fixed), written to dev f64 buffers.  It runs
 * the same linearisation and Schur kernel variant that ba_solve selects for
 * the batch. */
int ba_debug_reduced_system(ba_handle* h, const ba_problem* p, int32_t window,
                            double* S_out, double* s_out, void* stream);

/* Inspection entry point for tests: runs one 16x16x4 matrix-core product
 * (f32 when precision is BA_PREC_FP32, else f64) of A (16x4, row-major, dev)
 * and B (4x16, row-major, dev) into D (16x16, row-major, dev), through the
 * same operand and accumulator lane mapping the Schur kernel uses. */
int ba_debug_mfma(int32_t precision, const void* A, const void* B, void* D, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DPBA_H */
