/*
 * dpvo.h - C ABI of the gfx950 sliding-window driver of Deep Patch Visual
 * Odometry (Teed, Lipson, Deng, arXiv 2208.04726), built into libdpba.so.
 *
 * A handle keeps, on the device, the sliding window of many camera streams
 * and steps them together, one new frame per stream per vo_step, by the
 * rules of Sec. 3.3 "VO System":
 *   - window advance: a full window (`window` keyframes) drops its oldest
 *     keyframe with its patches and edges;
 *   - expansion ("Expansion"): the new frame's pose by a constant-velocity
 *     model, T_n = (T_{n-1} T_{n-2}^-1) T_{n-1}; its patches' inverse depth
 *     the median over all patches of the previous 3 keyframes; edges from each
 *     new patch to every keyframe within `radius` of its frame and from each
 *     patch of the last `radius` keyframes to the new frame;
 *   - optimization ("Optimization"): `iterations` bundle-adjustment steps
 *     (include/dpba.h) over every stream's window in one batched solve, the
 *     poses of all but the last `n_free` keyframes fixed;
 *   - keyframing ("Keyframing"): the flow magnitude between keyframes t-5 and
 *     t-3; below `flow_thresh` keyframe t-4 is removed, its pose relative to
 *     its previous neighbour recorded.
 * The targets and weights of the edges, which the paper's update operator
 * revises, come from a sensor table per stream (vo_set_sensor).
 *
 * Conventions (the paper fixes none of these):
 *   - the first two frames of a stream take their poses from the
 *     initialisation input, the first frame's patches a given inverse depth;
 *   - at least two poses stay fixed (the monocular gauge): n_fixed =
 *     max(min(2, n), n - n_free) of the window's n keyframes;
 *   - the flow magnitude is the mean, over the patches of keyframe t-5 whose
 *     homogeneous depth in keyframe t-3 exceeds z_min, of the distance between
 *     a patch centre and its reprojection into keyframe t-3 (infinite when no
 *     patch qualifies), in FP64;
 *   - the median of an even count is the mean of the two middle values.
 *
 * Device layout: stream s owns `window` keyframe slots and window *
 * patches_per_frame patch slots; its keyframes fill the first slots in window
 * order, unused slots hold identity poses and patches without edges, which
 * the solve leaves unchanged.  All patches of a keyframe enter and leave the
 * window together and share one set of target frames, so the patch graph is
 * one 64-bit row of target slots per keyframe slot.  Every step generates the
 * edge list from these rows, packed across the streams in (patch, target
 * frame) order, packs the windows of the streams with a new frame into
 * staging buffers and solves them in one bundle adjustment; idle streams
 * cost nothing in the solve.
 *
 * Errors: BA_OK (0) or BA_E_INVAL (-1) / BA_E_CAPACITY (-2) / BA_E_HIP (-3)
 * / BA_E_STATE (-4) of dpba.h.
 */
#ifndef DPVO_H
#define DPVO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vo_handle vo_handle;

typedef struct {
  int32_t n_streams;          /* S                                                  */
  int32_t window;             /* keyframes per window (paper: 22; at most 24 with
                                 BA_PREC_FP64, 64 with BA_PREC_FP32)                */
  int32_t patches_per_frame;  /* 1 .. 256 (paper: 96)                               */
  int32_t radius;             /* edge radius r, 0 .. 31 (paper: 13): a patch has at
                                 most 2 r + 1 edges, within the solver's 64       */
  int32_t n_free;             /* keyframes optimised (paper: 10)                    */
  int32_t precision;          /* BA_PREC_FP32 or BA_PREC_FP64                       */
  int32_t iterations;         /* Gauss-Newton iterations per step (paper: 2)        */
  int32_t table_radius;       /* R of the sensor tables                             */
  double flow_thresh;         /* keyframe removal threshold, pixels (paper: 64)     */
  double lambda;              /* damping (paper: 1e-4)                              */
  double z_min;               /* active-edge threshold on homogeneous depth         */
  double intrinsics[4];       /* fx, fy, cx, cy of every stream                     */
} vo_config;

/* Creates the handle and allocates every stream's device state and the
 * bundle-adjustment workspace.  BA_E_INVAL for out-of-range fields. */
int vo_create(const vo_config* cfg, vo_handle** out);

/* The sensor of the streams: for patch g = frame * patches_per_frame + i of
 * stream s and frame f, the target (pixels) and weight of edge (g, f) are
 * rows table_off[s] + g, column f - frame + table_radius of targets / weights
 * (dev [rows, 2 R + 1, 2], f64; FP32-exact values when precision is
 * BA_PREC_FP32).  table_off (host [S], first row of each stream) and
 * table_frames (host [S], frames of each stream) are copied; the device
 * arrays must stay valid while the handle steps.  An edge outside its
 * stream's table gets weight 0. */
int vo_set_sensor(vo_handle* h, const double* targets, const double* weights, const int64_t* table_off,
                  const int32_t* table_frames);

/* One new frame for every stream: frame_id (host [S], increasing per stream;
 * < 0 leaves the stream idle this step, its window unchanged), new_xy (dev
 * [S, patches_per_frame, 2], the new frame's patch centres in pixels),
 * init_poses (dev [S, 2, 7], the poses of a stream's first two frames),
 * init_depth (host [S], the inverse depth of a stream's first patches).
 * Enqueues the whole step on `stream` and waits for it (the next step's
 * fixed-pose counts depend on this step's keyframe decisions). */
int vo_step(vo_handle* h, const int32_t* frame_id, const double* new_xy, const double* init_poses,
            const double* init_depth, void* stream);

/* Host copies of the state after the last step: n_kf (host [S], keyframes in
 * the window), kf_id (host [S, window], frame ids in window order, -1 beyond
 * n_kf), flow (host [S], the step's flow magnitude, NaN when not computed or
 * the stream was idle) and removed (host [S], the frame id removed by the
 * step's keyframe decision or -1); any pointer may be NULL. */
int vo_read(vo_handle* h, int32_t* n_kf, int32_t* kf_id, double* flow, int32_t* removed);

/* What the last step took out of each window, for recovering the whole
 * trajectory ("Keyframing", Sec. 3.3): retired (host [S]) the frame id that
 * left the full window at the advance, or -1, with retired_pose (host [S, 7])
 * its final pose; removed (host [S]) the keyframe removed by the flow test,
 * or -1, with removed_prev (host [S]) the keyframe before it and removed_rel
 * (host [S, 7]) its pose relative to that keyframe, T_removed T_prev^-1,
 * taken after the step's optimisation.  Any pointer may be NULL. */
int vo_read_events(vo_handle* h, int32_t* retired, double* retired_pose, int32_t* removed, int32_t* removed_prev,
                   double* removed_rel);

/* Host copies of stream s's window: poses (host [window, 7]), inverse depths
 * (host [window * patches_per_frame], by keyframe slot), its edges as (patch
 * id g, frame id) pairs (host [n_edges] each; pass NULL to query the count)
 * and their count. */
int vo_read_window(vo_handle* h, int32_t s, double* poses, double* depth, int32_t* edge_patch,
                   int32_t* edge_frame, int64_t* n_edges);

/* BA status bits (dpba.h BA_W_*) of each stream's window in the last step
 * (host [S]; 0 for a stream that was idle); bit 16 marks an edge outside the stream's sensor table (its
 * weight is 0), bit 17 an edge count that disagrees with the graph (an
 * internal error: the step used the smaller count). */
int vo_status(vo_handle* h, int32_t* flags);

void vo_destroy(vo_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* DPVO_H */
