// Kernels and C ABI of the gfx950 bundle-adjustment library (include/dpba.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/dpba.h"
#include "dpba_common.h"
#include "dpba_prep.h"
#include "dpba_assemble.h"
#include "dpba_solve.h"
#include "dpba_chol_big.h"
#include "dpba_adjoint.h"

using namespace dpba;

// ---------------------------------------------------------------------------
// kernels
// The edge pass of the preparation, EPB edges per workgroup.
__global__ void __launch_bounds__(WG) k_prep_edges(Params P) {
  __shared__ int lds[1];
  if ((int)blockIdx.x >= P.counts[2]) return;
  wg_prep_edges(P, blockIdx.x, lds);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_prep(Params P, int edges_done) {
  __shared__ int lds[PREP_LDS_INTS];
  if ((int)blockIdx.x >= P.counts[0]) return;
  wg_prep<T>(P, blockIdx.x, lds, edges_done != 0);
}

template <typename T, int MAXT>
__global__ void __launch_bounds__(WG) k_assemble(Params P, int iter, int Rcap) {
  extern __shared__ __align__(16) char smem[];
  if ((int)blockIdx.x >= P.counts[1]) return;
  wg_assemble<T, MAXT>(P, blockIdx.x, iter, smem, Rcap);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_chol(Params P, int iter) {
  extern __shared__ __align__(16) char smem[];
  const int w = blockIdx.x;
  if (w >= P.counts[0]) return;
  const WinDesc& W = P.win[w];
  if (6 * (W.n_frames - W.n_fixed) > NCHOL_MAX) return;   // k_chol_big
  wg_chol<T>(P, w, iter, smem);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_chol_big(Params P, int iter) {
  extern __shared__ __align__(16) char smem[];
  const int w = blockIdx.x;
  if (w >= P.counts[0]) return;
  const WinDesc& W = P.win[w];
  if (6 * (W.n_frames - W.n_fixed) <= NCHOL_MAX) return;  // k_chol
  wg_chol_big<T>(P, w, iter, smem);
}

// Panel j of the factorisation of the windows with n > 126:
// blockIdx.x = window * (1 + groups) + b, b = 0 the panel workgroup, b >= 1
// the trailing-update workgroups.
__global__ void __launch_bounds__(WG) k_chol_panel(Params P, int j, int groups) {
  extern __shared__ __align__(16) char smem[];
  const int w = blockIdx.x / (1 + groups);
  if (w >= P.counts[0]) return;
  wg_chol_panel(P, w, j, blockIdx.x % (1 + groups), smem);
}

// Reduced systems of the windows with n > 126: blockIdx.x = window * tiles + tile.
__global__ void __launch_bounds__(WG) k_gather_big(Params P, int tiles) {
  const int w = blockIdx.x / tiles;
  if (w >= P.counts[0]) return;
  wg_gather_big(P, w, blockIdx.x % tiles);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_backsub(Params P, int iter, int Rcap, int nparts) {
  extern __shared__ __align__(16) char smem[];
  const int c = blockIdx.x / nparts;
  if (c >= P.counts[1]) return;
  wg_backsub<T>(P, c, blockIdx.x % nparts, nparts, iter, smem, Rcap);
}

__global__ void __launch_bounds__(WG) k_finalize(Params P) {
  if ((int)blockIdx.x >= P.counts[0]) return;
  wg_finalize(P, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_adj_init(Params P) {
  if ((int)blockIdx.x >= P.counts[0]) return;
  wg_adj_init<T>(P, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_chol_adj(Params P, int iter) {
  extern __shared__ __align__(16) char smem[];
  const int w = blockIdx.x;
  if (w >= P.counts[0]) return;
  if (6 * (P.win[w].n_frames - P.win[w].n_fixed) > NCHOL_MAX) return;   // k_chol_adj_big
  wg_chol_adj<T>(P, w, iter, smem);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_chol_adj_big(Params P, int iter) {
  extern __shared__ __align__(16) char smem[];
  if ((int)blockIdx.x >= P.counts[0]) return;
  wg_chol_adj_big<T>(P, blockIdx.x, iter, smem);
}

template <typename T>
__global__ void __launch_bounds__(WG) k_edge_adj(Params P, int iter, int Rcap) {
  extern __shared__ __align__(16) char smem[];
  if ((int)blockIdx.x >= P.counts[1]) return;
  wg_edge_adj<T>(P, blockIdx.x, iter, smem, Rcap);
}

__global__ void __launch_bounds__(WG) k_frame_adj(Params P) {
  if ((int)blockIdx.x >= P.counts[0]) return;
  wg_frame_adj(P, blockIdx.x);
}

// Persistent form: each workgroup takes whole windows (one chunk each) and
// runs preparation and every stage of every iteration without leaving the
// kernel.
template <typename T, int MAXT>
__global__ void __launch_bounds__(WG) k_fused(Params P, int Rcap) {
  extern __shared__ __align__(16) char smem[];
  const int nw = P.counts[0];
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
    wg_prep<T>(P, w, (int*)smem);
    __syncthreads();
    const int c = P.win[w].chunk_off;
    for (int it = 0; it < P.iterations; ++it) {
      wg_assemble<T, MAXT>(P, c, it, smem, Rcap);
      __syncthreads();
      wg_chol<T>(P, w, it, smem);
      __syncthreads();
      wg_backsub<T>(P, c, 0, 1, it, smem, Rcap);
      __syncthreads();
    }
    wg_finalize(P, w);
    __syncthreads();
  }
}

// Dense S, s of one window from the chunk partials (inspection).
template <typename T>
__global__ void __launch_bounds__(WG) k_debug_gather(Params P, int w, double* S, double* s) {
  extern __shared__ __align__(16) char smem[];
  const WinDesc W = P.win[w];
  const int n = 6 * (W.n_frames - W.n_fixed);
  const int lda = n + 1;
  double* A = (double*)(smem + 64);
  double* b = A + n * lda;
  if (n == 0) return;
  gather_partials(P, w, W, A, lda, b, n);
  for (int i = threadIdx.x; i < n * n; i += WG) {
    const int r = i / n, c = i % n;
    S[i] = (c <= r ? A[r * lda + c] : A[c * lda + r]) + (r == c ? P.lambda : 0.0);
  }
  for (int i = threadIdx.x; i < n; i += WG) s[i] = b[i];
}

// Dense S, s of a window with n > 126 from its gathered augmented system.
__global__ void __launch_bounds__(WG) k_debug_copy_big(Params P, int w, double* S, double* s) {
  const WinDesc W = P.win[w];
  const int n = 6 * (W.n_frames - W.n_fixed);
  const int ld = P.ld_big;
  const double* A = P.s_big + (int64_t)w * ld * ld;
  for (int i = threadIdx.x; i < n * n; i += WG) {
    const int r = i / n, c = i % n;
    S[i] = c <= r ? A[(int64_t)r * ld + c] : A[(int64_t)c * ld + r];
  }
  for (int i = threadIdx.x; i < n; i += WG) s[i] = -A[(int64_t)n * ld + i];
}

template <typename T>
__global__ void k_debug_mfma(const T* A, const T* B, T* D) {
  typedef typename AccT<T>::type Acc;
  const int l = threadIdx.x;
  Acc acc = Acc{T(0), T(0), T(0), T(0)};
  acc = mfma16(A[(l & 15) * 4 + (l >> 4)], B[(l >> 4) * 16 + (l & 15)], acc);
  for (int r = 0; r < 4; ++r) D[acc_row(T(0), l >> 4, r) * 16 + (l & 15)] = acc[r];
}

// Allocation-free path: descriptor words carried in the kernel arguments
// (copied by the runtime at launch, so no host buffer has to outlive the
// call) and stored into the static workspace.
constexpr int UPLOAD_WORDS = 992;
struct UploadBlock {
  int64_t dst;   // byte offset from the workspace base
  int32_t n;     // words
  int32_t pad;
  uint32_t w[UPLOAD_WORDS];
};
static_assert(sizeof(UploadBlock) + sizeof(char*) <= 4096, "kernel arguments must stay within 4 KB");
static_assert(sizeof(WinDesc) % 4 == 0 && sizeof(ChunkDesc) % 4 == 0, "descriptors are uploaded as 32-bit words");

__global__ void __launch_bounds__(256) k_upload(char* base, UploadBlock b) {
  uint32_t* d = (uint32_t*)(base + b.dst);
  for (int i = threadIdx.x; i < b.n; i += 256) d[i] = b.w[i];
}

__global__ void __launch_bounds__(256) k_copy_status(const int32_t* status, int32_t* out, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) out[i] = status[i];
}

// ---------------------------------------------------------------------------
// handle
struct ba_handle {
  ba_config cfg;
  int device = 0;
  int n_cu = 256;
  int64_t cap_chunks = 0;
  int64_t cap_partial = 0;   // elements
  int64_t cap_eblocks = 0;   // edge blocks of the split preparation
  WinDesc* d_win = nullptr;
  ChunkDesc* d_chunk = nullptr;
  WinDesc* h_win = nullptr;
  ChunkDesc* h_chunk = nullptr;
  hipEvent_t staging_ev = nullptr;
  bool staging_pending = false;
  hipStream_t last_stream = nullptr;
  int last_W = 0;
  int32_t* eflags = nullptr;
  int32_t *status = nullptr, *wmeta = nullptr, *cnt = nullptr, *ptr = nullptr, *fill = nullptr, *jrun = nullptr;
  int32_t *acnt = nullptr, *afill = nullptr, *plist = nullptr, *csr = nullptr, *arange = nullptr,
          *cstate = nullptr, *estart = nullptr, *sbstart = nullptr, *gj = nullptr;
  int4* sbd = nullptr;
  void *pxy = nullptr, *gt = nullptr, *gw = nullptr;
  int64_t cap_sb = 0;
  int32_t* gidx = nullptr;
  int32_t* d_counts = nullptr;
  int32_t* h_counts = nullptr;
  bool prepared = false;
  bool launch_fused = false;  // schedule of ba_prepare / ba_launch, fixed per handle
  ba_problem prep_problem;
  double *xib = nullptr, *xid = nullptr, *qxi = nullptr, *dbar = nullptr, *fcot = nullptr;
  double* partial = nullptr;
  double* s_big = nullptr;   // augmented reduced systems, windows with n > 126
  double* big_aux = nullptr; // their factorisation side data
  int ld_big = 0;
  double *dxi = nullptr, *pose_buf = nullptr, *depth_buf = nullptr;
  // per-kernel timing (ba_set_timing): event pairs around each launch
  struct TimedLaunch { int stage; hipEvent_t a, b; };
  int timing = 0;   // mask of timed stages
  std::vector<hipEvent_t> ev_pool;
  std::vector<TimedLaunch> timed;
  char err[256] = {0};
};

namespace {

// Records the message of an error on the handle (formatted into its fixed
// buffer: no host allocation on any path) and returns `code`.
int fail(ba_handle* h, int code, const char* fmt, ...) {
  if (h) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(h->err, sizeof(h->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define HIPCHK(h, call)                                                              \
  do {                                                                                \
    hipError_t _e = (call);                                                           \
    if (_e != hipSuccess)                                                             \
      return fail(h, BA_E_HIP, "%s: %s", #call, hipGetErrorString(_e));                 \
  } while (0)

template <typename T>
int set_kernel_attrs() {
  const int lds = 160 * 1024;
  if (hipFuncSetAttribute((const void*)k_assemble<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_assemble<T, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_assemble<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if constexpr (sizeof(T) == 4)
    if (hipFuncSetAttribute((const void*)k_assemble<T, 12>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_fused<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_fused<T, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_fused<T, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chol<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chol_big<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chol_panel, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_backsub<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_debug_gather<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chol_adj<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chol_adj_big<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_edge_adj<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
  return 0;
}

hipEvent_t take_event(ba_handle* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events on its stream when timing is on and
// the stream is not being captured into a graph.
struct KernelTimer {
  ba_handle* h;
  hipStream_t s;
  int stage;
  hipEvent_t a = nullptr;
  KernelTimer(ba_handle* h_, hipStream_t s_, int stage_) : h(h_), s(s_), stage(stage_) {
    if (!(h->timing & (1 << stage))) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    a = take_event(h);
    if (a && hipEventRecord(a, s) != hipSuccess) {
      h->ev_pool.push_back(a);
      a = nullptr;
    }
  }
  ~KernelTimer() {
    if (!a) return;
    hipEvent_t b = take_event(h);
    if (b && hipEventRecord(b, s) == hipSuccess) {
      h->timed.push_back({stage, a, b});
    } else {
      h->ev_pool.push_back(a);
      if (b) h->ev_pool.push_back(b);
    }
  }
};

// Chunk and partial-block capacities of a handle from its configuration.
// Chunks per call: the split schedule's chunking gives at most n_cu + W
// (about n_cu groups of source frames, plus one partial group per window),
// or F / chunk_frames + W with fixed chunking; the fused schedule one per
// window.  The capacity-sized launches of ba_launch use this bound.
void set_capacities(ba_handle* h) {
  const ba_config* cfg = &h->cfg;
  const int64_t W = cfg->max_windows, F = cfg->max_frames;
  const int64_t Dmax = 6LL * cfg->max_frames_per_window;
  int64_t cap_c = std::min<int64_t>(F, (int64_t)h->n_cu + W);
  if (cfg->chunk_frames > 0) cap_c = std::min<int64_t>(F, (F + cfg->chunk_frames - 1) / cfg->chunk_frames + W);
  h->cap_chunks = std::max<int64_t>(cap_c, W);
  // partial blocks: one chunk per window, and about two chunks per CU across
  // the batch (or the fixed chunking)
  int64_t blocks = std::max<int64_t>(W, std::min<int64_t>(F, 2LL * h->n_cu));
  if (cfg->chunk_frames > 0)
    blocks = std::max(blocks, std::min<int64_t>(F, W * ((cfg->max_frames_per_window + cfg->chunk_frames - 1) /
                                                          cfg->chunk_frames)));
  h->cap_partial = blocks * (Dmax * Dmax + 2 * Dmax);
  // edge blocks: every window's edges in blocks of EPB, so at most one partial
  // block per window beyond the total
  h->cap_eblocks = (std::max<int64_t>(cfg->max_edges, 0) + EPB - 1) / EPB + W;
}

// Every device buffer of a handle's workspace except the chunk partials,
// sized from its capacities; `take(&ptr, bytes)` provides each one.
template <class Take>
void carve_workspace(ba_handle* h, Take take) {
  const ba_config* cfg = &h->cfg;
  const int64_t W = cfg->max_windows, F = cfg->max_frames, Pn = std::max<int64_t>(cfg->max_patches, 1),
                E = std::max<int64_t>(cfg->max_edges, 1);
  const size_t esz = cfg->precision == BA_PREC_FP32 ? 4 : 8;
  take((void**)&h->d_win, sizeof(WinDesc) * W);
  take((void**)&h->d_chunk, sizeof(ChunkDesc) * h->cap_chunks);
  take((void**)&h->d_counts, 16);
  take((void**)&h->status, 4 * W);
  take((void**)&h->eflags, 4 * std::max<int64_t>(h->cap_eblocks, 1));
  take((void**)&h->wmeta, 16 * W);
  take((void**)&h->cnt, 4 * Pn);
  take((void**)&h->ptr, 4 * Pn);
  take((void**)&h->fill, 4 * Pn);
  take((void**)&h->jrun, 8 * Pn);
  take((void**)&h->acnt, 4 * (F + W));
  take((void**)&h->afill, 4 * F);
  take((void**)&h->plist, 4 * Pn);
  take((void**)&h->csr, 4 * E);
  take((void**)&h->arange, 8 * F);
  take((void**)&h->cstate, 8 * h->cap_chunks);
  if (6 * cfg->max_frames_per_window > NCHOL_MAX) {
    h->ld_big = big_ld(cfg->max_frames_per_window);
    take((void**)&h->s_big, 8 * (size_t)W * h->ld_big * h->ld_big);
    take((void**)&h->big_aux, 8 * (size_t)W * big_aux_stride(h->ld_big));
  }
  take((void**)&h->dxi, 8 * 6 * F);
  const int64_t slots = cfg->iterations + 1;
  take((void**)&h->pose_buf, 8 * slots * 7 * F);
  take((void**)&h->depth_buf, 8 * slots * Pn);
  take((void**)&h->gidx, 4 * E);
  take((void**)&h->xib, 8 * 6 * F);
  take((void**)&h->xid, 8 * 6 * F);
  take((void**)&h->qxi, 8 * 6 * F);
  take((void**)&h->dbar, 8 * 2 * Pn);
  take((void**)&h->fcot, 8 * RMAX * 6 * h->cap_chunks);
  h->cap_sb = Pn / 16 + F + 2 * W;
  take((void**)&h->estart, 4 * (Pn + W));
  take((void**)&h->sbstart, 4 * (F + W));
  take((void**)&h->sbd, 16 * h->cap_sb);
  take(&h->pxy, 16 * Pn);
  take((void**)&h->gj, 4 * E);
  take(&h->gt, 2 * esz * E);
  take(&h->gw, 2 * esz * E);
}

// Host-side checks of a configuration shared by ba_create and
// ba_solve_noalloc (capacities excepted).
int check_config_numerics(const ba_config* cfg) {
  if (!cfg) return BA_E_INVAL;
  if (cfg->precision != BA_PREC_FP64 && cfg->precision != BA_PREC_FP32) return BA_E_INVAL;
  if (cfg->iterations < 0 || cfg->iterations > 64) return BA_E_INVAL;
  if (!(cfg->lambda >= 0.0) || !std::isfinite(cfg->lambda) || !std::isfinite(cfg->z_min)) return BA_E_INVAL;
  if (cfg->schedule < 0 || cfg->schedule > 2) return BA_E_INVAL;
  if (cfg->chunk_frames < 0) return BA_E_INVAL;
  return BA_OK;
}

// Accumulator tiles per wave: the smallest instantiated count that holds a
// chunk's lower-triangle tiles in one pass (larger chunks take several passes
// with 8, or in FP32 with 12, whose running sums stay in memory).
int maxt_for(int tiles, bool fp32) {
  if (tiles <= NWAVES * 4) return 4;
  if (tiles <= NWAVES * 5) return 5;
  if (tiles <= NWAVES * 8 || !fp32) return 8;
  return 12;
}

// k_assemble with the tile count the plan selected (12 exists in FP32 only).
template <typename T>
void launch_assemble(int maxt, dim3 grid, int lds, hipStream_t s, const Params& P, int iter, int Rcap) {
  if (maxt == 4) hipLaunchKernelGGL((k_assemble<T, 4>), grid, dim3(WG), lds, s, P, iter, Rcap);
  else if (maxt == 5) hipLaunchKernelGGL((k_assemble<T, 5>), grid, dim3(WG), lds, s, P, iter, Rcap);
  else if constexpr (sizeof(T) == 4) {
    if (maxt == 12) hipLaunchKernelGGL((k_assemble<T, 12>), grid, dim3(WG), lds, s, P, iter, Rcap);
    else hipLaunchKernelGGL((k_assemble<T, 8>), grid, dim3(WG), lds, s, P, iter, Rcap);
  } else {
    hipLaunchKernelGGL((k_assemble<T, 8>), grid, dim3(WG), lds, s, P, iter, Rcap);
  }
}

struct Plan {
  int W = 0, C = 0, Rcap = 1, nmax = 0, maxt = 4, EB = 0;
  int64_t Emax = 0;        // edges of the largest window
  bool fused = false;
  bool capacity = false;   // grids sized for the handle's capacities (ba_launch)
  bool big = false;        // some window has more than 21 free frames
  bool small = false;      // some window has at most 21 (the LDS Cholesky's windows)
  int64_t F = 0, Pn = 0, E = 0;
};

int validate_and_plan(ba_handle* h, const ba_problem* p, Plan& pl) {
  const ba_config& cfg = h->cfg;
  if (!p) return fail(h, BA_E_INVAL, "problem is NULL");
  const int W = p->n_windows;
  if (W < 0) return fail(h, BA_E_INVAL, "n_windows < 0");
  if (W > cfg.max_windows) return fail(h, BA_E_CAPACITY, "n_windows exceeds max_windows");
  pl.W = W;
  if (W == 0) return BA_OK;
  if (!p->frame_off || !p->patch_off || !p->edge_off || !p->n_fixed || !p->intrinsics)
    return fail(h, BA_E_INVAL, "host offset / n_fixed / intrinsics pointer is NULL");
  if (p->frame_off[0] != 0 || p->patch_off[0] != 0 || p->edge_off[0] != 0)
    return fail(h, BA_E_INVAL, "offsets must start at 0");
  for (int w = 0; w < W; ++w) {
    const int64_t N = p->frame_off[w + 1] - p->frame_off[w];
    const int64_t M = p->patch_off[w + 1] - p->patch_off[w];
    const int64_t E = p->edge_off[w + 1] - p->edge_off[w];
    if (N < 0 || M < 0 || E < 0) return fail(h, BA_E_INVAL, "offsets must be non-decreasing");
    if (N > cfg.max_frames_per_window)
      return fail(h, BA_E_CAPACITY, "window %d has more frames than max_frames_per_window", w);
    if (M > INT32_MAX / 2 || E > INT32_MAX / 2) return fail(h, BA_E_CAPACITY, "window too large");
    pl.Emax = std::max(pl.Emax, E);
    const int nf = p->n_fixed[w];
    if (nf < 0 || nf > N) return fail(h, BA_E_INVAL, "n_fixed outside [0, frames] in window %d", w);
    const int n = 6 * (int)(N - nf);
    if (n <= NCHOL_MAX) pl.small = true;
    if (n > NCHOL_MAX) {
      if (!h->s_big)
        return fail(h, BA_E_CAPACITY, "window %d: more than 21 free frames", w);
      pl.big = true;
    }
    pl.nmax = std::max(pl.nmax, n);
    {
      // accumulator tiles per wave: lower-triangle 16x16 tiles of (n+1)^2 over 8 waves
      const int T16 = (n + 1 + 15) / 16;
      const int L = T16 * (T16 + 1) / 2;
      pl.maxt = std::max(pl.maxt, maxt_for(L, cfg.precision == BA_PREC_FP32));
    }
    pl.Rcap = std::max<int>(pl.Rcap, (int)N);
    const double* K = p->intrinsics + 4 * w;
    for (int m = 0; m < 4; ++m)
      if (!std::isfinite(K[m])) return fail(h, BA_E_INVAL, "non-finite intrinsics");
    if (K[0] == 0.0 || K[1] == 0.0) return fail(h, BA_E_INVAL, "zero focal length");
  }
  pl.F = p->frame_off[W];
  pl.Pn = p->patch_off[W];
  pl.E = p->edge_off[W];
  if (pl.F > cfg.max_frames || pl.Pn > cfg.max_patches || pl.E > cfg.max_edges)
    return fail(h, BA_E_CAPACITY, "batch totals exceed the handle's capacities");
  if (pl.F > 0 && (!p->poses_in || !p->poses_out)) return fail(h, BA_E_INVAL, "pose pointer is NULL");
  if (pl.Pn > 0 && (!p->patches_in || !p->anchor || !p->depth_out))
    return fail(h, BA_E_INVAL, "patch pointer is NULL");
  if (pl.E > 0 && (!p->kk || !p->jj || !p->targets || !p->weights))
    return fail(h, BA_E_INVAL, "edge pointer is NULL");
  return BA_OK;
}

// Chunking: split each window into runs of `c` consecutive source frames.
// The fused schedule uses one chunk per window.  `sched` is BA_SCHED_*.
int build_descriptors(ba_handle* h, const ba_problem* p, Plan& pl, int sched) {
  const ba_config& cfg = h->cfg;
  const int W = pl.W;
  int64_t total_anchor = 0;
  for (int w = 0; w < W; ++w) total_anchor += p->frame_off[w + 1] - p->frame_off[w];
  if (sched == BA_SCHED_FUSED) pl.fused = true;
  else if (sched == BA_SCHED_SPLIT) pl.fused = false;
  else pl.fused = false;   // AUTO: the split schedule, faster at every batch size measured
  // anchors per chunk for the split schedule: fixed, or aim for one assembly
  // workgroup per CU, with at least two source frames per chunk (a window cut
  // into single frames leaves the solve ~4 us per chunk partial to gather,
  // more than the assembly gains: measured faster for batches of 1-8 windows
  // of 22 x 96, the same from 12 windows up, where this bound does not bite)
  int c = 1;
  if (!pl.fused) {
    if (cfg.chunk_frames > 0) {
      c = cfg.chunk_frames;
    } else {
      const int64_t target = h->n_cu;
      c = (int)std::max<int64_t>(2, (total_anchor + target - 1) / target);
    }
  }
  for (;;) {
    int64_t chunks = 0, part = 0;
    for (int w = 0; w < W; ++w) {
      const int N = (int)(p->frame_off[w + 1] - p->frame_off[w]);
      const int cw = pl.fused ? std::max(N, 1) : c;
      const int nc = N == 0 ? 0 : (N + cw - 1) / cw;
      const int64_t D = 6LL * (N - p->n_fixed[w]);
      chunks += nc;
      part += nc * (D * D + 2 * D);
    }
    if (chunks <= h->cap_chunks && part <= h->cap_partial) break;
    // one chunk per window always fits the workspace ba_create sizes
    if (pl.fused || cfg.chunk_frames > 0 || c >= cfg.max_frames_per_window)
      return fail(h, BA_E_CAPACITY, "partial workspace too small");
    c *= 2;
  }
  if (h->staging_pending) {
    HIPCHK(h, hipEventSynchronize(h->staging_ev));
    h->staging_pending = false;
  }
  int64_t part_off = 0, sb_off = 0;
  int ci = 0, eb = 0;
  for (int w = 0; w < W; ++w) {
    WinDesc& d = h->h_win[w];
    const int N = (int)(p->frame_off[w + 1] - p->frame_off[w]);
    d.frame_off = p->frame_off[w];
    d.patch_off = p->patch_off[w];
    d.edge_off = p->edge_off[w];
    d.n_frames = N;
    d.n_patches = (int)(p->patch_off[w + 1] - p->patch_off[w]);
    d.n_edges = (int)(p->edge_off[w + 1] - p->edge_off[w]);
    d.n_fixed = p->n_fixed[w];
    d.fx = p->intrinsics[4 * w + 0];
    d.fy = p->intrinsics[4 * w + 1];
    d.cx = p->intrinsics[4 * w + 2];
    d.cy = p->intrinsics[4 * w + 3];
    const int cw = pl.fused ? std::max(N, 1) : c;
    const int nc = N == 0 ? 0 : (N + cw - 1) / cw;
    const int64_t D = 6LL * (N - d.n_fixed);
    d.chunk_off = ci;
    d.n_chunks = nc;
    d.part_off = part_off;
    d.part_stride = D * D + 2 * D;
    d.sb_off = sb_off;
    sb_off += (d.n_patches + 15) / 16 + N + 1;
    d.eb_off = eb;
    d.eb_n = (d.n_edges + EPB - 1) / EPB;
    eb += d.eb_n;
    for (int q = 0; q < nc; ++q) {
      ChunkDesc& cd = h->h_chunk[ci++];
      cd.window = w;
      cd.a_lo = q * cw;
      cd.a_hi = std::min(N, (q + 1) * cw);
      cd.pad = 0;
    }
    part_off += nc * d.part_stride;
  }
  pl.C = ci;
  pl.EB = eb;
  if (sb_off > h->cap_sb) return fail(h, BA_E_CAPACITY, "sub-batch table too small");
  return BA_OK;
}

void fill_params(ba_handle* h, const ba_problem* p, const Plan& pl, Params& P) {
  memset(&P, 0, sizeof(P));
  P.win = h->d_win;
  P.chunk = h->d_chunk;
  P.counts = h->d_counts;
  P.iterations = h->cfg.iterations;
  P.lambda = h->cfg.lambda;
  P.z_min = h->cfg.z_min;
  P.poses_in = p->poses_in;
  P.patches_in = p->patches_in;
  P.anchor = p->anchor;
  P.kk = p->kk;
  P.jj = p->jj;
  P.targets = p->targets;
  P.weights = p->weights;
  P.poses_out = p->poses_out;
  P.depth_out = p->depth_out;
  P.status = h->status;
  P.eflags = h->eflags;
  P.wmeta = h->wmeta;
  P.cnt = h->cnt;
  P.ptr = h->ptr;
  P.fill = h->fill;
  P.jrun = h->jrun;
  P.acnt = h->acnt;
  P.afill = h->afill;
  P.plist = h->plist;
  P.csr = h->csr;
  P.arange = h->arange;
  P.cstate = h->cstate;
  P.partial = h->partial;
  P.s_big = h->s_big;
  P.ld_big = h->ld_big;
  P.big_aux = h->big_aux;
  P.dxi = h->dxi;
  P.pose_buf = h->pose_buf;
  P.depth_buf = h->depth_buf;
  P.n_frames_total = h->cfg.max_frames;
  P.n_patches_total = std::max<int64_t>(h->cfg.max_patches, 1);
  P.estart = h->estart;
  P.sbstart = h->sbstart;
  P.sbd = h->sbd;
  P.pxy = h->pxy;
  P.gj = h->gj;
  P.gt = h->gt;
  P.gw = h->gw;
  P.gidx = h->gidx;
  P.xib = h->xib;
  P.xid = h->xid;
  P.qxi = h->qxi;
  P.dbar = h->dbar;
  P.fcot = h->fcot;
}

// Copies the staged descriptors and the window / chunk counts of `pl`.
int upload_descriptors(ba_handle* h, const Plan& pl, hipStream_t s) {
  h->h_counts[0] = pl.W;
  h->h_counts[1] = pl.C;
  h->h_counts[2] = pl.EB;
  HIPCHK(h, hipMemcpyAsync(h->d_counts, h->h_counts, 12, hipMemcpyHostToDevice, s));
  if (pl.W > 0)
    HIPCHK(h, hipMemcpyAsync(h->d_win, h->h_win, sizeof(WinDesc) * pl.W, hipMemcpyHostToDevice, s));
  if (pl.C > 0)
    HIPCHK(h, hipMemcpyAsync(h->d_chunk, h->h_chunk, sizeof(ChunkDesc) * pl.C, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipEventRecord(h->staging_ev, s));
  h->staging_pending = true;
  return BA_OK;
}

// Enqueues the forward solve.  The descriptors of `pl` must have been
// uploaded on `s` before.  With pl.capacity the grids and LDS sizes are those
// of the handle's capacities and the kernels read the batch size from the
// device counts; otherwise they are sized for the batch.
template <typename T>
int launch_solve(ba_handle* h, const ba_problem* p, const Plan& pl, hipStream_t s) {
  Params P;
  fill_params(h, p, pl, P);
  const int gW = pl.capacity ? h->cfg.max_windows : pl.W;
  const int gC = pl.capacity ? (int)h->cap_chunks : pl.C;
  const int Rcap = pl.Rcap;
  const int asm_lds = asm_layout(Rcap, (int)sizeof(T), pl.maxt).total;
  const int chol_lds = chol_lds_bytes(std::min(pl.nmax, NCHOL_MAX));
  const int big_lds = chol_big_lds_bytes(pl.nmax);
  const int bs_lds = backsub_lds_bytes(Rcap, (int)sizeof(T));
  // the back-substitution splits each chunk's sub-batches over several
  // workgroups, for about two workgroups per CU
  const int bs_parts = gC > 0 ? std::max(1, std::min(4, (2 * h->n_cu + gC - 1) / gC)) : 1;
  if (gW == 0) return BA_OK;
  if (pl.fused && pl.big) return fail(h, BA_E_CAPACITY, "the fused schedule holds at most 21 free frames per window");
  if (pl.fused) {
    const int lds = std::max(std::max(asm_lds, chol_lds), std::max(bs_lds, PREP_LDS_INTS * 4));
    const int grid = std::min(gW, 4 * h->n_cu);
    KernelTimer kt(h, s, BA_STAGE_FUSED);
    if (pl.maxt == 4) hipLaunchKernelGGL((k_fused<T, 4>), dim3(grid), dim3(WG), lds, s, P, Rcap);
    else if (pl.maxt == 5) hipLaunchKernelGGL((k_fused<T, 5>), dim3(grid), dim3(WG), lds, s, P, Rcap);
    else hipLaunchKernelGGL((k_fused<T, 8>), dim3(grid), dim3(WG), lds, s, P, Rcap);
    HIPCHK(h, hipGetLastError());
  } else {
    {
      // the edge pass over many workgroups, then the rest per window.  The
      // split pays when the batch leaves most CUs idle or a window is large;
      // with many windows of moderate size the extra launch costs more than
      // it saves.  Captured launches always split (any batch may follow).
      const bool split = pl.capacity || 4LL * pl.W <= h->n_cu || pl.Emax >= 16LL * EPB;
      const int64_t gEB = !split ? 0 : pl.capacity ? h->cap_eblocks : pl.EB;
      KernelTimer kt(h, s, BA_STAGE_PREP);
      if (gEB > 0) hipLaunchKernelGGL(k_prep_edges, dim3((unsigned)gEB), dim3(WG), 0, s, P);
      hipLaunchKernelGGL(k_prep<T>, dim3(gW), dim3(WG), 0, s, P, gEB > 0 ? 1 : 0);
    }
    HIPCHK(h, hipGetLastError());
    for (int it = 0; it < P.iterations; ++it) {
      if (gC > 0) {
        KernelTimer kt(h, s, BA_STAGE_ASSEMBLE);
        launch_assemble<T>(pl.maxt, dim3(gC), asm_lds, s, P, it, Rcap);
      }
      HIPCHK(h, hipGetLastError());
      {
        KernelTimer kt(h, s, BA_STAGE_CHOL);
        if (pl.small) hipLaunchKernelGGL(k_chol<T>, dim3(gW), dim3(WG), chol_lds, s, P, it);
        if (pl.big) {
          const int tiles = gather_tiles(pl.nmax);
          hipLaunchKernelGGL(k_gather_big, dim3(gW * tiles), dim3(WG), 0, s, P, tiles);
          for (int j = 0; PW * j < pl.nmax; ++j) {
            const int groups = upd_groups(pl.nmax, j);
            hipLaunchKernelGGL(k_chol_panel, dim3(gW * (1 + groups)), dim3(WG), chol_panel_lds_bytes(pl.nmax), s, P, j,
                               groups);
          }
          hipLaunchKernelGGL(k_chol_big<T>, dim3(gW), dim3(WG), big_lds, s, P, it);
        }
      }
      HIPCHK(h, hipGetLastError());
      if (gC > 0) {
        KernelTimer kt(h, s, BA_STAGE_BACKSUB);
        hipLaunchKernelGGL(k_backsub<T>, dim3(gC * bs_parts), dim3(WG), bs_lds, s, P, it, Rcap, bs_parts);
      }
      HIPCHK(h, hipGetLastError());
    }
    {
      KernelTimer kt(h, s, BA_STAGE_FINALIZE);
      hipLaunchKernelGGL(k_finalize, dim3(gW), dim3(WG), 0, s, P);
    }
    HIPCHK(h, hipGetLastError());
  }
  return BA_OK;
}

template <typename T>
int launch_backward(ba_handle* h, const ba_problem* p, const Plan& pl, const double* grad_poses,
                    const double* grad_depth, void* grad_targets, void* grad_weights,
                    hipStream_t s) {
  Params P;
  fill_params(h, p, pl, P);
  P.grad_poses = grad_poses;
  P.grad_depth = grad_depth;
  P.grad_targets = grad_targets;
  P.grad_weights = grad_weights;
  int r = upload_descriptors(h, pl, s);
  if (r != BA_OK) return r;
  const int Rcap = pl.Rcap, esz = (int)sizeof(T);
  const int asm_lds = asm_layout(Rcap, esz, pl.maxt).total;
  const int bs_lds = backsub_lds_bytes(Rcap, esz);
  const int nsmall = std::min(pl.nmax, NCHOL_MAX);   // windows above take the panel path
  const int chol_lds = chol_lds_bytes(nsmall);
  const int chol_adj_lds = chol_lds + 2 * 8 * nsmall + 64;
  const int adj_lds = edge_adj_lds_bytes(Rcap, esz);
  const int K = P.iterations;
  hipLaunchKernelGGL(k_prep<T>, dim3(pl.W), dim3(WG), 0, s, P, 0);
  HIPCHK(h, hipGetLastError());
  // windows with n > 126: the system gathered into device memory and
  // factorised by panels (the forward path's kernels)
  auto big_factor = [&](const Params& Q) {
    const int tiles = gather_tiles(pl.nmax);
    hipLaunchKernelGGL(k_gather_big, dim3(pl.W * tiles), dim3(WG), 0, s, Q, tiles);
    for (int j = 0; PW * j < pl.nmax; ++j) {
      const int groups = upd_groups(pl.nmax, j);
      hipLaunchKernelGGL(k_chol_panel, dim3(pl.W * (1 + groups)), dim3(WG), chol_panel_lds_bytes(pl.nmax), s, Q, j,
                         groups);
    }
  };
  // recompute the iterates x_1 .. x_{K-1}
  for (int it = 0; it + 1 < K; ++it) {
    launch_assemble<T>(pl.maxt, dim3(pl.C), asm_lds, s, P, it, Rcap);
    if (pl.small) hipLaunchKernelGGL(k_chol<T>, dim3(pl.W), dim3(WG), chol_lds, s, P, it);
    if (pl.big) {
      big_factor(P);
      hipLaunchKernelGGL(k_chol_big<T>, dim3(pl.W), dim3(WG), chol_big_lds_bytes(pl.nmax), s, P, it);
    }
    hipLaunchKernelGGL(k_backsub<T>, dim3(pl.C), dim3(WG), bs_lds, s, P, it, Rcap, 1);
    HIPCHK(h, hipGetLastError());
  }
  hipLaunchKernelGGL(k_adj_init<T>, dim3(pl.W), dim3(WG), 0, s, P);
  HIPCHK(h, hipGetLastError());
  Params PA = P;
  PA.adjoint = 1;
  for (int it = K - 1; it >= 0; --it) {
    launch_assemble<T>(pl.maxt, dim3(pl.C), asm_lds, s, PA, it, Rcap);
    if (pl.small) hipLaunchKernelGGL(k_chol_adj<T>, dim3(pl.W), dim3(WG), chol_adj_lds, s, PA, it);
    if (pl.big) {
      big_factor(PA);
      hipLaunchKernelGGL(k_chol_adj_big<T>, dim3(pl.W), dim3(WG), chol_adj_big_lds_bytes(pl.nmax), s, PA, it);
    }
    hipLaunchKernelGGL(k_edge_adj<T>, dim3(pl.C), dim3(WG), adj_lds, s, PA, it, Rcap);
    hipLaunchKernelGGL(k_frame_adj, dim3(pl.W), dim3(WG), 0, s, PA);
    HIPCHK(h, hipGetLastError());
  }
  return BA_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free solve.  The workspace of ba_solve_noalloc is carved, per
// call, from `scratch`, a device array of fixed size: each GPU the library
// runs on holds its own copy until the process ends.  Host code never uses
// the array's name as an address: its device address is taken once per device
// with hipGetSymbolAddress and kept in `NoallocDevice::base`.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;   // 64 MiB per GPU
constexpr int NOALLOC_MAX_DEVICES = 16;
constexpr int NOALLOC_MAX_WINDOWS = 256;
constexpr int NOALLOC_MAX_CHUNKS = 4096;

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

struct NoallocDevice {
  std::mutex mu;                 // one call at a time per device on the host side
  bool ready = false;
  char* base = nullptr;          // device address of `scratch` on this device
  ba_handle h;                   // workspace pointers into `scratch`, no allocation
  WinDesc hwin[NOALLOC_MAX_WINDOWS];
  ChunkDesc hchunk[NOALLOC_MAX_CHUNKS];
  int32_t hcounts[4];
};

NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];

// Once per device, with the device current: the address of its copy of
// `scratch`, the CU count, the kernels' LDS limits.
int noalloc_init(NoallocDevice& D, int dev) {
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return BA_E_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return BA_E_HIP;
  if (set_kernel_attrs<float>() != 0 || set_kernel_attrs<double>() != 0) return BA_E_HIP;
  D.base = (char*)ptr;
  D.h.device = dev;
  D.h.n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  D.h.h_win = D.hwin;
  D.h.h_chunk = D.hchunk;
  D.h.h_counts = D.hcounts;
  D.ready = true;
  return BA_OK;
}

// Stores `bytes` (a multiple of 4) from host `src` at device `dst` inside the
// workspace, through the arguments of k_upload launches on `s`.
int noalloc_upload(ba_handle* h, char* base, void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  const int64_t off = (int64_t)((char*)dst - base);
  UploadBlock b;
  for (size_t w0 = 0; w0 < words; w0 += UPLOAD_WORDS) {
    const int n = (int)std::min<size_t>(UPLOAD_WORDS, words - w0);
    b.dst = off + 4 * (int64_t)w0;
    b.n = n;
    b.pad = 0;
    memcpy(b.w, (const char*)src + 4 * w0, 4 * (size_t)n);
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, base, b);
    HIPCHK(h, hipGetLastError());
  }
  return BA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
extern "C" {

int ba_create(const ba_config* cfg, ba_handle** out) {
  if (!out) return BA_E_INVAL;
  *out = nullptr;
  if (check_config_numerics(cfg) != BA_OK) return BA_E_INVAL;
  if (cfg->max_windows < 1 || cfg->max_frames_per_window < 1 || cfg->max_frames_per_window > RMAX)
    return BA_E_INVAL;
  if (cfg->precision == BA_PREC_FP64 && cfg->max_frames_per_window > 24) return BA_E_INVAL;
  if (cfg->max_frames < 1 || cfg->max_patches < 0 || cfg->max_edges < 0) return BA_E_INVAL;

  ba_handle* h = new ba_handle();
  h->cfg = *cfg;
  auto cleanup = [&](int code) { ba_destroy(h); return code; };
  if (hipGetDevice(&h->device) != hipSuccess) return cleanup(BA_E_HIP);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) return cleanup(BA_E_HIP);
  h->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  const int r = cfg->precision == BA_PREC_FP32 ? set_kernel_attrs<float>() : set_kernel_attrs<double>();
  if (r != 0) return cleanup(BA_E_HIP);

  set_capacities(h);
  h->launch_fused = cfg->schedule == BA_SCHED_FUSED;
  bool ok = true;
  auto dmalloc = [&](void** ptr, size_t bytes) {
    if (!ok) return;
    if (hipMalloc(ptr, std::max<size_t>(bytes, 256)) != hipSuccess) ok = false;
  };
  carve_workspace(h, dmalloc);
  dmalloc((void**)&h->partial, 8 * h->cap_partial);
  if (!ok) return cleanup(BA_E_HIP);
  if (hipHostMalloc((void**)&h->h_win, sizeof(WinDesc) * cfg->max_windows) != hipSuccess) return cleanup(BA_E_HIP);
  if (hipHostMalloc((void**)&h->h_chunk, sizeof(ChunkDesc) * h->cap_chunks) != hipSuccess) return cleanup(BA_E_HIP);
  if (hipHostMalloc((void**)&h->h_counts, 16) != hipSuccess) return cleanup(BA_E_HIP);
  if (hipEventCreateWithFlags(&h->staging_ev, hipEventDisableTiming) != hipSuccess) return cleanup(BA_E_HIP);
  if (hipMemset(h->status, 0, 4 * cfg->max_windows) != hipSuccess) return cleanup(BA_E_HIP);
  *out = h;
  return BA_OK;
}

int ba_solve(ba_handle* h, const ba_problem* p, void* stream) {
  if (!h) return BA_E_INVAL;
  h->err[0] = 0;
  Plan pl;
  int r = validate_and_plan(h, p, pl);
  if (r != BA_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  h->last_W = pl.W;
  if (pl.W == 0) return BA_OK;
  int sched = h->cfg.schedule;
  if (pl.big) {
    if (sched == BA_SCHED_FUSED)
      return fail(h, BA_E_CAPACITY, "the fused schedule holds at most 21 free frames per window");
    sched = BA_SCHED_SPLIT;
  }
  r = build_descriptors(h, p, pl, sched);
  if (r != BA_OK) return r;
  r = upload_descriptors(h, pl, s);
  if (r != BA_OK) return r;
  return h->cfg.precision == BA_PREC_FP32 ? launch_solve<float>(h, p, pl, s)
                                          : launch_solve<double>(h, p, pl, s);
}

int ba_solve_noalloc(const ba_config* cfg, const ba_problem* p, int32_t* status_out, void* stream) {
  if (check_config_numerics(cfg) != BA_OK || !p || p->n_windows < 0) return BA_E_INVAL;
  const int W = p->n_windows;
  if (W == 0) return BA_OK;
  if (W > NOALLOC_MAX_WINDOWS) return BA_E_CAPACITY;
  if (!p->frame_off || !p->patch_off || !p->edge_off || !p->n_fixed || !p->intrinsics) return BA_E_INVAL;
  if (p->frame_off[0] != 0 || p->patch_off[0] != 0 || p->edge_off[0] != 0) return BA_E_INVAL;
  int64_t rmax = 1;
  for (int w = 0; w < W; ++w) {
    const int64_t N = p->frame_off[w + 1] - p->frame_off[w];
    if (N < 0 || p->patch_off[w + 1] < p->patch_off[w] || p->edge_off[w + 1] < p->edge_off[w]) return BA_E_INVAL;
    rmax = std::max(rmax, N);
  }
  if (rmax > RMAX || (cfg->precision == BA_PREC_FP64 && rmax > 24)) return BA_E_CAPACITY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BA_E_HIP;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return BA_E_CAPACITY;
  NoallocDevice& D = g_noalloc[dev];
  std::lock_guard<std::mutex> lock(D.mu);
  if (!D.ready) {
    const int r = noalloc_init(D, dev);
    if (r != BA_OK) return r;
  }
  ba_handle* h = &D.h;
  h->err[0] = 0;
  // capacities: exactly this batch
  h->cfg = *cfg;
  h->cfg.max_windows = W;
  h->cfg.max_frames_per_window = (int32_t)rmax;
  h->cfg.max_frames = std::max<int64_t>(1, p->frame_off[W]);
  h->cfg.max_patches = p->patch_off[W];
  h->cfg.max_edges = p->edge_off[W];
  set_capacities(h);
  h->cap_chunks = std::min<int64_t>(h->cap_chunks, NOALLOC_MAX_CHUNKS);
  h->s_big = nullptr;
  h->big_aux = nullptr;
  h->ld_big = 0;
  size_t off = 0;
  bool fits = true;
  auto take = [&](void** ptr, size_t bytes) {
    const size_t b = (std::max<size_t>(bytes, 256) + 255) & ~size_t(255);
    if (!fits || b > NOALLOC_SCRATCH_BYTES - off) {
      fits = false;
      *ptr = nullptr;
      return;
    }
    *ptr = D.base + off;
    off += b;
  };
  carve_workspace(h, take);
  if (!fits) return fail(h, BA_E_CAPACITY, "batch exceeds the %zu-byte static workspace", NOALLOC_SCRATCH_BYTES);
  // the chunk partials take the rest; the chunking grows when they do not fit
  h->partial = (double*)(D.base + off);
  h->cap_partial = (int64_t)((NOALLOC_SCRATCH_BYTES - off) / 8);
  Plan pl;
  int r = validate_and_plan(h, p, pl);
  if (r != BA_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  int sched = cfg->schedule;
  if (pl.big) {
    if (sched == BA_SCHED_FUSED)
      return fail(h, BA_E_CAPACITY, "the fused schedule holds at most 21 free frames per window");
    sched = BA_SCHED_SPLIT;
  }
  r = build_descriptors(h, p, pl, sched);
  if (r != BA_OK) return r;
  h->h_counts[0] = pl.W;
  h->h_counts[1] = pl.C;
  h->h_counts[2] = pl.EB;
  h->h_counts[3] = 0;
  r = noalloc_upload(h, D.base, h->d_counts, h->h_counts, 16, s);
  if (r == BA_OK) r = noalloc_upload(h, D.base, h->d_win, h->h_win, sizeof(WinDesc) * pl.W, s);
  if (r == BA_OK && pl.C > 0) r = noalloc_upload(h, D.base, h->d_chunk, h->h_chunk, sizeof(ChunkDesc) * pl.C, s);
  if (r != BA_OK) return r;
  r = cfg->precision == BA_PREC_FP32 ? launch_solve<float>(h, p, pl, s) : launch_solve<double>(h, p, pl, s);
  if (r != BA_OK) return r;
  if (status_out) {
    hipLaunchKernelGGL(k_copy_status, dim3((W + 255) / 256), dim3(256), 0, s, (const int32_t*)h->status, status_out, W);
    HIPCHK(h, hipGetLastError());
  }
  return BA_OK;
}

int ba_backward(ba_handle* h, const ba_problem* p, const double* grad_poses,
                const double* grad_depth, void* grad_targets, void* grad_weights, void* stream) {
  if (!h) return BA_E_INVAL;
  h->err[0] = 0;
  Plan pl;
  int r = validate_and_plan(h, p, pl);
  if (r != BA_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  h->last_W = pl.W;
  if (pl.W == 0) return BA_OK;
  if (h->cfg.iterations < 1) return fail(h, BA_E_STATE, "ba_backward needs at least one iteration");
  if ((pl.F > 0 && !grad_poses) || (pl.Pn > 0 && !grad_depth) ||
      (pl.E > 0 && (!grad_targets || !grad_weights)))
    return fail(h, BA_E_INVAL, "gradient pointer is NULL");
  r = build_descriptors(h, p, pl, BA_SCHED_SPLIT);
  if (r != BA_OK) return r;
  return h->cfg.precision == BA_PREC_FP32
             ? launch_backward<float>(h, p, pl, grad_poses, grad_depth, grad_targets, grad_weights, s)
             : launch_backward<double>(h, p, pl, grad_poses, grad_depth, grad_targets, grad_weights, s);
}

int ba_prepare(ba_handle* h, const ba_problem* p, void* stream) {
  if (!h) return BA_E_INVAL;
  h->err[0] = 0;
  h->prepared = false;
  Plan pl;
  int r = validate_and_plan(h, p, pl);
  if (r != BA_OK) return r;
  if (pl.big && h->launch_fused)
    return fail(h, BA_E_CAPACITY, "the fused schedule holds at most 21 free frames per window");
  r = build_descriptors(h, p, pl, h->launch_fused ? BA_SCHED_FUSED : BA_SCHED_SPLIT);
  if (r != BA_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  r = upload_descriptors(h, pl, s);
  if (r != BA_OK) return r;
  h->prep_problem = *p;
  h->last_stream = s;
  h->last_W = pl.W;
  h->prepared = true;
  return BA_OK;
}

int ba_launch(ba_handle* h, void* stream) {
  if (!h) return BA_E_INVAL;
  if (!h->prepared) return fail(h, BA_E_STATE, "ba_launch without ba_prepare");
  h->err[0] = 0;
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  Plan pl;
  pl.capacity = true;
  pl.fused = h->launch_fused;
  pl.Rcap = h->cfg.max_frames_per_window;
  pl.nmax = 6 * pl.Rcap;
  pl.big = !pl.fused && pl.nmax > NCHOL_MAX;
  pl.small = true;
  if (pl.fused) pl.nmax = std::min(NCHOL_MAX, pl.nmax);
  {
    // tile passes sized for windows with at least two fixed poses (the gauge
    // of the method); a window with fewer takes a second tile pass, with the
    // same results
    const int n2 = 6 * std::max(pl.Rcap - 2, 1);
    const int T16 = (std::min(pl.nmax, n2) + 1 + 15) / 16;
    pl.maxt = maxt_for(T16 * (T16 + 1) / 2, h->cfg.precision == BA_PREC_FP32);
  }
  const ba_problem* p = &h->prep_problem;
  return h->cfg.precision == BA_PREC_FP32 ? launch_solve<float>(h, p, pl, s)
                                          : launch_solve<double>(h, p, pl, s);
}

int ba_set_timing(ba_handle* h, int32_t enable) {
  if (!h) return BA_E_INVAL;
  h->timing = enable & BA_TIMING_ALL;
  return BA_OK;
}

int ba_kernel_times(ba_handle* h, double* ms_out, int32_t* launches_out) {
  if (!h || !ms_out || !launches_out) return BA_E_INVAL;
  for (int i = 0; i < BA_STAGE_COUNT; ++i) {
    ms_out[i] = 0.0;
    launches_out[i] = 0;
  }
  int rc = BA_OK;
  for (const auto& t : h->timed) {
    float ms = 0.f;
    if (rc == BA_OK) {
      hipError_t e = hipEventSynchronize(t.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
      if (e != hipSuccess) rc = fail(h, BA_E_HIP, "kernel timing: %s", hipGetErrorString(e));
    }
    if (rc == BA_OK && t.stage >= 0 && t.stage < BA_STAGE_COUNT) {
      ms_out[t.stage] += ms;
      launches_out[t.stage] += 1;
    }
    h->ev_pool.push_back(t.a);
    h->ev_pool.push_back(t.b);
  }
  h->timed.clear();
  return rc;
}

int ba_status(ba_handle* h, int32_t* host_flags) {
  if (!h || !host_flags) return BA_E_INVAL;
  // copy on the handle's own stream, so that other streams are not waited for
  if (h->last_W > 0)
    HIPCHK(h, hipMemcpyAsync(host_flags, h->status, 4 * h->last_W, hipMemcpyDeviceToHost, h->last_stream));
  HIPCHK(h, hipStreamSynchronize(h->last_stream));
  return BA_OK;
}

const char* ba_last_error(const ba_handle* h) { return h ? h->err : "null handle"; }

void ba_destroy(ba_handle* h) {
  if (!h) return;
  hipDeviceSynchronize();
  hipFree(h->d_win);
  hipFree(h->d_chunk);
  hipFree(h->status);
  hipFree(h->wmeta);
  hipFree(h->cnt);
  hipFree(h->ptr);
  hipFree(h->fill);
  hipFree(h->jrun);
  hipFree(h->acnt);
  hipFree(h->afill);
  hipFree(h->plist);
  hipFree(h->csr);
  hipFree(h->arange);
  hipFree(h->cstate);
  hipFree(h->partial);
  hipFree(h->s_big);
  hipFree(h->big_aux);
  hipFree(h->dxi);
  hipFree(h->pose_buf);
  hipFree(h->depth_buf);
  hipFree(h->estart);
  hipFree(h->sbstart);
  hipFree(h->sbd);
  hipFree(h->pxy);
  hipFree(h->gj);
  hipFree(h->gt);
  hipFree(h->gw);
  hipFree(h->gidx);
  hipFree(h->xib);
  hipFree(h->xid);
  hipFree(h->qxi);
  hipFree(h->dbar);
  hipFree(h->fcot);
  if (h->h_win) hipHostFree(h->h_win);
  if (h->h_chunk) hipHostFree(h->h_chunk);
  if (h->h_counts) hipHostFree(h->h_counts);
  hipFree(h->d_counts);
  if (h->staging_ev) hipEventDestroy(h->staging_ev);
  for (auto& t : h->timed) {
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  for (auto e : h->ev_pool) hipEventDestroy(e);
  delete h;
}

int ba_debug_reduced_system(ba_handle* h, const ba_problem* p, int32_t window, double* S_out,
                            double* s_out, void* stream) {
  if (!h) return BA_E_INVAL;
  h->err[0] = 0;
  Plan pl;
  int r = validate_and_plan(h, p, pl);
  if (r != BA_OK) return r;
  if (window < 0 || window >= pl.W) return fail(h, BA_E_INVAL, "window index out of range");
  if (!S_out || !s_out) return fail(h, BA_E_INVAL, "output pointer is NULL");
  r = build_descriptors(h, p, pl, BA_SCHED_SPLIT);
  if (r != BA_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  h->last_W = pl.W;
  Params P;
  fill_params(h, p, pl, P);
  P.iterations = 1;
  r = upload_descriptors(h, pl, s);
  if (r != BA_OK) return r;
  const bool f32 = h->cfg.precision == BA_PREC_FP32;
  const int esz = f32 ? 4 : 8;
  if (f32) hipLaunchKernelGGL(k_prep<float>, dim3(pl.W), dim3(WG), 0, s, P, 0);
  else hipLaunchKernelGGL(k_prep<double>, dim3(pl.W), dim3(WG), 0, s, P, 0);
  HIPCHK(h, hipGetLastError());
  if (pl.C > 0) {
    // the accumulator-tile variant ba_solve selects for this batch
    const int al = asm_layout(pl.Rcap, esz, pl.maxt).total;
    if (f32) {
      launch_assemble<float>(pl.maxt, dim3(pl.C), al, s, P, 0, pl.Rcap);
    } else {
      launch_assemble<double>(pl.maxt, dim3(pl.C), al, s, P, 0, pl.Rcap);
    }
    HIPCHK(h, hipGetLastError());
  }
  const int nw = 6 * (int)(p->frame_off[window + 1] - p->frame_off[window] - p->n_fixed[window]);
  if (nw > NCHOL_MAX) {
    const int tiles = gather_tiles(pl.nmax);
    hipLaunchKernelGGL(k_gather_big, dim3(pl.W * tiles), dim3(WG), 0, s, P, tiles);
    hipLaunchKernelGGL(k_debug_copy_big, dim3(1), dim3(WG), 0, s, P, window, S_out, s_out);
    HIPCHK(h, hipGetLastError());
    return BA_OK;
  }
  const int lds = chol_lds_bytes(std::min(pl.nmax, NCHOL_MAX));
  if (f32) hipLaunchKernelGGL(k_debug_gather<float>, dim3(1), dim3(WG), lds, s, P, window, S_out, s_out);
  else hipLaunchKernelGGL(k_debug_gather<double>, dim3(1), dim3(WG), lds, s, P, window, S_out, s_out);
  HIPCHK(h, hipGetLastError());
  return BA_OK;
}

int ba_debug_mfma(int32_t precision, const void* A, const void* B, void* D, void* stream) {
  if (!A || !B || !D) return BA_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  if (precision == BA_PREC_FP32)
    hipLaunchKernelGGL(k_debug_mfma<float>, dim3(1), dim3(64), 0, s, (const float*)A, (const float*)B, (float*)D);
  else if (precision == BA_PREC_FP64)
    hipLaunchKernelGGL(k_debug_mfma<double>, dim3(1), dim3(64), 0, s, (const double*)A, (const double*)B, (double*)D);
  else
    return BA_E_INVAL;
  return hipGetLastError() == hipSuccess ? BA_OK : BA_E_HIP;
}

}  // extern "C"
