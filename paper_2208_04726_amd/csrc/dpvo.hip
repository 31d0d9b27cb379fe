// Sliding-window driver (include/dpvo.h) on gfx950: the per-frame rules of
// Sec. 3.3 "VO System" applied on the device to many camera streams at once,
// around the batched bundle adjustment of include/dpba.h.
//
// The patch graph of a window is kept as one 64-bit row per keyframe slot:
// every patch of a keyframe is added, and leaves, together with its frame, so
// all patches of one keyframe share one set of target frames, and bit q of
// row p says that the patches of slot p have an edge to the frame in slot q.
// Removing a keyframe deletes its row and its bit column; the expansion sets
// one column and one row.  The edge list the bundle adjustment reads is
// generated from the rows in (patch, target frame) order, which is the order
// the solver consumes without regrouping, and packed without gaps: after
// every step the device predicts each stream's edge count after its next
// expansion, and the host reads it back with the keyframe counts.
//
// Per vo_step:
//   k_vo_expand   (one workgroup per stream): window advance, constant-
//                 velocity pose, median depth of the new patches, new edges;
//   k_vo_build    (many workgroups per stream): the bundle-adjustment arrays
//                 of every edge (window-local indices, sensor lookups);
//   ba_solve      over all streams' windows, in place on the state buffers;
//   k_vo_keyframe (one workgroup per stream): the solved depths into the
//                 state, the flow magnitude between keyframes t-5 and t-3, the
//                 removal of keyframe t-4, and the edge counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/dpba.h"
#include "../../include/dpvo.h"
#include "dpba_common.h"

namespace dpvo {

constexpr int WG = 1024;
constexpr int SORT_MAX = 1024;     // median sort: 3 keyframes' patches
constexpr int MAXN = 64;           // keyframe slots per window
constexpr int STATUS_TABLE = 1 << 16;
constexpr int STATUS_COUNT = 1 << 17;

struct State {
  int S, N, ppf, P, r, n_free, R;
  double thresh, z_min, fx, fy, cx, cy;
  int32_t* n_kf;        // [S]
  int32_t* kf_id;       // [S][N]
  double* poses;        // [S][N][7]
  double* patches;      // [S][P][3]  x, y, inverse depth
  uint64_t* adj;        // [S][N]     bit q of row p: patches of slot p -> frame of slot q
  int32_t* e_next;      // [S]        edges after the stream's next expansion
  int32_t* kk;          // bundle-adjustment arrays, packed by e_off
  int32_t* jj;
  void* tgt;            // [E][2] f32 or f64
  void* wgt;
  const int64_t* e_off; // [S+1] this step's first edge of every stream
  const int32_t* cslot; // [S]    this step's position of the stream among the active ones, or -1
  double* c_poses;      // [S][N][7] the active windows, packed in cslot order, for the solve
  double* c_patches;    // [S][P][3]
  double* depth_out;    // [S][P]    solved inverse depths, packed like c_patches
  double* flow;         // [S]
  int32_t* removed;     // [S]     keyframe removed by this step's keyframing, or -1
  int32_t* removed_prev;// [S]     its previous keyframe
  double* removed_rel;  // [S][7]  its pose relative to that keyframe, T_q T_{q-1}^-1
  int32_t* retired;     // [S]     keyframe that left the full window this step, or -1
  double* retired_pose; // [S][7]  its pose when it left
  int32_t* vstatus;     // [S]
  int32_t* active;      // [S] this step's frame id (-1 idle)
  const double* tab_t;  // sensor
  const double* tab_w;
  const int64_t* tab_off;   // [S] device copy
  const int32_t* tab_frames;
};

__host__ __device__ __forceinline__ uint64_t bits_below(int q) { return q >= 64 ? ~0ull : ((1ull << q) - 1); }
// bits lo .. hi inclusive
__host__ __device__ __forceinline__ uint64_t bit_range(int lo, int hi) { return bits_below(hi + 1) & ~bits_below(lo); }

// ---------------------------------------------------------------------------
// FP64 pose algebra (7-vectors t, q): composition and inverse.
__device__ void compose(const double* a, const double* b, double* out) {
  double Ra[9];
  dpba::quat_to_rot(a + 3, Ra);
  for (int i = 0; i < 3; ++i) out[i] = Ra[3 * i] * b[0] + Ra[3 * i + 1] * b[1] + Ra[3 * i + 2] * b[2] + a[i];
  const double ax = a[3], ay = a[4], az = a[5], aw = a[6];
  const double bx = b[3], by = b[4], bz = b[5], bw = b[6];
  double qx = aw * bx + bw * ax + (ay * bz - az * by);
  double qy = aw * by + bw * ay + (az * bx - ax * bz);
  double qz = aw * bz + bw * az + (ax * by - ay * bx);
  double qw = aw * bw - (ax * bx + ay * by + az * bz);
  const double n = sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  out[3] = qx / n;
  out[4] = qy / n;
  out[5] = qz / n;
  out[6] = qw / n;
}

__device__ void inverse(const double* a, double* out) {
  double R[9];
  dpba::quat_to_rot(a + 3, R);
  for (int i = 0; i < 3; ++i) out[i] = -(R[i] * a[0] + R[3 + i] * a[1] + R[6 + i] * a[2]);
  out[3] = -a[3];
  out[4] = -a[4];
  out[5] = -a[5];
  out[6] = a[6];
}

// Removes keyframe slot q of stream s (n keyframes): its row and bit column of
// the graph, then the slots after it move down by one.  All threads call.
__device__ void remove_slot(const State& st, int s, int q, int n) {
  const int t = threadIdx.x;
  uint64_t* adj = st.adj + (int64_t)s * st.N;
  double* pt = st.patches + (int64_t)s * st.P * 3;
  double* ps = st.poses + (int64_t)s * st.N * 7;
  int32_t* kid = st.kf_id + s * st.N;
  // rows, poses and ids: read everything first, then write
  uint64_t row = 0;
  double pv = 0.0;
  int id = -1;
  const uint64_t lo = bits_below(q);
  if (t < n && t != q) {
    const uint64_t x = adj[t];
    row = (x & lo) | ((x >> 1) & ~lo);
  }
  if (t < 7 * (n - 1 - q)) pv = ps[(q + 1) * 7 + t];
  if (t < n - 1 - q) id = kid[q + 1 + t];
  // patches of slots q+1 .. n-1, in chunks (the move goes down, so a chunk's
  // writes never reach a later chunk's reads)
  const int np = (n - 1 - q) * st.ppf * 3;
  constexpr int MAXV = 24;
  __syncthreads();
  if (t < n && t != q) adj[t < q ? t : t - 1] = row;
  if (t < 7 * (n - 1 - q)) ps[q * 7 + t] = pv;
  if (t < n - 1 - q) kid[q + t] = id;
  for (int base = 0; base < np; base += WG * MAXV) {
    double v[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const int i = base + k * WG + t;
      v[k] = i < np ? pt[(q + 1) * st.ppf * 3 + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const int i = base + k * WG + t;
      if (i < np) pt[q * st.ppf * 3 + i] = v[k];
    }
    __syncthreads();
  }
  __syncthreads();
  if (t == 0) {   // the freed slot: identity pose, no edges
    double* pose = ps + (n - 1) * 7;
    for (int i = 0; i < 7; ++i) pose[i] = i == 6 ? 1.0 : 0.0;
    kid[n - 1] = -1;
    adj[n - 1] = 0;
  }
  __syncthreads();
}

// Per-step outputs of every stream reset before the step.
__global__ void __launch_bounds__(256) k_vo_clear(State st) {
  for (int s = blockIdx.x * 256 + threadIdx.x; s < st.S; s += gridDim.x * 256) {
    st.vstatus[s] = 0;
    st.removed[s] = -1;
    st.removed_prev[s] = -1;
    st.retired[s] = -1;
    st.flow[s] = NAN;
  }
}

// Window advance and expansion of every active stream.
__global__ void __launch_bounds__(WG) k_vo_expand(State st, const double* new_xy, const double* init_poses,
                                                  const double* init_depth) {
  __shared__ double sortv[SORT_MAX];
  const int s = blockIdx.x, t = threadIdx.x;
  const int fid = st.active[s];
  if (fid < 0) return;
  int n = st.n_kf[s];
  if (n == st.N) {
    if (t < 7) st.retired_pose[s * 7 + t] = st.poses[(int64_t)s * st.N * 7 + t];
    if (t == 0) st.retired[s] = st.kf_id[s * st.N];
    remove_slot(st, s, 0, n);
    --n;
  }
  // new keyframe at slot n
  double* ps = st.poses + (int64_t)s * st.N * 7;
  uint64_t* adj = st.adj + (int64_t)s * st.N;
  const int q0 = max(0, n - st.r);
  if (t == 0) {
    double* pn = ps + n * 7;
    if (n < 2) {
      for (int i = 0; i < 7; ++i) pn[i] = init_poses[(s * 2 + n) * 7 + i];
    } else {
      double inv[7], vel[7];
      inverse(ps + (n - 2) * 7, inv);
      compose(ps + (n - 1) * 7, inv, vel);
      compose(vel, ps + (n - 1) * 7, pn);
    }
    st.kf_id[s * st.N + n] = fid;
  }
  // new edges: the patches of the last r keyframes to the new frame, the new
  // patches to keyframes n-r .. n
  if (t >= q0 && t < n) adj[t] |= 1ull << n;
  if (t == n) adj[n] = bit_range(q0, n);
  // median inverse depth of the previous three keyframes' patches
  double d0;
  if (n == 0) {
    d0 = init_depth[s];
  } else {
    const int p0 = max(0, n - 3);
    const int m = (n - p0) * st.ppf;
    int L = 1;
    while (L < m) L <<= 1;
    const double* pt = st.patches + (int64_t)s * st.P * 3;
    for (int i = t; i < L; i += WG) sortv[i] = i < m ? pt[(p0 * st.ppf + i) * 3 + 2] : DBL_MAX;
    __syncthreads();
    for (int k = 2; k <= L; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = t; i < L; i += WG) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const double a = sortv[i], b = sortv[ixj];
            const bool up = (i & k) == 0;
            if ((a > b) == up) {
              sortv[i] = b;
              sortv[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    d0 = (m & 1) ? sortv[m / 2] : 0.5 * (sortv[m / 2 - 1] + sortv[m / 2]);
  }
  double* pt = st.patches + (int64_t)s * st.P * 3;
  for (int i = t; i < st.ppf; i += WG) {
    double* p = pt + (n * st.ppf + i) * 3;
    p[0] = new_xy[((int64_t)s * st.ppf + i) * 2 + 0];
    p[1] = new_xy[((int64_t)s * st.ppf + i) * 2 + 1];
    p[2] = d0;
  }
  if (t == 0) st.n_kf[s] = n + 1;
}

// Bundle-adjustment arrays of every edge of the active streams: edge e of
// stream s is patch i of slot p with the c-th set bit of row p, for
// e = ppf * (edges of the rows before p) + i * popcount(row p) + c.
template <typename T>
__global__ void __launch_bounds__(256) k_vo_build(State st, int chunks) {
  __shared__ int rowoff[MAXN + 1];
  __shared__ int rowpop[MAXN];
  __shared__ int8_t bitpos[MAXN * MAXN];
  const int s = blockIdx.x / chunks;
  const int c = blockIdx.x % chunks;
  const int t = threadIdx.x;
  if (st.active[s] < 0) return;
  const int n = st.n_kf[s];
  const uint64_t* adj = st.adj + (int64_t)s * st.N;
  const int32_t* kid = st.kf_id + s * st.N;
  if (t < n) {
    uint64_t x = adj[t];
    rowpop[t] = __popcll(x);
    for (int k = 0; x; ++k, x &= x - 1) bitpos[t * MAXN + k] = (int8_t)__ffsll((long long)x) - 1;
  }
  __syncthreads();
  if (t == 0) {
    int o = 0;
    for (int p = 0; p < n; ++p) {
      rowoff[p] = o;
      o += st.ppf * rowpop[p];
    }
    rowoff[n] = o;
  }
  __syncthreads();
  // the window's poses and patches into the packed staging of the solve
  {
    const int a = st.cslot[s];
    const double* src = st.patches + (int64_t)s * st.P * 3;
    double* dst = st.c_patches + (int64_t)a * st.P * 3;
    for (int i = c * 256 + t; i < st.P * 3; i += chunks * 256) dst[i] = src[i];
    if (c == 0)
      for (int i = t; i < st.N * 7; i += 256) st.c_poses[(int64_t)a * st.N * 7 + i] = st.poses[(int64_t)s * st.N * 7 + i];
  }
  const int64_t e0 = st.e_off[s];
  const int ne = (int)(st.e_off[s + 1] - e0);
  if (ne != rowoff[n]) {   // the host's edge count disagrees with the graph
    if (c == 0 && t == 0) atomicOr(&st.vstatus[s], STATUS_COUNT);
  }
  const int nw = min(ne, rowoff[n]);
  T* tg = (T*)st.tgt + 2 * e0;
  T* wg = (T*)st.wgt + 2 * e0;
  int32_t* kk = st.kk + e0;
  int32_t* jj = st.jj + e0;
  const int R = st.R;
  const int64_t tab0 = st.tab_off[s];
  const int tabf = st.tab_frames[s];
  int bad = 0;
  for (int e = c * 256 + t; e < nw; e += chunks * 256) {
    int p = 0;
    while (p + 1 < n && rowoff[p + 1] <= e) ++p;
    const int local = e - rowoff[p], pc = rowpop[p];
    const int i = local / pc, q = bitpos[p * MAXN + local % pc];
    const int a = kid[p], f = kid[q];
    const int g = a * st.ppf + i;
    kk[e] = p * st.ppf + i;
    jj[e] = q;
    const int o = f - a + R;
    const bool ok = o >= 0 && o <= 2 * R && a < tabf && f < tabf;
    const int64_t row = (tab0 + g) * (2 * R + 1) + o;
    tg[2 * e] = ok ? (T)st.tab_t[2 * row] : T(0);
    tg[2 * e + 1] = ok ? (T)st.tab_t[2 * row + 1] : T(0);
    wg[2 * e] = ok ? (T)st.tab_w[2 * row] : T(0);
    wg[2 * e + 1] = ok ? (T)st.tab_w[2 * row + 1] : T(0);
    bad |= ok ? 0 : STATUS_TABLE;
  }
  if (bad) atomicOr(&st.vstatus[s], bad);
}

// Edges of the stream after its next expansion: the window advance drops slot
// 0's row and column, the expansion adds (n - q0) old rows' bits and a row of
// n - q0 + 1 bits.  Called by thread 0 with the stream's final state.
__device__ int next_edges(const State& st, int s) {
  const uint64_t* adj = st.adj + (int64_t)s * st.N;
  int n = st.n_kf[s];
  int bits = 0;
  for (int p = 0; p < n; ++p) bits += __popcll(adj[p]);
  if (n == st.N) {
    int col = 0;
    for (int p = 1; p < n; ++p) col += (int)(adj[p] & 1ull);
    bits -= __popcll(adj[0]) + col;
    --n;
  }
  const int q0 = max(0, n - st.r);
  bits += (n - q0) + (n - q0 + 1);
  return bits * st.ppf;
}

// Solved depths into the state, flow magnitude, keyframe removal.
__global__ void __launch_bounds__(WG) k_vo_keyframe(State st) {
  __shared__ double fsum[WG];
  __shared__ int fcnt[WG];
  const int s = blockIdx.x, t = threadIdx.x;
  if (st.active[s] < 0) return;
  const int n = st.n_kf[s];
  const int cs = st.cslot[s];
  double* pt = st.patches + (int64_t)s * st.P * 3;
  for (int i = t; i < n * st.ppf; i += WG) pt[i * 3 + 2] = st.depth_out[(int64_t)cs * st.P + i];
  for (int i = t; i < st.N * 7; i += WG) st.poses[(int64_t)s * st.N * 7 + i] = st.c_poses[(int64_t)cs * st.N * 7 + i];
  __syncthreads();
  double flow = NAN;
  int removed = -1;
  if (n >= 6) {
    const int a = n - 6, b = n - 4;
    const double* ps = st.poses + (int64_t)s * st.N * 7;
    double R[9], tv[3];
    dpba::relative_pose(ps + a * 7, ps + b * 7, R, tv);
    double sum = 0.0;
    int cnt = 0;
    for (int i = t; i < st.ppf; i += WG) {
      const double* p = pt + (a * st.ppf + i) * 3;
      const double x = (p[0] - st.cx) / st.fx, y = (p[1] - st.cy) / st.fy, d = p[2];
      const double X = R[0] * x + R[1] * y + R[2] + tv[0] * d;
      const double Y = R[3] * x + R[4] * y + R[5] + tv[1] * d;
      const double Z = R[6] * x + R[7] * y + R[8] + tv[2] * d;
      if (Z > st.z_min) {
        const double u = st.fx * X / Z + st.cx - p[0], v = st.fy * Y / Z + st.cy - p[1];
        sum += sqrt(u * u + v * v);
        ++cnt;
      }
    }
    fsum[t] = sum;
    fcnt[t] = cnt;
    __syncthreads();
    if (t == 0) {   // fixed order: patch by patch
      double tot = 0.0;
      int c = 0;
      for (int i = 0; i < min(WG, st.ppf); ++i) {
        tot += fsum[i];
        c += fcnt[i];
      }
      fsum[0] = c > 0 ? tot / c : INFINITY;
    }
    __syncthreads();
    flow = fsum[0];
    __syncthreads();
    if (flow < st.thresh) {
      const int q = n - 5;
      removed = st.kf_id[s * st.N + q];
      if (t == 0) {
        double inv[7];
        inverse(ps + (q - 1) * 7, inv);
        compose(ps + q * 7, inv, st.removed_rel + s * 7);
        st.removed_prev[s] = st.kf_id[s * st.N + q - 1];
      }
      remove_slot(st, s, q, n);
      if (t == 0) st.n_kf[s] = n - 1;
    }
  }
  __syncthreads();
  if (t == 0) {
    st.flow[s] = flow;
    st.removed[s] = removed;
    st.e_next[s] = next_edges(st, s);
  }
}

}  // namespace dpvo

using namespace dpvo;

struct vo_handle {
  vo_config cfg;
  State st;
  ba_handle* ba = nullptr;
  int64_t Ecap = 0;                 // edges of one window at most
  std::vector<int32_t> n_kf_host, e_next_host;
  std::vector<int64_t> frame_off, patch_off, edge_off;
  std::vector<int32_t> n_fixed, cslot;
  std::vector<int64_t> c_frame_off, c_patch_off, c_edge_off;
  std::vector<double> intr;
  int32_t* d_active = nullptr;
  int32_t* d_cslot = nullptr;
  int32_t* d_anchor = nullptr;     // [S][P] keyframe slot of every patch slot
  double* d_init_depth = nullptr;  // [S]
  int64_t* d_e_off = nullptr;      // [S+1]
  int64_t* d_tab_off = nullptr;
  int32_t* d_tab_frames = nullptr;
  bool sensor = false;
  std::vector<void*> allocs;
};

namespace {

int dmalloc(vo_handle* h, void** p, size_t bytes) {
  if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) return BA_E_HIP;
  h->allocs.push_back(*p);
  return BA_OK;
}

}  // namespace

extern "C" {

int vo_create(const vo_config* cfg, vo_handle** out) {
  if (!out) return BA_E_INVAL;
  *out = nullptr;
  if (!cfg) return BA_E_INVAL;
  const int maxw = cfg->precision == BA_PREC_FP64 ? 24 : MAXN;
  if (cfg->n_streams < 1 || cfg->window < 6 || cfg->window > maxw || cfg->patches_per_frame < 1 ||
      cfg->patches_per_frame > 256 || 3 * cfg->patches_per_frame > SORT_MAX || cfg->radius < 0 ||
      cfg->radius > 31 || cfg->radius >= cfg->window || cfg->n_free < 1 || cfg->iterations < 1 ||
      cfg->table_radius < cfg->radius || (cfg->precision != BA_PREC_FP32 && cfg->precision != BA_PREC_FP64) ||
      !(cfg->lambda >= 0.0))
    return BA_E_INVAL;
  vo_handle* h = new vo_handle();
  h->cfg = *cfg;
  const int S = cfg->n_streams, N = cfg->window, ppf = cfg->patches_per_frame;
  const int P = N * ppf;
  // a patch has at most 2 r + 1 edges: r + 1 when its frame arrives, and one
  // to each later frame added while its slot is within r of the newest
  h->Ecap = (int64_t)P * (2 * cfg->radius + 1);
  State& st = h->st;
  st.S = S;
  st.N = N;
  st.ppf = ppf;
  st.P = P;
  st.r = cfg->radius;
  st.n_free = cfg->n_free;
  st.R = cfg->table_radius;
  st.thresh = cfg->flow_thresh;
  st.z_min = cfg->z_min;
  st.fx = cfg->intrinsics[0];
  st.fy = cfg->intrinsics[1];
  st.cx = cfg->intrinsics[2];
  st.cy = cfg->intrinsics[3];
  const size_t esz = cfg->precision == BA_PREC_FP32 ? 4 : 8;
  const size_t E = (size_t)S * h->Ecap;
  int r = BA_OK;
  auto A = [&](void** p, size_t b) { if (r == BA_OK) r = dmalloc(h, p, b); };
  A((void**)&st.n_kf, 4 * S);
  A((void**)&st.kf_id, 4 * (size_t)S * N);
  A((void**)&st.poses, 8 * 7 * (size_t)S * N);
  A((void**)&st.patches, 8 * 3 * (size_t)S * P);
  A((void**)&st.adj, 8 * (size_t)S * N);
  A((void**)&st.e_next, 4 * S);
  A((void**)&st.kk, 4 * E);
  A((void**)&st.jj, 4 * E);
  A(&st.tgt, 2 * esz * E);
  A(&st.wgt, 2 * esz * E);
  A((void**)&st.depth_out, 8 * (size_t)S * P);
  A((void**)&st.c_poses, 8 * 7 * (size_t)S * N);
  A((void**)&st.c_patches, 8 * 3 * (size_t)S * P);
  A((void**)&h->d_cslot, 4 * S);
  A((void**)&st.flow, 8 * S);
  A((void**)&st.removed, 4 * S);
  A((void**)&st.removed_prev, 4 * S);
  A((void**)&st.removed_rel, 8 * 7 * S);
  A((void**)&st.retired, 4 * S);
  A((void**)&st.retired_pose, 8 * 7 * S);
  A((void**)&st.vstatus, 4 * S);
  A((void**)&h->d_active, 4 * S);
  A((void**)&h->d_e_off, 8 * (S + 1));
  A((void**)&h->d_tab_off, 8 * S);
  A((void**)&h->d_tab_frames, 4 * S);
  A((void**)&h->d_anchor, 4 * (size_t)S * P);
  A((void**)&h->d_init_depth, 8 * S);
  if (r != BA_OK) {
    vo_destroy(h);
    return r;
  }
  st.active = h->d_active;
  st.e_off = h->d_e_off;
  st.cslot = h->d_cslot;
  st.tab_off = h->d_tab_off;
  st.tab_frames = h->d_tab_frames;
  // empty windows: identity poses, unit inverse depths, no edges; the first
  // expansion adds the self-edges of the first frame's patches
  std::vector<double> poses((size_t)S * N * 7, 0.0), patches((size_t)S * P * 3, 0.0);
  for (size_t i = 0; i < (size_t)S * N; ++i) poses[i * 7 + 6] = 1.0;
  for (size_t i = 0; i < (size_t)S * P; ++i) patches[i * 3 + 2] = 1.0;
  std::vector<int32_t> ids((size_t)S * N, -1), zeros(S, 0), first(S, ppf), anchor((size_t)S * P);
  std::vector<uint64_t> rows((size_t)S * N, 0);
  for (size_t i = 0; i < anchor.size(); ++i) anchor[i] = (int32_t)((i % P) / ppf);
  bool ok = hipMemcpy(h->d_anchor, anchor.data(), 4 * anchor.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.poses, poses.data(), 8 * poses.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.patches, patches.data(), 8 * patches.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.kf_id, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.adj, rows.data(), 8 * rows.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.n_kf, zeros.data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.e_next, first.data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.removed, std::vector<int32_t>(S, -1).data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.removed_prev, std::vector<int32_t>(S, -1).data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.retired, std::vector<int32_t>(S, -1).data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.vstatus, zeros.data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess;
  std::vector<double> nan(S, NAN);
  ok = ok && hipMemcpy(st.flow, nan.data(), 8 * S, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    vo_destroy(h);
    return BA_E_HIP;
  }
  ba_config bc;
  memset(&bc, 0, sizeof(bc));
  bc.precision = cfg->precision;
  bc.iterations = cfg->iterations;
  bc.lambda = cfg->lambda;
  bc.z_min = cfg->z_min;
  bc.schedule = BA_SCHED_SPLIT;
  bc.max_windows = S;
  bc.max_frames_per_window = N;
  bc.chunk_frames = 0;
  bc.max_frames = (int64_t)S * N;
  bc.max_patches = (int64_t)S * P;
  bc.max_edges = (int64_t)E;
  r = ba_create(&bc, &h->ba);
  if (r != BA_OK) {
    vo_destroy(h);
    return r;
  }
  h->n_kf_host.assign(S, 0);
  h->e_next_host.assign(S, ppf);
  h->frame_off.resize(S + 1);
  h->patch_off.resize(S + 1);
  h->edge_off.assign(S + 1, 0);
  for (int s = 0; s <= S; ++s) {
    h->frame_off[s] = (int64_t)s * N;
    h->patch_off[s] = (int64_t)s * P;
  }
  h->n_fixed.assign(S, 0);
  h->cslot.assign(S, -1);
  h->c_frame_off.assign(S + 1, 0);
  h->c_patch_off.assign(S + 1, 0);
  h->c_edge_off.assign(S + 1, 0);
  h->intr.resize(4 * S);
  for (int s = 0; s < S; ++s)
    for (int i = 0; i < 4; ++i) h->intr[4 * s + i] = cfg->intrinsics[i];
  *out = h;
  return BA_OK;
}

int vo_set_sensor(vo_handle* h, const double* targets, const double* weights, const int64_t* table_off,
                  const int32_t* table_frames) {
  if (!h || !targets || !weights || !table_off || !table_frames) return BA_E_INVAL;
  const int S = h->cfg.n_streams;
  for (int s = 0; s < S; ++s)
    if (table_off[s] < 0 || table_frames[s] < 0) return BA_E_INVAL;
  if (hipMemcpy(h->d_tab_off, table_off, 8 * S, hipMemcpyHostToDevice) != hipSuccess) return BA_E_HIP;
  if (hipMemcpy(h->d_tab_frames, table_frames, 4 * S, hipMemcpyHostToDevice) != hipSuccess) return BA_E_HIP;
  h->st.tab_t = targets;
  h->st.tab_w = weights;
  h->sensor = true;
  return BA_OK;
}

int vo_step(vo_handle* h, const int32_t* frame_id, const double* new_xy, const double* init_poses,
            const double* init_depth, void* stream) {
  if (!h || !frame_id || !new_xy || !init_poses || !init_depth) return BA_E_INVAL;
  if (!h->sensor) return BA_E_STATE;
  const int S = h->cfg.n_streams, N = h->cfg.window;
  hipStream_t s = (hipStream_t)stream;
  State& st = h->st;
  // keyframes and edges after the expansion, known on the host from the last
  // step's read-back.  Only the streams with a new frame enter the solve,
  // their windows packed in stream order; idle streams keep their state.
  int na = 0;
  for (int i = 0; i < S; ++i) {
    const bool on = frame_id[i] >= 0;
    if (on && (h->e_next_host[i] < 0 || h->e_next_host[i] > h->Ecap)) return BA_E_STATE;
    h->edge_off[i + 1] = h->edge_off[i] + (on ? h->e_next_host[i] : 0);
    h->cslot[i] = on ? na : -1;
    if (on) {
      const int n = std::min(h->n_kf_host[i] + 1, N);
      h->n_fixed[na] = std::max(std::min(2, n), n - h->cfg.n_free);
      h->c_frame_off[na + 1] = (int64_t)(na + 1) * N;
      h->c_patch_off[na + 1] = (int64_t)(na + 1) * st.P;
      h->c_edge_off[na + 1] = h->edge_off[i + 1];
      ++na;
    }
  }
  // the host arrays are read before this call returns (it waits for the step)
  if (hipMemcpyAsync(h->d_active, frame_id, 4 * S, hipMemcpyHostToDevice, s) != hipSuccess) return BA_E_HIP;
  if (hipMemcpyAsync(h->d_init_depth, init_depth, 8 * S, hipMemcpyHostToDevice, s) != hipSuccess) return BA_E_HIP;
  if (hipMemcpyAsync(h->d_e_off, h->edge_off.data(), 8 * (S + 1), hipMemcpyHostToDevice, s) != hipSuccess)
    return BA_E_HIP;
  if (hipMemcpyAsync(h->d_cslot, h->cslot.data(), 4 * S, hipMemcpyHostToDevice, s) != hipSuccess) return BA_E_HIP;
  hipLaunchKernelGGL(k_vo_clear, dim3((S + 255) / 256), dim3(256), 0, s, st);
  if (na == 0) {
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return BA_E_HIP;
    return BA_OK;
  }
  hipLaunchKernelGGL(k_vo_expand, dim3(S), dim3(WG), 0, s, st, new_xy, init_poses, (const double*)h->d_init_depth);
  const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(64, (h->Ecap + 4095) / 4096));
  if (h->cfg.precision == BA_PREC_FP32)
    hipLaunchKernelGGL(k_vo_build<float>, dim3(S * chunks), dim3(256), 0, s, st, chunks);
  else
    hipLaunchKernelGGL(k_vo_build<double>, dim3(S * chunks), dim3(256), 0, s, st, chunks);
  if (hipGetLastError() != hipSuccess) return BA_E_HIP;
  ba_problem p;
  memset(&p, 0, sizeof(p));
  p.n_windows = na;
  p.frame_off = h->c_frame_off.data();
  p.patch_off = h->c_patch_off.data();
  p.edge_off = h->c_edge_off.data();
  p.n_fixed = h->n_fixed.data();
  p.intrinsics = h->intr.data();
  p.poses_in = st.c_poses;
  p.patches_in = st.c_patches;
  p.anchor = h->d_anchor;
  p.kk = st.kk;
  p.jj = st.jj;
  p.targets = st.tgt;
  p.weights = st.wgt;
  p.poses_out = st.c_poses;      // in place in the staging, copied back by k_vo_keyframe
  p.depth_out = st.depth_out;
  int rc = ba_solve(h->ba, &p, stream);
  if (rc != BA_OK) return rc;
  hipLaunchKernelGGL(k_vo_keyframe, dim3(S), dim3(WG), 0, s, st);
  if (hipGetLastError() != hipSuccess) return BA_E_HIP;
  if (hipMemcpyAsync(h->n_kf_host.data(), st.n_kf, 4 * S, hipMemcpyDeviceToHost, s) != hipSuccess) return BA_E_HIP;
  if (hipMemcpyAsync(h->e_next_host.data(), st.e_next, 4 * S, hipMemcpyDeviceToHost, s) != hipSuccess)
    return BA_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return BA_E_HIP;
  return BA_OK;
}

int vo_read(vo_handle* h, int32_t* n_kf, int32_t* kf_id, double* flow, int32_t* removed) {
  if (!h) return BA_E_INVAL;
  const int S = h->cfg.n_streams, N = h->cfg.window;
  State& st = h->st;
  if (n_kf && hipMemcpy(n_kf, st.n_kf, 4 * S, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  if (kf_id && hipMemcpy(kf_id, st.kf_id, 4 * (size_t)S * N, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  if (flow && hipMemcpy(flow, st.flow, 8 * S, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  if (removed && hipMemcpy(removed, st.removed, 4 * S, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  return BA_OK;
}

int vo_read_events(vo_handle* h, int32_t* retired, double* retired_pose, int32_t* removed, int32_t* removed_prev,
                   double* removed_rel) {
  if (!h) return BA_E_INVAL;
  const int S = h->cfg.n_streams;
  State& st = h->st;
  if (retired && hipMemcpy(retired, st.retired, 4 * S, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  if (retired_pose && hipMemcpy(retired_pose, st.retired_pose, 8 * 7 * S, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  if (removed && hipMemcpy(removed, st.removed, 4 * S, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  if (removed_prev && hipMemcpy(removed_prev, st.removed_prev, 4 * S, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  if (removed_rel && hipMemcpy(removed_rel, st.removed_rel, 8 * 7 * S, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  return BA_OK;
}

int vo_read_window(vo_handle* h, int32_t s, double* poses, double* depth, int32_t* edge_patch, int32_t* edge_frame,
                   int64_t* n_edges) {
  if (!h || s < 0 || s >= h->cfg.n_streams) return BA_E_INVAL;
  State& st = h->st;
  const int N = st.N, P = st.P, ppf = st.ppf;
  if (poses && hipMemcpy(poses, st.poses + (int64_t)s * N * 7, 8 * 7 * N, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  if (depth) {
    std::vector<double> pt((size_t)P * 3);
    if (hipMemcpy(pt.data(), st.patches + (int64_t)s * P * 3, 8 * pt.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return BA_E_HIP;
    for (int i = 0; i < P; ++i) depth[i] = pt[3 * i + 2];
  }
  int32_t n = 0;
  std::vector<uint64_t> rows(N);
  std::vector<int32_t> ids(N);
  if (hipMemcpy(&n, st.n_kf + s, 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(rows.data(), st.adj + (int64_t)s * N, 8 * N, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(ids.data(), st.kf_id + (int64_t)s * N, 4 * N, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  // (patch id, frame id) of every edge, in (slot, patch, target slot) order
  int64_t ne = 0;
  for (int p = 0; p < n; ++p) {
    for (int i = 0; i < ppf; ++i) {
      for (int q = 0; q < n; ++q) {
        if (!((rows[p] >> q) & 1ull)) continue;
        if (edge_patch) edge_patch[ne] = ids[p] * ppf + i;
        if (edge_frame) edge_frame[ne] = ids[q];
        ++ne;
      }
    }
  }
  if (n_edges) *n_edges = ne;
  return BA_OK;
}

int vo_status(vo_handle* h, int32_t* flags) {
  if (!h || !flags) return BA_E_INVAL;
  const int S = h->cfg.n_streams;
  // the last solve's windows are the streams that had a new frame, packed
  std::vector<int32_t> ba(S, 0), vs(S);
  if (std::any_of(h->cslot.begin(), h->cslot.end(), [](int32_t c) { return c >= 0; }) &&
      ba_status(h->ba, ba.data()) != BA_OK)
    return BA_E_HIP;
  if (hipMemcpy(vs.data(), h->st.vstatus, 4 * S, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  for (int s = 0; s < S; ++s) flags[s] = (h->cslot[s] >= 0 ? ba[h->cslot[s]] : 0) | vs[s];
  return BA_OK;
}

void vo_destroy(vo_handle* h) {
  if (!h) return;
  hipDeviceSynchronize();
  if (h->ba) ba_destroy(h->ba);
  for (void* p : h->allocs) hipFree(p);
  delete h;
}

}  // extern "C"
