// Sliding-window driver (include/dpvo.h) on gfx950: the per-frame rules of
// Sec. 3.3 "VO System" applied on the device to many camera streams at once,
// around the batched bundle adjustment of include/dpba.h.
//
// Per vo_step:
//   k_vo_expand   (one workgroup per stream): window advance, constant-
//                 velocity pose, median depth of the new patches, new edges;
//   k_vo_build    (many workgroups per stream): the bundle-adjustment arrays
//                 of every edge slot (window-local indices, sensor lookups,
//                 placeholder self-edges in the unused slots);
//   ba_solve      over all streams' windows, in place on the state buffers;
//   k_vo_keyframe (one workgroup per stream): the solved depths into the
//                 state, the flow magnitude between keyframes t-5 and t-3, and
//                 the removal of keyframe t-4.
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
constexpr int STATUS_TABLE = 1 << 16;

struct State {
  int S, N, ppf, P, Ecap, r, n_free, R;
  double thresh, z_min, fx, fy, cx, cy;
  int32_t* n_kf;        // [S]
  int32_t* kf_id;       // [S][N]
  double* poses;        // [S][N][7]
  double* patches;      // [S][P][3]  x, y, inverse depth
  int32_t* e_g;         // [S][Ecap]  patch id (frame * ppf + i)
  int32_t* e_f;         // [S][Ecap]  frame id
  int32_t* e_g2;        // [S][Ecap]  compaction scratch
  int32_t* e_f2;
  int32_t* n_e;         // [S]
  int32_t* kk;          // [S][Ecap]  bundle-adjustment arrays
  int32_t* jj;
  void* tgt;            // [S][Ecap][2] f32 or f64
  void* wgt;
  double* depth_out;    // [S][P]
  double* flow;         // [S]
  int32_t* removed;     // [S]
  int32_t* vstatus;     // [S]
  int32_t* active;      // [S] this step's frame id (-1 idle)
  const double* tab_t;  // sensor
  const double* tab_w;
  const int64_t* tab_off;   // [S] device copy
  const int32_t* tab_frames;
};

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

__device__ __forceinline__ void set_placeholder(const State& st, int s, int p) {
  double* pose = st.poses + ((int64_t)s * st.N + p) * 7;
  for (int i = 0; i < 7; ++i) pose[i] = i == 6 ? 1.0 : 0.0;
  st.kf_id[s * st.N + p] = -1;
}

// Workgroup exclusive scan of one int per thread; returns the total.
__device__ int wg_scan(int v, int* lds, int* out_excl) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int o = 1; o < WG; o <<= 1) {
    const int x = t >= o ? lds[t - o] : 0;
    __syncthreads();
    lds[t] += x;
    __syncthreads();
  }
  *out_excl = lds[t] - v;
  const int total = lds[WG - 1];
  __syncthreads();
  return total;
}

// Removes keyframe slot q of stream s (n keyframes): its edges and those of
// its patches, then the slots after it move down by one.  All threads call.
__device__ void remove_slot(const State& st, int s, int q, int n, int* lds) {
  const int t = threadIdx.x;
  const int fid = st.kf_id[s * st.N + q];
  // edges: order-preserving compaction through the scratch arrays
  const int ne = st.n_e[s];
  const int per = (ne + WG - 1) / WG;
  const int lo = min(ne, t * per), hi = min(ne, lo + per);
  int32_t* eg = st.e_g + (int64_t)s * st.Ecap;
  int32_t* ef = st.e_f + (int64_t)s * st.Ecap;
  int32_t* eg2 = st.e_g2 + (int64_t)s * st.Ecap;
  int32_t* ef2 = st.e_f2 + (int64_t)s * st.Ecap;
  int keep = 0;
  for (int e = lo; e < hi; ++e) keep += (ef[e] != fid && eg[e] / st.ppf != fid) ? 1 : 0;
  int off;
  const int total = wg_scan(keep, lds, &off);
  for (int e = lo; e < hi; ++e) {
    if (ef[e] != fid && eg[e] / st.ppf != fid) {
      eg2[off] = eg[e];
      ef2[off] = ef[e];
      ++off;
    }
  }
  __syncthreads();
  for (int e = t; e < total; e += WG) {
    eg[e] = eg2[e];
    ef[e] = ef2[e];
  }
  // slots q+1 .. n-1 move down: read everything first, then write
  const int np = (n - 1 - q) * st.ppf * 3;       // patch doubles to move
  const int nq = (n - 1 - q) * 7;                // pose doubles
  double* pt = st.patches + (int64_t)s * st.P * 3;
  double* ps = st.poses + (int64_t)s * st.N * 7;
  constexpr int MAXV = 24;                        // (64 slots * 256 patches * 3) / 1024 < 49; chunked below
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
  {
    double v = t < nq ? ps[(q + 1) * 7 + t] : 0.0;
    const int id = t < n - 1 - q ? st.kf_id[s * st.N + q + 1 + t] : -1;
    __syncthreads();
    if (t < nq) ps[q * 7 + t] = v;
    if (t < n - 1 - q) st.kf_id[s * st.N + q + t] = id;
  }
  __syncthreads();
  if (t == 0) {
    st.n_e[s] = total;
    set_placeholder(st, s, n - 1);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_vo_clear(int32_t* a, int n) {
  for (int i = threadIdx.x; i < n; i += 256) a[i] = 0;
}

// Window advance and expansion of every active stream.
__global__ void __launch_bounds__(WG) k_vo_expand(State st, const double* new_xy, const double* init_poses,
                                                  const double* init_depth) {
  __shared__ int lds[WG];
  __shared__ double sortv[SORT_MAX];
  const int s = blockIdx.x, t = threadIdx.x;
  const int fid = st.active[s];
  if (fid < 0) return;
  int n = st.n_kf[s];
  if (n == st.N) {
    remove_slot(st, s, 0, n, lds);
    --n;
  }
  // new keyframe at slot n
  double* ps = st.poses + (int64_t)s * st.N * 7;
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
  // new edges: patches of the last r keyframes -> the new frame, then the
  // new patches -> keyframes n-r .. n
  const int ne = st.n_e[s];
  const int q0 = max(0, n - st.r);
  const int nold = (n - q0) * st.ppf;
  const int nnew = (n - q0 + 1) * st.ppf;
  int32_t* eg = st.e_g + (int64_t)s * st.Ecap;
  int32_t* ef = st.e_f + (int64_t)s * st.Ecap;
  const int32_t* kid = st.kf_id + s * st.N;
  for (int i = t; i < nold + nnew; i += WG) {
    int g, f;
    if (i < nold) {
      const int p = q0 + i / st.ppf;
      g = kid[p] * st.ppf + i % st.ppf;
      f = fid;
    } else {
      const int k = i - nold;
      const int q = q0 + k / st.ppf;
      g = fid * st.ppf + k % st.ppf;
      f = q == n ? fid : kid[q];
    }
    eg[ne + i] = g;
    ef[ne + i] = f;
  }
  __syncthreads();
  if (t == 0) {
    st.n_e[s] = ne + nold + nnew;
    st.n_kf[s] = n + 1;
  }
}

// Bundle-adjustment arrays of every edge slot.
template <typename T>
__global__ void __launch_bounds__(256) k_vo_build(State st, int chunks) {
  const int s = blockIdx.x / chunks;
  const int c = blockIdx.x % chunks;
  const int ne = st.active[s] >= 0 ? st.n_e[s] : 0;   // idle streams: placeholders only
  const int n = st.n_kf[s];
  const int32_t* kid = st.kf_id + s * st.N;
  T* tg = (T*)st.tgt + (int64_t)s * st.Ecap * 2;
  T* wg = (T*)st.wgt + (int64_t)s * st.Ecap * 2;
  int32_t* kk = st.kk + (int64_t)s * st.Ecap;
  int32_t* jj = st.jj + (int64_t)s * st.Ecap;
  const int R = st.R;
  int bad = 0;
  for (int e = c * 256 + threadIdx.x; e < st.Ecap; e += chunks * 256) {
    if (e < ne) {
      const int g = st.e_g[(int64_t)s * st.Ecap + e], f = st.e_f[(int64_t)s * st.Ecap + e];
      const int a = g / st.ppf;
      int pa = 0, pf = 0;
      for (int p = 0; p < n; ++p) {
        if (kid[p] == a) pa = p;
        if (kid[p] == f) pf = p;
      }
      kk[e] = pa * st.ppf + g % st.ppf;
      jj[e] = pf;
      const int o = f - a + R;
      const bool ok = o >= 0 && o <= 2 * R && g < st.tab_frames[s] * st.ppf && f < st.tab_frames[s];
      const int64_t row = (st.tab_off[s] + g) * (2 * R + 1) + o;
      tg[2 * e] = ok ? (T)st.tab_t[2 * row] : T(0);
      tg[2 * e + 1] = ok ? (T)st.tab_t[2 * row + 1] : T(0);
      wg[2 * e] = ok ? (T)st.tab_w[2 * row] : T(0);
      wg[2 * e + 1] = ok ? (T)st.tab_w[2 * row + 1] : T(0);
      bad |= ok ? 0 : STATUS_TABLE;
    } else {
      // a self-edge of patch e % P: contributes exactly nothing
      const int k = e % st.P;
      kk[e] = k;
      jj[e] = k / st.ppf;
      tg[2 * e] = tg[2 * e + 1] = T(0);
      wg[2 * e] = wg[2 * e + 1] = T(0);
    }
  }
  if (bad) atomicOr(&st.vstatus[s], bad);
}

// Solved depths into the state, flow magnitude, keyframe removal.
__global__ void __launch_bounds__(WG) k_vo_keyframe(State st) {
  __shared__ int lds[WG];
  __shared__ double fsum[WG];
  __shared__ int fcnt[WG];
  const int s = blockIdx.x, t = threadIdx.x;
  if (st.active[s] < 0) return;
  const int n = st.n_kf[s];
  double* pt = st.patches + (int64_t)s * st.P * 3;
  for (int i = t; i < n * st.ppf; i += WG) pt[i * 3 + 2] = st.depth_out[(int64_t)s * st.P + i];
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
      lds[0] = c;
      fsum[0] = c > 0 ? tot / c : INFINITY;
    }
    __syncthreads();
    flow = fsum[0];
    __syncthreads();
    if (flow < st.thresh) {
      removed = st.kf_id[s * st.N + n - 5];
      remove_slot(st, s, n - 5, n, lds);
      if (t == 0) st.n_kf[s] = n - 1;
    }
  }
  if (t == 0) {
    st.flow[s] = flow;
    st.removed[s] = removed;
  }
}

}  // namespace dpvo

using namespace dpvo;

struct vo_handle {
  vo_config cfg;
  State st;
  ba_handle* ba = nullptr;
  std::vector<int32_t> n_kf_host;
  std::vector<int64_t> frame_off, patch_off, edge_off;
  std::vector<int32_t> n_fixed;
  std::vector<double> intr;
  int32_t* d_active = nullptr;
  int32_t* d_anchor = nullptr;     // [S][P] keyframe slot of every patch slot
  double* d_init_depth = nullptr;  // [S]
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
  const int maxw = cfg->precision == BA_PREC_FP64 ? 24 : 64;
  if (cfg->n_streams < 1 || cfg->window < 6 || cfg->window > maxw || cfg->patches_per_frame < 1 ||
      cfg->patches_per_frame > 256 || 3 * cfg->patches_per_frame > SORT_MAX || cfg->radius < 0 ||
      cfg->radius > 15 || cfg->radius >= cfg->window || cfg->n_free < 1 || cfg->iterations < 1 || cfg->table_radius < cfg->radius ||
      (cfg->precision != BA_PREC_FP32 && cfg->precision != BA_PREC_FP64) || !(cfg->lambda >= 0.0))
    return BA_E_INVAL;
  vo_handle* h = new vo_handle();
  h->cfg = *cfg;
  const int S = cfg->n_streams, N = cfg->window, ppf = cfg->patches_per_frame;
  const int P = N * ppf;
  const int Ecap = P * (2 * cfg->radius + 1);
  State& st = h->st;
  st.S = S;
  st.N = N;
  st.ppf = ppf;
  st.P = P;
  st.Ecap = Ecap;
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
  int r = BA_OK;
  auto A = [&](void** p, size_t b) { if (r == BA_OK) r = dmalloc(h, p, b); };
  A((void**)&st.n_kf, 4 * S);
  A((void**)&st.kf_id, 4 * (size_t)S * N);
  A((void**)&st.poses, 8 * 7 * (size_t)S * N);
  A((void**)&st.patches, 8 * 3 * (size_t)S * P);
  A((void**)&st.e_g, 4 * (size_t)S * Ecap);
  A((void**)&st.e_f, 4 * (size_t)S * Ecap);
  A((void**)&st.e_g2, 4 * (size_t)S * Ecap);
  A((void**)&st.e_f2, 4 * (size_t)S * Ecap);
  A((void**)&st.n_e, 4 * S);
  A((void**)&st.kk, 4 * (size_t)S * Ecap);
  A((void**)&st.jj, 4 * (size_t)S * Ecap);
  A(&st.tgt, 2 * esz * (size_t)S * Ecap);
  A(&st.wgt, 2 * esz * (size_t)S * Ecap);
  A((void**)&st.depth_out, 8 * (size_t)S * P);
  A((void**)&st.flow, 8 * S);
  A((void**)&st.removed, 4 * S);
  A((void**)&st.vstatus, 4 * S);
  A((void**)&h->d_active, 4 * S);
  A((void**)&h->d_tab_off, 8 * S);
  A((void**)&h->d_tab_frames, 4 * S);
  A((void**)&h->d_anchor, 4 * (size_t)S * P);
  A((void**)&h->d_init_depth, 8 * S);
  if (r != BA_OK) {
    vo_destroy(h);
    return r;
  }
  st.active = h->d_active;
  st.tab_off = h->d_tab_off;
  st.tab_frames = h->d_tab_frames;
  // empty windows: placeholder poses and patches, no edges
  std::vector<double> poses((size_t)S * N * 7, 0.0), patches((size_t)S * P * 3, 0.0);
  for (size_t i = 0; i < (size_t)S * N; ++i) poses[i * 7 + 6] = 1.0;
  for (size_t i = 0; i < (size_t)S * P; ++i) patches[i * 3 + 2] = 1.0;
  std::vector<int32_t> ids((size_t)S * N, -1), zeros(S, 0), anchor((size_t)S * P);
  for (size_t i = 0; i < anchor.size(); ++i) anchor[i] = (int32_t)((i % P) / ppf);
  bool ok = hipMemcpy(h->d_anchor, anchor.data(), 4 * anchor.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.poses, poses.data(), 8 * poses.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.patches, patches.data(), 8 * patches.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.kf_id, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.n_kf, zeros.data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(st.n_e, zeros.data(), 4 * S, hipMemcpyHostToDevice) == hipSuccess;
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
  bc.max_edges = (int64_t)S * Ecap;
  r = ba_create(&bc, &h->ba);
  if (r != BA_OK) {
    vo_destroy(h);
    return r;
  }
  h->n_kf_host.assign(S, 0);
  h->frame_off.resize(S + 1);
  h->patch_off.resize(S + 1);
  h->edge_off.resize(S + 1);
  for (int s = 0; s <= S; ++s) {
    h->frame_off[s] = (int64_t)s * N;
    h->patch_off[s] = (int64_t)s * P;
    h->edge_off[s] = (int64_t)s * Ecap;
  }
  h->n_fixed.assign(S, 0);
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
  // the host arrays are read before this call returns (it waits for the step)
  if (hipMemcpyAsync(h->d_active, frame_id, 4 * S, hipMemcpyHostToDevice, s) != hipSuccess) return BA_E_HIP;
  if (hipMemcpyAsync(h->d_init_depth, init_depth, 8 * S, hipMemcpyHostToDevice, s) != hipSuccess) return BA_E_HIP;
  hipLaunchKernelGGL(k_vo_clear, dim3(1), dim3(256), 0, s, st.vstatus, S);
  hipLaunchKernelGGL(k_vo_expand, dim3(S), dim3(WG), 0, s, st, new_xy, init_poses, (const double*)h->d_init_depth);
  const int chunks = std::max(1, std::min(64, (st.Ecap + 4095) / 4096));
  if (h->cfg.precision == BA_PREC_FP32)
    hipLaunchKernelGGL(k_vo_build<float>, dim3(S * chunks), dim3(256), 0, s, st, chunks);
  else
    hipLaunchKernelGGL(k_vo_build<double>, dim3(S * chunks), dim3(256), 0, s, st, chunks);
  if (hipGetLastError() != hipSuccess) return BA_E_HIP;
  // keyframes after the expansion (known on the host: the window grows by
  // one up to its capacity); idle streams keep every pose fixed
  for (int i = 0; i < S; ++i) {
    const int n = frame_id[i] >= 0 ? std::min(h->n_kf_host[i] + 1, N) : h->n_kf_host[i];
    h->n_fixed[i] = frame_id[i] >= 0 ? std::max(std::min(2, n), n - h->cfg.n_free) : N;
  }
  ba_problem p;
  memset(&p, 0, sizeof(p));
  p.n_windows = S;
  p.frame_off = h->frame_off.data();
  p.patch_off = h->patch_off.data();
  p.edge_off = h->edge_off.data();
  p.n_fixed = h->n_fixed.data();
  p.intrinsics = h->intr.data();
  p.poses_in = st.poses;
  p.patches_in = st.patches;
  p.anchor = h->d_anchor;
  p.kk = st.kk;
  p.jj = st.jj;
  p.targets = st.tgt;
  p.weights = st.wgt;
  p.poses_out = st.poses;        // in place: the window's poses are the state
  p.depth_out = st.depth_out;
  int rc = ba_solve(h->ba, &p, stream);
  if (rc != BA_OK) return rc;
  hipLaunchKernelGGL(k_vo_keyframe, dim3(S), dim3(WG), 0, s, st);
  if (hipGetLastError() != hipSuccess) return BA_E_HIP;
  if (hipMemcpyAsync(h->n_kf_host.data(), st.n_kf, 4 * S, hipMemcpyDeviceToHost, s) != hipSuccess) return BA_E_HIP;
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

int vo_read_window(vo_handle* h, int32_t s, double* poses, double* depth, int32_t* edge_patch, int32_t* edge_frame,
                   int64_t* n_edges) {
  if (!h || s < 0 || s >= h->cfg.n_streams) return BA_E_INVAL;
  State& st = h->st;
  const int N = st.N, P = st.P;
  if (poses && hipMemcpy(poses, st.poses + (int64_t)s * N * 7, 8 * 7 * N, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  if (depth) {
    std::vector<double> pt((size_t)P * 3);
    if (hipMemcpy(pt.data(), st.patches + (int64_t)s * P * 3, 8 * pt.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return BA_E_HIP;
    for (int i = 0; i < P; ++i) depth[i] = pt[3 * i + 2];
  }
  int32_t ne = 0;
  if (hipMemcpy(&ne, st.n_e + s, 4, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  if (n_edges) *n_edges = ne;
  if (edge_patch && hipMemcpy(edge_patch, st.e_g + (int64_t)s * st.Ecap, 4 * (size_t)ne, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  if (edge_frame && hipMemcpy(edge_frame, st.e_f + (int64_t)s * st.Ecap, 4 * (size_t)ne, hipMemcpyDeviceToHost) != hipSuccess)
    return BA_E_HIP;
  return BA_OK;
}

int vo_status(vo_handle* h, int32_t* flags) {
  if (!h || !flags) return BA_E_INVAL;
  const int S = h->cfg.n_streams;
  std::vector<int32_t> ba(S), vs(S);
  if (ba_status(h->ba, ba.data()) != BA_OK) return BA_E_HIP;
  if (hipMemcpy(vs.data(), h->st.vstatus, 4 * S, hipMemcpyDeviceToHost) != hipSuccess) return BA_E_HIP;
  for (int s = 0; s < S; ++s) flags[s] = ba[s] | vs[s];
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
