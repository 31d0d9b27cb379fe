// Edge linearisation and assembly of the depth-eliminated pose system.
//
// Objective (Sec. 3.1, Eq. 6): sum over edges e = (k, j), patch k anchored in
// frame i, of w_x r_x^2 + w_y r_y^2 with r = pi(p) - target, where
//   p = R_ji (xbar, ybar, 1) + t_ji d_k           (Eq. 2 on (x, y, 1, d), K of Eq. 3)
//   pi(p) = (fx X / Z + cx, fy Y / Z + cy)       (divide by the third element)
// Per edge, with Pi = d pi / d p and left perturbations of T_i, T_j:
//   J_j = Pi [d I | -hat(p)],  J_i = -J_j Ad(T_ji),  J_d = Pi t_ji.
// Damped normal equations over (free poses, depths) eliminate every depth by
// the Schur complement (Sec. 3.1): with C_k = lambda + sum_e J_d^T W J_d,
// w_k = sum_e J_d^T W r and E_ak = sum_e J_a^T W J_d,
//   S = B + lambda I - sum_k E_k E_k^T / C_k,   s = v - sum_k E_k w_k / C_k,
// where B, v collect J_a^T W J_b and J_a^T W r over all edges.
//
// One workgroup handles one chunk: a run of consecutive source frames of one
// window, and writes the chunk's share of S and s (lower triangle, dense over
// the free frames its patches touch) to a partial buffer that the Cholesky
// stage sums in a fixed order.  Within the chunk:
//   * patches are taken in sub-batches of SB; each patch is a lane segment of
//     the wave (one lane per edge), segment sums give C_k, w_k, E_ik;
//   * the scaled row u_k = (E_k, w_k) / sqrt(C_k) of every patch is staged in
//     LDS (column-major, dof x patch) and the outer products sum_k u_k u_k^T
//     are accumulated with 16x16x4 matrix-core instructions into register
//     tiles of the lower triangle;
//   * B and v are gathered per (source frame i, target frame j) pair as
//     Q_ij = sum_k J_j^T W J_j and V_ij = sum_k J_j^T W r (per-wave LDS tables,
//     summed in wave order), then mapped to the (i,i), (i,j), (j,j) blocks
//     through A = Ad(T_ji): B_jj += Q, B_ij -= A^T Q, B_ii += A^T Q A,
//     v_j += V, v_i -= A^T V.
#pragma once
#include "dpba_common.h"
#include "dpba_prep.h"

namespace dpba {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T> struct AccT;
template <> struct AccT<float> { typedef f32x4 type; };
template <> struct AccT<double> { typedef f64x4 type; };

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of the 16x16 result held in accumulator register r of a lane in lane
// group g = lane / 16 (the column is lane % 16).  The f32 16x16x4 product
// keeps four consecutive rows per lane group, the f64 product interleaves them.
__device__ __forceinline__ int acc_row(float, int g, int r) { return 4 * g + r; }
__device__ __forceinline__ int acc_row(double, int g, int r) { return 4 * r + g; }
// Slot of the tile element (row, col) in the entry image of the tile pass
// that starts at lower-triangle tile p0 and holds Lp tiles; -1 outside it.
__device__ __forceinline__ int img_slot(int row, int col, int p0, int Lp) {
  const int ti = row >> 4, tj = col >> 4;
  const int t = ((ti * (ti + 1)) >> 1) + tj - p0;
  if (t < 0 || t >= Lp) return -1;
  const int r16 = row & 15;   // FP32 accumulator rows: 4 * (lane / 16) + element
  return t * 256 + (16 * (r16 >> 2) + (col & 15)) * 4 + (r16 & 3);
}
// (m, n), m <= n, of the packed upper-triangle index e of a 6x6 block
__device__ __forceinline__ void unsym6(int e, int& m, int& n) {
  m = (e >= 6) + (e >= 11) + (e >= 15) + (e >= 18) + (e >= 20);
  n = e - (m * 6 - (m * (m - 1)) / 2) + m;
}

constexpr int SBMAX = 32;       // patches per sub-batch (K block of the Schur product)
constexpr int SBE = 1024;       // staged edges per sub-batch (SB x lane segment width)
constexpr int LDK = SBMAX + 4;  // LDS row length of the staged u rows
constexpr int RELW = 25;        // LDS words per relative pose: R(9) t(3) hat(t)R(9); odd stride, no bank conflicts

// LDS layout of the assembly and back-substitution stages, in bytes, for
// windows of at most Rcap frames.  Shared with the host to size the launch.
struct AsmLayout {
  int poses, rel, tbl, G, U, tiles, arng, stage, img, misc, total;
  int Tcap;
};
constexpr int LDS_BYTES = 160 * 1024;   // LDS of one compute unit
// FP32 assembly stages a source frame's B / v entries in an LDS image laid
// out like the matrix-core accumulators of one tile pass (tile, lane,
// element), so each lane folds a tile with one 16-byte load.  Elements of
// the image for windows of at most Tcap tile rows and passes of maxt tiles
// per wave.
__host__ __device__ inline int img_elems(int Tcap, int maxt) {
  const int lt = (Tcap * (Tcap + 1)) / 2, pp = NWAVES * maxt;
  return 256 * (lt < pp ? lt : pp);
}
__host__ __device__ inline int stage_bytes(int esize) {
  return SBE * (4 + 4 * esize) + SBMAX * (4 + 2 * esize + 16) + (SBMAX + 1) * 4;
}
// Lane segments of a wave add their pair-table entries into separate copies
// (two per wave for windows of at most 32 frames, 16 in FP64), so they need
// not take turns.  The count depends on the window alone, so a window's sums
// are the same whatever else is in the batch.
__host__ __device__ inline int table_slots(int n_frames, int esize) {
  return (esize == 4 ? n_frames <= 32 : n_frames <= 16) ? 2 : 1;
}
// Rows of pair tables per wave the LDS must hold for windows of up to Rcap
// frames: the larger of one copy of Rcap rows and two copies of the largest
// two-copy window.
__host__ __device__ inline int table_rows(int Rcap, int esize) {
  const int two = esize == 4 ? 32 : 16;
  const int a = table_slots(Rcap, esize) * Rcap, b = 2 * (Rcap < two ? Rcap : two);
  return a > b ? a : b;
}
__host__ __device__ inline int al16(int o) { return (o + 15) & ~15; }
// maxt of 4 or 5 adds the FP32 entry image when the LDS has room for it
// (img == 0 otherwise).
__host__ __device__ inline AsmLayout asm_layout(int Rcap, int esize, int maxt = 0) {
  AsmLayout L;
  const int Dcap = 6 * Rcap;
  L.Tcap = (Dcap + 1 + 15) / 16;
  int o = 0;
  L.poses = o; o = al16(o + Rcap * 7 * 8);
  L.rel = o;   o = al16(o + Rcap * RELW * esize);
  L.tbl = o;   o = al16(o + NWAVES * table_rows(Rcap, esize) * TBL * esize);
  L.G = o;     o = al16(o + (Rcap * 36 + 42) * esize);
  L.U = o;     o = al16(o + 16 * L.Tcap * LDK * esize);
  L.tiles = o; o = al16(o + 4 * ((L.Tcap * (L.Tcap + 1)) / 2 + 4));
  L.arng = o;  o = al16(o + 4 * 2 * RMAX);
  L.stage = o; o = al16(o + stage_bytes(esize));
  L.img = 0;
  if (esize == 4 && maxt > 0 && maxt <= 5) {   // the 8-tile passes keep the register budget for the gather
    const int ib = img_elems(L.Tcap, maxt) * esize;
    if (o + ib + 64 + 255 <= LDS_BYTES) { L.img = o; o = al16(o + ib); }
  }
  L.misc = o;  o += 64;
  L.total = (o + 255) & ~255;
  return L;
}
// back-substitution: poses, relative poses, pose steps, stage
__host__ __device__ inline int backsub_dx_offset(int Rcap, int esize) {
  return al16(al16(Rcap * 7 * 8) + Rcap * RELW * esize);
}
__host__ __device__ inline int backsub_stage_offset(int Rcap, int esize) {
  return al16(backsub_dx_offset(Rcap, esize) + Rcap * 6 * 8);
}
// then 64 bytes of flags and the target frame ranges of the chunk's source
// frames (2 * RMAX ints)
// and the per-target-frame vectors dx_j - Ad(T_ja) dx_a (6 doubles per frame)
__host__ __device__ inline int backsub_delta_offset(int Rcap, int esize) {
  return al16(backsub_stage_offset(Rcap, esize) + stage_bytes(esize) + 64 + 8 * RMAX);
}
__host__ __device__ inline int backsub_lds_bytes(int Rcap, int esize) {
  return backsub_delta_offset(Rcap, esize) + Rcap * 6 * 8;
}

// packed index of (m, n), m <= n, in the 21-entry upper triangle of a 6x6
__device__ __forceinline__ int sym6(int m, int n) {
  if (m > n) { int t = m; m = n; n = t; }
  return m * 6 - (m * (m - 1)) / 2 + (n - m);
}

template <typename T>
struct EdgeOut {
  T cd, wd;        // J_d^T W J_d, J_d^T W r
  T Ej[6];         // J_j^T W J_d
  T Ei[6];         // J_i^T W J_d = -Ad^T Ej
  T J0[6], J1[6];  // rows of J_j
  T r0, r1, w0, w1;
  T X, Y, Z, jd0, jd1;   // reprojected point, J_d
  bool active;
  int j;
};

// Linearise one edge.  rel: R (9), t (3), hat(t)R (9) of T_ji in LDS.
template <typename T, bool kEi = true>
__device__ __forceinline__ void linearize_edge(const T* rel, T xb, T yb, T d, T tx, T ty, T w0,
                                      T w1, T fx, T fy, T cx, T cy, T zmin, bool valid,
                                      EdgeOut<T>& o) {
  const T X = rel[0] * xb + rel[1] * yb + rel[2] + rel[9] * d;
  const T Y = rel[3] * xb + rel[4] * yb + rel[5] + rel[10] * d;
  const T Z = rel[6] * xb + rel[7] * yb + rel[8] + rel[11] * d;
  o.active = valid && (Z > zmin);
  const T iz = o.active ? recip(Z) : T(0);
  const T a = fx * iz, b = fy * iz;
  const T c0 = -fx * X * iz * iz, c1 = -fy * Y * iz * iz;
  o.w0 = o.active ? w0 : T(0);
  o.w1 = o.active ? w1 : T(0);
  o.r0 = o.active ? (fx * X * iz + cx - tx) : T(0);
  o.r1 = o.active ? (fy * Y * iz + cy - ty) : T(0);
  // rows of Pi [d I | -hat(p)]:  -Pi_c hat(p) = p x Pi_c
  o.J0[0] = d * a;  o.J0[1] = T(0);  o.J0[2] = d * c0;
  o.J0[3] = Y * c0; o.J0[4] = Z * a - X * c0; o.J0[5] = -Y * a;
  o.J1[0] = T(0);   o.J1[1] = d * b; o.J1[2] = d * c1;
  o.J1[3] = Y * c1 - Z * b; o.J1[4] = -X * c1; o.J1[5] = X * b;
  const T jd0 = a * rel[9] + c0 * rel[11];
  const T jd1 = b * rel[10] + c1 * rel[11];
  o.X = X; o.Y = Y; o.Z = Z; o.jd0 = jd0; o.jd1 = jd1;
  const T g0 = o.w0 * jd0, g1 = o.w1 * jd1;
  o.cd = g0 * jd0 + g1 * jd1;
  o.wd = g0 * o.r0 + g1 * o.r1;
  // (J0[1] = J1[0] = 0: those products are left out, not multiplied by zero)
  o.Ej[0] = g0 * o.J0[0];
  o.Ej[1] = g1 * o.J1[1];
#pragma unroll
  for (int m = 2; m < 6; ++m) o.Ej[m] = g0 * o.J0[m] + g1 * o.J1[m];
  // Ei = -Ad^T Ej with Ad^T = [[R^T, 0], [(hat(t)R)^T, R^T]]
  if constexpr (kEi) {
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    o.Ei[m] = -(rel[m] * o.Ej[0] + rel[3 + m] * o.Ej[1] + rel[6 + m] * o.Ej[2]);
    o.Ei[3 + m] = -(rel[12 + m] * o.Ej[0] + rel[15 + m] * o.Ej[1] + rel[18 + m] * o.Ej[2] +
                    rel[m] * o.Ej[3] + rel[3 + m] * o.Ej[4] + rel[6 + m] * o.Ej[5]);
  }
  }
}

// Broadcast a value computed by thread 0 to the workgroup.
__device__ __forceinline__ int wg_bcast_status(const int32_t* status, int w, int* slot) {
  if (threadIdx.x == 0) *slot = status[w];
  __syncthreads();
  const int s = *slot;
  __syncthreads();
  return s;
}


// One relative pose's LDS entry: R (9), t (3), hat(t) R (9).
template <typename T>
__device__ __forceinline__ void store_relpose(const double* R, const double* t, T* o) {
#pragma unroll
  for (int m = 0; m < 9; ++m) o[m] = (T)R[m];
#pragma unroll
  for (int m = 0; m < 3; ++m) o[9 + m] = (T)t[m];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o[12 + c] = (T)(-t[2] * R[3 + c] + t[1] * R[6 + c]);
    o[15 + c] = (T)(t[2] * R[c] - t[0] * R[6 + c]);
    o[18 + c] = (T)(-t[1] * R[c] + t[0] * R[3 + c]);
  }
}

// Relative poses T_ja for j in [lo, hi] into rel[(j - f_lo) * RELW].
template <typename T>
__device__ __forceinline__ void load_relposes(const double* poses, int a, int lo, int hi, int f_lo, T* rel) {
  for (int j = lo + (int)threadIdx.x; j <= hi; j += WG) {
    double R[9], t[3];
    relative_pose(poses + 7 * a, poses + 7 * j, R, t);
    store_relpose<T>(R, t, rel + (j - f_lo) * RELW);
  }
}

// A[p][q] of Ad(T_ji) = [[R, hat(t)R], [0, R]] from the LDS relative pose.
template <typename T>
__device__ __forceinline__ T adj_at(const T* rel, int p, int q) {
  if (p < 3) return q < 3 ? rel[3 * p + q] : rel[12 + 3 * p + (q - 3)];
  return q < 3 ? T(0) : rel[3 * (p - 3) + (q - 3)];
}

// Element (row, col) of a chunk's partial block: the lower triangle of the
// D x D pose block row-major, then rows D .. Daug-1 (the right-hand side and,
// in the adjoint, the cotangent column); -1 for an element outside it.
__device__ __forceinline__ int part_slot(int row, int col, int D, int Daug) {
  if (row < D && col <= row) return row * D + col;
  if (row >= D && row < Daug && col < D) return D * D + (row - D) * D + col;
  return -1;
}

// State after `iter` iterations: poses (slot iter of pose_buf) and inverse
// depths (slot iter of depth_buf, position order); slot 0 holds the inputs.
template <typename T>
__device__ inline const double* state_poses(const Params& P, const WinDesc& W, int iter) {
  return P.pose_buf + (int64_t)iter * 7 * P.n_frames_total + 7 * W.frame_off;
}
__device__ inline double* state_depth(const Params& P, const WinDesc& W, int iter) {
  return P.depth_buf + (int64_t)iter * P.n_patches_total + W.patch_off;
}

// ---------------------------------------------------------------------------
// Sub-batch staging.  A sub-batch is a run of at most SB positions of one
// source frame (descriptor from the preparation pass: first position,
// source frame << 8 | count, edge range [e0, e1)).  Its edges (target frame,
// target, weight) and per-patch data (patch index, edge offset, normalised
// pixel, inverse depth) are copied into LDS with coalesced loads.  The loads
// of the next sub-batch are issued into registers before the current one is
// processed and written to LDS after its edges have been consumed, so global
// latency overlaps the linearisation and the matrix-core work.
template <typename T>
struct Stage {
  int32_t* j; T* t; T* w; int32_t* pk; int32_t* pe; T* px; T* py; double* pd; double* pd2;
  __device__ Stage(char* base) {
    j = (int32_t*)base;
    t = (T*)(base + SBE * 4);
    w = (T*)(base + SBE * (4 + 2 * sizeof(T)));
    char* q = base + SBE * (4 + 4 * sizeof(T));
    pd = (double*)q; q += SBMAX * 8;
    pd2 = (double*)q; q += SBMAX * 8;
    px = (T*)q; q += SBMAX * sizeof(T);
    py = (T*)q; q += SBMAX * sizeof(T);
    pk = (int32_t*)q; q += SBMAX * 4;
    pe = (int32_t*)q;
  }
};

template <typename T>
struct StageRegs {
  int32_t j[2];
  T t[4], w[4];
  int32_t pk, pe;
  T px, py;
  double pd, pd2;
};

struct WinEdges {   // edge arrays in edge order (inputs, or the gathered copies)
  const int32_t* j;
  const void* t;
  const void* w;
};

__device__ __forceinline__ WinEdges win_edges(const Params& P, const WinDesc& W, int gathered, int esize) {
  WinEdges e;
  if (gathered) {
    e.j = P.gj + W.edge_off;
    e.t = (const char*)P.gt + 2 * esize * W.edge_off;
    e.w = (const char*)P.gw + 2 * esize * W.edge_off;
  } else {
    e.j = P.jj + W.edge_off;
    e.t = (const char*)P.targets + 2 * esize * W.edge_off;
    e.w = (const char*)P.weights + 2 * esize * W.edge_off;
  }
  return e;
}

// `iter` selects the inverse-depth state; `extra` (optional, position order)
// is staged alongside (the depth cotangents of the adjoint).
template <typename T>
__device__ __forceinline__ void stage_issue(const Params& P, const WinDesc& W, int w, const WinEdges& we,
                                   int4 d, int iter, const double* extra, StageRegs<T>& R) {
  const int tid = threadIdx.x;
  const int pos0 = d.x, n = d.y & 255, e0 = d.z, e1 = d.w;
  const T* tg = (const T*)we.t;
  const T* wt = (const T*)we.w;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int q = e0 + tid + r * WG;
    if (q < e1) {
      R.j[r] = we.j[q];
      R.t[2 * r] = tg[2 * q];
      R.t[2 * r + 1] = tg[2 * q + 1];
      R.w[2 * r] = wt[2 * q];
      R.w[2 * r + 1] = wt[2 * q + 1];
    }
  }
  // (registers the loads land in are not written otherwise: a write would
  // wait for the loads in flight)
  if (tid < n) {
    // edge offset of the patch, made relative to the sub-batch when stored
    R.pe = P.estart[W.patch_off + w + pos0 + tid];
    R.pk = P.plist[W.patch_off + pos0 + tid];
    const T* pxy = (const T*)P.pxy + 2 * (W.patch_off + pos0 + tid);
    R.px = pxy[0];
    R.py = pxy[1];
    R.pd = state_depth(P, W, iter)[pos0 + tid];
    if (extra) R.pd2 = extra[W.patch_off + pos0 + tid];
  }
}

template <typename T>
__device__ __forceinline__ void stage_store(int4 d, const StageRegs<T>& R, Stage<T>& S, bool extra) {
  const int tid = threadIdx.x;
  const int n = d.y & 255, ne = d.w - d.z;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int q = tid + r * WG;
    if (q < ne) {
      S.j[q] = R.j[r];
      S.t[2 * q] = R.t[2 * r];
      S.t[2 * q + 1] = R.t[2 * r + 1];
      S.w[2 * q] = R.w[2 * r];
      S.w[2 * q + 1] = R.w[2 * r + 1];
    }
  }
  if (tid < n) {
    S.pe[tid] = R.pe - d.z;
    S.pk[tid] = R.pk;
    S.px[tid] = R.px;
    S.py[tid] = R.py;
    S.pd[tid] = R.pd;
    if (extra) S.pd2[tid] = R.pd2;
  }
  if (tid == n) S.pe[n] = ne;
}

// One lane's edge of the staged sub-batch: slot `slot` (patch), lane `lseg`
// of its segment.
template <typename T>
struct LaneEdge {
  bool pv, has;
  int slot, deg, q, j;
  T t0, t1, w0, w1, xb, yb;
  double d;
};

template <typename T>
__device__ __forceinline__ LaneEdge<T> lane_edge(const Stage<T>& S, int slot, bool slot_ok, int n, int lseg, int a) {
  LaneEdge<T> L;
  L.slot = slot;
  L.pv = slot_ok && slot < n;
  const int s = L.pv ? slot : 0;
  const int base = S.pe[s];
  L.deg = L.pv ? S.pe[s + 1] - base : 0;
  L.has = lseg < L.deg;
  L.q = base + lseg;
  const int q = L.has ? L.q : 0;
  L.j = L.has ? S.j[q] : a;
  L.t0 = L.has ? S.t[2 * q] : T(0);
  L.t1 = L.has ? S.t[2 * q + 1] : T(0);
  L.w0 = L.has ? S.w[2 * q] : T(0);
  L.w1 = L.has ? S.w[2 * q + 1] : T(0);
  L.xb = S.px[s];
  L.yb = S.py[s];
  L.d = S.pd[s];
  return L;
}

// Frame range of a chunk: union of its anchors' ranges.
__device__ __forceinline__ void chunk_range(const Params& P, const WinDesc& W, const ChunkDesc& cd,
                                   int& f_lo, int& f_hi) {
  const int32_t* ar = P.arange + 2 * W.frame_off;
  f_lo = 1 << 30;
  f_hi = -1;
  for (int a = cd.a_lo; a < cd.a_hi; ++a) {
    f_lo = min(f_lo, ar[2 * a]);
    f_hi = max(f_hi, ar[2 * a + 1]);
  }
}

// Running sums of the tile elements across source frames.  FP32 assembly:
// each source frame's contribution (its B / v entries minus its outer
// products, formed in FP32) is added into FP64 registers `sh`, so no FP32
// value ever carries the whole window's sum.  FP64 assembly: the matrix-core
// accumulators themselves are the running sums (of the negated entries).
template <typename T, int MAXT>
__device__ __forceinline__ void wg_assemble(const Params& P, int c, int iter, char* smem, int Rcap) {
  typedef typename AccT<T>::type Acc;
  const AsmLayout L = asm_layout(Rcap, (int)sizeof(T), MAXT);
  double* lp = (double*)(smem + L.poses);
  T* rel = (T*)(smem + L.rel);
  T* tbl = (T*)(smem + L.tbl);
  T* G = (T*)(smem + L.G);
  T* U = (T*)(smem + L.U);
  int* tiles = (int*)(smem + L.tiles);
  int* arng = (int*)(smem + L.arng);   // target frame ranges of the chunk's source frames
  int* misc = (int*)(smem + L.misc);
  Stage<T> S(smem + L.stage);

  const ChunkDesc cd = P.chunk[c];
  const int w = cd.window;
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  if (tid == 0) *(T*)(misc + 8) = T(0);   // zero slot of the fold's entry lookup
  const int st = wg_bcast_status(P.status, w, misc);
  if (st != 0) {
    if (tid == 0) { P.cstate[2 * c] = 0; P.cstate[2 * c + 1] = 0; }
    return;
  }
  const int N = W.n_frames, nfix = W.n_fixed;
  int f_lo, f_hi;
  chunk_range(P, W, cd, f_lo, f_hi);
  const int lo_free = max(f_lo, nfix);
  const int D = (f_hi >= lo_free) ? 6 * (f_hi - lo_free + 1) : 0;
  if (tid == 0) { P.cstate[2 * c] = lo_free; P.cstate[2 * c + 1] = D; }
  double* part = P.partial + W.part_off + (int64_t)(c - W.chunk_off) * W.part_stride;
  if (D == 0) return;   // every frame the chunk touches is fixed: nothing to assemble

  // entry image (FP32 only); empty between source frames
  T* img = (sizeof(T) == 4 && MAXT <= 5 && L.img) ? (T*)(smem + L.img) : nullptr;
  if (img) {
    const int ne = img_elems(L.Tcap, MAXT) / 4;
    for (int i = tid; i < ne; i += WG) ((float4*)img)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const double* poses = state_poses<T>(P, W, iter);
  for (int i = tid; i < 7 * N; i += WG) lp[i] = poses[i];
  const int32_t* ar = P.arange + 2 * W.frame_off;
  for (int i = tid; i < 2 * (cd.a_hi - cd.a_lo); i += WG) arng[i] = ar[2 * cd.a_lo + i];
  const int32_t* sbs = P.sbstart + W.frame_off + w;
  const int4* sbd = P.sbd + W.sb_off;
  const WinEdges we = win_edges(P, W, P.wmeta[4 * w + 1], (int)sizeof(T));
  const T fx = (T)W.fx, fy = (T)W.fy, cx = (T)W.cx, cy = (T)W.cy;
  const T zmin = (T)P.z_min, lam = (T)P.lambda;
  const int SEG = seg_width(P.wmeta[4 * w]);
  const int SBw = sb_width(SEG);
  const int segs = 64 / SEG;                 // patches per wave pass
  const int spw = SBw / NWAVES;              // patch slots per wave per sub-batch
  const int npass = (spw + segs - 1) / segs;
  const int lseg = lane & (SEG - 1), sidx = lane / SEG;
  const int s_lo = sbs[cd.a_lo], s_hi = sbs[cd.a_hi];
  const int tslots = min(segs, table_slots(N, (int)sizeof(T)));   // pair-table copies per wave
  // staged columns beyond the pose dofs: w_k / sqrt(C_k) (column D) and, for
  // the adjoint, the depth cotangent / sqrt(C_k) (column D + 1)
  const int nextra = P.adjoint ? 2 : 1;
  const double* dbar_in = P.adjoint ? P.dbar + ((iter + 1) & 1) * P.n_patches_total : nullptr;

  // lower-triangle tiles of the (D+n_extra)^2 product, row-major
  const int Daug = D + nextra;
  const int T16 = (Daug + 15) / 16;
  const int Ltot = (T16 * (T16 + 1)) / 2;
  for (int t = tid; t < Ltot; t += WG) {
    int ti = 0;
    while (((ti + 1) * (ti + 2)) / 2 <= t) ++ti;
    tiles[t] = (ti << 16) | (t - (ti * (ti + 1)) / 2);
  }
  const int per_pass = NWAVES * MAXT;
  const int npasses_t = (Ltot + per_pass - 1) / per_pass;
  bool nonfinite = false;

  for (int tp = 0; tp < npasses_t; ++tp) {
    const int p0 = tp * per_pass;
    const int Lp = min(per_pass, Ltot - p0);
    // this wave's tiles of the pass: p0 + wv, p0 + wv + NWAVES, ... (spread
    // over the rows, so that the tiles a source frame reaches are shared out
    // evenly among the waves)
    const int ntl = Lp > wv ? (Lp - wv + NWAVES - 1) / NWAVES : 0;
    const int t_beg = p0 + wv;   // tile t of the wave is t_beg + NWAVES * t
    Acc acc[MAXT];
    // FP32 assembly keeps each tile element's FP64 running sum in registers,
    // except the 12-tile variant (windows whose chunks span about 34 free
    // frames, one tile pass instead of two): it has no register room for
    // them and keeps them in the chunk's partial block, each element read and
    // written by its own lane at the ends of source frames only
    constexpr bool kGlobalFold = sizeof(T) == 4 && MAXT > 8;
    double sh[kGlobalFold ? 1 : 4 * MAXT];
    // Regular source frames (every patch with the same target-frame sequence)
    // with one table copy per lane segment: each lane accumulates the
    // pair-table row of its one target frame, in registers for the whole
    // source frame in the FP32 passes of at most five tiles per wave
    constexpr bool kRegTbl = sizeof(T) == 4 && MAXT <= 5;
    T qacc[kRegTbl ? TBL : 1];
    bool regular = false;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) acc[t] = Acc{T(0), T(0), T(0), T(0)};
    if constexpr (!kGlobalFold) {
#pragma unroll
      for (int t = 0; t < 4 * MAXT; ++t) sh[t] = 0.0;
    }

    StageRegs<T> R;
    int4 dcur = make_int4(0, 0, 0, 0), dnxt = dcur;
    if (s_lo < s_hi) {
      dcur = sbd[s_lo];
      if (s_lo + 1 < s_hi) dnxt = sbd[s_lo + 1];
      stage_issue<T>(P, W, w, we, dcur, iter, dbar_in, R);
    }
    __syncthreads();   // previous pass done with the stage and the poses are in LDS
    if (s_lo < s_hi) stage_store<T>(dcur, R, S, dbar_in != nullptr);
    if constexpr (kGlobalFold) {
      // the running sums of this wave's tiles start from zero
      const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (t < ntl) {
          const int code = tiles[t_beg + NWAVES * t];
          const int ti = code >> 16, tj = code & 0xffff;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int sl = part_slot(16 * ti + acc_row(T(0), g, r), 16 * tj + l16, D, Daug);
            if (sl >= 0) part[sl] = 0.0;
          }
        }
      }
    }

    int a = -1, lo = 0, hi = -1, Ra = 0, nz_lo = 0, nz_hi = 0;
    unsigned tmask = 0;   // this wave's tiles reached by the current source frame
    bool a_free = false;
    for (int s = s_lo; s <= s_hi; ++s) {
      const int an = (s < s_hi) ? ((dcur.y >> 8) & 0xff) : -1;
      if (an != a && a >= 0) {
        // ---- pair blocks of the finished source frame a
        // regular frames with two segments per wave first add the segments'
        // rows (in registers or in LDS, the same sums), then the waves' copies
        // are added; otherwise every copy is added
        const int cstride = (regular && tslots == 2) ? 2 : 1;
        if (regular && tslots == 2) {
          if constexpr (kRegTbl) {
#pragma unroll
            for (int q = 0; q < TBL; ++q) qacc[q] = swap_add<32>(qacc[q]);
            // lane x holds target frame lo + x (zeros if no edge of it was
            // active), so every row of the wave's copy is written and the
            // copy needs no clearing
            if (sidx == 0 && lseg < Ra) {
              T* row = tbl + (wv * 2 * Ra + lseg) * TBL;
#pragma unroll
              for (int q = 0; q < TBL; ++q) row[q] = qacc[q];
            }
          } else {
            T* c0 = tbl + wv * 2 * Ra * TBL;
            for (int i = lane; i < Ra * TBL; i += 64) c0[i] = c0[i] + c0[Ra * TBL + i];
          }
        } else if (kRegTbl && regular && lseg < Ra) {
          // the lane's register row into its wave's table copy (every row,
          // as above)
          T* row = tbl + ((wv * tslots + sidx) * Ra + lseg) * TBL;
#pragma unroll
          for (int q = 0; q < TBL; ++q) row[q] = qacc[q];
        }
        lds_barrier();
        for (int i = tid; i < Ra * TBL; i += WG) {
          T sum = 0;
          for (int x = 0; x < NWAVES * tslots; x += cstride) sum += tbl[x * Ra * TBL + i];
          tbl[i] = sum;
          if (img) {
            // Q_j into the (j, j) block, V_j into the gradient row
            const int jr = i / TBL, e = i - jr * TBL, j = lo + jr;
            if (j != a && j >= lo_free) {
              const int J6 = 6 * (j - lo_free);
              int row = D, col = J6 + e - 21;
              if (e < 21) {
                int m, n;
                unsym6(e, m, n);
                row = J6 + n;
                col = J6 + m;
              }
              const int sl = img_slot(row, col, p0, Lp);
              if (sl >= 0) img[sl] = sum;
            }
          }
        }
        lds_barrier();
        // G_j = A_j^T Q_j
        for (int i = tid; i < Ra * 36; i += WG) {
          const int jr = i / 36, m = (i % 36) / 6, n = i % 6;
          const T* rj = rel + (lo + jr - f_lo) * RELW;
          const T* Q = tbl + jr * TBL;
          const int mm = m < 3 ? m : m - 3;
          // rows p = 0..2 of A carry R (m < 3) or hat(t)R (m >= 3); rows 3..5
          // carry R for m >= 3 only
          const T* top = m < 3 ? rj : rj + 12;
          T sum = top[mm] * Q[sym6(0, n)] + top[3 + mm] * Q[sym6(1, n)] + top[6 + mm] * Q[sym6(2, n)];
          if (m >= 3)
            sum += rj[mm] * Q[sym6(3, n)] + rj[3 + mm] * Q[sym6(4, n)] + rj[6 + mm] * Q[sym6(5, n)];
          G[i] = sum;
          if (img && a_free) {
            // -A^T Q_j into the (a, j) block (its transpose when j > a)
            const int j = lo + jr;
            if (j != a && j >= lo_free) {
              const int A6 = 6 * (a - lo_free), J6 = 6 * (j - lo_free);
              const int sl = a > j ? img_slot(A6 + m, J6 + n, p0, Lp) : img_slot(J6 + n, A6 + m, p0, Lp);
              if (sl >= 0) img[sl] = -sum;
            }
          }
        }
        lds_barrier();
        // anchor block sum_j A^T Q A and anchor gradient -sum_j A^T V (targets in
        // fixed frames included: J_i = -J_j Ad(T_ji) whatever frame j is)
        // (42 entries, each a sum over the target frames: 12 interleaved
        // partial sums per entry, staged in the consumed U buffer, then added
        // in order)
        T* AQA = G + Ra * 36;
        constexpr int NP = 12;
        if (a_free) {
          if (tid < 42 * NP) {
            const int i = tid / NP, part = tid % NP;
            T sum = 0;
            if (i < 36) {
              const int m = i / 6, n = i % 6;
              for (int jr = part; jr < Ra; jr += NP) {
                if (lo + jr == a) continue;
                const T* rj = rel + (lo + jr - f_lo) * RELW;
#pragma unroll
                for (int q2 = 0; q2 < 6; ++q2) sum += G[jr * 36 + m * 6 + q2] * adj_at(rj, q2, n);
              }
            } else {
              const int m = i - 36;
              for (int jr = part; jr < Ra; jr += NP) {
                if (lo + jr == a) continue;
                const T* rj = rel + (lo + jr - f_lo) * RELW;
                const T* Q = tbl + jr * TBL;
#pragma unroll
                for (int p = 0; p < 6; ++p) sum -= adj_at(rj, p, m) * Q[21 + p];
              }
            }
            U[tid] = sum;
          }
          lds_barrier();
          if (tid < 42) {
            T sum = 0;
#pragma unroll
            for (int part = 0; part < NP; ++part) sum += U[tid * NP + part];
            AQA[tid] = sum;
            if (img) {
              const int A6 = 6 * (a - lo_free);
              int sl = -1;
              if (tid < 36) {
                const int m = tid / 6, n = tid % 6;
                if (m >= n) sl = img_slot(A6 + m, A6 + n, p0, Lp);
              } else {
                sl = img_slot(D, A6 + tid - 36, p0, Lp);
              }
              if (sl >= 0) img[sl] = sum;
            }
          }
        }
        lds_barrier();
        // Each lane folds this source frame's B / v entries of its tile
        // elements and the staged outer products into its running sums:
        //   (j,j) += Q_j, (a,j) -= A^T Q_j, (a,a) += sum A^T Q A, v_j += V_j,
        //   v_a -= sum A^T V, and -= sum_k u_k u_k^T.
        // The entry is located by selects (an element index into the stage's
        // LDS, a zero slot for entries the source frame does not touch), so the
        // lanes do not diverge and a tile's four loads are issued together.
        if constexpr (sizeof(T) == 4 && MAXT <= 5) {
          if (img) {
            // the image holds the entries at the accumulator positions; the
            // tiles read are cleared for the next source frame
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
              if (tmask & (1u << t)) {
                float4* src = (float4*)img + (t_beg + NWAVES * t - p0) * 64 + lane;
                const float4 v = *src;
                *src = make_float4(0.f, 0.f, 0.f, 0.f);
                const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  sh[t * 4 + r] += (double)vv[r] - (double)acc[t][r];
                  acc[t][r] = T(0);
                }
              }
            }
          }
        }
        if (!img) {
          const int l16 = lane & 15, g = lane >> 4;
          constexpr int ES = (int)sizeof(T);
          const int o_tbl = L.tbl / ES, o_G = L.G / ES, o_AQA = o_G + Ra * 36;
          const int o_zero = (L.misc + 32) / ES;
          const T* base = (const T*)smem;
          // kGlobalFold: the running sums of a group of FG tiles are loaded
          // together (one memory round trip per group) before their entries
          constexpr int FG = kGlobalFold ? 4 : 1;
          double old[FG][4];
          int osl[FG][4];
#pragma unroll
          for (int t = 0; t < MAXT; ++t) {
            if constexpr (kGlobalFold) {
              if (t % FG == 0) {
#pragma unroll
                for (int q = 0; q < FG; ++q) {
                  const bool in = t + q < MAXT && (tmask & (1u << (t + q)));
                  const int code = in ? tiles[t_beg + NWAVES * (t + q)] : 0;
                  const int ti = code >> 16, tj = code & 0xffff;
#pragma unroll
                  for (int r = 0; r < 4; ++r) {
                    osl[q][r] = in ? part_slot(16 * ti + acc_row(T(0), g, r), 16 * tj + l16, D, Daug) : -1;
                    old[q][r] = osl[q][r] >= 0 ? part[osl[q][r]] : 0.0;
                  }
                }
              }
            }
            // tiles the source frame does not reach hold no products and no
            // B / v entries of it
            if (tmask & (1u << t)) {
              const int code = tiles[t_beg + NWAVES * t];
              const int ti = code >> 16, tj = code & 0xffff;
              const int col = 16 * tj + l16;
              const int cf = col / 6, n = col - 6 * cf, fc = lo_free + cf;
              const bool cin = fc >= lo && fc <= hi;
              int idx[4];
              bool neg[4];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = 16 * ti + acc_row(T(0), g, r);
                const int rf = row / 6, m = row - 6 * rf, fr = lo_free + rf;
                const bool rin = fr >= lo && fr <= hi;
                const int mn = min(m, n), mx = max(m, n);
                const int i_v = fc == a ? o_AQA + 36 + n : (cin ? o_tbl + (fc - lo) * TBL + 21 + n : o_zero);
                const int i_d = fr == a ? o_AQA + m * 6 + n
                                        : (rin ? o_tbl + (fr - lo) * TBL + mn * 6 - (mn * (mn - 1)) / 2 + (mx - mn) : o_zero);
                const bool ga = fr == a && cin, gb = fc == a && rin;
                const int i_g = ga ? o_G + (fc - lo) * 36 + m * 6 + n : o_G + (fr - lo) * 36 + n * 6 + m;
                const bool lower = row < D && col <= row;
                int i = o_zero;
                i = (row == D && col < D && a_free | (fc != a)) ? i_v : i;
                i = (lower && fr == fc && (a_free | (fr != a))) ? i_d : i;
                i = (lower && fr != fc && (ga || gb)) ? i_g : i;
                idx[r] = i;
                neg[r] = lower && fr != fc && (ga || gb);
              }
              T val[4];
#pragma unroll
              for (int r = 0; r < 4; ++r) val[r] = base[idx[r]];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const T v = neg[r] ? -val[r] : val[r];
                if constexpr (kGlobalFold) {
                  const int sl = osl[t % FG][r];
                  if (sl >= 0) part[sl] = old[t % FG][r] + ((double)v - (double)acc[t][r]);
                  acc[t][r] = T(0);
                } else if constexpr (sizeof(T) == 4) {
                  sh[t * 4 + r] += (double)v - (double)acc[t][r];
                  acc[t][r] = T(0);
                } else {
                  acc[t][r] -= v;
                }
              }
            }
          }
        }
        lds_barrier();
      }
      if (s == s_hi) break;
      const bool started = an != a;
      if (an != a) {
        // ---- start of source frame an: relative poses, empty pair tables
        a = an;
        lo = arng[2 * (a - cd.a_lo)];
        hi = arng[2 * (a - cd.a_lo) + 1];
        Ra = hi - lo + 1;
        load_relposes<T>(lp, a, lo, hi, f_lo, rel);
        // one table copy per lane segment and one target frame per lane: the
        // rows are summed in the same order in registers (five-tile FP32
        // passes) or in LDS (otherwise), so the sums do not depend on the
        // kernel variant a batch selects
        regular = sizeof(T) == 4 && (dcur.y & SB_REGULAR) && tslots == segs;   // FP32 assembly
        // the tables start from zero, except the register rows' copies, which
        // the frame end writes in full
        if (!(kRegTbl && regular)) {
          const int nt = NWAVES * tslots * Ra * TBL, n4 = (nt * (int)sizeof(T)) / 16;
          for (int i = tid; i < n4; i += WG) ((float4*)tbl)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
          for (int i = (n4 * 16) / (int)sizeof(T) + tid; i < nt; i += WG) tbl[i] = T(0);
        }
        if constexpr (kRegTbl) {
#pragma unroll
          for (int q = 0; q < TBL; ++q) qacc[q] = T(0);
        }
        nz_lo = 6 * (max(lo, lo_free) - lo_free);
        nz_hi = (hi >= lo_free) ? 6 * (hi - lo_free + 1) : 0;
        a_free = a >= nfix;
        // this wave's tiles that the source frame's outer products reach
        tmask = 0;
        for (int t = 0; t < ntl; ++t) {
          const int code = tiles[t_beg + NWAVES * t];
          const int ti = code >> 16, tj = code & 0xffff;
          const bool rows_nz = (16 * ti < nz_hi && 16 * ti + 16 > nz_lo) ||
                               (16 * ti < Daug && D < 16 * ti + 16);
          const bool cols_nz = (16 * tj < nz_hi && 16 * tj + 16 > nz_lo) ||
                               (16 * tj < Daug && D < 16 * tj + 16);
          if (rows_nz && cols_nz) tmask |= 1u << t;
        }
        tmask = __builtin_amdgcn_readfirstlane(tmask);
      }
      const int nsb = dcur.y & 255;
      // prefetch the next sub-batch and the descriptor of the one after
      int dnn = 0;
      const bool pre = s + 2 < s_hi;
      if (s + 1 < s_hi) stage_issue<T>(P, W, w, we, dnxt, iter, dbar_in, R);
      if (pre) dnn = desc_prefetch(sbd + s + 2);
      // The staged rows start from zero.  A regular source frame writes every
      // (target, patch) entry it owns in each sub-batch (zero for an inactive
      // edge), so U is cleared at the frame's start only, plus the columns of
      // a short last sub-batch that the products read past its patches.
      const int nkb = (nsb + 15) >> 4;
      const bool clear_all = !regular || started;
      if (clear_all) {
        for (int i = tid; i < (16 * T16 * LDK * (int)sizeof(T)) / 16; i += WG) ((float4*)U)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      } else if (nsb & 15) {
        const int nc = 16 * nkb - nsb;
        for (int i = tid; i < 16 * T16 * nc; i += WG) U[(i / nc) * LDK + nsb + i % nc] = T(0);
      }
      if (clear_all || (nsb & 15)) lds_barrier();

      // ---- linearise this wave's patches, one lane segment per patch
      T* mytbl = tbl + wv * tslots * Ra * TBL;
      for (int ps = 0; ps < npass; ++ps) {
        const int slot_in_wave = ps * segs + sidx;
        const LaneEdge<T> le = lane_edge<T>(S, wv * spw + slot_in_wave, slot_in_wave < spw, nsb, lseg, a);
        if (le.has && !(__builtin_isfinite(le.t0) && __builtin_isfinite(le.t1) &&
                        __builtin_isfinite(le.w0) && __builtin_isfinite(le.w1)))
          nonfinite = true;
        EdgeOut<T> eo;
        const int j = le.j;
        linearize_edge<T>(rel + (j - f_lo) * RELW, le.xb, le.yb, (T)le.d, le.t0, le.t1, le.w0,
                          le.w1, fx, fy, cx, cy, zmin, le.has && (j != a), eo);
        // pair tables Q_aj (21) and V_aj (6); segments of a wave take turns,
        // and duplicate (k, j) edges inside a segment are added one lane at a time
        bool anydup = false;
        if (sizeof(T) == 4 && regular) {
          if (eo.active) {
            T* racc = qacc;
            if constexpr (!kRegTbl) racc = mytbl + (sidx * Ra + (j - lo)) * TBL;
            // Q += w0 J0 J0^T + w1 J1 J1^T, V += w0 r0 J0 + w1 r1 J1, with the
            // structural zeros J0[1] = J1[0] = 0 left out
            int q = 0;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
              const T a0 = eo.w0 * eo.J0[m], a1 = eo.w1 * eo.J1[m];
#pragma unroll
              for (int n = m; n < 6; ++n, ++q) {
                const bool z0 = m == 1 || n == 1, z1 = m == 0 || n == 0;
                if (z0 && z1) continue;
                if (z0) racc[q] = a1 * eo.J1[n] + racc[q];
                else if (z1) racc[q] = a0 * eo.J0[n] + racc[q];
                else racc[q] = a1 * eo.J1[n] + (a0 * eo.J0[n] + racc[q]);
              }
            }
            const T b0 = eo.w0 * eo.r0, b1 = eo.w1 * eo.r1;
            racc[21] = b0 * eo.J0[0] + racc[21];
            racc[22] = b1 * eo.J1[1] + racc[22];
#pragma unroll
            for (int m = 2; m < 6; ++m) racc[21 + m] = b1 * eo.J1[m] + (b0 * eo.J0[m] + racc[21 + m]);
          }
        } else {
        const int jprev = __shfl_up(j, 1, 64);
        const bool dup = eo.active && lseg > 0 && jprev == j;
        anydup = __any(dup);
        T* tb = mytbl + ((sidx % tslots) * Ra + (j - lo)) * TBL;
        for (int sgi = 0; sgi < segs; sgi += tslots) {
          for (int ln = 0; ln < (anydup ? SEG : 1); ++ln) {
            if (sidx - sidx % tslots == sgi && eo.active && (!anydup || lseg == ln)) {
              int q = 0;
#pragma unroll
              for (int m = 0; m < 6; ++m)
#pragma unroll
                for (int n = m; n < 6; ++n, ++q)
                  tb[q] += eo.w0 * eo.J0[m] * eo.J0[n] + eo.w1 * eo.J1[m] * eo.J1[n];
#pragma unroll
              for (int m = 0; m < 6; ++m)
                tb[21 + m] += eo.w0 * eo.r0 * eo.J0[m] + eo.w1 * eo.r1 * eo.J1[m];
            }
          }
        }
        }
        T red[8] = {eo.cd, eo.wd, eo.Ei[0], eo.Ei[1], eo.Ei[2], eo.Ei[3], eo.Ei[4], eo.Ei[5]};
        seg_sum8(red, SEG);
        const T Ck = lam + red[0];
        const T Wk = red[1];
        const T* Eik = red + 2;
        const T rs = rsqrt_(Ck);
        // staged row u_k: E_jk / sqrt(C_k) at target columns, E_ik / sqrt(C_k) at
        // the source frame's columns, w_k / sqrt(C_k) at column D
        const int slot = le.slot;
        T* ucol = U + (6 * (j - lo_free)) * LDK + slot;
        if (regular) {
          if (le.pv && le.has && j != a && j >= lo_free) {
#pragma unroll
            for (int m = 0; m < 6; ++m) ucol[m * LDK] = eo.active ? eo.Ej[m] * rs : T(0);
          }
        } else {
          for (int ln = 0; ln < (anydup ? SEG : 1); ++ln) {
            if (le.pv && eo.active && j >= lo_free && (!anydup || lseg == ln)) {
#pragma unroll
              for (int m = 0; m < 6; ++m) ucol[m * LDK] += eo.Ej[m] * rs;
            }
          }
        }
        if (le.pv && lseg == 0) {
          if (a_free) {
            T* ua = U + (6 * (a - lo_free)) * LDK + slot;
#pragma unroll
            for (int m = 0; m < 6; ++m) ua[m * LDK] = Eik[m] * rs;
          }
          U[D * LDK + slot] = Wk * rs;
          if (nextra == 2) U[(D + 1) * LDK + slot] = (T)S.pd2[slot] * rs;
        }
      }
      lds_barrier();

      // ---- matrix-core outer products of the staged rows
      {
        const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
          if (tmask & (1u << t)) {
            const int code = tiles[t_beg + NWAVES * t];
            const int ti = code >> 16, tj = code & 0xffff;
            {
              const T* ua = U + (16 * ti + l16) * LDK + 4 * g;
              const T* ub = U + (16 * tj + l16) * LDK + 4 * g;
              for (int kb = 0; kb < nkb; ++kb) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                  acc[t] = mfma16(ua[16 * kb + s4], ub[16 * kb + s4], acc[t]);
              }
            }
          }
        }
      }
      if (s + 1 < s_hi) stage_store<T>(dnxt, R, S, dbar_in != nullptr);
      lds_barrier();
      dcur = dnxt;
      {
      // taken on every path, so no load is in flight into the next iteration
      const int4 dt = desc_take(dnn);
      if (pre) dnxt = dt;
    }
    }

    // ---- chunk partial: lower triangle of S and s, FP64
    {
      const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (!kGlobalFold && t < ntl) {
          const int code = tiles[t_beg + NWAVES * t];
          const int ti = code >> 16, tj = code & 0xffff;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int sl = part_slot(16 * ti + acc_row(T(0), g, r), 16 * tj + l16, D, Daug);
            double v = -(double)acc[t][r];
            if constexpr (sizeof(T) == 4 && !kGlobalFold) v = sh[t * 4 + r];
            if (sl >= 0) part[sl] = v;
          }
        }
      }
    }
    __syncthreads();
  }
  if (nonfinite) atomicOr(&P.status[w], W_NONFINITE);
}

}  // namespace dpba
