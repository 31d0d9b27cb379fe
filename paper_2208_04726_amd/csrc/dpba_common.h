// Shared definitions of the gfx950 bundle-adjustment kernels: launch
// constants, window / chunk descriptors, workspace layout, wave helpers and
// the FP64 SE(3) helpers used for relative poses and the retraction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpba {

constexpr int WG = 512;            // threads per workgroup (8 wave64s)
constexpr int NWAVES = WG / 64;
constexpr int RMAX = 64;           // frames per window (and per chunk range)
constexpr int NCHOL_MAX = 126;     // reduced pose system held in LDS (21 free frames)
constexpr int TBL = 27;            // pair table entries: 21 (6x6 sym) + 6

// status bits (match include/dpba.h)
constexpr int W_NOT_SPD = 1;
constexpr int W_NONFINITE = 2;
constexpr int W_BAD_INDEX = 4;
constexpr int W_DEGREE = 8;

// ---------------------------------------------------------------------------
// Descriptors, built on the host for every call and copied to the device.
struct WinDesc {
  int64_t frame_off, patch_off, edge_off;
  int32_t n_frames, n_patches, n_edges, n_fixed;
  double fx, fy, cx, cy;
  int32_t chunk_off, n_chunks;    // chunks of this window in the chunk table
  int64_t part_off;               // first element of this window's partials
  int64_t part_stride;            // elements per chunk partial (D*D + D, D = 6*(N-nfix))
  int64_t sb_off;                 // first sub-batch descriptor of this window
  int32_t eb_off, eb_n;           // edge blocks of the split preparation (EPB edges each)
};

struct ChunkDesc {
  int32_t window, a_lo, a_hi, pad;  // anchor frames [a_lo, a_hi) of the window
};

struct Params {
  const WinDesc* win;
  const ChunkDesc* chunk;
  const int32_t* counts;  // device [3]: windows, chunks, edge blocks of this call (grids may be larger)
  int32_t iterations;
  double lambda, z_min;
  // problem (caller buffers)
  const double* poses_in;
  const double* patches_in;
  const int32_t* anchor;
  const int32_t* kk;
  const int32_t* jj;
  const void* targets;
  const void* weights;
  double* poses_out;
  double* depth_out;
  // workspace
  int32_t* status;      // [W]
  int32_t* eflags;      // [edge blocks] flags of each block of the edge pass (bad index, unsorted, duplicate)
  int32_t* wmeta;       // [W*4]: max degree, edges-sorted flag, anchors-sorted flag
  int32_t* cnt;         // [P] edges per patch
  int32_t* ptr;         // [P] first CSR slot of each patch (window-local)
  int32_t* fill;        // [P] scatter cursor
  int32_t* jrun;        // [P][2] target frames of the first and last edge of a patch's run (edges in order)
  int32_t* acnt;        // [F+W] patches per anchor -> offsets
  int32_t* afill;       // [F] scatter cursor
  int32_t* plist;       // [P] patch at each position (positions sorted by (anchor, index))
  int32_t* csr;         // [E] edges sorted by (patch, target, index), window-local
  int32_t* estart;      // [P+W] first edge (edge order) of each position
  int32_t* sbstart;     // [F+W] first sub-batch of each source frame
  int4* sbd;            // sub-batches: (first position, frame << 8 | count, e0, e1)
  void* pxy;            // [P*2] T, normalised pixel of each position
  int32_t* gj;          // [E] gathered target frames (edge order)
  void* gt;             // [E*2] T gathered targets
  void* gw;             // [E*2] T gathered weights
  int32_t* arange;      // [F*2] frame range touched by each anchor's patches
  int32_t* cstate;      // [C*2] chunk: first free frame of its range, D
  double* partial;      // chunk partials of S (lower, D x D) and s (D), FP64
  double* s_big;        // [W][ld_big^2] augmented reduced systems of windows with n > 126
  int32_t ld_big;
  double* big_aux;      // [W][ld_big + 40] factorisation side data of those windows
  double* dxi;          // [F*6] pose steps
  double* pose_buf;     // [K+1][F*7] pose state after each iteration (slot 0: inputs)
  double* depth_buf;    // [K+1][P] inverse-depth state after each iteration, position order
  int64_t n_frames_total;   // slot strides
  int64_t n_patches_total;
  int32_t* gidx;        // [E] input index of each edge-order position (gathered layout)
  // adjoint
  int32_t adjoint;      // assembly adds the depth-cotangent column
  const double* grad_poses;   // [F*7] cotangent of poses_out
  const double* grad_depth;   // [P] cotangent of depth_out (patch order)
  void* grad_targets;   // [E*2] T out
  void* grad_weights;   // [E*2] T out
  double* xib;          // [F*6] pose cotangent (left tangent) of the current state
  double* xid;          // [F*6] direct part through the retraction
  double* qxi;          // [F*6] adjoint solve, pose part
  double* dbar;         // [2][P] depth cotangents, position order (ping-pong)
  double* fcot;         // [C][RMAX*6] per-chunk pose cotangent partials
};

// ---------------------------------------------------------------------------
// wave / workgroup helpers
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
// Sub-batch descriptor prefetch: lane k loads component k % 4, so the load is
// a per-lane one whose wait falls where the descriptor is taken (lane reads,
// a loop iteration later), not behind the other loads in flight.
__device__ __forceinline__ int desc_prefetch(const int4* d) {
  return ((const int*)d)[lane_id() & 3];
}
__device__ __forceinline__ int4 desc_take(int v) {
  return make_int4(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 1),
                   __builtin_amdgcn_readlane(v, 2), __builtin_amdgcn_readlane(v, 3));
}
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Lane exchanges of the segment sums, done in the vector ALU: DPP quad
// permutations (the lane 1 and 2 apart), the half-row and row mirrors (the
// other half of each 8- and 16-lane group) and the row swaps of gfx950 (the
// other 16-lane row of each 32, the other 32-lane half of the wave).  Every
// step adds two lane groups that already hold equal partial sums, so all
// lanes of a segment end with the bitwise-identical total, and the order of
// the additions depends only on the segment width.  All 64 lanes must be
// active.
template <int CTRL>
__device__ __forceinline__ float dpp_get(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_get(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// v plus the same lane of the other 16-lane row (ROW = 16) or 32-lane half (32)
template <int ROW>
__device__ __forceinline__ float swap_add(float v) {
  const int b = __float_as_int(v);
  const auto r = ROW == 16 ? __builtin_amdgcn_permlane16_swap(b, b, false, false)
                           : __builtin_amdgcn_permlane32_swap(b, b, false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
template <int ROW>
__device__ __forceinline__ double swap_add(double v) {
  const long long b = __double_as_longlong(v);
  const int l = (int)(b & 0xffffffffLL), h = (int)(b >> 32);
  const auto lo = ROW == 16 ? __builtin_amdgcn_permlane16_swap(l, l, false, false)
                            : __builtin_amdgcn_permlane32_swap(l, l, false, false);
  const auto hi = ROW == 16 ? __builtin_amdgcn_permlane16_swap(h, h, false, false)
                            : __builtin_amdgcn_permlane32_swap(h, h, false, false);
  const double x = __longlong_as_double(((long long)hi[0] << 32) | (unsigned int)lo[0]);
  const double y = __longlong_as_double(((long long)hi[1] << 32) | (unsigned int)lo[1]);
  return x + y;
}

// Sums of v[0..N) over aligned power-of-two lane segments of width seg.
template <int N, typename T>
__device__ __forceinline__ void seg_sum_n(T* v, int seg) {
  if (seg > 1) {
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] += dpp_get<0xB1>(v[m]);   // quad_perm [1,0,3,2]
  }
  if (seg > 2) {
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] += dpp_get<0x4E>(v[m]);   // quad_perm [2,3,0,1]
  }
  if (seg > 4) {
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] += dpp_get<0x141>(v[m]);  // row_half_mirror
  }
  if (seg > 8) {
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] += dpp_get<0x140>(v[m]);  // row_mirror
  }
  if (seg > 16) {
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = swap_add<16>(v[m]);
  }
  if (seg > 32) {
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = swap_add<32>(v[m]);
  }
}

template <typename T>
__device__ __forceinline__ T seg_sum(T v, int seg) {
  seg_sum_n<1>(&v, seg);
  return v;
}

template <typename T>
__device__ __forceinline__ void seg_sum8(T* v, int seg) {
  seg_sum_n<8>(v, seg);
}

// Reciprocal and reciprocal square root: the hardware approximations (about
// 1 ulp) in FP32, correctly rounded division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ bool isfinite_d(double x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool isfinite_f(float x) { return __builtin_isfinite(x); }

// Workgroup barrier for LDS traffic only: waits for this wave's LDS (and
// scalar) operations, not for its global loads, so loads issued ahead (the
// prefetch of the next sub-batch) stay in flight across it.  Use only where
// no global memory written before it is read after it by another wave.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt, expcnt unconstrained
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Makes what the lanes of a wave wrote to LDS visible to the other lanes of
// the same wave (fences at wave scope around a wave barrier).  Without it the
// compiler, reasoning lane by lane, may move a lane's read above a store that
// only another lane performs.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive scan of data[0..n) in place by the whole workgroup; returns the
// total.  lds must hold WG ints.  All threads must call it.
__device__ __forceinline__ int wg_exclusive_scan(int32_t* data, int n, int* lds) {
  const int tid = threadIdx.x;
  const int per = (n + WG - 1) / WG;
  const int b = tid * per, e = min(n, b + per);
  int s = 0;
  for (int i = b; i < e; ++i) s += data[i];
  lds[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over WG partial sums
  for (int o = 1; o < WG; o <<= 1) {
    int v = (tid >= o) ? lds[tid - o] : 0;
    __syncthreads();
    lds[tid] += v;
    __syncthreads();
  }
  int run = lds[tid] - s;
  const int total = lds[WG - 1];
  for (int i = b; i < e; ++i) {
    int c = data[i];
    data[i] = run;
    run += c;
  }
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------------------
// FP64 SE(3) helpers.  Pose 7-vector: t (3), unit quaternion (x, y, z, w).
__device__ __forceinline__ void quat_to_rot(const double* q, double* R) {
  const double x = q[0], y = q[1], z = q[2], w = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

// Relative pose T_ji = T_j T_i^{-1}: R = R_j R_i^T, t = t_j - R t_i.
__device__ __forceinline__ void relative_pose(const double* pi, const double* pj, double* R, double* t) {
  double Ri[9], Rj[9];
  quat_to_rot(pi + 3, Ri);
  quat_to_rot(pj + 3, Rj);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      R[3 * a + b] = Rj[3 * a] * Ri[3 * b] + Rj[3 * a + 1] * Ri[3 * b + 1] + Rj[3 * a + 2] * Ri[3 * b + 2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    t[a] = pj[a] - (R[3 * a] * pi[0] + R[3 * a + 1] * pi[1] + R[3 * a + 2] * pi[2]);
}

// T <- Exp(xi) T, xi = (rho, phi).  Exp(xi) = (R(phi), V(phi) rho) with
// Rodrigues' R = I + A K + B K^2, V = I + B K + C K^2, K = hat(phi); the
// rotation is applied to the quaternion as q_exp (x) q, then renormalised.
// Series forms of A, B, C and of the half-angle terms below theta = 1e-2.
__device__ __forceinline__ void retract_left(const double* xi, const double* pin, double* pout) {
  const double rx = xi[0], ry = xi[1], rz = xi[2];
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th2 = px * px + py * py + pz * pz;
  double A, B, C, hs, hc;
  if (th2 < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0 - th2 * th2 * th2 / 5040.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0 - th2 * th2 * th2 / 40320.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0 - th2 * th2 * th2 / 362880.0;
    hs = 0.5 - th2 / 48.0 + th2 * th2 / 3840.0;
    hc = 1.0 - th2 / 8.0 + th2 * th2 / 384.0;
  } else {
    const double th = sqrt(th2);
    const double s = sin(th), c = cos(th);
    A = s / th;
    B = (1.0 - c) / th2;
    C = (th - s) / (th2 * th);
    hs = sin(0.5 * th) / th;
    hc = cos(0.5 * th);
  }
  // K = hat(phi), K2 = K K
  const double K[9] = {0, -pz, py, pz, 0, -px, -py, px, 0};
  double K2[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      K2[3 * a + b] = K[3 * a] * K[b] + K[3 * a + 1] * K[3 + b] + K[3 * a + 2] * K[6 + b];
  double R[9], V[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    const double I = (m == 0 || m == 4 || m == 8) ? 1.0 : 0.0;
    R[m] = I + A * K[m] + B * K2[m];
    V[m] = I + B * K[m] + C * K2[m];
  }
  const double rho[3] = {rx, ry, rz};
#pragma unroll
  for (int a = 0; a < 3; ++a)
    pout[a] = R[3 * a] * pin[0] + R[3 * a + 1] * pin[1] + R[3 * a + 2] * pin[2] +
              V[3 * a] * rho[0] + V[3 * a + 1] * rho[1] + V[3 * a + 2] * rho[2];
  // q_exp = (hs * phi, hc);  q' = q_exp (x) q  (Hamilton)
  const double ax = hs * px, ay = hs * py, az = hs * pz, aw = hc;
  const double bx = pin[3], by = pin[4], bz = pin[5], bw = pin[6];
  double qx = aw * bx + bw * ax + (ay * bz - az * by);
  double qy = aw * by + bw * ay + (az * bx - ax * bz);
  double qz = aw * bz + bw * az + (ax * by - ay * bx);
  double qw = aw * bw - (ax * bx + ay * by + az * bz);
  const double inv = 1.0 / sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  pout[3] = qx * inv; pout[4] = qy * inv; pout[5] = qz * inv; pout[6] = qw * inv;
}

}  // namespace dpba
