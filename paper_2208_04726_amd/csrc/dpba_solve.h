// Reduced pose solve, depth back-substitution and retraction (FP64).
//
// With the depths eliminated (Sec. 3.1, Schur complement), the pose step of a
// window solves S dxi = -s, S = B + lambda I - E C^{-1} E^T, by a Cholesky
// factorisation; then every depth is recovered from its own row,
//   dd_k = -(w_k + sum_a E_ak^T dxi_a) / C_k,
// and the state is updated, T_a <- Exp(dxi_a) T_a for free frames and
// d_k <- d_k + dd_k.  The chunk partials of S and s are summed here in chunk
// order, so the sum is the same in every run.
#pragma once
#include "dpba_assemble.h"

namespace dpba {

constexpr int CBS_LDS = 32 * 33;   // inverse diagonal block of the blocked factorisation (and spare)
// LDS of the solve: 64 B header, A (n x (n+1)), b, x, the inverse diagonal
// block and solve scratch (the adjoint's column buffers fit in the same space).
__host__ __device__ inline int chol_lds_bytes(int n) {
  const int lda = n + 1;
  return 64 + (n * lda + 2 * n + 8) * 8 + (CBS_LDS + 2 * 128) * 8;
}

// Sum the chunk partials of window w into A (n x lda, lower) and b (n).
// With b2 (adjoint), also the depth-cotangent row: b2 = -sum_k E_k dbar_k / C_k.
// Chunks are added in chunk order, one at a time (their blocks overlap); the
// next chunk's entries are loaded into registers while the current one is
// added, so each chunk does not wait for a memory round trip.  Thread tid
// takes the entries e = tid + k WG of a chunk's lower triangle.
constexpr int GATHER_K = ((NCHOL_MAX * (NCHOL_MAX + 1)) / 2 + WG - 1) / WG;
__device__ __forceinline__ void tri_index(int e, int& r, int& c) {
  r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  if (((r + 1) * (r + 2)) / 2 <= e) ++r;
  if ((r * (r + 1)) / 2 > e) --r;
  c = e - (r * (r + 1)) / 2;
}
struct GatherChunk {
  int off, Dc;
  double v[GATHER_K];
  double vb, vb2;
};
__device__ __forceinline__ void gather_load(const Params& P, const WinDesc& W, int cc, bool adj, GatherChunk& g) {
  const int tid = threadIdx.x;
  const int c = W.chunk_off + cc;
  const int lo_free = P.cstate[2 * c], Dc = P.cstate[2 * c + 1];
  g.off = 6 * (lo_free - W.n_fixed);
  g.Dc = Dc;
  const double* part = P.partial + W.part_off + (int64_t)cc * W.part_stride;
  const int ntri = (Dc * (Dc + 1)) / 2;
#pragma unroll
  for (int k = 0; k < GATHER_K; ++k) {
    const int e = tid + k * WG;
    int r, col;
    tri_index(e, r, col);
    g.v[k] = e < ntri ? part[r * Dc + col] : 0.0;
  }
  g.vb = tid < Dc ? part[Dc * Dc + tid] : 0.0;
  g.vb2 = (adj && tid < Dc) ? part[Dc * Dc + Dc + tid] : 0.0;
}
__device__ __forceinline__ void gather_partials(const Params& P, int w, const WinDesc& W, double* A,
                                       int lda, double* b, int n, double* b2 = nullptr) {
  const int tid = threadIdx.x;
  for (int i = tid; i < n * lda; i += WG) A[i] = 0.0;
  for (int i = tid; i < n; i += WG) b[i] = 0.0;
  if (b2)
    for (int i = tid; i < n; i += WG) b2[i] = 0.0;
  __syncthreads();
  const int nc = W.n_chunks;
  const bool adj = b2 != nullptr;
  GatherChunk cur, nxt;
  int cc = 0;
  while (cc < nc && P.cstate[2 * (W.chunk_off + cc) + 1] == 0) ++cc;   // chunks without free frames
  if (cc < nc) gather_load(P, W, cc, adj, nxt);
  while (cc < nc) {
    cur = nxt;
    int cn = cc + 1;
    while (cn < nc && P.cstate[2 * (W.chunk_off + cn) + 1] == 0) ++cn;
    if (cn < nc) gather_load(P, W, cn, adj, nxt);
    const int ntri = (cur.Dc * (cur.Dc + 1)) / 2;
#pragma unroll
    for (int k = 0; k < GATHER_K; ++k) {
      const int e = tid + k * WG;
      if (e < ntri) {
        int r, col;
        tri_index(e, r, col);
        A[(cur.off + r) * lda + cur.off + col] += cur.v[k];
      }
    }
    if (tid < cur.Dc) {
      b[cur.off + tid] += cur.vb;
      if (b2) b2[cur.off + tid] += cur.vb2;
    }
    __syncthreads();
    cc = cn;
  }
}

// Cholesky of the n x n lower triangle in A (LDS), n <= 128, in place.  The
// matrix is spread over the workgroup's registers: thread (tr, tc) =
// (tid % 32, tid / 32) owns rows tr + 32 a and columns tc + 16 b.  Column k is
// published through an LDS buffer (two alternating buffers, one barrier per
// column) and every thread applies the rank-one update to its own elements.
// Writes BA_W_* bits (non-positive or non-finite pivot) to *flag (thread 0).
__device__ __forceinline__ void wg_cholesky(double* A, int lda, int n, double* colbuf, int* flag) {
  const int tid = threadIdx.x;
  const int tr = tid & 31, tc = tid >> 5;
  double Ar[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = tr + 32 * a, j = tc + 16 * b;
      Ar[a][b] = (i < n && j <= i) ? A[i * lda + j] : 0.0;
    }
  int bad = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * b + kk;
      if (k >= n) break;
      double* buf = colbuf + (k & 1) * 128;
      if (tc == kk) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = tr + 32 * a;
          if (i >= k && i < n) buf[i] = Ar[a][b];
        }
      }
      __syncthreads();
      double d = buf[k];
      if (!(d > 0.0) || !isfinite_d(d)) {
        bad |= isfinite_d(d) ? W_NOT_SPD : W_NONFINITE;
        d = 1.0;
      }
      const double lkk = sqrt(d);
      const double inv = 1.0 / lkk;
      double li[4], lj[8];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int i = tr + 32 * a;
        li[a] = (i > k && i < n) ? buf[i] * inv : 0.0;
      }
#pragma unroll
      for (int bb = 0; bb < 8; ++bb) {
        const int j = tc + 16 * bb;
        lj[bb] = (j > k && j < n) ? buf[j] * inv : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int bb = 0; bb < 8; ++bb) Ar[a][bb] -= li[a] * lj[bb];
      if (tc == kk) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = tr + 32 * a;
          if (i == k) Ar[a][b] = lkk;
          else if (i > k && i < n) Ar[a][b] = li[a];
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = tr + 32 * a, j = tc + 16 * b;
      if (i < n && j <= i) A[i * lda + j] = Ar[a][b];
    }
  if (tid == 0) *flag = bad;
}

// L L^T x = rhs by one wave (lanes hold entries l and l + 64); L in LDS.
__device__ __forceinline__ void wave_cholesky_solve(const double* A, int lda, int n, const double* rhs,
                                           double* x) {
  const int l = lane_id();
  double y0 = l < n ? rhs[l] : 0.0, y1 = l + 64 < n ? rhs[l + 64] : 0.0;
  for (int k = 0; k < n; ++k) {   // L y = rhs
    const double v = __shfl(k < 64 ? y0 : y1, k & 63, 64);
    const double yk = v / A[k * lda + k];
    if (l > k && l < n) y0 -= A[l * lda + k] * yk;
    if (l + 64 > k && l + 64 < n) y1 -= A[(l + 64) * lda + k] * yk;
    if (l == k) y0 = yk;
    if (l + 64 == k) y1 = yk;
  }
  for (int k = n - 1; k >= 0; --k) {   // L^T x = y
    const double v = __shfl(k < 64 ? y0 : y1, k & 63, 64);
    const double xk = v / A[k * lda + k];
    if (l < k) y0 -= A[k * lda + l] * xk;
    if (l + 64 < k) y1 -= A[k * lda + l + 64] * xk;
    if (l == k) y0 = xk;
    if (l + 64 == k) y1 = xk;
  }
  if (l < n) x[l] = y0;
  if (l + 64 < n) x[l + 64] = y1;
}

constexpr int CBS = 16;   // panel width of the blocked factorisation

// Lane j of each row of 16 lanes, broadcast to the whole row (DPP
// row_newbcast): a vector-register move, no round trip through scalar
// registers.  j must fold to a constant (the callers' loops are unrolled).
__device__ __forceinline__ int row_bcast_i32(int v, int j) {
  switch (j) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x150, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x151, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x152, 0xf, 0xf, false);
    case 3: return __builtin_amdgcn_mov_dpp(v, 0x153, 0xf, 0xf, false);
    case 4: return __builtin_amdgcn_mov_dpp(v, 0x154, 0xf, 0xf, false);
    case 5: return __builtin_amdgcn_mov_dpp(v, 0x155, 0xf, 0xf, false);
    case 6: return __builtin_amdgcn_mov_dpp(v, 0x156, 0xf, 0xf, false);
    case 7: return __builtin_amdgcn_mov_dpp(v, 0x157, 0xf, 0xf, false);
    case 8: return __builtin_amdgcn_mov_dpp(v, 0x158, 0xf, 0xf, false);
    case 9: return __builtin_amdgcn_mov_dpp(v, 0x159, 0xf, 0xf, false);
    case 10: return __builtin_amdgcn_mov_dpp(v, 0x15a, 0xf, 0xf, false);
    case 11: return __builtin_amdgcn_mov_dpp(v, 0x15b, 0xf, 0xf, false);
    case 12: return __builtin_amdgcn_mov_dpp(v, 0x15c, 0xf, 0xf, false);
    case 13: return __builtin_amdgcn_mov_dpp(v, 0x15d, 0xf, 0xf, false);
    case 14: return __builtin_amdgcn_mov_dpp(v, 0x15e, 0xf, 0xf, false);
    default: return __builtin_amdgcn_mov_dpp(v, 0x15f, 0xf, 0xf, false);
  }
}
// FP64: one 64-bit DPP move (gfx950 moves 64-bit values with row_newbcast).
__device__ __forceinline__ double row_bcast_f64(double v, int j) {
  switch (j) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x150, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x151, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x152, 0xf, 0xf, false);
    case 3: return __builtin_amdgcn_mov_dpp(v, 0x153, 0xf, 0xf, false);
    case 4: return __builtin_amdgcn_mov_dpp(v, 0x154, 0xf, 0xf, false);
    case 5: return __builtin_amdgcn_mov_dpp(v, 0x155, 0xf, 0xf, false);
    case 6: return __builtin_amdgcn_mov_dpp(v, 0x156, 0xf, 0xf, false);
    case 7: return __builtin_amdgcn_mov_dpp(v, 0x157, 0xf, 0xf, false);
    case 8: return __builtin_amdgcn_mov_dpp(v, 0x158, 0xf, 0xf, false);
    case 9: return __builtin_amdgcn_mov_dpp(v, 0x159, 0xf, 0xf, false);
    case 10: return __builtin_amdgcn_mov_dpp(v, 0x15a, 0xf, 0xf, false);
    case 11: return __builtin_amdgcn_mov_dpp(v, 0x15b, 0xf, 0xf, false);
    case 12: return __builtin_amdgcn_mov_dpp(v, 0x15c, 0xf, 0xf, false);
    case 13: return __builtin_amdgcn_mov_dpp(v, 0x15d, 0xf, 0xf, false);
    case 14: return __builtin_amdgcn_mov_dpp(v, 0x15e, 0xf, 0xf, false);
    default: return __builtin_amdgcn_mov_dpp(v, 0x15f, 0xf, 0xf, false);
  }
}

// 1/sqrt(x) for x > 0 in FP64: the hardware estimate refined by two Newton
// steps (within a few ulps).
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Factorisation of one diagonal block by wave 0 (lane l < kb holds row l,
// loaded by the caller into Lr; lanes kb.. hold identity rows), followed by
// the inverse of the factor.  The factor's rows are written to Ld (row stride
// ldd), the reciprocals of its diagonal to dinv, and Linv (LDS, CBS x CBS,
// row stride CBS + 1) receives L^{-1} (lower, zeros elsewhere).  Lane values
// are exchanged by broadcasts within the first row of 16 lanes (the other
// rows compute on their own lanes' values, which are never stored); the
// updates are branch-free (entries above the diagonal hold garbage that is
// never read).  Pivot problems accumulate BA_W_* bits into bad (meaningful in
// lanes below 16).
__device__ __forceinline__ void wave_factor_invert(double (&Lr)[CBS], int kb, double* Ld, int ldd,
                                          double* Linv, double* dinv, int& bad) {
  const int lane = lane_id();
  // Column `lane` of L^{-1}, X[i][j] = (delta_ij - sum_{k<i} L[i][k] X[k][j]) / L[i][i],
  // accumulated alongside the factorisation: column k of L, broadcast once at
  // step k, updates both the trailing rows and the pending X[i] (i > k), in
  // the same order (k ascending) as the row-by-row recurrence.
  double ilv[CBS], Xc[CBS];
#pragma unroll
  for (int i = 0; i < CBS; ++i) Xc[i] = (lane == i) ? 1.0 : 0.0;
#pragma unroll
  for (int kk = 0; kk < CBS; ++kk) {
    double piv = row_bcast_f64(Lr[kk], kk);
    if (!(piv > 0.0) || !isfinite_d(piv)) {
      bad |= isfinite_d(piv) ? W_NOT_SPD : W_NONFINITE;
      piv = 1.0;
    }
    const double il = rsqrt_f64(piv);
    ilv[kk] = il;
    Lr[kk] = (lane == kk) ? piv * il : Lr[kk] * il;
    Xc[kk] = (lane <= kk) ? Xc[kk] * il : 0.0;
#pragma unroll
    for (int jj = kk + 1; jj < CBS; ++jj) {
      const double c = row_bcast_f64(Lr[kk], jj);   // L[jj][kk]
      Lr[jj] -= Lr[kk] * c;
      Xc[jj] -= c * Xc[kk];
    }
    // finish each step before the next (empty statements that take the rows
    // as operands): scheduled ahead along the pivot chain, the other
    // updates' broadcasts would all wait in registers
#pragma unroll
    for (int q = 0; q < CBS; q += 4) {
      asm volatile("" : "+v"(Lr[q]), "+v"(Lr[q + 1]), "+v"(Lr[q + 2]), "+v"(Lr[q + 3]));
      asm volatile("" : "+v"(Xc[q]), "+v"(Xc[q + 1]), "+v"(Xc[q + 2]), "+v"(Xc[q + 3]));
    }
  }
  if (lane < kb) {
#pragma unroll
    for (int t = 0; t < CBS; ++t)
      if (t <= lane) Ld[lane * ldd + t] = Lr[t];
    double d = 0.0;
#pragma unroll
    for (int t = 0; t < CBS; ++t) d = (t == lane) ? ilv[t] : d;
    dinv[lane] = d;
  }
  if (lane < CBS) {
#pragma unroll
    for (int i = 0; i < CBS; ++i) Linv[i * (CBS + 1) + lane] = (i < kb) ? Xc[i] : 0.0;
  }
}

// Rows below a diagonal block: X = A_rows L^{-T}, 16 rows per wave step with
// 16x16x4 FP64 matrix-core products (K = 32).  rows(r) returns the address of
// column k0 of row r (r < m) of the source; results go to dst(r) (and, when
// given, to a second destination).  Rows are read before they are written by
// the same wave, so the product may be in place.  trsm_row_block forms row
// block rb (rows 16 rb ..) with the calling wave; panel_trsm_mfma deals the
// blocks to the waves.
template <typename Src, typename Dst, typename Dst2>
__device__ __forceinline__ void trsm_row_block(int rb, int m, int kb, const double* Linv, Src rows, Dst dst, Dst2 dst2,
                                               int* nzb) {
  const int lane = lane_id();
  const int l16 = lane & 15, g = lane >> 4;
  const int ra = min(16 * rb + l16, m - 1);   // operand row (clamped; extra rows not stored)
  const double* src = rows(ra);
  double av[CBS / 4];
#pragma unroll
  for (int kq = 0; kq < CBS / 4; ++kq) {
    const int k = 4 * kq + g;
    av[kq] = k < kb ? src[k] : 0.0;
  }
  f64x4 acc[CBS / 16];
#pragma unroll
  for (int h = 0; h < CBS / 16; ++h) acc[h] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kq = 0; kq < CBS / 4; ++kq) {
    const int k = 4 * kq + g;
#pragma unroll
    for (int h = 0; h < CBS / 16; ++h) acc[h] = mfma16(av[kq], Linv[(16 * h + l16) * (CBS + 1) + k], acc[h]);
  }
  bool nz = false;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * rb + acc_row(0.0, g, r);
    if (row < m) {
#pragma unroll
      for (int h = 0; h < CBS / 16; ++h) {
        if (16 * h + l16 < kb) {
          dst(row)[16 * h + l16] = acc[h][r];
          dst2(row, 16 * h + l16, acc[h][r]);
          nz |= acc[h][r] != 0.0;
        }
      }
    }
  }
  // row blocks whose panel entries are all zero (outside the envelope of
  // the matrix: frames that share no patch) contribute nothing to the
  // trailing update, which then skips their tiles
  const bool any = __any(nz);
  if (lane == 0) nzb[rb] = any ? 1 : 0;
}
template <typename Src, typename Dst, typename Dst2>
__device__ __forceinline__ void panel_trsm_mfma(int m, int kb, const double* Linv, Src rows, Dst dst, Dst2 dst2,
                                       int* nzb) {
  const int nblk = (m + 15) / 16;
  for (int rb = wave_id(); rb < nblk; rb += NWAVES) trsm_row_block(rb, m, kb, Linv, rows, dst, dst2, nzb);
}

// Blocked right-looking Cholesky of the augmented (n+1) x (n+1) matrix in LDS
// (lower triangle of rows 0..n-1, row n = right-hand side b): on return rows
// < n hold L and row n holds y = L^{-1} b, so the forward substitution is
// folded into the factorisation.  Per CBS-column panel:
//   * wave 0 factorises the diagonal block in registers (lane l = row l) and
//     inverts the factor;
//   * the rows below it, the right-hand side included, become A L^{-T}
//     (matrix-core products);
//   * the trailing lower triangle is updated with 16x16x4 FP64 matrix-core
//     products whose operands are read straight from the matrix.
// Linv: CBS * (CBS + 1) doubles of LDS.  Pivot problems set BA_W_* bits in *flag.
__device__ __forceinline__ void wg_cholesky_lds(double* A, int lda, int n, double* Linv, double* dinv, int* flag) {
  const int lane = lane_id(), wv = wave_id();
  int* nzb = (int*)(Linv + CBS * (CBS + 1));   // 32 row-block flags
  int bad = 0;
  // factor and invert the diagonal block at k0 (wave 0)
  auto factor = [&](int k0) {
    const int kb = min(CBS, n - k0);
    double Lr[CBS];
#pragma unroll
    for (int t = 0; t < CBS; ++t)
      Lr[t] = (lane < kb && t <= lane) ? A[(k0 + lane) * lda + k0 + t] : (t == lane ? 1.0 : 0.0);
    wave_factor_invert(Lr, kb, A + k0 * lda + k0, lda, Linv, dinv + k0, bad);
  };
  if (wv == 0) factor(0);
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += CBS) {
    const int kb = min(CBS, n - k0);
    const int r0 = k0 + kb;
    const int m = n + 1 - r0;
    auto rows = [&](int r) { return (const double*)(A + (r0 + r) * lda + k0); };
    auto dst = [&](int r) { return A + (r0 + r) * lda + k0; };
    auto none = [](int, int, double) {};
    panel_trsm_mfma(m, kb, Linv, rows, dst, none, nzb);
    __syncthreads();
    if (m > 1) {
      // kb == CBS here (a shorter panel is the last one, with m == 1)
      const int T = (m + 15) / 16;
      const int ntile = T * (T + 1) / 2;
      const int l16 = lane & 15, g = lane >> 4;
      auto update = [&](int t) {
        int ti = 0;
        while (((ti + 1) * (ti + 2)) / 2 <= t) ++ti;
        const int tj = t - (ti * (ti + 1)) / 2;
        if (!nzb[ti] || !nzb[tj]) return;
        f64x4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * ti + acc_row(0.0, g, r), col = 16 * tj + l16;
          const bool ok = row < m && col <= row && r0 + col < n;
          acc[r] = ok ? A[(r0 + row) * lda + r0 + col] : 0.0;
        }
        // operand rows past the matrix read its last row; their products land
        // in accumulator entries that are not stored
        const double* pa = A + min(r0 + 16 * ti + l16, n) * lda + k0 + g;
        const double* pb = A + min(r0 + 16 * tj + l16, n) * lda + k0 + g;
#pragma unroll
        for (int kq = 0; kq < CBS / 4; ++kq) acc = mfma16(-pa[4 * kq], pb[4 * kq], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * ti + acc_row(0.0, g, r), col = 16 * tj + l16;
          if (row < m && col <= row && r0 + col < n) A[(r0 + row) * lda + r0 + col] = acc[r];
        }
      };
      // Look-ahead: wave 0 updates the leading tile, which holds the next
      // diagonal block, and factors that block while the other waves update
      // the rest of the trailing matrix.
      if (wv == 0) {
        update(0);
        wave_sync();
        if (r0 < n) factor(r0);
      } else {
        for (int t = wv; t < ntile; t += NWAVES - 1) update(t);
      }
    }
    __syncthreads();
  }
  if (wv == 0 && lane == 0) *flag = bad;
  __syncthreads();
}

// L^T x = y with L and y (row n) from wg_cholesky_lds; x in LDS.  z: n doubles
// of LDS scratch.
__device__ __forceinline__ void wg_backsolve_lds(const double* A, int lda, int n, const double* dinv, double* x,
                                        double* z) {
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  for (int j = tid; j < n; j += WG) z[j] = A[n * lda + j];
  __syncthreads();
  const int nb = (n + CBS - 1) / CBS;
  for (int bk = nb - 1; bk >= 0; --bk) {
    const int b0 = bk * CBS, bs = min(CBS, n - b0);
    if (wv == 0) {
      double Lc[CBS];
#pragma unroll
      for (int s2 = 0; s2 < CBS; ++s2)
        Lc[s2] = (lane < bs && s2 < bs && s2 >= lane) ? A[(b0 + s2) * lda + b0 + lane] : 0.0;
      double zz = lane < bs ? z[b0 + lane] : 0.0;
#pragma unroll
      for (int s2 = CBS - 1; s2 >= 0; --s2) {
        if (s2 < bs) {
          const double xs = row_bcast_f64(zz, s2) * dinv[b0 + s2];
          if (lane == s2) zz = xs;
          else if (lane < s2) zz -= Lc[s2] * xs;
        }
      }
      if (lane < bs) x[b0 + lane] = zz;
    }
    __syncthreads();
    for (int j = tid; j < b0; j += WG) {
      double v = z[j];
      for (int s2 = 0; s2 < bs; ++s2) v -= A[(b0 + s2) * lda + j] * x[b0 + s2];
      z[j] = v;
    }
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ void wg_chol(const Params& P, int w, int iter, char* smem) {
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x;
  int* misc = (int*)smem;
  const int st = wg_bcast_status(P.status, w, misc);
  const int N = W.n_frames, nfix = W.n_fixed;
  const int n = 6 * (N - nfix);
  const double* poses = state_poses<T>(P, W, iter);
  double* next = P.pose_buf + (int64_t)(iter + 1) * 7 * P.n_frames_total + 7 * W.frame_off;
  double* dxi = P.dxi + 6 * W.frame_off;
  if (st != 0) {
    for (int i = tid; i < 6 * N; i += WG) dxi[i] = 0.0;
    return;
  }
  const int lda = n + 1;
  double* A = (double*)(smem + 64);
  double* b = A + n * lda;
  double* x = b + n;
  double* colbuf = x + n + 8;
  if (n > 0) {
    gather_partials(P, w, W, A, lda, b, n);
    for (int i = tid; i < n; i += WG) {
      A[i * lda + i] += P.lambda;
      b[i] = -b[i];
    }
    __syncthreads();
    // colbuf: the inverse diagonal block, 32 row-block flags, the reciprocal
    // diagonal of L, then n doubles of solve scratch
    wg_cholesky_lds(A, lda, n, colbuf, colbuf + CBS * (CBS + 1) + 16, misc + 1);
    wg_backsolve_lds(A, lda, n, colbuf + CBS * (CBS + 1) + 16, x, colbuf + CBS * (CBS + 1) + 16 + NCHOL_MAX);
    __syncthreads();
    if (tid == 0) misc[2] = misc[1];
    __syncthreads();
    if (tid < n && !isfinite_d(x[tid])) atomicOr(&misc[2], W_NONFINITE);
    __syncthreads();
    if (tid == 0 && misc[2]) atomicOr(&P.status[w], misc[2]);
  } else if (tid == 0) {
    misc[2] = 0;
  }
  __syncthreads();
  const int bad = misc[2];
  for (int i = tid; i < 6 * N; i += WG) {
    const int a = i / 6;
    dxi[i] = (a >= nfix && !bad) ? x[6 * (a - nfix) + i % 6] : 0.0;
  }
  for (int a = tid; a < N; a += WG) {
    const double* p = poses + 7 * a;
    double* q = next + 7 * a;
    if (a >= nfix && !bad) {
      retract_left(x + 6 * (a - nfix), p, q);
    } else {
      for (int m = 0; m < 7; ++m) q[m] = p[m];
    }
  }
}

// dd_k for the chunk's patches, from the same staged sub-batches as the
// assembly; writes the depth state (position order) or, on the last
// iteration, depth_out (patch order).
template <typename T>
__device__ __forceinline__ void wg_backsub(const Params& P, int c, int part, int nparts, int iter, char* smem,
                                           int Rcap) {
  double* lp = (double*)smem;
  T* rel = (T*)(smem + al16(Rcap * 7 * 8));
  double* dx = (double*)(smem + backsub_dx_offset(Rcap, (int)sizeof(T)));
  double* dl = (double*)(smem + backsub_delta_offset(Rcap, (int)sizeof(T)));
  const int o = backsub_stage_offset(Rcap, (int)sizeof(T));
  Stage<T> S(smem + o);
  int* misc = (int*)(smem + o + stage_bytes((int)sizeof(T)));
  const ChunkDesc cd = P.chunk[c];
  const int w = cd.window;
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const bool last = iter == P.iterations - 1;
  const int st = wg_bcast_status(P.status, w, misc);
  const int32_t* acnt = P.acnt + W.frame_off + w;
  const int32_t* plist = P.plist + W.patch_off;
  if (st != 0) {
    if (last && part == 0) {
      // failed window: its outputs are its inputs
      if (!(st & W_BAD_INDEX)) {
        for (int q = acnt[cd.a_lo] + tid; q < acnt[cd.a_hi]; q += WG) {
          const int k = plist[q];
          P.depth_out[W.patch_off + k] = P.patches_in[3 * (W.patch_off + k) + 2];
        }
      } else if (cd.a_lo == 0) {
        for (int k = tid; k < W.n_patches; k += WG)
          P.depth_out[W.patch_off + k] = P.patches_in[3 * (W.patch_off + k) + 2];
      }
    }
    return;
  }
  const int N = W.n_frames;
  const double* poses = state_poses<T>(P, W, iter);
  for (int i = tid; i < 7 * N; i += WG) lp[i] = poses[i];
  for (int i = tid; i < 6 * N; i += WG) dx[i] = P.dxi[6 * W.frame_off + i];
  const int32_t* ar = P.arange + 2 * W.frame_off;
  int* arng = misc + 16;   // target frame ranges of the chunk's source frames
  for (int i = tid; i < 2 * (cd.a_hi - cd.a_lo); i += WG) arng[i] = ar[2 * cd.a_lo + i];
  const int32_t* sbs = P.sbstart + W.frame_off + w;
  const int4* sbd = P.sbd + W.sb_off;
  const WinEdges we = win_edges(P, W, P.wmeta[4 * w + 1], (int)sizeof(T));
  const T fx = (T)W.fx, fy = (T)W.fy, cx = (T)W.cx, cy = (T)W.cy;
  const T zmin = (T)P.z_min, lam = (T)P.lambda;
  const int SEG = seg_width(P.wmeta[4 * w]);
  const int SBw = sb_width(SEG);
  const int segs = 64 / SEG;
  const int spw = SBw / NWAVES;
  const int npass = (spw + segs - 1) / segs;
  const int lseg = lane & (SEG - 1), sidx = lane / SEG;
  // this workgroup's share of the chunk's sub-batches (patches are
  // independent here)
  const int c_lo = sbs[cd.a_lo], c_n = sbs[cd.a_hi] - c_lo;
  const int s_lo = c_lo + (c_n * part) / nparts, s_hi = c_lo + (c_n * (part + 1)) / nparts;
  if (s_lo >= s_hi) return;

  StageRegs<T> R;
  int4 dcur = sbd[s_lo], dnxt = dcur;
  if (s_lo + 1 < s_hi) dnxt = sbd[s_lo + 1];
  stage_issue<T>(P, W, w, we, dcur, iter, nullptr, R);
  __syncthreads();
  stage_store<T>(dcur, R, S, false);
  int a = -1;
  double* dnext = state_depth(P, W, iter + 1);
  for (int s = s_lo; s < s_hi; ++s) {
    const int an = (dcur.y >> 8) & 0xff, nsb = dcur.y & 255, pos0 = dcur.x;
    if (an != a) {
      a = an;
      const int lo = arng[2 * (a - cd.a_lo)], hi = arng[2 * (a - cd.a_lo) + 1];
      // relative poses, and since E_ik^T dx_a = -sum_j E_jk^T Ad(T_ja) dx_a,
      // per target frame the vector dx_j - Ad(T_ja) dx_a, so an edge adds
      // E_jk^T (dx_j - Ad dx_a)
      for (int j = lo + tid; j <= hi; j += WG) {
        double R[9], t[3];
        relative_pose(lp + 7 * a, lp + 7 * j, R, t);
        store_relpose<T>(R, t, rel + j * RELW);
        const double* xa = dx + 6 * a;
        double Rp[3], Rr[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          Rr[r] = R[3 * r] * xa[0] + R[3 * r + 1] * xa[1] + R[3 * r + 2] * xa[2];
          Rp[r] = R[3 * r] * xa[3] + R[3 * r + 1] * xa[4] + R[3 * r + 2] * xa[5];
        }
        // Ad (rho, phi) = (R rho + t x (R phi), R phi)
        const double ad[6] = {Rr[0] + t[1] * Rp[2] - t[2] * Rp[1], Rr[1] + t[2] * Rp[0] - t[0] * Rp[2],
                              Rr[2] + t[0] * Rp[1] - t[1] * Rp[0], Rp[0], Rp[1], Rp[2]};
#pragma unroll
        for (int m = 0; m < 6; ++m) dl[6 * j + m] = dx[6 * j + m] - ad[m];
      }
    }
    int dnn = 0;
    const bool pre = s + 2 < s_hi;
    if (s + 1 < s_hi) stage_issue<T>(P, W, w, we, dnxt, iter, nullptr, R);
    if (pre) dnn = desc_prefetch(sbd + s + 2);
    lds_barrier();
    for (int ps = 0; ps < npass; ++ps) {
      const int slot_in_wave = ps * segs + sidx;
      const LaneEdge<T> le = lane_edge<T>(S, wv * spw + slot_in_wave, slot_in_wave < spw, nsb, lseg, a);
      EdgeOut<T> eo;
      const int j = le.j;
      linearize_edge<T, false>(rel + j * RELW, le.xb, le.yb, (T)le.d, le.t0, le.t1, le.w0, le.w1, fx,
                               fy, cx, cy, zmin, le.has && (j != a), eo);
      double t = 0.0;
      if (eo.active) {
        const double* dj = dl + 6 * j;
#pragma unroll
        for (int m = 0; m < 6; ++m) t += (double)eo.Ej[m] * dj[m];
      }
      T red[2] = {eo.cd, eo.wd};
      seg_sum_n<2>(red, SEG);
      const double tk = seg_sum(t, SEG);
      const T Ck = lam + red[0];
      const T Wk = red[1];
      if (le.pv && lseg == 0) {
        const double dnew = le.d - ((double)Wk + tk) / (double)Ck;
        if (last) P.depth_out[W.patch_off + S.pk[le.slot]] = dnew;
        else dnext[pos0 + le.slot] = dnew;
      }
    }
    lds_barrier();
    if (s + 1 < s_hi) stage_store<T>(dnxt, R, S, false);
    dcur = dnxt;
    {
      // taken on every path, so no load is in flight into the next iteration
      const int4 dt = desc_take(dnn);
      if (pre) dnxt = dt;
    }
  }
}

// Final poses: the last state, or the inputs of a failed window.
__device__ __forceinline__ void wg_finalize(const Params& P, int w) {
  const WinDesc W = P.win[w];
  const int st = P.status[w];
  const double* src = (st != 0 || P.iterations == 0)
                          ? P.poses_in + 7 * W.frame_off
                          : P.pose_buf + (int64_t)P.iterations * 7 * P.n_frames_total + 7 * W.frame_off;
  double* dst = P.poses_out + 7 * W.frame_off;
  for (int i = threadIdx.x; i < 7 * W.n_frames; i += WG) dst[i] = src[i];
  if (P.iterations == 0)
    for (int k = threadIdx.x; k < W.n_patches; k += WG)
      P.depth_out[W.patch_off + k] = P.patches_in[3 * (W.patch_off + k) + 2];
}

}  // namespace dpba
