// Reduced pose solve for windows with more than 21 free frames (n > 126):
// the depth-eliminated system (Sec. 3.1, Schur complement) no longer fits in
// the LDS of one workgroup, so it is summed into an (n+1) x (n+1) FP64 matrix
// in device memory (row n carries the right-hand side -s) by many
// workgroups, then factorised in place by one workgroup per window with a
// blocked right-looking Cholesky:
//   * each 16 x 16 diagonal block is factorised and inverted by one wave;
//   * the rows below it (the right-hand-side row included, which folds the
//     forward substitution L y = -s into the factorisation) are multiplied by
//     the inverse with matrix-core products;
//   * the trailing lower triangle is updated with 16x16x4 FP64 matrix-core
//     products from the panel held in LDS.
// The back substitution L^T dxi = y runs by 16-row blocks from the bottom,
// then the free poses are retracted as in the small-window solve.
#pragma once
#include "dpba_solve.h"

namespace dpba {

constexpr int NBIG_MAX = 6 * RMAX;   // reduced system size of a 64-frame window
constexpr int CB = CBS;              // panel width
constexpr int PLD = CB + 1;          // LDS row stride of the panel
constexpr int GT = 64;               // gather tile

// 64 x 64 lower tiles of the augmented (n+1) square.
__host__ __device__ inline int gather_tiles(int n) {
  const int t = (n + 1 + GT - 1) / GT;
  return t * (t + 1) / 2;
}
__host__ __device__ inline int big_ld(int rcap) { return 6 * rcap + 1; }

// LDS: panel ((n+1) rows padded to 16, CB columns), the diagonal block's
// factor and its inverse, row-block flags, the right-hand side / solution,
// the reciprocal diagonal of L.
__host__ __device__ inline int chol_big_lds_bytes(int n) {
  const int rows = ((n + 1 + 15) / 16) * 16;
  return 64 + (rows * PLD + 2 * CB * PLD + 16 + 3 * (n + 8)) * 8;
}

// One 64 x 64 tile of the augmented system of window w, summed from the chunk
// partials in chunk order (the order of the small-window gather):
// rows < n hold S + lambda I (lower triangle), row n holds -s.
__device__ __forceinline__ void wg_gather_big(const Params& P, int w, int tile) {
  const WinDesc W = P.win[w];
  const int nfix = W.n_fixed;
  const int n = 6 * (W.n_frames - nfix);
  if (n <= NCHOL_MAX || P.status[w] != 0) return;
  if (tile >= gather_tiles(n)) return;
  int bi = 0;
  while (((bi + 1) * (bi + 2)) / 2 <= tile) ++bi;
  const int bj = tile - (bi * (bi + 1)) / 2;
  const int ld = P.ld_big;
  double* A = P.s_big + (int64_t)w * ld * ld;
  constexpr int EPT = GT * GT / WG;   // elements per thread
  double v[EPT];
  int rr[EPT], cc_[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = threadIdx.x + u * WG;
    rr[u] = GT * bi + e / GT;
    cc_[u] = GT * bj + e % GT;
    v[u] = 0.0;
  }
  const int r_lo = GT * bi, r_hi = min(GT * bi + GT - 1, n);
  const int c_lo = GT * bj, c_hi = min(GT * bj + GT - 1, n - 1);
  // chunks in order; a chunk whose columns miss the tile, or whose rows miss
  // it (the right-hand-side row n belongs to every chunk), is skipped
  for (int cc = 0; cc < W.n_chunks; ++cc) {
    const int ci = W.chunk_off + cc;
    const int lo_free = P.cstate[2 * ci], Dc = P.cstate[2 * ci + 1];
    if (Dc == 0) continue;
    const int off = 6 * (lo_free - nfix);
    if (c_hi < off || c_lo >= off + Dc) continue;
    if (!(r_hi >= off && r_lo < off + Dc) && !(r_lo <= n && n <= r_hi)) continue;
    const double* part = P.partial + W.part_off + (int64_t)cc * W.part_stride;
    double a[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int r = rr[u], c = cc_[u];
      a[u] = 0.0;
      if (r <= n && c <= r && c < n && c >= off && c < off + Dc) {
        if (r == n) a[u] = part[Dc * Dc + (c - off)];
        else if (r < off + Dc) a[u] = part[(r - off) * Dc + (c - off)];
      }
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) v[u] += a[u];
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int r = rr[u], c = cc_[u];
    if (r > n || c > r || c >= n) continue;
    A[(int64_t)r * ld + c] = (r == n) ? -v[u] : (r == c ? v[u] + P.lambda : v[u]);
  }
}

// Blocked Cholesky of the augmented matrix A (lower, ld) in place; on return
// rows < n hold L and row n holds y = L^{-1} b.  Pivot problems set BA_W_*
// bits in *flag.  Per 16-column panel: wave 0 factorises and inverts the
// diagonal block; the rows below become A L^{-T} (matrix-core products, kept
// in the LDS panel and written back); the trailing lower triangle is updated
// from the LDS panel, four 16x16 tiles per wave in flight.
__device__ __forceinline__ void wg_cholesky_big(double* A, int ld, int n, char* smem, double* dinv, int* flag) {
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int rows_pad = ((n + 1 + 15) / 16) * 16;
  double* Pn = (double*)(smem + 64);           // panel rows below the diagonal block
  double* Linv = Pn + rows_pad * PLD;          // inverse of the diagonal block
  double* Ld = Linv + CB * PLD;                // the diagonal block's factor
  int* nzb = (int*)(Ld + CB * PLD);            // nonzero flags of the panel's row blocks
  int bad = 0;
  for (int k0 = 0; k0 < n; k0 += CB) {
    const int kb = min(CB, n - k0);
    const int r0 = k0 + kb;             // first row below the block
    const int m = n + 1 - r0;           // rows below, the right-hand-side row included
    if (wv == 0) {
      double Lr[CB];
#pragma unroll
      for (int t = 0; t < CB; ++t)
        Lr[t] = (lane < kb && t <= lane) ? A[(int64_t)(k0 + lane) * ld + k0 + t] : (t == lane ? 1.0 : 0.0);
      wave_factor_invert(Lr, kb, Ld, PLD, Linv, dinv + k0, bad);
      if (lane < kb) {
#pragma unroll
        for (int t = 0; t < CB; ++t)
          if (t <= lane) A[(int64_t)(k0 + lane) * ld + k0 + t] = Lr[t];
      }
    }
    // zero the panel rows past the matrix (operands of the last tiles)
    for (int i = m + tid; i < rows_pad - r0; i += WG)
#pragma unroll
      for (int t = 0; t < CB; ++t) Pn[i * PLD + t] = 0.0;
    __syncthreads();
    {
      auto rows = [&](int r) { return (const double*)(A + (int64_t)(r0 + r) * ld + k0); };
      auto dst = [&](int r) { return Pn + r * PLD; };
      auto dst2 = [&](int r, int c, double v) { A[(int64_t)(r0 + r) * ld + k0 + c] = v; };
      panel_trsm_mfma(m, kb, Linv, rows, dst, dst2, nzb);
    }
    __syncthreads();
    // ---- trailing update A[r][c] -= sum_t P[r][t] P[c][t], c <= r, c < n
    if (m > 1) {
      const int T = (m + 15) / 16;
      const int ntile = T * (T + 1) / 2;
      const int l16 = lane & 15, g = lane >> 4;
      constexpr int TU = 4;   // tiles per wave in flight
      for (int t0 = wv; t0 < ntile; t0 += TU * NWAVES) {
        f64x4 acc[TU];
        int ti[TU], tj[TU];
        bool has[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
          const int t = t0 + u * NWAVES;
          int a = 0;
          while (((a + 1) * (a + 2)) / 2 <= t) ++a;
          ti[u] = a;
          tj[u] = t - (a * (a + 1)) / 2;
          has[u] = t < ntile && nzb[ti[u]] && nzb[tj[u]];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * ti[u] + acc_row(0.0, g, r), col = 16 * tj[u] + l16;
            const bool ok = has[u] && row < m && col <= row && r0 + col < n;
            acc[u][r] = ok ? A[(int64_t)(r0 + row) * ld + r0 + col] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < TU; ++u) {
          if (has[u]) {
            const double* pa = Pn + (16 * ti[u] + l16) * PLD + g;
            const double* pb = Pn + (16 * tj[u] + l16) * PLD + g;
#pragma unroll
            for (int kq = 0; kq < CB / 4; ++kq) acc[u] = mfma16(-pa[4 * kq], pb[4 * kq], acc[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < TU; ++u) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * ti[u] + acc_row(0.0, g, r), col = 16 * tj[u] + l16;
            if (has[u] && row < m && col <= row && r0 + col < n)
              A[(int64_t)(r0 + row) * ld + r0 + col] = acc[u][r];
          }
        }
      }
    }
    __syncthreads();
  }
  if (wv == 0 && lane == 0) *flag = bad;
  __syncthreads();
}

// L^T x = y, L in A (lower, ld), y = row n of A; x into LDS `x` (n entries).
__device__ __forceinline__ void wg_backsolve_big(const double* A, int ld, int n, const double* dinv, double* x,
                                        double* z) {
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  for (int j = tid; j < n; j += WG) z[j] = A[(int64_t)n * ld + j];
  __syncthreads();
  const int nb = (n + CB - 1) / CB;
  for (int b = nb - 1; b >= 0; --b) {
    const int b0 = b * CB, bs = min(CB, n - b0);
    if (wv == 0) {
      // lane t holds column t of the diagonal block and z_t
      double Lc[CB];
#pragma unroll
      for (int s = 0; s < CB; ++s) Lc[s] = (lane < bs && s < bs && s >= lane) ? A[(int64_t)(b0 + s) * ld + b0 + lane] : 0.0;
      double zz = lane < bs ? z[b0 + lane] : 0.0;
#pragma unroll
      for (int s = CB - 1; s >= 0; --s) {
        if (s < bs) {
          const double xs = readlane_f64(zz, s) * dinv[b0 + s];
          if (lane == s) zz = xs;
          else if (lane < s) zz -= Lc[s] * xs;
        }
      }
      if (lane < bs) x[b0 + lane] = zz;
    }
    __syncthreads();
    for (int j = tid; j < b0; j += WG) {
      double v = z[j];
      for (int s = 0; s < bs; ++s) v -= A[(int64_t)(b0 + s) * ld + j] * x[b0 + s];
      z[j] = v;
    }
    __syncthreads();
  }
}

// Solve and retraction of a window with n > 126 (the system was gathered by
// wg_gather_big).
template <typename T>
__device__ __forceinline__ void wg_chol_big(const Params& P, int w, int iter, char* smem) {
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
  const int ld = P.ld_big;
  double* A = P.s_big + (int64_t)w * ld * ld;
  const int rows_pad = ((n + 1 + 15) / 16) * 16;
  double* x = (double*)(smem + 64) + rows_pad * PLD + 2 * CB * PLD + 16;
  double* z = x + n + 8;
  double* dinv = z + n + 8;
  wg_cholesky_big(A, ld, n, smem, dinv, misc + 1);
  wg_backsolve_big(A, ld, n, dinv, x, z);
  if (tid == 0) {
    int bad = misc[1];
    for (int i = 0; i < n; ++i)
      if (!isfinite_d(x[i])) bad |= W_NONFINITE;
    misc[2] = bad;
    if (bad) atomicOr(&P.status[w], bad);
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
    if (a >= nfix && !bad) retract_left(x + 6 * (a - nfix), p, q);
    else
      for (int m = 0; m < 7; ++m) q[m] = p[m];
  }
}

}  // namespace dpba
