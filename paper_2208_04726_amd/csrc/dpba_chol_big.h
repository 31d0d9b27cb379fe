// Reduced pose solve for windows with more than 21 free frames (n > 126):
// the depth-eliminated system (Sec. 3.1, Schur complement) no longer fits in
// the LDS of one workgroup, so it is summed into an (n+1) x (n+1) FP64 matrix
// in device memory (row n carries the right-hand side -s) by many
// workgroups, then factorised in place by a blocked right-looking Cholesky
// with one launch per 32-column panel j (two 16-column sub-blocks):
//   * one workgroup per window applies panel j-1 to column block j in LDS;
//     per sub-block it factorises and inverts the 16 x 16 diagonal block
//     (one wave) and turns the rows below it (the right-hand-side row
//     included, which folds the forward substitution L y = -s into the
//     factorisation) into A L^{-T} with matrix-core products, the first
//     sub-block's rows updating the second's columns in between (with a
//     look-ahead: the second diagonal block is factorised while the other
//     waves finish the first sub-block's rows);
//   * in the same launch, many more workgroups apply panel j-1 to the rest
//     of the trailing lower triangle (16x16x4 FP64 matrix-core products),
//     so the update of a window is spread over the chip instead of one CU.
// Every entry receives the same products in the same order as in a
// one-workgroup factorisation with 16-column panels.  The back substitution L^T dxi = y runs by
// 16-row blocks from the bottom, then the free poses are retracted as in the
// small-window solve.
#pragma once
#include "dpba_solve.h"

namespace dpba {

constexpr int NBIG_MAX = 6 * RMAX;   // reduced system size of a 64-frame window
constexpr int CB = CBS;              // sub-block width
constexpr int PLD = CB + 1;          // LDS row stride of a diagonal block's inverse
constexpr int GT = 64;               // gather tile

// 64 x 64 lower tiles of the augmented (n+1) square.
__host__ __device__ inline int gather_tiles(int n) {
  const int t = (n + 1 + GT - 1) / GT;
  return t * (t + 1) / 2;
}
__host__ __device__ inline int big_ld(int rcap) { return 6 * rcap + 1; }

// The factorisation advances by panels of two 16-column sub-blocks.
constexpr int PW = 2 * CB;     // panel width (the column-major panel copies assume 32)
static_assert(PW == 32, "side data holds 32-column panel copies");
constexpr int CLD = PW + 1;    // LDS row stride of a panel's column block

// Per-window side data of the factorisation (FP64 words, after the window's
// slot): the reciprocal diagonal of L (ld words), the adjoint's second
// right-hand side as gathered (ld words), then as ints, for the last two
// panels (panel & 1), the nonzero flags of the 16-row blocks below each
// sub-block (32 + 32), and the pivot flags of the factorisation (one int);
// then, for the last two panels, a column-major copy of the panel's columns
// of L (PW columns of ld words), which the next launch reads with coalesced
// loads (16 consecutive rows of a column per lane group).
__host__ __device__ inline int big_aux_stride(int ld) { return 2 * ld + 72 + 2 * 32 * ld; }
struct BigAux {
  double* dinv;
  double* b2;
  int* nzb;    // panel p: nzb + 64 * (p & 1), first sub-block, then + 32 the second
  int* bad;
  double* pt;  // panel p: pt + (p & 1) * PW * ld, entry L[r][32 p + c] at c * ld + r
};
__device__ __forceinline__ BigAux big_aux(const Params& P, int w) {
  double* base = P.big_aux + (int64_t)w * big_aux_stride(P.ld_big);
  int* ints = (int*)(base + 2 * P.ld_big);
  return {base, base + P.ld_big, ints, ints + 128, base + 2 * P.ld_big + 72};
}

constexpr int TU_PANEL = 4;   // row tiles per wave in flight, panel workgroup
constexpr int TU_UPD = 2;     // tiles per wave in flight, update workgroups
constexpr int UPD_TILES = TU_UPD * NWAVES;   // tiles per update workgroup

// Lower 16x16 tiles right of column block j of the trailing matrix at panel
// j (rows and columns from 32 j, tile columns 2 and up), which the update
// workgroups of launch j take from panel j - 1.
__host__ __device__ inline int upd_tiles(int n, int j) {
  const int m = n + 1 - PW * j;
  if (j == 0 || m <= 0) return 0;
  const int T = (m + 15) / 16;
  return T >= 2 ? (T - 2) * (T - 1) / 2 : 0;
}
__host__ __device__ inline int upd_groups(int n, int j) { return (upd_tiles(n, j) + UPD_TILES - 1) / UPD_TILES; }

// LDS of a panel launch: flags, the diagonal block's inverse, row-block
// flags, the column block ((n+1) rows padded to 16, stride CLD).
__host__ __device__ constexpr int chol_panel_lds_bytes(int n) {
  return 64 + CB * PLD * 8 + 64 * 4 + ((n + 1 + 15) / 16) * 16 * CLD * 8 + CB * PLD * 8;
}
// LDS of the back substitution: flags, the solution, two blocks of it.
__host__ __device__ constexpr int chol_big_lds_bytes(int n) { return 64 + (n + 8) * 8 + 2 * CB * 8; }
static_assert((NBIG_MAX + 1 + 15) / 16 <= 32, "row-block flags of a sub-block hold 32 entries");
static_assert(chol_panel_lds_bytes(NBIG_MAX) <= 160 * 1024 && chol_big_lds_bytes(NBIG_MAX) <= 160 * 1024,
              "the largest reduced system fits the LDS of a workgroup");

// One 64 x 64 tile of the augmented system of window w, summed from the chunk
// partials in chunk order (the order of the small-window gather):
// rows < n hold S + lambda I (lower triangle), row n holds -s.  In the
// adjoint (P.adjoint) the tiles of row n also sum the partials' second
// right-hand side (the depth-cotangent column) into the side data.
//
// A chunk whose columns miss the tile, or whose rows miss it (the
// right-hand-side row n belongs to every chunk), is skipped.  The chunks'
// descriptors arrive with one vector load (a window has at most RMAX <= 64
// chunks, one per lane), a ballot marks the chunks that reach the tile, and
// their entries are loaded GB chunks at a time, so a pass waits on one
// memory round trip for GB chunks; they are then added in chunk order.
constexpr int GEPT = GT * GT / WG;   // tile elements per thread
static_assert(RMAX <= 64, "the chunks of a window fit the lanes of a wave");

template <bool ADJ>
__device__ __forceinline__ void gather_big_passes(const Params& P, const WinDesc& W, int n, uint64_t mask, int lo_l,
                                                  int dc_l, const int (&rr)[GEPT], const int (&cc_)[GEPT],
                                                  double (&v)[GEPT], double (&v2)[GEPT]) {
  constexpr int GB = ADJ ? 4 : 8;   // chunks per pass
  while (mask) {
    int ch[GB];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      ch[q] = mask ? __ffsll((unsigned long long)mask) - 1 : -1;
      mask &= mask - 1;
    }
    double a[GB][GEPT], a2[GB][GEPT];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int cc = max(ch[q], 0);
      const int off = 6 * (__builtin_amdgcn_readlane(lo_l, cc) - W.n_fixed);
      const int Dc = __builtin_amdgcn_readlane(dc_l, cc);
      const double* part = P.partial + W.part_off + (int64_t)cc * W.part_stride;
      // unconditional loads (index 0 where the element takes nothing from
      // the chunk) and selects afterwards: loads under divergent branches
      // would each wait for all loads in flight
#pragma unroll
      for (int u = 0; u < GEPT; ++u) {
        const int r = rr[u], c = cc_[u];
        const bool in = ch[q] >= 0 && r <= n && c <= r && c < n && c >= off && c < off + Dc;
        const bool rhs = in && r == n, body = in && r != n && r < off + Dc;
        const int i1 = rhs ? Dc * Dc + (c - off) : (body ? (r - off) * Dc + (c - off) : 0);
        const double x = part[i1];
        a[q][u] = (rhs || body) ? x : 0.0;
        if (ADJ) {
          const double y = part[rhs ? Dc * Dc + Dc + (c - off) : 0];
          a2[q][u] = rhs ? y : 0.0;
        } else {
          a2[q][u] = 0.0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      if (ch[q] >= 0) {
#pragma unroll
        for (int u = 0; u < GEPT; ++u) {
          v[u] += a[q][u];
          if (ADJ) v2[u] += a2[q][u];
        }
      }
    }
  }
}

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
  double v[GEPT], v2[GEPT];
  int rr[GEPT], cc_[GEPT];
#pragma unroll
  for (int u = 0; u < GEPT; ++u) {
    const int e = threadIdx.x + u * WG;
    rr[u] = GT * bi + e / GT;
    cc_[u] = GT * bj + e % GT;
    v[u] = 0.0;
    v2[u] = 0.0;
  }
  const bool adj = P.adjoint != 0;
  const int r_lo = GT * bi, r_hi = min(GT * bi + GT - 1, n);
  const int c_lo = GT * bj, c_hi = min(GT * bj + GT - 1, n - 1);
  const int lane = lane_id();
  const bool has = lane < W.n_chunks;
  const int lo_l = has ? P.cstate[2 * (W.chunk_off + lane)] : 0;
  const int dc_l = has ? P.cstate[2 * (W.chunk_off + lane) + 1] : 0;
  const int off_l = 6 * (lo_l - nfix);
  const bool hit = has && dc_l != 0 && !(c_hi < off_l || c_lo >= off_l + dc_l) &&
                   ((r_hi >= off_l && r_lo < off_l + dc_l) || (r_lo <= n && n <= r_hi));
  const uint64_t mask = __ballot(hit);
  if (adj) gather_big_passes<true>(P, W, n, mask, lo_l, dc_l, rr, cc_, v, v2);
  else gather_big_passes<false>(P, W, n, mask, lo_l, dc_l, rr, cc_, v, v2);
  double* b2 = big_aux(P, w).b2;
#pragma unroll
  for (int u = 0; u < GEPT; ++u) {
    const int r = rr[u], c = cc_[u];
    if (r > n || c > r || c >= n) continue;
    A[(int64_t)r * ld + c] = (r == n) ? -v[u] : (r == c ? v[u] + P.lambda : v[u]);
    if (adj && r == n) b2[c] = v2[u];
  }
}

// Applies panel j-1 (columns kp = k0 - 32 .. k0 - 1 of L, read from its
// column-major copy Pt: two 16-column sub-blocks) to lower 16x16 tiles of
// the trailing matrix at r0 = k0: tile
// (ti, tj) covers rows r0 + 16 ti .. and columns r0 + 16 tj ..;
// A[r][c] -= sum_t L[r][kp+t] L[c][kp+t] for c <= r, c < n, r <= n, as four
// 16x16x4 FP64 matrix-core steps per sub-block, first sub-block first.  A
// sub-block is skipped for a tile whose row blocks below it are zero
// (nzb_a: flags of the first sub-block, row blocks from k0 - 16; nzb_b: the
// second, from k0).  The wave takes tiles t_beg, t_beg + NWAVES, .. below
// t_end, TU at a time; tile_of maps an index to (ti, tj).
template <int TU, typename TileOf>
__device__ __forceinline__ void apply_panel(double* A, const double* Pt, int ld, int n, int k0, int t_beg, int t_end,
                                            TileOf tile_of, const int* nzb_a, const int* nzb_b) {
  const int lane = lane_id(), l16 = lane & 15, g = lane >> 4;
  const int m = n + 1 - k0;
  for (int t0 = t_beg; t0 < t_end; t0 += TU * NWAVES) {
    f64x4 acc[TU];
    double pa[TU][8], pb[TU][8];
    int ti[TU], tj[TU];
    bool ha[TU], hb[TU];
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      const int t = t0 + u * NWAVES;
      ti[u] = 0;
      tj[u] = 0;
      if (t < t_end) tile_of(t, ti[u], tj[u]);
      ha[u] = t < t_end && nzb_a[ti[u] + 1] && nzb_a[tj[u] + 1];
      hb[u] = t < t_end && nzb_b[ti[u]] && nzb_b[tj[u]];
      const int ra = 16 * ti[u] + l16, ca = 16 * tj[u] + l16;
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) {
        pa[u][kq] = (ha[u] && ra < m) ? Pt[(int64_t)(g + 4 * kq) * ld + k0 + ra] : 0.0;
        pb[u][kq] = (ha[u] && ca < m) ? Pt[(int64_t)(g + 4 * kq) * ld + k0 + ca] : 0.0;
        pa[u][4 + kq] = (hb[u] && ra < m) ? Pt[(int64_t)(CB + g + 4 * kq) * ld + k0 + ra] : 0.0;
        pb[u][4 + kq] = (hb[u] && ca < m) ? Pt[(int64_t)(CB + g + 4 * kq) * ld + k0 + ca] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti[u] + acc_row(0.0, g, r), col = 16 * tj[u] + l16;
        const bool ok = (ha[u] || hb[u]) && row < m && col <= row && k0 + col < n;
        acc[u][r] = ok ? A[(int64_t)(k0 + row) * ld + k0 + col] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < TU; ++u) {
      if (ha[u]) {
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) acc[u] = mfma16(-pa[u][kq], pb[u][kq], acc[u]);
      }
      if (hb[u]) {
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) acc[u] = mfma16(-pa[u][4 + kq], pb[u][4 + kq], acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < TU; ++u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti[u] + acc_row(0.0, g, r), col = 16 * tj[u] + l16;
        if ((ha[u] || hb[u]) && row < m && col <= row && k0 + col < n)
          A[(int64_t)(k0 + row) * ld + k0 + col] = acc[u][r];
      }
    }
  }
}

// Launch j of the factorisation of window w (k0 = 32 j).  Workgroup b = 0
// brings column block j (32 columns) up to date with panel j-1 in LDS, then
// per 16-column sub-block: one wave factorises and inverts the diagonal
// block, the rows below become A L^{-T} (written to A and to the panel's
// column-major copy), and after the first sub-block the second one's
// columns receive its update in LDS.
// Workgroups b >= 1 apply panel j-1 to their share of the tiles right of
// column block j.  The two sets of entries are disjoint, and both only read
// panel j-1, which launch j-1 finished.  Pivot problems accumulate BA_W_*
// bits in the side data.
__device__ __forceinline__ void wg_chol_panel(const Params& P, int w, int j, int b, char* smem) {
  const WinDesc W = P.win[w];
  const int n = 6 * (W.n_frames - W.n_fixed);
  // the status word is not written during the factorisation
  if (n <= NCHOL_MAX || P.status[w] != 0) return;
  const int k0 = PW * j;
  if (k0 >= n) return;   // a window with fewer panels
  const int ld = P.ld_big;
  double* A = P.s_big + (int64_t)w * ld * ld;
  const BigAux ax = big_aux(P, w);
  const int* pa_prev = ax.nzb + 64 * ((j + 1) & 1);   // panel j-1, first sub-block
  const int* pb_prev = pa_prev + 32;                  // and second
  const double* pt_prev = ax.pt + ((j + 1) & 1) * PW * ld;   // panel j-1, column-major
  double* pt_cur = ax.pt + (j & 1) * PW * ld;
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int l16 = lane & 15, g = lane >> 4;
  if (b > 0) {
    const int t_end = min(b * UPD_TILES, upd_tiles(n, j));
    apply_panel<TU_UPD>(A, pt_prev, ld, n, k0, (b - 1) * UPD_TILES + wv, t_end,
                        [](int t, int& ti, int& tj) {
                          int a = 0;
                          while (((a + 1) * (a + 2)) / 2 <= t) ++a;
                          ti = a + 2;
                          tj = t - (a * (a + 1)) / 2 + 2;
                        },
                        pa_prev, pb_prev);
    return;
  }
  double* Linv = (double*)(smem + 64);
  int* nzb = (int*)(Linv + CB * PLD);   // 32 + 32 flags
  double* Cb = (double*)(nzb + 64);     // column block j, rows k0 .. n (LDS, stride CLD)
  const int mc = n + 1 - k0;
  const int kw = min(PW, n - k0);
  {
    // column block j with panel j-1 applied: row tiles ti, column tiles tc
    // = 0, 1 (the entries and order of apply_panel)
    const int T = (mc + 15) / 16;
    double qa[2][4], qb[2][4];
    bool ca[2], cb[2];
#pragma unroll
    for (int tc = 0; tc < 2; ++tc) {
      ca[tc] = j > 0 && pa_prev[tc + 1];
      cb[tc] = j > 0 && pb_prev[tc];
      const int rr = 16 * tc + l16;
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) {
        qa[tc][kq] = (ca[tc] && rr < mc) ? pt_prev[(int64_t)(g + 4 * kq) * ld + k0 + rr] : 0.0;
        qb[tc][kq] = (cb[tc] && rr < mc) ? pt_prev[(int64_t)(CB + g + 4 * kq) * ld + k0 + rr] : 0.0;
      }
    }
    for (int t0 = wv; t0 < T; t0 += TU_PANEL * NWAVES) {
      f64x4 acc[TU_PANEL][2];
      double pa[TU_PANEL][8];
      bool ra_nz[TU_PANEL], rb_nz[TU_PANEL];
#pragma unroll
      for (int u = 0; u < TU_PANEL; ++u) {
        const int ti = t0 + u * NWAVES;
        ra_nz[u] = ti < T && j > 0 && pa_prev[ti + 1];
        rb_nz[u] = ti < T && j > 0 && pb_prev[ti];
        const int ra = 16 * ti + l16;
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
          pa[u][kq] = (ra_nz[u] && ra < mc) ? pt_prev[(int64_t)(g + 4 * kq) * ld + k0 + ra] : 0.0;
          pa[u][4 + kq] = (rb_nz[u] && ra < mc) ? pt_prev[(int64_t)(CB + g + 4 * kq) * ld + k0 + ra] : 0.0;
        }
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * ti + acc_row(0.0, g, r), col = 16 * tc + l16;
            const bool ok = ti < T && row < mc && col <= row && k0 + col < n;
            acc[u][tc][r] = ok ? A[(int64_t)(k0 + row) * ld + k0 + col] : 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TU_PANEL; ++u) {
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
          if (ra_nz[u] && ca[tc]) {
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) acc[u][tc] = mfma16(-pa[u][kq], qa[tc][kq], acc[u][tc]);
          }
          if (rb_nz[u] && cb[tc]) {
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) acc[u][tc] = mfma16(-pa[u][4 + kq], qb[tc][kq], acc[u][tc]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TU_PANEL; ++u) {
        const int ti = t0 + u * NWAVES;
        if (ti < T) {
#pragma unroll
          for (int tc = 0; tc < 2; ++tc) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * ti + acc_row(0.0, g, r), col = 16 * tc + l16;
              const bool ok = row < mc && col <= row && k0 + col < n;
              Cb[row * CLD + col] = ok ? acc[u][tc][r] : 0.0;
            }
          }
        }
      }
    }
  }
  int bad = 0;
  double* Linv1 = Cb + ((n + 1 - k0 + 15) / 16) * 16 * CLD;   // the second sub-block's inverse
  // wave 0: factor and invert the diagonal block of sub-block sb (columns
  // 16 sb .. of the column block) into Li
  auto factor = [&](int sb, double* Li) {
    const int c0 = CB * sb, kb = min(CB, kw - c0);
    double Lr[CB];
#pragma unroll
    for (int t = 0; t < CB; ++t)
      Lr[t] = (lane < kb && t <= lane) ? Cb[(c0 + lane) * CLD + c0 + t] : (t == lane ? 1.0 : 0.0);
    wave_factor_invert(Lr, kb, A + (int64_t)(k0 + c0) * ld + k0 + c0, ld, Li, ax.dinv + k0 + c0, bad);
  };
  // rows below sub-block sb: X = A L^{-T} in the column block (LDS), in A and
  // in the column-major copy of the panel; row block rb by the calling wave
  auto trsm = [&](int sb, const double* Li, int rb) {
    const int c0 = CB * sb, kb = min(CB, kw - c0);
    const int r0 = k0 + c0 + kb, m = n + 1 - r0;
    auto rows = [&](int r) { return (const double*)(Cb + (c0 + kb + r) * CLD + c0); };
    auto dst = [&](int r) { return Cb + (c0 + kb + r) * CLD + c0; };
    auto dst2 = [&](int r, int c, double v) {
      A[(int64_t)(r0 + r) * ld + k0 + c0 + c] = v;
      pt_cur[(int64_t)(c0 + c) * ld + r0 + r] = v;
    };
    trsm_row_block(rb, m, kb, Li, rows, dst, dst2, nzb + 32 * sb);
  };
  const int m0 = n + 1 - (k0 + min(CB, kw)), nb0 = (m0 + 15) / 16;   // rows below sub-block 0
  // Sub-block 0: wave 0 factors it and forms row block 0 below it (the
  // second sub-block's diagonal rows), whose products every later tile of
  // the second sub-block's update needs.
  __syncthreads();
  if (wv == 0) {
    factor(0, Linv);
    wave_sync();
    if (nb0 > 0) trsm(0, Linv, 0);
  }
  __syncthreads();
  if (kw <= CB) {
    // one sub-block (the last panel of a window): its remaining rows
    for (int rb = 1 + wv; rb < nb0; rb += NWAVES) trsm(0, Linv, rb);
  } else {
    // Look-ahead.  The second sub-block's columns (rows from 16) lose the
    // first sub-block's products tile by tile, tiles (ti, 0) at r0 = k0 + 16
    // as in a 16-column factorisation; tile ti needs row block ti of the
    // first sub-block's rows and row block 0.  Wave 0 updates tile 0 (the
    // second diagonal block) and factors it, while the other waves form the
    // first sub-block's remaining row blocks and update their tiles.
    const int m1 = m0, T1 = nb0;
    const int* nz1 = nzb;
    double qb1[4];
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) qb1[kq] = (nz1[0] && l16 < m1) ? Cb[(CB + l16) * CLD + g + 4 * kq] : 0.0;
    auto update1 = [&](int ti) {
      const bool has = nz1[ti] && nz1[0];
      const int ra = 16 * ti + l16;
      f64x4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti + acc_row(0.0, g, r);
        acc[r] = (row < m1 && l16 <= row) ? Cb[(CB + row) * CLD + CB + l16] : 0.0;
      }
      if (has) {
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
          const double av = ra < m1 ? Cb[(CB + ra) * CLD + g + 4 * kq] : 0.0;
          acc = mfma16(-av, qb1[kq], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * ti + acc_row(0.0, g, r);
          if (row < m1 && l16 <= row && k0 + CB + l16 < n) Cb[(CB + row) * CLD + CB + l16] = acc[r];
        }
      }
    };
    if (wv == 0) {
      update1(0);
      wave_sync();
      factor(1, Linv1);
    } else {
      // a wave reads back only the rows (and the flag) it has just written
      for (int rb = wv; rb < T1; rb += NWAVES - 1) {
        trsm(0, Linv, rb);
        wave_sync();
        update1(rb);
      }
    }
    __syncthreads();
    const int m2 = n + 1 - (k0 + kw), nb1 = (m2 + 15) / 16;
    for (int rb = wv; rb < nb1; rb += NWAVES) trsm(1, Linv1, rb);
  }
  __syncthreads();
  {
    const int m2 = n + 1 - (k0 + kw);
    if (tid < nb0) ax.nzb[64 * (j & 1) + tid] = nzb[tid];
    if (kw > CB && tid < (m2 + 15) / 16) ax.nzb[64 * (j & 1) + 32 + tid] = nzb[32 + tid];
  }
  if (wv == 0 && lane == 0) *ax.bad = (j == 0 ? 0 : *ax.bad) | bad;
}

// Blocks of the triangular solves whose rows are in flight while a block is
// solved (a ring of SOLVE_AHEAD + 1 register blocks): enough to cover the
// memory latency with the few microseconds a block takes.
constexpr int SOLVE_AHEAD = 4;
constexpr int SOLVE_RING = SOLVE_AHEAD + 1;

// One 16-row block b of the back substitution L^T x = y (rows b0 .. b0+bs-1).
// Thread t < n holds entry t of the running right-hand side in `z` and, in
// `cur`, its column of the block's rows: cur[s] = L[b0 + s][t] for t <= b0 + s.
// The wave holding entries b0 .. b0+15 (one wave: b0 is a multiple of 16)
// solves the block's triangle from its registers, lane b0 + r taking x_r;
// then every thread above the block subtracts the block's products.  `nxt`
// receives the rows of block b - SOLVE_AHEAD (loads in flight across the
// steps).
__device__ __forceinline__ void backsolve_block(const double* A, int ld, int n, int b, double& z, double dv,
                                                double (&cur)[CB], double (&nxt)[CB], double* x, double* xl) {
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  {
    // unconditional loads at clamped addresses: the entries are read only
    // where they belong to the triangle (below the diagonal, inside the
    // matrix), and straight-line loads let each block wait for its own rows
    // only, not for the loads in flight behind them
    const int p0 = max(b - SOLVE_AHEAD, 0) * CB;
#pragma unroll
    for (int s = 0; s < CB; ++s) nxt[s] = A[(int64_t)min(p0 + s, n - 1) * ld + min(tid, n - 1)];
  }
  const int b0 = b * CB, bs = min(CB, n - b0);
  double* xb = xl + (b & 1) * CB;
  if (wv == b0 / 64) {
    const int lb = b0 & 63;
#pragma unroll
    for (int s = CB - 1; s >= 0; --s) {
      if (s < bs) {
        const double xs = row_bcast_f64(z, s) * row_bcast_f64(dv, s);   // lanes lb .. lb+15 form one DPP row
        if (lane == lb + s) z = xs;
        else if (lane >= lb && lane < lb + s) z -= cur[s] * xs;
      }
    }
    if (lane >= lb && lane < lb + bs) {
      xb[lane - lb] = z;
      x[b0 + lane - lb] = z;
    }
  }
  __syncthreads();
  if (tid < b0) {
#pragma unroll
    for (int s = 0; s < CB; ++s)
      if (s < bs) z -= cur[s] * xb[s];
  }
}

// L^T x = y, L in A (lower, ld), y = row n of A (or y0 in LDS), 1/L_ii in
// dinv; x into LDS `x` (n entries); xl: 2 x 16 doubles of LDS.  By 16-row blocks from the
// bottom (backsolve_block), the rows of each block fetched SOLVE_AHEAD blocks
// ahead (block nb - 1 - k of round r in ring slot k: the loop is unrolled
// over the ring); the block's values are double-buffered in xl, so each
// block needs one barrier.
static_assert(NBIG_MAX < WG, "a row of the reduced system is staged one entry per thread");
__device__ __forceinline__ void wg_backsolve_big(const double* A, int ld, int n, const double* dinv, double* x,
                                        double* xl, const double* y0 = nullptr) {
  const int tid = threadIdx.x;
  double z = tid < n ? (y0 ? y0[tid] : A[(int64_t)n * ld + tid]) : 0.0;
  const double dv = tid < n ? dinv[tid] : 0.0;
  double ring[SOLVE_RING][CB];
  const int nb = (n + CB - 1) / CB;
#pragma unroll
  for (int q = 0; q < SOLVE_AHEAD; ++q) {
    const int p0 = max(nb - 1 - q, 0) * CB;
#pragma unroll
    for (int s = 0; s < CB; ++s) ring[q][s] = A[(int64_t)min(p0 + s, n - 1) * ld + min(tid, n - 1)];
  }
  for (int b = nb - 1; b >= 0; b -= SOLVE_RING) {
#pragma unroll
    for (int q = 0; q < SOLVE_RING; ++q)
      if (b - q >= 0) backsolve_block(A, ld, n, b - q, z, dv, ring[q], ring[(q + SOLVE_AHEAD) % SOLVE_RING], x, xl);
  }
  __syncthreads();
}

// One 16-row block b of the forward substitution L y = r: thread t < n
// holds entry t of the running right-hand side in `z` and, in `cur`, its
// row's entries in the block's columns: cur[s] = L[t][b0 + s] for
// b0 + s <= t.  The wave holding entries b0 .. b0+15 solves the block's
// triangle from its registers; then every thread below the block subtracts
// the block's products.  `nxt` receives the columns of block b + SOLVE_AHEAD.
__device__ __forceinline__ void forwardsolve_block(const double* A, int ld, int n, int b, double& z, double dv,
                                                   double (&cur)[CB], double (&nxt)[CB], double* y, double* yl) {
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  {
    // unconditional loads at clamped addresses, as in the back substitution
    const int p0 = (b + SOLVE_AHEAD) * CB;
#pragma unroll
    for (int s = 0; s < CB; ++s) nxt[s] = A[(int64_t)min(tid, n - 1) * ld + min(p0 + s, n - 1)];
  }
  const int b0 = b * CB, bs = min(CB, n - b0);
  double* yb = yl + (b & 1) * CB;
  if (wv == b0 / 64) {
    const int lb = b0 & 63;
#pragma unroll
    for (int s = 0; s < CB; ++s) {
      if (s < bs) {
        const double ys = row_bcast_f64(z, s) * row_bcast_f64(dv, s);
        if (lane == lb + s) z = ys;
        else if (lane > lb + s && lane < lb + bs) z -= cur[s] * ys;
      }
    }
    if (lane >= lb && lane < lb + bs) {
      yb[lane - lb] = z;
      y[b0 + lane - lb] = z;
    }
  }
  __syncthreads();
  if (tid >= b0 + bs && tid < n) {
#pragma unroll
    for (int s = 0; s < CB; ++s)
      if (s < bs) z -= cur[s] * yb[s];
  }
}

// L y = r, L in A (lower, ld), r in LDS (n entries), 1/L_ii in dinv; y into
// LDS `y` (may be r); yl: 2 x 16 doubles of LDS.  By 16-row blocks from the
// top (forwardsolve_block), columns fetched SOLVE_AHEAD blocks ahead (ring
// slots as in the back substitution).
__device__ __forceinline__ void wg_forwardsolve_big(const double* A, int ld, int n, const double* dinv,
                                                    const double* r, double* y, double* yl) {
  const int tid = threadIdx.x;
  double z = tid < n ? r[tid] : 0.0;
  const double dv = tid < n ? dinv[tid] : 0.0;
  __syncthreads();   // r read before y (possibly the same array) is written
  double ring[SOLVE_RING][CB];
#pragma unroll
  for (int q = 0; q < SOLVE_AHEAD; ++q) {
#pragma unroll
    for (int s = 0; s < CB; ++s) ring[q][s] = A[(int64_t)min(tid, n - 1) * ld + min(q * CB + s, n - 1)];
  }
  const int nb = (n + CB - 1) / CB;
  for (int b = 0; b < nb; b += SOLVE_RING) {
#pragma unroll
    for (int q = 0; q < SOLVE_RING; ++q)
      if (b + q < nb) forwardsolve_block(A, ld, n, b + q, z, dv, ring[q], ring[(q + SOLVE_AHEAD) % SOLVE_RING], y, yl);
  }
  __syncthreads();
}

// Back substitution and retraction of a window with n > 126 (the system was
// gathered by wg_gather_big and factorised by the panel launches).
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
  double* x = (double*)(smem + 64);
  double* xl = x + n + 8;
  const BigAux ax = big_aux(P, w);
  if (tid == 0) misc[2] = *ax.bad;
  wg_backsolve_big(A, ld, n, ax.dinv, x, xl);
  if (tid < n && !isfinite_d(x[tid])) atomicOr(&misc[2], W_NONFINITE);
  __syncthreads();
  if (tid == 0 && misc[2]) atomicOr(&P.status[w], misc[2]);
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
