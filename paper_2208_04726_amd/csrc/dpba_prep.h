// Per-window graph preparation, one workgroup per window.
//
// The patch graph (Sec. 3 "Patch Graph") arrives as an unordered edge list
// (k, j).  This pass validates it and lays the window out in the order every
// later stage consumes it:
//   * positions: the window's patches sorted by (source frame, patch index);
//     pk[pos] is the patch at a position, acnt[a] the first position of
//     source frame a;
//   * edge order: the edges of position 0, then of position 1, ...; inside a
//     patch by (target frame, edge index).  estart[pos] is the first edge of a
//     position.  When the input is already in this order (the usual case) the
//     input arrays are used as they are; otherwise the target frame, target
//     and weight of each edge are gathered into workspace arrays in this order;
//   * per position: the normalised pixel ((x - cx) / fx, (y - cy) / fy) and
//     the inverse depth of the state (position order);
//   * sub-batches: runs of at most SB positions of one source frame, each with
//     its position and edge ranges (sbd), and per source frame the index of
//     its first sub-batch (sbstart);
//   * per source frame, the range of frames its patches touch (arange).
// Every order depends only on the graph, so results are bitwise reproducible
// whatever the input order of the edges.
#pragma once
#include "dpba_common.h"

namespace dpba {

// Sub-batch width (patches) and lane segment width (edges per patch) for a
// window's largest patch degree: one segment of lanes per patch, at most 1024
// staged edges per sub-batch.
constexpr int PU = 16;   // edges (patches) per thread in flight in the preparation loops
// LDS of the preparation pass (ints): scan scratch, flags, per-frame ranges,
// and per frame a regularity flag and the extremes of its patches' first and
// last target frames
// Scan tiles: SCAN_PER consecutive entries per thread, staged through LDS
// with one pad word per 32 (the per-thread runs then fall in distinct banks).
constexpr int SCAN_PER = 8;
constexpr int SCAN_TILE = SCAN_PER * WG;
constexpr int SCAN_TILE_PAD = SCAN_TILE + SCAN_TILE / 32;
// Stable ordering of unsorted patches: per wave and frame the counts of a
// tile, and per frame the patches placed so far.
constexpr int PREP_LDS_INTS = WG + 16 + 7 * RMAX + SCAN_TILE_PAD + NWAVES * RMAX + RMAX;
// bit of a sub-batch descriptor's .y: every patch of the source frame has the
// same strictly increasing sequence of target frames
constexpr int SB_REGULAR = 1 << 16;

__host__ __device__ inline int seg_width(int maxdeg) { return maxdeg <= 16 ? 16 : (maxdeg <= 32 ? 32 : 64); }
__host__ __device__ inline int sb_width(int seg) { return seg == 64 ? 16 : 32; }

__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }

// Exclusive prefix sum of data[0, n) in place, by tiles of SCAN_TILE entries:
// coalesced loads into LDS, each thread sums its SCAN_PER consecutive
// entries, a wave scan of the thread sums and one of the wave totals, then
// coalesced stores (also into `copy` when given).  `part` holds NWAVES ints,
// `tile` SCAN_TILE_PAD.  Returns the total.  All threads call.
__device__ int wg_scan_tiled(int32_t* data, int n, int* part, int* tile, int32_t* copy = nullptr) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += SCAN_TILE) {
    const int m = min(SCAN_TILE, n - base);
#pragma unroll
    for (int u = 0; u < SCAN_PER; ++u) {
      const int i = u * WG + tid;
      tile[scan_pad(i)] = i < m ? data[base + i] : 0;
    }
    __syncthreads();
    int v[SCAN_PER], sum = 0;
#pragma unroll
    for (int u = 0; u < SCAN_PER; ++u) {
      v[u] = tile[scan_pad(tid * SCAN_PER + u)];
      sum += v[u];
    }
    int incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int x = __shfl_up(incl, o, 64);
      if (lane >= o) incl += x;
    }
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < NWAVES; ++q) {
      before += q < wv ? part[q] : 0;
      total += part[q];
    }
    int run = carry + before + incl - sum;
#pragma unroll
    for (int u = 0; u < SCAN_PER; ++u) {
      tile[scan_pad(tid * SCAN_PER + u)] = run;
      run += v[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SCAN_PER; ++u) {
      const int i = u * WG + tid;
      if (i < m) {
        const int v = tile[scan_pad(i)];
        data[base + i] = v;
        if (copy) copy[base + i] = v;
      }
    }
    carry += total;
    __syncthreads();
  }
  return carry;
}

// Edges per block of the split edge pass.
constexpr int EPB = PU * WG;

// The edge pass over edges [lo, hi) of window W (window-local indices, in
// batches of PU per thread from lo + tid): index checks, order checks, and
// where each patch's run of edges starts (fill) and ends (cnt), which gives
// the counts when the edges turn out to be sorted, and the target frames of
// the run's first and last edge (jrun).
__device__ __forceinline__ void prep_edge_range(const Params& P, const WinDesc& W, int lo, int hi, bool& bad,
                                                bool& uns_e, bool& dup_e) {
  const int M = W.n_patches, N = W.n_frames, E = W.n_edges;
  const int32_t* kk = P.kk + W.edge_off;
  const int32_t* jj = P.jj + W.edge_off;
  int32_t* cnt = P.cnt + W.patch_off;
  int32_t* fill = P.fill + W.patch_off;
  int32_t* jrun = P.jrun + 2 * W.patch_off;
  for (int e0 = lo + (int)threadIdx.x; e0 < hi; e0 += PU * WG) {
    int k[PU], j[PU], kp[PU], jp[PU], kn[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = e0 + u * WG;
      const bool in = e < hi;
      k[u] = in ? kk[e] : 0;
      j[u] = in ? jj[e] : 0;
      kp[u] = (in && e > 0) ? kk[e - 1] : -1;
      jp[u] = (in && e > 0) ? jj[e - 1] : -1;
      kn[u] = (in && e + 1 < E) ? kk[e + 1] : -1;
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = e0 + u * WG;
      if (e < hi) {
        const bool kbad = k[u] < 0 || k[u] >= M;
        bad |= (kbad || j[u] < 0 || j[u] >= N);
        uns_e |= (kp[u] > k[u] || (kp[u] == k[u] && jp[u] > j[u]));
        dup_e |= kp[u] == k[u] && jp[u] == j[u];
        if (!kbad) {
          if (kp[u] != k[u]) {
            fill[k[u]] = e;
            jrun[2 * k[u]] = j[u];
          }
          if (kn[u] != k[u]) {
            cnt[k[u]] = e + 1;
            jrun[2 * k[u] + 1] = j[u];
          }
        }
      }
    }
  }
}

// Split edge pass: block b takes edges [EPB * (b - eb_off), ...) of the window
// whose blocks contain b, and writes its flags to eflags[b] (bit 0 bad index,
// bit 1 unsorted, bit 2 duplicate).  Blocks never span windows, so no flag
// word is shared and none needs clearing.
__device__ __forceinline__ void wg_prep_edges(const Params& P, int b, int* lds) {
  int lo = 0, hi = P.counts[0] - 1;   // last window with eb_off <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (P.win[mid].eb_off <= b) lo = mid; else hi = mid - 1;
  }
  const WinDesc W = P.win[lo];
  const int e_lo = EPB * (b - W.eb_off), e_hi = min(W.n_edges, e_lo + EPB);
  if (threadIdx.x == 0) lds[0] = 0;
  __syncthreads();
  bool bad = false, uns_e = false, dup_e = false;
  prep_edge_range(P, W, e_lo, e_hi, bad, uns_e, dup_e);
  const int f = (__any(bad) ? 1 : 0) | (__any(uns_e) ? 2 : 0) | (__any(dup_e) ? 4 : 0);
  if (f && lane_id() == 0) atomicOr(&lds[0], f);
  __syncthreads();
  if (threadIdx.x == 0) P.eflags[b] = lds[0];
}

template <typename T>
__device__ __forceinline__ void wg_prep(const Params& P, int w, int* lds, bool edges_done = false) {
  const WinDesc W = P.win[w];
  const int N = W.n_frames, M = W.n_patches, E = W.n_edges;
  const int tid = threadIdx.x;
  int32_t* cnt = P.cnt + W.patch_off;
  int32_t* ptr = P.ptr + W.patch_off;
  int32_t* fill = P.fill + W.patch_off;
  int32_t* pk = P.plist + W.patch_off;
  int32_t* acnt = P.acnt + W.frame_off + w;   // N + 1 entries
  int32_t* afill = P.afill + W.frame_off;
  int32_t* ar = P.arange + 2 * W.frame_off;
  int32_t* csr = P.csr + W.edge_off;
  int32_t* est = P.estart + W.patch_off + w;  // M + 1 entries
  int32_t* sbs = P.sbstart + W.frame_off + w; // N + 1 entries
  int4* sbd = P.sbd + W.sb_off;
  const int32_t* anc = P.anchor + W.patch_off;
  const int32_t* kk = P.kk + W.edge_off;
  const int32_t* jj = P.jj + W.edge_off;
  // lds: [0, WG) scan scratch; flags at WG: [0] bad index, [1] edges unsorted,
  // [2] patches unsorted, [3] max degree, [4] non-finite, [5] duplicate edge;
  // per-frame range at WG+16, then per frame: regular, min / max first target
  // frame, min / max last target frame
  int* flags = lds + WG;
  int* lr = lds + WG + 16;   // [2 * RMAX]
  int* rg = lr + 2 * RMAX;   // [5 * RMAX]
  int* tile = rg + 5 * RMAX;           // [SCAN_TILE_PAD] scan staging
  int* wcnt = tile + SCAN_TILE_PAD;    // [NWAVES * RMAX] stable patch ordering
  int* frun = wcnt + NWAVES * RMAX;    // [RMAX]

  if (tid < 16) flags[tid] = 0;
  for (int a = tid; a < N; a += WG) {
    lr[2 * a] = a;
    lr[2 * a + 1] = a;
    rg[a] = 1;
    rg[a + RMAX] = 1 << 30;
    rg[a + 2 * RMAX] = -1;
    rg[a + 3 * RMAX] = 1 << 30;
    rg[a + 4 * RMAX] = -1;
  }
  // run ends / run starts of the edges per patch (read when the edges are
  // sorted); after the split edge pass they hold this call's runs, and stale
  // values for patches without edges, which the count below recognises
  if (!edges_done) {
    for (int k = tid; k < M; k += WG) {
      cnt[k] = 0;
      fill[k] = 0;
    }
  }
  __syncthreads();

  // ---- validation and order checks (coalesced, no atomics on the data path)
  bool bad = false, uns_e = false, uns_p = false, nonfin = false, dup_e = false;
  for (int a = tid; a < N; a += WG) {
    const double* p = P.poses_in + 7 * (W.frame_off + a);
    for (int m = 0; m < 7; ++m) nonfin |= !isfinite_d(p[m]);
  }
  for (int k0 = tid; k0 < M; k0 += PU * WG) {
    int a[PU], ap[PU];
    double x[PU], y[PU], d[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int k = k0 + u * WG;
      const bool in = k < M;
      a[u] = in ? anc[k] : 0;
      ap[u] = (in && k > 0) ? anc[k - 1] : -1;
      const double* pt = P.patches_in + 3 * (W.patch_off + (in ? k : 0));
      x[u] = in ? pt[0] : 0.0;
      y[u] = in ? pt[1] : 0.0;
      d[u] = in ? pt[2] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int k = k0 + u * WG;
      if (k < M) {
        bad |= (a[u] < 0 || a[u] >= N);
        uns_p |= ap[u] > a[u];
        nonfin |= !(isfinite_d(x[u]) && isfinite_d(y[u]) && isfinite_d(d[u]));
        // first position of each source frame, for anchors in frame order
        // (frames without patches start where the next frame does); the
        // unsorted path below recomputes them
        for (int f = max(ap[u] + 1, 0); f <= min(a[u], N); ++f) acnt[f] = k;
        if (k == M - 1)
          for (int f = max(a[u] + 1, 0); f <= N; ++f) acnt[f] = M;
      }
    }
  }
  // edges in batches of PU per thread, so that the loads of a batch are in
  // flight together (or the flags of the split edge pass)
  if (!edges_done) {
    prep_edge_range(P, W, 0, E, bad, uns_e, dup_e);
  } else {
    int f = 0;
    for (int b = tid; b < W.eb_n; b += WG) f |= P.eflags[W.eb_off + b];
    bad |= (f & 1) != 0;
    uns_e |= (f & 2) != 0;
    dup_e |= (f & 4) != 0;
  }
  if (__any(bad) && lane_id() == 0) atomicOr(&flags[0], 1);
  if (__any(uns_e) && lane_id() == 0) atomicOr(&flags[1], 1);
  if (__any(uns_p) && lane_id() == 0) atomicOr(&flags[2], 1);
  if (__any(nonfin) && lane_id() == 0) atomicOr(&flags[4], 1);
  if (__any(dup_e) && lane_id() == 0) atomicOr(&flags[5], 1);   // meaningful for sorted edges
  __syncthreads();
  if (flags[0]) {
    if (tid == 0) {
      P.status[w] = W_BAD_INDEX | (flags[4] ? W_NONFINITE : 0);
      P.wmeta[4 * w] = 0;
    }
    return;
  }
  const int unsorted_e = flags[1], unsorted_p = flags[2];

  // ---- edges per patch and first CSR slot of each patch
  if (unsorted_e) {
    for (int k = tid; k < M; k += WG) {
      cnt[k] = 0;
      fill[k] = 0;
    }
    __syncthreads();
    for (int e = tid; e < E; e += WG) atomicAdd(&cnt[kk[e]], 1);
    __syncthreads();
  }
  int mx = 0;
  for (int k0 = tid; k0 < M; k0 += PU * WG) {
    int f0[PU], ce[PU], c[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int k = k0 + u * WG;
      const bool in = k < M;
      f0[u] = (in && !unsorted_e) ? fill[k] : 0;
      ce[u] = in ? cnt[k] : 0;
    }
    if (unsorted_e) {
#pragma unroll
      for (int u = 0; u < PU; ++u) c[u] = ce[u];
    } else if (edges_done) {
      // after the split pass a patch has a run of this call exactly when its
      // recorded start is an edge of the patch with no edge of the patch
      // before it (no edge names a patch without edges)
      int ka[PU], kb[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const bool ok = k0 + u * WG < M && f0[u] >= 0 && f0[u] < E;
        ka[u] = ok ? kk[f0[u]] : -1;
        kb[u] = (ok && f0[u] > 0) ? kk[f0[u] - 1] : -1;
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int k = k0 + u * WG;
        c[u] = (ka[u] == k && kb[u] != k) ? ce[u] - f0[u] : 0;
      }
    } else {
      // sorted edges: the run end minus the run start (0 for a patch without edges)
#pragma unroll
      for (int u = 0; u < PU; ++u) c[u] = ce[u] - f0[u];
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int k = k0 + u * WG;
      if (k < M) {
        cnt[k] = c[u];
        ptr[k] = c[u];
        mx = max(mx, c[u]);
      }
    }
  }
  atomicMax(&flags[3], mx);
  __syncthreads();
  // with patches in frame order, positions are patch indices and the edge
  // offsets per position are the CSR offsets: one scan writes both
  wg_scan_tiled(ptr, M, lds, tile, unsorted_p ? nullptr : est);
  if (unsorted_e) {
    for (int e = tid; e < E; e += WG) {
      const int k = kk[e];
      csr[ptr[k] + atomicAdd(&fill[k], 1)] = e;
    }
    __syncthreads();
    for (int k = tid; k < M; k += WG) {   // order each patch's edges by (target, index)
      const int b = ptr[k], n = cnt[k];
      for (int x = 1; x < n; ++x) {
        const int e = csr[b + x];
        const int je = jj[e];
        int y = x - 1;
        while (y >= 0) {
          const int f = csr[b + y];
          const int jf = jj[f];
          if (jf < je || (jf == je && f < e)) break;
          csr[b + y + 1] = f;
          --y;
        }
        csr[b + y + 1] = e;
      }
      bool dup = false;
      for (int x = 1; x < n; ++x) dup |= jj[csr[b + x]] == jj[csr[b + x - 1]];
      if (dup) flags[5] = 1;
    }
  }

  // ---- positions: patches by (source frame, index)
  if (!unsorted_p) {
    if (M == 0)
      for (int a = tid; a <= N; a += WG) acnt[a] = 0;
    for (int k = tid; k < M; k += WG) pk[k] = k;
  } else {
    // stable counting sort by source frame: frame sizes, their prefix sum,
    // then tiles of WG patches in index order; inside a tile a patch's rank
    // among the earlier patches of its frame comes from the ballots of its
    // wave and the per-frame counts of the earlier waves
    for (int a = tid; a <= N; a += WG) acnt[a] = 0;
    for (int a = tid; a < RMAX; a += WG) frun[a] = 0;
    __syncthreads();
    for (int k = tid; k < M; k += WG) atomicAdd(&acnt[anc[k]], 1);
    __syncthreads();
    wg_scan_tiled(acnt, N + 1, lds, tile);
    const int lane = tid & 63, wv = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1;
    for (int base = 0; base < M; base += WG) {
      const int k = base + tid;
      const int a = k < M ? anc[k] : -1;
      for (int q = tid; q < NWAVES * RMAX; q += WG) wcnt[q] = 0;
      __syncthreads();
      uint64_t left = __ballot(k < M);
      int rank = 0;
      while (left) {
        const int lead = __ffsll((long long)left) - 1;
        const int a0 = __shfl(a, lead, 64);
        const uint64_t same = __ballot(a == a0) & left;
        if (a == a0) rank = __popcll(same & lt);
        if (lane == lead) wcnt[wv * RMAX + a0] = __popcll(same);
        left &= ~same;
      }
      __syncthreads();
      if (k < M) {
        int before = frun[a];
        for (int q = 0; q < wv; ++q) before += wcnt[q * RMAX + a];
        pk[acnt[a] + before + rank] = k;
      }
      __syncthreads();
      for (int a2 = tid; a2 < N; a2 += WG) {
        int t = 0;
        for (int q = 0; q < NWAVES; ++q) t += wcnt[q * RMAX + a2];
        frun[a2] += t;
      }
      __syncthreads();
    }
  }
  __syncthreads();

  // ---- edge order offsets per position (patches out of frame order)
  for (int q0 = tid; unsorted_p && q0 < M; q0 += PU * WG) {
    int k[PU], c[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int q = q0 + u * WG;
      k[u] = q < M ? (unsorted_p ? pk[q] : q) : 0;
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) c[u] = q0 + u * WG < M ? cnt[k[u]] : 0;
#pragma unroll
    for (int u = 0; u < PU; ++u)
      if (q0 + u * WG < M) est[q0 + u * WG] = c[u];
  }
  __syncthreads();
  if (unsorted_p) wg_scan_tiled(est, M, lds, tile);
  if (tid == 0) est[M] = E;
  // per-position pixel rays, initial depths, frame ranges
  T* pxy = (T*)P.pxy + 2 * W.patch_off;
  double* dep = P.depth_buf + W.patch_off;   // slot 0
  for (int i = tid; i < 7 * N; i += WG) P.pose_buf[7 * W.frame_off + i] = P.poses_in[7 * W.frame_off + i];
  for (int q0 = tid; q0 < M; q0 += PU * WG) {
    int k[PU], n[PU], a[PU], b[PU], j0[PU], j1[PU];
    int2 jr[PU];
    double x[PU], y[PU], d[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int q = q0 + u * WG;
      k[u] = q < M ? (unsorted_p ? pk[q] : q) : 0;
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const bool in = q0 + u * WG < M;
      const double* pt = P.patches_in + 3 * (W.patch_off + k[u]);
      x[u] = in ? pt[0] : 0.0;
      y[u] = in ? pt[1] : 0.0;
      d[u] = in ? pt[2] : 0.0;
      n[u] = in ? cnt[k[u]] : 0;
      a[u] = in ? anc[k[u]] : 0;
      b[u] = in ? ptr[k[u]] : 0;
      // edges in order: the run's first and last target frames, recorded by
      // the edge pass (meaningful for a patch with edges)
      jr[u] = (in && !unsorted_e) ? ((const int2*)(P.jrun + 2 * W.patch_off))[k[u]] : make_int2(0, 0);
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      j0[u] = j1[u] = 0;
      if (n[u] > 0) {
        j0[u] = unsorted_e ? jj[csr[b[u]]] : jr[u].x;
        j1[u] = unsorted_e ? jj[csr[b[u] + n[u] - 1]] : jr[u].y;
      }
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int q = q0 + u * WG;
      // positions are in frame order, so neighbouring lanes mostly carry the
      // same frame and the same first / last target: a lane equal to its left
      // neighbour leaves the per-frame extremes to it (fewer LDS atomics on
      // the same few words)
      const int al = __shfl_up(a[u], 1, 64), j0l = __shfl_up(j0[u], 1, 64);
      const int j1l = __shfl_up(j1[u], 1, 64), nl = __shfl_up(n[u], 1, 64);
      const bool same = lane_id() > 0 && al == a[u] && j0l == j0[u] && j1l == j1[u] && (nl > 0) == (n[u] > 0);
      if (q < M) {
        pxy[2 * q] = (T)((x[u] - W.cx) / W.fx);
        pxy[2 * q + 1] = (T)((y[u] - W.cy) / W.fy);
        dep[q] = d[u];
        if (n[u] > 0 && !same) {
          atomicMin(&lr[2 * a[u]], j0[u]);
          atomicMax(&lr[2 * a[u] + 1], j1[u]);
          atomicMin(&rg[a[u] + RMAX], j0[u]);
          atomicMax(&rg[a[u] + 2 * RMAX], j0[u]);
          atomicMin(&rg[a[u] + 3 * RMAX], j1[u]);
          atomicMax(&rg[a[u] + 4 * RMAX], j1[u]);
        }
        // sorted targets fill [j0, j1] exactly when there are j1 - j0 + 1
        // of them and none repeats
        if (n[u] == 0 || n[u] != j1[u] - j0[u] + 1) rg[a[u]] = 0;
      }
    }
  }
  __syncthreads();
  // gathered edge arrays when the input is not already in edge order
  const bool gathered = unsorted_e || unsorted_p;
  if (gathered) {
    int32_t* gj = P.gj + W.edge_off;
    T* gt = (T*)P.gt + 2 * W.edge_off;
    T* gw = (T*)P.gw + 2 * W.edge_off;
    const T* tg = (const T*)P.targets + 2 * W.edge_off;
    const T* wt = (const T*)P.weights + 2 * W.edge_off;
    for (int q = tid; q < M; q += WG) {
      const int k = pk[q];
      const int b = ptr[k], n = cnt[k], o = est[q];
      for (int x = 0; x < n; ++x) {
        const int e = unsorted_e ? csr[b + x] : b + x;
        gj[o + x] = jj[e];
        P.gidx[W.edge_off + o + x] = e;
        gt[2 * (o + x)] = tg[2 * e];
        gt[2 * (o + x) + 1] = tg[2 * e + 1];
        gw[2 * (o + x)] = wt[2 * e];
        gw[2 * (o + x) + 1] = wt[2 * e + 1];
      }
    }
  }
  // Regular source frames: every patch has the same strictly increasing
  // target-frame sequence (contiguous, unique, with the same first and last
  // frame).  Lane x of a patch's segment then meets one target frame for the
  // whole source frame.
  {
    int* reg = lr + 2 * RMAX;
    for (int a = tid; a < N; a += WG)
      reg[a] = !flags[5] && reg[a] && reg[a + RMAX] == reg[a + 2 * RMAX] && reg[a + 3 * RMAX] == reg[a + 4 * RMAX];
  }
  __syncthreads();
  // sub-batches per source frame
  const int maxdeg = flags[3];
  const int SBw = sb_width(seg_width(maxdeg));
  // wave 0, one frame per lane (at most 64): sub-batch counts and their
  // prefix sum (also kept in LDS: the scan scratch, free again here); then
  // one thread per sub-batch writes its descriptor
  int* sbl = lds;   // [RMAX + 1] first sub-batch of each frame
  if (tid < 64) {
    const int a = tid;
    const int p0 = a < N ? acnt[a] : 0, p1 = a < N ? acnt[a + 1] : 0;
    const int c = (p1 - p0 + SBw - 1) / SBw;
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (tid >= off) incl += v;
    }
    if (a < N) {
      sbs[a] = incl - c;
      sbl[a] = incl - c;
      if (a == N - 1) {
        sbs[N] = incl;
        sbl[N] = incl;
      }
      ar[2 * a] = lr[2 * a];
      ar[2 * a + 1] = lr[2 * a + 1];
    }
    if (N == 0 && a == 0) {
      sbs[0] = 0;
      sbl[0] = 0;
    }
  }
  __syncthreads();
  const int nsb = sbl[N];
  for (int s = tid; s < nsb; s += WG) {
    int a = 0;   // frame of sub-batch s: the last frame whose first sub-batch is <= s
    for (int step = 32; step > 0; step >>= 1)
      if (a + step < N && sbl[a + step] <= s) a += step;
    const int p1 = acnt[a + 1];
    const int q = acnt[a] + (s - sbl[a]) * SBw;
    const int n = min(SBw, p1 - q);
    const int flag = (lr[2 * RMAX + a] ? SB_REGULAR : 0) | (a << 8);
    sbd[s] = make_int4(q, flag | n, est[q], est[q + n]);
  }
  __syncthreads();
  if (tid == 0) {
    int st = flags[4] ? W_NONFINITE : 0;
    if (maxdeg > 64) st |= W_DEGREE;
    P.status[w] = st;
    P.wmeta[4 * w + 0] = maxdeg;
    P.wmeta[4 * w + 1] = gathered ? 1 : 0;
    P.wmeta[4 * w + 2] = unsorted_p;
  }
}

}  // namespace dpba
