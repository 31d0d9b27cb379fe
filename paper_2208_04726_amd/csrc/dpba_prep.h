// Per-window graph preparation, one workgroup per window.
//
// The patch graph (Sec. 3 "Patch Graph") arrives as an unordered edge list
// (k, j).  This pass validates indices, counts edges per patch and patches per
// source frame, and builds two deterministic orderings used by every later
// stage:
//   plist: the window's patches sorted by (source frame, patch index);
//   csr:   each patch's edges sorted by (target frame, edge index).
// Both orders depend only on the graph, not on the input order of equal keys'
// scheduling, so results are bitwise reproducible.  Inputs that already come
// grouped (the usual case) are detected and take the identity orderings.
// It also records, per source frame, the range of frames its patches touch.
#pragma once
#include "dpba_common.h"

namespace dpba {

__device__ void wg_prep(const Params& P, int w, int* lds) {
  const WinDesc W = P.win[w];
  const int N = W.n_frames, M = W.n_patches, E = W.n_edges;
  const int tid = threadIdx.x;
  int32_t* cnt = P.cnt + W.patch_off;
  int32_t* ptr = P.ptr + W.patch_off;
  int32_t* fill = P.fill + W.patch_off;
  int32_t* plist = P.plist + W.patch_off;
  int32_t* acnt = P.acnt + W.frame_off + w;   // N + 1 entries
  int32_t* afill = P.afill + W.frame_off;
  int32_t* ar = P.arange + 2 * W.frame_off;
  int32_t* csr = P.csr + W.edge_off;
  const int32_t* anc = P.anchor + W.patch_off;
  const int32_t* kk = P.kk + W.edge_off;
  const int32_t* jj = P.jj + W.edge_off;
  int* flags = lds + WG;  // [0] bad index, [1] edges unsorted, [2] patches unsorted, [3] max degree, [4] non-finite

  if (tid < 8) flags[tid] = 0;
  for (int k = tid; k < M; k += WG) { cnt[k] = 0; fill[k] = 0; }
  for (int a = tid; a <= N; a += WG) acnt[a] = 0;
  for (int a = tid; a < N; a += WG) { afill[a] = 0; ar[2 * a] = a; ar[2 * a + 1] = a; }
  __syncthreads();

  for (int a = tid; a < N; a += WG) {
    const double* p = P.poses_in + 7 * (W.frame_off + a);
    bool fin = true;
    for (int m = 0; m < 7; ++m) fin = fin && isfinite_d(p[m]);
    if (!fin) atomicOr(&flags[4], 1);
  }
  for (int k = tid; k < M; k += WG) {
    const int a = anc[k];
    if (a < 0 || a >= N) {
      atomicOr(&flags[0], 1);
    } else {
      atomicAdd(&acnt[a], 1);
    }
    if (k > 0 && anc[k - 1] > a) atomicOr(&flags[2], 1);
    const double* pt = P.patches_in + 3 * (W.patch_off + k);
    if (!(isfinite_d(pt[0]) && isfinite_d(pt[1]) && isfinite_d(pt[2]))) atomicOr(&flags[4], 1);
  }
  for (int e = tid; e < E; e += WG) {
    const int k = kk[e], j = jj[e];
    if (k < 0 || k >= M || j < 0 || j >= N) {
      atomicOr(&flags[0], 1);
    } else {
      atomicAdd(&cnt[k], 1);
    }
    if (e > 0) {
      const int kp = kk[e - 1], jp = jj[e - 1];
      if (kp > k || (kp == k && jp > j)) atomicOr(&flags[1], 1);
    }
  }
  __syncthreads();
  const int bad = flags[0];
  if (bad) {
    if (tid == 0) {
      P.status[w] = W_BAD_INDEX | (flags[4] ? W_NONFINITE : 0);
      P.wmeta[4 * w] = 0;
    }
    return;
  }
  for (int k = tid; k < M; k += WG) {
    ptr[k] = cnt[k];
    atomicMax(&flags[3], cnt[k]);
  }
  __syncthreads();
  wg_exclusive_scan(ptr, M, lds);
  wg_exclusive_scan(acnt, N + 1, lds);
  const int unsorted_e = flags[1], unsorted_p = flags[2];

  if (unsorted_p) {
    for (int k = tid; k < M; k += WG) {
      const int a = anc[k];
      const int slot = atomicAdd(&afill[a], 1);
      plist[acnt[a] + slot] = k;
    }
  } else {
    for (int k = tid; k < M; k += WG) plist[k] = k;
  }
  if (unsorted_e) {
    for (int e = tid; e < E; e += WG) {
      const int k = kk[e];
      const int slot = atomicAdd(&fill[k], 1);
      csr[ptr[k] + slot] = e;
    }
  } else {
    for (int e = tid; e < E; e += WG) csr[e] = e;
  }
  __syncthreads();

  // per-patch ordering by (target frame, edge index) and anchor frame ranges
  for (int k = tid; k < M; k += WG) {
    const int b = ptr[k], n = cnt[k];
    if (unsorted_e) {
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
    }
    const int a = anc[k];
    int lo = a, hi = a;
    for (int x = 0; x < n; ++x) {
      const int j = jj[csr[b + x]];
      lo = min(lo, j);
      hi = max(hi, j);
    }
    atomicMin(&ar[2 * a], lo);
    atomicMax(&ar[2 * a + 1], hi);
  }
  if (unsorted_p) {
    for (int a = tid; a < N; a += WG) {
      const int b = acnt[a], n = acnt[a + 1] - b;
      for (int x = 1; x < n; ++x) {
        const int v = plist[b + x];
        int y = x - 1;
        while (y >= 0 && plist[b + y] > v) {
          plist[b + y + 1] = plist[b + y];
          --y;
        }
        plist[b + y + 1] = v;
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    P.status[w] = flags[4] ? W_NONFINITE : 0;
    P.wmeta[4 * w + 0] = flags[3];
    P.wmeta[4 * w + 1] = unsorted_e;
    P.wmeta[4 * w + 2] = unsorted_p;
  }
}

}  // namespace dpba
