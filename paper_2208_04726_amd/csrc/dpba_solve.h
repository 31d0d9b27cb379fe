// Reduced pose solve, depth back-substitution and retraction (FP64).
//
// With the depths eliminated (Sec. 3.1, Schur complement), the pose step of a
// window solves S dxi = -s, S = B + lambda I - E C^{-1} E^T, by a Cholesky
// factorisation held in LDS; then every depth is recovered from its own row,
//   dd_k = -(w_k + sum_a E_ak^T dxi_a) / C_k,
// and the state is updated, T_a <- Exp(dxi_a) T_a for free frames and
// d_k <- d_k + dd_k.  The chunk partials of S and s are summed here in chunk
// order, so the sum is the same in every run.
#pragma once
#include "dpba_assemble.h"

namespace dpba {

__host__ __device__ inline int chol_lds_bytes(int n) {
  const int lda = n + 1;
  return (n * lda + 2 * n + 8) * 8 + 64;
}

// Sum the chunk partials of window w into A (n x lda, lower) and b (n).
template <typename T>
__device__ inline void gather_partials(const Params& P, int w, const WinDesc& W, double* A,
                                       int lda, double* b, int n) {
  const int tid = threadIdx.x;
  const int nfix = W.n_fixed;
  for (int i = tid; i < n * lda; i += WG) A[i] = 0.0;
  for (int i = tid; i < n; i += WG) b[i] = 0.0;
  __syncthreads();
  for (int cc = 0; cc < W.n_chunks; ++cc) {
    const int c = W.chunk_off + cc;
    const int lo_free = P.cstate[2 * c], Dc = P.cstate[2 * c + 1];
    if (Dc == 0) continue;
    const int off = 6 * (lo_free - nfix);
    const double* part = P.partial + W.part_off + (int64_t)cc * W.part_stride;
    for (int i = tid; i < Dc * Dc; i += WG) {
      const int r = i / Dc, col = i % Dc;
      if (col <= r) A[(off + r) * lda + off + col] += part[i];
    }
    for (int r = tid; r < Dc; r += WG) b[off + r] += part[Dc * Dc + r];
    __syncthreads();
  }
}

template <typename T>
__device__ void wg_chol(const Params& P, int w, int iter, char* smem) {
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x;
  int* misc = (int*)smem;
  const int st = wg_bcast_status(P.status, w, misc);
  const int N = W.n_frames, nfix = W.n_fixed;
  const int n = 6 * (N - nfix);
  const double* poses = state_poses<T>(P, W, iter);
  double* next = P.pose_buf + (int64_t)((iter + 1) & 1) * 7 * P.n_frames_total + 7 * W.frame_off;
  double* dxi = P.dxi + 6 * W.frame_off;
  if (st != 0) {
    for (int i = tid; i < 6 * N; i += WG) dxi[i] = 0.0;
    return;
  }
  const int lda = n + 1;
  double* A = (double*)(smem + 64);
  double* b = A + n * lda;
  double* x = b + n;
  if (n > 0) {
    gather_partials<T>(P, w, W, A, lda, b, n);
    for (int i = tid; i < n; i += WG) A[i * lda + i] += P.lambda;
    if (tid == 0) misc[1] = 0;
    __syncthreads();
    // right-looking Cholesky, lower triangle in place
    for (int k = 0; k < n; ++k) {
      if (tid == 0) {
        double d = A[k * lda + k];
        if (!(d > 0.0) || !isfinite_d(d)) {
          misc[1] |= isfinite_d(d) ? W_NOT_SPD : W_NONFINITE;
          d = 1.0;
        }
        A[k * lda + k] = sqrt(d);
      }
      __syncthreads();
      const double lkk = A[k * lda + k];
      for (int i = k + 1 + tid; i < n; i += WG) A[i * lda + k] /= lkk;
      __syncthreads();
      const int m = n - k - 1;
      for (int idx = tid; idx < m * m; idx += WG) {
        const int ii = idx / m, jj = idx % m;
        if (jj <= ii) A[(k + 1 + ii) * lda + k + 1 + jj] -= A[(k + 1 + ii) * lda + k] * A[(k + 1 + jj) * lda + k];
      }
      __syncthreads();
    }
    // L y = -s ; L^T dxi = y
    for (int i = tid; i < n; i += WG) x[i] = -b[i];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      if (tid == 0) x[k] /= A[k * lda + k];
      __syncthreads();
      const double xk = x[k];
      for (int i = k + 1 + tid; i < n; i += WG) x[i] -= A[i * lda + k] * xk;
      __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
      if (tid == 0) x[k] /= A[k * lda + k];
      __syncthreads();
      const double xk = x[k];
      for (int i = tid; i < k; i += WG) x[i] -= A[k * lda + i] * xk;
      __syncthreads();
    }
    if (tid == 0) {
      int bad = misc[1];
      for (int i = 0; i < n; ++i)
        if (!isfinite_d(x[i])) bad |= W_NONFINITE;
      misc[2] = bad;
      if (bad) atomicOr(&P.status[w], bad);
    }
    __syncthreads();
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

__host__ __device__ inline int backsub_lds_bytes(int Rcap, int esize) {
  return RMAX * RELW * esize + Rcap * 6 * 8 + 64;
}

// dd_k for the chunk's patches; writes the depth state (or depth_out on the
// last iteration).
template <typename T>
__device__ void wg_backsub(const Params& P, int c, int iter, char* smem, int Rcap) {
  T* rel = (T*)smem;
  double* dx = (double*)(smem + RMAX * RELW * sizeof(T));
  int* misc = (int*)(smem + RMAX * RELW * sizeof(T) + Rcap * 6 * 8);
  const ChunkDesc cd = P.chunk[c];
  const int w = cd.window;
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const bool last = iter == P.iterations - 1;
  const int st = wg_bcast_status(P.status, w, misc);
  const int32_t* acnt = P.acnt + W.frame_off + w;
  const int32_t* plist = P.plist + W.patch_off;
  if (st != 0) {
    if (last) {
      // failed window: its outputs are its inputs
      const int pb = (cd.a_lo < W.n_frames && !(st & W_BAD_INDEX)) ? acnt[cd.a_lo] : 0;
      const int pe = (cd.a_lo < W.n_frames && !(st & W_BAD_INDEX)) ? acnt[cd.a_hi] : 0;
      if (!(st & W_BAD_INDEX)) {
        for (int q = pb + tid; q < pe; q += WG) {
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
  const int nfix = W.n_fixed;
  int f_lo, f_hi;
  chunk_range(P, W, cd, f_lo, f_hi);
  const double* poses = state_poses<T>(P, W, iter);
  const double* dxi = P.dxi + 6 * W.frame_off;
  for (int i = tid; i < 6 * (f_hi - f_lo + 1); i += WG) dx[i] = dxi[6 * f_lo + i];
  const int32_t* ar = P.arange + 2 * W.frame_off;
  const int32_t* cnt = P.cnt + W.patch_off;
  const int32_t* ptr = P.ptr + W.patch_off;
  const int32_t* csr = P.csr + W.edge_off;
  const int32_t* jjw = P.jj + W.edge_off;
  const T* tg = (const T*)P.targets + 2 * W.edge_off;
  const T* wt = (const T*)P.weights + 2 * W.edge_off;
  const T fx = (T)W.fx, fy = (T)W.fy, cx = (T)W.cx, cy = (T)W.cy;
  const T zmin = (T)P.z_min, lam = (T)P.lambda;
  const int maxdeg = P.wmeta[4 * w];
  const int SEG = seg_width(maxdeg);
  const int segs = 64 / SEG;
  const int lseg = lane & (SEG - 1), sidx = lane / SEG;
  const int nch = (maxdeg + SEG - 1) / SEG;
  double* dout = last ? P.depth_out + W.patch_off : P.depth_buf + W.patch_off;

  for (int a = cd.a_lo; a < cd.a_hi; ++a) {
    const int lo = ar[2 * a], hi = ar[2 * a + 1];
    load_relposes<T>(poses, a, lo, hi, f_lo, rel);
    __syncthreads();
    const int pb = acnt[a], pe = acnt[a + 1];
    const double* dxa = dx + 6 * (a - f_lo);
    for (int q0 = pb + wv * segs; q0 < pe; q0 += NWAVES * segs) {
      const int q = q0 + sidx;
      const bool pv = q < pe;
      const int k = pv ? plist[q] : 0;
      const int deg = pv ? cnt[k] : 0;
      const int base = pv ? ptr[k] : 0;
      const double* pt = P.patches_in + 3 * (W.patch_off + k);
      const double d0 = state_depth(P, W, iter, k);
      const T xb = (T)((pt[0] - W.cx) / W.fx);
      const T yb = (T)((pt[1] - W.cy) / W.fy);
      const T dk = (T)d0;
      T s_cd = 0, s_wd = 0;
      double s_t = 0.0;
      for (int ch = 0; ch < nch; ++ch) {
        const int es = ch * SEG + lseg;
        const bool has = es < deg;
        const int e = has ? csr[base + es] : 0;
        const int j = has ? jjw[e] : a;
        EdgeOut<T> eo;
        linearize_edge<T>(rel + (j - f_lo) * RELW, xb, yb, dk, has ? tg[2 * e] : T(0),
                          has ? tg[2 * e + 1] : T(0), has ? wt[2 * e] : T(0),
                          has ? wt[2 * e + 1] : T(0), fx, fy, cx, cy, zmin, has && (j != a), eo);
        s_cd += eo.cd;
        s_wd += eo.wd;
        if (eo.active) {
          const double* dxj = dx + 6 * (j - f_lo);
          double t = 0.0;
#pragma unroll
          for (int m = 0; m < 6; ++m) t += (double)eo.Ej[m] * dxj[m] + (double)eo.Ei[m] * dxa[m];
          s_t += t;
        }
      }
      const T Ck = lam + seg_sum(s_cd, SEG);
      const T Wk = seg_sum(s_wd, SEG);
      const double tk = seg_sum(s_t, SEG);
      if (pv && lseg == 0) dout[k] = d0 - ((double)Wk + tk) / (double)Ck;
    }
    __syncthreads();
  }
}

// Final poses: the last state, or the inputs of a failed window.
__device__ inline void wg_finalize(const Params& P, int w) {
  const WinDesc W = P.win[w];
  const int st = P.status[w];
  const double* src = (st != 0 || P.iterations == 0)
                          ? P.poses_in + 7 * W.frame_off
                          : P.pose_buf + (int64_t)(P.iterations & 1) * 7 * P.n_frames_total + 7 * W.frame_off;
  double* dst = P.poses_out + 7 * W.frame_off;
  for (int i = threadIdx.x; i < 7 * W.n_frames; i += WG) dst[i] = src[i];
  if (P.iterations == 0)
    for (int k = threadIdx.x; k < W.n_patches; k += WG)
      P.depth_out[W.patch_off + k] = P.patches_in[3 * (W.patch_off + k) + 2];
}

}  // namespace dpba
