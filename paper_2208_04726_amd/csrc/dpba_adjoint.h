// Adjoint of the K-step Gauss-Newton map (vector-Jacobian product with
// respect to targets and weights).
//
// The paper trains through the bundle-adjustment iterations (Sec. 3.1) with
// the initial state held constant (Sec. 3.2, poses and patches detached before
// each update).  One step maps x_n to x_{n+1} = x_n (+) delta_n with
// H_n delta_n = -g_n, H_n = sum_e J_e^T W_e J_e + lambda I, g_n = sum_e J_e^T W_e r_e.
// Given the cotangent of x_{n+1} the pullback through one step is
//   * retraction T' = Exp(dxi) T:  dxi_bar = J_l(dxi)^T xi_bar',
//                                  xi_bar(direct) = Ad(Exp(dxi))^T xi_bar';
//     d' = d + dd:                 dd_bar = d_bar', d_bar(direct) = d_bar';
//   * linear solve: q = H^{-1} delta_bar (same Schur path, second right-hand
//     side on the same Cholesky factor), then per active edge with
//     a = J_e q and b = J_e delta:
//       target_bar += W a,   weight_bar_c += -a_c (r_c + b_c),
//       x_bar += -J_e^T W a + grad_x < Jbar_e, J_e(x) >,
//       Jbar_e = -[W (r + b) q_e^T + W a delta_e^T];
//     the last term differentiates the Jacobian itself (second derivatives of
//     the projection and of the relative pose), written out below.
// The iterates x_1 .. x_{K-1} are recomputed from x_0 inside the backward
// call; nothing is kept from the forward call.
#pragma once
#include "dpba_solve.h"
#include "dpba_chol_big.h"

namespace dpba {

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Exp(xi) = (R, t) for xi = (rho, phi): Rodrigues with series below 1e-2 rad.
__device__ __forceinline__ void se3_exp(const double* xi, double* R, double* t) {
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th2 = px * px + py * py + pz * pz;
  double A, B, C;
  if (th2 < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0 - th2 * th2 * th2 / 5040.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0 - th2 * th2 * th2 / 40320.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0 - th2 * th2 * th2 / 362880.0;
  } else {
    const double th = sqrt(th2);
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[9] = {0, -pz, py, pz, 0, -px, -py, px, 0};
  double K2[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      K2[3 * a + b] = K[3 * a] * K[b] + K[3 * a + 1] * K[3 + b] + K[3 * a + 2] * K[6 + b];
  double V[9];
  for (int m = 0; m < 9; ++m) {
    const double I = (m == 0 || m == 4 || m == 8) ? 1.0 : 0.0;
    R[m] = I + A * K[m] + B * K2[m];
    V[m] = I + B * K[m] + C * K2[m];
  }
  for (int a = 0; a < 3; ++a) t[a] = V[3 * a] * xi[0] + V[3 * a + 1] * xi[1] + V[3 * a + 2] * xi[2];
}

// ad(xi)^T z for ad(xi) = [[hat(phi), hat(rho)], [0, hat(phi)]]:
// (-phi x z_rho, -rho x z_rho - phi x z_phi).
__device__ __forceinline__ void ad_T(const double* xi, const double* z, double* o) {
  double c1[3], c2[3], c3[3];
  cross3(xi + 3, z, c1);
  cross3(xi, z, c2);
  cross3(xi + 3, z + 3, c3);
  for (int m = 0; m < 3; ++m) {
    o[m] = -c1[m];
    o[3 + m] = -c2[m] - c3[m];
  }
}

// J_l(xi)^T v with J_l = sum_m ad(xi)^m / (m+1)!  (left Jacobian of SE(3)).
__device__ __forceinline__ void left_jacobian_T(const double* xi, const double* v, double* out) {
  double term[6], nxt[6];
  for (int m = 0; m < 6; ++m) { term[m] = v[m]; out[m] = v[m]; }
  for (int k = 1; k <= 16; ++k) {
    ad_T(xi, term, nxt);
    const double s = 1.0 / (double)(k + 1);
    for (int m = 0; m < 6; ++m) { term[m] = nxt[m] * s; out[m] += term[m]; }
  }
}

// Ad(Exp(xi))^T v = (R^T v_rho, R^T (v_phi - t x v_rho)).
__device__ __forceinline__ void adjoint_exp_T(const double* xi, const double* v, double* out) {
  double R[9], t[3], c[3];
  se3_exp(xi, R, t);
  cross3(t, v, c);
  const double u[3] = {v[3] - c[0], v[4] - c[1], v[5] - c[2]};
  for (int m = 0; m < 3; ++m) {
    out[m] = R[m] * v[0] + R[3 + m] * v[1] + R[6 + m] * v[2];
    out[3 + m] = R[m] * u[0] + R[3 + m] * u[1] + R[6 + m] * u[2];
  }
}

// Cotangent of a pose 7-vector (t, q) mapped to the left tangent:
// d vec7(Exp(e) T)/de at 0 has dt = rho - t x phi ... transposed:
//   rho_bar = g_t,  phi_bar = t x g_t + (qw g_qv + qv x g_qv) / 2 - qv g_qw / 2.
__device__ __forceinline__ void pose7_cotangent(const double* p, const double* g, double* out) {
  double c[3], c2[3];
  cross3(p, g, c);
  cross3(p + 3, g + 3, c2);
  const double qw = p[6];
  for (int m = 0; m < 3; ++m) {
    out[m] = g[m];
    out[3 + m] = c[m] + 0.5 * (qw * g[3 + m] + c2[m]) - 0.5 * p[3 + m] * g[6];
  }
}

// Zero the gradient outputs of a window and lay out the depth cotangent of
// the final state in position order.
template <typename T>
__device__ __forceinline__ void wg_adj_init(const Params& P, int w) {
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x;
  T* gt = (T*)P.grad_targets + 2 * W.edge_off;
  T* gw = (T*)P.grad_weights + 2 * W.edge_off;
  for (int i = tid; i < 2 * W.n_edges; i += WG) { gt[i] = T(0); gw[i] = T(0); }
  if (P.status[w] != 0) return;
  double* db = P.dbar + (int64_t)(P.iterations & 1) * P.n_patches_total + W.patch_off;
  const int32_t* pk = P.plist + W.patch_off;
  for (int q = tid; q < W.n_patches; q += WG) db[q] = P.grad_depth[W.patch_off + pk[q]];
}

// Reduced pose solves of the adjoint step at x_n: the forward step dxi and
// q_xi = S^{-1} (dxi_bar - sum_k E_k d_bar_k / C_k), with
// dxi_bar = J_l(dxi)^T xi_bar_{n+1}; also the direct cotangent
// Ad(Exp(dxi))^T xi_bar_{n+1}.
template <typename T>
__device__ __forceinline__ void wg_chol_adj(const Params& P, int w, int it, char* smem) {
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x;
  int* misc = (int*)smem;
  const int st = wg_bcast_status(P.status, w, misc);
  const int N = W.n_frames, nfix = W.n_fixed;
  const int n = 6 * (N - nfix);
  double* dxi = P.dxi + 6 * W.frame_off;
  double* qxi = P.qxi + 6 * W.frame_off;
  double* xid = P.xid + 6 * W.frame_off;
  double* xib = P.xib + 6 * W.frame_off;
  if (st != 0 || n == 0) {
    for (int i = tid; i < 6 * N; i += WG) { dxi[i] = 0.0; qxi[i] = 0.0; xid[i] = 0.0; }
    return;
  }
  const double* poses = state_poses<T>(P, W, it);
  const int lda = n + 1;
  double* A = (double*)(smem + 64);
  double* b = A + n * lda;
  double* x = b + n;
  double* b2 = x + n;
  double* x2 = b2 + n;
  double* colbuf = x2 + n + 8;
  gather_partials(P, w, W, A, lda, b, n, b2);
  for (int i = tid; i < n; i += WG) {
    A[i * lda + i] += P.lambda;
    b[i] = -b[i];
  }
  __syncthreads();
  wg_cholesky(A, lda, n, colbuf, misc + 1);
  __syncthreads();
  if (tid < 64) wave_cholesky_solve(A, lda, n, b, x);
  __syncthreads();
  for (int a = nfix + tid; a < N; a += WG) {
    const double* dx = x + 6 * (a - nfix);
    double xin[6];
    if (it == P.iterations - 1) {
      double pn[7];
      retract_left(dx, poses + 7 * a, pn);
      pose7_cotangent(pn, P.grad_poses + 7 * (W.frame_off + a), xin);
    } else {
      for (int m = 0; m < 6; ++m) xin[m] = xib[6 * a + m];
    }
    double dbarx[6], dir[6];
    left_jacobian_T(dx, xin, dbarx);
    adjoint_exp_T(dx, xin, dir);
    for (int m = 0; m < 6; ++m) {
      b2[6 * (a - nfix) + m] += dbarx[m];
      xid[6 * a + m] = dir[m];
    }
  }
  __syncthreads();
  if (tid < 64) wave_cholesky_solve(A, lda, n, b2, x2);
  __syncthreads();
  if (tid == 0) misc[2] = misc[1];
  __syncthreads();
  if (tid < n && !(isfinite_d(x[tid]) && isfinite_d(x2[tid]))) atomicOr(&misc[2], W_NONFINITE);
  __syncthreads();
  if (tid == 0 && misc[2]) atomicOr(&P.status[w], misc[2]);
  for (int i = tid; i < 6 * N; i += WG) {
    const int a = i / 6;
    dxi[i] = a >= nfix ? x[6 * (a - nfix) + i % 6] : 0.0;
    qxi[i] = a >= nfix ? x2[6 * (a - nfix) + i % 6] : 0.0;
    if (a < nfix) xid[i] = 0.0;
  }
}

// The reduced solves of wg_chol_adj for a window with n > 126: the system and
// both right-hand sides were gathered by wg_gather_big (adjoint mode) and
// factorised by the panel launches, which also carried out L y = -s.  Here:
// dxi from L^T dxi = y; the second right-hand side completed with
// J_l(dxi)^T xi_bar per free frame; q_xi from L z = rhs, L^T q_xi = z.
template <typename T>
__device__ __forceinline__ void wg_chol_adj_big(const Params& P, int w, int it, char* smem) {
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x;
  int* misc = (int*)smem;
  const int N = W.n_frames, nfix = W.n_fixed;
  const int n = 6 * (N - nfix);
  if (n <= NCHOL_MAX) return;   // wg_chol_adj
  const int st = wg_bcast_status(P.status, w, misc);
  double* dxi = P.dxi + 6 * W.frame_off;
  double* qxi = P.qxi + 6 * W.frame_off;
  double* xid = P.xid + 6 * W.frame_off;
  double* xib = P.xib + 6 * W.frame_off;
  if (st != 0) {
    for (int i = tid; i < 6 * N; i += WG) { dxi[i] = 0.0; qxi[i] = 0.0; xid[i] = 0.0; }
    return;
  }
  const double* poses = state_poses<T>(P, W, it);
  const int ld = P.ld_big;
  const double* A = P.s_big + (int64_t)w * ld * ld;
  const BigAux ax = big_aux(P, w);
  double* x = (double*)(smem + 64);
  double* xl = x + n + 8;
  double* b2 = xl + 2 * CB;
  double* x2 = b2 + n + 8;
  if (tid == 0) misc[2] = *ax.bad;
  wg_backsolve_big(A, ld, n, ax.dinv, x, xl);
  for (int i = tid; i < n; i += WG) b2[i] = ax.b2[i];
  __syncthreads();
  for (int a = nfix + tid; a < N; a += WG) {
    const double* dx = x + 6 * (a - nfix);
    double xin[6];
    if (it == P.iterations - 1) {
      double pn[7];
      retract_left(dx, poses + 7 * a, pn);
      pose7_cotangent(pn, P.grad_poses + 7 * (W.frame_off + a), xin);
    } else {
      for (int m = 0; m < 6; ++m) xin[m] = xib[6 * a + m];
    }
    double dbarx[6], dir[6];
    left_jacobian_T(dx, xin, dbarx);
    adjoint_exp_T(dx, xin, dir);
    for (int m = 0; m < 6; ++m) {
      b2[6 * (a - nfix) + m] += dbarx[m];
      xid[6 * a + m] = dir[m];
    }
  }
  __syncthreads();
  wg_forwardsolve_big(A, ld, n, ax.dinv, b2, b2, xl);
  wg_backsolve_big(A, ld, n, ax.dinv, x2, xl, b2);
  if (tid < n && !(isfinite_d(x[tid]) && isfinite_d(x2[tid]))) atomicOr(&misc[2], W_NONFINITE);
  __syncthreads();
  if (tid == 0 && misc[2]) atomicOr(&P.status[w], misc[2]);
  for (int i = tid; i < 6 * N; i += WG) {
    const int a = i / 6;
    dxi[i] = a >= nfix ? x[6 * (a - nfix) + i % 6] : 0.0;
    qxi[i] = a >= nfix ? x2[6 * (a - nfix) + i % 6] : 0.0;
    if (a < nfix) xid[i] = 0.0;
  }
}
__host__ __device__ constexpr int chol_adj_big_lds_bytes(int n) { return 64 + 3 * (n + 8) * 8 + 2 * CB * 8; }

// Second-order term of one (u, v) pair: gradient of u^T J(x) v with respect
// to the edge's left perturbation eps = eps_j - Ad(T_ji) eps_i (g[0..5]) and
// its inverse depth (g[6]).  With w_i = Ad v_i, w = v_j - w_i,
// m = d w_rho + w_phi x p + t v_d (the point motion of v) and n = Pi^T u.
__device__ __forceinline__ void jac_pair_grad(const double* u, const double* wi, const double* wv,
                                     double vd, const double* p, double d, const double* t,
                                     double fx, double fy, double* g) {
  const double X = p[0], Y = p[1], Z = p[2];
  const double iz = 1.0 / Z, iz2 = iz * iz;
  double m[3], c[3];
  cross3(wv + 3, p, c);
  for (int k = 0; k < 3; ++k) m[k] = d * wv[k] + c[k] + t[k] * vd;
  const double ux = u[0] * fx, uy = u[1] * fy;
  const double n[3] = {ux * iz, uy * iz, -(ux * X + uy * Y) * iz2};
  // d (u^T Pi(p) m) / dp with m held
  double G[3] = {-ux * m[2] * iz2, -uy * m[2] * iz2,
                 -(ux * m[0] + uy * m[1]) * iz2 + 2.0 * (ux * X + uy * Y) * m[2] * iz2 * iz};
  cross3(n, wv + 3, c);
  for (int k = 0; k < 3; ++k) G[k] += c[k];
  double c1[3], c2[3], c3[3], pn[3], c4[3];
  cross3(wi + 3, n, c1);       // w_i_phi x n
  cross3(wi, n, c2);           // w_i_rho x n
  cross3(p, n, pn);            // p x n
  cross3(wi + 3, pn, c3);      // w_i_phi x (p x n)
  cross3(t, n, c4);            // t x n
  double pG[3];
  cross3(p, G, pG);
  for (int k = 0; k < 3; ++k) {
    g[k] += d * G[k] - d * c1[k] + vd * n[k];
    g[3 + k] += pG[k] - d * c2[k] - c3[k] + vd * c4[k];
  }
  g[6] += G[0] * t[0] + G[1] * t[1] + G[2] * t[2] + n[0] * wv[0] + n[1] * wv[1] + n[2] * wv[2];
}

// Ad(T) z from the LDS relative pose (R, t, hat(t) R).
template <typename T>
__device__ __forceinline__ void rel_adj(const T* rel, const double* z, double* o) {
  for (int r = 0; r < 3; ++r) {
    o[r] = (double)rel[3 * r] * z[0] + (double)rel[3 * r + 1] * z[1] + (double)rel[3 * r + 2] * z[2] +
           (double)rel[12 + 3 * r] * z[3] + (double)rel[13 + 3 * r] * z[4] + (double)rel[14 + 3 * r] * z[5];
    o[3 + r] = (double)rel[3 * r] * z[3] + (double)rel[3 * r + 1] * z[4] + (double)rel[3 * r + 2] * z[5];
  }
}
// Ad(T)^T z
template <typename T>
__device__ __forceinline__ void rel_adj_T(const T* rel, const double* z, double* o) {
  for (int c = 0; c < 3; ++c) {
    o[c] = (double)rel[c] * z[0] + (double)rel[3 + c] * z[1] + (double)rel[6 + c] * z[2];
    o[3 + c] = (double)rel[12 + c] * z[0] + (double)rel[15 + c] * z[1] + (double)rel[18 + c] * z[2] +
               (double)rel[c] * z[3] + (double)rel[3 + c] * z[4] + (double)rel[6 + c] * z[5];
  }
}

__host__ __device__ inline int edge_adj_lds_bytes(int Rcap, int esize) {
  int o = backsub_stage_offset(Rcap, esize) + stage_bytes(esize);
  o = al16(o);
  o += Rcap * 6 * 8;                          // q_xi per frame
  o += NWAVES * 2 * Rcap * 6 * 8;             // target cotangent tables
  o += NWAVES * 4 * 6 * 8;                    // source-frame cotangent per segment
  o += Rcap * 6 * 8;                          // per-frame sum of the chunk
  return o + 64;
}

// Per-edge adjoint of iteration `it` for one chunk: target and weight
// gradients, the depth cotangent of x_it (position order) and the chunk's
// pose-cotangent partial.
template <typename T>
__device__ __forceinline__ void wg_edge_adj(const Params& P, int c, int it, char* smem, int Rcap) {
  double* lp = (double*)smem;
  T* rel = (T*)(smem + al16(Rcap * 7 * 8));
  double* dx = (double*)(smem + backsub_dx_offset(Rcap, (int)sizeof(T)));
  const int so = backsub_stage_offset(Rcap, (int)sizeof(T));
  Stage<T> S(smem + so);
  char* q0 = smem + al16(so + stage_bytes((int)sizeof(T)));
  double* qx = (double*)q0;
  double* gT = qx + Rcap * 6;
  double* gA = gT + NWAVES * 2 * Rcap * 6;
  double* facc = gA + NWAVES * 4 * 6;
  int* misc = (int*)(facc + Rcap * 6);

  const ChunkDesc cd = P.chunk[c];
  const int w = cd.window;
  const WinDesc W = P.win[w];
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int st = wg_bcast_status(P.status, w, misc);
  const int N = W.n_frames, nfix = W.n_fixed;
  double* fc = P.fcot + (int64_t)c * RMAX * 6;
  if (st != 0) {
    for (int i = tid; i < 6 * N; i += WG) fc[i] = 0.0;
    return;
  }
  const double* poses = state_poses<T>(P, W, it);
  for (int i = tid; i < 7 * N; i += WG) lp[i] = poses[i];
  for (int i = tid; i < 6 * N; i += WG) {
    dx[i] = P.dxi[6 * W.frame_off + i];
    qx[i] = P.qxi[6 * W.frame_off + i];
    facc[i] = 0.0;
  }
  const int32_t* ar = P.arange + 2 * W.frame_off;
  const int32_t* sbs = P.sbstart + W.frame_off + w;
  const int4* sbd = P.sbd + W.sb_off;
  const int gathered = P.wmeta[4 * w + 1];
  const WinEdges we = win_edges(P, W, gathered, (int)sizeof(T));
  const T fx = (T)W.fx, fy = (T)W.fy, cx = (T)W.cx, cy = (T)W.cy;
  const T zmin = (T)P.z_min, lam = (T)P.lambda;
  const int SEG = seg_width(P.wmeta[4 * w]);
  const int SBw = sb_width(SEG);
  const int segs = 64 / SEG;
  const int spw = SBw / NWAVES;
  const int npass = (spw + segs - 1) / segs;
  const int lseg = lane & (SEG - 1), sidx = lane / SEG;
  const int tslots = min(segs, 2);
  const double* dbar_in = P.dbar + (int64_t)((it + 1) & 1) * P.n_patches_total;
  double* dbar_out = P.dbar + (int64_t)(it & 1) * P.n_patches_total + W.patch_off;
  T* gtg = (T*)P.grad_targets + 2 * W.edge_off;
  T* gwt = (T*)P.grad_weights + 2 * W.edge_off;
  const int s_lo = sbs[cd.a_lo], s_hi = sbs[cd.a_hi];

  StageRegs<T> R;
  int4 dcur = make_int4(0, 0, 0, 0), dnxt = dcur;
  if (s_lo < s_hi) {
    dcur = sbd[s_lo];
    if (s_lo + 1 < s_hi) dnxt = sbd[s_lo + 1];
    stage_issue<T>(P, W, w, we, dcur, it, dbar_in, R);
  }
  __syncthreads();
  if (s_lo < s_hi) stage_store<T>(dcur, R, S, dbar_in != nullptr);
  int a = -1, lo = 0, hi = -1, Ra = 0;
  for (int s = s_lo; s <= s_hi; ++s) {
    const int an = (s < s_hi) ? ((dcur.y >> 8) & 0xff) : -1;
    if (an != a && a >= 0) {
      // fold this source frame's tables into the per-frame sums, fixed order
      __syncthreads();
      for (int i = tid; i < Ra * 6; i += WG) {
        double sum = 0.0;
        for (int x = 0; x < NWAVES * tslots; ++x) sum += gT[x * Ra * 6 + i];
        facc[6 * lo + i] += sum;
      }
      __syncthreads();
      if (tid < 6) {
        double sum = 0.0;
        for (int x = 0; x < NWAVES * 4; ++x) sum += gA[x * 6 + tid];
        facc[6 * a + tid] += sum;
      }
      __syncthreads();
    }
    if (s == s_hi) break;
    if (an != a) {
      a = an;
      lo = ar[2 * a];
      hi = ar[2 * a + 1];
      Ra = hi - lo + 1;
      load_relposes<T>(lp, a, lo, hi, 0, rel);
      for (int i = tid; i < NWAVES * tslots * Ra * 6; i += WG) gT[i] = 0.0;
      for (int i = tid; i < NWAVES * 4 * 6; i += WG) gA[i] = 0.0;
    }
    const int nsb = dcur.y & 255, pos0 = dcur.x, e0 = dcur.z;
    int dnn = 0;
    const bool pre = s + 2 < s_hi;
    if (s + 1 < s_hi) stage_issue<T>(P, W, w, we, dnxt, it, dbar_in, R);
    if (pre) dnn = desc_prefetch(sbd + s + 2);
    __syncthreads();
    const double* dxa = dx + 6 * a;
    const double* qxa = qx + 6 * a;
    const T* rela = rel + a * RELW;   // identity relative pose of the source frame (unused)
    (void)rela;
    double* mygT = gT + wv * tslots * Ra * 6;
    for (int ps = 0; ps < npass; ++ps) {
      const int slot_in_wave = ps * segs + sidx;
      const LaneEdge<T> le = lane_edge<T>(S, wv * spw + slot_in_wave, slot_in_wave < spw, nsb, lseg, a);
      EdgeOut<T> eo;
      const int j = le.j;
      const T* rj = rel + j * RELW;
      linearize_edge<T>(rj, le.xb, le.yb, (T)le.d, le.t0, le.t1, le.w0, le.w1, fx, fy, cx, cy,
                        zmin, le.has && (j != a), eo);
      // forward step and adjoint solve, depth rows (FP64)
      double tD = 0.0, tQ = 0.0;
      if (eo.active) {
        const double* dxj = dx + 6 * j;
        const double* qxj = qx + 6 * j;
        for (int m = 0; m < 6; ++m) {
          tD += (double)eo.Ej[m] * dxj[m] + (double)eo.Ei[m] * dxa[m];
          tQ += (double)eo.Ej[m] * qxj[m] + (double)eo.Ei[m] * qxa[m];
        }
      }
      T rc[2] = {eo.cd, eo.wd};
      double rr[2] = {tD, tQ};
      seg_sum_n<2>(rc, SEG);
      seg_sum_n<2>(rr, SEG);
      const T rc0 = rc[0], rc1 = rc[1];
      const double r2 = rr[0], r3 = rr[1];
      const double Ck = (double)(lam + rc0);
      const double ddk = -((double)rc1 + r2) / Ck;
      const double dbk = le.pv ? S.pd2[le.slot] : 0.0;
      const double qdk = (dbk - r3) / Ck;

      // per-edge adjoint
      double gv[7] = {0, 0, 0, 0, 0, 0, 0};
      if (eo.active) {
        const double J0[6] = {eo.J0[0], eo.J0[1], eo.J0[2], eo.J0[3], eo.J0[4], eo.J0[5]};
        const double J1[6] = {eo.J1[0], eo.J1[1], eo.J1[2], eo.J1[3], eo.J1[4], eo.J1[5]};
        const double w0 = eo.w0, w1 = eo.w1, r0 = eo.r0, r1 = eo.r1;
        const double jd0 = eo.jd0, jd1 = eo.jd1;
        double wiq[6], wid[6], wq[6], wD[6];
        rel_adj<T>(rj, qxa, wiq);
        rel_adj<T>(rj, dxa, wid);
        for (int m = 0; m < 6; ++m) {
          wq[m] = qx[6 * j + m] - wiq[m];
          wD[m] = dx[6 * j + m] - wid[m];
        }
        double a0 = jd0 * qdk, a1 = jd1 * qdk, b0 = jd0 * ddk, b1 = jd1 * ddk;
        for (int m = 0; m < 6; ++m) {
          a0 += J0[m] * wq[m];
          a1 += J1[m] * wq[m];
          b0 += J0[m] * wD[m];
          b1 += J1[m] * wD[m];
        }
        const int q = e0 + le.q;
        const int eidx = gathered ? P.gidx[W.edge_off + q] : q;
        gtg[2 * eidx] += (T)(w0 * a0);
        gtg[2 * eidx + 1] += (T)(w1 * a1);
        gwt[2 * eidx] += (T)(-a0 * (r0 + b0));
        gwt[2 * eidx + 1] += (T)(-a1 * (r1 + b1));
        const double p[3] = {eo.X, eo.Y, eo.Z};
        const double t3[3] = {(double)rj[9], (double)rj[10], (double)rj[11]};
        const double dd = le.d;
        const double dfx = W.fx, dfy = W.fy;
        // first order: -J^T W a
        {
          const double iz = 1.0 / p[2];
          const double ux = w0 * a0 * dfx, uy = w1 * a1 * dfy;
          const double n1[3] = {ux * iz, uy * iz, -(ux * p[0] + uy * p[1]) * iz * iz};
          double pn[3];
          cross3(p, n1, pn);
          for (int k = 0; k < 3; ++k) { gv[k] -= dd * n1[k]; gv[3 + k] -= pn[k]; }
          gv[6] -= t3[0] * n1[0] + t3[1] * n1[1] + t3[2] * n1[2];
        }
        // second order: pairs (-W (r + b), q) and (-W a, delta)
        const double u1[2] = {-w0 * (r0 + b0), -w1 * (r1 + b1)};
        jac_pair_grad(u1, wiq, wq, qdk, p, dd, t3, dfx, dfy, gv);
        const double u2[2] = {-w0 * a0, -w1 * a1};
        jac_pair_grad(u2, wid, wD, ddk, p, dd, t3, dfx, dfy, gv);
      }
      // source frame share -Ad^T g_eps, summed over the patch's edges
      double ga[7];
      rel_adj_T<T>(rj, gv, ga);
      for (int m = 0; m < 6; ++m) ga[m] = -ga[m];
      ga[6] = gv[6];
      seg_sum_n<7>(ga, SEG);
      if (le.pv && lseg == 0) {
        dbar_out[pos0 + le.slot] = dbk + ga[6];
        double* acc = gA + (wv * 4 + sidx) * 6;
        for (int m = 0; m < 6; ++m) acc[m] += ga[m];
      }
      // target-frame share g_eps into the wave's table
      const int jprev = __shfl_up(j, 1, 64);
      const bool dup = eo.active && lseg > 0 && jprev == j;
      const bool anydup = __any(dup);
      double* tb = mygT + ((sidx % tslots) * Ra + (j - lo)) * 6;
      for (int sgi = 0; sgi < segs; sgi += tslots) {
        for (int ln = 0; ln < (anydup ? SEG : 1); ++ln) {
          if (sidx - sidx % tslots == sgi && eo.active && (!anydup || lseg == ln)) {
            for (int m = 0; m < 6; ++m) tb[m] += gv[m];
          }
        }
      }
    }
    __syncthreads();
    if (s + 1 < s_hi) stage_store<T>(dnxt, R, S, dbar_in != nullptr);
    dcur = dnxt;
    {
      // taken on every path, so no load is in flight into the next iteration
      const int4 dt = desc_take(dnn);
      if (pre) dnxt = dt;
    }
  }
  __syncthreads();
  for (int i = tid; i < 6 * N; i += WG) fc[i] = facc[i];
}

// x_bar_n for the poses: direct part plus every chunk's partial; fixed frames 0.
__device__ __forceinline__ void wg_frame_adj(const Params& P, int w) {
  const WinDesc W = P.win[w];
  const int N = W.n_frames, nfix = W.n_fixed;
  if (P.status[w] != 0) return;
  for (int i = threadIdx.x; i < 6 * N; i += WG) {
    const int a = i / 6;
    double s = 0.0;
    if (a >= nfix) {
      s = P.xid[6 * W.frame_off + i];
      for (int cc = 0; cc < W.n_chunks; ++cc) s += P.fcot[(int64_t)(W.chunk_off + cc) * RMAX * 6 + i];
    }
    P.xib[6 * W.frame_off + i] = s;
  }
}

}  // namespace dpba
