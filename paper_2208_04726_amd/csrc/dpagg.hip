// Soft aggregation (include/dpagg.h) on gfx950: Eq. 5 of Sec. 3.1 over the
// patch or frame neighbourhoods of the patch graph.
//
// 1. The neighbourhoods as a CSR: a key per edge (its patch, or its source
//    and target frame), a counting sort, and each segment put in edge order
//    by a rank sort (so that every sum below runs in a fixed order).
// 2. k_agg_gate: the hidden states of 64 consecutive CSR rows are staged in
//    LDS; the 8 waves multiply them by the gate and value layers on the
//    16x16x32 bfloat16 matrix cores (FP32 accumulation), each wave a band of
//    output channels of both layers; the epilogue forms sigma and
//    sigma * phi and sums them down the rows of each neighbourhood piece of
//    the chunk, writing one partial per (chunk, neighbourhood).
// 3. k_agg_mean sums each neighbourhood's partials in chunk order and
//    divides; k_agg_psi passes 16 neighbourhoods at a time through psi (FP32
//    on the vector ALU: every thread one output channel of a 128-channel
//    slice, its weight row read once for all 16);
//    k_agg_bcast writes each neighbourhood's row to its edges, a 64-row chunk
//    of the CSR per workgroup.
// The CSR depends only on the graph: with graph_ready set, a call reuses the
// one an earlier call left in the workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/dpba.h"
#include "../../include/dpagg.h"

namespace dpagg {

constexpr int CH = 64;          // CSR rows per chunk
constexpr int NW = 8;           // waves of the gate kernel
constexpr int GB = 16;          // neighbourhoods per output workgroup

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

struct Layout {                 // workspace offsets (bytes)
  int64_t key, off, fill, seg, segs, gfirst, pbase, part, psi, ymean, total;
};

__host__ __device__ inline int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

__host__ __device__ inline Layout layout(int64_t E, int64_t G, int D) {
  const int64_t NC = (E + CH - 1) / CH;
  Layout L;
  int64_t o = 0;
  L.key = o;    o += align256(4 * std::max<int64_t>(E, 1));
  L.off = o;    o += align256(4 * (G + 1));
  L.fill = o;   o += align256(4 * std::max<int64_t>(G, 1));
  L.seg = o;    o += align256(4 * std::max<int64_t>(E, 1));
  L.segs = o;   o += align256(4 * std::max<int64_t>(E, 1));
  L.gfirst = o; o += align256(4 * std::max<int64_t>(NC, 1));
  L.pbase = o;  o += align256(4 * (NC + 1));
  L.part = o;   o += align256(4 * 2 * (int64_t)D * (G + NC));   // pieces <= groups + chunks
  L.psi = o;    o += align256(4 * (int64_t)D * std::max<int64_t>(G, 1));
  L.ymean = o;  o += align256(4 * (int64_t)D * std::max<int64_t>(G, 1));
  L.total = o;
  return L;
}

struct Params {
  int mode, D, F;
  int64_t E, M, G;
  const uint16_t* x;
  const int32_t* kk;
  const int32_t* jj;
  const int32_t* anchor;
  const uint16_t* wg;
  const float* bg;
  const uint16_t* wv;
  const float* bv;
  const uint16_t* wo;
  const float* bo;
  float* out;
  int32_t* status;
  int32_t* key;     // [E] neighbourhood of each edge, -1 if its indices are bad
  int32_t* off;     // [G+1] CSR offsets (off[G] = valid edges)
  int32_t* fill;    // [G] scatter cursor
  int32_t* seg;     // [E] edges of each neighbourhood, scatter order
  int32_t* segs;    // [E] the same in edge order
  int32_t* gfirst;  // [NC] first neighbourhood of each chunk
  int32_t* pbase;   // [NC+1] first partial of each chunk
  float* part;      // [pieces][2][D]: sum sigma*phi, sum sigma
  float* psi;       // [G][D]: the output row of each neighbourhood
  float* ymean;     // [G][D]: the aggregate of each neighbourhood
};

__global__ void __launch_bounds__(256) k_agg_zero(int32_t* a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a[i] = 0;
}

// Key of every edge; counts; zero output for edges with bad indices.
__global__ void __launch_bounds__(256) k_agg_keys(Params P) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < P.E; e += (int64_t)gridDim.x * 256) {
    const int k = P.kk[e], j = P.jj[e];
    int64_t key = -1;
    if (k >= 0 && k < P.M && j >= 0 && j < P.F) {
      if (P.mode == DPA_PATCH) {
        key = k;
      } else {
        const int a = P.anchor[k];
        if (a >= 0 && a < P.F) key = (int64_t)a * P.F + j;
      }
    }
    P.key[e] = (int32_t)key;
    if (key >= 0) {
      atomicAdd(&P.off[key], 1);
    } else {
      for (int c = 0; c < P.D; ++c) P.out[e * P.D + c] = 0.f;
      if (P.status) atomicOr(P.status, BA_W_BAD_INDEX);
    }
  }
}

// Exclusive prefix sum of a[0 .. n) in place (a[n] = total), and a copy into
// b[0 .. n) when b is given; one workgroup of 1024.
__global__ void __launch_bounds__(1024) k_agg_scan(int32_t* a, int32_t* b, int64_t n) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = std::min<int64_t>(n, t * per), hi = std::min<int64_t>(n, lo + per);
  int s = 0;
  for (int64_t i = lo; i < hi; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t ? part[t - 1] : 0;
  for (int64_t i = lo; i < hi; ++i) {
    const int c = a[i];
    a[i] = run;
    if (b) b[i] = run;
    run += c;
  }
  if (t == 1023) a[n] = part[1023];
}

// With the graph reused: rows of edges with bad indices are zero again.
__global__ void __launch_bounds__(256) k_agg_badrows(Params P) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < P.E; e += (int64_t)gridDim.x * 256)
    if (P.key[e] < 0)
      for (int c = 0; c < P.D; ++c) P.out[e * P.D + c] = 0.f;
}

__global__ void __launch_bounds__(256) k_agg_scatter(Params P) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < P.E; e += (int64_t)gridDim.x * 256) {
    const int key = P.key[e];
    if (key >= 0) P.seg[atomicAdd(&P.fill[key], 1)] = (int32_t)e;
  }
}

// One wave per neighbourhood: each entry's place is the number of smaller
// edge indices in its segment.
__global__ void __launch_bounds__(512) k_agg_rank(Params P) {
  const int64_t g = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 6);
  if (g >= P.G) return;
  const int l = threadIdx.x & 63;
  const int b = P.off[g], n = P.off[g + 1] - b;
  for (int i = l; i < n; i += 64) {
    const int v = P.seg[b + i];
    int r = 0;
    for (int q = 0; q < n; ++q) r += P.seg[b + q] < v;
    P.segs[b + r] = v;
  }
}

// Per chunk: its first neighbourhood and its number of pieces (a piece per
// neighbourhood from the first to the last one the chunk's rows reach).
__global__ void __launch_bounds__(1024) k_agg_plan(Params P, int64_t NC) {
  const int64_t Ev = P.off[P.G];
  for (int64_t c = threadIdx.x; c < NC; c += 1024) {
    const int64_t r0 = c * CH, r1 = std::min<int64_t>(Ev, r0 + CH);
    // last g with off[g] <= r0, and last g with off[g] < r1
    int64_t lo = 0, hi = P.G - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (P.off[mid] <= r0) lo = mid; else hi = mid - 1;
    }
    const int64_t gf = lo;
    lo = gf;
    hi = P.G - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (P.off[mid] < r1) lo = mid; else hi = mid - 1;
    }
    P.gfirst[c] = (int32_t)gf;
    P.pbase[c] = (int32_t)(lo - gf + 1);   // pieces of the chunk (k_agg_scan makes offsets)
  }
}

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) { return __builtin_bit_cast(bf16x8, *(const uint4*)p); }

// Gate and value layers of 64 CSR rows, sigma and sigma * phi, summed down
// each neighbourhood piece.  CT = 16-channel column tiles per wave.
template <int D>
__global__ void __launch_bounds__(64 * NW) k_agg_gate(Params P) {
  constexpr int KB = D / 32;
  constexpr int CT = D / (16 * NW);
  extern __shared__ __align__(16) char smem[];
  uint16_t* xs = (uint16_t*)smem;                                      // [CH][D]
  int32_t* rgrp = (int32_t*)(smem + CH * D * 2);                       // [CH]
  float* scratch = (float*)(smem + CH * D * 2 + CH * 4);              // [NW][2][CH][16]
  const int c = blockIdx.x;
  const int64_t Ev = P.off[P.G];
  const int64_t r0 = (int64_t)c * CH;
  const int nrows = (int)std::min<int64_t>(CH, Ev - r0);
  if (nrows <= 0) return;   // whole workgroup: chunks past the valid edges
  const int t = threadIdx.x, wave = t >> 6, l = t & 63;
  // stage the chunk's rows (zeros past the last row)
  for (int i = t; i < CH * (D / 8); i += 64 * NW) {
    const int r = i / (D / 8), q = i - r * (D / 8);
    uint4 v = make_uint4(0, 0, 0, 0);
    if (r < nrows) v = *(const uint4*)(P.x + (int64_t)P.segs[r0 + r] * D + q * 8);
    *(uint4*)(xs + r * D + q * 8) = v;
  }
  for (int r = t; r < CH; r += 64 * NW) rgrp[r] = r < nrows ? P.key[P.segs[r0 + r]] : -1;
  __syncthreads();
  const int ch0 = wave * CT * 16;
  const int col = l & 15, kq = l >> 4;
  f32x4 acc[2][4][CT];
#pragma unroll
  for (int L = 0; L < 2; ++L)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[L][rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  // weight operands of the next K step are loaded while this one's
  // products run
  bf16x8 bg[CT], bv[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int64_t w = (int64_t)(ch0 + ct * 16 + col) * D + kq * 8;
    bg[ct] = load8(P.wg + w);
    bv[ct] = load8(P.wv + w);
  }
  for (int kb = 0; kb < KB; ++kb) {
    bf16x8 a[4], ng[CT], nv[CT];
    const int kn = kb + 1 < KB ? kb + 1 : kb;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int64_t w = (int64_t)(ch0 + ct * 16 + col) * D + kn * 32 + kq * 8;
      ng[ct] = load8(P.wg + w);
      nv[ct] = load8(P.wv + w);
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) a[rt] = load8(xs + (rt * 16 + col) * D + kb * 32 + kq * 8);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        acc[0][rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], bg[ct], acc[0][rt][ct], 0, 0, 0);
        acc[1][rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], bv[ct], acc[1][rt][ct], 0, 0, 0);
      }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      bg[ct] = ng[ct];
      bv[ct] = nv[ct];
    }
  }
  float* sc = scratch + wave * (2 * CH * 16);
  const int gf = P.gfirst[c];
  const int pb = P.pbase[c];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int chan = ch0 + ct * 16 + col;
    const float bgc = P.bg[chan], bvc = P.bv[chan];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + 4 * kq + r;
        const float s = 1.0f / (1.0f + expf(-(acc[0][rt][ct][r] + bgc)));
        sc[row * 16 + col] = s * (acc[1][rt][ct][r] + bvc);
        sc[CH * 16 + row * 16 + col] = s;
      }
    wave_lds_sync();
    // lanes 0-15: sigma * phi of channel col; lanes 16-31: sigma
    if (l < 32) {
      const int which = l >> 4;
      const float* src = sc + which * CH * 16;
      float sum = 0.f;
      int cur = nrows > 0 ? rgrp[0] : -1;
      for (int row = 0; row < nrows; ++row) {
        const int g = rgrp[row];
        if (g != cur) {
          P.part[((int64_t)(pb + cur - gf) * 2 + which) * D + chan] = sum;
          sum = 0.f;
          cur = g;
        }
        sum += src[row * 16 + col];
      }
      if (nrows > 0) P.part[((int64_t)(pb + cur - gf) * 2 + which) * D + chan] = sum;
    }
    wave_lds_sync();
  }
}

// The aggregate of every neighbourhood, y[g][c] = sum of its pieces' sigma*phi
// over the sum of their sigma, summed in chunk order; one thread per channel.
__global__ void __launch_bounds__(256) k_agg_mean(Params P) {
  const int64_t total = P.G * P.D;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t g = i / P.D;
    const int c = (int)(i - g * P.D);
    const int b = P.off[g], e = P.off[g + 1];
    float v = 0.f;
    if (e > b) {
      float A = 0.f, B = 0.f;
      for (int ch = b / CH; ch <= (e - 1) / CH; ++ch) {
        const int64_t piece = P.pbase[ch] + (g - P.gfirst[ch]);
        A += P.part[(piece * 2 + 0) * P.D + c];
        B += P.part[(piece * 2 + 1) * P.D + c];
      }
      v = A / B;
    }
    P.ymean[i] = v;
  }
}

// psi of GB neighbourhoods for a 128-channel slice of the outputs (blockIdx.y),
// one thread per output channel, its weight row read once for all GB.
template <int D>
__global__ void __launch_bounds__(128) k_agg_psi(Params P) {
  __shared__ float y[GB][D];
  const int t = threadIdx.x;
  const int64_t g0 = (int64_t)blockIdx.x * GB;
  for (int i = t; i < GB * D; i += 128) {
    const int q = i / D, c = i - q * D;
    y[q][c] = g0 + q < P.G ? P.ymean[(g0 + q) * D + c] : 0.f;
  }
  __syncthreads();
  const int ch = blockIdx.y * 128 + t;
  float o[GB];
#pragma unroll
  for (int q = 0; q < GB; ++q) o[q] = 0.f;
  const uint16_t* w = P.wo + (int64_t)ch * D;
  for (int k = 0; k < D; k += 8) {
    const uint4 v = *(const uint4*)(w + k);
    const uint32_t h[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float w0 = __uint_as_float(h[i] << 16), w1 = __uint_as_float(h[i] & 0xffff0000u);
#pragma unroll
      for (int q = 0; q < GB; ++q) o[q] += w0 * y[q][k + 2 * i] + w1 * y[q][k + 2 * i + 1];
    }
  }
  const float bo = P.bo[ch];
  for (int q = 0; q < GB; ++q) {
    const int64_t g = g0 + q;
    if (g >= P.G) break;
    P.psi[g * D + ch] = o[q] + bo;
  }
}

// Every edge of a 64-row chunk of the CSR receives its neighbourhood's row.
template <int D>
__global__ void __launch_bounds__(256) k_agg_bcast(Params P) {
  const int64_t Ev = P.off[P.G];
  const int64_t r0 = (int64_t)blockIdx.x * CH;
  const int nrows = (int)std::min<int64_t>(CH, Ev - r0);
  for (int i = threadIdx.x; i < nrows * (D / 4); i += 256) {
    const int r = i / (D / 4), q = i - r * (D / 4);
    const int e = P.segs[r0 + r];
    const int g = P.key[e];
    *(float4*)(P.out + (int64_t)e * D + 4 * q) = *(const float4*)(P.psi + (int64_t)g * D + 4 * q);
  }
}

template <int D>
int launch(const Params& P, int64_t NC, hipStream_t s) {
  const int lds = CH * D * 2 + CH * 4 + NW * 2 * CH * 16 * 4;
  if (hipFuncSetAttribute((const void*)k_agg_gate<D>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return BA_E_HIP;
  hipLaunchKernelGGL(k_agg_gate<D>, dim3((unsigned)NC), dim3(64 * NW), lds, s, P);
  hipLaunchKernelGGL(k_agg_mean, dim3((unsigned)std::min<int64_t>((P.G * D + 255) / 256, 16384)), dim3(256), 0, s,
                     P);
  hipLaunchKernelGGL(k_agg_psi<D>, dim3((unsigned)((P.G + GB - 1) / GB), D / 128), dim3(128), 0, s, P);
  hipLaunchKernelGGL(k_agg_bcast<D>, dim3((unsigned)NC), dim3(256), 0, s, P);
  return BA_OK;
}

}  // namespace dpagg

using namespace dpagg;

extern "C" {

int64_t dpa_workspace_bytes(int32_t mode, int32_t dim, int64_t n_edges, int64_t n_patches, int32_t n_frames) {
  if ((mode != DPA_PATCH && mode != DPA_FRAME) || n_edges < 0 || n_patches < 0 || n_frames < 0) return -1;
  if (dim != 128 && dim != 256 && dim != 384 && dim != 512) return -1;
  const int64_t G = mode == DPA_PATCH ? n_patches : (int64_t)n_frames * n_frames;
  return layout(n_edges, G, dim).total;
}

int dpa_softagg(const dpa_problem* p, void* stream) {
  if (!p) return BA_E_INVAL;
  const int64_t need = dpa_workspace_bytes(p->mode, p->dim, p->n_edges, p->n_patches, p->n_frames);
  if (need < 0) return BA_E_INVAL;
  if (p->n_edges == 0) return BA_OK;
  if (p->n_edges > 0x7fffffffLL || p->n_patches > 0x7fffffffLL || p->n_frames < 1 || p->n_patches < 1)
    return BA_E_INVAL;
  const int64_t G = p->mode == DPA_PATCH ? p->n_patches : (int64_t)p->n_frames * p->n_frames;
  if (G > 0x7fffffffLL) return BA_E_INVAL;
  if (!p->x || !p->kk || !p->jj || (p->mode == DPA_FRAME && !p->anchor) || !p->w_gate || !p->b_gate || !p->w_val ||
      !p->b_val || !p->w_out || !p->b_out || !p->out || !p->workspace)
    return BA_E_INVAL;
  if (p->workspace_bytes < need) return BA_E_INVAL;
  const int D = p->dim;
  const Layout L = layout(p->n_edges, G, D);
  char* ws = (char*)p->workspace;
  Params P{};
  P.mode = p->mode;
  P.D = D;
  P.F = p->n_frames;
  P.E = p->n_edges;
  P.M = p->n_patches;
  P.G = G;
  P.x = p->x;
  P.kk = p->kk;
  P.jj = p->jj;
  P.anchor = p->anchor;
  P.wg = p->w_gate;
  P.bg = p->b_gate;
  P.wv = p->w_val;
  P.bv = p->b_val;
  P.wo = p->w_out;
  P.bo = p->b_out;
  P.out = p->out;
  P.status = p->status;
  P.key = (int32_t*)(ws + L.key);
  P.off = (int32_t*)(ws + L.off);
  P.fill = (int32_t*)(ws + L.fill);
  P.seg = (int32_t*)(ws + L.seg);
  P.segs = (int32_t*)(ws + L.segs);
  P.gfirst = (int32_t*)(ws + L.gfirst);
  P.pbase = (int32_t*)(ws + L.pbase);
  P.part = (float*)(ws + L.part);
  P.psi = (float*)(ws + L.psi);
  P.ymean = (float*)(ws + L.ymean);
  // chunks: the valid edges are at most E; chunks past the valid ones exit
  const int64_t NC = (p->n_edges + CH - 1) / CH;
  hipStream_t s = (hipStream_t)stream;
  const unsigned ge = (unsigned)std::min<int64_t>((p->n_edges + 255) / 256, 8192);
  if (!p->graph_ready) {
    hipLaunchKernelGGL(k_agg_zero, dim3((unsigned)std::min<int64_t>((G + 1 + 255) / 256, 4096)), dim3(256), 0, s,
                       P.off, G + 1);
    hipLaunchKernelGGL(k_agg_keys, dim3(ge), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_agg_scan, dim3(1), dim3(1024), 0, s, P.off, P.fill, G);
    hipLaunchKernelGGL(k_agg_scatter, dim3(ge), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_agg_rank, dim3((unsigned)((G + 7) / 8)), dim3(512), 0, s, P);
    hipLaunchKernelGGL(k_agg_plan, dim3(1), dim3(1024), 0, s, P, NC);
    hipLaunchKernelGGL(k_agg_scan, dim3(1), dim3(1024), 0, s, P.pbase, (int32_t*)nullptr, NC);
  } else {
    hipLaunchKernelGGL(k_agg_badrows, dim3(ge), dim3(256), 0, s, P);
  }
  int r = BA_OK;
  if (D == 128) r = launch<128>(P, NC, s);
  else if (D == 256) r = launch<256>(P, NC, s);
  else if (D == 384) r = launch<384>(P, NC, s);
  else r = launch<512>(P, NC, s);
  if (r != BA_OK) return r;
  return hipGetLastError() == hipSuccess ? BA_OK : BA_E_HIP;
}

}  // extern "C"
