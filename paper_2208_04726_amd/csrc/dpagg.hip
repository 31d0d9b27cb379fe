// Soft aggregation (include/dpagg.h) on gfx950: Eq. 5 of Sec. 3.1 over the
// patch or frame neighbourhoods of the patch graph.
//
// 1. The neighbourhoods as a CSR: a key per edge (its patch, or its source
//    and target frame), a counting sort, and each segment put in edge order
//    by a rank sort (so that every sum below runs in a fixed order).
// 2. k_agg_gate: a workgroup takes a 128-channel slice of the gate and value
//    layers, each wave the weights of 16 channels for every K step in
//    registers, and runs through a group of 64-row CSR chunks: the chunk's
//    hidden states staged in LDS (the next chunk's loaded meanwhile), the
//    products on the 16x16x32 bfloat16 matrix cores (FP32 accumulation); the
//    epilogue forms sigma and sigma * phi and sums them down the rows of each
//    neighbourhood piece of the chunk, writing one partial per (chunk,
//    neighbourhood) for the slice's channels.
// 3. k_agg_mean sums each neighbourhood's partials in chunk order and
//    divides; k_agg_psi passes 16 neighbourhoods x 64 channels at a time
//    through psi on the FP32 matrix cores (bfloat16 weights widened exactly);
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

// Gate and value layers of `cpw` consecutive 64-row chunks of the CSR for one
// 128-channel slice of both layers (blockIdx.x = chunk group * NS + slice):
// every wave keeps the weights of its 16 channels for all K steps in
// registers (read once per workgroup), the chunk's rows are staged in LDS
// while the next chunk's rows are loaded into registers; sigma and
// sigma * phi are summed down each neighbourhood piece of the chunk.
template <int D>
__global__ void __launch_bounds__(64 * NW) k_agg_gate(Params P, int64_t NC, int cpw) {
  constexpr int KB = D / 32;
  constexpr int XS = D + 8;                   // LDS row stride (bf16): rows 16 bytes apart in the banks
  constexpr int NS = D / (16 * NW);           // channel slices
  constexpr int XQ = CH * (D / 8) / (64 * NW);  // 16-byte row pieces per thread
  static_assert(CH * (D / 8) % (64 * NW) == 0, "rows stage evenly");
  extern __shared__ __align__(16) char smem[];
  uint16_t* xs = (uint16_t*)smem;                                      // [CH][XS]
  int32_t* rgrp = (int32_t*)(smem + CH * XS * 2);                      // [CH]
  float* scratch = (float*)(smem + CH * XS * 2 + CH * 4);             // [NW][2][16][CH]
  const int slice = blockIdx.x % NS;
  const int64_t c_begin = (int64_t)(blockIdx.x / NS) * cpw;
  const int64_t c_end = std::min<int64_t>(NC, c_begin + cpw);
  const int64_t Ev = P.off[P.G];
  const int t = threadIdx.x, wave = t >> 6, l = t & 63;
  const int col = l & 15, kq = l >> 4;
  const int chan = slice * 16 * NW + wave * 16 + col;
  bf16x8 wgk[KB], wvk[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const int64_t w = (int64_t)chan * D + kb * 32 + kq * 8;
    wgk[kb] = load8(P.wg + w);
    wvk[kb] = load8(P.wv + w);
  }
  const float bgc = P.bg[chan], bvc = P.bv[chan];
  // rows of chunk c into registers (zeros past the valid rows), and the key
  // of row t for t < CH.  The CSR entries of a chunk are loaded one chunk
  // ahead of its rows (si, st), so a chunk's rows need one round trip.
  uint4 xr[XQ];
  int si[XQ];
  int st = -1, rk = -1;
  auto fetch_segs = [&](int64_t c) {
    const int64_t r0 = c * CH;
    const int nr = c < c_end ? (int)std::min<int64_t>(CH, Ev - r0) : 0;
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int r = (t + u * 64 * NW) / (D / 8);
      si[u] = r < nr ? P.segs[r0 + r] : -1;
    }
    st = t < CH && t < nr ? P.segs[r0 + t] : -1;
  };
  auto fetch_rows = [&]() {
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int i = t + u * 64 * NW;
      const int q = i % (D / 8);
      xr[u] = si[u] >= 0 ? *(const uint4*)(P.x + (int64_t)si[u] * D + q * 8) : make_uint4(0, 0, 0, 0);
    }
    rk = st >= 0 ? P.key[st] : -1;
  };
  if (c_begin < c_end) {
    fetch_segs(c_begin);
    fetch_rows();
    fetch_segs(c_begin + 1);
  }
  float* sc = scratch + wave * (2 * CH * 16);
  for (int64_t c = c_begin; c < c_end; ++c) {
    const int64_t r0 = c * CH;
    const int nrows = (int)std::min<int64_t>(CH, Ev - r0);
    if (nrows <= 0) break;   // whole workgroup: chunks past the valid edges
    __syncthreads();         // the previous chunk's rows and keys are no longer read
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int i = t + u * 64 * NW;
      const int r = i / (D / 8), q = i - r * (D / 8);
      *(uint4*)(xs + r * XS + q * 8) = xr[u];
    }
    if (t < CH) rgrp[t] = rk;
    __syncthreads();
    if (c + 1 < c_end) {
      fetch_rows();          // chunk c + 1, from the CSR entries loaded last time
      fetch_segs(c + 2);
    }
    f32x4 acc[2][4];
#pragma unroll
    for (int L = 0; L < 2; ++L)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) acc[L][rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      bf16x8 a[4];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) a[rt] = load8(xs + (rt * 16 + col) * XS + kb * 32 + kq * 8);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        acc[0][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], wgk[kb], acc[0][rt], 0, 0, 0);
        acc[1][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], wvk[kb], acc[1][rt], 0, 0, 0);
      }
    }
    const int gf = P.gfirst[c];
    const int pb = P.pbase[c];
    // sigma * phi and sigma, column-major per wave ([which][col][row]) so that
    // each summing lane reads its column's rows with 16-byte loads
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      float4 sp, sg4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float sg = 1.0f / (1.0f + expf(-(acc[0][rt][r] + bgc)));
        (&sp.x)[r] = sg * (acc[1][rt][r] + bvc);
        (&sg4.x)[r] = sg;
      }
      *(float4*)(sc + col * CH + rt * 16 + 4 * kq) = sp;
      *(float4*)(sc + (16 + col) * CH + rt * 16 + 4 * kq) = sg4;
    }
    wave_lds_sync();
    // lanes 0-15: sigma * phi of channel col; lanes 16-31: sigma; the rows
    // summed in order, in registers, 16 at a time
    if (l < 32) {
      const int which = l >> 4;
      const float* src = sc + (which * 16 + col) * CH;
      float sum = 0.f;
      int cur = rgrp[0];
      for (int r0b = 0; r0b < nrows; r0b += 16) {
        float v[16];
        int g[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          *(float4*)(v + 4 * q) = *(const float4*)(src + r0b + 4 * q);
          *(int4*)(g + 4 * q) = *(const int4*)(rgrp + r0b + 4 * q);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          if (r0b + q < nrows) {
            if (g[q] != cur) {
              P.part[((int64_t)(pb + cur - gf) * 2 + which) * D + chan] = sum;
              sum = 0.f;
              cur = g[q];
            }
            sum += v[q];
          }
        }
      }
      P.part[((int64_t)(pb + cur - gf) * 2 + which) * D + chan] = sum;
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

// psi of 16 neighbourhoods x 64 output channels per workgroup (blockIdx.x,
// blockIdx.y) on the FP32 matrix cores, a 16-channel tile per wave: lane
// (i, q) = (lane % 16, lane / 16) supplies row i of the means and column i of
// the (bfloat16, widened exactly) weights for input channels k = q * D/4 + s
// at step s, so each lane reads contiguous runs of both.
template <int D>
__global__ void __launch_bounds__(256) k_agg_psi(Params P) {
  constexpr int KQ = D / 4;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = l & 15, q = l >> 4;
  const int64_t g0 = (int64_t)blockIdx.x * 16;
  const int c0 = blockIdx.y * 64 + wave * 16;
  const int64_t g = g0 + i < P.G ? g0 + i : 0;   // rows past the last neighbourhood: any row, not stored
  const float* yrow = P.ymean + g * D + q * KQ;
  const uint16_t* wrow = P.wo + (int64_t)(c0 + i) * D + q * KQ;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s0 = 0; s0 < KQ; s0 += 8) {
    const float4 a0 = *(const float4*)(yrow + s0), a1 = *(const float4*)(yrow + s0 + 4);
    const uint4 wv = *(const uint4*)(wrow + s0);
    const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
    const uint32_t h[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2 * u], __uint_as_float(h[u] << 16), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2 * u + 1], __uint_as_float(h[u] & 0xffff0000u), acc, 0, 0, 0);
    }
  }
  const float bo = P.bo[c0 + i];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t gg = g0 + 4 * q + r;
    if (gg < P.G) P.psi[gg * D + c0 + i] = acc[r] + bo;
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
  const int lds = CH * (D + 8) * 2 + CH * 4 + NW * 2 * CH * 16 * 4;
  if (hipFuncSetAttribute((const void*)k_agg_gate<D>, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return BA_E_HIP;
  // chunks per workgroup: about one workgroup per CU over all slices, so
  // each slice's weights are read once per CU
  constexpr int NS = D / (16 * NW);
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
    n_cu = 256;
  const int cpw = (int)std::max<int64_t>(1, (NC * NS + n_cu - 1) / n_cu);
  const int64_t groups = (NC + cpw - 1) / cpw;
  if (groups > 0) hipLaunchKernelGGL(k_agg_gate<D>, dim3((unsigned)(groups * NS)), dim3(64 * NW), lds, s, P, NC, cpw);
  hipLaunchKernelGGL(k_agg_mean, dim3((unsigned)std::min<int64_t>((P.G * D + 255) / 256, 16384)), dim3(256), 0, s,
                     P);
  hipLaunchKernelGGL(k_agg_psi<D>, dim3((unsigned)((P.G + 15) / 16), D / 64), dim3(256), 0, s, P);
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
