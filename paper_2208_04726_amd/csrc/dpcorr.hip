// Correlation features (include/dpcorr.h) on gfx950: Eq. 4 of Sec. 3.1 at
// both levels of the matching-feature pyramid, and the average pooling that
// makes the second level.
//
// One wave per edge.  Correlation is linear in the sampled features, so each
// bilinear sample of Eq. 4 is the same bilinear combination of the inner
// products at its four integer neighbours.  Per edge and level the wave
//   1. takes the integer box that holds every lattice point the p*p pixels'
//      7x7 grids touch (for 3x3 patches about 10x10 points: the pixels'
//      8x8 lattices overlap),
//   2. forms the inner products of all p*p patch features with all box
//      features as one matrix product, G (p*p x D) times F_box^T (D x box),
//      on the 16x16x32 bfloat16 matrix cores with FP32 accumulation (each
//      box feature is read once, straight into the operand registers),
//   3. writes the products to LDS and combines each output from its four
//      lattice neighbours with the pixel's bilinear weights (FP32),
//      storing the p*p*49 outputs of the level contiguously.
// A pixel whose whole lattice lies outside the map contributes zeros; when
// the pixels are spread so far that the union box exceeds NBMAX points, the
// pixels are taken one at a time with their own 8x8 lattices.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/dpba.h"
#include "../../include/dpcorr.h"

namespace dpcorr {

constexpr int WAVES = 4;            // edges per workgroup
constexpr int RAD = 3;              // 7 x 7 grid (Eq. 4)
constexpr int GRID = 2 * RAD + 1;
constexpr int LAT = GRID + 1;       // lattice points per pixel and axis
constexpr int NBMAX = 160;          // union box points per level (10 tiles of 16)
constexpr int PMAX = 16;            // patch pixels (rows of the matrix-core tile)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct PixelBox {       // per pixel of the current level, in LDS
  float x, y;           // level coordinates
  int ix, iy;           // floor of the coordinates
  int bx0, by0, wb;     // lattice box of the pixel's products: origin and width
  int live;             // 0: every lattice point outside the map
};

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t* p) {
  const uint4 v = *(const uint4*)p;
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero_bf16x8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// LDS written by some lanes of a wave and then read by others of the same
// wave: wait for this wave's LDS operations and keep the compiler from
// moving memory operations across.
__device__ __forceinline__ void wave_lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

struct Params {
  int D, P2;
  int H0, W0, H1, W1;
  float inv_s1;
  int64_t M, E;
  int F;
  const uint16_t* f0;
  const uint16_t* f1;
  const uint16_t* gmap;
  const float* coords;
  const int32_t* kk;
  const int32_t* jj;
  float* out;
  int32_t* status;
};

// Products of the patch features (operand a: lane row l & 15, channels
// 8*(l >> 4) .. + 7 of each 32-channel block) with the features of the `nb`
// lattice points of the box with origin (bx0, by0) and width wb; rows < P2
// (only row `row_keep` when it is >= 0) go to raw[row * NBMAX + point].
// Tiles are taken TG at a time, every load of the group issued before its
// matrix-core products.
template <int KB, int TG>
__device__ __forceinline__ void box_products(const bf16x8 (&a)[KB], const uint16_t* fm, int H, int W, int bx0,
                                             int by0, int wb, int nb, int row_keep, float* raw, int P2) {
  const int l = threadIdx.x & 63;
  const int kq = l >> 4, col = l & 15;
  const int D = KB * 32;
  for (int t0 = 0; t0 < nb; t0 += 16 * TG) {
    bf16x8 b[TG][KB];
#pragma unroll
    for (int g = 0; g < TG; ++g) {
      const int n = t0 + 16 * g + col;
      const int bx = bx0 + n % wb, by = by0 + n / wb;
      const bool ok = n < nb && bx >= 0 && bx < W && by >= 0 && by < H;
      const uint16_t* src = fm + ((int64_t)(ok ? by : 0) * W + (ok ? bx : 0)) * D + kq * 8;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) b[g][kb] = ok ? load_bf16x8(src + kb * 32) : zero_bf16x8();
    }
#pragma unroll
    for (int g = 0; g < TG; ++g) {
      const int n = t0 + 16 * g + col;
      if (t0 + 16 * g >= nb) break;   // uniform: the group's remaining tiles are empty
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kb], b[g][kb], acc, 0, 0, 0);
      if (n < nb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 4 * kq + r;
          if (row < P2 && (row_keep < 0 || row == row_keep)) raw[row * NBMAX + n] = acc[r];
        }
      }
    }
  }
}

// Tiles per load group.  Measured on MI355X for D = 128 (22 x 96 graph,
// 39,552 edges): groups of 2 tiles with a 5-waves-per-SIMD register target,
// 0.212 ms; groups of 4 (138 registers, 3 waves), 0.243 ms; one tile at a
// time, 0.245 ms.
template <int KB>
struct TileGroup {
  static constexpr int value = 2;
};

// LDS of a workgroup: per wave the lattice products of its P2 rows and the
// pixel boxes.
__host__ __device__ constexpr int corr_lds_bytes(int P2) {
  return WAVES * (P2 * NBMAX * 4 + PMAX * (int)sizeof(PixelBox));
}

template <int KB>
__device__ __forceinline__ void corr_edge(const Params& P, char* smem) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * WAVES + wave;
  if (e >= P.E) return;   // the whole wave leaves; no workgroup barrier follows
  const int P2 = P.P2;
  const int D = KB * 32;
  const int k = P.kk[e], j = P.jj[e];
  float* out_e = P.out + e * (2 * P2 * GRID * GRID);
  if (k < 0 || k >= P.M || j < 0 || j >= P.F) {
    for (int o = l; o < 2 * P2 * GRID * GRID; o += 64) out_e[o] = 0.f;
    if (l == 0 && P.status) atomicOr(P.status, BA_W_BAD_INDEX);
    return;
  }
  float* raw = (float*)(smem + wave * (P2 * NBMAX * 4));
  PixelBox* pix = (PixelBox*)(smem + WAVES * P2 * NBMAX * 4) + wave * PMAX;
  // operand a: patch feature rows (zero beyond the patch's pixels)
  bf16x8 a[KB];
  {
    const int m = l & 15, kq = l >> 4;
    const uint16_t* g = P.gmap + ((int64_t)k * P2 + (m < P2 ? m : 0)) * D + kq * 8;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) a[kb] = m < P2 ? load_bf16x8(g + kb * 32) : zero_bf16x8();
  }
  for (int level = 0; level < 2; ++level) {
    const int H = level ? P.H1 : P.H0, W = level ? P.W1 : P.W0;
    const float sc = level ? P.inv_s1 : 1.0f;
    const uint16_t* fm = (level ? P.f1 : P.f0) + (int64_t)j * H * W * D;
    // pixels: coordinates, and whether any lattice point can be inside
    int ix = 0, iy = 0, live = 0;
    float x = 0.f, y = 0.f;
    if (l < P2) {
      x = P.coords[(e * P2 + l) * 2 + 0] * sc;
      y = P.coords[(e * P2 + l) * 2 + 1] * sc;
      // the lattice spans floor - 3 .. floor + 4: beyond these limits (or
      // not finite) every point is outside
      live = (x > -6.0f && x < (float)W + 5.0f && y > -6.0f && y < (float)H + 5.0f) ? 1 : 0;
      if (live) {
        ix = (int)floorf(x);
        iy = (int)floorf(y);
      }
    }
    const int big = 1 << 30;
    const int lo_x = wave_min(live ? ix : big), hi_x = wave_max(live ? ix : -big);
    const int lo_y = wave_min(live ? iy : big), hi_y = wave_max(live ? iy : -big);
    const bool any = lo_x != big;
    const int wb = any ? hi_x - lo_x + LAT : 0, hb = any ? hi_y - lo_y + LAT : 0;
    const bool united = any && wb * hb <= NBMAX;
    if (l < P2) {
      PixelBox b;
      b.x = x;
      b.y = y;
      b.ix = ix;
      b.iy = iy;
      b.live = live;
      b.bx0 = united ? lo_x - RAD : ix - RAD;
      b.by0 = united ? lo_y - RAD : iy - RAD;
      b.wb = united ? wb : LAT;
      pix[l] = b;
    }
    if (united) {
      box_products<KB, TileGroup<KB>::value>(a, fm, H, W, lo_x - RAD, lo_y - RAD, wb, wb * hb, -1, raw, P2);
    } else if (any) {
      for (int m = 0; m < P2; ++m) {
        const int lm = __shfl(live, m);
        if (!lm) continue;
        const int bx = __shfl(ix, m) - RAD, by = __shfl(iy, m) - RAD;
        box_products<KB, TileGroup<KB>::value>(a, fm, H, W, bx, by, LAT, LAT * LAT, m, raw, P2);
      }
    }
    wave_lds_sync();
    // bilinear combination of the lattice products
    float* out_l = out_e + level * P2 * GRID * GRID;
    for (int o = l; o < P2 * GRID * GRID; o += 64) {
      const int m = o / (GRID * GRID), rem = o - m * (GRID * GRID);
      const int al = rem / GRID, be = rem - al * GRID;
      const PixelBox b = pix[m];
      float v = 0.f;
      if (b.live) {
        const float fx = b.x - (float)b.ix, fy = b.y - (float)b.iy;
        const int c = (b.iy - RAD + al - b.by0) * b.wb + (b.ix - RAD + be - b.bx0);
        const float* r = raw + m * NBMAX;
        v = (1.f - fy) * ((1.f - fx) * r[c] + fx * r[c + 1]) + fy * ((1.f - fx) * r[c + b.wb] + fx * r[c + b.wb + 1]);
      }
      out_l[o] = v;
    }
    wave_lds_sync();
  }
}

// D = 64, 128: a register target of 5 waves per SIMD (measured faster, see
// TileGroup); D = 256 keeps the default (the target would spill).
template <int KB>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(5))) k_corr(Params P) {
  extern __shared__ __align__(16) char smem[];
  corr_edge<KB>(P, smem);
}

__global__ void __launch_bounds__(64 * WAVES) k_corr_wide(Params P) {
  extern __shared__ __align__(16) char smem[];
  corr_edge<8>(P, smem);
}

// Average pooling: one thread per 8 channels of an output pixel.
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0u;   // NaN stays NaN
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;                                // nearest, ties to even
}

__global__ void __launch_bounds__(256) k_pool(const uint16_t* in, int F, int H, int W, int D, int s, uint16_t* out) {
  const int h = H / s, w = W / s, g8 = D / 8;
  const int64_t total = (int64_t)F * h * w * g8;
  const float inv = 1.0f / (float)(s * s);
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int c8 = (int)(t % g8);
    int64_t r = t / g8;
    const int ox = (int)(r % w);
    r /= w;
    const int oy = (int)(r % h);
    const int f = (int)(r / h);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int dy = 0; dy < s; ++dy) {
      for (int dx = 0; dx < s; ++dx) {
        const uint4 v = *(const uint4*)(in + (((int64_t)f * H + oy * s + dy) * W + ox * s + dx) * D + c8 * 8);
        const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc[2 * i] += bf16_to_f32(q[i] & 0xffffu);
          acc[2 * i + 1] += bf16_to_f32(q[i] >> 16);
        }
      }
    }
    uint4 o;
    o.x = f32_to_bf16(acc[0] * inv) | (f32_to_bf16(acc[1] * inv) << 16);
    o.y = f32_to_bf16(acc[2] * inv) | (f32_to_bf16(acc[3] * inv) << 16);
    o.z = f32_to_bf16(acc[4] * inv) | (f32_to_bf16(acc[5] * inv) << 16);
    o.w = f32_to_bf16(acc[6] * inv) | (f32_to_bf16(acc[7] * inv) << 16);
    *(uint4*)(out + (((int64_t)f * h + oy) * w + ox) * D + c8 * 8) = o;
  }
}

__global__ void k_debug_mfma_bf16(const uint16_t* A, const uint16_t* B, float* Dm) {
  const int l = threadIdx.x;
  const int row = l & 15, kq = l >> 4;
  uint16_t av[8], bv[8];
  for (int i = 0; i < 8; ++i) {
    av[i] = A[row * 32 + kq * 8 + i];        // A[row][k]
    bv[i] = B[(kq * 8 + i) * 16 + row];      // B[k][col], col = l & 15
  }
  const bf16x8 a = __builtin_bit_cast(bf16x8, av);
  const bf16x8 b = __builtin_bit_cast(bf16x8, bv);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) Dm[(4 * kq + r) * 16 + (l & 15)] = acc[r];
}

}  // namespace dpcorr

using namespace dpcorr;

extern "C" {

int dpc_correlation(const dpc_corr_problem* p, void* stream) {
  if (!p) return BA_E_INVAL;
  if (p->n_edges < 0 || p->n_frames < 0 || p->n_patches < 0) return BA_E_INVAL;
  if (p->n_edges == 0) return BA_OK;
  const int D = p->channels, P2 = p->patch_pixels;
  if (D != 64 && D != 128 && D != 256) return BA_E_INVAL;
  if (P2 != 1 && P2 != 4 && P2 != 9 && P2 != 16) return BA_E_INVAL;
  if (p->height0 < 1 || p->width0 < 1 || p->height1 < 1 || p->width1 < 1) return BA_E_INVAL;
  if (!(p->scale1 > 0.0f) || !std::isfinite(p->scale1)) return BA_E_INVAL;
  if (p->n_frames < 1 || p->n_patches < 1) return BA_E_INVAL;
  if (!p->level0 || !p->level1 || !p->gmap || !p->coords || !p->kk || !p->jj || !p->out) return BA_E_INVAL;
  Params P{};   // every field zero unless set below
  P.D = D;
  P.P2 = P2;
  P.H0 = p->height0;
  P.W0 = p->width0;
  P.H1 = p->height1;
  P.W1 = p->width1;
  P.inv_s1 = 1.0f / p->scale1;
  P.M = p->n_patches;
  P.E = p->n_edges;
  P.F = p->n_frames;
  P.f0 = p->level0;
  P.f1 = p->level1;
  P.gmap = p->gmap;
  P.coords = p->coords;
  P.kk = p->kk;
  P.jj = p->jj;
  P.out = p->out;
  P.status = p->status;
  const int64_t blocks = (p->n_edges + WAVES - 1) / WAVES;
  if (blocks > 0x7fffffffLL) return BA_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const int lds = corr_lds_bytes(P2);
  if (D == 64) hipLaunchKernelGGL(k_corr<2>, dim3((unsigned)blocks), dim3(64 * WAVES), lds, s, P);
  else if (D == 128) hipLaunchKernelGGL(k_corr<4>, dim3((unsigned)blocks), dim3(64 * WAVES), lds, s, P);
  else hipLaunchKernelGGL(k_corr_wide, dim3((unsigned)blocks), dim3(64 * WAVES), lds, s, P);
  return hipGetLastError() == hipSuccess ? BA_OK : BA_E_HIP;
}

int dpc_avg_pool(const uint16_t* in, int32_t n_frames, int32_t height, int32_t width, int32_t channels, int32_t s,
                 uint16_t* out, void* stream) {
  if (n_frames < 0 || height < 0 || width < 0 || channels < 8 || channels % 8 != 0 || s < 1 || s > 8)
    return BA_E_INVAL;
  const int64_t total = (int64_t)n_frames * (height / s) * (width / s) * (channels / 8);
  if (total == 0) return BA_OK;
  if (!in || !out) return BA_E_INVAL;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_pool, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, in, n_frames, height, width,
                     channels, s, out);
  return hipGetLastError() == hipSuccess ? BA_OK : BA_E_HIP;
}

int dpc_debug_mfma_bf16(const uint16_t* A, const uint16_t* B, float* D, void* stream) {
  if (!A || !B || !D) return BA_E_INVAL;
  hipLaunchKernelGGL(k_debug_mfma_bf16, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, D);
  return hipGetLastError() == hipSuccess ? BA_OK : BA_E_HIP;
}

}  // extern "C"
