/*
 * dpcorr.h - C ABI of the gfx950 correlation features of Deep Patch Visual
 * Odometry (Teed, Lipson, Deng, arXiv 2208.04726), built into libdpba.so.
 *
 * For every edge (k, j) of the patch graph and every pixel (u, v) of patch
 * k, the update operator correlates the patch feature g_uv with the features
 * of frame j bilinearly sampled on a 7 x 7 integer grid centred at the
 * pixel's reprojection P'_kj(u, v) (Sec. 3.1 "Correlation", Eq. 4), at both
 * levels of the matching-feature pyramid, the second level made by average
 * pooling (Sec. 3 "Feature and Patch Extraction"), the two results
 * concatenated (Appendix "Correlation Operation").
 *
 * Conventions (the paper fixes none of these):
 *   - feature maps are bfloat16, [frame, row y, column x, channel] with the
 *     channels contiguous; patch features bfloat16 [patch, pixel u*p+v,
 *     channel]; products are accumulated in FP32;
 *   - integer coordinates are pixel centres; a pixel outside the map is a
 *     zero feature (zero padding of the bilinear sample);
 *   - reprojected coordinates are (x, y) in pixels of the first level; the
 *     second level samples at (x, y) / scale1;
 *   - output (alpha, beta) is the grid offset (dy, dx) = (alpha-3, beta-3);
 *     an edge's output is [level][pixel][alpha][beta], FP32;
 *   - a pixel with a non-finite coordinate correlates with zero features.
 *
 * Memory: "dev" pointers are device pointers on the current HIP device, owned
 * by the caller; nothing is allocated.  Calls enqueue work on `stream` (a
 * hipStream_t as void*, NULL = default stream) and return at once.
 * Errors: BA_OK (0) or BA_E_INVAL (-1) / BA_E_HIP (-3) of dpba.h, checked
 * before anything is enqueued (launch failures excepted).
 */
#ifndef DPCORR_H
#define DPCORR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_frames;        /* F                                                  */
  int32_t channels;        /* D: 64, 128 or 256                                  */
  int32_t height0, width0; /* first-level map, dev bf16 [F, height0, width0, D]  */
  int32_t height1, width1; /* second-level map, dev bf16 [F, height1, width1, D] */
  float scale1;            /* > 0: second-level coordinates = first-level / scale1 */
  int32_t patch_pixels;    /* p*p: 1, 4, 9 or 16                                 */
  int64_t n_patches;       /* M                                                  */
  int64_t n_edges;         /* E                                                  */
  const uint16_t* level0;  /* dev bf16                                           */
  const uint16_t* level1;  /* dev bf16                                           */
  const uint16_t* gmap;    /* dev bf16 [M, p*p, D]                               */
  const float* coords;     /* dev f32 [E, p*p, 2]: (x, y) of each reprojected patch pixel, first-level pixels */
  const int32_t* kk;       /* dev [E] patch of each edge                         */
  const int32_t* jj;       /* dev [E] target frame of each edge                  */
  float* out;              /* dev f32 [E, 2, p*p, 7, 7]                          */
  int32_t* status;         /* dev [1] or NULL: bit 4 (BA_W_BAD_INDEX) is or-ed in when
                              an edge's kk or jj is out of range; that edge's
                              outputs are zero                                   */
} dpc_corr_problem;

/* Eq. 4 at both pyramid levels for every edge of *p.  BA_E_INVAL for a null
 * pointer (with E > 0), unsupported channels / patch_pixels, non-positive
 * sizes or scale1. */
int dpc_correlation(const dpc_corr_problem* p, void* stream);

/* The second pyramid level (Sec. 3: average pooling, s x s filter, stride
 * s): out[f, y, x, :] = mean of in[f, s*y + a, s*x + b, :] over a, b < s,
 * accumulated in FP32 and rounded to the nearest bfloat16 (ties to even).
 * in: dev bf16 [F, H, W, D]; out: dev bf16 [F, H / s, W / s, D] (rows and
 * columns beyond the last whole block are dropped).  D a multiple of 8,
 * 1 <= s <= 8.  BA_E_INVAL otherwise. */
int dpc_avg_pool(const uint16_t* in, int32_t n_frames, int32_t height, int32_t width,
                 int32_t channels, int32_t s, uint16_t* out, void* stream);

/* Inspection entry point for tests: one 16x16x32 bfloat16 matrix-core
 * product D = A B of A (16x32, row-major, dev bf16) and B (32x16, row-major,
 * dev bf16) into D (16x16, row-major, dev f32), through the operand and
 * accumulator lane mapping the correlation kernel uses. */
int dpc_debug_mfma_bf16(const uint16_t* A, const uint16_t* B, float* D, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DPCORR_H */
