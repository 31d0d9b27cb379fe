/*
 * dpagg.h - C ABI of the gfx950 soft aggregation of Deep Patch Visual
 * Odometry (Teed, Lipson, Deng, arXiv 2208.04726), built into libdpba.so.
 *
 * The update operator exchanges information between the edges of the patch
 * graph with a channel-wise soft aggregation (Sec. 3.1 "SoftMax Aggregation",
 * Eq. 5): for edge e with neighbours N(e) and hidden states x,
 *
 *     out_e = psi( sum_{x in N(e)} sigma(x) * phi(x) / sum_{x in N(e)} sigma(x) )
 *
 * with phi and psi linear layers and sigma a linear layer followed by a
 * sigmoid, in two instantiations: patch aggregation (neighbours share the
 * patch) and frame aggregation (neighbours share the target frame, and their
 * patches share the source frame).
 *
 * Conventions (the paper fixes none of these):
 *   - N(e) contains e: the neighbours of e are all edges with its key;
 *   - the layers map the hidden dimension onto itself, y = W x + b, W stored
 *     [out, in] in bfloat16, b in FP32; hidden states bfloat16 [E, dim];
 *   - products in FP32 on the matrix cores (bfloat16 operands), sums and
 *     the output in FP32; the sums of a neighbourhood run in edge order, so
 *     results are deterministic and independent of scheduling.
 *
 * Memory: "dev" pointers are device pointers on the current HIP device, owned
 * by the caller; the caller provides the workspace (dpa_workspace_bytes);
 * nothing is allocated.  Calls enqueue work on `stream` and return at once.
 * Errors: BA_OK (0) or BA_E_INVAL (-1) / BA_E_HIP (-3) of dpba.h, checked
 * before anything is enqueued (launch failures excepted).
 */
#ifndef DPAGG_H
#define DPAGG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DPA_PATCH = 0, DPA_FRAME = 1 };

typedef struct {
  int32_t mode;            /* DPA_PATCH or DPA_FRAME                               */
  int32_t dim;             /* hidden dimension: 128, 256, 384 or 512               */
  int64_t n_edges;         /* E                                                    */
  int64_t n_patches;       /* M                                                    */
  int32_t n_frames;        /* F: frames of the window (source and target frames)  */
  int32_t graph_ready;     /* nonzero: the workspace holds the neighbourhoods an
                              earlier call built for the same mode, sizes, kk, jj
                              and anchor (unchanged since), and they are reused;
                              zero: they are built (the update operator keeps its
                              graph across iterations)                             */
  const uint16_t* x;       /* dev bf16 [E, dim]: hidden state of each edge          */
  const int32_t* kk;       /* dev [E] patch of each edge                           */
  const int32_t* jj;       /* dev [E] target frame of each edge                    */
  const int32_t* anchor;   /* dev [M] source frame of each patch (DPA_FRAME)       */
  const uint16_t* w_gate;  /* dev bf16 [dim, dim]: sigma's linear layer            */
  const float* b_gate;     /* dev f32 [dim]                                        */
  const uint16_t* w_val;   /* dev bf16 [dim, dim]: phi                             */
  const float* b_val;      /* dev f32 [dim]                                        */
  const uint16_t* w_out;   /* dev bf16 [dim, dim]: psi                             */
  const float* b_out;      /* dev f32 [dim]                                        */
  float* out;              /* dev f32 [E, dim]                                     */
  void* workspace;         /* dev, dpa_workspace_bytes(...) bytes, clobbered       */
  int64_t workspace_bytes;
  int32_t* status;         /* dev [1] or NULL: bit 4 (BA_W_BAD_INDEX) is or-ed in
                              when an edge's kk, jj or its patch's source frame is
                              out of range; that edge's output is zero             */
} dpa_problem;

/* Workspace of dpa_softagg for these sizes (bytes), or -1 if they are invalid. */
int64_t dpa_workspace_bytes(int32_t mode, int32_t dim, int64_t n_edges, int64_t n_patches, int32_t n_frames);

/* Eq. 5 for every edge of *p.  BA_E_INVAL for a bad mode or dim, negative or
 * oversize counts, null pointers (with E > 0) or a workspace smaller than
 * dpa_workspace_bytes. */
int dpa_softagg(const dpa_problem* p, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DPAGG_H */
