// Adam on the shared parameters (Sec. 4.1: Adam, Kingma & Ba 2015, with
// bias correction) and the BF16 copies the products read.
#pragma once
#include "common.h"

namespace edpc {

// The Adam step (Kingma & Ba 2015, bias-corrected) on 8 parameters P with
// moments M, V and gradients gv, in place; lr_bc = lr / (1 - beta1^tau),
// inv_bc2 = 1 / (1 - beta2^tau).
__device__ __forceinline__ void adam8_math(float P[8], float M[8], float V[8], const float gv[8],
                                           float lr_bc, float inv_bc2, const AdamCfg& ac) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    M[k] = ac.beta1 * M[k] + (1.0f - ac.beta1) * gv[k];
    V[k] = ac.beta2 * V[k] + (1.0f - ac.beta2) * gv[k] * gv[k];
    P[k] = P[k] - lr_bc * M[k] / (sqrtf(V[k] * inv_bc2) + ac.eps);
  }
}

typedef float f32v4 __attribute__((ext_vector_type(4)));

// Loads of 8 consecutive parameters and their moments (moments are touched
// once per step: non-temporal).
__device__ __forceinline__ void adam8_load(const float* pp, const float* mp, const float* vp,
                                           float P[8], float M[8], float V[8]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float4 p4 = ((const float4*)pp)[h];
    const f32v4 mv = __builtin_nontemporal_load((const f32v4*)mp + h);
    const f32v4 vv = __builtin_nontemporal_load((const f32v4*)vp + h);
    P[4 * h] = p4.x; P[4 * h + 1] = p4.y; P[4 * h + 2] = p4.z; P[4 * h + 3] = p4.w;
    M[4 * h] = mv.x; M[4 * h + 1] = mv.y; M[4 * h + 2] = mv.z; M[4 * h + 3] = mv.w;
    V[4 * h] = vv.x; V[4 * h + 1] = vv.y; V[4 * h + 2] = vv.z; V[4 * h + 3] = vv.w;
  }
}

__device__ __forceinline__ void adam8_store(float* pp, float* mp, float* vp, const float P[8],
                                            const float M[8], const float V[8]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    ((float4*)pp)[h] = make_float4(P[4 * h], P[4 * h + 1], P[4 * h + 2], P[4 * h + 3]);
    __builtin_nontemporal_store(f32v4{M[4 * h], M[4 * h + 1], M[4 * h + 2], M[4 * h + 3]},
                                (f32v4*)mp + h);
    __builtin_nontemporal_store(f32v4{V[4 * h], V[4 * h + 1], V[4 * h + 2], V[4 * h + 3]},
                                (f32v4*)vp + h);
  }
}

// Adam on 8 consecutive parameters with gradients gv; the updated values are
// returned in out.
__device__ __forceinline__ void adam8(float* pp, const float gv[8], float* mp, float* vp, float lr_bc,
                                      float inv_bc2, const AdamCfg& ac, float out[8]) {
  float P[8], M[8], V[8];
  adam8_load(pp, mp, vp, P, M, V);
  adam8_math(P, M, V, gv, lr_bc, inv_bc2, ac);
  adam8_store(pp, mp, vp, P, M, V);
#pragma unroll
  for (int k = 0; k < 8; ++k) out[k] = P[k];
}

// 8 values rounded to BF16, packed in order into 16 bytes.
__device__ __forceinline__ uint4 pack_bf16x8(const float v[8]) {
  return make_uint4((uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                    (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16),
                    (uint32_t)f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16),
                    (uint32_t)f2bf(v[6]) | ((uint32_t)f2bf(v[7]) << 16));
}

__device__ __forceinline__ void load8(const float* q, float out[8]) {
  const float4 a = ((const float4*)q)[0], b = ((const float4*)q)[1];
  out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
  out[4] = b.x; out[5] = b.y; out[6] = b.z; out[7] = b.w;
}


// Adam over the shared parameters fused with the fragment-copy refresh:
// matrix jobs are walked in 32 x 64 tiles (rows a multiple of 32, columns a
// multiple of 64), the other tensors in items of 256 elements; one
// workgroup per item.  The gradient of an element-range job may be formed
// here from per-row-block partials (bias, LayerNorm and embedding
// gradients): the sum over the step's row blocks in block order.
constexpr int kAdamTileRows = 32;
constexpr int kAdamTileCols = 64;
constexpr int kAdamVecItem = 256;
struct AdamJob {
  size_t off;        // element offset in the flat parameter buffers
  int rows, cols;    // matrix (cols > 0) or element range (cols == 0, rows = count)
  uint4* nt;         // fragment copies (matrix jobs)
  uint4* nn;
  const float* red;  // element-range jobs: partials of element 0 of row block 0, or null
  int red_ld;        // stride between row blocks in red
  int red_block;     // rows per partial (the step's partials: ceil(rows / red_block))
  int item_begin;    // first work item of this job
};

// One item (kAdamVecItem elements) of an element-range job: the gradient is
// the sum of the job's per-row-block partials in block order (when it has
// them), then scalar Adam.  One thread per element.
__device__ __forceinline__ void adam_elements(const StepState* st, const AdamJob& jb, int local,
                                              float* p, float* g, float* m, float* v,
                                              const AdamCfg& ac, float lr_bc, float inv_bc2) {
  const int e = local * kAdamVecItem + (int)threadIdx.x;
  if (e >= jb.rows) return;
  const size_t o = jb.off + e;
  float gr;
  if (jb.red) {
    gr = ordered_sum(jb.red + e, (size_t)jb.red_ld, (st->rows + jb.red_block - 1) / jb.red_block);
    g[o] = gr;
  } else {
    gr = g[o];
  }
  const float mm = ac.beta1 * m[o] + (1.0f - ac.beta1) * gr;
  const float vv = ac.beta2 * v[o] + (1.0f - ac.beta2) * gr * gr;
  p[o] -= lr_bc * mm / (sqrtf(vv * inv_bc2) + ac.eps);
  m[o] = mm;
  v[o] = vv;
}

}  // namespace edpc
