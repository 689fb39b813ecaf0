// Shared definitions of the EDPC HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace edpc {

typedef uint16_t bf16_t;  // storage type of BF16 values (bit pattern)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Round-to-nearest-even FP32 -> BF16 (the gfx950 conversion instruction;
// NaN stays NaN).
__device__ __forceinline__ bf16_t f2bf(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }

// Per-step scalars, written on the device by the step-advance kernel so that
// the same launch sequence (or a captured graph of it) serves every step.
struct StepState {
  int32_t step;      // position i in the streams
  int32_t rows;      // active rows (streams) this step
  float inv_rows;    // 1 / rows (the mean of Eq. 2)
  float bc1, bc2;    // Adam bias corrections 1 - beta^tau
  uint32_t tau;      // Adam step number (1 for the first update)
  int32_t model;     // 1 if the model runs this step (step >= context)
  int32_t base;      // step before a captured window; its steps count from it
};

// Adam constants (Kingma & Ba 2015; lr from the configuration).
struct AdamCfg {
  float lr, beta1, beta2, eps;
};

// Adam's bias correction 1 - beta^tau, formed as -expm1(tau log1p(beta - 1))
// so that it keeps full FP32 relative accuracy at small tau (1 - powf loses
// log2(1 / (1 - beta^tau)) bits to cancellation, about 8 bits at beta 0.999
// and tau 3).  beta - 1 is exact in FP32 for beta in [0.5, 1]; beta = 0
// gives 1.  tau = 0 (no update yet) gives 0.
__device__ __forceinline__ float adam_bias_correction(float beta, uint32_t tau) {
  if (tau == 0) return 0.0f;
  if (beta <= 0.0f) return 1.0f;
  return -expm1f((float)tau * log1pf(beta - 1.0f));
}

__device__ __forceinline__ float gelu_f(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = expf(-0.5f * x * x) * 0.39894228040143268f;
  return cdf + x * pdf;
}

// Fixed-order wave reductions (butterfly over the 64 lanes).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    uint32_t w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// Global-memory view of a generic pointer.  Pointers read from device memory
// (job tables) are generic to the compiler, which then emits flat accesses;
// flat loads also count against the LDS wait counter, so every LDS access
// after them waits for the loads.  Accessing through this view gives global
// loads and stores.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// 16-byte global loads and stores through the global view (HIP's vector
// classes cannot be assigned across address spaces, so the data moves as a
// native 4 x 32-bit vector).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_global16(const void* p) {
  const u32x4 v = *(const __attribute__((address_space(1))) u32x4*)p;
  return __builtin_bit_cast(uint4, v);
}
__device__ __forceinline__ void st_global16(void* p, uint4 x) {
  *(__attribute__((address_space(1))) u32x4*)p = __builtin_bit_cast(u32x4, x);
}
// A 16-byte load issued unconditionally: where `ok` is false it reads 16
// zero bytes kept in device memory.  With no branch around the load and no
// select after it, the compiler counts outstanding loads exactly and needs
// the data only where it is consumed, so tiles staged ahead stay in flight
// under the matrix products instead of being waited for right away.
__device__ __align__(16) static const uint32_t kZero16[4] = {0u, 0u, 0u, 0u};
__device__ __forceinline__ uint4 ld_global16_or_zero(const void* p, bool ok) {
  return ld_global16(ok ? p : (const void*)kZero16);
}

// p[0] + p[stride] + ... + p[(n-1) stride], added strictly in index order;
// the loads are issued 32 at a time so their latencies overlap (slots past n
// add an exact zero).
__device__ __forceinline__ float ordered_sum(const float* __restrict__ pg, size_t stride, int n) {
  const auto p = gl(pg);
  float s = 0.f;
  for (int k = 0; k < n; k += 32) {
    float v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) v[q] = k + q < n ? p[(size_t)(k + q) * stride] : 0.f;
#pragma unroll
    for (int q = 0; q < 32; ++q) s += v[q];
  }
  return s;
}

}  // namespace edpc
