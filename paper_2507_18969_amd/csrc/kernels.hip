// Row-wise / element-wise kernels of one model step and the coder lanes.
#include "kernels.h"
#include "head_row.h"

namespace edpc {

static inline unsigned blocks_for(size_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

// ---------------------------------------------------------------------------
// Step state
// ---------------------------------------------------------------------------
// rows = number of streams with length > step (lens sorted decreasing).  A
// 256-way search: each round every thread tests one of 256 evenly spaced
// positions of the open range and the count of true tests narrows the range to
// one gap between positions, so n streams take ceil(log_256 n) rounds of one
// load each instead of log_2 n dependent loads.
constexpr int kScheduleThreads = 256;

__global__ void __launch_bounds__(kScheduleThreads) step_schedule_kernel(StepState* st, Schedule sc,
                                                                         int step) {
  if (step < 0) step = st->step + 1;
  const int rows = active_rows(sc, step);
  __syncthreads();  // every thread has read st->step
  if (threadIdx.x == 0) write_step_state(st, sc, step, rows);
}

void k_step_schedule(StepState* st, Schedule sc, int step, hipStream_t s) {
  hipLaunchKernelGGL(step_schedule_kernel, dim3(1), dim3(kScheduleThreads), 0, s, st, sc, step);
}

__global__ void step_set_kernel(StepState* st, int step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->step = step;
    st->base = step;
  }
}

void k_step_set(StepState* st, int step, hipStream_t s) {
  hipLaunchKernelGGL(step_set_kernel, dim3(1), dim3(64), 0, s, st, step);
}

__global__ void step_explicit_kernel(StepState* st, int rows, uint32_t tau, float beta1,
                                     float beta2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->step = -1;
  st->rows = rows;
  st->inv_rows = rows > 0 ? 1.0f / (float)rows : 0.0f;
  st->model = 1;
  st->tau = tau;
  st->bc1 = adam_bias_correction(beta1, tau);
  st->bc2 = adam_bias_correction(beta2, tau);
}

void k_step_explicit(StepState* st, int rows, uint32_t tau, float beta1, float beta2,
                     hipStream_t s) {
  hipLaunchKernelGGL(step_explicit_kernel, dim3(1), dim3(64), 0, s, st, rows, tau, beta1, beta2);
}

// ---------------------------------------------------------------------------
// Context window gather and byte embedding
// ---------------------------------------------------------------------------
__global__ void gather_kernel(const StepState* __restrict__ st, StreamIO io, int C,
                              uint8_t* __restrict__ ctx, uint8_t* __restrict__ tgt,
                              bool decoding) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx / C, c = idx % C;
  if (r >= st->rows) return;
  const int i = st->step;
  const uint32_t s = io.slot[r];
  const uint8_t* base = decoding ? io.dst : io.src;
  const uint64_t o = io.off[s];
  ctx[idx] = base[io_at(io, o, (uint64_t)(i - C + c))];
  if (!decoding && c == 0) tgt[r] = io.src[io_at(io, o, (uint64_t)i)];
}

void k_gather(const StepState* st, StreamIO io, int C, uint8_t* ctx, uint8_t* tgt, int max_rows,
              bool decoding, hipStream_t s) {
  const size_t n = (size_t)max_rows * C;
  hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, st, io, C, ctx, tgt,
                     decoding);
}

__global__ void embed_kernel(const StepState* __restrict__ st, const uint8_t* __restrict__ ctx,
                             const float* __restrict__ emb, int C, int E, float* __restrict__ x32,
                             bf16_t* __restrict__ x16) {
  const int F = C * E;
  const int q4 = F >> 2;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = idx / q4, f = (idx % q4) * 4;
  if (r >= st->rows) return;
  const int c = f / E, e = f % E;
  const int v = ctx[r * C + c];
  const float4 val = *(const float4*)(emb + v * E + e);
  if (x32) *(float4*)(x32 + (size_t)r * F + f) = val;
  if (x16) {
    ushort4 h = make_ushort4(f2bf(val.x), f2bf(val.y), f2bf(val.z), f2bf(val.w));
    *(ushort4*)(x16 + (size_t)r * F + f) = h;
  }
}

void k_embed(const StepState* st, const uint8_t* ctx, const float* emb, int C, int E, float* x32,
             bf16_t* x16, int max_rows, hipStream_t s) {
  const size_t n = (size_t)max_rows * C * E / 4;
  hipLaunchKernelGGL(embed_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, st, ctx, emb, C, E,
                     x32, x16);
}

// Streaming (non-temporal) 16-byte accesses for the Adam moments of the FDM:
// every element of m_U, v_U is read and written once per step, while U is
// read again by the next step's forward product and keeps normal caching.
__device__ __forceinline__ float4 nt_load4(const float* p) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 v = __builtin_nontemporal_load((const f4*)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store4(float* p, float4 x) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 v = {x.x, x.y, x.z, x.w};
  __builtin_nontemporal_store(v, (f4*)p);
}

// Rows of U_s whose loads are issued together in the FDM kernels.
constexpr int kFdmBatch = 4;

// ---------------------------------------------------------------------------
// Feature Distribution Matrix (Eq. 15): y_s = x'_s U_s, one workgroup per row.
// U_s is [Lin, Lout] (square for the FDM itself; the low-rank ablation's
// per-stream factors A_s [F, F'] and B_s [F', F] use the same kernels).
// Thread (g, t): t covers columns 4t..4t+3, group g rows l = g, g+G, ...
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) fdm_fwd_kernel(const StepState* __restrict__ st,
                                                      const float* __restrict__ x1,
                                                      const float* __restrict__ U,
                                                      const uint32_t* __restrict__ slot, int Lin,
                                                      int Lout, float* __restrict__ y32,
                                                      bf16_t* __restrict__ y16) {
  const int r = blockIdx.x;
  if (r >= st->rows) return;
  __shared__ float xs[256];
  __shared__ float part[1024];
  const int tpr = Lout >> 2, G = 256 / tpr;
  const int t = threadIdx.x % tpr, g = threadIdx.x / tpr;
  for (int l = threadIdx.x; l < Lin; l += 256) xs[l] = x1[(size_t)r * Lin + l];
  __syncthreads();
  const float* Us = U + (size_t)slot[r] * Lin * Lout;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (g < G) {
    // rows l = g, g + G, ... in order; loads issued kFdmBatch rows at a time
    int l = g;
    for (; l + (kFdmBatch - 1) * G < Lin; l += kFdmBatch * G) {
      float4 u[kFdmBatch];
#pragma unroll
      for (int q = 0; q < kFdmBatch; ++q) u[q] = *(const float4*)(Us + (size_t)(l + q * G) * Lout + 4 * t);
#pragma unroll
      for (int q = 0; q < kFdmBatch; ++q) {
        const float xv = xs[l + q * G];
        acc.x += xv * u[q].x;
        acc.y += xv * u[q].y;
        acc.z += xv * u[q].z;
        acc.w += xv * u[q].w;
      }
    }
    for (; l < Lin; l += G) {
      const float4 u = *(const float4*)(Us + (size_t)l * Lout + 4 * t);
      const float xv = xs[l];
      acc.x += xv * u.x;
      acc.y += xv * u.y;
      acc.z += xv * u.z;
      acc.w += xv * u.w;
    }
    *(float4*)(part + g * Lout + 4 * t) = acc;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < Lout; k += 256) {
    float y = 0.f;
    for (int gg = 0; gg < G; ++gg) y += part[gg * Lout + k];
    if (y32) y32[(size_t)r * Lout + k] = y;
    if (y16) y16[(size_t)r * Lout + k] = f2bf(y);
  }
}

void k_fdm_fwd(const StepState* st, const float* x1, const float* U, const uint32_t* slot, int Lin,
               int Lout, float* y32, bf16_t* y16, int max_rows, hipStream_t s) {
  hipLaunchKernelGGL(fdm_fwd_kernel, dim3(max_rows), dim3(256), 0, s, st, x1, U, slot, Lin, Lout,
                     y32, y16);
}

// Adjoint of Eq. 15 fused with the Adam step on U_s:
//   dx'_s = U_s dy_s (with U before the update), dU_s = x'_s (x) dy_s.
__global__ void __launch_bounds__(256) fdm_bwd_kernel(
    const StepState* __restrict__ st, const float* __restrict__ x1, const float* __restrict__ dy,
    float* __restrict__ U, float* __restrict__ mU, float* __restrict__ vU,
    float* __restrict__ dU_keep, const uint32_t* __restrict__ slot, int Lin, int Lout, AdamCfg ac,
    bool update,
    float* __restrict__ dx1_32, bf16_t* __restrict__ dx1_16) {
  const int r = blockIdx.x;
  if (r >= st->rows) return;
  __shared__ float xs[256];
  __shared__ float ds[256];
  const int tpr = Lout >> 2, G = 256 / tpr;
  const int t = threadIdx.x % tpr, g = threadIdx.x / tpr;
  for (int l = threadIdx.x; l < Lin; l += 256) xs[l] = x1[(size_t)r * Lin + l];
  for (int k = threadIdx.x; k < Lout; k += 256) ds[k] = dy[(size_t)r * Lout + k];
  __syncthreads();
  if (g >= G) return;
  const size_t base_s = (size_t)slot[r] * Lin * Lout;
  const float4 d4 = *(const float4*)(ds + 4 * t);
  const float b1 = ac.beta1, b2 = ac.beta2;
  const float lr_bc = ac.lr / st->bc1;
  const float inv_bc2 = 1.0f / st->bc2;
  // one row l of U_s: dx'[l] (from U before the update), dU, Adam
  auto row = [&](int l, float4 u, float4 m, float4 v) {
    const size_t idx = base_s + (size_t)l * Lout + 4 * t;
    float part = u.x * d4.x + u.y * d4.y + u.z * d4.z + u.w * d4.w;
    for (int o = tpr >> 1; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
    if (t == 0) {
      if (dx1_32) dx1_32[(size_t)r * Lin + l] = part;
      if (dx1_16) dx1_16[(size_t)r * Lin + l] = f2bf(part);
    }
    const float xv = xs[l];
    const float gr[4] = {xv * d4.x, xv * d4.y, xv * d4.z, xv * d4.w};
    if (dU_keep) *(float4*)(dU_keep + idx) = make_float4(gr[0], gr[1], gr[2], gr[3]);
    if (update) {
      float* up = (float*)&u;
      float* mp = (float*)&m;
      float* vp = (float*)&v;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        mp[j] = b1 * mp[j] + (1.0f - b1) * gr[j];
        vp[j] = b2 * vp[j] + (1.0f - b2) * gr[j] * gr[j];
        up[j] -= lr_bc * mp[j] / (sqrtf(vp[j] * inv_bc2) + ac.eps);
      }
      *(float4*)(U + idx) = u;
      nt_store4(mU + idx, m);
      nt_store4(vU + idx, v);
    }
  };
  // rows l = g, g + G, ...; the loads of kFdmBatch rows are issued before any
  // of them is used, so that each thread keeps 3 kFdmBatch 16-byte loads in
  // flight (the rows are independent: each updates its own slice of U_s)
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  int l = g;
  for (; l + (kFdmBatch - 1) * G < Lin; l += kFdmBatch * G) {
    float4 u[kFdmBatch], m[kFdmBatch], v[kFdmBatch];
#pragma unroll
    for (int q = 0; q < kFdmBatch; ++q) {
      const size_t idx = base_s + (size_t)(l + q * G) * Lout + 4 * t;
      u[q] = *(const float4*)(U + idx);
      m[q] = update ? nt_load4(mU + idx) : z4;
      v[q] = update ? nt_load4(vU + idx) : z4;
    }
#pragma unroll
    for (int q = 0; q < kFdmBatch; ++q) row(l + q * G, u[q], m[q], v[q]);
  }
  for (; l < Lin; l += G) {
    const size_t idx = base_s + (size_t)l * Lout + 4 * t;
    row(l, *(const float4*)(U + idx), update ? nt_load4(mU + idx) : z4,
        update ? nt_load4(vU + idx) : z4);
  }
}

void k_fdm_bwd(const StepState* st, const float* x1, const float* dy, float* U, float* mU,
               float* vU, float* dU_keep, const uint32_t* slot, int Lin, int Lout, AdamCfg ac,
               bool update, float* dx1_32, bf16_t* dx1_16, int max_rows, hipStream_t s) {
  hipLaunchKernelGGL(fdm_bwd_kernel, dim3(max_rows), dim3(256), 0, s, st, x1, dy, U, mU, vU,
                     dU_keep, slot, Lin, Lout, ac, update, dx1_32, dx1_16);
}

// ---------------------------------------------------------------------------
// LayerNorm (Eq. 9): one wave per row, biased variance, eps 1e-5.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) ln_fwd_kernel(const StepState* __restrict__ st,
                                                     const float* __restrict__ h,
                                                     const float* __restrict__ gamma,
                                                     const float* __restrict__ beta, int F,
                                                     float* __restrict__ z32,
                                                     bf16_t* __restrict__ z16,
                                                     float* __restrict__ mean,
                                                     float* __restrict__ rstd) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= st->rows) return;
  const float* hr = h + (size_t)r * F;
  float s = 0.f;
  for (int f = 4 * lane; f < F; f += 256) {
    const float4 x = *(const float4*)(hr + f);
    s += (x.x + x.y) + (x.z + x.w);
  }
  const float mu = wave_sum(s) / (float)F;
  float q = 0.f;
  for (int f = 4 * lane; f < F; f += 256) {
    const float4 x = *(const float4*)(hr + f);
    const float a = x.x - mu, b = x.y - mu, c = x.z - mu, d = x.w - mu;
    q += (a * a + b * b) + (c * c + d * d);
  }
  const float var = wave_sum(q) / (float)F;
  const float rs = 1.0f / sqrtf(var + 1e-5f);
  if (lane == 0) {
    mean[r] = mu;
    rstd[r] = rs;
  }
  for (int f = 4 * lane; f < F; f += 256) {
    const float4 x = *(const float4*)(hr + f);
    const float4 gm = *(const float4*)(gamma + f);
    const float4 bt = *(const float4*)(beta + f);
    float4 z;
    z.x = (x.x - mu) * rs * gm.x + bt.x;
    z.y = (x.y - mu) * rs * gm.y + bt.y;
    z.z = (x.z - mu) * rs * gm.z + bt.z;
    z.w = (x.w - mu) * rs * gm.w + bt.w;
    if (z32) *(float4*)(z32 + (size_t)r * F + f) = z;
    if (z16)
      *(ushort4*)(z16 + (size_t)r * F + f) = make_ushort4(f2bf(z.x), f2bf(z.y), f2bf(z.z), f2bf(z.w));
  }
}

// Register-resident variant for F = 256 * NV: each lane holds NV float4.
template <int NV>
__global__ void __launch_bounds__(256) ln_fwd_reg_kernel(const StepState* __restrict__ st,
                                                         const float* __restrict__ h,
                                                         const float* __restrict__ gamma,
                                                         const float* __restrict__ beta,
                                                         float* __restrict__ z32,
                                                         bf16_t* __restrict__ z16,
                                                         float* __restrict__ mean,
                                                         float* __restrict__ rstd) {
  constexpr int F = 256 * NV;
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= st->rows) return;
  const float* hr = h + (size_t)r * F;
  float4 x[NV];
  float s = 0.f;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    x[v] = *(const float4*)(hr + 4 * (lane + 64 * v));
    s += (x[v].x + x[v].y) + (x[v].z + x[v].w);
  }
  const float mu = wave_sum(s) / (float)F;
  float q = 0.f;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const float a = x[v].x - mu, b = x[v].y - mu, c = x[v].z - mu, d = x[v].w - mu;
    q += (a * a + b * b) + (c * c + d * d);
  }
  const float var = wave_sum(q) / (float)F;
  const float rs = 1.0f / sqrtf(var + 1e-5f);
  if (lane == 0) {
    mean[r] = mu;
    rstd[r] = rs;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int f = 4 * (lane + 64 * v);
    const float4 gm = *(const float4*)(gamma + f);
    const float4 bt = *(const float4*)(beta + f);
    float4 z;
    z.x = (x[v].x - mu) * rs * gm.x + bt.x;
    z.y = (x[v].y - mu) * rs * gm.y + bt.y;
    z.z = (x[v].z - mu) * rs * gm.z + bt.z;
    z.w = (x[v].w - mu) * rs * gm.w + bt.w;
    if (z32) *(float4*)(z32 + (size_t)r * F + f) = z;
    if (z16)
      *(ushort4*)(z16 + (size_t)r * F + f) = make_ushort4(f2bf(z.x), f2bf(z.y), f2bf(z.z), f2bf(z.w));
  }
}

void k_ln_fwd(const StepState* st, const float* h, const float* gamma, const float* beta, int F,
              float* z32, bf16_t* z16, float* mean, float* rstd, int max_rows, hipStream_t s) {
  const dim3 g(blocks_for(max_rows, 4)), b(256);
  switch (F % 256 == 0 ? F / 256 : 0) {
    case 1: hipLaunchKernelGGL(ln_fwd_reg_kernel<1>, g, b, 0, s, st, h, gamma, beta, z32, z16, mean, rstd); return;
    case 2: hipLaunchKernelGGL(ln_fwd_reg_kernel<2>, g, b, 0, s, st, h, gamma, beta, z32, z16, mean, rstd); return;
    case 4: hipLaunchKernelGGL(ln_fwd_reg_kernel<4>, g, b, 0, s, st, h, gamma, beta, z32, z16, mean, rstd); return;
    case 8: hipLaunchKernelGGL(ln_fwd_reg_kernel<8>, g, b, 0, s, st, h, gamma, beta, z32, z16, mean, rstd); return;
    default:
      hipLaunchKernelGGL(ln_fwd_kernel, g, b, 0, s, st, h, gamma, beta, F, z32, z16, mean, rstd);
  }
}

// dh = dh_next + rstd * (dxhat - mean(dxhat) - xhat * mean(dxhat * xhat)),
// dxhat = dz * gamma, xhat = (h - mean) * rstd.
__global__ void __launch_bounds__(256) ln_bwd_kernel(
    const StepState* __restrict__ st, const float* __restrict__ h, const float* __restrict__ mean,
    const float* __restrict__ rstd, const float* __restrict__ gamma, const float* __restrict__ dz,
    const float* __restrict__ dh_next, int F, float* __restrict__ dh32,
    bf16_t* __restrict__ dh16) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= st->rows) return;
  const float mu = mean[r], rs = rstd[r];
  const float* hr = h + (size_t)r * F;
  const float* dzr = dz + (size_t)r * F;
  float s1 = 0.f, s2 = 0.f;
  for (int f = 4 * lane; f < F; f += 256) {
    const float4 x = *(const float4*)(hr + f);
    const float4 d = *(const float4*)(dzr + f);
    const float4 gm = *(const float4*)(gamma + f);
    const float dx0 = d.x * gm.x, dx1 = d.y * gm.y, dx2 = d.z * gm.z, dx3 = d.w * gm.w;
    s1 += (dx0 + dx1) + (dx2 + dx3);
    s2 += (dx0 * ((x.x - mu) * rs) + dx1 * ((x.y - mu) * rs)) +
          (dx2 * ((x.z - mu) * rs) + dx3 * ((x.w - mu) * rs));
  }
  const float m1 = wave_sum(s1) / (float)F;
  const float m2 = wave_sum(s2) / (float)F;
  for (int f = 4 * lane; f < F; f += 256) {
    const float4 x = *(const float4*)(hr + f);
    const float4 d = *(const float4*)(dzr + f);
    const float4 gm = *(const float4*)(gamma + f);
    const float4 dn = *(const float4*)(dh_next + (size_t)r * F + f);
    float4 o;
    o.x = dn.x + rs * (d.x * gm.x - m1 - ((x.x - mu) * rs) * m2);
    o.y = dn.y + rs * (d.y * gm.y - m1 - ((x.y - mu) * rs) * m2);
    o.z = dn.z + rs * (d.z * gm.z - m1 - ((x.z - mu) * rs) * m2);
    o.w = dn.w + rs * (d.w * gm.w - m1 - ((x.w - mu) * rs) * m2);
    *(float4*)(dh32 + (size_t)r * F + f) = o;
    if (dh16)
      *(ushort4*)(dh16 + (size_t)r * F + f) = make_ushort4(f2bf(o.x), f2bf(o.y), f2bf(o.z), f2bf(o.w));
  }
}

template <int NV>
__global__ void __launch_bounds__(256) ln_bwd_reg_kernel(
    const StepState* __restrict__ st, const float* __restrict__ h, const float* __restrict__ mean,
    const float* __restrict__ rstd, const float* __restrict__ gamma, const float* __restrict__ dz,
    const float* __restrict__ dh_next, float* __restrict__ dh32, bf16_t* __restrict__ dh16) {
  constexpr int F = 256 * NV;
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= st->rows) return;
  const float mu = mean[r], rs = rstd[r];
  float xh[NV][4], dx[NV][4];
  float s1 = 0.f, s2 = 0.f;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int f = 4 * (lane + 64 * v);
    const float4 x = *(const float4*)(h + (size_t)r * F + f);
    const float4 d = *(const float4*)(dz + (size_t)r * F + f);
    const float4 gm = *(const float4*)(gamma + f);
    xh[v][0] = (x.x - mu) * rs; xh[v][1] = (x.y - mu) * rs;
    xh[v][2] = (x.z - mu) * rs; xh[v][3] = (x.w - mu) * rs;
    dx[v][0] = d.x * gm.x; dx[v][1] = d.y * gm.y; dx[v][2] = d.z * gm.z; dx[v][3] = d.w * gm.w;
    s1 += (dx[v][0] + dx[v][1]) + (dx[v][2] + dx[v][3]);
    s2 += (dx[v][0] * xh[v][0] + dx[v][1] * xh[v][1]) + (dx[v][2] * xh[v][2] + dx[v][3] * xh[v][3]);
  }
  const float m1 = wave_sum(s1) / (float)F;
  const float m2 = wave_sum(s2) / (float)F;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int f = 4 * (lane + 64 * v);
    const float4 dn = *(const float4*)(dh_next + (size_t)r * F + f);
    float4 o;
    o.x = dn.x + rs * (dx[v][0] - m1 - xh[v][0] * m2);
    o.y = dn.y + rs * (dx[v][1] - m1 - xh[v][1] * m2);
    o.z = dn.z + rs * (dx[v][2] - m1 - xh[v][2] * m2);
    o.w = dn.w + rs * (dx[v][3] - m1 - xh[v][3] * m2);
    *(float4*)(dh32 + (size_t)r * F + f) = o;
    if (dh16)
      *(ushort4*)(dh16 + (size_t)r * F + f) = make_ushort4(f2bf(o.x), f2bf(o.y), f2bf(o.z), f2bf(o.w));
  }
}

// The LayerNorm adjoint with the column sums folded in.  The 4 waves of a
// workgroup share each row (thread t takes columns t, t + 256, ...), so a
// thread's share of the column sums over the group's rows stays in CPT x 3
// registers; the row statistics of the adjoint are summed over the 4 waves
// through LDS, in wave order.  Rows r0 .. r0 + kLnFoldRows - 1 in order.
template <int CPT>
__global__ void __launch_bounds__(256) ln_bwd_fold_kernel(
    const StepState* __restrict__ st, const float* __restrict__ h, const float* __restrict__ mean,
    const float* __restrict__ rstd, const float* __restrict__ gamma, const float* __restrict__ dz,
    const float* __restrict__ dh_next, float* __restrict__ dh32, bf16_t* __restrict__ dh16,
    float* __restrict__ part) {
  constexpr int F = 256 * CPT;
  __shared__ float red[2][4][2];  // per-row wave partials, alternating by row
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rows = st->rows;
  const int r0 = blockIdx.x * kLnFoldRows;
  if (r0 >= rows) return;
  const int r1 = min(rows, r0 + kLnFoldRows);
  float gm[CPT], sb[CPT], sg[CPT], so[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    gm[u] = gamma[t + 256 * u];
    sb[u] = sg[u] = so[u] = 0.f;
  }
  for (int r = r0; r < r1; ++r) {
    const int buf = (r - r0) & 1;
    const float mu = mean[r], rs = rstd[r];
    float xh[CPT], d[CPT], dn[CPT];
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const size_t o = (size_t)r * F + t + 256 * u;
      xh[u] = (h[o] - mu) * rs;
      d[u] = dz[o];
      dn[u] = dh_next[o];
      const float dx = d[u] * gm[u];
      s1 += dx;
      s2 += dx * xh[u];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      red[buf][w][0] = s1;
      red[buf][w][1] = s2;
    }
    // (the next row's barrier keeps the row after next from rewriting
    // red[buf] before every thread has read it)
    __syncthreads();
    const float m1 = ((red[buf][0][0] + red[buf][1][0]) + (red[buf][2][0] + red[buf][3][0])) / (float)F;
    const float m2 = ((red[buf][0][1] + red[buf][1][1]) + (red[buf][2][1] + red[buf][3][1])) / (float)F;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const size_t o = (size_t)r * F + t + 256 * u;
      const float dx = d[u] * gm[u];
      const float v = dn[u] + rs * (dx - m1 - xh[u] * m2);
      dh32[o] = v;
      if (dh16) dh16[o] = f2bf(v);
      sb[u] += d[u];
      sg[u] += d[u] * xh[u];
      so[u] += dn[u];
    }
  }
  float* pg = part + (size_t)blockIdx.x * 3 * F;
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    pg[t + 256 * u] = sb[u];
    pg[F + t + 256 * u] = sg[u];
    pg[2 * F + t + 256 * u] = so[u];
  }
}

bool ln_bwd_folds(int F) { return F == 256 || F == 512 || F == 1024 || F == 2048; }

size_t ln_fold_part_elems(int max_rows, int F) {
  return (size_t)((max_rows + kLnFoldRows - 1) / kLnFoldRows) * 3 * (size_t)F;
}

void k_ln_bwd(const StepState* st, const float* h, const float* mean, const float* rstd,
              const float* gamma, const float* dz, const float* dh_next, int F, float* dh32,
              bf16_t* dh16, float* part, int max_rows, hipStream_t s) {
  if (part && ln_bwd_folds(F)) {
    const dim3 g(blocks_for(max_rows, kLnFoldRows)), b(256);
    switch (F / 256) {
      case 1: hipLaunchKernelGGL(ln_bwd_fold_kernel<1>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16, part); return;
      case 2: hipLaunchKernelGGL(ln_bwd_fold_kernel<2>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16, part); return;
      case 4: hipLaunchKernelGGL(ln_bwd_fold_kernel<4>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16, part); return;
      case 8: hipLaunchKernelGGL(ln_bwd_fold_kernel<8>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16, part); return;
    }
  }
  const dim3 g(blocks_for(max_rows, 4)), b(256);
  switch (F % 256 == 0 ? F / 256 : 0) {
    case 1: hipLaunchKernelGGL(ln_bwd_reg_kernel<1>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16); return;
    case 2: hipLaunchKernelGGL(ln_bwd_reg_kernel<2>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16); return;
    case 4: hipLaunchKernelGGL(ln_bwd_reg_kernel<4>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16); return;
    case 8: hipLaunchKernelGGL(ln_bwd_reg_kernel<8>, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, dh32, dh16); return;
    default:
      hipLaunchKernelGGL(ln_bwd_kernel, g, b, 0, s, st, h, mean, rstd, gamma, dz, dh_next, F, dh32, dh16);
  }
}

// ---------------------------------------------------------------------------
// Head: softmax (Eq. 1) -> 16-bit integer CDF -> range-coder lane ->
// cross-entropy adjoint (Eq. 2).  One wave per row; lane l holds symbols
// 4l .. 4l+3.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) head_kernel(const StepState* __restrict__ st, HeadArgs a,
                                                   StreamIO io) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= st->rows) return;
  const float4 z4 = *(const float4*)(a.logits + (size_t)r * 256 + 4 * lane);
  const float z[4] = {z4.x, z4.y, z4.z, z4.w};
  float p[4];
  int x = 0;
  const bool have_target = head_row(st, a, io, r, lane, z, p, &x);
  if (have_target && a.want_grad) {
    const float ir = st->inv_rows;
    float4 d4;
    d4.x = (p[0] - (4 * lane + 0 == x ? 1.0f : 0.0f)) * ir;
    d4.y = (p[1] - (4 * lane + 1 == x ? 1.0f : 0.0f)) * ir;
    d4.z = (p[2] - (4 * lane + 2 == x ? 1.0f : 0.0f)) * ir;
    d4.w = (p[3] - (4 * lane + 3 == x ? 1.0f : 0.0f)) * ir;
    if (a.dz32) *(float4*)(a.dz32 + (size_t)r * 256 + 4 * lane) = d4;
    if (a.dz16)
      *(ushort4*)(a.dz16 + (size_t)r * 256 + 4 * lane) =
          make_ushort4(f2bf(d4.x), f2bf(d4.y), f2bf(d4.z), f2bf(d4.w));
  }
}

void k_head(const StepState* st, HeadArgs a, StreamIO io, int max_rows, hipStream_t s) {
  hipLaunchKernelGGL(head_kernel, dim3(blocks_for(max_rows, 4)), dim3(256), 0, s, st, a, io);
}

// ---------------------------------------------------------------------------
// Column sums over the active rows (bias and LayerNorm affine gradients).
// Two passes with a fixed order: rows are cut into chunks of kColChunk; a
// block sums 64 columns of one chunk (4 interleaved row slices added in slice
// order) into partial[chunk][col]; the second pass adds the chunks in order.
// ---------------------------------------------------------------------------
constexpr int kColChunk = 64;

__global__ void __launch_bounds__(256) colsum_partial_kernel(const StepState* __restrict__ st,
                                                             const ColsumJob* __restrict__ jobs,
                                                             int n_jobs, int total_cols,
                                                             float* __restrict__ partial) {
  const int rows = st->rows;
  const int r0 = blockIdx.y * kColChunk;
  if (r0 >= rows) return;
  int j = 0;
  while (j + 1 < n_jobs && (int)blockIdx.x >= jobs[j + 1].col_block_begin) ++j;
  const ColsumJob jb = jobs[j];
  const int lc = ((int)blockIdx.x - jb.col_block_begin) * 64 + (threadIdx.x & 63);
  const int slice = threadIdx.x >> 6;
  const int r1 = min(rows, r0 + kColChunk);
  float acc = 0.f;
  const auto src = gl(jb.src);
  if (lc < jb.cols) {
    if (jb.h) {
      const auto h = gl(jb.h), mean = gl(jb.mean), rstd = gl(jb.rstd);
#pragma unroll 4
      for (int r = r0 + slice; r < r1; r += 4) {
        const float xh = (h[(size_t)r * jb.ld + lc] - mean[r]) * rstd[r];
        acc += src[(size_t)r * jb.ld + lc] * xh;
      }
    } else {
#pragma unroll 4
      for (int r = r0 + slice; r < r1; r += 4) acc += src[(size_t)r * jb.ld + lc];
    }
  }
  __shared__ float part[4][64];
  part[slice][threadIdx.x & 63] = acc;
  __syncthreads();
  if (slice == 0 && lc < jb.cols) {
    const int t = threadIdx.x;
    partial[(size_t)blockIdx.y * total_cols + jb.col_offset + lc] =
        (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
  }
}

__global__ void colsum_reduce_kernel(const StepState* __restrict__ st,
                                     const ColsumJob* __restrict__ jobs, int n_jobs,
                                     int total_cols, const float* __restrict__ partial,
                                     int chunk) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total_cols) return;
  int j = 0;
  while (j + 1 < n_jobs && c >= jobs[j + 1].col_offset) ++j;
  const ColsumJob& jb = jobs[j];
  float s;
  if (jb.part) {
    const int ng = (st->rows + jb.part_rows - 1) / jb.part_rows;
    s = ordered_sum(jb.part + (c - jb.col_offset), (size_t)jb.part_ld, ng);
  } else {
    const int nch = (st->rows + chunk - 1) / chunk;
    s = ordered_sum(partial + c, (size_t)total_cols, nch);
  }
  gl(jb.dst)[c - jb.col_offset] = s * (jb.scale == 0.0f ? st->inv_rows : jb.scale);
}

size_t colsum_partial_elems(int max_rows, int total_cols) {
  return (size_t)((max_rows + kColChunk - 1) / kColChunk) * total_cols;
}

void k_colsum(const StepState* st, const ColsumJob* jobs, int n_jobs, int total_blocks,
              int total_cols, float* partial, int max_rows, hipStream_t s) {
  if (total_blocks == 0) return;
  dim3 grid(total_blocks, (max_rows + kColChunk - 1) / kColChunk);
  hipLaunchKernelGGL(colsum_partial_kernel, grid, dim3(256), 0, s, st, jobs, n_jobs, total_cols,
                     partial);
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3(blocks_for(total_cols, 256)), dim3(256), 0, s, st,
                     jobs, n_jobs, total_cols, (const float*)partial, kColChunk);
}

void k_colsum_reduce(const StepState* st, const ColsumJob* jobs, int n_jobs, int total_cols,
                     const float* partial, int chunk_rows, hipStream_t s) {
  if (total_cols == 0) return;
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3(blocks_for(total_cols, 256)), dim3(256), 0, s, st,
                     jobs, n_jobs, total_cols, partial, chunk_rows);
}

// ---------------------------------------------------------------------------
// Embedding gradient: dEmb[v] = sum over (row, position) with ctx = v of the
// matching E-slice of dX.  A block takes a chunk of rows, staged through LDS
// a few rows at a time; thread v keeps the E sums of byte value v in
// registers and adds the matching pairs in row-major pair order.  The chunk
// partials are then added in chunk order.
// ---------------------------------------------------------------------------
template <int E>
__global__ void __launch_bounds__(256) emb_grad_partial_kernel(
    const StepState* __restrict__ st, const uint8_t* __restrict__ ctx, const float* __restrict__ dx,
    int C, int chunk_rows, int sub_rows, float* __restrict__ partial) {
  // dEmb_chunk[v][e] = sum over the chunk's (row, position) pairs of
  // [ctx = v] * dX[row][position*E + e]: a matrix product on the BF16 MFMA
  // whose A operand, the one-hot of the context bytes, is formed in registers
  // (exact in BF16).  An FP32 value x is the exact sum of three BF16 values
  // (x rounded to 8 significant bits, then the rounding errors of what is
  // left), so dX enters as three BF16 operands accumulated in FP32: an FP32
  // sum of the same terms, 3 MFMA instructions per 32 pairs where the FP32
  // MFMA (K = 4) takes 8.
  // Wave w owns byte values 64w .. 64w+63; pairs are visited in row-major
  // order, 32 per step.
  extern __shared__ float smem_f[];
  float* lds_dx = smem_f;                                            // [sub_rows][F]
  uint8_t* lds_ctx = (uint8_t*)(smem_f + (size_t)sub_rows * C * E);  // [sub_rows][C]
  constexpr int NE = E / 16;
  const int rows = st->rows;
  const int F = C * E;
  const int r0 = blockIdx.x * chunk_rows;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  f32x4 acc[4][NE];
#pragma unroll
  for (int vb = 0; vb < 4; ++vb)
#pragma unroll
    for (int nb = 0; nb < NE; ++nb) acc[vb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int r_end = min(rows, r0 + chunk_rows);
  // The next sub-batch of rows is loaded into registers while the current
  // one feeds the MFMAs from LDS: up to 8192 floats of dX (8 float4 a
  // thread) and 512 context bytes (sub_rows * C <= 8192 / E).  Wider rows
  // (F > 8192, one row a sub-batch) are copied straight to LDS instead.
  constexpr int kStage = 8;
  const bool staged = sub_rows * F <= 4 * kStage * 256;
  float4 nx[kStage];
  uint32_t nc[2] = {0u, 0u};
  auto fetch = [&](int rs) {
    const int nr = min(sub_rows, r_end - rs);
    const float4* src = (const float4*)(dx + (size_t)rs * F);
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int k = (int)threadIdx.x + 256 * q;
      nx[q] = k < nr * F / 4 ? src[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = (int)threadIdx.x + 256 * q;
      nc[q] = k < nr * C ? (uint32_t)ctx[(size_t)rs * C + k] : 0u;
    }
  };
  if (staged && r0 < r_end) fetch(r0);
  for (int rs = r0; rs < r_end; rs += sub_rows) {
    const int nr = min(sub_rows, r_end - rs);
    __syncthreads();  // the previous sub-batch's LDS reads are done
    if (staged) {
#pragma unroll
      for (int q = 0; q < kStage; ++q) {
        const int k = (int)threadIdx.x + 256 * q;
        if (k < nr * F / 4) ((float4*)lds_dx)[k] = nx[q];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = (int)threadIdx.x + 256 * q;
        if (k < nr * C) lds_ctx[k] = (uint8_t)nc[q];
      }
    } else {
      const float4* src = (const float4*)(dx + (size_t)rs * F);
      for (int k = threadIdx.x; k < nr * F / 4; k += 256) ((float4*)lds_dx)[k] = src[k];
      for (int k = threadIdx.x; k < nr * C; k += 256) lds_ctx[k] = ctx[(size_t)rs * C + k];
    }
    __syncthreads();
    if (staged && rs + sub_rows < r_end) fetch(rs + sub_rows);
    // lane group g = lane / 16 takes pairs p0 .. p0 + 7 of each 32-pair step;
    // pairs past the chunk's end take no byte value and a zero dX
    const int np = nr * C;
    for (int k0 = 0; k0 < np; k0 += 32) {
      const int p0 = k0 + 8 * (lane >> 4);
      int off[8];  // LDS offset of each pair's dX, or -1
      uint32_t bytes[8];
      if (C % 8 == 0) {  // the 8 pairs lie in one row: all valid or none
        const bool live = p0 < np;
        const int pr = live ? p0 / C : 0, pc = live ? p0 - pr * C : 0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          off[v] = live ? pr * F + (pc + v) * E : -1;
          bytes[v] = live ? (uint32_t)lds_ctx[p0 + v] : 0xFFFFu;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int p = p0 + v;
          const int pr = p / C;
          off[v] = p < np ? pr * F + (p - pr * C) * E : -1;
          bytes[v] = p < np ? (uint32_t)lds_ctx[p] : 0xFFFFu;
        }
      }
#pragma unroll
      for (int nb = 0; nb < NE; ++nb) {
        const float* d = lds_dx + 16 * nb + (lane & 15);
        uint32_t hi[4], mid[4], lo[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          uint32_t ph = 0, pm = 0, pl = 0;
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int o = off[2 * h + u];
            const float x = o >= 0 ? d[o] : 0.0f;
            const bf16_t b0 = f2bf(x);
            const float r1 = x - bf2f(b0);
            const bf16_t b1 = f2bf(r1);
            const bf16_t b2 = f2bf(r1 - bf2f(b1));
            ph |= (uint32_t)b0 << (16 * u);
            pm |= (uint32_t)b1 << (16 * u);
            pl |= (uint32_t)b2 << (16 * u);
          }
          hi[h] = ph;
          mid[h] = pm;
          lo[h] = pl;
        }
        const bf16x8 bh = __builtin_bit_cast(bf16x8, make_uint4(hi[0], hi[1], hi[2], hi[3]));
        const bf16x8 bm = __builtin_bit_cast(bf16x8, make_uint4(mid[0], mid[1], mid[2], mid[3]));
        const bf16x8 bl = __builtin_bit_cast(bf16x8, make_uint4(lo[0], lo[1], lo[2], lo[3]));
#pragma unroll
        for (int vb = 0; vb < 4; ++vb) {
          const uint32_t me = (uint32_t)(64 * w + 16 * vb + (lane & 15));
          uint32_t q[4];
#pragma unroll
          for (int h = 0; h < 4; ++h)
            q[h] = (bytes[2 * h] == me ? 0x3F80u : 0u) |
                   ((bytes[2 * h + 1] == me ? 0x3F80u : 0u) << 16);
          const bf16x8 a = __builtin_bit_cast(bf16x8, make_uint4(q[0], q[1], q[2], q[3]));
          acc[vb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc[vb][nb], 0, 0, 0);
          acc[vb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bm, acc[vb][nb], 0, 0, 0);
          acc[vb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[vb][nb], 0, 0, 0);
        }
      }
    }
  }
  float* out = partial + (size_t)blockIdx.x * 256 * E;
#pragma unroll
  for (int vb = 0; vb < 4; ++vb)
#pragma unroll
    for (int nb = 0; nb < NE; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = 64 * w + 16 * vb + 4 * (lane >> 4) + r;
        out[(size_t)v * E + 16 * nb + (lane & 15)] = acc[vb][nb][r];
      }
}

__global__ void emb_grad_reduce_kernel(const StepState* __restrict__ st,
                                       const float* __restrict__ partial, int chunk_rows, int n,
                                       float* __restrict__ demb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int nb = (st->rows + chunk_rows - 1) / chunk_rows;
  demb[k] = ordered_sum(partial + k, (size_t)n, nb);
}

void emb_grad_plan(int max_rows, int C, int E, int* chunk_rows, int* sub_rows) {
  const int F = C * E;
  int sub = 8192 / F;
  sub = sub < 1 ? 1 : (sub > 16 ? 16 : sub);
  int chunk = sub;
  while ((max_rows + chunk - 1) / chunk > 256) chunk += sub;
  *chunk_rows = chunk;
  *sub_rows = sub;
}

void k_emb_grad_reduce(const StepState* st, const float* partial, int chunk_rows, int E,
                       float* demb, hipStream_t s) {
  const int n = 256 * E;
  hipLaunchKernelGGL(emb_grad_reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, st, partial,
                     chunk_rows, n, demb);
}

void k_emb_grad(const StepState* st, const uint8_t* ctx, const float* dx, int C, int E,
                float* partial, int chunk_rows, int sub_rows, int max_rows, float* demb,
                hipStream_t s) {
  const int nb = (max_rows + chunk_rows - 1) / chunk_rows;
  const size_t smem = (size_t)sub_rows * C * E * sizeof(float) + (size_t)sub_rows * C + 32;
#define EMB_CASE(EE)                                                                            \
  case EE:                                                                                      \
    if (smem > 65536)  /* the widest feature vectors need more than the default LDS */          \
      (void)hipFuncSetAttribute((const void*)emb_grad_partial_kernel<EE>,                       \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);         \
    hipLaunchKernelGGL(emb_grad_partial_kernel<EE>, dim3(nb), dim3(256), smem, s, st, ctx, dx, C, \
                       chunk_rows, sub_rows, partial);                                          \
    break;
  switch (E) {
    EMB_CASE(16)
    EMB_CASE(32)
    EMB_CASE(64)
  }
#undef EMB_CASE
  const int n = 256 * E;
  hipLaunchKernelGGL(emb_grad_reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, st, partial,
                     chunk_rows, n, demb);
}

// ---------------------------------------------------------------------------
// Adam on the shared parameters (FP32 master, optional BF16 shadow).
// ---------------------------------------------------------------------------
__global__ void adam_kernel(const StepState* __restrict__ st, float* __restrict__ p,
                            const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, bf16_t* __restrict__ p16, size_t n,
                            AdamCfg ac) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float lr_bc = ac.lr / st->bc1;
  const float inv_bc2 = 1.0f / st->bc2;
  const float gr = g[i];
  const float mm = ac.beta1 * m[i] + (1.0f - ac.beta1) * gr;
  const float vv = ac.beta2 * v[i] + (1.0f - ac.beta2) * gr * gr;
  const float pp = p[i] - lr_bc * mm / (sqrtf(vv * inv_bc2) + ac.eps);
  m[i] = mm;
  v[i] = vv;
  p[i] = pp;
  if (p16) p16[i] = f2bf(pp);
}

void k_adam(const StepState* st, float* p, const float* g, float* m, float* v, bf16_t* p16,
            size_t n, AdamCfg ac, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, st, p, g, m, v, p16, n,
                     ac);
}

// ---------------------------------------------------------------------------
// Initialisation (SplitMix64, Steele, Lea & Flood 2014)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void init_uniform_kernel(float* __restrict__ dst, size_t n, uint64_t seed, uint32_t tid,
                                    uint64_t start, float bound) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint64_t r = splitmix64(seed + ((uint64_t)tid << 40) + start + j);
  const int k = (int)(r >> 40) - (1 << 23);
  const float a = (float)k * (1.0f / 8388608.0f);
  dst[j] = a * bound;
}

void k_init_uniform(float* dst, size_t n, uint64_t seed, uint32_t tid, uint64_t start, float bound,
                    hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(init_uniform_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst, n, seed,
                     tid, start, bound);
}

__global__ void fill_kernel(float* dst, size_t n, float v) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) dst[j] = v;
}
void k_fill(float* dst, size_t n, float v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst, n, v);
}

__global__ void to_bf16_kernel(const float* src, bf16_t* dst, size_t n) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) dst[j] = f2bf(src[j]);
}
void k_to_bf16(const float* src, bf16_t* dst, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
}

// ---------------------------------------------------------------------------
// Coder lanes (one thread per stream)
// ---------------------------------------------------------------------------
// The first t bytes of each stream: frequency 256 each (Algorithm 1, "with
// equal probability"); also initialises the coder state.
__global__ void uniform_prefix_kernel(StreamIO io, int n_streams, int C, bool decoding) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_streams) return;
  const uint64_t len = io.lens[s];
  const uint64_t n = len < (uint64_t)C ? len : (uint64_t)C;
  if (!decoding) {
    RcEnc e;
    rc_enc_init(e);
    uint8_t* out = io.pay + io.pay_off[s];
    const uint64_t cap = io.pay_cap[s];
    for (uint64_t i = 0; i < n; ++i) rc_encode(e, out, cap, 256u * io.src[io_at(io, io.off[s], i)], 256u);
    io.enc[s] = e;
  } else {
    RcDec d;
    const uint8_t* in = io.pay_in + io.pay_off[s];
    const uint64_t plen = io.pay_cap[s];
    rc_dec_init(d, in, plen);
    for (uint64_t i = 0; i < n; ++i) {
      // largest x with (range * 256x) >> 16 <= d
      uint32_t lo = 0, hi = 256;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (((d.range * (uint64_t)(256u * mid)) >> 16) <= d.d) lo = mid; else hi = mid;
      }
      io.dst[io_at(io, io.off[s], i)] = (uint8_t)lo;
      rc_consume(d, in, plen, 256u * lo, 256u * lo + 256u);
    }
    io.dec[s] = d;
  }
}

void k_uniform_prefix(StreamIO io, int n_streams, int C, bool decoding, hipStream_t s) {
  hipLaunchKernelGGL(uniform_prefix_kernel, dim3(blocks_for(n_streams, 64)), dim3(64), 0, s, io,
                     n_streams, C, decoding);
}

__global__ void rc_finish_kernel(StreamIO io, int n_streams) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_streams) return;
  RcEnc e = io.enc[s];
  rc_finish(e, io.pay + io.pay_off[s], io.pay_cap[s]);
  io.enc[s] = e;
}

void k_rc_finish(StreamIO io, int n_streams, hipStream_t s) {
  hipLaunchKernelGGL(rc_finish_kernel, dim3(blocks_for(n_streams, 64)), dim3(64), 0, s, io,
                     n_streams);
}

__global__ void rc_table_encode_kernel(const uint32_t* __restrict__ cum,
                                       const uint8_t* __restrict__ sym, size_t n_steps,
                                       size_t n_streams, uint8_t* __restrict__ out, size_t cap,
                                       uint64_t* __restrict__ out_lens) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_streams) return;
  RcEnc e;
  rc_enc_init(e);
  uint8_t* o = out + s * cap;
  for (size_t t = 0; t < n_steps; ++t) {
    const uint32_t* c = cum + (t * n_streams + s) * 257;
    const uint32_t x = sym[t * n_streams + s];
    rc_encode(e, o, cap, c[x], c[x + 1] - c[x]);
  }
  rc_finish(e, o, cap);
  out_lens[s] = e.pos;
}

void k_rc_table_encode(const uint32_t* cum, const uint8_t* sym, size_t n_steps, size_t n_streams,
                       uint8_t* out, size_t cap, uint64_t* out_lens, hipStream_t s) {
  hipLaunchKernelGGL(rc_table_encode_kernel, dim3(blocks_for(n_streams, 64)), dim3(64), 0, s, cum,
                     sym, n_steps, n_streams, out, cap, out_lens);
}

__global__ void rc_table_decode_kernel(const uint32_t* __restrict__ cum,
                                       const uint8_t* __restrict__ in,
                                       const uint64_t* __restrict__ in_lens, size_t cap,
                                       size_t n_steps, size_t n_streams, uint8_t* __restrict__ sym) {
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_streams) return;
  const uint8_t* p = in + s * cap;
  const uint64_t len = in_lens[s] < cap ? in_lens[s] : cap;
  RcDec d;
  rc_dec_init(d, p, len);
  for (size_t t = 0; t < n_steps; ++t) {
    const uint32_t* c = cum + (t * n_streams + s) * 257;
    const uint32_t x = rc_find(d, c);
    rc_consume(d, p, len, c[x], c[x + 1]);
    sym[t * n_streams + s] = (uint8_t)x;
  }
}

void k_rc_table_decode(const uint32_t* cum, const uint8_t* in, const uint64_t* in_lens, size_t cap,
                       size_t n_steps, size_t n_streams, uint8_t* sym, hipStream_t s) {
  hipLaunchKernelGGL(rc_table_decode_kernel, dim3(blocks_for(n_streams, 64)), dim3(64), 0, s, cum,
                     in, in_lens, cap, n_steps, n_streams, sym);
}

// CRC-32 (IEEE 802.3, reflected polynomial 0xEDB88320), one thread per stream.
__global__ void crc32_kernel(const uint8_t* __restrict__ data, const uint64_t* __restrict__ off,
                             const uint64_t* __restrict__ lens, int n, uint32_t* __restrict__ crc) {
  __shared__ uint32_t table[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    uint32_t c = (uint32_t)i;
    for (int k = 0; k < 8; ++k) c = (c & 1u) ? (0xEDB88320u ^ (c >> 1)) : (c >> 1);
    table[i] = c;
  }
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint8_t* p = data + off[s];
  const uint64_t len = lens[s];
  uint32_t c = 0xFFFFFFFFu;
  for (uint64_t i = 0; i < len; ++i) c = table[(c ^ p[i]) & 0xFFu] ^ (c >> 8);
  crc[s] = c ^ 0xFFFFFFFFu;
}

void k_crc32(const uint8_t* data, const uint64_t* off, const uint64_t* lens, int n, uint32_t* crc,
             hipStream_t s) {
  hipLaunchKernelGGL(crc32_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, s, data, off, lens, n, crc);
}

__global__ void gather_payloads_kernel(const uint8_t* __restrict__ pay,
                                       const uint64_t* __restrict__ pay_off,
                                       const uint64_t* __restrict__ len,
                                       const uint64_t* __restrict__ dst_off,
                                       uint8_t* __restrict__ dst) {
  const int s = blockIdx.x;
  const uint8_t* src = pay + pay_off[s];
  uint8_t* d = dst + dst_off[s];
  const uint64_t n = len[s];
  for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = src[i];
}

void k_gather_payloads(const uint8_t* pay, const uint64_t* pay_off, const uint64_t* len,
                       const uint64_t* dst_off, uint8_t* dst, int n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(gather_payloads_kernel, dim3(n), dim3(256), 0, s, pay, pay_off, len, dst_off,
                     dst);
}

}  // namespace edpc

namespace edpc {

// One wave per stream.  A carry adds one to the last byte before the coder's
// write position that is not 0xFF and zeroes the 0xFF bytes after it, so the
// bytes before that byte are final.
__global__ void __launch_bounds__(64) pay_drain_kernel(const RcEnc* __restrict__ enc,
                                                       const uint8_t* __restrict__ pay,
                                                       const uint64_t* __restrict__ pay_off,
                                                       uint64_t* __restrict__ done, int n, int all,
                                                       uint8_t* __restrict__ out, uint32_t stride,
                                                       uint32_t* __restrict__ out_len) {
  const int s = blockIdx.x;
  if (s >= n) return;
  const uint8_t* p = pay + pay_off[s];
  const uint64_t pos = enc[s].pos, d0 = done[s];
  uint64_t fin = pos;
  if (!all) {
    fin = d0;
    for (uint64_t i = pos; i > d0; --i)  // wave-uniform scan, usually one step
      if (p[i - 1] != 0xFF) { fin = i - 1; break; }
  }
  if (fin > d0 + stride) fin = d0 + stride;
  const uint32_t cnt = (uint32_t)(fin > d0 ? fin - d0 : 0);
  uint8_t* o = out + (size_t)s * stride;
  for (uint32_t i = threadIdx.x; i < cnt; i += 64) o[i] = p[d0 + i];
  __syncthreads();
  if (threadIdx.x == 0) {
    out_len[s] = cnt;
    done[s] = d0 + cnt;
  }
}

void k_pay_drain(const RcEnc* enc, const uint8_t* pay, const uint64_t* pay_off, uint64_t* done,
                 int n, bool all, uint8_t* out, uint32_t stride, uint32_t* out_len, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(pay_drain_kernel, dim3(n), dim3(64), 0, s, enc, pay, pay_off, done, n,
                     all ? 1 : 0, out, stride, out_len);
}

}  // namespace edpc
