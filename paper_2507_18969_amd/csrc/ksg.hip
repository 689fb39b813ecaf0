// Kraskov's mutual-information estimator on the GPU (Sec. 3.1.1, Eq. 7):
// the analysis the paper uses to compare refinement blocks with one, two
// and three branches (the IFR metric, Eq. 8).
//
//   1. D_z[i][j] = max_c |z_ic - z_jc| and D_y likewise: tiled like a matrix
//      product, but with max(|a - b|) in place of the multiply-add, so it
//      runs on the vector ALUs (two instructions per pair and dimension).
//   2. per sample i, one workgroup: eps_i = the v-th smallest of
//      max(D_z[i][j], D_y[i][j]) over j != i (ties with multiplicity), then
//      c_z(i) = #{j != i: D_z[i][j] < eps_i}, c_y(i) likewise.
//   3. on the host: psi(v) + psi(c) - mean(psi(c_z + 1) + psi(c_y + 1)),
//      psi at integers from harmonic numbers.
// Distances are FP32 (correctly rounded differences, exact maxima), so the
// neighbour counts are those of any FP32 evaluation of the definition.
#include <cmath>
#include <vector>

#include "model.h"

namespace edpc {

constexpr int kKsgTile = 64;   // 64 x 64 sample pairs per workgroup
constexpr int kKsgDim = 32;    // dimensions per LDS stage
constexpr int kKsgMaxV = 16;   // largest neighbour order v

__global__ void __launch_bounds__(256) maxnorm_kernel(const float* __restrict__ x, int c, int d,
                                                      float* __restrict__ D) {
  __shared__ __align__(16) float si[kKsgDim][kKsgTile + 4];
  __shared__ __align__(16) float sj[kKsgDim][kKsgTile + 4];
  const int i0 = blockIdx.y * kKsgTile, j0 = blockIdx.x * kKsgTile;
  const int t = threadIdx.x;
  const int ti = t / 16, tj = t % 16;  // 4 x 4 pairs each
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
  for (int d0 = 0; d0 < d; d0 += kKsgDim) {
    // stage 64 samples x 32 dimensions of each side, transposed (zeros past
    // the ends add |0 - 0| = 0, which leaves a maximum of absolute values)
    for (int e = t; e < kKsgTile * kKsgDim; e += 256) {
      const int r = e / kKsgDim, q = e % kKsgDim;
      const int dd = d0 + q;
      si[q][r] = (i0 + r < c && dd < d) ? x[(size_t)(i0 + r) * d + dd] : 0.0f;
      sj[q][r] = (j0 + r < c && dd < d) ? x[(size_t)(j0 + r) * d + dd] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < kKsgDim; ++q) {
      const float4 a = *(const float4*)&si[q][4 * ti];
      const float4 b = *(const float4*)&sj[q][4 * tj];
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] = fmaxf(acc[u][w], fabsf(av[u] - bv[w]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + 4 * ti + u;
    if (i >= c) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int j = j0 + 4 * tj + w;
      if (j < c) D[(size_t)i * c + j] = acc[u][w];
    }
  }
}

// Lexicographic (value, thread) minimum over the workgroup: pops exactly one
// element per round even when several threads hold equal values.
__device__ __forceinline__ void block_argmin(float& v, int& who, float* sv, int* sw) {
  const int t = threadIdx.x;
  sv[t] = v;
  sw[t] = who;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) {
      const float a = sv[t], b = sv[t + o];
      const int wa = sw[t], wb = sw[t + o];
      if (b < a || (b == a && wb < wa)) {
        sv[t] = b;
        sw[t] = wb;
      }
    }
    __syncthreads();
  }
  v = sv[0];
  who = sw[0];
  __syncthreads();
}

__global__ void __launch_bounds__(256) ksg_select_kernel(const float* __restrict__ Dz,
                                                         const float* __restrict__ Dy, int c, int v,
                                                         float* __restrict__ eps_out,
                                                         int32_t* __restrict__ counts) {
  __shared__ float sv[256];
  __shared__ int sw[256];
  __shared__ int sc[2][256];
  const int i = blockIdx.x, t = threadIdx.x;
  const float* rz = Dz + (size_t)i * c;
  const float* ry = Dy + (size_t)i * c;
  // the v smallest joint distances this thread sees, ascending
  float best[kKsgMaxV];
#pragma unroll
  for (int q = 0; q < kKsgMaxV; ++q) best[q] = INFINITY;
  for (int j = t; j < c; j += 256) {
    if (j == i) continue;
    float x = fmaxf(rz[j], ry[j]);
#pragma unroll
    for (int q = 0; q < kKsgMaxV; ++q) {  // insertion keeps duplicates
      if (q < v && x < best[q]) {
        const float tmp = best[q];
        best[q] = x;
        x = tmp;
      }
    }
  }
  // v rounds: the smallest head over the workgroup leaves its list
  int head = 0;
  float eps = 0.0f;
  for (int r = 0; r < v; ++r) {
    float m = head < v ? best[0] : INFINITY;
    int who = t;
    block_argmin(m, who, sv, sw);
    eps = m;
    if (who == t) {  // pop this thread's head
#pragma unroll
      for (int q = 0; q + 1 < kKsgMaxV; ++q) best[q] = best[q + 1];
      best[kKsgMaxV - 1] = INFINITY;
      ++head;
    }
  }
  int nz = 0, ny = 0;
  for (int j = t; j < c; j += 256) {
    if (j == i) continue;
    nz += rz[j] < eps ? 1 : 0;
    ny += ry[j] < eps ? 1 : 0;
  }
  sc[0][t] = nz;
  sc[1][t] = ny;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) {
      sc[0][t] += sc[0][t + o];
      sc[1][t] += sc[1][t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (eps_out) eps_out[i] = eps;
    counts[2 * i] = sc[0][0];
    counts[2 * i + 1] = sc[1][0];
  }
}

double mutual_info(const float* d_z, size_t dz, const float* d_y, size_t dy, size_t c, uint32_t v,
                   int32_t* d_counts, float* d_eps, hipStream_t s) {
  if (c < 2 || c > 32768) fail(EDPC_E_INVALID_ARG, "number of samples must be in 2..32768");
  if (v < 1 || v >= c || v > (uint32_t)kKsgMaxV) fail(EDPC_E_INVALID_ARG, "v must be in 1..min(16, c - 1)");
  if (dz < 1 || dy < 1 || dz > (1u << 20) || dy > (1u << 20)) fail(EDPC_E_INVALID_ARG, "bad dimension");
  std::vector<void*> tmp;
  auto alloc = [&](size_t bytes) {
    void* p = nullptr;
    hip_check(hipMalloc(&p, bytes), "hipMalloc");
    tmp.push_back(p);
    return p;
  };
  double mi = 0.0;
  try {
    float* Dz = (float*)alloc(c * c * sizeof(float));
    float* Dy = (float*)alloc(c * c * sizeof(float));
    int32_t* cnt = d_counts ? d_counts : (int32_t*)alloc(2 * c * sizeof(int32_t));
    const unsigned tiles = (unsigned)((c + kKsgTile - 1) / kKsgTile);
    hipLaunchKernelGGL(maxnorm_kernel, dim3(tiles, tiles), dim3(256), 0, s, d_z, (int)c, (int)dz, Dz);
    hipLaunchKernelGGL(maxnorm_kernel, dim3(tiles, tiles), dim3(256), 0, s, d_y, (int)c, (int)dy, Dy);
    hipLaunchKernelGGL(ksg_select_kernel, dim3((unsigned)c), dim3(256), 0, s, Dz, Dy, (int)c, (int)v,
                       d_eps, cnt);
    hip_check(hipGetLastError(), "ksg launch");
    std::vector<int32_t> h(2 * c);
    hip_check(hipMemcpyAsync(h.data(), cnt, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s),
              "copy");
    hip_check(hipStreamSynchronize(s), "ksg");
    // psi(n) = -gamma + H(n - 1) at integers
    std::vector<double> H(c + 2, 0.0);
    for (size_t m = 1; m < H.size(); ++m) H[m] = H[m - 1] + 1.0 / (double)m;
    const double gamma = 0.57721566490153286061;
    auto psi = [&](size_t n) { return -gamma + H[n - 1]; };
    double sum = 0.0;
    for (size_t i = 0; i < c; ++i) sum += psi((size_t)h[2 * i] + 1) + psi((size_t)h[2 * i + 1] + 1);
    mi = psi(v) + psi(c) - sum / (double)c;
  } catch (...) {
    for (void* p : tmp) (void)hipFree(p);
    throw;
  }
  for (void* p : tmp) (void)hipFree(p);
  return mi;
}

}  // namespace edpc
