// Head of one row, run by one wave (lane l holds symbols 4l .. 4l+3):
// softmax (Eq. 1) -> 16-bit integer CDF -> range-coder lane (encode, or
// decode the symbol) -> per-row loss; optional probabilities / CDF outputs.
// Returns whether the row has a target (and so a loss and gradient); p and
// *x_out receive the probabilities and the coded symbol.
#pragma once
#include "kernels.h"

namespace edpc {

__device__ __forceinline__ bool head_row(const StepState* __restrict__ st, const HeadArgs& a,
                                         const StreamIO& io, int r, int lane, const float z[4],
                                         float p[4], int* x_out) {
  const float m = wave_max(fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3])));
  float e[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) e[j] = expf(z[j] - m);
  const float S = wave_sum((e[0] + e[1]) + (e[2] + e[3]));
#pragma unroll
  for (int j = 0; j < 4; ++j) p[j] = e[j] / S;

  // quantise: q = 1 + floor(p * (2^16 - 256)) in FP32; remainder to the
  // largest bin (lowest symbol on ties)
  int q[4];
  uint32_t key = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    q[j] = 1 + (int)floorf(p[j] * 65280.0f);
    const uint32_t k = ((uint32_t)q[j] << 8) | (uint32_t)(255 - (4 * lane + j));
    key = k > key ? k : key;
  }
  key = wave_max_u(key);
  const int am = 255 - (int)(key & 255u);
  const int qsum = wave_sum_i((q[0] + q[1]) + (q[2] + q[3]));
  if ((am >> 2) == lane) q[am & 3] += 65536 - qsum;

  // exclusive prefix sums
  const int ls = (q[0] + q[1]) + (q[2] + q[3]);
  int incl = ls;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  int cum[4];
  cum[0] = incl - ls;
  cum[1] = cum[0] + q[0];
  cum[2] = cum[1] + q[1];
  cum[3] = cum[2] + q[2];

  const uint32_t s = io.slot ? io.slot[r] : 0u;
  int x = 0;
  if (a.mode == 2) {
    // decode: symbol x = #{v : (range * cum[v]) >> 16 <= d} - 1
    uint64_t d = 0, rng = 0;
    if (lane == 0) {
      d = io.dec[s].d;
      rng = io.dec[s].range;
    }
    d = __shfl(d, 0, 64);
    rng = __shfl(rng, 0, 64);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) cnt += (((rng * (uint64_t)cum[j]) >> 16) <= d) ? 1 : 0;
    x = wave_sum_i(cnt) - 1;
  } else if (a.target) {
    x = a.target[r];
  }
  const int jx = x & 3;
  const int cx = __shfl(jx == 0 ? cum[0] : jx == 1 ? cum[1] : jx == 2 ? cum[2] : cum[3], x >> 2, 64);
  const int qx = __shfl(jx == 0 ? q[0] : jx == 1 ? q[1] : jx == 2 ? q[2] : q[3], x >> 2, 64);
  const float zx = __shfl(jx == 0 ? z[0] : jx == 1 ? z[1] : jx == 2 ? z[2] : z[3], x >> 2, 64);

  if (lane == 0) {
    if (a.mode == 1) {
      RcEnc en = io.enc[s];
      rc_encode(en, io.pay + io.pay_off[s], io.pay_cap[s], (uint32_t)cx, (uint32_t)qx);
      io.enc[s] = en;
    } else if (a.mode == 2) {
      RcDec de = io.dec[s];
      rc_consume(de, io.pay_in + io.pay_off[s], io.pay_cap[s], (uint32_t)cx, (uint32_t)(cx + qx));
      io.dec[s] = de;
      io.dst[io.off[s] + (uint64_t)st->step] = (uint8_t)x;
      if (a.target_out) a.target_out[r] = (uint8_t)x;
    }
  }
  const bool have_target = a.mode != 0 || a.target != nullptr;
  if (have_target && lane == 0 && a.loss_rows) a.loss_rows[r] = logf(S) - (zx - m);
  if (a.probs) *(float4*)(a.probs + (size_t)r * 256 + 4 * lane) = make_float4(p[0], p[1], p[2], p[3]);
  if (a.cum_out) {
    uint32_t* co = a.cum_out + (size_t)r * 257;
#pragma unroll
    for (int j = 0; j < 4; ++j) co[4 * lane + j] = (uint32_t)cum[j];
    if (lane == 63) co[256] = 65536u;
  }
  *x_out = x;
  return have_target;
}

}  // namespace edpc
