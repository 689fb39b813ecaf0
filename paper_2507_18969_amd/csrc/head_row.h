// Head of one row, run by one wave (lane l holds symbols 4l .. 4l+3):
// softmax (Eq. 1) -> 16-bit integer CDF -> range-coder lane (encode, or
// decode the symbol) -> per-row loss; optional probabilities / CDF outputs.
// Returns whether the row has a target (and so a loss and gradient); p and
// *x_out receive the probabilities and the coded symbol.
#pragma once
#include "kernels.h"

namespace edpc {

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Softmax (Eq. 1) and quantised 16-bit CDF of one row, one wave per row.
// The per-lane quadruples are vectors, so that row_cdf's runtime index
// (the remainder's bin) is a register insert; an array indexed at run time
// keeps the whole struct in scratch memory.
struct RowCdf {
  f32x4 p;      // probabilities of symbols 4l .. 4l+3
  i32x4 q;      // frequencies
  i32x4 cum;    // exclusive prefix sums of the frequencies
  float m, S;   // largest logit and the sum of exp(z - m)
};

__device__ __forceinline__ void row_cdf(int lane, const float z[4], RowCdf& c) {
  c.m = wave_max(fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3])));
  float e[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) e[j] = expf(z[j] - c.m);
  c.S = wave_sum((e[0] + e[1]) + (e[2] + e[3]));
#pragma unroll
  for (int j = 0; j < 4; ++j) c.p[j] = e[j] / c.S;

  // quantise: q = 1 + floor(p * (2^16 - 256)) in FP32; remainder to the
  // largest bin (lowest symbol on ties)
  uint32_t key = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    c.q[j] = 1 + (int)floorf(c.p[j] * 65280.0f);
    const uint32_t k = ((uint32_t)c.q[j] << 8) | (uint32_t)(255 - (4 * lane + j));
    key = k > key ? k : key;
  }
  key = wave_max_u(key);
  const int am = 255 - (int)(key & 255u);
  const int qsum = wave_sum_i((c.q[0] + c.q[1]) + (c.q[2] + c.q[3]));
  if ((am >> 2) == lane) c.q[am & 3] += 65536 - qsum;

  // exclusive prefix sums
  const int ls = (c.q[0] + c.q[1]) + (c.q[2] + c.q[3]);
  int incl = ls;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  c.cum[0] = incl - ls;
  c.cum[1] = c.cum[0] + c.q[0];
  c.cum[2] = c.cum[1] + c.q[1];
  c.cum[3] = c.cum[2] + c.q[2];
}

// Decoder symbol search: x = #{v : (range * cum[v]) >> 16 <= d} - 1.
__device__ __forceinline__ int row_decode_symbol(const RowCdf& c, uint64_t d, uint64_t rng) {
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) cnt += (((rng * (uint64_t)c.cum[j]) >> 16) <= d) ? 1 : 0;
  return wave_sum_i(cnt) - 1;
}

// Interval (cum, freq) and logit of symbol x, broadcast to the wave.
__device__ __forceinline__ void row_pick(const RowCdf& c, const float z[4], int x, int* cx, int* qx,
                                         float* zx) {
  const int jx = x & 3;
  // copied out first: a choice among loads of the struct is turned into one
  // load from a computed address, which would put the struct in scratch
  const int c0 = c.cum[0], c1 = c.cum[1], c2 = c.cum[2], c3 = c.cum[3];
  const int q0 = c.q[0], q1 = c.q[1], q2 = c.q[2], q3 = c.q[3];
  const float z0 = z[0], z1 = z[1], z2 = z[2], z3 = z[3];
  *cx = __shfl(jx == 0 ? c0 : jx == 1 ? c1 : jx == 2 ? c2 : c3, x >> 2, 64);
  *qx = __shfl(jx == 0 ? q0 : jx == 1 ? q1 : jx == 2 ? q2 : q3, x >> 2, 64);
  *zx = __shfl(jx == 0 ? z0 : jx == 1 ? z1 : jx == 2 ? z2 : z3, x >> 2, 64);
}

// Optional per-row outputs: probabilities and the CDF with its closing 2^16.
__device__ __forceinline__ void row_outputs(const HeadArgs& a, int r, int lane, const RowCdf& c) {
  if (a.probs)
    *(float4*)(a.probs + (size_t)r * 256 + 4 * lane) = make_float4(c.p[0], c.p[1], c.p[2], c.p[3]);
  if (a.cum_out) {
    uint32_t* co = a.cum_out + (size_t)r * 257;
#pragma unroll
    for (int j = 0; j < 4; ++j) co[4 * lane + j] = (uint32_t)c.cum[j];
    if (lane == 63) co[256] = 65536u;
  }
}

__device__ __forceinline__ bool head_row(const StepState* __restrict__ st, const HeadArgs& a,
                                         const StreamIO& io, int r, int lane, const float z[4],
                                         float p[4], int* x_out) {
  RowCdf c;
  row_cdf(lane, z, c);
#pragma unroll
  for (int j = 0; j < 4; ++j) p[j] = c.p[j];

  const uint32_t s = io.slot ? io.slot[r] : 0u;
  int x = 0;
  if (a.mode == 2) {
    uint64_t d = 0, rng = 0;
    if (lane == 0) {
      d = io.dec[s].d;
      rng = io.dec[s].range;
    }
    d = __shfl(d, 0, 64);
    rng = __shfl(rng, 0, 64);
    x = row_decode_symbol(c, d, rng);
  } else if (a.target) {
    x = a.target[r];
  }
  int cx, qx;
  float zx;
  row_pick(c, z, x, &cx, &qx, &zx);

  if (lane == 0) {
    if (a.mode == 1) {
      RcEnc en = io.enc[s];
      rc_encode(en, io.pay + io.pay_off[s], io.pay_cap[s], (uint32_t)cx, (uint32_t)qx);
      io.enc[s] = en;
    } else if (a.mode == 2) {
      RcDec de = io.dec[s];
      rc_consume(de, io.pay_in + io.pay_off[s], io.pay_cap[s], (uint32_t)cx, (uint32_t)(cx + qx));
      io.dec[s] = de;
      io.dst[io_at(io, io.off[s], (uint64_t)st->step)] = (uint8_t)x;
      if (a.target_out) a.target_out[r] = (uint8_t)x;
    }
  }
  const bool have_target = a.mode != 0 || a.target != nullptr;
  if (have_target && lane == 0 && a.loss_rows) a.loss_rows[r] = logf(c.S) - (zx - c.m);
  row_outputs(a, r, lane, c);
  *x_out = x;
  return have_target;
}

}  // namespace edpc
