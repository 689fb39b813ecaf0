// Multiply-first 32-bit range coder (G. N. N. Martin, 1979), compiled for
// both the GPU lanes and the host.  One coder per stream; the model supplies
// a 16-bit integer CDF per symbol (the "Arithmetic Coding" step of Sec. 2.1).
//
//   state: low < 2^32 (+carry), range in [2^24, 2^32]; start low=0,
//          range=2^32, nothing written.
//   encode(c, q): lo = (range*c) >> 16, hi = (range*(c+q)) >> 16;
//          low += lo; range = hi - lo; a carry past 2^32 adds one to the
//          bytes already written (trailing 0xFF become 0x00); then while
//          range < 2^24 write low>>24, low = (low<<8) mod 2^32, range <<= 8.
//   finish: v = (low + 0xFFFF) & ~0xFFFF (with carry); write v's top two
//          bytes.  An empty stream writes nothing.
//   decode keeps d = code - low in [0, range), picks the symbol x with
//          lo(x) <= d < lo(x+1), and shifts in zero bytes past the end.
// With 16-bit frequencies >= 1 a symbol writes at most two bytes, so a
// payload never exceeds 2 * n_symbols + 2 bytes.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define EDPC_HD __host__ __device__ __forceinline__
#else
#define EDPC_HD inline
#endif

namespace edpc {

constexpr uint64_t kRcTop = 1ull << 32;
constexpr uint64_t kRcBot = 1ull << 24;

struct RcEnc {
  uint64_t low;
  uint64_t range;
  uint64_t pos;  // bytes written so far
  uint64_t n;    // symbols coded
};

struct RcDec {
  uint64_t d;
  uint64_t range;
  uint64_t pos;  // next byte to read
  uint64_t pad;
};

EDPC_HD void rc_enc_init(RcEnc& e) { e.low = 0; e.range = kRcTop; e.pos = 0; e.n = 0; }

EDPC_HD void rc_carry(uint8_t* out, uint64_t pos) {
  // The coded value never reaches 1.0, so a zero-free byte exists before
  // the start; the bound keeps a corrupted state from walking off the buffer.
  uint64_t i = pos;
  while (i > 0) {
    --i;
    if (out[i] != 0xFF) { out[i] = (uint8_t)(out[i] + 1); return; }
    out[i] = 0;
  }
}

// Encode one symbol of cumulative count c and frequency q (out of 2^16).
// `cap` bounds the writes; the payload bound makes overflow impossible when
// cap >= 2 * n + 2, but a wrong caller cannot write past the buffer.
EDPC_HD void rc_encode(RcEnc& e, uint8_t* out, uint64_t cap, uint32_t c, uint32_t q) {
  const uint64_t lo = (e.range * (uint64_t)c) >> 16;
  const uint64_t hi = (e.range * (uint64_t)(c + q)) >> 16;
  e.low += lo;
  e.range = hi - lo;
  if (e.low >= kRcTop) {
    rc_carry(out, e.pos < cap ? e.pos : cap);
    e.low -= kRcTop;
  }
  // At most two shifts for valid tables (q >= 1); the bound also ends the
  // loop for an invalid table (q = 0 would leave range = 0).
  for (int k = 0; k < 4 && e.range < kRcBot; ++k) {
    if (e.pos < cap) out[e.pos] = (uint8_t)(e.low >> 24);
    e.pos++;
    e.low = (e.low << 8) & 0xFFFFFFFFull;
    e.range <<= 8;
  }
  e.n++;
}

EDPC_HD void rc_finish(RcEnc& e, uint8_t* out, uint64_t cap) {
  if (e.n == 0) return;
  uint64_t v = (e.low + 0xFFFFull) & ~0xFFFFull;
  if (v >= kRcTop) {
    rc_carry(out, e.pos < cap ? e.pos : cap);
    v -= kRcTop;
  }
  if (e.pos < cap) out[e.pos] = (uint8_t)(v >> 24);
  e.pos++;
  if (e.pos < cap) out[e.pos] = (uint8_t)(v >> 16);
  e.pos++;
}

EDPC_HD uint32_t rc_byte(const uint8_t* in, uint64_t len, uint64_t pos) {
  return pos < len ? (uint32_t)in[pos] : 0u;
}

EDPC_HD void rc_dec_init(RcDec& dd, const uint8_t* in, uint64_t len) {
  dd.range = kRcTop;
  dd.d = 0;
  dd.pos = 0;
  dd.pad = 0;
  for (int k = 0; k < 4; ++k) { dd.d = (dd.d << 8) | rc_byte(in, len, dd.pos); dd.pos++; }
}

// Symbol whose interval holds d: the largest x with (range*cum[x])>>16 <= d.
EDPC_HD uint32_t rc_find(const RcDec& dd, const uint32_t* cum) {
  uint32_t lo_x = 0, hi_x = 256;
  while (hi_x - lo_x > 1) {
    const uint32_t mid = (lo_x + hi_x) >> 1;
    if (((dd.range * (uint64_t)cum[mid]) >> 16) <= dd.d) lo_x = mid; else hi_x = mid;
  }
  return lo_x;
}

// Consume symbol with cumulative bounds c0 = cum[x], c1 = cum[x+1].
EDPC_HD void rc_consume(RcDec& dd, const uint8_t* in, uint64_t len, uint32_t c0, uint32_t c1) {
  const uint64_t lo = (dd.range * (uint64_t)c0) >> 16;
  const uint64_t hi = (dd.range * (uint64_t)c1) >> 16;
  dd.d -= lo;
  dd.range = hi - lo;
  for (int k = 0; k < 4 && dd.range < kRcBot; ++k) {
    dd.d = (dd.d << 8) | rc_byte(in, len, dd.pos);
    dd.pos++;
    dd.range <<= 8;
  }
}

}  // namespace edpc
