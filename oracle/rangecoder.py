"""32-bit multiply-first range coder in exact integers (oracle side).

Test infrastructure only.  The paper codes each byte by arithmetic coding
with Pr(i) (Sec. 2.1, "Data Encoding"; Algorithm 1, encode and decode steps)
and gives no coder details.  This is range coding (G. N. N. Martin, 1979) with
the following reading:

* state: ``low`` (< 2**32, plus a carry), ``range`` in [2**24, 2**32];
  start ``low = 0``, ``range = 2**32``; no leading byte is emitted;
* encode symbol with cumulative count c and frequency q out of T = 2**bits:
  ``lo = (range*c) >> bits``, ``hi = (range*(c+q)) >> bits``,
  ``low += lo``, ``range = hi - lo`` (products are exact, < 2**48);
* a carry (low >= 2**32) adds one to the bytes already written, turning
  trailing 0xFF bytes into 0x00;
* renormalise while ``range < 2**24``: write ``low >> 24``,
  ``low = (low << 8) mod 2**32``, ``range <<= 8`` (at most two bytes per
  symbol for 16-bit frequencies);
* finish: ``v = (low + 0xFFFF) & ~0xFFFF`` (with carry), write its top two
  bytes.  An empty stream writes nothing;
* decode keeps ``d = code - low`` in [0, range), finds the symbol x with
  lo(x) <= d < lo(x+1), subtracts lo(x), sets range = lo(x+1) - lo(x) and
  shifts in bytes past the end as zeros.

Pinned by: exhaustive decode(encode(x)) == x on tiny alphabets and lengths,
random round trips, the code-length bound (ideal + 2 bytes + truncation
slack), and the uniform case, where 16-bit frequencies of 256 shift the
stream's bytes through verbatim (tests/test_oracle_coder.py).
"""

from __future__ import annotations

TOP = 1 << 32
BOT = 1 << 24
MASK32 = TOP - 1


class RangeEncoder:
    def __init__(self, bits: int = 16):
        self.bits = bits
        self.low = 0
        self.range = TOP
        self.out = bytearray()
        self.n = 0

    def _carry(self):
        i = len(self.out) - 1
        while self.out[i] == 0xFF:
            self.out[i] = 0
            i -= 1
        self.out[i] += 1

    def encode(self, cum: int, freq: int):
        lo = (self.range * cum) >> self.bits
        hi = (self.range * (cum + freq)) >> self.bits
        self.low += lo
        self.range = hi - lo
        if self.low >= TOP:
            self._carry()
            self.low -= TOP
        while self.range < BOT:
            self.out.append(self.low >> 24)
            self.low = (self.low << 8) & MASK32
            self.range <<= 8
        self.n += 1

    def finish(self) -> bytes:
        if self.n == 0:
            return bytes(self.out)
        v = (self.low + 0xFFFF) & ~0xFFFF
        if v >= TOP:
            self._carry()
            v -= TOP
        self.out.append(v >> 24)
        self.out.append((v >> 16) & 0xFF)
        return bytes(self.out)


class RangeDecoder:
    def __init__(self, data: bytes, bits: int = 16):
        self.bits = bits
        self.data = data
        self.pos = 0
        self.range = TOP
        self.d = 0
        for _ in range(4):
            self.d = (self.d << 8) | self._next()

    def _next(self) -> int:
        b = self.data[self.pos] if self.pos < len(self.data) else 0
        self.pos += 1
        return b

    def decode(self, cum) -> int:
        """Decode one symbol given the cumulative table cum[0..n] (cum[n] = T)."""
        n = len(cum) - 1
        r = self.range
        lo_x, hi_x = 0, n  # invariant: lo(lo_x) <= d < lo(hi_x) with lo(n) = range
        while hi_x - lo_x > 1:
            mid = (lo_x + hi_x) // 2
            if ((r * cum[mid]) >> self.bits) <= self.d:
                lo_x = mid
            else:
                hi_x = mid
        x = lo_x
        lo = (r * cum[x]) >> self.bits
        hi = (r * cum[x + 1]) >> self.bits
        self.d -= lo
        self.range = hi - lo
        while self.range < BOT:
            self.d = (self.d << 8) | self._next()
            self.range <<= 8
        return x
