"""Pins for the oracle's CDF quantiser and range coder."""

import itertools
import math
import os

import numpy as np
import pytest

from oracle.quantize import cumulative, quantize
from oracle.rangecoder import RangeDecoder, RangeEncoder

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, *v = line.split()
                out[k] = v
    return out


def _encode(cum, q, symbols, bits=16):
    e = RangeEncoder(bits)
    for x in symbols:
        e.encode(int(cum[x]), int(q[x]))
    return e.finish()


def _decode(payload, cum, n, bits=16):
    d = RangeDecoder(payload, bits)
    return [d.decode(list(cum)) for _ in range(n)]


# ---------------------------------------------------------------- quantiser

def test_quantize_invariants_random():
    r = np.random.default_rng(0)
    for scale in (0.1, 1.0, 5.0, 30.0):
        z = r.standard_normal((64, 256)) * scale
        p = np.exp(z - z.max(1, keepdims=True))
        p /= p.sum(1, keepdims=True)
        q = quantize(p)
        assert np.all(q.sum(1) == 65536)
        assert q.min() >= 1
        exact = p * 65280.0
        am = np.argmax(q, axis=1)
        mask = np.ones_like(q, dtype=bool)
        mask[np.arange(64), am] = False
        # away from the remainder bin each count is 1 + floor(p * 65280)
        assert np.all(np.abs(q - 1 - exact)[mask] < 1.0 + 1e-3)
        cum = cumulative(q)
        assert np.all(cum[:, 0] == 0) and np.all(cum[:, -1] == 65536)
        assert np.all(np.diff(cum, axis=1) >= 1)


def test_quantize_special_cases():
    q = quantize(np.full((1, 256), 1.0 / 256))
    assert np.all(q == 256)
    p = np.zeros((1, 256))
    p[0, 77] = 1.0
    q = quantize(p)[0]
    assert q[77] == 65536 - 255 and np.all(np.delete(q, 77) == 1)
    # the remainder goes to the argmax bin, the lowest index on ties:
    # 0.4 * 65280 = 26112 -> 26113 for bins 5 and 9, 0.2/254 * 65280 = 51.4 ->
    # 52 elsewhere, so R = 65536 - (2 * 26113 + 254 * 52) = 102 lands on bin 5.
    p = np.full((1, 256), 0.2 / 254)
    p[0, 5] = p[0, 9] = 0.4
    q = quantize(p)[0]
    assert q[9] == 26113 and q[5] == 26113 + 102 and q[0] == 52


# ---------------------------------------------------------------- coder

def test_handworked_example():
    g = _golden("rangecoder_handworked.txt")
    q = [int(v) for v in g["freq"]]
    cum = [0] + list(itertools.accumulate(q))
    sym = [int(v) for v in g["symbols"]]
    expect = bytes(int(v, 16) for v in g["payload"])
    assert _encode(cum, q, sym) == expect
    assert _decode(expect, cum, len(sym)) == sym

    qu = [int(g["freq_uniform"][0])] * 256
    cumu = [0] + list(itertools.accumulate(qu))
    symu = [int(v) for v in g["symbols_uniform"]]
    expectu = bytes(int(v, 16) for v in g["payload_uniform"])
    assert _encode(cumu, qu, symu) == expectu


@pytest.mark.parametrize("freqs", [[1, 65535], [65535, 1], [3, 65530, 3], [21845, 21845, 21846]])
def test_exhaustive_tiny_roundtrip(freqs):
    cum = [0] + list(itertools.accumulate(freqs))
    n = len(freqs)
    for length in range(0, 5):
        for syms in itertools.product(range(n), repeat=length):
            pay = _encode(cum, freqs, syms)
            assert _decode(pay, cum, length) == list(syms)


class CountingEncoder(RangeEncoder):
    carries = 0

    def _carry(self):
        CountingEncoder.carries += 1
        super()._carry()


def test_random_roundtrip_and_length_bound_with_carries():
    r = np.random.default_rng(1)
    CountingEncoder.carries = 0
    for trial in range(40):
        n = int(r.integers(1, 3000))
        # skewed random tables per symbol (like an adaptive model)
        enc = CountingEncoder(16)
        tables, syms, ideal = [], [], 0.0
        for _ in range(n):
            z = r.standard_normal(256) * r.choice([0.5, 3.0, 10.0])
            p = np.exp(z - z.max())
            p /= p.sum()
            q = quantize(p[None])[0]
            cum = cumulative(q[None])[0]
            x = int(r.choice(256, p=p))
            enc.encode(int(cum[x]), int(q[x]))
            tables.append(cum)
            syms.append(x)
            ideal += 16 - math.log2(q[x])
        pay = enc.finish()
        dec = RangeDecoder(pay, 16)
        assert [dec.decode(list(t)) for t in tables] == syms
        # interval bound: bytes <= ceil(ideal / 8) + 2, plus the truncation
        # slack of the multiply-first interval (< 256/2^24 bits per symbol)
        slack = n * 256.0 / (2 ** 24 * math.log(2))
        assert len(pay) <= math.ceil((ideal + slack) / 8.0) + 2
        assert len(pay) >= math.floor(ideal / 8.0)
    assert CountingEncoder.carries > 0


def test_carry_through_ff_bytes():
    # Force a long run of 0xFF: coding the top symbol of a [1, 65535] table
    # many times pushes low up against 2^32.
    freqs = [65535, 1]
    cum = [0, 65535, 65536]
    CountingEncoder.carries = 0
    for pattern in ([1] * 3 + [0] * 40 + [1], [0] * 200 + [1, 1, 0, 1]):
        enc = CountingEncoder(16)
        for x in pattern:
            enc.encode(cum[x], freqs[x])
        pay = enc.finish()
        assert _decode(pay, cum, len(pattern)) == pattern
    assert CountingEncoder.carries > 0


def test_empty_stream_writes_nothing():
    assert RangeEncoder().finish() == b""


def test_uniform_prefix_verbatim():
    r = np.random.default_rng(3)
    data = bytes(r.integers(0, 256, 50).tolist())
    pay = _encode(list(range(0, 65537, 256)), [256] * 256, data)
    assert pay == data + b"\x00"
