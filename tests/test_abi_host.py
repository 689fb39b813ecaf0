"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every declared symbol, the host-compiled coder is byte-identical to
the oracle's coder, configuration and container errors are reported."""

import os
import re
import struct
import zlib

import numpy as np
import pytest

import paper_2507_18969_amd as E
from oracle.quantize import cumulative, quantize
from oracle.rangecoder import RangeEncoder

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    L = E.lib()
    with open(os.path.join(ROOT, "include", "edpc.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"\b(edpc_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(E.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name
    assert L.edpc_abi_version() == 2


def test_host_coder_matches_oracle_coder():
    r = np.random.default_rng(5)
    for n in (0, 1, 2, 17, 1500):
        z = r.standard_normal((max(n, 1), 256)) * r.choice([0.5, 4.0, 15.0])
        p = np.exp(z - z.max(1, keepdims=True))
        p /= p.sum(1, keepdims=True)
        q = quantize(p)
        cum = cumulative(q)
        sym = np.array([r.choice(256, p=pp) for pp in p[:n]], dtype=np.uint8)
        e = RangeEncoder()
        for t in range(n):
            e.encode(int(cum[t, sym[t]]), int(q[t, sym[t]]))
        ref = e.finish()
        got = E.edpc_rc_encode_host(cum[:max(n, 1)], sym)
        assert got == ref
        assert np.array_equal(E.edpc_rc_decode_host(cum, got, n), sym)


def test_config_validation():
    E.edpc_config_validate(E.edpc_config_default())
    for bad in (dict(embed=12), dict(embed=8), dict(context=6), dict(latent=48), dict(branches=4), dict(cdf_bits=12),
                dict(hidden=100), dict(context=0), dict(precision=7), dict(beta1=1.0)):
        with pytest.raises(E.EdpcError) as ei:
            E.edpc_config_validate(E.edpc_config_default(**bad))
        assert ei.value.status == -1
    c = E.edpc_config_default()
    c.struct_size = 12
    with pytest.raises(E.EdpcError):
        E.edpc_config_validate(c)


def test_low_rank_config_validation():
    # the low-rank factors run through the per-stream kernels: F = context *
    # embed a power of two <= 256, and the flag excludes the F x F ablation
    E.edpc_config_validate(E.edpc_config_default(context=16, embed=16, latent=64, low_rank=True))
    for bad in (dict(context=32, embed=16, latent=64, low_rank=True),
                dict(context=12, embed=16, latent=64, low_rank=True),
                dict(context=16, embed=16, latent=256, low_rank=True, lte=False)):
        with pytest.raises(E.EdpcError) as ei:
            E.edpc_config_validate(E.edpc_config_default(**bad))
        assert ei.value.status == -1


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_bench_ablation_configs_validate(precision):
    # every Table 4 variant the bench's ablation workload runs is accepted, and
    # carries the flag bits of its variant
    import bench
    import gen
    base = gen.WORKLOADS["small"].model
    for name, over in bench.ABLATIONS:
        cfg = bench.ablation_cfg(E, base, over, precision)
        E.edpc_config_validate(cfg)
        assert bool(cfg.flags & E.EDPC_CFG_NO_LTE) == (over.get("lte") is False), name
        assert bool(cfg.flags & E.EDPC_CFG_LOW_RANK) == bool(over.get("low_rank")), name


def test_encode_bound():
    c = E.edpc_config_default()
    assert E.edpc_encode_bound(c, [10, 0, 5]) == 96 + 20 * 3 + (22 + 2 + 12)
    with pytest.raises(E.EdpcError):
        E.edpc_encode_bound(c, [])


def _header(lens, pay_lens, crcs, cfg=None, version=1, kernel=5 << 48, arch=950):
    """Container header written from the documented layout (independent of
    the library's writer)."""
    c = cfg or E.edpc_config_default()
    n = len(lens)
    b = b"EDPC" + struct.pack("<HHII", version, 0, 96 + 20 * n, n)
    b += struct.pack("<9I", c.context, c.embed, c.latent, c.blocks, c.hidden, c.branches,
                     c.cdf_bits, c.precision, c.flags)
    b += struct.pack("<4f", c.lr, c.beta1, c.beta2, c.eps)
    b += struct.pack("<QQII", c.seed, kernel, arch, 0)
    for l, p, k in zip(lens, pay_lens, crcs):
        b += struct.pack("<QQI", l, p, k)
    return b + struct.pack("<I", zlib.crc32(b))


def test_decode_info_reads_documented_layout():
    h = _header([100, 0, 7], [80, 0, 9], [1, 2, 3])
    cfg, lens, hl, total = E.edpc_decode_info(h)
    assert list(lens) == [100, 0, 7] and hl == len(h) and total == 107
    assert cfg.context == 16 and cfg.latent == 64


@pytest.mark.parametrize("mutate,status", [
    (lambda h: h[:10], -4),                       # shorter than the fixed header
    (lambda h: h[:-3], -4),                       # shorter than its header
    (lambda h: b"EDPX" + h[4:], -4),              # bad magic
    (lambda h: h[:30] + bytes([h[30] ^ 1]) + h[31:], -5),  # header CRC
])
def test_decode_info_errors(mutate, status):
    h = _header([100, 5], [80, 4], [1, 2])
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode_info(mutate(h))
    assert ei.value.status == status


def test_decode_info_rejects_version_and_bad_lengths():
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode_info(_header([10], [8], [0], version=2))
    assert ei.value.status == -6
    with pytest.raises(E.EdpcError) as ei:  # payload longer than 2 * len + 2
        E.edpc_decode_info(_header([10], [23], [0]))
    assert ei.value.status == -4
    with pytest.raises(E.EdpcError) as ei:  # non-empty payload for an empty stream
        E.edpc_decode_info(_header([0], [2], [0]))
    assert ei.value.status == -4


def test_decode_info_rejects_lengths_beyond_the_codec_limits():
    # crafted headers with valid CRCs: lengths whose arithmetic would wrap
    # (2 * len + 2, the sums of lengths) must be reported as corrupt before
    # any offset is formed from them
    big = E.EDPC_MAX_STREAM_LEN
    cfg, lens, _, total = E.edpc_decode_info(_header([big, 3], [12, 4], [0, 0]))
    assert list(lens) == [big, 3] and total == big + 3
    for lens_, pays in (([big + 1], [8]), ([1 << 63], [8]), ([(1 << 64) - 1], [2]),
                        ([5, 1 << 62], [4, 4])):
        with pytest.raises(E.EdpcError) as ei:
            E.edpc_decode_info(_header(lens_, pays, [0] * len(lens_)))
        assert ei.value.status == -4, (lens_, pays)
    # payload length that wraps 2 * len + 2
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode_info(_header([1 << 63], [(1 << 64) - 1], [0]))
    assert ei.value.status == -4


def test_decode_info_rejects_stream_count_beyond_limit():
    # only the fixed part is given: the count is refused before the header
    # length (which would be 20 bytes per stream) is consulted
    h = bytearray(_header([4], [3], [0]))
    struct.pack_into("<II", h, 8, 96 + 20 * (E.EDPC_MAX_STREAMS + 1), E.EDPC_MAX_STREAMS + 1)
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode_info(bytes(h[:96]))
    assert ei.value.status == -4


def test_encode_bound_rejects_overlong_streams():
    c = E.edpc_config_default()
    assert E.edpc_encode_bound(c, [E.EDPC_MAX_STREAM_LEN]) == 96 + 20 + 2 * E.EDPC_MAX_STREAM_LEN + 2
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_encode_bound(c, [E.EDPC_MAX_STREAM_LEN + 1])
    assert ei.value.status == -1


def test_config_flags_for_launch_choices():
    # the launch sequence and graph replay are configuration bits, not
    # environment settings
    c = E.edpc_config_default(precision="bf16", layerwise=True, graphs=False)
    assert c.flags & E.EDPC_CFG_LAYERWISE and c.flags & E.EDPC_CFG_NO_GRAPHS
    E.edpc_config_validate(c)
    c.flags |= 0x40
    with pytest.raises(E.EdpcError):
        E.edpc_config_validate(c)


def _exact_buffer(data: bytes):
    """A malloc'd copy of exactly len(data) bytes (so a read past its end is
    a heap overflow that the sanitizer build reports)."""
    import ctypes
    libc = ctypes.CDLL(None)
    libc.malloc.restype = ctypes.c_void_p
    libc.malloc.argtypes = [ctypes.c_size_t]
    libc.free.argtypes = [ctypes.c_void_p]
    p = libc.malloc(max(len(data), 1))
    ctypes.memmove(p, data, len(data))
    return p, libc


def test_decode_info_survives_mutated_headers():
    # random field corruptions with the header CRC recomputed (so parsing gets
    # past the checksum) and random truncations: every call either succeeds
    # with a consistent result or reports a documented error
    import ctypes
    r = np.random.default_rng(11)
    for it in range(600):
        n = int(r.integers(1, 6))
        lens = [int(x) for x in r.integers(0, 1 << 20, size=n)]
        pays = [min(2 * l + 2, int(r.integers(0, 2 * l + 3))) if l else 0 for l in lens]
        h = bytearray(_header(lens, pays, [0] * n))
        for _ in range(int(r.integers(1, 4))):
            h[int(r.integers(0, len(h) - 4))] = int(r.integers(0, 256))
        struct.pack_into("<I", h, len(h) - 4, zlib.crc32(bytes(h[:-4])))
        cut = len(h) if r.random() < 0.7 else int(r.integers(0, len(h)))
        p, libc = _exact_buffer(bytes(h[:cut]))
        try:
            cfg = E.edpc_config()
            cnt, hl, dl = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
            st = E.lib().edpc_decode_info(ctypes.c_void_p(p), cut, ctypes.byref(cfg), ctypes.byref(cnt),
                                          None, 0, ctypes.byref(hl), ctypes.byref(dl))
            assert st in (0, -1, -4, -5, -6), (it, st)
            if st == 0:
                assert hl.value <= cut and cnt.value == (hl.value - 96) // 20
        finally:
            libc.free(ctypes.c_void_p(p))


def test_host_decoder_reads_only_its_payload():
    # random payloads of every short length against peaked and flat CDFs: the
    # host decoder stops at in_len (garbage in, symbols out, no overread)
    import ctypes
    r = np.random.default_rng(12)
    for it in range(300):
        n = int(r.integers(1, 40))
        z = r.standard_normal((n, 256)) * r.choice([0.5, 8.0, 30.0])
        p = np.exp(z - z.max(1, keepdims=True))
        p /= p.sum(1, keepdims=True)
        cum = np.ascontiguousarray(cumulative(quantize(p)), dtype=np.uint32)
        pay = r.integers(0, 256, size=int(r.integers(0, 12)), dtype=np.uint8).tobytes()
        buf, libc = _exact_buffer(pay)
        sym = np.zeros(n, dtype=np.uint8)
        try:
            st = E.lib().edpc_rc_decode_host(cum.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(buf),
                                             len(pay), n, sym.ctypes.data_as(ctypes.c_void_p))
            assert st == 0
        finally:
            libc.free(ctypes.c_void_p(buf))
