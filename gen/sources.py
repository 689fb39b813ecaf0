"""Synthetic byte sources (stand-ins for the paper's corpora, Sec. 4.1 Table 1).

All randomness is drawn from counter-based SplitMix64 (Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): output n of a
stream keyed by k is ``splitmix64(k + n)``, where ``splitmix64(x)`` adds the
golden-ratio increment once and applies the published 64-bit finaliser.
Uniform doubles take the top 53 bits.

Sources
-------
* order-``o`` Markov bytes with a Zipf(s) law per context over a seeded
  permutation of the 256 symbols (text-like data);
* uniform random bytes (already-compressed / backup-like data);
* run-length bytes, geometric run lengths (structured binary);
* int16 little-endian samples of a noisy sinusoid (sound-like data);
* i.i.d. bytes over a four-letter alphabet with probabilities 1/2, 1/4,
  1/8, 1/8 (entropy 1.75 bits): a source an online model learns within a
  few hundred steps, so that coded probabilities become strongly peaked.

Every function is deterministic in its seeds.  Nothing here models or codes
the data; it only produces it.
"""

from __future__ import annotations

import math

import functools

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

#: Table seed used by every workload (arXiv id of the paper).
TABLE_SEED = 250718969


def splitmix64(x) -> np.ndarray:
    """SplitMix64 output for counter value(s) ``x`` (uint64, wrapping)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _u64(v: int) -> np.uint64:
    return np.uint64(v & _MASK64)


def uniform01(x) -> np.ndarray:
    """Uniform double in [0, 1) from the top 53 bits of ``splitmix64(x)``."""
    return (splitmix64(x) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _counter(key, n0: int, n: int) -> np.ndarray:
    """Uniforms n0..n0+n-1 of the counter stream keyed by ``key``."""
    with np.errstate(over="ignore"):
        idx = np.uint64(key) + np.arange(n0, n0 + n, dtype=np.uint64)
    return uniform01(idx)


def zipf_pmf(s: float, n: int = 256) -> np.ndarray:
    """Zipf law over ranks 1..n: w_r proportional to r**-s."""
    r = np.arange(1, n + 1, dtype=np.float64)
    w = r ** (-s)
    return w / w.sum()


def zipf_entropy_bits(s: float, n: int = 256) -> float:
    w = zipf_pmf(s, n)
    return float(-(w * np.log2(w)).sum())


def _rank_from_uniform(u: np.ndarray, cdf: np.ndarray) -> np.ndarray:
    """Inverse-CDF draw of a 0-based rank."""
    r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, len(cdf) - 1).astype(np.int64)


@functools.lru_cache(maxsize=4)
def markov_order2_table(order: int, table_seed: int = TABLE_SEED) -> np.ndarray:
    """65536 x 256 table of seeded permutations of the byte alphabet.

    Row c is the permutation for context key c: symbols sorted by the
    SplitMix64 key ``splitmix64(k_c + j)``, ``k_c = splitmix64(seed ^ (o<<56) ^ c)``.
    Entry ``[c, r]`` is the symbol of 0-based rank r.  Built in row blocks
    (same result, less memory at once) and kept per process, read-only.
    """
    out = np.empty((65536, 256), dtype=np.uint8)
    j = np.arange(256, dtype=np.uint64)[None, :]
    for c0 in range(0, 65536, 4096):
        c = np.arange(c0, c0 + 4096, dtype=np.uint64)
        kc = splitmix64(_u64(table_seed) ^ np.uint64(order << 56) ^ c)
        with np.errstate(over="ignore"):
            keys = splitmix64(kc[:, None] + j)
        out[c0:c0 + 4096] = np.argsort(keys, axis=1, kind="stable")
    out.setflags(write=False)
    return out


def stream_seed(s, table_seed: int = TABLE_SEED):
    """Per-stream sampling seed: splitmix64(table_seed + 1 + s)."""
    with np.errstate(over="ignore"):
        return splitmix64(np.uint64(table_seed + 1) + np.asarray(s, dtype=np.uint64))


def markov2_streams(n_streams: int, length: int, zipf_s: float = 1.2,
                    table_seed: int = TABLE_SEED, first_stream: int = 0) -> np.ndarray:
    """``[n_streams, length]`` uint8 from the order-2 Markov Zipf source.

    The first two bytes of each stream are uniform; afterwards byte i is the
    symbol of Zipf-drawn rank in the permutation of context (x[i-2], x[i-1]).
    Stream s uses uniforms ``uniform01(stream_seed(s) + i)``.  Row k is stream
    ``first_stream + k``; a shorter ``length`` yields an exact prefix.
    """
    table = markov_order2_table(2, table_seed)
    cdf = np.cumsum(zipf_pmf(zipf_s))
    seeds = stream_seed(np.arange(first_stream, first_stream + n_streams), table_seed)
    out = np.zeros((n_streams, length), dtype=np.uint8)
    chunk = 4096
    prev2 = np.zeros(n_streams, dtype=np.int64)
    prev1 = np.zeros(n_streams, dtype=np.int64)
    for i0 in range(0, length, chunk):
        n = min(chunk, length - i0)
        with np.errstate(over="ignore"):
            idx = seeds[:, None] + np.arange(i0, i0 + n, dtype=np.uint64)[None, :]
        u = uniform01(idx)
        ranks = _rank_from_uniform(u, cdf)
        for j in range(n):
            i = i0 + j
            if i < 2:
                x = np.floor(u[:, j] * 256.0).astype(np.int64)
            else:
                x = table[prev2 * 256 + prev1, ranks[:, j]].astype(np.int64)
            out[:, i] = x
            prev2, prev1 = prev1, x
    return out


#: Law of the skewed source: ranks 0..3 with these probabilities, written as
#: the bytes "a".."d".
SKEWED_PROBS = (0.5, 0.25, 0.125, 0.125)
SKEWED_FIRST_BYTE = 0x61


def skewed_streams(n_streams: int, length: int, table_seed: int = TABLE_SEED,
                   first_stream: int = 0) -> np.ndarray:
    """``[n_streams, length]`` uint8 of i.i.d. skewed bytes.

    Byte i of stream s is the inverse-CDF rank of
    ``uniform01(stream_seed(s, table_seed + 2) + i)`` under SKEWED_PROBS,
    offset to SKEWED_FIRST_BYTE.  A shorter ``length`` yields an exact prefix.
    """
    cdf = np.cumsum(np.asarray(SKEWED_PROBS, dtype=np.float64))
    seeds = stream_seed(np.arange(first_stream, first_stream + n_streams), table_seed + 2)
    with np.errstate(over="ignore"):
        idx = seeds[:, None] + np.arange(length, dtype=np.uint64)[None, :]
    ranks = _rank_from_uniform(uniform01(idx), cdf)
    return (SKEWED_FIRST_BYTE + ranks).astype(np.uint8)


# --------------------------------------------------------------------------
# Mixture source (ragged streams)
# --------------------------------------------------------------------------

SEG_MARKOV3, SEG_UNIFORM, SEG_RUNS, SEG_SINE = 0, 1, 2, 3


def _hash3_table(table_seed: int) -> np.ndarray:
    """16-bit permutation-table row for every 3-byte context."""
    c = np.arange(1 << 24, dtype=np.uint64)
    h = splitmix64(c ^ _u64(table_seed ^ (3 << 56))) >> np.uint64(48)
    return h.astype(np.int64)


def ragged_lengths(n_streams: int, total: int, lo: int, hi: int,
                   table_seed: int = TABLE_SEED) -> np.ndarray:
    """Log-uniform lengths in [lo, hi], rescaled so they sum to ``total``.

    The rescaling keeps the log-uniform shape and the stream count while
    fixing the total; the remainder of the integer rounding goes one byte each
    to the first streams.
    """
    u = _counter(splitmix64(_u64(table_seed ^ (0xC3 << 48))), 0, n_streams)
    lam = np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
    scaled = np.floor(lam * (total / lam.sum())).astype(np.int64)
    rem = total - int(scaled.sum())
    scaled[:rem] += 1
    return scaled


def _segments(s: int, length: int, table_seed: int):
    key = int(splitmix64(_u64(table_seed ^ (0xC3 << 40) ^ s)))
    segs = []
    pos = 0
    k = 0
    while pos < length:
        u = _counter(key, 2 * k, 2)
        typ = min(int(u[0] * 4.0), 3)
        seg_len = int(1024.0 * 64.0 ** float(u[1]))
        seg_len = min(seg_len, length - pos)
        ckey = int(splitmix64(_u64(key + ((k + 1) << 32))))
        segs.append((typ, pos, seg_len, ckey))
        pos += seg_len
        k += 1
    return segs


def _fill_uniform(buf, start, n, ckey):
    buf[start:start + n] = np.floor(_counter(ckey, 0, n) * 256.0).astype(np.uint8)


def _fill_runs(buf, start, n, ckey, p=1.0 / 20.0):
    filled = 0
    n0 = 0
    while filled < n:
        m = max(16, 2 * (n - filled) // 20 + 16)
        u = _counter(ckey, n0, 2 * m)
        n0 += 2 * m
        u_len = 1.0 - u[0::2]  # in (0, 1]
        run = 1 + np.floor(np.log(u_len) / math.log(1.0 - p)).astype(np.int64)
        val = np.floor(u[1::2] * 256.0).astype(np.uint8)
        chunk = np.repeat(val, run)
        take = min(len(chunk), n - filled)
        buf[start + filled:start + filled + take] = chunk[:take]
        filled += take


def _fill_sine(buf, start, n, ckey, amplitude=16384.0, sigma=0.05):
    n_samp = (n + 1) // 2
    f = 0.001 + 0.049 * float(_counter(ckey, 0, 1)[0])
    u = _counter(ckey, 1, 2 * n_samp)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    noise = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    t = np.arange(n_samp, dtype=np.float64)
    v = np.sin(2.0 * math.pi * f * t) + sigma * noise
    q = np.clip(np.rint(amplitude * v), -32768, 32767).astype("<i2")
    buf[start:start + n] = q.view(np.uint8)[:n]


def mixture_streams(lens: np.ndarray, zipf_s: float = 1.1,
                    table_seed: int = TABLE_SEED, prefix: int | None = None):
    """Concatenated streams of seeded segments of the four source kinds.

    Segment type is uniform over {order-3 Markov Zipf(1.1), uniform bytes,
    runs, int16 sine}; segment length is log-uniform in [1 KiB, 64 KiB],
    truncated at the end of the stream.  Order-3 contexts select one of the
    65536 order-3 permutation rows through a 16-bit SplitMix64 hash; the first
    three bytes of each Markov segment are uniform.

    ``prefix`` truncates every stream to at most that many bytes (an exact
    prefix of the full stream).  Returns (flat uint8 data, lengths).
    """
    lens = np.asarray(lens, dtype=np.int64)
    full_lens = lens
    out_lens = lens if prefix is None else np.minimum(lens, prefix)
    offs = np.concatenate([[0], np.cumsum(out_lens)])
    buf = np.zeros(int(offs[-1]), dtype=np.uint8)
    markov = []
    for s in range(len(lens)):
        for typ, pos, n, ckey in _segments(s, int(full_lens[s]), table_seed):
            if pos >= out_lens[s]:
                break
            n = min(n, int(out_lens[s]) - pos)
            start = int(offs[s]) + pos
            if typ == SEG_UNIFORM:
                _fill_uniform(buf, start, n, ckey)
            elif typ == SEG_RUNS:
                _fill_runs(buf, start, n, ckey)
            elif typ == SEG_SINE:
                _fill_sine(buf, start, n, ckey)
            else:
                markov.append((start, n, ckey))
    if markov:
        _fill_markov3(buf, markov, zipf_s, table_seed)
    return buf, out_lens


def _fill_markov3(buf, segs, zipf_s, table_seed):
    table = markov_order2_table(3, table_seed)
    h3 = _hash3_table(table_seed)
    cdf = np.cumsum(zipf_pmf(zipf_s))
    starts = np.array([s[0] for s in segs], dtype=np.int64)
    lens = np.array([s[1] for s in segs], dtype=np.int64)
    keys = np.array([s[2] for s in segs], dtype=np.uint64)
    order = np.argsort(-lens, kind="stable")
    starts, lens, keys = starts[order], lens[order], keys[order]
    ctx = np.zeros(len(segs), dtype=np.int64)
    chunk = 2048
    maxlen = int(lens.max())
    for j0 in range(0, maxlen, chunk):
        act = int((lens > j0).sum())
        n = min(chunk, maxlen - j0)
        with np.errstate(over="ignore"):
            idx = keys[:act, None] + np.arange(j0, j0 + n, dtype=np.uint64)[None, :]
        u = uniform01(idx)
        ranks = _rank_from_uniform(u, cdf)
        for jj in range(n):
            j = j0 + jj
            a = int((lens[:act] > j).sum())
            if a == 0:
                break
            if j < 3:
                x = np.floor(u[:a, jj] * 256.0).astype(np.int64)
            else:
                x = table[h3[ctx[:a]], ranks[:a, jj]].astype(np.int64)
            buf[starts[:a] + j] = x.astype(np.uint8)
            ctx[:a] = ((ctx[:a] << 8) | x) & 0xFFFFFF
