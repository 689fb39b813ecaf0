"""Pins for the oracle's compression loop (Algorithm 1 over many streams)
and for the reading of the LTE's shapes against the paper's printed counts."""

import math
import os

import numpy as np

import gen
import oracle
from oracle.codec import split_streams
from oracle.model import Config, Model, param_specs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SMALL = Config.from_dict(gen.WORKLOADS["small"].model)


def _streams(prefix, n=None, ragged=False):
    d, l = gen.make_streams("small", prefix=prefix, n_streams=n)
    st = split_streams(d, l)
    if ragged:  # cut to uneven lengths, some shorter than the context
        cuts = [prefix, 5, prefix // 2, 0, 17, prefix - 3, 16, 1][: len(st)]
        st = [s[:c] for s, c in zip(st, cuts)]
    return st


def test_roundtrip_ragged_with_short_and_empty_streams():
    st = _streams(96, ragged=True)
    pay, info = oracle.encode(st, SMALL)
    dec, _ = oracle.decode(pay, [len(s) for s in st], SMALL)
    assert dec == st
    for s, p in zip(st, pay):
        if len(s) == 0:
            assert p == b""
        # the first t bytes are coded with equal probability: they appear
        # verbatim at the front of the payload
        k = min(len(s), SMALL.context)
        assert p[:k] == s[:k]
        # ideal length bound (+2 bytes of flush)
        ideal = info["ideal_bits"][st.index(s)]
        assert len(p) <= math.ceil(ideal / 8.0 + 1e-3) + 2


def test_identity_case_zero_head_no_learning():
    # W_h = 0, b_h = 0, lr = 0 -> p = 1/256 exactly -> q = 256 for every byte:
    # the payload is the stream followed by one 0x00 byte.
    cfg = SMALL.with_(zero_head=True, lr=0.0)
    st = _streams(80, n=3)
    pay, _ = oracle.encode(st, cfg)
    assert pay == [s + b"\x00" for s in st]


def test_causality_prefix_probabilities():
    seen = {}

    def hook_full(i, act, cache, q, model):
        seen[("full", i)] = cache["p"].copy()

    def hook_short(i, act, cache, q, model):
        seen[("short", i)] = cache["p"].copy()

    st = _streams(60, n=3)
    oracle.encode(st, SMALL, hook=hook_full)
    oracle.encode([s[:40] for s in st], SMALL, hook=hook_short)
    for i in range(SMALL.context, 40):
        assert np.array_equal(seen[("full", i)], seen[("short", i)])


def test_learning_beats_static_model_on_skewed_source():
    # i.i.d. bytes over four symbols with probabilities 1/2, 1/4, 1/8, 1/8
    # (entropy 1.75 bits): a static model (lr = 0) with random weights codes
    # near 8 bits/byte, the online model must learn the law within 1.5k bytes
    r = np.random.default_rng(11)
    st = [bytes(r.choice(4, size=1536, p=[0.5, 0.25, 0.125, 0.125]).astype(np.uint8).tolist())
          for _ in range(4)]
    pay, _ = oracle.encode(st, SMALL)
    bpb = 8.0 * sum(map(len, pay)) / sum(map(len, st))
    pay0, _ = oracle.encode(st, SMALL.with_(lr=0.0))
    bpb0 = 8.0 * sum(map(len, pay0)) / sum(map(len, st))
    assert bpb0 > 7.0
    assert bpb < 4.0, (bpb, bpb0)


def test_source_conditional_entropy_matches_zipf():
    # order-2 Markov source: every context is Zipf(1.2) over a permutation,
    # so -log2 P(x_i | x_{i-2}, x_{i-1}) averages H(Zipf_1.2 on 256 symbols)
    from gen import sources
    data = sources.markov2_streams(64, 4096, 1.2)
    table = sources.markov_order2_table(2)
    w = sources.zipf_pmf(1.2)
    inv = np.argsort(table, axis=1)  # symbol -> rank
    ctx = data[:, :-2].astype(np.int64) * 256 + data[:, 1:-1]
    ranks = inv[ctx, data[:, 2:]]
    emp = float(-np.log2(w[ranks]).mean())
    h = sources.zipf_entropy_bits(1.2)
    assert abs(h - 5.29) < 0.01
    assert abs(emp - h) < 0.03


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


def test_lte_shapes_against_paper_table4():
    """Per-instance FDM of shape F' x F' (Sec. 3.2) reproduces the parameter
    differences printed in the ablation table at b = 4096, F = 256, r = 4."""
    g = _golden("paper_table4_fdm.txt")
    b, F, L = int(g["batch"]), int(g["feat"]), int(g["latent"])
    cfg = Config(context=16, embed=16, latent=L, blocks=0, hidden=8)
    assert cfg.feat == F
    m = Model(cfg, 1)
    fdm_per_stream = m.U[0].size
    sizes = {name: int(np.prod(shape)) for name, shape, _, _ in param_specs(cfg)}
    # "w/o LTE": the oracle's ablation model, a per-instance F x F FDM in place
    # of (W1, b1, per-instance U, W2, b2)
    cfg_n = cfg.with_(latent=F, lte=False)
    sizes_n = {name: int(np.prod(shape)) for name, shape, _, _ in param_specs(cfg_n)}
    delta_no_lte = (b * Model(cfg_n, 1).U[0].size + sum(sizes_n.values())
                    - b * fdm_per_stream - sum(sizes.values()))
    printed = g["params_without_lte"] - g["params_edpc"]
    assert abs(delta_no_lte - printed) / printed < 3e-3
    # "low-rank factorization": the oracle's ablation model, per-instance
    # factors A_s, U_s, B_s and no shared W1, b1, W2, b2 (with per-instance
    # biases the difference would be 1.3e6 larger, outside the bound)
    cfg_r = cfg.with_(low_rank=True)
    m_r = Model(cfg_r, 1)
    sizes_r = {name: int(np.prod(shape)) for name, shape, _, _ in param_specs(cfg_r)}
    delta_low_rank = (b * (m_r.A[0].size + m_r.B[0].size) + sum(sizes_r.values())
                      - sum(sizes.values()))
    printed_lr = g["params_low_rank"] - g["params_edpc"]
    assert abs(delta_low_rank - printed_lr) / printed_lr < 3e-3
    # FDM-module FLOPs: (2FF' + 2F'^2 + 2F'F) against 2F^2 without the LTE
    red = 100.0 * (1.0 - (4 * F * L + 2 * L * L) / (2.0 * F * F))
    assert abs(red - g["lte_flop_reduction_percent"]) < 0.02
