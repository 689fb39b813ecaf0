"""Pins for the oracle's counter-based initialiser."""

import math

import numpy as np

from oracle import rng
from oracle.model import Config, init_fdm, init_shared, param_specs


def test_splitmix64_published_outputs():
    # SplitMix64 (Steele, Lea & Flood 2014) generator state 0: its first two
    # outputs are mix(0 + gamma) and mix(2 * gamma).  The first is the widely
    # quoted value 0xE220A8397B1DCDAF (java.util.SplittableRandom(0).nextLong()
    # == -2152535657050944081).
    assert rng.splitmix64_int(0) == 0xE220A8397B1DCDAF
    assert rng.splitmix64_int(0) - (1 << 64) == -2152535657050944081
    assert rng.splitmix64_int(rng.GOLDEN) == 0x6E789E6AA1B965F4


def test_vectorised_matches_scalar():
    xs = [0, 1, 2, 12345, (1 << 63) + 7, (1 << 64) - 1, 4 << 40]
    vec = rng.splitmix64_vec(np.array(xs, dtype=np.uint64))
    assert [int(v) for v in vec] == [rng.splitmix64_int(x) for x in xs]


def test_init_values_on_grid_and_in_range():
    a = rng.uniform_pm1_f32(seed=0, tensor_id=3, start=0, count=100000)
    assert a.dtype == np.float32
    k = a.astype(np.float64) * 2 ** 23
    assert np.all(k == np.round(k))
    assert a.min() >= -1.0 and a.max() < 1.0
    assert abs(a.mean()) < 0.01
    assert abs(a.var() - 1.0 / 3.0) < 0.01
    # element j of a tensor depends only on (seed, id, j): a slice equals the
    # tail of a longer draw
    b = rng.uniform_pm1_f32(seed=0, tensor_id=3, start=500, count=100)
    assert np.array_equal(a[500:600], b)


def test_init_scalar_recipe():
    # element 0 of tensor id 2 with seed 5: r = SplitMix64(5 + 2<<40), computed
    # here from the scalar definition.
    r = rng.splitmix64_int(5 + (2 << 40))
    k = (r >> 40) - (1 << 23)
    bound = np.float32(1.0 / math.sqrt(256))
    expect = np.float32(np.float32(k * 2.0 ** -23) * bound)
    got = rng.init_tensor(5, 2, (1,), 1.0 / math.sqrt(256))[0]
    assert got == expect


def test_fdm_slices_indexed_by_stream():
    cfg = Config(latent=8)
    u_all = init_fdm(cfg, range(5))
    u_3 = init_fdm(cfg, [3])[0]
    assert np.array_equal(u_all[3], u_3)
    assert not np.array_equal(u_all[2], u_all[3])
    assert np.abs(u_all).max() <= 1.0 / math.sqrt(8)


def test_shared_init_shapes_and_constants():
    cfg = Config(context=4, embed=3, latent=5, blocks=2, hidden=7)
    sh = init_shared(cfg)
    for name, shape, tid, bound in param_specs(cfg):
        assert sh[name].shape == shape
        if tid is None:
            assert np.all(sh[name] == np.float32(bound))
        else:
            assert np.abs(sh[name]).max() <= np.float32(bound)
    zh = init_shared(cfg.with_(zero_head=True))
    assert not zh["wh"].any() and not zh["bh"].any()
