"""Pins for the oracle's Kraskov estimator and IFR (Sec. 3.1.1, Eqs. 3-8)
against facts other than its own formula: the mutual information of a
Gaussian pair, independence, a hand-worked case, and a library neighbour
search (scipy's k-d tree under the max norm)."""

import math
import os

import numpy as np
from scipy.spatial import cKDTree

from oracle.ifr import ifr, ksg_counts, ksg_mi, max_norm_distances

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ksg_handworked.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = [float(x) for x in line[1:]]
    return out


def test_handworked_four_points():
    g = _golden()
    z = np.array(g["z"], dtype=np.float32)[:, None]
    y = np.array(g["y"], dtype=np.float32)[:, None]
    v = int(g["v"][0])
    eps, cz, cy = ksg_counts(z, y, v)
    assert list(eps) == g["eps"] and list(cz) == g["cz"] and list(cy) == g["cy"]
    assert abs(ksg_mi(z, y, v) - g["mi_numerator"][0] / g["mi_denominator"][0]) < 1e-12


def _gauss_pairs(rho, c, d, seed):
    r = np.random.default_rng(seed)
    a = r.standard_normal((c, d))
    b = rho * a + math.sqrt(1.0 - rho * rho) * r.standard_normal((c, d))
    return a.astype(np.float32), b.astype(np.float32)


def test_gaussian_closed_form():
    # I = -log(1 - rho^2) / 2 per independent coordinate pair; the estimator's
    # error at 1500 samples, v = 3, is a few hundredths
    for rho, d in ((0.6, 1), (0.9, 1), (0.6, 3)):
        z, y = _gauss_pairs(rho, 1500, d, seed=int(rho * 100) + d)
        truth = -0.5 * d * math.log(1.0 - rho * rho)
        est = ksg_mi(z, y, 3)
        assert abs(est - truth) < 0.06 * d, (rho, d, est, truth)


def test_independent_variables():
    r = np.random.default_rng(3)
    z = r.standard_normal((1500, 2)).astype(np.float32)
    y = r.standard_normal((1500, 2)).astype(np.float32)
    assert abs(ksg_mi(z, y, 3)) < 0.04


def test_counts_match_library_neighbour_search():
    # dyadic grid data: every difference is exact in FP32 and FP64, and there
    # are many ties (equal distances, duplicated points)
    r = np.random.default_rng(11)
    z = (r.integers(0, 8, size=(300, 3)) / 4.0).astype(np.float32)
    y = (r.integers(0, 8, size=(300, 2)) / 4.0).astype(np.float32)
    for v in (1, 3, 5):
        eps, cz, cy = ksg_counts(z, y, v)
        joint = np.concatenate([z, y], axis=1).astype(np.float64)
        d, _ = cKDTree(joint).query(joint, k=v + 1, p=np.inf)
        assert np.array_equal(eps.astype(np.float64), d[:, v])
        # strictly inside eps: the grid step is 1/4, so radius eps - 1/8
        rz = cKDTree(z.astype(np.float64)).query_ball_point(z.astype(np.float64), eps - 0.125,
                                                            p=np.inf, return_length=True)
        ry = cKDTree(y.astype(np.float64)).query_ball_point(y.astype(np.float64), eps - 0.125,
                                                            p=np.inf, return_length=True)
        # (a duplicated point gives eps = 0: nothing is strictly closer)
        rz = np.where(eps == 0, 0, np.asarray(rz) - 1)
        ry = np.where(eps == 0, 0, np.asarray(ry) - 1)
        assert np.array_equal(cz, rz) and np.array_equal(cy, ry)


def test_distances_are_fp32_max_norm():
    r = np.random.default_rng(2)
    x = r.standard_normal((20, 7)).astype(np.float32)
    dm = max_norm_distances(x)
    for i in range(20):
        for j in range(20):
            assert dm[i, j] == max(abs(np.float32(a) - np.float32(b)) for a, b in zip(x[i], x[j]))
    assert np.all(np.diag(dm) == 0)


def test_ifr_is_a_ratio_of_mutual_informations():
    z, y = _gauss_pairs(0.8, 600, 1, seed=4)
    i1 = ksg_mi(z, y, 3)
    assert ifr(i1, i1) == 1.0
    assert ifr(2.0 * i1, i1) == 2.0
