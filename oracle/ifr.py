"""Mutual information by Kraskov's estimator and the Information Flow
Refinement metric (oracle side).  Test infrastructure only.

Sec. 3.1.1 measures how much a refinement block's added feature X^(k) (the
sum of its k branches) leaves the skip connection S redundant, through the
mutual information I(S; S + X^(k)) (Eqs. 3-6), estimated with Kraskov's
non-parametric estimator (Eq. 7; Kraskov, Stoegbauer & Grassberger 2004,
their first estimator):

    I(Z; Y) ~ psi(v) + psi(c) - (1/c) sum_i [psi(c_z(i) + 1) + psi(c_y(i) + 1)]

over c samples (rows), v nearest neighbours.  For sample i, eps_i is the
distance to its v-th nearest neighbour in the joint space (Z, Y) under the
maximum norm, max(||z_i - z_j||_inf, ||y_i - y_j||_inf), other samples only,
ties counted with multiplicity; c_z(i) (c_y(i)) is the number of samples j
!= i with ||z_i - z_j||_inf < eps_i (strictly).  IFR_{k1->k2} is the ratio
I^(k1) / I^(k2) (Eq. 8).

Distances are taken in FP32 (each |z_ic - z_jc| a correctly rounded FP32
difference, the maximum exact), the precision of the GPU kernel, so that the
integer neighbour counts are decided identically on both sides; digamma and
the average are FP64.  Pinned by tests/test_oracle_ifr.py: the closed form
-log(1 - rho^2) / 2 of a bivariate Gaussian, independence, a hand-worked
four-point case, and a library neighbour search (scipy's k-d tree under the
max norm) on data where every difference is exact.
"""

from __future__ import annotations

import numpy as np
from scipy.special import digamma


def max_norm_distances(x: np.ndarray) -> np.ndarray:
    """[c, c] FP32 matrix of ||x_i - x_j||_inf for rows of x (FP32)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    c = x.shape[0]
    out = np.empty((c, c), dtype=np.float32)
    for i in range(c):  # row by row keeps memory at O(c d)
        out[i] = np.abs(x[i][None, :] - x).max(axis=1)
    return out


def ksg_counts(z: np.ndarray, y: np.ndarray, v: int):
    """(eps [c] FP32, c_z [c], c_y [c]) of Kraskov's first estimator."""
    dz = max_norm_distances(z)
    dy = max_norm_distances(y)
    c = dz.shape[0]
    if not 1 <= v < c:
        raise ValueError("need 1 <= v < number of samples")
    joint = np.maximum(dz, dy)
    eps = np.empty(c, dtype=np.float32)
    cz = np.empty(c, dtype=np.int64)
    cy = np.empty(c, dtype=np.int64)
    for i in range(c):
        others = np.delete(np.arange(c), i)
        d = np.sort(joint[i, others], kind="stable")
        eps[i] = d[v - 1]
        cz[i] = int((dz[i, others] < eps[i]).sum())
        cy[i] = int((dy[i, others] < eps[i]).sum())
    return eps, cz, cy


def ksg_mi(z: np.ndarray, y: np.ndarray, v: int = 3) -> float:
    """I(Z; Y) in nats by Eq. 7."""
    _, cz, cy = ksg_counts(z, y, v)
    c = cz.shape[0]
    return float(digamma(v) + digamma(c) - np.mean(digamma(cz + 1) + digamma(cy + 1)))


def ifr(i_k1: float, i_k2: float) -> float:
    """IFR_{k1 -> k2} = I^(k1)(S; S + X^(k1)) / I^(k2)(S; S + X^(k2)) (Eq. 8)."""
    return i_k1 / i_k2
