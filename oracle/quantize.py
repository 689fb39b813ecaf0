"""Integer CDF from Pr(i) (oracle side).  Test infrastructure only.

The paper codes x_i "with" Pr(i) (Sec. 2.1, "Data Encoding") and does not say
how the distribution is made integer.  Reading used, with total T = 2**bits
(16-bit CDF) and minimum frequency 1:

    q_v  = 1 + floor(fl32(fl32(p_v) * (T - 256)))          v = 0..255
    R    = T - sum_v q_v                                    (signed)
    q[argmax_v q_v] += R                                    lowest index on ties
    cum[0] = 0, cum[v+1] = cum[v] + q_v, cum[256] = T

The floor is taken in FP32 (the GPU kernel's precision), so that both sides
decide the integers in the same precision.

Pinned by: sum/positivity invariants, the uniform and one-hot special cases,
and |q_v - p_v (T-256)| <= 1 away from the argmax bin
(tests/test_oracle_coder.py).
"""

from __future__ import annotations

import numpy as np


def quantize(p: np.ndarray, bits: int = 16) -> np.ndarray:
    """Frequencies [n, 256] int64 from probabilities [n, 256]."""
    p = np.atleast_2d(p)
    T = 1 << bits
    p32 = p.astype(np.float32)
    scaled = p32 * np.float32(T - 256)
    q = 1 + np.floor(scaled).astype(np.int64)
    rem = T - q.sum(axis=1)
    am = np.argmax(q, axis=1)
    q[np.arange(q.shape[0]), am] += rem
    return q


def cumulative(q: np.ndarray) -> np.ndarray:
    """Exclusive prefix sums [n, 257]."""
    q = np.atleast_2d(q)
    cum = np.zeros((q.shape[0], q.shape[1] + 1), dtype=np.int64)
    np.cumsum(q, axis=1, out=cum[:, 1:])
    return cum
