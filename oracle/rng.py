"""Counter-based initialisation (oracle side).  Test infrastructure only.

The paper starts encoder and decoder from the same randomly initialised
parameters and stores no weights (Sec. 2.1, "Overall Process"; Sec. 3.2 says
the FDM is "initialized randomly").  How the random values are drawn is not
stated; the reading used here:

    r   = SplitMix64(seed + (tensor_id << 40) + j)      (mod 2**64)
    a   = ((r >> 40) - 2**23) / 2**23                   exact in FP32, in [-1, 1)
    w   = fl32(a * fl32(bound))                          one FP32 multiply

for element j (row-major) of tensor ``tensor_id``.  SplitMix64 is Steele, Lea
and Flood (2014): add 0x9E3779B97F4A7C15, then the two xor-shift-multiply
rounds and a final xor-shift.  Values are produced in FP32 so that the GPU
library, which implements the same published generator independently, starts
from bit-identical weights.

Pinned by: the published first output of SplitMix64 from state 0, and
exact FP32 representability / range checks (tests/test_oracle_rng.py).
"""

from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
M64 = (1 << 64) - 1


def splitmix64_int(x: int) -> int:
    """One SplitMix64 output for counter ``x`` (Python integers)."""
    z = (x + GOLDEN) & M64
    z = ((z ^ (z >> 30)) * MIX1) & M64
    z = ((z ^ (z >> 27)) * MIX2) & M64
    return z ^ (z >> 31)


def splitmix64_vec(x: np.ndarray) -> np.ndarray:
    """Vectorised SplitMix64 over a uint64 array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        return z ^ (z >> np.uint64(31))


def uniform_pm1_f32(seed: int, tensor_id: int, start: int, count: int) -> np.ndarray:
    """FP32 values a_j in [-1, 1) on a 2**-23 grid, j = start .. start+count-1."""
    base = (seed + (tensor_id << 40) + start) & M64
    with np.errstate(over="ignore"):
        ctr = np.uint64(base) + np.arange(count, dtype=np.uint64)
    r = splitmix64_vec(ctr)
    k = (r >> np.uint64(40)).astype(np.int64) - (1 << 23)
    return (k.astype(np.float32) * np.float32(2.0 ** -23)).astype(np.float32)


def init_tensor(seed: int, tensor_id: int, shape, bound: float, start: int = 0) -> np.ndarray:
    """FP32 tensor with entries fl32(a_j * fl32(bound))."""
    n = int(np.prod(shape))
    a = uniform_pm1_f32(seed, tensor_id, start, n)
    return (a * np.float32(bound)).astype(np.float32).reshape(shape)
