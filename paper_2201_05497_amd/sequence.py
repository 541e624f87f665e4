"""Random subset choices of LM-SPDHG (Algorithm 2 picks, before every
update, a data subset with probability p_k = 1/(2n) each or the prior with
probability 1/2; Section 3).

The draws come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), a counter-based generator:
output u of the stream started at `seed` depends only on (seed, u), so the
choices of a reconstruction resumed at update u are those of an unbroken
run.  The top bit of the output picks the prior; otherwise the low 63 bits
modulo n pick the data subset (modulo bias below n / 2^63).
"""
from __future__ import annotations

import numpy as np

__all__ = ["splitmix64", "subset_sequence"]

_MASK = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15  # the generator's increment
_MUL1 = 0xBF58476D1CE4E5B9
_MUL2 = 0x94D049BB133111EB


def splitmix64(seed: int, u: int) -> int:
    """Output number u (0-based) of the stream started at seed."""
    z = (seed + (u + 1) * _GOLDEN) & _MASK
    z = ((z ^ (z >> 30)) * _MUL1) & _MASK
    z = ((z ^ (z >> 27)) * _MUL2) & _MASK
    return z ^ (z >> 31)


def subset_sequence(seed: int, u0: int, count: int, n_subsets: int) -> np.ndarray:
    """Choices of updates u0 .. u0 + count - 1: n_subsets (the prior) or a
    data subset 0 .. n_subsets - 1, as int32."""
    out = np.empty(count, dtype=np.int32)
    for j in range(count):
        z = splitmix64(seed, u0 + j)
        out[j] = n_subsets if z >> 63 else (z & ((1 << 63) - 1)) % n_subsets
    return out
