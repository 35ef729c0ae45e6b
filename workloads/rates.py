"""Seeded per-channel noise rates.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written out from its published
definition: the state advances by the golden-gamma constant and each output is
the state passed through a two-multiply xor-shift finaliser. A uniform double
in [0, 1) takes the top 53 bits.
"""

from __future__ import annotations

import math

import numpy as np

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


def splitmix64_uniform(seed: int, count: int) -> np.ndarray:
    """`count` uniform doubles in [0, 1) from SplitMix64 seeded with `seed`."""
    out = np.empty(count, dtype=np.float64)
    state = seed & _MASK
    scale = 1.0 / float(1 << 53)
    for i in range(count):
        state = (state + _GAMMA) & _MASK
        z = state
        z = ((z ^ (z >> 30)) * _M1) & _MASK
        z = ((z ^ (z >> 27)) * _M2) & _MASK
        z ^= z >> 31
        out[i] = (z >> 11) * scale
    return out


def log_uniform_rates(n_channels: int, seed: int, lo: float = 1e-4, hi: float = 5e-3) -> np.ndarray:
    """Per-channel rates drawn i.i.d. log-uniform in [lo, hi): exp(ln lo + u ln(hi/lo))."""
    u = splitmix64_uniform(seed, n_channels)
    return np.exp(math.log(lo) + u * math.log(hi / lo))
