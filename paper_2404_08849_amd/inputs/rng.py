"""Seeded synthetic-input randomness: SplitMix64 (Steele, Lea & Flood 2014).

Every random number that an initial state or perturbation uses comes from
here, so the CPU oracle and the GPU path are always fed byte-identical
arrays.  Uniforms take the top 53 bits of a SplitMix64 output; normal
deviates use the Box-Muller transform on two uniforms.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    """Return the first ``n`` SplitMix64 outputs for ``seed`` as uint64."""
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        z = state + _GAMMA * np.arange(1, n + 1, dtype=np.uint64)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, n):
    """``n`` doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed, n):
    """``n`` standard normal deviates by Box-Muller (cosine branch)."""
    u = uniform(seed, 2 * n)
    u1 = 1.0 - u[0::2]           # (0, 1]: log is finite
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
