"""Counter-based normal stream for the rank-growth columns.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the k-th output of a generator seeded with s is
mix(s + k * 0x9E3779B97F4A7C15) mod 2^64 with the published finaliser

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31).

Normals use the Box-Muller transform on two 53-bit uniforms.  Element t of event
e uses counters k1 = e * 2^40 + 2 t + 1 and k2 = k1 + 1:
u1 = ((mix(k1) >> 11) + 1) 2^-53 in (0, 1], u2 = (mix(k2) >> 11) 2^-53,
x = sqrt(-2 ln u1) cos(2 pi u2).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix_output(seed: int, k: np.ndarray) -> np.ndarray:
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix(np.uint64(seed) + k * GAMMA)


def normals(seed: int, event: int, count: int) -> np.ndarray:
    t = np.arange(count, dtype=np.uint64)
    base = np.uint64(event) << np.uint64(40)
    k1 = base + np.uint64(2) * t + np.uint64(1)
    k2 = k1 + np.uint64(1)
    u1 = ((splitmix_output(seed, k1) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (splitmix_output(seed, k2) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
