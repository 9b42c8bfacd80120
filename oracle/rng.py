"""Realisation angles of the shape-noise maps, FP64 side (test infrastructure).

The paper builds noise maps from many copies of the catalogue with the
galaxies' orientations randomly rotated (Sect. 1, Sect. 5.3); it names no
generator. Reading: realisation r rotates source j by the angle pi u with
u = ((k >> 41) + 0.5) 2^-23 and k the j-th 64-bit word of the
Philox4x64-10 stream keyed by (seed, r) (Salmon et al. 2011), which
numpy.random.Philox implements: word j is output j mod 4 of the block at
counter j // 4 + 1. The 23-bit fraction plus one half is exact in float32,
so this side and the device draw identical u.

Pins: tests/test_oracle_rng.py re-derives the words from the published
round function and constants in plain Python integers, and checks the
uniformity of u.
"""
from __future__ import annotations

import numpy as np


def philox_words(seed: int, r: int, n: int) -> np.ndarray:
    """The first n 64-bit words of the stream keyed by (seed, r)."""
    g = np.random.Philox(key=np.array([seed, r], dtype=np.uint64))  # a list would pass through float
    return g.random_raw(n) if n > 0 else np.zeros(0, np.uint64)


def noise_angles(seed: int, r_first: int, n_real: int, n_src: int) -> np.ndarray:
    """u[r][j] in (0, 1) as float32, realisation r_first + r, source j."""
    u = np.empty((n_real, n_src), dtype=np.float32)
    for r in range(n_real):
        k = philox_words(seed, r_first + r, n_src)
        u[r] = ((k >> np.uint64(41)).astype(np.float64) + 0.5) * 2.0 ** -23
    return u
