"""Realisation angles of the shape-noise maps, FP64 side (test infrastructure).

The paper builds noise maps from many copies of the catalogue with the
galaxies' orientations randomly rotated (Sect. 1, Sect. 5.3); it names no
generator. Reading: realisation r rotates source j by the angle pi u with
u = ((k >> 41) + 0.5) 2^-23 and k the j-th 64-bit word of the
Philox4x64-10 stream keyed by (seed, r) (Salmon et al. 2011), which
numpy.random.Philox implements: word j is output j mod 4 of the block at
counter j // 4 + 1. The 23-bit fraction plus one half is exact in float32,
so this side and the device draw identical u.

Galaxy-level realisations draw one angle per galaxy and realisation from
the 32-bit variant: realisation r rotates galaxy i (its catalogue index) by
u = ((x >> 9) + 0.5) 2^-23 with x word r mod 4 of Philox4x32-10 at counter
(i mod 2^32, i // 2^32, r // 4, 0) and key (seed mod 2^32, seed // 2^32).
numpy has no Philox4x32; philox4x32_10 below is the published round
function (two 32 x 32 -> 64-bit products per round with the published
multipliers, the key bumped by the published Weyl constants), vectorised
over counters in uint64 arithmetic.

Pins: tests/test_oracle_rng.py re-derives the 64-bit words from the published
round function and constants in plain Python integers, checks the 32-bit
generator against the published known-answer vectors of Philox4x32-10, and
checks the uniformity of u.
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


_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 of the counters (c0, c1, c2, c3) (uint32 values held in
    uint64 arrays or scalars) under the key (k0, k1); returns the four output
    words as uint64 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & _LO for x in (c0, c1, c2, c3)]
    k0 = np.uint64(k0) & _LO
    k1 = np.uint64(k1) & _LO
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & _LO, p1 & _LO, ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & _LO, p0 & _LO]
        k0 = (k0 + _W0) & _LO
        k1 = (k1 + _W1) & _LO
    return c


def galaxy_angles(seed: int, r_first: int, n_real: int, n_gal: int) -> np.ndarray:
    """u[r][i] in (0, 1) as float32, realisation r_first + r, galaxy i."""
    i = np.arange(n_gal, dtype=np.uint64)
    lo, hi = i & _LO, i >> np.uint64(32)
    u = np.empty((n_real, n_gal), dtype=np.float32)
    for r in range(n_real):
        ra = r_first + r
        w = philox4x32_10(lo, hi, np.uint64(ra >> 2), np.uint64(0), seed & 0xFFFFFFFF, seed >> 32)[ra & 3]
        u[r] = ((w >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    return u
