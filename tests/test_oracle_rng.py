"""Pins of oracle/rng.py: the Philox4x64-10 words from the published round
function (plain Python integers, no numpy), the counter convention, and
the distribution of the angle fractions."""
import numpy as np

from oracle import rng as R

# multipliers and Weyl key increments of Philox4x64 (Salmon et al. 2011)
M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
MASK = (1 << 64) - 1


def _philox4x64_10(ctr, key):
    x = list(ctr)
    k0, k1 = key
    for _ in range(10):
        p0, p1 = M0 * x[0], M1 * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k0, p1 & MASK, (p0 >> 64) ^ x[3] ^ k1, p0 & MASK]
        k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
    return x


def test_words_follow_the_published_rounds():
    for seed, r in [(0, 0), (12345, 7), (2 ** 63 + 5, 255)]:
        w = R.philox_words(seed, r, 11)
        for j in range(11):
            assert int(w[j]) == _philox4x64_10([j // 4 + 1, 0, 0, 0], [seed, r])[j % 4], (seed, r, j)


def test_angles_exact_and_uniform():
    u = R.noise_angles(9, 3, 4, 50001)
    k = R.philox_words(9, 5, 50001)
    ref = ((k >> np.uint64(41)).astype(np.float64) + 0.5) / 2.0 ** 23
    assert np.array_equal(u[2].astype(np.float64), ref)  # exact in float32
    assert u.min() > 0 and u.max() < 1
    # mean 1/2 and variance 1/12 within five standard errors
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
    # different realisations are different streams
    assert not np.array_equal(u[0], u[1])
