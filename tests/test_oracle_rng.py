"""Pins of oracle/rng.py: the Philox4x64-10 words from the published round
function (plain Python integers, no numpy), the counter convention, and
the distribution of the angle fractions; the galaxy-level Philox4x32-10
against the generator's published known-answer vectors."""
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


# known-answer vectors of Philox4x32-10 published with the generator
# (Salmon et al. 2011, the Random123 test vectors): (counter, key, output)
KAT_4X32 = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox4x32_known_answers():
    for ctr, key, out in KAT_4X32:
        got = R.philox4x32_10(*ctr, *key)
        assert [int(x) for x in got] == list(out), (ctr, key)
    # vectorised over counters: every lane equals its own scalar evaluation
    c0 = np.array([0, 1, 0xFFFFFFFF, 12345], dtype=np.uint64)
    v = R.philox4x32_10(c0, 7, 3, 0, 99, 5)
    for j, x in enumerate(c0):
        s = R.philox4x32_10(int(x), 7, 3, 0, 99, 5)
        assert [int(w[j]) for w in v] == [int(w) for w in s]


def test_galaxy_angles_stream_and_distribution():
    seed = 2 ** 40 + 17
    u = R.galaxy_angles(seed, 5, 7, 3001)  # realisations 5 .. 11 cross two blocks of four
    for r in range(7):
        ra = 5 + r
        for i in (0, 1, 2999, 3000):
            w = R.philox4x32_10(i, 0, ra // 4, 0, seed & 0xFFFFFFFF, seed >> 32)[ra % 4]
            assert u[r, i] == np.float32(((int(w) >> 9) + 0.5) / 2 ** 23)
    # a galaxy index past 2^32 uses the counter's second word
    big = R.philox4x32_10(5, 1, 0, 0, 1, 0)
    assert [int(x) for x in big] != [int(x) for x in R.philox4x32_10(5, 0, 0, 0, 1, 0)]
    uu = R.galaxy_angles(3, 0, 8, 40000)
    assert uu.min() > 0 and uu.max() < 1
    n = uu.size
    assert abs(uu.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(uu.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
