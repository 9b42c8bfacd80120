"""Pins of oracle/detect.py (detection step, Sect. 6.1)."""
import math

import numpy as np

from oracle import detect as D
from oracle import healpix_ref as hp
from tests.test_oracle_neighbours import _brute_neighbours


def test_detect_equals_definition_with_brute_neighbours():
    """Random maps at NSIDE 8 over the whole sphere and over a cap (edge
    pixels excluded), with and without threshold and noise map, against the
    definition written out with the brute-force neighbour sets."""
    N = 8
    brute = _brute_neighbours(N)
    rng = np.random.default_rng(0)
    allp = np.arange(hp.npix(N))
    for cap in (None, 0.9):
        pix = allp if cap is None else allp[hp.pix2vec(N, allp)[:, 0] > math.cos(cap)]
        val = rng.normal(size=pix.size)
        sd = rng.uniform(0.5, 2.0, size=pix.size)
        inmap = dict(zip(pix.tolist(), val.tolist()))
        for thr, use_sd in ((-np.inf, False), (0.5, False), (0.8, True)):
            want = []
            for p, v, s in zip(pix, val, sd):
                nbs = brute[p]
                if all(q in inmap for q in nbs) and all(v > inmap[q] for q in nbs):
                    if (v / s if use_sd else v) >= thr:
                        want.append(p)
            got = D.detect_peaks(N, pix, val, thr, sd if use_sd else None)
            assert np.array_equal(got, np.array(want, np.int64)), (cap, thr, use_sd)


def test_single_bump_and_plateau():
    N = 32
    pix = np.arange(hp.npix(N))
    c = hp.pix2vec(N, np.array([5000]))[0]
    val = hp.pix2vec(N, pix) @ c  # maximum at pixel 5000 only
    assert np.array_equal(D.detect_peaks(N, pix, val), [5000])
    assert D.detect_peaks(N, pix, np.ones(pix.size)).size == 0  # strict: no peak on a plateau
    assert D.detect_peaks(N, pix, val, threshold=1.5).size == 0
