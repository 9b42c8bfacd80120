"""Pins of the oracle's catalogue partition and pixel sums (oracle/binning.py)."""
import math

import numpy as np

from oracle import binning as B
from oracle import healpix_ref as hp
from synth import small_catalogue


def test_partition_invariants():
    nside = 32
    cat = small_catalogue(20000, seed=1, cap_radius=0.4, centre=(6.0, 0.3))
    pix, order, off = B.partition(nside, cat["ra"], cat["dec"])
    assert off[0] == 0 and off[-1] == pix.size
    assert np.all(np.diff(off) >= 0)
    sp = pix[order]
    # every sorted row lies in its pixel's range, and the range is exact
    for n in np.unique(sp)[:200]:
        rows = np.nonzero(sp == n)[0]
        assert rows[0] == off[n] and rows[-1] == off[n + 1] - 1
    # stable: equal pixels keep catalogue order
    for n in np.unique(sp)[:200]:
        seg = order[off[n]:off[n + 1]]
        assert np.all(np.diff(seg) > 0)


def test_pixel_sums_fsum():
    nside = 8
    cat = small_catalogue(3000, seed=2)
    u, W, G1, G2, E2 = B.pixel_sums(nside, cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"])
    pix = hp.radec2pix(nside, cat["ra"], cat["dec"])
    for k, n in enumerate(u[:150]):
        m = pix == n
        w = cat["w"][m].astype(float)
        g1 = cat["g1"][m].astype(float)
        g2 = cat["g2"][m].astype(float)
        assert abs(W[k] - math.fsum(w)) <= 1e-13 * abs(W[k])
        assert abs(G1[k] - math.fsum(w * g1)) <= 1e-13 * np.sum(np.abs(w * g1))
        assert abs(G2[k] - math.fsum(w * g2)) <= 1e-13 * np.sum(np.abs(w * g2))
        assert abs(E2[k] - math.fsum(w * w * (g1 * g1 + g2 * g2))) <= 1e-13 * E2[k]
