"""Catalogue partition and pixel sums in plain numpy.

* partition (Sect. 3.4): the pixel of each galaxy (RING numbering), the
  catalogue reordered so that galaxies of one pixel are contiguous (stable:
  equal pixels keep catalogue order), and the offset table, so that pixel n
  owns sorted rows [off[n], off[n+1]);
* pixel sums (Sect. 3.2, step 2): per pixel the sum of weights W, the
  weighted shear sums G1, G2 and E2 = sum w^2 |g|^2 (the per-pixel input of
  the noise estimate, Eq. map_noise).

Pins (tests/test_oracle_binning.py): offsets are a prefix sum of the counts;
every sorted row lies in its pixel's range; the permutation is stable;
per-pixel sums equal a Python loop with math.fsum on a small catalogue.
"""
from __future__ import annotations

import numpy as np

from . import healpix_ref as hp


def partition(nside, ra, dec):
    pix = hp.radec2pix(nside, ra, dec)
    order = np.argsort(pix, kind="stable")
    counts = np.bincount(pix, minlength=hp.npix(nside))
    off = np.zeros(hp.npix(nside) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return pix, order, off


def pixel_sums(nside, ra, dec, g1, g2, w=None):
    """Returns (pix_unique, W, G1, G2, E2) over occupied pixels, sorted."""
    pix = hp.radec2pix(nside, ra, dec)
    g1 = np.asarray(g1, np.float64)
    g2 = np.asarray(g2, np.float64)
    w = np.ones_like(g1) if w is None else np.asarray(w, np.float64)
    u, inv = np.unique(pix, return_inverse=True)
    W = np.bincount(inv, weights=w, minlength=u.size)
    G1 = np.bincount(inv, weights=w * g1, minlength=u.size)
    G2 = np.bincount(inv, weights=w * g2, minlength=u.size)
    E2 = np.bincount(inv, weights=w * w * (g1 * g1 + g2 * g2), minlength=u.size)
    return u, W, G1, G2, E2
