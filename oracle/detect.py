"""Detection step of the paper (Sect. 6.1), FP64 side (test infrastructure).

After the aperture-mass maps are computed, every map pixel whose value is
higher than those of its eight direct HEALPix neighbours is a detection;
the paper then varies a threshold to trace purity against completeness.
Readings where the text is silent:

* "higher than" is strict: a pixel equal to a neighbour is not a peak;
* a pixel with a neighbour outside the map (the field's edge, an
  unlisted pixel) is not a detection: it cannot be shown to be a maximum;
* the threshold applies to the value itself, or, when a noise map is given
  (the standard deviation of the noise realisations of the same pixel),
  to the value divided by it (a signal-to-noise cut; pixels without a
  positive noise value are not detections);
* pixels touching a corner where three base faces meet have seven
  neighbours.

Neighbours come from oracle.healpix_ref.neighbours (pinned against a brute
force over cell corners). Pins: tests/test_oracle_detect.py.
"""
from __future__ import annotations

import numpy as np

from . import healpix_ref as hp


def detect_peaks(nside: int, pix, values, threshold: float = -np.inf, noise_sd=None, chunk: int = 200000):
    """Sorted RING pixels of the detections in a map given as strictly
    increasing pixels `pix` with `values` (and optional `noise_sd`)."""
    pix = np.asarray(pix, np.int64)
    val = np.asarray(values, np.float64)
    if pix.size > 1 and np.any(np.diff(pix) <= 0):
        raise ValueError("pixels must be strictly increasing")
    keep = []
    for s in range(0, pix.size, chunk):
        p = pix[s:s + chunk]
        v = val[s:s + chunk]
        nb = hp.neighbours(nside, p)
        idx = np.searchsorted(pix, np.where(nb >= 0, nb, 0))
        idx = np.minimum(idx, pix.size - 1)
        present = (pix[idx] == nb) | (nb < 0)
        nv = np.where(nb >= 0, val[idx], -np.inf)
        ok = present.all(axis=1) & (v[:, None] > nv).all(axis=1)
        if noise_sd is None:
            ok &= v >= threshold
        else:
            sd = np.asarray(noise_sd, np.float64)[s:s + chunk]
            with np.errstate(divide="ignore", invalid="ignore"):
                ok &= (sd > 0) & (v / np.where(sd > 0, sd, 1.0) >= threshold)
        keep.append(p[ok])
    return np.concatenate(keep) if keep else np.zeros(0, np.int64)
