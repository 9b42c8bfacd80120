"""Pins of the oracle's face coordinates and pixel neighbours
(oracle/healpix_ref.py), used by the detection step (Sect. 6.1: a pixel
above its eight direct neighbours is a detection)."""
import math

import numpy as np
import pytest

from oracle import healpix_ref as hp


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 256])
def test_face_chart_round_trip_and_cells(nside):
    """Every pixel is one cell of one face; the face chart maps each cell's
    centre (alpha, beta) = (i + 1/2, j + 1/2) to the pixel centre given by
    the ring formulas (an independent route), and back."""
    p = np.arange(hp.npix(nside)) if nside <= 16 else np.random.default_rng(1).integers(0, hp.npix(nside), 20000)
    f, ia, ib = hp.pix2face(nside, p)
    assert ia.min() >= 0 and ia.max() < nside and ib.min() >= 0 and ib.max() < nside
    if nside <= 16:
        assert np.unique((f * nside + ia) * nside + ib).size == p.size
        assert np.all(np.bincount(f, minlength=12) == nside * nside)
    z, omz, phi = hp.face_point(nside, f, ia + 0.5, ib + 0.5)
    zc, sc, phic = hp.pix2zphi(nside, p)
    assert np.max(np.abs(z - zc)) < 1e-12
    dphi = np.angle(np.exp(1j * (phi - phic)))
    assert np.max(np.abs(dphi * sc)) < 1e-12
    f2, a2, b2 = hp.face_coords(nside, z, np.mod(phi / (0.5 * math.pi), 4.0), omz)
    assert np.array_equal(f2, f) and np.max(np.abs(a2 - ia - 0.5)) < 1e-9 and np.max(np.abs(b2 - ib - 0.5)) < 1e-9


def _brute_neighbours(nside):
    """Neighbour sets by brute force: every cell corner (integer face
    coordinates) is placed on the sphere, the pixels of 96 points on a small
    circle around it are the pixels meeting there, and any two pixels meeting
    at a corner are neighbours."""
    nb = [set() for _ in range(hp.npix(nside))]
    k = np.arange(nside + 1)
    for f in range(12):
        a, b = np.meshgrid(k, k, indexing="ij")
        z, omz, phi = hp.face_point(nside, np.full(a.size, f), a.ravel().astype(float), b.ravel().astype(float))
        s = np.sqrt(omz * (2.0 - omz))
        v = np.stack([s * np.cos(phi), s * np.sin(phi), z], 1)
        # orthonormal tangent frame at each corner
        ref = np.where(np.abs(v[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
        e1 = np.cross(v, ref)
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(v, e1)
        ang = np.linspace(0, 2 * math.pi, 96, endpoint=False)
        rho = 1e-4
        for c in range(v.shape[0]):
            pts = v[c][None, :] + rho * (np.cos(ang)[:, None] * e1[c] + np.sin(ang)[:, None] * e2[c])
            pts /= np.linalg.norm(pts, axis=1, keepdims=True)
            cells = np.unique(hp.radec2pix(nside, np.arctan2(pts[:, 1], pts[:, 0]), np.arcsin(pts[:, 2])))
            for x in cells:
                nb[x].update(int(y) for y in cells if y != x)
    return nb


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_neighbours_equal_brute_force(nside):
    nb = hp.neighbours(nside, np.arange(hp.npix(nside)))
    brute = _brute_neighbours(nside)
    for p in range(hp.npix(nside)):
        got = [int(q) for q in nb[p] if q >= 0]
        assert len(got) == len(set(got)) and set(got) == brute[p], (nside, p, sorted(got), sorted(brute[p]))
    if nside >= 2:  # eight neighbours, seven at the 24 pixels touching a three-face corner
        cnt = (nb >= 0).sum(1)
        assert np.sum(cnt == 7) == 24 and np.sum(cnt == 8) == hp.npix(nside) - 24


def test_neighbours_in_the_belt_follow_the_ring_lattice():
    """Away from the caps the grid is a regular lattice in (phi, z): the
    neighbours are the pixels one and two rings away at the expected
    azimuths (an independent index rule)."""
    N = 64
    rt = hp.ring_table(N)
    rng = np.random.default_rng(2)
    for _ in range(200):
        i = int(rng.integers(N + 3, 3 * N - 2))  # ring, 1-based
        j = int(rng.integers(0, 4 * N))
        p = rt["first"][i - 1] + j
        shifted = (i - N) % 2 == 0
        up = [j, j + 1] if shifted else [j - 1, j]  # ring i-1 has the other shift
        want = {rt["first"][i - 1] + (j - 1) % (4 * N), rt["first"][i - 1] + (j + 1) % (4 * N),
                rt["first"][i - 3] + j, rt["first"][i + 1] + j}
        want |= {rt["first"][i - 2] + q % (4 * N) for q in up} | {rt["first"][i] + q % (4 * N) for q in up}
        got = set(int(q) for q in hp.neighbours(N, np.array([p]))[0])
        assert got == want
