"""Pins of the oracle's HEALPix RING geometry (oracle/healpix_ref.py)."""
import math
import os

import numpy as np
import pytest

from oracle import healpix_ref as hp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 64, 1024, 4096])
def test_ring_counts_sum(nside):
    rt = hp.ring_table(nside)
    assert rt["n"].sum() == 12 * nside * nside
    # first pixels are the running sum of the ring sizes
    assert np.array_equal(rt["first"][1:], np.cumsum(rt["n"])[:-1])
    assert rt["first"][0] == 0


def test_golden_base_centres():
    """Centres fixed by the construction for NSIDE 1 and 2 (tests/golden)."""
    data = np.loadtxt(os.path.join(GOLDEN, "healpix_centres.txt"), comments="#")
    for nside, pix, z, phi_over_pi in data:
        zz, s, phi = hp.pix2zphi(int(nside), np.array([int(pix)]))
        assert abs(zz[0] - z) < 1e-15
        assert abs(phi[0] / math.pi - phi_over_pi) < 1e-15


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 64])
def test_roundtrip_all(nside):
    p = np.arange(hp.npix(nside))
    ra, dec = hp.pix2radec(nside, p)
    assert np.array_equal(hp.radec2pix(nside, ra, dec), p)


@pytest.mark.parametrize("nside", [4096, 8192, 16384])
def test_roundtrip_random(nside):
    rng = np.random.default_rng(nside)
    p = rng.integers(0, hp.npix(nside), 200000)
    # rings near the poles and the cap/belt seams
    extra = np.concatenate([np.arange(40), hp.npix(nside) - 1 - np.arange(40),
                            2 * nside * (nside - 1) + np.arange(-20, 20),
                            hp.npix(nside) - 2 * nside * (nside - 1) + np.arange(-20, 20)])
    p = np.concatenate([p, extra])
    ra, dec = hp.pix2radec(nside, p)
    assert np.array_equal(hp.radec2pix(nside, ra, dec), p)


@pytest.mark.parametrize("nside", [2, 16])
def test_equal_area_chi2(nside):
    """Uniform points fill the 12 N^2 pixels equally (equal-area scheme)."""
    rng = np.random.default_rng(7)
    n = 400 * hp.npix(nside)
    ra = rng.uniform(0, 2 * math.pi, n)
    dec = np.arcsin(rng.uniform(-1, 1, n))
    c = np.bincount(hp.radec2pix(nside, ra, dec), minlength=hp.npix(nside))
    exp = n / hp.npix(nside)
    chi2 = ((c - exp) ** 2 / exp).sum()
    dof = hp.npix(nside) - 1
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof)


@pytest.mark.parametrize("nside", [4, 32])
def test_belt_cells_are_diamonds(nside):
    """In the equatorial belt each cell is the (phi, z) diamond
    |phi - phi_c| / (pi/(4N)) + |z - z_c| / (2/(3N)) < 1 around its centre."""
    rng = np.random.default_rng(3)
    n = 200000
    lim = 2.0 / 3.0 - 2.0 / (3.0 * nside)
    z = rng.uniform(-lim, lim, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    pix = hp.radec2pix(nside, phi, np.arcsin(z))
    zc, _, phic = hp.pix2zphi(nside, pix)
    dphi = np.abs(np.mod(phi - phic + math.pi, 2 * math.pi) - math.pi)
    lhs = dphi / (math.pi / (4 * nside)) + np.abs(z - zc) / (2.0 / (3.0 * nside))
    assert np.all(lhs <= 1.0 + 1e-9)


def test_cap_cells_contain_centre_neighbourhood():
    """Points very close to a cap centre fall in that pixel, and every point
    lies within the largest cell radius of its centre."""
    nside = 64
    rng = np.random.default_rng(4)
    p = rng.integers(0, 2 * nside * (nside - 1), 2000)
    ra, dec = hp.pix2radec(nside, p)
    eps = 1e-3 * math.sqrt(math.pi / 3) / nside
    assert np.array_equal(hp.radec2pix(nside, ra + eps * rng.uniform(-1, 1, p.size) / np.cos(dec),
                                       dec + eps * rng.uniform(-1, 1, p.size)), p)
    n = 100000
    ra = rng.uniform(0, 2 * math.pi, n)
    dec = np.arcsin(rng.uniform(2 / 3, 1, n))
    pix = hp.radec2pix(nside, ra, dec)
    v = np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], -1)
    d = np.arccos(np.clip((v * hp.pix2vec(nside, pix)).sum(1), -1, 1))
    assert d.max() < 2.0 * math.sqrt(math.pi / 3) / nside


def test_disc_brute_size():
    """Disc sizes approach the cap area over the pixel area."""
    nside = 256
    r = 3 * math.pi / 180
    v = hp.pix2vec(nside, np.array([323456]))[0]
    n = hp.disc_brute(nside, v, r).size
    expect = 2 * math.pi * (1 - math.cos(r)) / (4 * math.pi / hp.npix(nside))
    assert abs(n - expect) / expect < 0.02
