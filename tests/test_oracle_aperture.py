"""Pins of the oracle's aperture sums and maps (oracle/aperture.py).

Each test fixes the oracle against something other than itself:
  * a 50-digit mpmath all-pairs brute force that builds the tangential
    projection from tangent-plane vectors (not from the polar-angle formula);
  * hand-derived sign conventions;
  * the closed-form aperture mass of a singular isothermal sphere, integrated
    by mpmath quadrature, against a catalogue laid on quadrature nodes;
  * identities: B-mode nulling, E<->B duality, linearity, HEALPix symmetries,
    pixel variant == galaxy variant on pixel centres;
  * shape-noise statistics.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import aperture as A
from oracle import filters as F
from oracle import healpix_ref as hp
from synth import small_catalogue

DEG = math.pi / 180
ARCMIN = DEG / 60


# ----------------------------------------------------------------------------
# helpers written independently of the oracle
# ----------------------------------------------------------------------------

def _mp_vec(ra, dec):
    return [mp.cos(dec) * mp.cos(ra), mp.cos(dec) * mp.sin(ra), mp.sin(dec)]


def _mp_q(kind, x):
    if x >= 1:
        return mp.mpf(0)
    if kind == F.POLY:
        return 6 / mp.pi * x * x * (1 - x * x)
    t = x / mp.mpf("0.15")
    r = mp.mpf(1) if t == 0 else mp.tanh(t) / t
    return r / (1 + mp.exp(6 - 150 * x) + mp.exp(-47 + 50 * x))


def mp_brute(cat, c_ra, c_dec, theta_ap, kind):
    """All-pairs sums at 50 digits. The tangential shear is read off the
    tangent plane of each galaxy: with d = r_centre - r_gal, x = d.e_East,
    y = d.e_North, the bearing towards the centre is beta = atan2(x, y) and
    a tangential shear pattern g = g_t exp(-2 i beta) must give g+ = g_t:
    g+ = g1 cos 2beta - g2 sin 2beta, gx = g1 sin 2beta + g2 cos 2beta."""
    mp.mp.dps = 50
    th = mp.mpf(theta_ap)
    C = 4 * mp.sin(th / 2) ** 2
    out = np.zeros((len(c_ra), 5))
    gv = [_mp_vec(mp.mpf(a), mp.mpf(d)) for a, d in zip(cat["ra"], cat["dec"])]
    for k, (ca, cd) in enumerate(zip(c_ra, c_dec)):
        rc = _mp_vec(mp.mpf(ca), mp.mpf(cd))
        SE = SB = W = V = N = mp.mpf(0)
        for i, r in enumerate(gv):
            d = [rc[0] - r[0], rc[1] - r[1], rc[2] - r[2]]
            c2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
            if not c2 < C:
                continue
            a = mp.mpf(cat["ra"][i])
            de = mp.mpf(cat["dec"][i])
            w = mp.mpf(float(cat["w"][i]))
            g1 = mp.mpf(float(cat["g1"][i]))
            g2 = mp.mpf(float(cat["g2"][i]))
            theta = 2 * mp.asin(mp.sqrt(c2) / 2)
            q = _mp_q(kind, theta / th)
            if c2 == 0:
                gp = gx = mp.mpf(0)
            else:
                eE = [-mp.sin(a), mp.cos(a), 0]
                eN = [-mp.sin(de) * mp.cos(a), -mp.sin(de) * mp.sin(a), mp.cos(de)]
                x = sum(d[j] * eE[j] for j in range(3))
                y = sum(d[j] * eN[j] for j in range(3))
                b = mp.atan2(x, y)
                gp = g1 * mp.cos(2 * b) - g2 * mp.sin(2 * b)
                gx = g1 * mp.sin(2 * b) + g2 * mp.cos(2 * b)
            SE += w * q * gp
            SB += w * q * gx
            W += w
            V += w * w * (g1 * g1 + g2 * g2) * q * q
            N += 1
        out[k] = [float(SE), float(SB), float(W), float(V), float(N)]
    return out


def _dest(ra0, dec0, theta, bearing):
    """Point at great-circle distance theta along the initial bearing
    (North through East) from (ra0, dec0), by rotating in the tangent frame."""
    r0 = np.array([math.cos(dec0) * math.cos(ra0), math.cos(dec0) * math.sin(ra0), math.sin(dec0)])
    eE = np.array([-math.sin(ra0), math.cos(ra0), 0.0])
    eN = np.array([-math.sin(dec0) * math.cos(ra0), -math.sin(dec0) * math.sin(ra0), math.cos(dec0)])
    t = np.cos(bearing)[:, None] * eN + np.sin(bearing)[:, None] * eE
    r = np.cos(theta)[:, None] * r0 + np.sin(theta)[:, None] * t
    return np.mod(np.arctan2(r[:, 1], r[:, 0]), 2 * math.pi), np.arcsin(np.clip(r[:, 2], -1, 1))


def _tangential(ra, dec, ra0, dec0, gt):
    """Shear of amplitude gt oriented tangentially about (ra0, dec0), from
    tangent-plane vectors at each galaxy."""
    r0 = np.array([math.cos(dec0) * math.cos(ra0), math.cos(dec0) * math.sin(ra0), math.sin(dec0)])
    r = np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], -1)
    t = r0[None, :] - (r @ r0)[:, None] * r
    eE = np.stack([-np.sin(ra), np.cos(ra), np.zeros_like(ra)], -1)
    eN = np.stack([-np.sin(dec) * np.cos(ra), -np.sin(dec) * np.sin(ra), np.cos(dec)], -1)
    b = np.arctan2((t * eE).sum(1), (t * eN).sum(1))
    return gt * np.cos(2 * b), -gt * np.sin(2 * b)


def _raw(cat, c_ra, c_dec, th, kind):
    src = A.galaxy_sources(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"])
    s = A.sums_kdtree(src, np.asarray(c_ra), np.asarray(c_dec), th, F.q_of(kind))
    return np.stack([s["S_E"], s["S_B"], s["W"], s["V"], s["N"]], 1), s


# ----------------------------------------------------------------------------
# P1: brute force at 50 digits
# ----------------------------------------------------------------------------

SCENARIOS = [
    # (name, centre of the catalogue cap, cap radius, theta_ap, filter)
    ("midlat_poly_5deg", (1.0, 0.5), 9 * DEG, 5 * DEG, F.POLY),
    ("pole_tanh_30deg", (0.3, 85 * DEG), 40 * DEG, 30 * DEG, F.TANH),
    ("rawrap_tanh_5deg", (0.0, 0.0), 8 * DEG, 5 * DEG, F.TANH),
    ("south_poly_30deg", (4.0, -60 * DEG), 35 * DEG, 30 * DEG, F.POLY),
]


@pytest.mark.parametrize("name,centre,capr,th,kind", SCENARIOS)
def test_mp_bruteforce(name, centre, capr, th, kind):
    cat = small_catalogue(220, seed=hash(name) % 1000, cap_radius=capr, centre=centre)
    rng = np.random.default_rng(1)
    sub = small_catalogue(6, seed=11, cap_radius=capr * 0.7, centre=centre, signal=False)
    c_ra = np.concatenate([sub["ra"], cat["ra"][:2]])   # two centres sit on galaxies
    c_dec = np.concatenate([sub["dec"], cat["dec"][:2]])
    if name.startswith("pole"):
        c_ra = np.append(c_ra, 1.234)
        c_dec = np.append(c_dec, math.pi / 2)            # centre exactly at the pole
    got, s = _raw(cat, c_ra, c_dec, th, kind)
    assert not s["tie"].any()
    ref = mp_brute(cat, c_ra, c_dec, th, kind)
    assert ref[:, 4].min() > 5
    for col in range(5):
        scale = np.sqrt(np.mean(ref[:, col] ** 2)) + 1e-300
        assert np.max(np.abs(got[:, col] - ref[:, col])) <= 1e-12 * scale, (name, col)
    del rng


def test_sign_convention_by_hand():
    """g1 = 1 at a galaxy due East of the centre is radial (E-W elongation)
    and gives g+ = -1; due North it is tangential and gives g+ = +1; at the
    North-East diagonal g2 = 1 is radial and gives g+ = -1."""
    ra0, dec0 = 1.0, 0.2
    d = 1 * DEG
    cases = [
        (ra0 + d / math.cos(dec0), dec0, 1.0, 0.0, -1.0),
        (ra0, dec0 + d, 1.0, 0.0, +1.0),
    ]
    for ra, dec, g1, g2, expect in cases:
        psi = A.polar_angle(np.array([ra]), np.array([dec]), ra0, dec0)
        gp, gx = A.tangential_cross(np.array([g1]), np.array([g2]), psi)
        assert abs(gp[0] - expect) < 2e-2
    # diagonal, near the equator where the frame is nearly flat
    ra, dec = 0.01 * DEG, 0.01 * DEG
    psi = A.polar_angle(np.array([ra]), np.array([dec]), 0.0, 0.0)
    gp, _ = A.tangential_cross(np.array([0.0]), np.array([1.0]), psi)
    assert abs(gp[0] + 1.0) < 1e-6


# ----------------------------------------------------------------------------
# P2/P3: closed-form SIS aperture mass on a quadrature catalogue
# ----------------------------------------------------------------------------

def _gl_catalogue(ra0, dec0, th, breaks, nodes, n_az, theta_e):
    xs, ws = np.polynomial.legendre.leggauss(nodes)
    radii, rw = [], []
    for a, b in zip(breaks[:-1], breaks[1:]):
        radii.append(0.5 * (b - a) * xs + 0.5 * (a + b))
        rw.append(0.5 * (b - a) * ws)
    radii = np.concatenate(radii) * th
    rw = np.concatenate(rw) * th
    az = 2 * math.pi * (np.arange(n_az) + 0.5) / n_az
    R, B = np.meshgrid(radii, az, indexing="ij")
    Wt = (rw * np.sin(radii))[:, None] * np.full((1, n_az), 2 * math.pi / n_az)
    ra, dec = _dest(ra0, dec0, R.ravel(), B.ravel())
    gt = theta_e / (2 * R.ravel())
    g1, g2 = _tangential(ra, dec, ra0, dec0, gt)
    return {"ra": ra, "dec": dec, "g1": g1, "g2": g2, "w": Wt.ravel()}


@pytest.mark.parametrize("kind,th", [(F.POLY, 2 * DEG), (F.TANH, 10 * ARCMIN), (F.POLY, 20 * DEG)])
def test_sis_closed_form(kind, th):
    ra0, dec0 = 0.7, 0.4
    theta_e = 2.0 * ARCMIN
    if kind == F.POLY:
        breaks = [0.0, 1.0]
        nodes = 24
    else:
        breaks = [0.0, 0.02, 0.03, 0.036, 0.04, 0.044, 0.05, 0.06, 0.08, 0.12, 0.2, 0.35, 0.6, 0.85, 1.0]
        nodes = 24
    cat = _gl_catalogue(ra0, dec0, th, breaks, nodes, 48, theta_e)
    # galaxies built exactly at the aperture edge are impossible (open interval)
    out = A.aperture_mass_galaxy(cat, np.array([ra0]), np.array([dec0]), th, kind, A.NORM_SUMMED_CAP)
    assert not out["tie"].any()
    mp.mp.dps = 30
    tt = mp.mpf(th)
    f = lambda t: (mp.mpf(theta_e) / (2 * t)) * _mp_q(kind, t / tt) * mp.sin(t)
    pts = [mp.mpf(b) * tt for b in breaks]
    ref = 2 * mp.pi * mp.quad(f, pts) / tt ** 2
    assert abs(out["W"][0] - 4 * math.pi * math.sin(th / 2) ** 2) < 1e-13 * out["W"][0]
    assert abs(out["M_E"][0] - float(ref)) < 1e-11 * abs(float(ref))
    assert abs(out["M_B"][0]) < 1e-13 * abs(float(ref))


def test_b_nulling_random_tangential():
    rng = np.random.default_rng(5)
    ra0, dec0 = 2.0, -0.3
    n = 5000
    th = 3 * DEG
    ra, dec = _dest(ra0, dec0, np.sqrt(rng.uniform(0, 1, n)) * th * 1.2, rng.uniform(0, 2 * math.pi, n))
    g1, g2 = _tangential(ra, dec, ra0, dec0, rng.uniform(-0.3, 0.3, n))
    cat = {"ra": ra, "dec": dec, "g1": g1, "g2": g2, "w": rng.uniform(0.5, 2, n)}
    got, _ = _raw(cat, [ra0], [dec0], th, F.TANH)
    assert abs(got[0, 1]) < 1e-13 * np.sum(np.abs(g1) + np.abs(g2))


# ----------------------------------------------------------------------------
# P4/P5: duality and linearity
# ----------------------------------------------------------------------------

def _rand_cat(seed, n=4000):
    return small_catalogue(n, seed=seed, cap_radius=6 * DEG, centre=(3.0, -0.4))


def test_eb_duality_and_linearity():
    c = _rand_cat(1)
    c2 = _rand_cat(2)
    c2 = dict(c2, ra=c["ra"], dec=c["dec"], w=c["w"])
    cen = small_catalogue(50, seed=3, cap_radius=4 * DEG, centre=(3.0, -0.4), signal=False)
    th = 1.5 * DEG
    a, _ = _raw(c, cen["ra"], cen["dec"], th, F.TANH)
    rot = dict(c, g1=c["g2"], g2=-c["g1"])
    b, _ = _raw(rot, cen["ra"], cen["dec"], th, F.TANH)
    sc = np.abs(a[:, :2]).max()
    assert np.max(np.abs(b[:, 0] - a[:, 1])) < 1e-12 * sc
    assert np.max(np.abs(b[:, 1] + a[:, 0])) < 1e-12 * sc
    al, be = 0.7, -1.9
    f64 = lambda v: np.asarray(v, np.float64)
    lin = dict(c, g1=al * f64(c["g1"]) + be * f64(c2["g1"]), g2=al * f64(c["g2"]) + be * f64(c2["g2"]))
    d, _ = _raw(lin, cen["ra"], cen["dec"], th, F.TANH)
    e, _ = _raw(c2, cen["ra"], cen["dec"], th, F.TANH)
    for col in (0, 1):
        assert np.max(np.abs(d[:, col] - (al * a[:, col] + be * e[:, col]))) < 1e-12 * sc
    assert np.array_equal(d[:, 2], a[:, 2]) and np.array_equal(d[:, 4], a[:, 4])


# ----------------------------------------------------------------------------
# P6/P7: pixel variant: HEALPix symmetries, equality with the galaxy variant
# ----------------------------------------------------------------------------

def _rand_pixmap(nside, seed):
    rng = np.random.default_rng(seed)
    pix = np.arange(hp.npix(nside))
    W = rng.poisson(20, pix.size).astype(np.float64)
    W[rng.uniform(size=pix.size) < 0.05] = 0.0
    G1 = np.where(W > 0, rng.normal(0, 1, pix.size) * np.sqrt(W), 0.0)
    G2 = np.where(W > 0, rng.normal(0, 1, pix.size) * np.sqrt(W), 0.0)
    E2 = np.where(W > 0, W * 0.135 + G1 * G1 * 0.01, 0.0)
    return {"nside": nside, "pix": pix, "W": W, "G1": G1, "G2": G2, "E2": E2}


def _rot90(nside, pix):
    ring, j = hp.pix2ring(nside, pix)
    rt = hp.ring_table(nside)
    n = rt["n"][ring - 1]
    return rt["first"][ring - 1] + np.mod(j + n // 4, n)


def _mirror(nside, pix):
    ring, j = hp.pix2ring(nside, pix)
    rt = hp.ring_table(nside)
    return rt["first"][4 * nside - ring - 1] + j


@pytest.mark.parametrize("kind,th", [(F.TANH, 4 * DEG), (F.POLY, 9 * DEG)])
def test_pixel_symmetries(kind, th):
    nside = 16
    m = _rand_pixmap(nside, 9)
    rng = np.random.default_rng(2)
    out = rng.choice(hp.npix(nside), 300, replace=False)
    base = A.aperture_mass_pixel(m, out, th, kind)
    # (i) azimuthal quarter turn maps the grid onto itself; values follow pixels
    m1 = dict(m, pix=_rot90(nside, m["pix"]))
    r1 = A.aperture_mass_pixel(m1, _rot90(nside, out), th, kind)
    # (ii) reflection through the equator: g2 flips, E even, B odd
    m2 = dict(m, pix=_mirror(nside, m["pix"]), G2=-m["G2"])
    r2 = A.aperture_mass_pixel(m2, _mirror(nside, out), th, kind)
    ok = ~(base["tie"] | r1["tie"] | r2["tie"])
    assert ok.sum() > 250
    sc = np.sqrt(np.mean(base["M_E"][ok] ** 2))
    for k in ("M_E", "M_B", "sigma", "W", "N"):
        assert np.max(np.abs(r1[k][ok] - base[k][ok])) < 1e-12 * max(sc, np.abs(base[k]).max()), k
    assert np.max(np.abs(r2["M_E"][ok] - base["M_E"][ok])) < 1e-12 * sc
    assert np.max(np.abs(r2["M_B"][ok] + base["M_B"][ok])) < 1e-12 * sc


def test_pixel_equals_galaxy_on_centres():
    nside = 32
    m = _rand_pixmap(nside, 4)
    m["W"] = np.maximum(m["W"], 1.0)
    m["E2"] = m["G1"] ** 2 + m["G2"] ** 2
    out = np.random.default_rng(0).choice(hp.npix(nside), 200, replace=False)
    th = 5 * DEG
    p = A.aperture_mass_pixel(m, out, th, F.TANH, norm=A.NORM_RAW)
    ra, dec = hp.pix2radec(nside, m["pix"])
    cat = {"ra": ra, "dec": dec, "g1": m["G1"] / m["W"], "g2": m["G2"] / m["W"], "w": m["W"]}
    cra, cdec = hp.pix2radec(nside, out)
    g = A.aperture_mass_galaxy(cat, cra, cdec, th, F.TANH, norm=A.NORM_RAW)
    for k in ("M_E", "M_B", "sigma", "W", "N"):
        sc = np.abs(g[k]).max()
        assert np.max(np.abs(p[k] - g[k])) < 1e-12 * sc, k


# ----------------------------------------------------------------------------
# Averaged normalisation (Sect. 2.4): three routes that do not use the
# pixel-level weighting of the oracle
# ----------------------------------------------------------------------------

def test_averaged_equals_galaxy_variant_with_pixel_density_weights():
    """Galaxy by galaxy, the averaged approach divides each galaxy's filtered
    shear by the effective density of its pixel, n_j = (galaxies in pixel j) /
    Omega_pix: a galaxy-variant sum with weights w_i = Omega_pix / n_gal(j)
    over galaxies placed at their pixel centres, divided by theta_ap^2.
    A wrong power of the weight in the variance or a weight taken from the
    wrong pixel fails here."""
    nside = 32
    rng = np.random.default_rng(21)
    pix = np.arange(hp.npix(nside))
    ngal = rng.poisson(2.0, pix.size)          # about 13% of the pixels are empty
    gpix = np.repeat(pix, ngal)
    g1 = rng.normal(0, 0.3, gpix.size) + 0.05
    g2 = rng.normal(0, 0.3, gpix.size)
    omega = 4 * math.pi / hp.npix(nside)
    ra, dec = hp.pix2radec(nside, gpix)
    cat = {"ra": ra, "dec": dec, "g1": g1, "g2": g2, "w": omega / ngal[gpix]}
    m = {"nside": nside, "pix": pix, "W": ngal.astype(np.float64),
         "G1": np.bincount(gpix, g1, pix.size), "G2": np.bincount(gpix, g2, pix.size),
         "E2": np.bincount(gpix, g1 * g1 + g2 * g2, pix.size)}
    out = np.concatenate([np.arange(0, 20), rng.choice(hp.npix(nside), 150, replace=False)])
    cra, cdec = hp.pix2radec(nside, out)
    for th, kind in [(5 * DEG, F.TANH), (12 * DEG, F.POLY)]:
        a = A.aperture_mass_pixel(m, out, th, kind, norm=A.NORM_AVERAGED)
        g = A.aperture_mass_galaxy(cat, cra, cdec, th, kind, norm=A.NORM_RAW)
        ok = ~(a["tie"] | g["tie"])
        assert ok.sum() > 100
        ref = {"M_E": g["M_E"] / th ** 2, "M_B": g["M_B"] / th ** 2,
               "sigma": np.sqrt(0.5 * g["sigma"]) / th ** 2}   # RAW: the sigma channel is V
        for k in ("M_E", "M_B", "sigma"):
            sc = np.abs(ref[k][ok]).max()
            assert np.max(np.abs(a[k][ok] - ref[k][ok])) < 1e-12 * sc, k
        assert np.array_equal(a["W"], A.aperture_mass_pixel(m, out, th, kind)["W"])


def test_averaged_equals_summed_with_one_galaxy_per_pixel():
    """With one galaxy in every occupied pixel the density of each pixel,
    1 / Omega_pix, is also the aperture's mean density N / (N Omega_pix), so
    the averaged maps equal the summed pixel-count maps."""
    nside = 64
    rng = np.random.default_rng(22)
    pix = np.arange(hp.npix(nside))
    W = (rng.uniform(size=pix.size) < 0.7).astype(np.float64)
    G1 = W * rng.normal(0, 0.3, pix.size)
    G2 = W * rng.normal(0, 0.3, pix.size)
    m = {"nside": nside, "pix": pix, "W": W, "G1": G1, "G2": G2, "E2": G1 * G1 + G2 * G2}
    out = rng.choice(hp.npix(nside), 200, replace=False)
    th = 4 * DEG
    a = A.aperture_mass_pixel(m, out, th, F.TANH, norm=A.NORM_AVERAGED)
    b = A.aperture_mass_pixel(m, out, th, F.TANH, norm=A.NORM_SUMMED_PIXCOUNT)
    ok = ~a["tie"]
    for k in ("M_E", "M_B", "sigma", "W", "N"):
        sc = np.abs(b[k][ok]).max()
        assert np.max(np.abs(a[k][ok] - b[k][ok])) < 1e-12 * sc, k


def test_averaged_unchanged_when_galaxies_repeat():
    """Repeating every galaxy of pixel j k_j times multiplies the pixel's G, W
    and E2 by k_j: its mean shear, and so the averaged M_E and M_B, stay as
    they are (the summed maps move), while the variance term of the pixel
    scales by 1 / k_j."""
    nside = 32
    m = _rand_pixmap(nside, 23)
    rng = np.random.default_rng(24)
    k = rng.integers(1, 5, m["pix"].size).astype(np.float64)
    m2 = dict(m, W=m["W"] * k, G1=m["G1"] * k, G2=m["G2"] * k, E2=m["E2"] * k)
    out = rng.choice(hp.npix(nside), 150, replace=False)
    th = 8 * DEG
    a = A.aperture_mass_pixel(m, out, th, F.TANH, norm=A.NORM_AVERAGED)
    b = A.aperture_mass_pixel(m2, out, th, F.TANH, norm=A.NORM_AVERAGED)
    ok = ~a["tie"]
    for key in ("M_E", "M_B"):
        sc = np.abs(a[key][ok]).max()
        assert np.max(np.abs(a[key][ok] - b[key][ok])) < 1e-12 * sc, key
    s1 = A.aperture_mass_pixel(m, out, th, F.TANH)
    s2 = A.aperture_mass_pixel(m2, out, th, F.TANH)
    assert np.max(np.abs(s1["M_E"][ok] - s2["M_E"][ok])) > 1e-3 * np.abs(s1["M_E"][ok]).max()
    # uniform repetition: sigma scales by 1 / sqrt(k)
    m3 = dict(m, W=m["W"] * 4, G1=m["G1"] * 4, G2=m["G2"] * 4, E2=m["E2"] * 4)
    c = A.aperture_mass_pixel(m3, out, th, F.TANH, norm=A.NORM_AVERAGED)
    assert np.max(np.abs(c["sigma"][ok] - 0.5 * a["sigma"][ok])) < 1e-12 * np.abs(a["sigma"][ok]).max()


@pytest.mark.parametrize("nside,th", [(32, 6 * DEG), (64, 30 * DEG), (8, 50 * DEG)])
def test_ring_candidates_match_kdtree(nside, th):
    m = _rand_pixmap(nside, 1)
    keep = np.random.default_rng(5).uniform(size=m["pix"].size) < 0.7   # a sparse map
    m = {k: (v[keep] if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    out = np.concatenate([np.arange(0, 30), hp.npix(nside) - 1 - np.arange(30),
                          np.random.default_rng(6).choice(hp.npix(nside), 100, replace=False)])
    a = A.aperture_mass_pixel(m, out, th, F.POLY, candidates="rings")
    b = A.aperture_mass_pixel(m, out, th, F.POLY, candidates="kdtree")
    assert a["pairs"] == b["pairs"]
    for k in ("M_E", "M_B", "sigma", "W", "N"):
        assert np.max(np.abs(a[k] - b[k])) <= 1e-12 * (np.abs(b[k]).max() + 1e-300), k


# ----------------------------------------------------------------------------
# P9: shape-noise realisations
# ----------------------------------------------------------------------------

def test_noise_realisations_statistics():
    """Rotating each pixel sum by a uniform spin-2 phase leaves W and V alone;
    over realisations the mean of M_E vanishes and its variance equals
    sigma^2 computed with E2 = |G|^2 (Eq. map_noise)."""
    nside = 16
    m = _rand_pixmap(nside, 8)
    m["E2"] = m["G1"] ** 2 + m["G2"] ** 2
    out = np.arange(0, hp.npix(nside), 37)
    th = 8 * DEG
    base = A.aperture_mass_pixel(m, out, th, F.POLY)
    R = 400
    acc = np.zeros((R, out.size))
    for r in range(R):
        u = np.random.default_rng([17, r]).random(m["pix"].size, dtype=np.float32)
        G1, G2 = A.rotate_realisation(m["G1"], m["G2"], u)
        mr = dict(m, G1=G1, G2=G2, E2=G1 ** 2 + G2 ** 2)
        o = A.aperture_mass_pixel(mr, out, th, F.POLY)
        assert np.allclose(o["sigma"], base["sigma"], rtol=1e-12)
        acc[r] = o["M_E"]
    var = acc.var(0)
    ratio = var / base["sigma"] ** 2
    assert abs(ratio.mean() - 1.0) < 4 * math.sqrt(2.0 / R) / math.sqrt(out.size) + 0.01
    assert np.abs(acc.mean(0)).mean() < 4 * base["sigma"].mean() / math.sqrt(R)


# ----------------------------------------------------------------------------
# Galaxy-level shape-noise realisations (random orientation of every galaxy)
# ----------------------------------------------------------------------------

def _gal_cat(n, seed, cap=10 * DEG):
    rng = np.random.default_rng(seed)
    ra = rng.uniform(-cap, cap, n) % (2 * math.pi)
    dec = rng.uniform(-cap, cap, n)
    return {"ra": ra, "dec": dec, "g1": rng.normal(0, 0.3, n) + 0.05, "g2": rng.normal(0, 0.3, n),
            "w": rng.uniform(0.5, 1.5, n)}


def test_galaxy_realisations_quarter_turns_and_statistics():
    """Exact identities of the spin-2 phase: u + 1/2 negates the E and B maps,
    and the four quarter-turn shifts of any u sum to zero. Over independent
    uniform angles the mean of M_E vanishes and its variance is sigma^2 of
    Eq. map_noise (the expectation of cos^2 of a uniform angle is 1/2)."""
    cat = _gal_cat(3000, 31)
    rng = np.random.default_rng(32)
    c_ra = rng.uniform(-5 * DEG, 5 * DEG, 40) % (2 * math.pi)
    c_dec = rng.uniform(-5 * DEG, 5 * DEG, 40)
    th = 3 * DEG
    u = rng.random(3000)
    maps = [A.aperture_mass_galaxy(A.rotate_galaxies(cat, (u + k / 4) % 1.0), c_ra, c_dec, th, F.TANH)
            for k in range(4)]
    sc = np.abs(maps[0]["M_E"]).max()
    for key in ("M_E", "M_B"):
        assert np.max(np.abs(maps[2][key] + maps[0][key])) < 1e-12 * sc
        assert np.max(np.abs(sum(mp[key] for mp in maps))) < 1e-12 * sc
    base = A.aperture_mass_galaxy(cat, c_ra, c_dec, th, F.TANH)
    assert np.allclose(maps[1]["sigma"], base["sigma"], rtol=1e-12)
    R = 300
    acc = np.array([A.aperture_mass_galaxy(A.rotate_galaxies(cat, np.random.default_rng([33, r]).random(3000)),
                                           c_ra, c_dec, th, F.TANH)["M_E"] for r in range(R)])
    ratio = acc.var(0) / base["sigma"] ** 2
    assert abs(ratio.mean() - 1.0) < 4 * math.sqrt(2.0 / R) / math.sqrt(c_ra.size) + 0.01
    assert np.abs(acc.mean(0)).mean() < 4 * base["sigma"].mean() / math.sqrt(R)


def test_galaxy_realisation_binned_equals_pixel_realisation_at_one_galaxy_per_pixel():
    """With one galaxy in each occupied pixel, rotating the galaxies and
    binning them again gives the pixel sums rotated by the same angles: the
    galaxy-level realisation of the pixel variant equals the pixel-level one."""
    from oracle import binning as B

    nside = 64
    rng = np.random.default_rng(34)
    pix = np.sort(rng.choice(hp.npix(nside), 20000, replace=False))
    ra, dec = hp.pix2radec(nside, pix)
    cat = {"ra": ra, "dec": dec, "g1": rng.normal(0, 0.3, pix.size), "g2": rng.normal(0, 0.3, pix.size),
           "w": np.ones(pix.size)}
    u = rng.random(pix.size)
    out = rng.choice(hp.npix(nside), 150, replace=False)
    th = 4 * DEG
    rc = A.rotate_galaxies(cat, u)
    p_u, W, G1, G2, E2 = B.pixel_sums(nside, rc["ra"], rc["dec"], rc["g1"], rc["g2"], rc["w"])
    assert np.array_equal(p_u, pix)
    a = A.aperture_mass_pixel({"nside": nside, "pix": p_u, "W": W, "G1": G1, "G2": G2, "E2": E2}, out, th, F.TANH)
    H1, H2 = A.rotate_realisation(cat["g1"], cat["g2"], u)
    b = A.aperture_mass_pixel({"nside": nside, "pix": pix, "W": np.ones(pix.size), "G1": H1, "G2": H2,
                               "E2": cat["g1"] ** 2 + cat["g2"] ** 2}, out, th, F.TANH)
    ok = ~a["tie"]
    for key in ("M_E", "M_B", "sigma", "W", "N"):
        sc = np.abs(b[key][ok]).max()
        assert np.max(np.abs(a[key][ok] - b[key][ok])) < 1e-12 * sc, key


# ----------------------------------------------------------------------------
# sphS_pixB: pixel sums at the barycentre of their galaxies (Sect. 3.3)
# ----------------------------------------------------------------------------

def test_barycentre_one_galaxy_per_pixel_is_the_brute_force():
    """A pixel holding one galaxy has that galaxy as its barycentre and its
    sums as its values: pixB equals the galaxy variant."""
    nside = 64
    rng = np.random.default_rng(41)
    pix = np.sort(rng.choice(hp.npix(nside), 8000, replace=False))
    c = hp.pix2vec(nside, pix)
    # one galaxy inside each pixel, off its centre
    t = np.cross(c, rng.normal(size=c.shape))
    t /= np.linalg.norm(t, axis=1)[:, None]
    v = c + 0.2 * math.sqrt(4 * math.pi / hp.npix(nside)) * t
    v /= np.linalg.norm(v, axis=1)[:, None]
    ra = np.arctan2(v[:, 1], v[:, 0]) % (2 * math.pi)
    dec = np.arcsin(np.clip(v[:, 2], -1, 1))
    assert np.array_equal(np.sort(hp.radec2pix(nside, ra, dec)), pix)
    cat = {"ra": ra, "dec": dec, "g1": rng.normal(0, 0.3, pix.size), "g2": rng.normal(0, 0.3, pix.size),
           "w": rng.uniform(0.5, 1.5, pix.size)}
    out = rng.choice(hp.npix(nside), 200, replace=False)
    c_ra, c_dec = hp.pix2radec(nside, out)
    th = 4 * DEG
    a = A.aperture_mass_barycentre(cat, nside, c_ra, c_dec, th, F.TANH, norm=A.NORM_SUMMED_CAP)
    g = A.aperture_mass_galaxy(cat, c_ra, c_dec, th, F.TANH, norm=A.NORM_SUMMED_CAP)
    ok = ~(a["tie"] | g["tie"])
    for key in ("M_E", "M_B", "sigma", "W", "N"):
        sc = np.abs(g[key][ok]).max()
        assert np.max(np.abs(a[key][ok] - g[key][ok])) < 1e-12 * sc, key


def test_barycentre_of_symmetric_pairs_is_the_pixel_centre():
    """Two galaxies at the same small distance on either side of a pixel
    centre along a great circle have the centre as barycentre: pixB equals
    the pixel variant with the same sums."""
    nside = 32
    rng = np.random.default_rng(42)
    pix = np.sort(rng.choice(hp.npix(nside), 3000, replace=False))
    c = hp.pix2vec(nside, pix)
    t = np.cross(c, rng.normal(size=c.shape))
    t /= np.linalg.norm(t, axis=1)[:, None]
    eps = 0.15 * math.sqrt(4 * math.pi / hp.npix(nside))
    v = np.concatenate([math.cos(eps) * c + math.sin(eps) * t, math.cos(eps) * c - math.sin(eps) * t])
    ra = np.arctan2(v[:, 1], v[:, 0]) % (2 * math.pi)
    dec = np.arcsin(np.clip(v[:, 2], -1, 1))
    n = v.shape[0]
    cat = {"ra": ra, "dec": dec, "g1": rng.normal(0, 0.3, n), "g2": rng.normal(0, 0.3, n), "w": np.ones(n)}
    from oracle import binning as B

    p_u, W, G1, G2, E2 = B.pixel_sums(nside, ra, dec, cat["g1"], cat["g2"], cat["w"])
    assert np.array_equal(p_u, pix) and np.all(W == 2)
    out = rng.choice(hp.npix(nside), 200, replace=False)
    c_ra, c_dec = hp.pix2radec(nside, out)
    th = 6 * DEG
    a = A.aperture_mass_barycentre(cat, nside, c_ra, c_dec, th, F.POLY)
    b = A.aperture_mass_pixel({"nside": nside, "pix": p_u, "W": W, "G1": G1, "G2": G2, "E2": E2}, out, th, F.POLY)
    ok = ~(a["tie"] | b["tie"])
    for key in ("M_E", "M_B", "sigma", "W", "N"):
        sc = np.abs(b[key][ok]).max()
        assert np.max(np.abs(a[key][ok] - b[key][ok])) < 1e-9 * sc, key


def test_barycentre_across_ra_zero_and_at_the_pole():
    """The barycentre of galaxies on both sides of RA = 0, or around a pole,
    lies among them (a mean of RA would put it half a turn away)."""
    nside = 16
    pra, pdec = hp.pix2radec(nside, np.arange(hp.npix(nside)))
    k = np.nonzero((pra == 0.0) & (np.abs(pdec) < 0.2))[0][0]   # a pixel centred on RA = 0
    ra = np.array([0.01, 2 * math.pi - 0.01, 0.005, 2 * math.pi - 0.02])
    dec = pdec[k] + np.array([0.01, -0.01, 0.0, 0.005])
    assert np.all(hp.radec2pix(nside, ra, dec) == k)
    src = A.barycentre_sources(nside, ra, dec, np.zeros(4), np.zeros(4))
    assert src.ra.size == 1
    d = min(src.ra[0], 2 * math.pi - src.ra[0])
    assert d < 0.01 and abs(src.dec[0] - pdec[k]) < 0.01
    # two galaxies of the first polar pixel, far apart in RA: the barycentre is
    # the midpoint of the great-circle arc, nearer the pole than either galaxy
    # (a mean of Dec would stay at their declination)
    ra = np.array([0.1, 1.4])
    dec = np.full(2, 0.5 * math.pi - 0.02)
    assert np.all(hp.radec2pix(nside, ra, dec) == 0)
    src = A.barycentre_sources(nside, ra, dec, np.zeros(2), np.zeros(2))
    half = 0.5 * math.acos(np.clip(A.radec2vec(ra[:1], dec[:1]) @ A.radec2vec(ra[1:], dec[1:])[0], -1, 1)[0])
    expect = math.acos(math.cos(0.02) / math.cos(half))   # colatitude of the arc's midpoint
    assert src.ra.size == 1 and abs(src.ra[0] - 0.75) < 1e-12
    assert abs((0.5 * math.pi - src.dec[0]) - expect) < 1e-9 and src.dec[0] > dec[0] + 1e-3


# ----------------------------------------------------------------------------
# sphS_posB: pixels retrieved by their centres, galaxies at their own positions
# ----------------------------------------------------------------------------

def test_posB_with_galaxies_at_pixel_centres_is_the_brute_force():
    """A galaxy at its pixel's centre is inside the aperture exactly when the
    centre is: posB equals the galaxy variant."""
    nside = 64
    rng = np.random.default_rng(51)
    pix = np.sort(rng.choice(hp.npix(nside), 6000, replace=False))
    pix = np.repeat(pix, rng.integers(1, 4, pix.size))       # 1-3 galaxies per pixel
    ra, dec = hp.pix2radec(nside, pix)
    cat = {"ra": ra, "dec": dec, "g1": rng.normal(0, 0.3, pix.size), "g2": rng.normal(0, 0.3, pix.size),
           "w": rng.uniform(0.5, 1.5, pix.size)}
    out = rng.choice(hp.npix(nside), 200, replace=False)
    c_ra, c_dec = hp.pix2radec(nside, out)
    th = 5 * DEG
    a = A.aperture_mass_posB(cat, nside, c_ra, c_dec, th, F.TANH)
    g = A.aperture_mass_galaxy(cat, c_ra, c_dec, th, F.TANH)
    ok = ~(a["tie"] | g["tie"])
    for key in ("M_E", "M_B", "sigma", "W", "N"):
        sc = np.abs(g[key][ok]).max()
        assert np.max(np.abs(a[key][ok] - g[key][ok])) < 1e-12 * sc, key


def test_posB_boundary_galaxies():
    """Membership follows the pixel centre: a galaxy outside the aperture in a
    pixel centred inside it counts in W and N with a zero filter; a galaxy
    inside the aperture in a pixel centred outside it does not count. The
    member count differs from the brute force only by galaxies of pixels
    that cross the aperture's edge."""
    nside = 32
    th = 6 * DEG
    rng = np.random.default_rng(52)
    n = 40000
    z = rng.uniform(math.cos(15 * DEG), 1.0, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    ra = phi
    dec = np.arcsin(z)
    cat = {"ra": ra, "dec": dec, "g1": rng.normal(0, 0.3, n), "g2": rng.normal(0, 0.3, n)}
    c_ra, c_dec = np.array([0.3]), np.array([0.5 * math.pi - 0.05])
    a = A.aperture_mass_posB(cat, nside, c_ra, c_dec, th, F.POLY, norm=A.NORM_RAW)
    g = A.aperture_mass_galaxy(cat, c_ra, c_dec, th, F.POLY, norm=A.NORM_RAW)
    cv = A.radec2vec(c_ra, c_dec)[0]
    gv = A.radec2vec(ra, dec)
    gpix = hp.radec2pix(nside, ra, dec)
    C = 4 * math.sin(0.5 * th) ** 2
    pin = np.sum((hp.pix2vec(nside, gpix) - cv) ** 2, axis=1) < C
    gin = np.sum((gv - cv) ** 2, axis=1) < C
    assert a["N"][0] == pin.sum() and g["N"][0] == gin.sum()
    assert (pin & ~gin).sum() > 0 and (gin & ~pin).sum() > 0
    # E sums: the same filter on the galaxies inside both, nothing from the others
    both = A.aperture_mass_galaxy({k: v[pin & gin] for k, v in cat.items()}, c_ra, c_dec, th, F.POLY,
                                  norm=A.NORM_RAW)
    assert abs(a["M_E"][0] - both["M_E"][0]) < 1e-12 * abs(g["M_E"][0]) + 1e-15
    # the boundary pixels bound the difference: half a pixel diagonal around the edge
    r = np.arccos(np.clip(gv @ cv, -1, 1))
    edge = np.abs(r - th) < 2.0 * math.sqrt(4 * math.pi / hp.npix(nside))
    assert np.all(edge[pin != gin])


def test_averaged_galaxy_route_equals_pixel_route():
    """Averaged approach for galaxies (density of each galaxy's final-map
    pixel) against the pinned averaged pixel variant: one galaxy per pixel at
    the pixel centre with weight W_j and shear G_j / W_j is the same source
    set, so the maps must agree; and with several galaxies per pixel the
    factor is Omega_pix over the pixel's summed weight."""
    from oracle import aperture as A
    from oracle import filters as F
    from oracle import healpix_ref as hp

    nside = 32
    rng = np.random.default_rng(5)
    pix = np.arange(hp.npix(nside))
    pix = pix[hp.pix2vec(nside, pix)[:, 0] > np.cos(0.5)]
    W = rng.uniform(5, 30, pix.size)
    G1 = rng.normal(0, 0.3, pix.size) * W
    G2 = rng.normal(0, 0.3, pix.size) * W
    E2 = (G1 ** 2 + G2 ** 2) / W
    ra, dec = hp.pix2radec(nside, pix)
    cat = {"ra": ra, "dec": dec, "g1": G1 / W, "g2": G2 / W, "w": W}
    out_pix = pix[:: 7]
    th = 6 * np.pi / 180
    c_ra, c_dec = hp.pix2radec(nside, out_pix)
    g = A.aperture_mass_galaxy(cat, c_ra, c_dec, th, F.TANH, norm=A.NORM_AVERAGED, avg_nside=nside)
    p = A.aperture_mass_pixel({"nside": nside, "pix": pix, "W": W, "G1": G1, "G2": G2, "E2": W * E2},
                              out_pix, th, F.TANH, norm=A.NORM_AVERAGED)
    for k in ("M_E", "M_B", "sigma"):
        assert np.max(np.abs(g[k] - p[k])) <= 1e-12 * np.max(np.abs(p[k]))
    c = A.galaxy_density_factors(nside, np.repeat(ra[:3], 2), np.repeat(dec[:3], 2), np.array([1, 3, 2, 2, 5, 5.0]))
    omega = 4 * np.pi / hp.npix(nside)
    assert np.allclose(c, omega / np.array([4, 4, 4, 4, 10, 10.0]), rtol=1e-15)
