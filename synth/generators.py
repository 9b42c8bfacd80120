"""Seeded synthetic catalogues and pixel maps with the statistics of the
paper's evaluation workload (Sect. 4 and Sect. 5: shape noise of 0.26 per
component, a Stage-IV-like source density, a circular field centred on the
equator).

Conventions of the produced arrays:

* angles in radians; right ascension in [0, 2*pi), declination in [-pi/2, pi/2];
* shear (g1, g2) in the local frame whose x axis points East (+ra) and whose
  y axis points North (+dec): g1 > 0 is an East-West elongation, g2 > 0 an
  elongation along the North-East diagonal;
* pixel maps use the HEALPix RING numbering; a pixel entry carries the sum of
  weights W, the weighted shear sums G1, G2 and the sum of w^2 |g|^2 (E2).

The lensing signal is a superposition of singular isothermal spheres (SIS):
tangential shear theta_E / (2 theta) around each halo, held at 1/2 inside
the Einstein radius theta_E (the weak-lensing regime) and truncated at
``trunc`` radians for CPU cost (generator parameters only; every consumer
reads the same arrays).

Nothing here computes an aperture mass. The generator needs pixel centres to
place signal on a pixel map and to select the pixels of a field; it carries
its own small routine for that, used for nothing else.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ARCMIN = math.pi / 10800.0
DEG = math.pi / 180.0
SIGMA_E = 0.26


# ----------------------------------------------------------------------------
# small geometry helpers (generator-private)
# ----------------------------------------------------------------------------

def _unit(ra, dec):
    cd = np.cos(dec)
    return np.stack([cd * np.cos(ra), cd * np.sin(ra), np.sin(dec)], axis=-1)


def _bearing_shear(ra_g, dec_g, ra_h, dec_h, gamma_t):
    """Shear of a galaxy tangentially aligned about a halo.

    The initial bearing beta from the galaxy towards the halo (measured from
    North through East, navigation convention) fixes the radial direction; a
    tangential ellipse is elongated perpendicular to it, which in the
    (East, North) frame gives g = gamma_t * exp(-2 i beta).
    """
    dra = ra_h - ra_g
    y = np.sin(dra) * np.cos(dec_h)
    x = np.cos(dec_g) * np.sin(dec_h) - np.sin(dec_g) * np.cos(dec_h) * np.cos(dra)
    beta = np.arctan2(y, x)
    return gamma_t * np.cos(2 * beta), -gamma_t * np.sin(2 * beta)


def _sis_gamma(theta_e, theta):
    """Tangential shear of a singular isothermal sphere, theta_E / (2 theta),
    held at its Einstein-radius value 1/2 inside theta_E: closer in, the
    lens is strong and the weak-shear formula (which diverges at the centre)
    no longer describes the sources."""
    return theta_e / (2.0 * np.maximum(theta, theta_e))


def _sep(ra1, dec1, ra2, dec2):
    """Great-circle separation by the haversine form."""
    s = np.sin(0.5 * (dec2 - dec1)) ** 2 + np.cos(dec1) * np.cos(dec2) * np.sin(0.5 * (ra2 - ra1)) ** 2
    return 2 * np.arcsin(np.sqrt(np.clip(s, 0.0, 1.0)))


def cap_radius_from_area(area_deg2: float) -> float:
    """Radius (rad) of a spherical cap of the given area (deg^2)."""
    sr = area_deg2 * DEG * DEG
    return math.acos(1.0 - sr / (2 * math.pi))


# ----------------------------------------------------------------------------
# galaxy catalogues
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class CatalogueSpec:
    n_gal: int
    cap_radius: float | None  # None = full sphere; else cap centred at (0, 0)
    n_halos: int
    seed: int
    trunc: float = 0.5 * DEG
    weights: bool = False


def _halos(rng, n, cap_radius):
    if cap_radius is None:
        ra = rng.uniform(0, 2 * math.pi, n)
        dec = np.arcsin(rng.uniform(-1, 1, n))
    else:
        ra, dec = _uniform_cap_rejection(rng, n, cap_radius)
    theta_e = rng.uniform(0.5 * ARCMIN, 3.0 * ARCMIN, n)
    return ra, dec, theta_e


def _uniform_cap_rejection(rng, n, R):
    out_ra, out_dec = [], []
    got = 0
    while got < n:
        m = 2 * (n - got) + 16
        # the cap centred at (0, 0) lies inside |ra| < R, |dec| < R
        amax = R if R < math.pi / 2 else math.pi
        sd = math.sin(min(R, math.pi / 2))
        ra = rng.uniform(-amax, amax, m)
        dec = np.arcsin(rng.uniform(-sd, sd, m))
        keep = np.cos(dec) * np.cos(ra) > math.cos(R)
        out_ra.append(ra[keep])
        out_dec.append(dec[keep])
        got += int(keep.sum())
    ra = np.concatenate(out_ra)[:n]
    dec = np.concatenate(out_dec)[:n]
    return np.mod(ra, 2 * math.pi), dec


def _banded_cap_positions(rng, density_sr, R, band):
    """Uniform positions in a cap of radius R centred at (0, 0).

    Declination bands of height ``band`` are filled independently; inside a
    band right ascension is drawn already sorted (normalised exponential
    spacings), which lets the signal pass find a halo's neighbours by
    bisection. Returns (ra in (-pi, pi], dec, band_edges_dec, band_offsets).
    """
    nb = int(math.ceil(2 * R / band))
    edges = np.linspace(-R, R, nb + 1)
    ras, decs, offs = [], [], [0]
    cR = math.cos(R)
    for b in range(nb):
        lo, hi = edges[b], edges[b + 1]
        dmin = 0.0 if lo <= 0.0 <= hi else min(abs(lo), abs(hi))
        ratio = cR / math.cos(dmin)
        if ratio >= 1.0:
            offs.append(offs[-1])
            continue
        amax = math.acos(ratio)
        area = 2 * amax * (math.sin(hi) - math.sin(lo))
        n = int(rng.poisson(density_sr * area))
        e = rng.standard_exponential(n + 1)
        c = np.cumsum(e)
        ra = -amax + 2 * amax * (c[:n] / c[n])
        dec = np.arcsin(rng.uniform(math.sin(lo), math.sin(hi), n))
        keep = np.cos(dec) * np.cos(ra) > cR
        ras.append(ra[keep])
        decs.append(dec[keep])
        offs.append(offs[-1] + int(keep.sum()))
    ra = np.concatenate(ras) if ras else np.zeros(0)
    dec = np.concatenate(decs) if decs else np.zeros(0)
    return ra, dec, edges, np.asarray(offs, dtype=np.int64)


def _add_sis_banded(g1, g2, ra, dec, edges, offs, halos, trunc):
    h_ra, h_dec, h_te = halos
    h_ra = np.where(h_ra > math.pi, h_ra - 2 * math.pi, h_ra)
    nb = len(edges) - 1
    for k in range(len(h_ra)):
        ha, hd, te = h_ra[k], h_dec[k], h_te[k]
        dmax = min(abs(hd) + trunc, math.pi / 2 - 1e-9)
        da = trunc / math.cos(dmax) + 1e-12
        b0 = max(0, int(np.searchsorted(edges, hd - trunc, side="right")) - 1)
        b1 = min(nb - 1, int(np.searchsorted(edges, hd + trunc, side="right")) - 1)
        for b in range(b0, b1 + 1):
            s, e = offs[b], offs[b + 1]
            if e <= s:
                continue
            seg = ra[s:e]
            i0 = s + int(np.searchsorted(seg, ha - da))
            i1 = s + int(np.searchsorted(seg, ha + da))
            if i1 <= i0:
                continue
            th = _sep(ra[i0:i1], dec[i0:i1], ha, hd)
            m = (th < trunc) & (th > 0)
            if not m.any():
                continue
            idx = np.nonzero(m)[0] + i0
            gt = _sis_gamma(te, th[m])
            a, b_ = _bearing_shear(ra[idx], dec[idx], ha, hd, gt)
            g1[idx] += a
            g2[idx] += b_


def galaxy_catalogue(spec: CatalogueSpec):
    """Galaxy catalogue: dict of ra, dec (float64), g1, g2, w (float32)."""
    rng = np.random.default_rng(spec.seed)
    halos = _halos(rng, spec.n_halos, spec.cap_radius)
    if spec.cap_radius is None:
        n = spec.n_gal
        ra = rng.uniform(0, 2 * math.pi, n)
        dec = np.arcsin(rng.uniform(-1, 1, n))
        g1 = rng.normal(0, SIGMA_E, n)
        g2 = rng.normal(0, SIGMA_E, n)
        # brute force over the (few) halos
        for k in range(spec.n_halos):
            th = _sep(ra, dec, halos[0][k], halos[1][k])
            m = (th < spec.trunc) & (th > 0)
            idx = np.nonzero(m)[0]
            a, b = _bearing_shear(ra[idx], dec[idx], halos[0][k], halos[1][k], _sis_gamma(halos[2][k], th[m]))
            g1[idx] += a
            g2[idx] += b
    else:
        R = spec.cap_radius
        area = 2 * math.pi * (1 - math.cos(R))
        ra, dec, edges, offs = _banded_cap_positions(rng, spec.n_gal / area, R, spec.trunc)
        n = ra.size
        g1 = rng.normal(0, SIGMA_E, n)
        g2 = rng.normal(0, SIGMA_E, n)
        _add_sis_banded(g1, g2, ra, dec, edges, offs, halos, spec.trunc)
        ra = np.mod(ra, 2 * math.pi)
    w = rng.uniform(0.5, 1.5, n).astype(np.float32) if spec.weights else np.ones(n, np.float32)
    return {
        "ra": np.ascontiguousarray(ra, dtype=np.float64),
        "dec": np.ascontiguousarray(dec, dtype=np.float64),
        "g1": g1.astype(np.float32),
        "g2": g2.astype(np.float32),
        "w": w,
        "halos": halos,
    }


def small_catalogue(n, seed, *, cap_radius=None, centre=(0.0, 0.0), weights=True, n_halos=3,
                    signal=True):
    """Small random catalogue for unit tests: uniform on the sphere or in a
    cap about ``centre``; random weights; shape noise plus SIS signal."""
    rng = np.random.default_rng(seed)
    if cap_radius is None:
        ra = rng.uniform(0, 2 * math.pi, n)
        dec = np.arcsin(rng.uniform(-1, 1, n))
    else:
        # uniform in a cap around centre via rotation of a cap about the pole
        ct = rng.uniform(math.cos(cap_radius), 1.0, n)
        st = np.sqrt(1 - ct * ct)
        az = rng.uniform(0, 2 * math.pi, n)
        v = np.stack([st * np.cos(az), st * np.sin(az), ct], -1)
        a0, d0 = centre
        # rotate pole -> centre: about y by (pi/2 - d0), then about z by a0
        t = math.pi / 2 - d0
        ry = np.array([[math.cos(t), 0, math.sin(t)], [0, 1, 0], [-math.sin(t), 0, math.cos(t)]])
        rz = np.array([[math.cos(a0), -math.sin(a0), 0], [math.sin(a0), math.cos(a0), 0], [0, 0, 1]])
        v = v @ (rz @ ry).T
        ra = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * math.pi)
        dec = np.arcsin(np.clip(v[:, 2], -1, 1))
    g1 = rng.normal(0, SIGMA_E, n)
    g2 = rng.normal(0, SIGMA_E, n)
    if signal and n_halos:
        k = rng.integers(0, n, n_halos)
        for j in k:
            th = _sep(ra, dec, ra[j], dec[j])
            m = th > 0
            gt = np.zeros(n)
            gt[m] = 2.0 * ARCMIN / (2 * np.maximum(th[m], 1 * ARCMIN))
            a, b = _bearing_shear(ra, dec, ra[j], dec[j], gt)
            g1 += a
            g2 += b
    w = rng.uniform(0.2, 2.0, n) if weights else np.ones(n)
    return {
        "ra": ra.astype(np.float64),
        "dec": dec.astype(np.float64),
        "g1": g1.astype(np.float32),
        "g2": g2.astype(np.float32),
        "w": w.astype(np.float32),
    }


# ----------------------------------------------------------------------------
# pixel-level maps (RING numbering)
# ----------------------------------------------------------------------------

def _ring_table(nside):
    """Per ring (1..4N-1): z, sin(theta), pixel count, first index, half-shift."""
    N = nside
    i = np.arange(1, 4 * N, dtype=np.int64)
    n = np.where(i < N, 4 * i, np.where(i > 3 * N, 4 * (4 * N - i), 4 * N))
    cap_n = i < N
    cap_s = i > 3 * N
    ip = np.where(cap_s, 4 * N - i, i).astype(np.float64)
    one_minus = ip * ip / (3.0 * N * N)  # 1 - |z| in the caps
    z = np.where(cap_n, 1 - one_minus, np.where(cap_s, -(1 - one_minus), (4.0 / 3.0) - 2.0 * i / (3.0 * N)))
    s = np.where(cap_n | cap_s, np.sqrt(np.maximum(one_minus * (2 - one_minus), 0.0)),
                 np.sqrt(np.maximum((1 - z) * (1 + z), 0.0)))
    start = np.where(i < N, 2 * i * (i - 1),
                     np.where(i <= 3 * N, 2 * N * (N - 1) + 4 * N * (i - N),
                              12 * N * N - 2 * (4 * N - i) * (4 * N - i + 1)))
    half = np.where(cap_n | cap_s, 0.5, np.where(((i - N) % 2) == 0, 0.5, 0.0))
    return {"z": z, "s": s, "n": n, "start": start, "half": half}


@dataclasses.dataclass
class PixelMapSpec:
    nside: int
    cap_radius: float           # cap centred at (0, 0)
    density_arcmin2: float      # galaxies per arcmin^2
    halos_per_deg2: float
    seed: int
    trunc: float = 0.5 * DEG


def pixel_level_map(spec: PixelMapSpec):
    """Pixel map of a field: per pixel inside the cap, a Poisson galaxy count
    N_j, G = N_j * gamma_SIS(r_j) + sqrt(N_j) * 0.26 * normal per component,
    E2 = N_j * 2 * 0.26^2 + N_j * |gamma_SIS|^2 (its expectation), W = N_j.

    Returns dict(nside, pix (int64 sorted), W, G1, G2, E2 (float32)).
    """
    N = spec.nside
    R = spec.cap_radius
    rng = np.random.default_rng(spec.seed)
    rt = _ring_table(N)
    cR = math.cos(R)
    # rings whose latitude band reaches the cap
    lat = np.arcsin(rt["z"])
    rings = np.nonzero(np.abs(lat) < R)[0]
    if rings.size == 0:
        raise ValueError("empty field")
    r0, r1 = int(rings[0]), int(rings[-1])
    base = int(rt["start"][r0])
    end = int(rt["start"][r1] + rt["n"][r1])
    dense_n = end - base
    inside = np.zeros(dense_n, dtype=bool)
    for r in range(r0, r1 + 1):
        s = rt["s"][r]
        if s <= 0 or cR / s >= 1.0:
            continue
        amax = math.acos(cR / s)
        n = int(rt["n"][r])
        dphi = 2 * math.pi / n
        h = rt["half"][r]
        # pixels with |phi| < amax, phi_j = (j + h) dphi (mod 2 pi)
        jhi = int(math.floor(amax / dphi - h))       # j in [0, jhi]
        jlo = int(math.ceil(n - amax / dphi - h))    # j in [jlo, n)
        a = int(rt["start"][r]) - base
        jhi = min(jhi, n - 1)
        if jhi >= 0:
            inside[a: a + jhi + 1] = True
        if jlo < n:
            inside[a + max(jlo, 0): a + n] = True
    idx = np.nonzero(inside)[0]
    npx = idx.size
    omega = 4 * math.pi / (12 * N * N)
    lam = spec.density_arcmin2 * omega / (ARCMIN * ARCMIN)
    cnt = rng.poisson(lam, npx).astype(np.float64)
    g1s = np.zeros(dense_n, dtype=np.float64)
    g2s = np.zeros(dense_n, dtype=np.float64)
    # halos
    area_deg2 = 2 * math.pi * (1 - cR) / (DEG * DEG)
    nh = int(round(spec.halos_per_deg2 * area_deg2))
    h_ra, h_dec = _uniform_cap_rejection(rng, nh, R) if nh else (np.zeros(0), np.zeros(0))
    h_te = rng.uniform(0.5 * ARCMIN, 3.0 * ARCMIN, nh)
    tr = spec.trunc
    for k in range(nh):
        ha, hd, te = h_ra[k], h_dec[k], h_te[k]
        rr = np.nonzero(np.abs(lat[r0:r1 + 1] - hd) < tr)[0] + r0
        if rr.size == 0:
            continue
        segs = []
        for r in rr:
            s = rt["s"][r]
            if s <= 1e-12:
                continue
            half_w = min(math.pi, tr / s + 2 * 2 * math.pi / rt["n"][r])
            n = int(rt["n"][r])
            dphi = 2 * math.pi / n
            h = rt["half"][r]
            jc = ha / dphi - h
            ja = int(math.floor(jc - half_w / dphi))
            jb = int(math.ceil(jc + half_w / dphi))
            if jb - ja + 1 >= n:
                j = np.arange(n)
            else:
                j = np.mod(np.arange(ja, jb + 1), n)
            segs.append((r, j))
        if not segs:
            continue
        rix = np.concatenate([np.full(j.size, r) for r, j in segs])
        jix = np.concatenate([j for _, j in segs])
        phi = (jix + rt["half"][rix]) * (2 * math.pi / rt["n"][rix])
        dec = np.arcsin(rt["z"][rix])
        th = _sep(phi, dec, ha, hd)
        m = (th < tr) & (th > 0)
        if not m.any():
            continue
        gt = _sis_gamma(te, th[m])
        a, b = _bearing_shear(phi[m], dec[m], ha, hd, gt)
        d = (rt["start"][rix[m]] - base + jix[m]).astype(np.int64)
        np.add.at(g1s, d, a)
        np.add.at(g2s, d, b)
    sig1 = g1s[idx]
    sig2 = g2s[idx]
    del g1s, g2s
    sq = np.sqrt(cnt)
    G1 = cnt * sig1 + sq * SIGMA_E * rng.standard_normal(npx)
    G2 = cnt * sig2 + sq * SIGMA_E * rng.standard_normal(npx)
    E2 = cnt * (2 * SIGMA_E ** 2) + cnt * (sig1 * sig1 + sig2 * sig2)
    return {
        "nside": N,
        "pix": (idx + base).astype(np.int64),
        "W": cnt.astype(np.float32),
        "G1": G1.astype(np.float32),
        "G2": G2.astype(np.float32),
        "E2": E2.astype(np.float32),
        "halos": (h_ra, h_dec, h_te),
    }


def noise_angles(seed: int, r_first: int, n_real: int, n_in: int) -> np.ndarray:
    """Uniform numbers u in [0, 1) for shape-noise realisations, one row per
    realisation r (seeded by (seed, r) so any subset can be regenerated);
    the rotation angle of input element j in realisation r is pi * u[r, j]."""
    out = np.empty((n_real, n_in), dtype=np.float32)
    for k in range(n_real):
        out[k] = np.random.default_rng([seed, r_first + k]).random(n_in, dtype=np.float32)
    return out


# ----------------------------------------------------------------------------
# the five workload presets
# ----------------------------------------------------------------------------

def config1_catalogue(seed=1):
    """1e6 galaxies on the full sphere, 20 SIS halos (output NSIDE 64,
    theta_ap = 2 deg, polynomial filter, FP64)."""
    return galaxy_catalogue(CatalogueSpec(n_gal=1_000_000, cap_radius=None, n_halos=20, seed=seed,
                                          trunc=1.0 * DEG))


def config2_catalogue(seed=2, n_gal=50_000_000):
    """5e7 galaxies in a 1000 deg^2 cap, 500 halos (output NSIDE 2048 inside the
    cap, theta_ap = 10', tanh filter, FP32 with FP64 geometry)."""
    R = cap_radius_from_area(1000.0)
    return galaxy_catalogue(CatalogueSpec(n_gal=n_gal, cap_radius=R, n_halos=int(round(500 * n_gal / 5e7)),
                                          seed=seed)), R


def config3_pixelmap(seed=3, area_deg2=15000.0, nside=4096):
    """NSIDE-4096 pixel map over a 15000 deg^2 cap, 30 gal/arcmin^2,
    20000 halos (1.333 per deg^2)."""
    R = cap_radius_from_area(area_deg2)
    return pixel_level_map(PixelMapSpec(nside=nside, cap_radius=R, density_arcmin2=30.0,
                                        halos_per_deg2=20000.0 / 15000.0, seed=seed)), R


def config4_catalogue(seed=4, area_deg2=5000.0, density_arcmin2=50_000_000 / (1000 * 3600.0)):
    """Config-2 statistics over a 5000 deg^2 cap (about 2.5e8 galaxies)."""
    R = cap_radius_from_area(area_deg2)
    n = int(round(density_arcmin2 * area_deg2 * 3600.0))
    nh = int(round(0.5 * area_deg2))
    return galaxy_catalogue(CatalogueSpec(n_gal=n, cap_radius=R, n_halos=nh, seed=seed)), R


def config5_instances(seed=5, n_inst=64):
    """Parameters of the 64-instance mixed batch: NSIDE in {512..4096}, cap area
    log-uniform in [100, 15000] deg^2, theta_ap log-uniform in [2', 40'],
    filter in {poly, tanh}; pixel-level maps with config-2 statistics."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        nside = int(rng.choice([512, 1024, 2048, 4096]))
        area = float(math.exp(rng.uniform(math.log(100.0), math.log(15000.0))))
        th = float(math.exp(rng.uniform(math.log(2.0), math.log(40.0)))) * ARCMIN
        filt = int(rng.integers(0, 2))
        out.append({"nside": nside, "area_deg2": area, "theta_ap": th, "filter": filt,
                    "seed": int(rng.integers(0, 2**31 - 1))})
    return out
