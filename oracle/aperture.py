"""Spherical shear-based aperture mass in plain numpy FP64.

What is computed (the paper's Sect. 2.3-2.4 and Sect. 3.1-3.2):

For an aperture centre p and every source element i strictly inside the
aperture (great-circle distance theta_pi < theta_ap; Sect. 3.1 step 1):

* the separation from the great-circle formula (Sect. 2.3), evaluated here
  as theta = 2 asin(|r_p - r_i| / 2) from unit vectors (the same angle,
  better conditioned for small apertures);
* the polar angle psi of the paper's Sect. 2.3, tan psi =
  sin(a_i - a_0) / (cos d_i tan d_0 - sin d_i cos(a_i - a_0)), taken as
  atan2 of numerator and denominator both multiplied by cos d_0 > 0;
* tangential and cross shear (Eq. gammat):
  g+ = g1 cos 2psi + g2 sin 2psi, gx = -g1 sin 2psi + g2 cos 2psi;
  a source at the centre (closer than 1e-10 rad) has no defined psi and
  contributes g+ = gx = 0 (it still counts in W, N and V);
* the filter q(theta/theta_ap) (Sect. 3.1 step 3).

Sums over the aperture (Eq. map and Eq. map_noise, Sect. 3.1 step 4):

  S_E = sum q A+,   S_B = sum q Ax,   W = sum Wsrc,   V = sum q^2 Vsrc,
  N = sum Nsrc,

where a source carries (A1, A2, Wsrc, Vsrc, Nsrc):
  galaxy variant: (w g1, w g2, w, w^2 |g|^2, 1);
  pixel variant:  (G1, G2, W_j, E2_j, [W_j > 0]) with G, W_j, E2_j the
                  per-pixel sums of Sect. 3.2 step 2, placed at the pixel
                  centre (Sect. 3.2 steps 4-5).

Summed normalisation (Sect. 2.4 and Sect. 3.1 step 5): the density in the
aperture is n = W / A, so with Q = q / theta_ap^2
  M_E = (A / theta_ap^2) S_E / W,  M_B = (A / theta_ap^2) S_B / W,
  sigma = (A / theta_ap^2) sqrt(V / 2) / W          (Eq. map_noise)
with A the aperture area: the spherical cap 2 pi (1 - cos theta_ap) for the
galaxy variant; N_occ * Omega_pix (occupied pixels in the aperture times the
pixel area) for the pixel variant. W = 0 gives M = sigma = 0.

Averaged normalisation (Sect. 2.4, the "averaged approach"): each galaxy
is normalised by the effective density of its own pixel, W_j / Omega_pix,
instead of the aperture's mean density. Summing the galaxies of pixel j
gives the pixel the weight c_j = Omega_pix / W_j on its shear sum, so
  M_E = (1 / theta_ap^2) sum_j q_j c_j G+_j,   M_B likewise with Gx,
  sigma = (1 / theta_ap^2) sqrt(sum_j q_j^2 c_j^2 E2_j / 2)
(Eq. map_noise with per-galaxy weights c_j / theta_ap^2); empty pixels add
nothing; W and N are the summed maps' channels. Pixel variant only, with
Omega_pix the area of a source pixel.

Membership is decided in FP64 on the squared chord against
C_ap = 4 sin^2(theta_ap/2). Pairs within TIE_REL * C_ap of the boundary are
reported as ties: the decision there depends on last-bit rounding, so
comparisons skip those apertures.

Pins (tests/test_oracle_aperture.py): 50-digit mpmath all-pairs brute force
built on tangent-plane vectors rather than the polar-angle formula; the
closed-form aperture mass of a singular isothermal sphere integrated by
quadrature; B-mode nulling for a purely tangential field; E<->B duality;
linearity; invariance under the HEALPix symmetries; pixel variant equal to
the galaxy variant on a catalogue of pixel centres; averaged maps equal to
the galaxy variant with per-galaxy weights Omega_pix / (galaxies in the
pixel), to the summed pixel-count maps when every occupied pixel holds one
galaxy, and unchanged when every galaxy of a pixel is repeated.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree

from . import healpix_ref as hp
from .filters import q_of

TIE_REL = 1e-10
# A source within 1e-10 rad of the centre counts as coincident: its polar
# angle is undefined (and the last-bit rounding of two unit vectors of the
# same point already makes their difference nonzero), so it adds no shear
# term; it still counts in W, N and V.
COINCIDENT_C2 = 1e-20

NORM_SUMMED_CAP = 0
NORM_SUMMED_PIXCOUNT = 1
NORM_RAW = 2
NORM_AVERAGED = 3


def radec2vec(ra, dec):
    ra = np.asarray(ra, dtype=np.float64)
    dec = np.asarray(dec, dtype=np.float64)
    cd = np.cos(dec)
    return np.stack([cd * np.cos(ra), cd * np.sin(ra), np.sin(dec)], axis=-1)


def polar_angle(ra_i, dec_i, ra0, dec0):
    """psi of source i about centre 0 (Sect. 2.3), quadrant fixed by atan2
    with numerator and denominator multiplied by cos(dec0) >= 0."""
    da = ra_i - ra0
    num = np.sin(da) * np.cos(dec0)
    den = np.cos(dec_i) * np.sin(dec0) - np.sin(dec_i) * np.cos(dec0) * np.cos(da)
    return np.arctan2(num, den)


def tangential_cross(g1, g2, psi):
    """Eq. gammat."""
    c = np.cos(2 * psi)
    s = np.sin(2 * psi)
    return g1 * c + g2 * s, -g1 * s + g2 * c


@dataclasses.dataclass
class Sources:
    ra: np.ndarray
    dec: np.ndarray
    A1: np.ndarray
    A2: np.ndarray
    Wsrc: np.ndarray
    Vsrc: np.ndarray
    Nsrc: np.ndarray

    @property
    def vec(self):
        return radec2vec(self.ra, self.dec)


def galaxy_sources(ra, dec, g1, g2, w=None) -> Sources:
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    w = np.ones_like(g1) if w is None else np.asarray(w, dtype=np.float64)
    return Sources(np.asarray(ra, np.float64), np.asarray(dec, np.float64), w * g1, w * g2, w,
                   w * w * (g1 * g1 + g2 * g2), np.ones_like(g1))


def pixel_sources(nside, pix, W, G1, G2, E2) -> Sources:
    ra, dec = hp.pix2radec(nside, np.asarray(pix, np.int64))
    W = np.asarray(W, np.float64)
    return Sources(ra, dec, np.asarray(G1, np.float64), np.asarray(G2, np.float64), W,
                   np.asarray(E2, np.float64), (W > 0).astype(np.float64))


def barycentre_sources(nside, ra, dec, g1, g2, w=None) -> Sources:
    """Pixel-based variant with barycentre positions (Sect. 3.3, label
    sphS_pixB): the galaxies of each occupied pixel are summed as in the
    pixel variant (Sect. 3.2 step 2) and the sums are placed at the pixel's
    barycentre instead of its centre. The barycentre is the normalised mean
    of the galaxies' unit vectors (the paper averages RA and Dec; that mean
    breaks across RA = 0 and near the poles, and elsewhere the two agree to
    second order in the pixel size). Every occupied pixel counts once in N."""
    from . import binning

    ra = np.asarray(ra, np.float64)
    dec = np.asarray(dec, np.float64)
    pix = hp.radec2pix(nside, ra, dec)
    v = radec2vec(ra, dec)
    occ, inv = np.unique(pix, return_inverse=True)
    m = np.stack([np.bincount(inv, v[:, k], occ.size) for k in range(3)], axis=1)
    m /= np.linalg.norm(m, axis=1)[:, None]
    b_ra = np.arctan2(m[:, 1], m[:, 0]) % (2 * math.pi)
    b_dec = np.arctan2(m[:, 2], np.hypot(m[:, 0], m[:, 1]))
    p_u, W, G1, G2, E2 = binning.pixel_sums(nside, ra, dec, g1, g2, w)
    assert np.array_equal(p_u, occ)
    return Sources(b_ra, b_dec, G1, G2, W, E2, np.ones(occ.size))


def aperture_mass_barycentre(cat, nside, c_ra, c_dec, theta_ap, filter_kind, norm=NORM_SUMMED_PIXCOUNT,
                             filter_params=None):
    """sphS_pixB (Sect. 3.3): pixel sums at their pixels' barycentres, every
    source within theta_ap of the centre, summed normalisation with
    A = (occupied pixels in the aperture) x Omega_pix or the cap area."""
    src = barycentre_sources(nside, cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat.get("w"))
    if norm == NORM_AVERAGED:  # each pixel by its own density (Sect. 2.4), as in the pixel variant
        W = src.Wsrc
        src = _averaged(src, np.where(W > 0, 4.0 * math.pi / hp.npix(nside) / np.where(W > 0, W, 1.0), 0.0))
    s = sums_kdtree(src, c_ra, c_dec, theta_ap, q_of(filter_kind, filter_params))
    out = (_averaged_out(s, theta_ap) if norm == NORM_AVERAGED
           else normalise(s, theta_ap, norm, omega_pix=4.0 * math.pi / hp.npix(nside)))
    out["tie"] = s["tie"]
    out["pairs"] = s["pairs"]
    return out


def aperture_mass_posB(cat, nside, c_ra, c_dec, theta_ap, filter_kind, norm=NORM_SUMMED_CAP, filter_params=None):
    """sphS_posB (Sect. 3.4, catalogue partitioned by HEALPix pixel): the
    aperture is retrieved as the pixels whose centres lie within theta_ap of
    the aperture centre, and every galaxy of those pixels is a member (W, V,
    N); its filter is evaluated at its own position, q(theta_i / theta_ap),
    and is zero beyond theta_ap (the filter's support). Galaxies inside the
    aperture in pixels centred outside it are not counted."""
    ra = np.asarray(cat["ra"], np.float64)
    dec = np.asarray(cat["dec"], np.float64)
    src = galaxy_sources(ra, dec, cat["g1"], cat["g2"], cat.get("w"))
    if norm == NORM_AVERAGED:  # per galaxy by its pixel's density (Sect. 2.4); the partition is the final map's grid
        src = _averaged(src, galaxy_density_factors(nside, ra, dec, cat.get("w")))
    src_vec = src.vec
    qfun = q_of(filter_kind, filter_params)
    c_ra = np.asarray(c_ra, np.float64)
    c_dec = np.asarray(c_dec, np.float64)
    n_cen = c_ra.size
    c_vec = radec2vec(c_ra, c_dec)
    C_ap = 4.0 * math.sin(0.5 * theta_ap) ** 2
    gpix = hp.radec2pix(nside, ra, dec)
    order = np.argsort(gpix, kind="stable")
    occ, first, count = np.unique(gpix[order], return_index=True, return_counts=True)
    pc = hp.pix2vec(nside, occ)
    tree = cKDTree(pc)
    lists = tree.query_ball_point(c_vec, 2.0 * math.sin(0.5 * theta_ap) * (1.0 + 1e-9) + 1e-15)
    cc, pp = [], []
    for i, lst in enumerate(lists):
        cc.append(np.full(len(lst), i, np.int64))
        pp.append(np.asarray(lst, np.int64))
    cc = np.concatenate(cc)
    pp = np.concatenate(pp)
    d = c_vec[cc] - pc[pp]
    pc2 = np.einsum("ij,ij->i", d, d)
    tie_pix = np.abs(pc2 - C_ap) <= TIE_REL * C_ap
    keep = pc2 < C_ap
    tie = np.bincount(cc[tie_pix], minlength=n_cen) > 0
    cc, pp = cc[keep], pp[keep]
    # every galaxy of every retrieved pixel
    n_g = count[pp]
    ci = np.repeat(cc, n_g)
    start = np.repeat(first[pp], n_g)
    within = np.arange(ci.size) - np.repeat(np.cumsum(n_g) - n_g, n_g)
    si = order[start + within]
    d = c_vec[ci] - src_vec[si]
    c2 = np.einsum("ij,ij->i", d, d)
    tie |= np.bincount(ci[np.abs(c2 - C_ap) <= TIE_REL * C_ap], minlength=n_cen) > 0
    theta = 2.0 * np.arcsin(np.sqrt(c2) * 0.5)
    q = np.where(c2 < C_ap, qfun(np.minimum(theta / theta_ap, 1.0)), 0.0)
    psi = polar_angle(src.ra[si], src.dec[si], c_ra[ci], c_dec[ci])
    gp, gx = tangential_cross(src.A1[si], src.A2[si], psi)
    at_centre = c2 < COINCIDENT_C2
    gp = np.where(at_centre, 0.0, gp)
    gx = np.where(at_centre, 0.0, gx)
    sums = {
        "S_E": np.bincount(ci, weights=q * gp, minlength=n_cen),
        "S_B": np.bincount(ci, weights=q * gx, minlength=n_cen),
        "W": np.bincount(ci, weights=src.Wsrc[si], minlength=n_cen),
        "V": np.bincount(ci, weights=q * q * src.Vsrc[si], minlength=n_cen),
        "N": np.bincount(ci, weights=src.Nsrc[si], minlength=n_cen),
    }
    out = _averaged_out(sums, theta_ap) if norm == NORM_AVERAGED else normalise(sums, theta_ap, norm)
    out["tie"] = tie
    out["pairs"] = int(ci.size)
    return out


def _pair_sums(src: Sources, src_vec, cand_centre, cand_src, c_ra, c_dec, c_vec, theta_ap, qfun, n_cen):
    """Sums over the candidate pairs (centre index, source index) that pass
    the FP64 membership test."""
    C_ap = 4.0 * math.sin(0.5 * theta_ap) ** 2
    d = c_vec[cand_centre] - src_vec[cand_src]
    c2 = np.einsum("ij,ij->i", d, d)
    tie = np.abs(c2 - C_ap) <= TIE_REL * C_ap
    inside = c2 < C_ap
    ci = cand_centre[inside]
    si = cand_src[inside]
    c2 = c2[inside]
    theta = 2.0 * np.arcsin(np.sqrt(c2) * 0.5)
    q = qfun(theta / theta_ap)
    psi = polar_angle(src.ra[si], src.dec[si], c_ra[ci], c_dec[ci])
    gp, gx = tangential_cross(src.A1[si], src.A2[si], psi)
    at_centre = c2 < COINCIDENT_C2
    gp = np.where(at_centre, 0.0, gp)
    gx = np.where(at_centre, 0.0, gx)
    out = {
        "S_E": np.bincount(ci, weights=q * gp, minlength=n_cen),
        "S_B": np.bincount(ci, weights=q * gx, minlength=n_cen),
        "W": np.bincount(ci, weights=src.Wsrc[si], minlength=n_cen),
        "V": np.bincount(ci, weights=q * q * src.Vsrc[si], minlength=n_cen),
        "N": np.bincount(ci, weights=src.Nsrc[si], minlength=n_cen),
        "tie": np.bincount(cand_centre[tie], minlength=n_cen) > 0,
        "pairs": int(inside.sum()),
    }
    return out


def sums_kdtree(src: Sources, c_ra, c_dec, theta_ap, qfun, chunk=4096):
    """Aperture sums with candidates from a KD-tree on the source unit
    vectors (the neighbour search the paper suggests in Sect. 3.1)."""
    c_ra = np.asarray(c_ra, np.float64)
    c_dec = np.asarray(c_dec, np.float64)
    n_cen = c_ra.size
    src_vec = src.vec
    c_vec = radec2vec(c_ra, c_dec)
    tree = cKDTree(src_vec)
    rad = 2.0 * math.sin(0.5 * theta_ap) * (1.0 + 1e-9) + 1e-15
    acc = None
    for a in range(0, n_cen, chunk):
        b = min(n_cen, a + chunk)
        lists = tree.query_ball_point(c_vec[a:b], rad)
        lens = np.fromiter((len(x) for x in lists), dtype=np.int64, count=b - a)
        cc = np.repeat(np.arange(a, b, dtype=np.int64), lens)
        ss = np.fromiter((k for x in lists for k in x), dtype=np.int64, count=int(lens.sum()))
        part = _pair_sums(src, src_vec, cc, ss, c_ra, c_dec, c_vec, theta_ap, qfun, n_cen)
        if acc is None:
            acc = part
        else:
            for k in ("S_E", "S_B", "W", "V", "N"):
                acc[k] = acc[k] + part[k]
            acc["tie"] = acc["tie"] | part["tie"]
            acc["pairs"] += part["pairs"]
    return acc


def _ring_window_candidates(nside, out_pix, theta_ap, in_index_of):
    """Candidate (output position, input position) pairs for the pixel
    variant: every input pixel of every ring that a necessary condition does
    not exclude. The condition follows from the exact identity
      |r_p - r_j|^2 = (z_p - z_j)^2 + (s_p - s_j)^2 + 4 s_p s_j sin^2(dphi/2),
    which requires s_p s_j sin^2(dphi/2) < sin^2(theta_ap/2) and
    |colat_p - colat_j| < theta_ap for a member. One pixel of margin is
    added on each side; the FP64 chord test decides membership afterwards."""
    rt = hp.ring_table(nside)
    colat = np.arctan2(rt["sin"], rt["z"])
    ring_p, _ = hp.pix2ring(nside, out_pix)
    z_p, s_p, phi_p = hp.pix2zphi(nside, out_pix)
    sh = math.sin(0.5 * theta_ap)
    cc, ss = [], []
    for k in range(out_pix.size):
        cp = colat[ring_p[k] - 1]
        rings = np.nonzero(np.abs(colat - cp) < theta_ap * (1 + 1e-9) + 1e-12)[0]
        if rings.size == 0:
            continue
        n = rt["n"][rings]
        sj = rt["sin"][rings]
        prod = s_p[k] * sj
        arg = np.where(prod > 0, sh / np.sqrt(np.maximum(prod, 1e-300)), 2.0)
        full = arg >= 1.0
        half = np.where(full, math.pi, 2.0 * np.arcsin(np.minimum(arg, 1.0)))
        step = 2 * math.pi / n
        ja = np.floor((phi_p[k] - half) / step - rt["off"][rings]).astype(np.int64) - 1
        jb = np.ceil((phi_p[k] + half) / step - rt["off"][rings]).astype(np.int64) + 1
        cnt = np.where(full | (jb - ja + 1 >= n), n, jb - ja + 1)
        ja = np.where(full | (jb - ja + 1 >= n), 0, ja)
        tot = int(cnt.sum())
        rep_ring = np.repeat(np.arange(rings.size), cnt)
        within = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        j = np.mod(ja[rep_ring] + within, n[rep_ring])
        pix = rt["first"][rings][rep_ring] + j
        pos = in_index_of(pix)
        ok = pos >= 0
        cc.append(np.full(int(ok.sum()), k, dtype=np.int64))
        ss.append(pos[ok])
    if not cc:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(cc), np.concatenate(ss)


def sums_pixel(nside, in_pix, W, G1, G2, E2, out_pix, theta_ap, qfun, candidates="rings"):
    """Aperture sums of the pixel-based variant (Sect. 3.2) at the centres of
    ``out_pix`` (RING, same NSIDE as the input map)."""
    in_pix = np.asarray(in_pix, np.int64)
    out_pix = np.asarray(out_pix, np.int64)
    src = pixel_sources(nside, in_pix, W, G1, G2, E2)
    c_ra, c_dec = hp.pix2radec(nside, out_pix)
    if candidates == "kdtree":
        return sums_kdtree(src, c_ra, c_dec, theta_ap, qfun)
    order = np.argsort(in_pix)
    sorted_pix = in_pix[order]

    def in_index_of(pix):
        k = np.searchsorted(sorted_pix, pix)
        k = np.minimum(k, sorted_pix.size - 1)
        hit = sorted_pix[k] == pix
        return np.where(hit, order[k], -1)

    cc, ss = _ring_window_candidates(nside, out_pix, theta_ap, in_index_of)
    c_vec = radec2vec(c_ra, c_dec)
    return _pair_sums(src, src.vec, cc, ss, c_ra, c_dec, c_vec, theta_ap, qfun, out_pix.size)


def normalise(sums, theta_ap, mode, omega_pix=None):
    """Summed normalisation (Sect. 2.4; Sect. 3.1 step 5; Sect. 3.2 step 2).
    Returns dict with M_E, M_B, sigma, W, N."""
    W = sums["W"]
    if mode == NORM_RAW:
        return {"M_E": sums["S_E"], "M_B": sums["S_B"], "sigma": sums["V"], "W": W, "N": sums["N"]}
    if mode == NORM_SUMMED_CAP:
        A = np.full_like(W, 4.0 * math.pi * math.sin(0.5 * theta_ap) ** 2)  # 2 pi (1 - cos theta_ap)
    elif mode == NORM_SUMMED_PIXCOUNT:
        if omega_pix is None:
            raise ValueError("pixel-count normalisation needs the pixel area")
        A = sums["N"] * omega_pix
    else:
        raise ValueError(mode)
    f = np.where(W > 0, A / (theta_ap * theta_ap) / np.where(W > 0, W, 1.0), 0.0)
    return {
        "M_E": f * sums["S_E"],
        "M_B": f * sums["S_B"],
        "sigma": f * np.sqrt(0.5 * sums["V"]),
        "W": W,
        "N": sums["N"],
    }


def galaxy_density_factors(nside, ra, dec, w=None):
    """Averaged approach for galaxies (Sect. 2.4): each galaxy is divided by
    the effective density of its pixel of the final map, W_pix / Omega_pix,
    i.e. multiplied by c_i = Omega_pix / W_pix(i), with W_pix the summed
    weight of the galaxies in that pixel (NSIDE of the map)."""
    ra = np.asarray(ra, np.float64)
    w = np.ones_like(ra) if w is None else np.asarray(w, np.float64)
    pix = hp.radec2pix(nside, ra, np.asarray(dec, np.float64))
    occ, inv = np.unique(pix, return_inverse=True)
    W = np.bincount(inv, weights=w, minlength=occ.size)
    omega = 4.0 * math.pi / hp.npix(nside)
    return np.where(W[inv] > 0, omega / np.where(W[inv] > 0, W[inv], 1.0), 0.0)


def _averaged(src: Sources, c) -> Sources:
    """Sources whose shear terms carry the factor c and squared terms c^2
    (W and N unchanged: those channels stay the summed ones)."""
    return Sources(src.ra, src.dec, c * src.A1, c * src.A2, src.Wsrc, c * c * src.Vsrc, src.Nsrc)


def _averaged_out(s, theta_ap):
    return {"M_E": s["S_E"] / theta_ap ** 2, "M_B": s["S_B"] / theta_ap ** 2,
            "sigma": np.sqrt(0.5 * s["V"]) / theta_ap ** 2, "W": s["W"], "N": s["N"]}


def aperture_mass_galaxy(cat, c_ra, c_dec, theta_ap, filter_kind, norm=NORM_SUMMED_CAP, filter_params=None,
                         avg_nside=None):
    """Brute-force galaxy variant (Sect. 3.1, label sphS_pos); the averaged
    normalisation (Sect. 2.4) needs the NSIDE of the final map, avg_nside."""
    src = galaxy_sources(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat.get("w"))
    if norm == NORM_AVERAGED:
        src = _averaged(src, galaxy_density_factors(avg_nside, cat["ra"], cat["dec"], cat.get("w")))
    s = sums_kdtree(src, c_ra, c_dec, theta_ap, q_of(filter_kind, filter_params))
    out = _averaged_out(s, theta_ap) if norm == NORM_AVERAGED else normalise(s, theta_ap, norm)
    out["tie"] = s["tie"]
    out["pairs"] = s["pairs"]
    return out


def averaged_sources(nside, W, G1, G2, E2):
    """The pixel sums of the averaged approach (Sect. 2.4): pixel j's galaxies
    are each divided by the pixel's effective density W_j / Omega_pix, so its
    shear sum takes the factor c_j = Omega_pix / W_j and its sum of squared
    shears (the variance term) c_j^2; c_j = 0 for an empty pixel. Returns
    (G1 c, G2 c, E2 c^2)."""
    omega_pix = 4.0 * math.pi / hp.npix(nside)
    W = np.asarray(W, np.float64)
    c = np.where(W > 0, omega_pix / np.where(W > 0, W, 1.0), 0.0)
    return (c * np.asarray(G1, np.float64), c * np.asarray(G2, np.float64),
            c * c * np.asarray(E2, np.float64))


def aperture_mass_pixel(pmap, out_pix, theta_ap, filter_kind, norm=NORM_SUMMED_PIXCOUNT, filter_params=None,
                        candidates="rings"):
    """Pixel-based variant (Sect. 3.2, label sphS_pix); summed (Sect. 3.1
    step 5) or averaged (Sect. 2.4) normalisation."""
    nside = pmap["nside"]
    G1, G2, E2 = pmap["G1"], pmap["G2"], pmap["E2"]
    if norm == NORM_AVERAGED:
        G1, G2, E2 = averaged_sources(nside, pmap["W"], G1, G2, E2)
    s = sums_pixel(nside, pmap["pix"], pmap["W"], G1, G2, E2, out_pix, theta_ap,
                   q_of(filter_kind, filter_params), candidates=candidates)
    if norm == NORM_AVERAGED:
        # the sums already carry Omega_pix / W_j: only Q = q / theta_ap^2 is left
        out = {"M_E": s["S_E"] / theta_ap ** 2, "M_B": s["S_B"] / theta_ap ** 2,
               "sigma": np.sqrt(0.5 * s["V"]) / theta_ap ** 2, "W": s["W"], "N": s["N"]}
    else:
        out = normalise(s, theta_ap, norm, omega_pix=4.0 * math.pi / hp.npix(nside))
    out["tie"] = s["tie"]
    out["pairs"] = s["pairs"]
    return out


def rotate_realisation(G1, G2, u):
    """One shape-noise realisation of a pixel map: each pixel's shear sum is
    rotated by the spin-2 phase exp(2 i phi), phi = pi u (the random
    orientation of the paper's Sect. 1 / Sect. 5.3 noise maps, applied per
    pixel). Returns (G1', G2')."""
    phi = math.pi * np.asarray(u, dtype=np.float64)
    c = np.cos(2 * phi)
    s = np.sin(2 * phi)
    G1 = np.asarray(G1, np.float64)
    G2 = np.asarray(G2, np.float64)
    return G1 * c - G2 * s, G1 * s + G2 * c


def rotate_galaxies(cat, u):
    """One galaxy-level shape-noise realisation (the random orientations of
    Sect. 1 / Sect. 5.3 given to every galaxy): galaxy i's shear is rotated by
    the spin-2 phase exp(2 i pi u_i); positions and weights stay. The pixel
    variant bins the rotated catalogue again (Sect. 3.2 step 2). Returns a
    new catalogue dict."""
    g1, g2 = rotate_realisation(cat["g1"], cat["g2"], u)
    return dict(cat, g1=g1, g2=g2)
