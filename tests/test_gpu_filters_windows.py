"""Filters and window widths that the workloads do not reach, through the C
ABI against the FP64 oracle:

* the filter tables as the kernels read them (smart_filter_pieces) against
  the exact filter on a dense grid: the table in x and the general walk's
  tables in sin(theta), for the default tanh filter, a tanh filter with
  other parameters and a table filter;
* maps with a table filter (Catmull-Rom samples) and with a non-default tanh
  filter, pixel and galaxy variants;
* belt items whose windows hold 122-185 members per table ring (the widest
  staged LDS span) and more than 185 (records read from global memory), in
  single runs and in one mixed batch with an ordinary job.
"""
import math

import numpy as np
import pytest

from oracle import aperture as A
from oracle import filters as F
from oracle import healpix_ref as hp
from synth import small_catalogue

pytestmark = pytest.mark.gpu

DEG = math.pi / 180
ARCMIN = DEG / 60
TANH_OTHER = (0.1, 5.0, 120.0, 40.0, 44.0)
# a smooth filter given by 33 samples (32 intervals divide the 2048 table pieces)
TABLE_X = np.linspace(0.0, 1.0, 33)
TABLE_Q = F.q_poly(TABLE_X) * (1.0 + 0.3 * np.sin(5.0 * TABLE_X))


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_11181_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _L():
    from paper_2609_11181_amd import lib

    return lib


def _filters(ctx):
    L = _L()
    return [
        ("tanh", ctx.filter(L.FILTER_TANH), F.TANH, None),
        ("tanh_other", ctx.filter(L.FILTER_TANH, TANH_OTHER), F.TANH, TANH_OTHER),
        ("table", ctx.filter(L.FILTER_TABLE, list(TABLE_Q)), F.TABLE, TABLE_Q),
    ]


def _eval_pieces(c, t):
    """q at table coordinate t as the kernels form it: FP64 c0, the cubic
    part in FP32 at the FP32-rounded local coordinate."""
    i = np.minimum(t.astype(np.int64), c.shape[0] - 1)
    fd = t - i
    f = fd.astype(np.float32)
    c32 = c[i, 1:].astype(np.float32)
    p = f * (f * c32[:, 2] + c32[:, 1]) + c32[:, 0]
    return c[i, 0] + fd * p.astype(np.float64)


@pytest.mark.parametrize("theta", [5 * ARCMIN, 20 * ARCMIN, 2 * DEG, 0.25])
def test_filter_pieces_against_exact_filter(ctx, theta):
    """The x table to 1e-8 of the filter maximum for every filter (the
    table filter's x table holds its Catmull-Rom cubics exactly: its knots
    are table knots); the sin(theta) tables to 1e-8 for the closed forms, and
    for the table filter up to 2 degrees; at 0.25 rad to 5e-8 for the table
    filter, whose spline knots fall inside the pieces of the grid in
    sin theta (a jump of the second derivative inside a piece; about 2e-8
    there)."""
    for name, fid, kind, params in _filters(ctx):
        q = F.q_of(kind, params)
        qmax = np.max(np.abs(q(np.linspace(0, 1, 100001)[:-1])))
        cx = ctx.filter_pieces(fid)
        assert cx.shape == (2048, 4)
        x = np.linspace(0, 1, 400001)[:-1]
        ex = np.max(np.abs(_eval_pieces(cx, x * 2048) - q(x)))
        assert ex < 1e-8 * qmax, (name, ex / qmax)
        cs = ctx.filter_pieces(fid, theta)
        assert cs.shape == (2049, 4)
        ymax = math.sin(theta)
        y = np.linspace(0, ymax, 400001)[:-1]
        es = np.max(np.abs(_eval_pieces(cs, y * (2048 / ymax)) - q(np.arcsin(y) / theta)))
        tol = 1e-8 if kind != F.TABLE or theta <= 2 * DEG else 5e-8
        assert es < tol * qmax, (name, theta, es / qmax)
        assert abs(cs[2048, 0] - q(1 - 1e-12)) < 1e-10 * qmax and np.all(cs[2048, 1:] == 0)


def _pixmap(nside, seed, cap, dec0=0.0):
    rng = np.random.default_rng(seed)
    pix = np.arange(hp.npix(nside))
    v = hp.pix2vec(nside, pix)
    pix = pix[v @ A.radec2vec(0.0, dec0) > math.cos(cap)]
    n = pix.size
    W = rng.poisson(20, n).astype(np.float32)
    G1 = (rng.normal(0, 0.26, n) * np.sqrt(W) + 0.02 * W).astype(np.float32)
    G2 = (rng.normal(0, 0.26, n) * np.sqrt(W)).astype(np.float32)
    E2 = (W * 2 * 0.26 ** 2).astype(np.float32)
    return {"nside": nside, "pix": pix, "W": W, "G1": G1, "G2": G2, "E2": E2}


def _err(out, ref, ok, key, ch):
    rms = math.sqrt(np.mean(ref[key][ok] ** 2))
    return float(np.max(np.abs(out[ch][ok] - ref[key][ok])) / rms)


def _check(out, ref, tol=1e-6):
    ok = ~ref["tie"]
    for ch, key in enumerate(("M_E", "M_B", "sigma")):
        e = _err(out, ref, ok, key, ch)
        assert e <= tol, (key, e)
    assert np.array_equal(out[4][ok].astype(np.float64), ref["N"][ok])


def _belt_runs(nside, rings, j0, length):
    """Runs of `length` consecutive pixels from azimuth index j0 on the
    given (belt) rings: each run is a belt item."""
    rt = hp.ring_table(nside)
    return np.unique(np.concatenate([rt["first"][r - 1] + (j0 + np.arange(length)) % rt["n"][r - 1] for r in rings]))


@pytest.mark.parametrize("which", ["tanh_other", "table"])
def test_pixel_and_galaxy_maps_with_other_filters(ctx, which):
    L = _L()
    name, fid, kind, params = [f for f in _filters(ctx) if f[0] == which][0]
    nside = 128
    m = _pixmap(nside, 21, 20 * DEG)
    data = ctx.pixel_map(nside, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
    rng = np.random.default_rng(22)
    inner = m["pix"][hp.pix2vec(nside, m["pix"])[:, 0] > math.cos(12 * DEG)]
    out_pix = np.unique(np.concatenate([_belt_runs(nside, [2 * nside - 3, 2 * nside, 2 * nside + 5], 500, 40),
                                        rng.choice(inner, 700, replace=False)]))
    ths = [40 * ARCMIN, 3 * DEG]
    plan = ctx.plan(data, L.VAR_PIXEL, nside, out_pix, ths, [fid, fid])
    out = plan.run(L.NORM_SUMMED_PIXCOUNT).cpu().numpy()
    for k, th in enumerate(ths):
        _check(out[k], A.aperture_mass_pixel(m, out_pix, th, kind, filter_params=params))
    cat = small_catalogue(150000, seed=23, cap_radius=6 * DEG, centre=(0.02, 0.0))
    gd = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=256)
    v = hp.pix2vec(128, np.arange(hp.npix(128)))
    op = np.nonzero(v[:, 0] > math.cos(5 * DEG))[0]
    th = 45 * ARCMIN
    gp = ctx.plan(gd, L.VAR_GALAXY, 128, op, [th], [fid])
    go = gp.run(L.NORM_SUMMED_CAP).cpu().numpy()[0]
    ra, dec = hp.pix2radec(128, op)
    _check(go, A.aperture_mass_galaxy(cat, ra, dec, th, kind, filter_params=params))


# (NSIDE, theta_ap, centre declination): members per table ring about
# 4 NSIDE theta / (pi cos dec); a belt disc spans about 3 NSIDE theta rings
# (at most 384, so 4 NSIDE theta / pi < 163 at the equator: windows over 185
# members occur towards the belt's edge)
WIDE = [(512, 0.2, 0.0), (1024, 0.125, 30 * DEG)]


def _wide_case(ctx, nside, th, dec0, seed):
    members = 4 * nside * th / (math.pi * math.cos(dec0))
    assert (122 <= members <= 185) if nside == 512 else members > 185
    m = _pixmap(nside, seed, th + 3 * DEG, dec0)
    data = ctx.pixel_map(nside, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
    # the belt ring at declination dec0: z = 4/3 - 2 i / (3 nside)
    ring = int(round((4.0 / 3.0 - math.sin(dec0)) * 1.5 * nside))
    # two tiles of 256 entries: a run across ring `ring`'s end (two belt
    # items) and a run inside ring `ring` + 7 (one belt item)
    out_pix = np.concatenate([_belt_runs(nside, [ring], 4 * nside - 128, 256),
                              _belt_runs(nside, [ring + 7], 4 * nside - 300, 256)])
    return m, data, np.sort(out_pix)


@pytest.mark.parametrize("nside,th,dec0", WIDE)
def test_wide_belt_windows(ctx, nside, th, dec0):
    import torch

    L = _L()
    m, data, out_pix = _wide_case(ctx, nside, th, dec0, 30 + nside)
    fid = ctx.filter(L.FILTER_TANH)
    plan = ctx.plan(data, L.VAR_PIXEL, nside, out_pix, [th], [fid])
    belt, gen = plan.tiles(0)
    assert belt.shape[0] == 3 and gen.shape[0] == 0
    out = plan.run(L.NORM_SUMMED_PIXCOUNT)
    torch.cuda.synchronize()
    sel = np.arange(0, out_pix.size, 3)
    ref = A.aperture_mass_pixel(m, out_pix[sel], th, F.TANH)
    _check(out.cpu().numpy()[0][:, sel], ref)


def test_wide_windows_in_mixed_batch(ctx):
    """The two wide-window jobs and an ordinary one in one persistent launch:
    bit-identical to their single runs (same device code, same order)."""
    import torch

    L = _L()
    fid = ctx.filter(L.FILTER_TANH)
    plans, keep = [], []
    for (nside, th, dec0), seed in zip(WIDE, (41, 42)):
        m, data, out_pix = _wide_case(ctx, nside, th, dec0, seed)
        plans.append(ctx.plan(data, L.VAR_PIXEL, nside, out_pix, [th], [fid]))
        keep.append(data)
    m = _pixmap(256, 43, 10 * DEG)
    d3 = ctx.pixel_map(256, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
    plans.append(ctx.plan(d3, L.VAR_PIXEL, 256, m["pix"], [30 * ARCMIN], [ctx.filter(L.FILTER_POLY)]))
    single = [p.run(L.NORM_SUMMED_PIXCOUNT).clone() for p in plans]
    outs = [p.empty_out() for p in plans]
    ctx.mixed_batch(plans, [L.NORM_SUMMED_PIXCOUNT] * 3, outs)
    torch.cuda.synchronize()
    for a, b in zip(single, outs):
        assert torch.equal(a, b)
