"""The five workloads at their full sizes, in the launch configuration the
benchmark times, checked against the FP64 oracle on sampled apertures (the
oracle computes them one by one):

1. brute-force galaxy variant in FP64: 1e6 galaxies on the sphere, all
   49152 NSIDE-64 apertures, theta_ap = 2 deg, polynomial filter (whole map);
2. galaxy variant, mixed precision: 5e7 galaxies in a 1000 deg^2 field,
   NSIDE-2048 apertures in the field, theta_ap = 10', tanh filter;
3. pixel variant at NSIDE 4096 over 15000 deg^2, three scales (the
   benchmark workload);
4. 256 shape-noise realisations x 3 scales of a 5000 deg^2 field binned at
   NSIDE 2048, split-BF16 MFMA path;
5. a mixed batch of the 64 drawn instances (NSIDE, field area, aperture and
   filter of each) at their full field areas, one persistent launch; each
   instance checked on centres around a random pixel of its field, the
   oracle reading the pixels within reach of them.
"""
import math

import numpy as np
import pytest

from oracle import aperture as A
from oracle import filters as F
from oracle import healpix_ref as hp
import synth
from synth import ARCMIN, DEG

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_11181_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _err(gpu, ref, key, ok):
    rms = math.sqrt(np.mean(ref[key][ok] ** 2))
    return float(np.max(np.abs(gpu[ok] - ref[key][ok])) / rms)


def test_config1_fp64_full_map(ctx):
    from paper_2609_11181_amd import lib as L

    cat = synth.config1_catalogue()
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=256)
    out_pix = np.arange(hp.npix(64))
    th = 2 * DEG
    plan = ctx.plan(data, L.VAR_GALAXY, 64, out_pix, [th], [ctx.filter(L.FILTER_POLY)], precision=L.PREC_FP64)
    out = plan.run(L.NORM_SUMMED_CAP).cpu().numpy()[0]
    ra, dec = hp.pix2radec(64, out_pix)
    ref = A.aperture_mass_galaxy(cat, ra, dec, th, F.POLY)
    ok = ~ref["tie"]
    assert ok.sum() >= out_pix.size - 5
    for c, key in enumerate(("M_E", "M_B", "sigma")):
        assert _err(out[c], ref, key, ok) <= 3e-12, key
    assert np.array_equal(out[4][ok], ref["N"][ok])


def _near(v, anchor, radius):
    return np.nonzero(v @ anchor > math.cos(radius))[0]


def test_config2_galaxy_mixed_precision(ctx):
    from paper_2609_11181_amd import lib as L

    cat, R = synth.config2_catalogue()
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=4096)
    nside = 2048
    # every aperture whose centre lies in the field
    rt = hp.ring_table(nside)
    rings = np.nonzero(np.abs(np.arcsin(rt["z"])) < R)[0]
    pix = np.arange(rt["first"][rings[0]], rt["first"][rings[-1]] + rt["n"][rings[-1]])
    v = hp.pix2vec(nside, pix)
    out_pix = pix[v[:, 0] > math.cos(R)]
    vo = v[v[:, 0] > math.cos(R)]
    th = 10 * ARCMIN
    plan = ctx.plan(data, L.VAR_GALAXY, nside, out_pix, [th], [ctx.filter(L.FILTER_TANH)])
    out = plan.run(L.NORM_SUMMED_CAP).cpu().numpy()[0]
    assert out_pix.size > 1.2e6
    gv = A.radec2vec(cat["ra"], cat["dec"])
    rng = np.random.default_rng(2)
    # 600 apertures in a 1-degree patch inside the field, 300 at its edge
    for anchor, n in ((A.radec2vec(0.1, -0.05), 600), (A.radec2vec(R - 0.2 * DEG, 0.0), 300)):
        sel = np.sort(rng.choice(_near(vo, anchor, 1 * DEG), n, replace=False))
        keep = gv @ anchor > math.cos(1 * DEG + th + 0.002)
        sub = {k: cat[k][keep] for k in ("ra", "dec", "g1", "g2", "w")}
        ra, dec = hp.pix2radec(nside, out_pix[sel])
        ref = A.aperture_mass_galaxy(sub, ra, dec, th, F.TANH)
        ok = ~ref["tie"]
        for ch, key in enumerate(("M_E", "M_B", "sigma")):
            assert _err(out[ch][sel], ref, key, ok) <= 1e-6, key
        assert np.array_equal(out[4][sel][ok], ref["N"][ok])


def test_config3_pixel_nside4096(ctx):
    """Maps with double outputs (SMART_PREC_FP32_OUT64: the FP32 output
    format alone rounds a map value to 2^-24 of itself, 1.2e-6 of the RMS at
    a 20-RMS peak), errors relative to the RMS of the whole map, on patches
    inside the field, at its edge, in the polar rings and around the map's
    largest |M_E| at each scale; the FP32-output plan writes exactly these
    values rounded to float."""
    import torch
    from paper_2609_11181_amd import lib as L

    pm, R = synth.config3_pixelmap()
    data = ctx.pixel_map(4096, pm["pix"], pm["W"], pm["G1"], pm["G2"], pm["E2"])
    scales = [5 * ARCMIN, 10 * ARCMIN, 20 * ARCMIN]
    fid = ctx.filter(L.FILTER_TANH)
    plan = ctx.plan(data, L.VAR_PIXEL, 4096, pm["pix"], scales, [fid] * 3, precision=L.PREC_FP32_OUT64)
    out = plan.run(L.NORM_SUMMED_PIXCOUNT)
    assert out.dtype == torch.float64
    assert plan.last_pairs() > 1.6e11
    map_rms = torch.sqrt(torch.mean(out[:, :3] ** 2, dim=2)).cpu().numpy()  # [scale][channel]
    peaks = torch.argmax(torch.abs(out[:, 0]), dim=1).cpu().numpy()
    plan32 = ctx.plan(data, L.VAR_PIXEL, 4096, pm["pix"], scales, [fid] * 3)
    out32 = plan32.run(L.NORM_SUMMED_PIXCOUNT)
    assert torch.equal(out32, out.float())
    del out32, plan32
    rng = np.random.default_rng(3)
    vp = hp.pix2vec(4096, pm["pix"])
    # a patch inside the field, one at its edge and one in the polar rings,
    # then small patches around each scale's largest |M_E|
    anchors = [(A.radec2vec(-0.3, 0.2), 1 * DEG, None), (A.radec2vec(R - 0.3 * DEG, 0.0), 1 * DEG, None),
               (A.radec2vec(0.0, math.asin(0.93)), 1 * DEG, None)]
    anchors += [(vp[p], 0.2 * DEG, p) for p in peaks]
    worst = 0.0
    for anchor, rad, peak in anchors:
        cand = _near(vp, anchor, rad)
        sel = np.sort(rng.choice(cand, min(500, cand.size), replace=False))
        if peak is not None:
            sel = np.unique(np.concatenate([sel, [peak]]))
        near = vp @ anchor > math.cos(rad + scales[-1] + 0.002)
        sub = {"nside": 4096, "pix": pm["pix"][near]}
        for k in ("W", "G1", "G2", "E2"):
            sub[k] = pm[k][near]
        o = out[:, :, sel].cpu().numpy()
        for k, th in enumerate(scales):
            ref = A.aperture_mass_pixel(sub, pm["pix"][sel], th, F.TANH)
            ok = ~ref["tie"]
            for ch, key in enumerate(("M_E", "M_B", "sigma")):
                e = float(np.max(np.abs(o[k, ch][ok] - ref[key][ok]))) / map_rms[k, ch]
                worst = max(worst, e)
                assert e <= 1e-6, (k, key, peak, e)
            assert np.array_equal(o[k, 4][ok], ref["N"][ok])
    print("worst error / map RMS", worst)


def test_config4_batched_noise(ctx):
    import torch
    from paper_2609_11181_amd import lib as L

    cat, R = synth.config4_catalogue()
    cols = [torch.from_numpy(cat[k]).cuda() for k in ("ra", "dec", "g1", "g2")]
    del cat
    data = ctx.bin_galaxies(*cols, None, nside_bin=2048, pixel_sums=True)
    del cols
    src = data.sources()
    n_src = src.numel()
    scales = [5 * ARCMIN, 10 * ARCMIN, 20 * ARCMIN]
    plan = ctx.plan(data, L.VAR_PIXEL, 2048, src, scales, [ctx.filter(L.FILTER_TANH)] * 3)
    n_real = 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(44)
    u = torch.rand((n_real, n_src), generator=gen, device="cuda", dtype=torch.float32)
    out = plan.noise_batch(u, n_real, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3)
    inf = data.info()
    _, _, sums = data.export(sums=True)
    srcs = src.cpu().numpy()
    s = sums.cpu().numpy()[srcs - inf["pix_first"]]
    v = hp.pix2vec(2048, srcs)
    rng = np.random.default_rng(4)
    c = A.radec2vec(0.2, 0.1)
    inner = np.nonzero(v @ c > math.cos(1 * DEG))[0]
    sel = np.sort(rng.choice(inner, 1024, replace=False))
    near = v @ c > math.cos(1 * DEG + scales[-1] + 0.01)
    sub = {"nside": 2048, "pix": srcs[near], "W": s[near, 2], "G1": s[near, 0], "G2": s[near, 1], "E2": s[near, 3]}
    for r in (0, 1, n_real - 1):
        G1, G2 = A.rotate_realisation(sub["G1"], sub["G2"], u[r].cpu().numpy()[near])
        mr = dict(sub, G1=G1, G2=G2)
        o = out[:, r][:, :, sel].cpu().numpy()
        for k, th in enumerate(scales):
            ref = A.aperture_mass_pixel(mr, srcs[sel], th, F.TANH)
            ok = ~ref["tie"]
            for e, key in enumerate(("M_E", "M_B")):
                assert _err(o[k, e], ref, key, ok) <= 1e-4, (r, k, key)


def _near_anchor(m, nside, theta_ap, rng, radius=0.5 * DEG):
    """A random pixel of the field, the list positions of the field's pixels
    within `radius` of it (the centres to check) and those within reach of
    them (the sources the oracle needs)."""
    anchor = m["pix"][rng.integers(0, m["pix"].size)]
    a = hp.pix2vec(nside, np.array([anchor]))[0]
    rt = hp.ring_table(nside)
    colat = np.arctan2(rt["sin"], rt["z"])
    reach = radius + theta_ap + 0.01
    rings = np.nonzero(np.abs(colat - math.acos(a[2])) < reach)[0]
    lo = rt["first"][rings[0]]
    hi = rt["first"][rings[-1]] + rt["n"][rings[-1]]
    sel = np.nonzero((m["pix"] >= lo) & (m["pix"] < hi))[0]
    dist = np.arccos(np.clip(hp.pix2vec(nside, m["pix"][sel]) @ a, -1.0, 1.0))
    return sel[dist < radius], sel[dist < reach]


def test_config5_mixed_batch(ctx):
    import torch
    from paper_2609_11181_amd import lib as L

    inst = synth.config5_instances()
    plans, maps = [], []
    for k, d in enumerate(inst):
        R = synth.generators.cap_radius_from_area(d["area_deg2"])
        m = synth.pixel_level_map(synth.PixelMapSpec(nside=d["nside"], cap_radius=R, density_arcmin2=13.9,
                                                     halos_per_deg2=0.5, seed=d["seed"]))
        data = ctx.pixel_map(d["nside"], m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
        fid = ctx.filter(L.FILTER_POLY if d["filter"] == 0 else L.FILTER_TANH)
        plans.append(ctx.plan(data, L.VAR_PIXEL, d["nside"], m["pix"], [d["theta_ap"]], [fid]))
        maps.append(m)
    print("mixed batch of", sum(m["pix"].size for m in maps), "pixels in", len(maps), "maps", flush=True)
    outs = [p.empty_out() for p in plans]
    ctx.mixed_batch(plans, [L.NORM_SUMMED_PIXCOUNT] * len(plans), outs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    worst = 0.0
    for k, (d, m) in enumerate(zip(inst, maps)):
        inner, near = _near_anchor(m, d["nside"], d["theta_ap"], rng)
        pick = np.sort(rng.choice(inner, min(128, inner.size), replace=False))
        sub = {"nside": d["nside"], "pix": m["pix"][near]}
        for c in ("W", "G1", "G2", "E2"):
            sub[c] = m[c][near]
        kind = F.POLY if d["filter"] == 0 else F.TANH
        ref = A.aperture_mass_pixel(sub, m["pix"][pick], d["theta_ap"], kind)
        o = outs[k][0].cpu().numpy()[:, pick]
        ok = ~ref["tie"]
        rms = math.sqrt(np.mean(ref["M_E"][ok] ** 2))
        diff = np.max(np.abs(o[0][ok] - ref["M_E"][ok]))
        assert (diff == 0.0) if rms == 0.0 else (diff / rms <= 1e-6), (k, d)
        assert np.array_equal(o[4][ok], ref["N"][ok]), (k, d)
        worst = max(worst, diff / rms if rms > 0 else 0.0)
        maps[k] = None
    print("worst error / sample RMS", worst)
