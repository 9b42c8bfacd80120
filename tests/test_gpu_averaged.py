"""Averaged normalisation (Sect. 2.4) on the GPU: smart_run, the batched
noise realisations and mixed batches with SMART_NORM_AVERAGED against the
FP64 oracle (FP32 path within 1e-6 of the map RMS, split-BF16x3 within
1e-4), on maps with empty pixels; the plans it does not apply to reject it."""
import math

import numpy as np
import pytest

from oracle import aperture as A
from oracle import filters as F
from oracle import healpix_ref as hp
from synth import noise_angles

pytestmark = pytest.mark.gpu

DEG = math.pi / 180
ARCMIN = DEG / 60


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_11181_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _cap_map(nside, cap, seed, lam=6.0):
    """Poisson galaxy counts (about e^-lam of the pixels empty, 8% more
    masked) with shear sums and squared-shear sums consistent with them, in a
    cap centred at (ra, dec) = (180 deg, 0) so that each ring's pixels in the
    cap are one run of consecutive pixel numbers."""
    rng = np.random.default_rng(seed)
    pix = np.arange(hp.npix(nside))
    v = hp.pix2vec(nside, pix)
    pix = pix[-v[:, 0] > math.cos(cap)]
    n = pix.size
    W = rng.poisson(lam, n).astype(np.float32)
    W[rng.uniform(size=n) < 0.08] = 0.0
    G1 = np.where(W > 0, rng.normal(0, 0.26, n) * np.sqrt(W) + 0.05 * W, 0.0).astype(np.float32)
    G2 = np.where(W > 0, rng.normal(0, 0.26, n) * np.sqrt(W), 0.0).astype(np.float32)
    E2 = np.where(W > 0, 2 * 0.26 ** 2 * W + 0.01 * G1.astype(np.float64) ** 2, 0.0).astype(np.float32)
    return {"nside": nside, "pix": pix, "W": W, "G1": G1, "G2": G2, "E2": E2}


def _rel(gpu, ref, ok):
    rms = math.sqrt(np.mean(ref[ok] ** 2))
    return float(np.max(np.abs(gpu[ok].astype(np.float64) - ref[ok])) / rms)


def test_averaged_run_vs_oracle(ctx):
    from paper_2609_11181_amd import lib as L

    nside = 128
    m = _cap_map(nside, 40 * DEG, 31)
    rng = np.random.default_rng(32)
    # every map pixel (belt runs and polar-cap tiles) plus isolated centres
    out_pix = np.unique(np.concatenate([m["pix"], rng.choice(hp.npix(nside), 500, replace=False)]))
    ths = [1.0 * DEG, 3.0 * DEG]
    kinds = [F.TANH, F.POLY]
    data = ctx.pixel_map(nside, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
    plan = ctx.plan(data, L.VAR_PIXEL, nside, out_pix, ths, [ctx.filter(k) for k in kinds])
    assert plan.tiles(0)[0].shape[0] > 0 and plan.tiles(0)[1].shape[0] > 0   # both tile kinds
    summed = plan.run(L.NORM_SUMMED_PIXCOUNT).cpu().numpy()
    out = plan.run(L.NORM_AVERAGED).cpu().numpy()
    again = plan.run(L.NORM_AVERAGED).cpu().numpy()
    assert np.array_equal(out, again)
    # W and N are the summed maps' channels
    assert np.array_equal(out[:, 3:], summed[:, 3:])
    pick = np.sort(rng.choice(out_pix.size, 1500, replace=False))
    for k, (th, kind) in enumerate(zip(ths, kinds)):
        ref = A.aperture_mass_pixel(m, out_pix[pick], th, kind, norm=A.NORM_AVERAGED)
        ok = ~ref["tie"]
        errs = {key: _rel(out[k, c][pick], ref[key], ok) for c, key in enumerate(["M_E", "M_B", "sigma"])}
        print(th, kind, errs)
        assert max(errs.values()) <= 1e-6, (th, errs)
        assert np.array_equal(out[k, 4][pick][ok].astype(np.float64), ref["N"][ok])


def test_averaged_noise_batch_vs_oracle(ctx):
    import torch
    from paper_2609_11181_amd import lib as L

    nside = 512
    m = _cap_map(nside, 8 * DEG, 33)
    data = ctx.pixel_map(nside, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
    rng = np.random.default_rng(34)
    out_pix = np.unique(np.concatenate([m["pix"][: m["pix"].size // 2], rng.choice(m["pix"], 300, replace=False)]))
    n_real = 40
    u = noise_angles(35, 0, n_real, m["pix"].size)
    u_dev = torch.from_numpy(u).cuda()
    ths = [20 * ARCMIN, 45 * ARCMIN]
    kinds = [F.TANH, F.POLY]
    plan = ctx.plan(data, L.VAR_PIXEL, nside, out_pix, ths, [ctx.filter(k) for k in kinds])
    outs = {p: plan.noise_batch(u_dev, n_real, L.NORM_AVERAGED, p).cpu().numpy() for p in (2, 1)}
    for prec, tol in ((2, 1e-4), (1, 1e-6)):
        out = outs[prec]
        assert np.isfinite(out).all()
        for k, (th, kind) in enumerate(zip(ths, kinds)):
            for r in (0, 17, n_real - 1):
                G1, G2 = A.rotate_realisation(m["G1"], m["G2"], u[r])
                ref = A.aperture_mass_pixel(dict(m, G1=G1, G2=G2), out_pix, th, kind, norm=A.NORM_AVERAGED)
                ok = ~ref["tie"]
                for e, key in enumerate(["M_E", "M_B"]):
                    err = _rel(out[k, r, e], ref[key], ok)
                    assert err <= tol, (prec, k, r, key, err)


def test_averaged_in_mixed_batch_and_rejections(ctx):
    import torch
    from paper_2609_11181_amd import lib as L

    plans, singles = [], []
    for k, (nside, cap, th, norm) in enumerate([(128, 20 * DEG, [2 * DEG], L.NORM_AVERAGED),
                                                (256, 6 * DEG, [30 * ARCMIN, 10 * ARCMIN], L.NORM_SUMMED_PIXCOUNT),
                                                (64, 60 * DEG, [5 * DEG], L.NORM_AVERAGED)]):
        m = _cap_map(nside, cap, 40 + k)
        data = ctx.pixel_map(nside, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
        plan = ctx.plan(data, L.VAR_PIXEL, nside, m["pix"], th, [ctx.filter(F.TANH)] * len(th))
        singles.append(plan.run(norm).cpu().numpy())
        plans.append((plan, norm))
    outs = [p.empty_out().fill_(np.nan) for p, _ in plans]
    ctx.mixed_batch([p for p, _ in plans], [n for _, n in plans], outs)
    torch.cuda.synchronize()
    for k, (o, s) in enumerate(zip(outs, singles)):
        assert np.array_equal(o.cpu().numpy(), s), k
    # FP64 plans reject the averaged form, and galaxy plans whose output grid
    # is not the binning grid (each galaxy needs its pixel of the final map)
    m = _cap_map(64, 20 * DEG, 50)
    data = ctx.pixel_map(64, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
    p64 = ctx.plan(data, L.VAR_PIXEL, 64, m["pix"][:100], [3 * DEG], [ctx.filter(F.TANH)], precision=0)
    with pytest.raises(L.SmartError):
        p64.run(L.NORM_AVERAGED)
    with pytest.raises(L.SmartError):
        p64.run(4)
    ra, dec = hp.pix2radec(64, m["pix"])
    gdata = ctx.bin_galaxies(ra, dec, np.zeros(ra.size), np.zeros(ra.size), nside_bin=128)
    pg = ctx.plan(gdata, L.VAR_GALAXY, 64, m["pix"][:100], [3 * DEG], [ctx.filter(F.TANH)])
    with pytest.raises(L.SmartError):
        pg.run(L.NORM_AVERAGED)


@pytest.mark.parametrize("variant", ["pos", "posB", "pixB"])
def test_averaged_galaxy_sources(ctx, variant):
    """Averaged approach (Sect. 2.4) with galaxy sources: the brute force,
    posB and barycentre data, every galaxy (barycentre source) divided by
    the density of its pixel of the final map, against the oracle; output
    NSIDE = binning NSIDE (another NSIDE is refused)."""
    from paper_2609_11181_amd import lib as L
    from synth import small_catalogue

    nside = 128
    cat = small_catalogue(120000, seed=71, cap_radius=5 * DEG, centre=(0.03, 0.01))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=nside, pixel_sums=True)
    v = hp.pix2vec(nside, np.arange(hp.npix(nside)))
    out_pix = np.nonzero(v[:, 0] > math.cos(4 * DEG))[0]
    th = 50 * ARCMIN
    fid = ctx.filter(F.TANH)
    c_ra, c_dec = hp.pix2radec(nside, out_pix)
    if variant == "pixB":
        d = data.barycentre()
        plan = ctx.plan(d, L.VAR_GALAXY, nside, out_pix, [th], [fid])
        ref = A.aperture_mass_barycentre(cat, nside, c_ra, c_dec, th, F.TANH, norm=A.NORM_AVERAGED)
    elif variant == "posB":
        plan = ctx.plan(data, L.VAR_GALAXY_POSB, nside, out_pix, [th], [fid])
        ref = A.aperture_mass_posB(cat, nside, c_ra, c_dec, th, F.TANH, norm=A.NORM_AVERAGED)
    else:
        plan = ctx.plan(data, L.VAR_GALAXY, nside, out_pix, [th], [fid])
        ref = A.aperture_mass_galaxy(cat, c_ra, c_dec, th, F.TANH, norm=A.NORM_AVERAGED, avg_nside=nside)
    out = plan.run(L.NORM_AVERAGED).cpu().numpy()[0]
    ok = ~ref["tie"]
    for ch, key in enumerate(("M_E", "M_B", "sigma")):
        rms = math.sqrt(np.mean(ref[key][ok] ** 2))
        assert np.max(np.abs(out[ch][ok] - ref[key][ok])) <= 1e-6 * rms, key
    assert np.array_equal(out[4][ok], ref["N"][ok])
    if variant == "pos":
        other = ctx.plan(data, L.VAR_GALAXY, 64, out_pix[:10] // 4, [th], [fid])
        with pytest.raises(L.SmartError):
            other.run(L.NORM_AVERAGED)
