"""The two forms of the FP32 galaxy kernel (one lane per aperture centre,
one wave per centre) against the FP64 oracle (brute force, sphS_posB and
barycentre data, Sect. 3.1, 3.3 and 3.4), within 1e-6 of the map RMS and N
exact for both forms; the form a plan starts with follows the mean candidate
count and run length of its sampled centres; a wave-form disc of more than 64 partition
rings takes several passes; the autotuner's galaxy choice is cached."""
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


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_11181_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _rel(gpu, ref, ok):
    rms = math.sqrt(np.mean(ref[ok] ** 2))
    return float(np.max(np.abs(gpu[ok].astype(np.float64) - ref[ok])) / rms)


def _centres(no, cap, n, seed):
    v = hp.pix2vec(no, np.arange(hp.npix(no)))
    pix = np.nonzero(v[:, 0] > math.cos(cap))[0]
    if pix.size > n:
        pix = np.sort(np.random.default_rng(seed).choice(pix, n, replace=False))
    return pix


def _check(out, ref):
    ok = ~ref["tie"]
    errs = {key: _rel(out[c], ref[key], ok) for c, key in enumerate(["M_E", "M_B", "sigma"])}
    assert max(errs.values()) <= 1e-6, errs
    assert np.array_equal(out[4][ok].astype(np.float64), ref["N"][ok])
    return errs


# (galaxies, cap, binning NSIDE, output NSIDE, theta_ap, filter, form the plan starts with)
CASES = [
    (20000, 5 * DEG, 1024, 128, 30 * ARCMIN, F.TANH, 0),    # about 200 candidates per centre in short runs
    (150000, 5 * DEG, 256, 128, 60 * ARCMIN, F.POLY, 1),    # about 6000
    (150000, 6 * DEG, 1024, 128, 2.5 * DEG, F.TANH, 1),     # about 90 partition rings per disc
]


@pytest.mark.parametrize("n,cap,nb,no,th,kind,first", CASES)
def test_both_forms_vs_oracle(ctx, n, cap, nb, no, th, kind, first):
    from paper_2609_11181_amd import lib as L

    cat = small_catalogue(n, seed=nb + n % 97, cap_radius=cap, centre=(0.02, 0.01))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=nb)
    out_pix = _centres(no, cap - 0.5 * th, 400, nb)
    plan = ctx.plan(data, L.VAR_GALAXY, no, out_pix, [th], [ctx.filter(kind)])
    assert plan.galaxy_form(0) == first
    c_ra, c_dec = hp.pix2radec(no, out_pix)
    ref = A.aperture_mass_galaxy(cat, c_ra, c_dec, th, kind)
    outs = []
    for form in (L.GAL_LANE, L.GAL_WAVE):
        plan.set_galaxy_form(0, form)
        out = plan.run(L.NORM_SUMMED_CAP).cpu().numpy()[0]
        print(n, nb, th, form, _check(out, ref))
        outs.append(out)
    # the two forms sum the same members in different orders
    ok = ~ref["tie"]
    for c in range(3):
        scale = math.sqrt(np.mean(outs[0][c][ok].astype(np.float64) ** 2))
        assert np.max(np.abs(outs[0][c][ok] - outs[1][c][ok])) <= 2e-6 * scale
    assert np.allclose(outs[0][3], outs[1][3], rtol=1e-6)
    assert np.array_equal(outs[0][4], outs[1][4])


def test_forms_per_scale_and_posB_barycentre(ctx):
    """One plan whose scales start in different forms; sphS_posB and
    barycentre sources in both forms."""
    from paper_2609_11181_amd import lib as L

    cap = 5 * DEG
    cat = small_catalogue(60000, seed=5, cap_radius=cap, centre=(0.0, -0.02))
    nb = 256
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=nb, pixel_sums=True)
    out_pix = _centres(nb, cap - 1 * DEG, 300, 7)
    ths = [5 * ARCMIN, 80 * ARCMIN]
    fid = ctx.filter(F.TANH)
    plan = ctx.plan(data, L.VAR_GALAXY, nb, out_pix, ths, [fid, fid])
    assert [plan.galaxy_form(k) for k in range(2)] == [L.GAL_LANE, L.GAL_WAVE]
    out = plan.run(L.NORM_SUMMED_CAP).cpu().numpy()
    c_ra, c_dec = hp.pix2radec(nb, out_pix)
    for k, th in enumerate(ths):
        _check(out[k], A.aperture_mass_galaxy(cat, c_ra, c_dec, th, F.TANH))
    th = 40 * ARCMIN
    pb = ctx.plan(data, L.VAR_GALAXY_POSB, nb, out_pix, [th], [fid])
    ref = A.aperture_mass_posB(cat, nb, c_ra, c_dec, th, F.TANH)
    bary = data.barycentre()
    pc = ctx.plan(bary, L.VAR_GALAXY, nb, out_pix, [th], [fid])
    ref_b = A.aperture_mass_barycentre(cat, nb, c_ra, c_dec, th, F.TANH, norm=A.NORM_SUMMED_CAP)
    for form in (L.GAL_LANE, L.GAL_WAVE):
        pb.set_galaxy_form(0, form)
        _check(pb.run(L.NORM_SUMMED_CAP).cpu().numpy()[0], ref)
        pc.set_galaxy_form(0, form)
        _check(pc.run(L.NORM_SUMMED_CAP).cpu().numpy()[0], ref_b)


def test_autotune_galaxy_cache_and_errors(ctx, tmp_path):
    from paper_2609_11181_amd import lib as L

    cap = 4 * DEG
    cat = small_catalogue(30000, seed=9, cap_radius=cap, centre=(1.0, 0.2))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=256)
    fid = ctx.filter(F.TANH)
    out_pix = _centres_near(256, A.radec2vec(1.0, 0.2), cap, 2000, 3)
    ths = [20 * ARCMIN, 70 * ARCMIN]
    plan = ctx.plan(data, L.VAR_GALAXY, 256, out_pix, ths, [fid, fid])
    before = plan.run(L.NORM_SUMMED_CAP).cpu().numpy()
    cache = tmp_path / "tune.txt"
    plan.autotune(5000, cache)
    forms = [plan.galaxy_form(k) for k in range(2)]
    assert all(f in (L.GAL_LANE, L.GAL_WAVE) for f in forms)
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and all(ln.startswith("key=gal/") and " form=" in ln for ln in lines)
    after = plan.run(L.NORM_SUMMED_CAP).cpu().numpy()
    assert np.array_equal(before[:, 4], after[:, 4])
    rms = np.sqrt(np.mean(before[:, 0].astype(np.float64) ** 2))
    assert np.max(np.abs(before[:, 0] - after[:, 0])) <= 2e-6 * rms
    # a second plan of the same workload looks the choices up (no measuring)
    again = ctx.plan(data, L.VAR_GALAXY, 256, out_pix, ths, [fid, fid])
    for k in range(2):
        again.set_galaxy_form(k, 1 - forms[k])
    again.autotune(0, cache)
    assert [again.galaxy_form(k) for k in range(2)] == forms
    with pytest.raises(L.SmartError):
        plan.set_galaxy_form(2, L.GAL_LANE)
    with pytest.raises(L.SmartError):
        plan.set_galaxy_form(0, 2)
    p64 = ctx.plan(data, L.VAR_GALAXY, 256, out_pix[:10], [ths[0]], [fid], precision=L.PREC_FP64)
    with pytest.raises(L.SmartError):
        p64.galaxy_form(0)


def _centres_near(no, anchor, rad, n, seed):
    v = hp.pix2vec(no, np.arange(hp.npix(no)))
    pix = np.nonzero(v @ anchor > math.cos(rad))[0]
    if pix.size > n:
        pix = np.sort(np.random.default_rng(seed).choice(pix, n, replace=False))
    return pix


def test_visiting_order_covers_every_output(ctx):
    """The wave form visits a plan's centres in tiles of rings and azimuth
    (an order built at plan creation); every output is written once with the
    sums of its own centre. Whole maps, bit for bit: a shuffled output list
    (with a repeated pixel) gives the sorted list's values at the permuted
    positions, for both forms, over more centres than one tile row holds."""
    import torch
    from paper_2609_11181_amd import lib as L

    cat = small_catalogue(100000, seed=7, cap_radius=4 * DEG, centre=(0.0, 0.0))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=512)
    v = hp.pix2vec(256, np.arange(hp.npix(256)))
    pix = np.nonzero(v[:, 0] > math.cos(3.5 * DEG))[0]  # about 2000 centres over many tiles
    rng = np.random.default_rng(3)
    perm = rng.permutation(pix.size)
    shuffled = np.concatenate([pix[perm], pix[perm[:1]]])
    th = 20 * ARCMIN
    fid = ctx.filter(F.TANH)
    a = ctx.plan(data, L.VAR_GALAXY, 256, pix, [th], [fid])
    b = ctx.plan(data, L.VAR_GALAXY, 256, shuffled, [th], [fid])
    for form in (L.GAL_WAVE, L.GAL_LANE):
        a.set_galaxy_form(0, form)
        b.set_galaxy_form(0, form)
        oa = a.run(L.NORM_SUMMED_CAP)
        ob = b.run(L.NORM_SUMMED_CAP)
        torch.cuda.synchronize()
        oa = oa.cpu().numpy()[0]
        ob = ob.cpu().numpy()[0]
        assert np.array_equal(ob[:, : pix.size], oa[:, perm]), form
        assert np.array_equal(ob[:, pix.size], oa[:, perm[0]]), form
        assert np.all(oa[4] > 0), form
