"""sphS_posB on the GPU (SMART_VAR_GALAXY_POSB): apertures retrieved as the
binning pixels centred inside them, each galaxy's filter at its own position,
against the FP64 oracle within 1e-6 of the map RMS; the W and N channels
count every galaxy of the retrieved pixels exactly."""
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


@pytest.mark.parametrize("nb,no,th,kind,norm", [(256, 128, 40 * ARCMIN, F.TANH, 0), (128, 128, 90 * ARCMIN, F.POLY, 2),
                                                (512, 256, 15 * ARCMIN, F.TANH, 0)])
def test_posB_vs_oracle(ctx, nb, no, th, kind, norm):
    from paper_2609_11181_amd import lib as L

    cap = 6 * DEG
    cat = small_catalogue(150000, seed=nb + 11, cap_radius=cap, centre=(0.02, 0.0))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=nb)
    v = hp.pix2vec(no, np.arange(hp.npix(no)))
    out_pix = np.nonzero(v[:, 0] > math.cos(cap + 0.5 * th))[0]
    if out_pix.size > 3000:
        out_pix = np.sort(np.random.default_rng(nb).choice(out_pix, 3000, replace=False))
    plan = ctx.plan(data, L.VAR_GALAXY_POSB, no, out_pix, [th], [ctx.filter(kind)])
    out = plan.run(norm).cpu().numpy()[0]
    c_ra, c_dec = hp.pix2radec(no, out_pix)
    ref = A.aperture_mass_posB(cat, nb, c_ra, c_dec, th, kind, norm=norm)
    ok = ~ref["tie"]
    errs = {key: _rel(out[c], ref[key], ok) for c, key in enumerate(["M_E", "M_B", "sigma"])}
    print(nb, no, th, kind, norm, errs)
    assert max(errs.values()) <= 1e-6, errs
    assert np.max(np.abs(out[3][ok] - ref["W"][ok]) / np.maximum(ref["W"][ok], 1)) <= 2e-7
    assert np.array_equal(out[4][ok].astype(np.float64), ref["N"][ok])
    # it differs from the brute force (galaxies near the aperture's edge)
    brute = ctx.plan(data, L.VAR_GALAXY, no, out_pix, [th], [ctx.filter(kind)]).run(norm).cpu().numpy()[0]
    assert not np.array_equal(brute[4], out[4])


def test_posB_rejects_fp64(ctx):
    from paper_2609_11181_amd import lib as L

    cat = small_catalogue(5000, seed=3, cap_radius=3 * DEG, centre=(1.0, 0.3))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=128)
    with pytest.raises(L.SmartError):
        ctx.plan(data, L.VAR_GALAXY_POSB, 128, np.arange(10), [30 * ARCMIN], [ctx.filter(F.TANH)], precision=0)


def test_plan_and_norm_refusals(ctx):
    """sphS_posB selects galaxies of a binned catalogue: barycentre data
    (already one source per pixel) is refused; the pixel-count area is
    refused for galaxy sources (N counts galaxies there, not pixels), and
    accepted for barycentre data."""
    from paper_2609_11181_amd import lib as L

    cat = small_catalogue(5000, seed=3, cap_radius=3 * DEG, centre=(1.0, 0.3))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=128, pixel_sums=True)
    fid = ctx.filter(F.TANH)
    bary = data.barycentre()
    with pytest.raises(L.SmartError):
        ctx.plan(bary, L.VAR_GALAXY_POSB, 128, np.arange(10), [30 * ARCMIN], [fid])
    for var in (L.VAR_GALAXY, L.VAR_GALAXY_POSB):
        plan = ctx.plan(data, var, 128, np.arange(10), [30 * ARCMIN], [fid])
        with pytest.raises(L.SmartError):
            plan.run(L.NORM_SUMMED_PIXCOUNT)
        plan.run(L.NORM_SUMMED_CAP)
    ctx.plan(bary, L.VAR_GALAXY, 128, np.arange(10), [30 * ARCMIN], [fid]).run(L.NORM_SUMMED_PIXCOUNT)
