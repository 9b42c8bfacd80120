"""sphS_pixB on the GPU (smart_barycentre_map + galaxy-variant FP32 plans):
pixel sums at their galaxies' barycentres against the FP64 oracle within 1e-6
of the map RMS, on a field that straddles RA = 0; the plans and inputs it
does not apply to are rejected."""
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


@pytest.mark.parametrize("nb,th,kind,norm", [(256, 40 * ARCMIN, F.TANH, 1), (128, 90 * ARCMIN, F.POLY, 0),
                                             (512, 25 * ARCMIN, F.TANH, 2)])
def test_barycentre_variant_vs_oracle(ctx, nb, th, kind, norm):
    from paper_2609_11181_amd import lib as L

    cap = 6 * DEG
    cat = small_catalogue(150000, seed=nb + 7, cap_radius=cap, centre=(0.02, 0.0))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=nb, pixel_sums=True)
    bdata = data.barycentre()
    n_occ = data.sources().numel()
    assert bdata.info()["n_gal"] == n_occ
    no = 128
    v = hp.pix2vec(no, np.arange(hp.npix(no)))
    out_pix = np.nonzero(v[:, 0] > math.cos(cap + 0.5 * th))[0]
    plan = ctx.plan(bdata, L.VAR_GALAXY, no, out_pix, [th], [ctx.filter(kind)])
    out = plan.run(norm).cpu().numpy()[0]
    c_ra, c_dec = hp.pix2radec(no, out_pix)
    ref = A.aperture_mass_barycentre(cat, nb, c_ra, c_dec, th, kind, norm=norm)
    ok = ~ref["tie"]
    errs = {key: _rel(out[c], ref[key], ok) for c, key in enumerate(["M_E", "M_B", "sigma"])}
    print(nb, th, kind, norm, errs)
    assert max(errs.values()) <= 1e-6, errs
    assert np.max(np.abs(out[3][ok] - ref["W"][ok]) / np.maximum(ref["W"][ok], 1)) <= 2e-7
    assert np.array_equal(out[4][ok].astype(np.float64), ref["N"][ok])
    assert abs(plan.last_pairs() - ref["N"].sum()) < 0.5
    # the catalogue's own maps are untouched by building the barycentre data
    pplan = ctx.plan(data, L.VAR_PIXEL, nb, data.sources().cpu().numpy()[:50], [th], [ctx.filter(kind)])
    assert np.isfinite(pplan.run(norm).cpu().numpy()).all()


def test_barycentre_rejections(ctx):
    from paper_2609_11181_amd import lib as L

    cat = small_catalogue(20000, seed=5, cap_radius=3 * DEG, centre=(1.0, 0.3))
    plain = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=128)
    with pytest.raises(L.SmartError):
        plain.barycentre()                      # no pixel sums
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=128, pixel_sums=True)
    bdata = data.barycentre()
    with pytest.raises(L.SmartError):
        bdata.barycentre()                      # already barycentre data
    fid = ctx.filter(F.TANH)
    pix = data.sources().cpu().numpy()[:20]
    with pytest.raises(L.SmartError):
        ctx.plan(bdata, L.VAR_PIXEL, 128, pix, [30 * ARCMIN], [fid])
    with pytest.raises(L.SmartError):
        ctx.plan(bdata, L.VAR_GALAXY, 128, pix, [30 * ARCMIN], [fid], precision=0)
