"""Galaxy-level shape-noise realisations (smart_noise_galaxy_batch, and the
seeded matrix-core form smart_noise_galaxy_seeded) against
the FP64 oracle with the same angles: the brute-force galaxy variant and the
pixel variant on the re-binned rotated catalogue, FP32 path within 1e-6 of
the map RMS; zero angles reproduce smart_run bit for bit."""
import math

import numpy as np
import pytest

from oracle import aperture as A
from oracle import binning as B
from oracle import filters as F
from oracle import healpix_ref as hp
from synth import noise_angles, small_catalogue

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


def test_galaxy_level_realisations_vs_oracle(ctx):
    import torch
    from paper_2609_11181_amd import lib as L

    n, cap, nb = 60000, 5 * DEG, 256
    cat = small_catalogue(n, seed=61, cap_radius=cap, centre=(0.02, 0.0))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=nb, pixel_sums=True)
    n_real = 12
    u = noise_angles(62, 0, n_real, n)
    u_dev = torch.from_numpy(u).cuda()
    ths = [30 * ARCMIN, 50 * ARCMIN]
    fids = [ctx.filter(F.TANH), ctx.filter(F.POLY)]
    kinds = [F.TANH, F.POLY]
    rng = np.random.default_rng(63)

    # brute-force galaxy variant, outputs on a coarser grid
    no = 128
    v = hp.pix2vec(no, np.arange(hp.npix(no)))
    out_g = np.nonzero(v[:, 0] > math.cos(cap + 0.3 * DEG))[0]
    plan_g = ctx.plan(data, L.VAR_GALAXY, no, out_g, ths, fids)
    got = plan_g.noise_galaxy_batch(u_dev, n_real, L.NORM_SUMMED_CAP).cpu().numpy()
    c_ra, c_dec = hp.pix2radec(no, out_g)
    for r in (0, 7, n_real - 1):
        rc = A.rotate_galaxies(cat, u[r].astype(np.float64))
        for k, (th, kind) in enumerate(zip(ths, kinds)):
            ref = A.aperture_mass_galaxy(rc, c_ra, c_dec, th, kind)
            ok = ~ref["tie"]
            for e, key in enumerate(["M_E", "M_B"]):
                err = _rel(got[k, r, e], ref[key], ok)
                assert err <= 1e-6, ("galaxy", r, k, key, err)
    # zero angles: the rotation is the identity, the maps are smart_run's
    zero = torch.zeros(1, n, dtype=torch.float32, device="cuda")
    z = plan_g.noise_galaxy_batch(zero, 1, L.NORM_SUMMED_CAP).cpu().numpy()
    main = plan_g.run(L.NORM_SUMMED_CAP).cpu().numpy()
    assert np.array_equal(z[:, 0], main[:, 0:2])

    # pixel variant: the pixel sums of the rotated catalogue, outputs on the binning grid
    src = data.sources().cpu().numpy()
    out_p = np.sort(rng.choice(src, min(3000, src.size), replace=False))
    plan_p = ctx.plan(data, L.VAR_PIXEL, nb, out_p, ths, fids)
    for norm in (L.NORM_SUMMED_PIXCOUNT, L.NORM_AVERAGED):
        got = plan_p.noise_galaxy_batch(u_dev, n_real, norm).cpu().numpy()
        for r in (0, n_real - 1):
            rc = A.rotate_galaxies(cat, u[r].astype(np.float64))
            p_u, W, G1, G2, E2 = B.pixel_sums(nb, rc["ra"], rc["dec"], rc["g1"], rc["g2"], rc["w"])
            m = {"nside": nb, "pix": p_u, "W": W, "G1": G1, "G2": G2, "E2": E2}
            for k, (th, kind) in enumerate(zip(ths, kinds)):
                ref = A.aperture_mass_pixel(m, out_p, th, kind, norm=norm)
                ok = ~ref["tie"]
                for e, key in enumerate(["M_E", "M_B"]):
                    err = _rel(got[k, r, e], ref[key], ok)
                    assert err <= 1e-6, ("pixel", norm, r, k, key, err)
    z = plan_p.noise_galaxy_batch(zero, 1, L.NORM_SUMMED_PIXCOUNT).cpu().numpy()
    main = plan_p.run(L.NORM_SUMMED_PIXCOUNT).cpu().numpy()
    assert np.array_equal(z[:, 0], main[:, 0:2])

    # a pixel map made from sums has no galaxies to rotate
    pm = ctx.pixel_map(nb, p_u, W.astype(np.float32), G1.astype(np.float32), G2.astype(np.float32),
                       E2.astype(np.float32))
    plan_m = ctx.plan(pm, L.VAR_PIXEL, nb, out_p[:10], ths[:1], fids[:1])
    with pytest.raises(L.SmartError):
        plan_m.noise_galaxy_batch(zero, 1, L.NORM_SUMMED_PIXCOUNT)


def test_galaxy_level_seeded_mfma(ctx):
    """smart_noise_galaxy_angles draws the oracle's Philox4x32-10 angles bit
    for bit; smart_noise_galaxy_seeded (rotated pixel sums contracted on the
    matrix cores) matches the oracle on the re-binned rotated catalogue and
    smart_noise_galaxy_batch on the same angles within 1e-4 of the map RMS
    (split-BF16x3 terms), for a realisation range that starts off a block of
    four and ends in a partial chunk, both normalisations; its moments over
    split ranges equal the sums over its maps."""
    import torch
    from oracle import rng as R
    from paper_2609_11181_amd import lib as L

    n, cap, nb = 60000, 5 * DEG, 256
    cat = small_catalogue(n, seed=71, cap_radius=cap, centre=(0.02, 0.0))
    data = ctx.bin_galaxies(cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"], nside_bin=nb, pixel_sums=True)
    seed, r0, nr = 2 ** 37 + 5, 3, 37
    u_dev = ctx.noise_galaxy_angles(seed, r0, nr, n)
    u = R.galaxy_angles(seed, r0, nr, n)
    assert np.array_equal(u_dev.cpu().numpy(), u)

    ths = [30 * ARCMIN, 50 * ARCMIN]
    kinds = [F.TANH, F.POLY]
    fids = [ctx.filter(k) for k in kinds]
    rng = np.random.default_rng(72)
    src = data.sources().cpu().numpy()
    out_p = np.sort(rng.choice(src, min(3000, src.size), replace=False))
    plan = ctx.plan(data, L.VAR_PIXEL, nb, out_p, ths, fids)
    for norm in (L.NORM_SUMMED_PIXCOUNT, L.NORM_AVERAGED):
        got = plan.noise_galaxy_seeded(seed, r0, nr, norm)
        ref_b = plan.noise_galaxy_batch(u_dev, nr, norm)
        g, b = got.cpu().numpy(), ref_b.cpu().numpy()
        for k in range(len(ths)):
            for r in range(nr):
                for e in range(2):
                    rms = math.sqrt(np.mean(b[k, r, e].astype(np.float64) ** 2))
                    err = np.max(np.abs(g[k, r, e].astype(np.float64) - b[k, r, e])) / rms
                    assert err <= 1e-4, ("batch", norm, k, r, e, err)
        for r in (0, 1, 32, nr - 1):
            rc = A.rotate_galaxies(cat, u[r].astype(np.float64))
            p_u, W, G1, G2, E2 = B.pixel_sums(nb, rc["ra"], rc["dec"], rc["g1"], rc["g2"], rc["w"])
            m = {"nside": nb, "pix": p_u, "W": W, "G1": G1, "G2": G2, "E2": E2}
            for k, (th, kind) in enumerate(zip(ths, kinds)):
                ref = A.aperture_mass_pixel(m, out_p, th, kind, norm=norm)
                ok = ~ref["tie"]
                for e, key in enumerate(["M_E", "M_B"]):
                    err = _rel(g[k, r, e], ref[key], ok)
                    assert err <= 1e-4, ("oracle", norm, r, k, key, err)
        mom = plan.noise_galaxy_seeded(seed, r0, 5, norm, moments=True)
        plan.noise_galaxy_seeded(seed, r0 + 5, nr - 5, norm, moments=True, out=mom)
        md = got.double()
        want = torch.stack([md[:, :, 0].sum(1), (md[:, :, 0] ** 2).sum(1), md[:, :, 1].sum(1),
                            (md[:, :, 1] ** 2).sum(1)], dim=1)
        scale = torch.abs(want).amax(dim=2, keepdim=True)
        assert torch.max(torch.abs(mom - want) / scale) < 1e-9

    # other plans and data are refused
    plan_g = ctx.plan(data, L.VAR_GALAXY, nb, out_p[:10], ths[:1], fids[:1])
    with pytest.raises(L.SmartError):
        plan_g.noise_galaxy_seeded(seed, 0, 1, L.NORM_SUMMED_CAP)
    with pytest.raises(L.SmartError):
        plan.noise_galaxy_seeded(seed, 0, 0, L.NORM_SUMMED_PIXCOUNT)
    with pytest.raises(L.SmartError):
        plan.noise_galaxy_seeded(seed, 2 ** 33, 1, L.NORM_SUMMED_PIXCOUNT)
    p_u, W, G1, G2, E2 = B.pixel_sums(nb, cat["ra"], cat["dec"], cat["g1"], cat["g2"], cat["w"])
    pm = ctx.pixel_map(nb, p_u, W.astype(np.float32), G1.astype(np.float32), G2.astype(np.float32),
                       E2.astype(np.float32))
    plan_m = ctx.plan(pm, L.VAR_PIXEL, nb, out_p[:10], ths[:1], fids[:1])
    with pytest.raises(L.SmartError):
        plan_m.noise_galaxy_seeded(seed, 0, 1, L.NORM_SUMMED_PIXCOUNT)
