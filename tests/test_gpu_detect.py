"""GPU parity of the detection step (smart_detect_peaks, Sect. 6.1) against
the oracle (oracle/detect.py): the detected pixel indices must be equal,
bit for bit, on whole-sphere maps (every kind of pixel, the seven-neighbour
corners included), on a cap (field edges), with a threshold and with a noise
map, and on the full NSIDE-4096 workload map (15000 deg^2, 5' aperture
mass), compared on patches by the oracle."""
import math

import numpy as np
import pytest

from oracle import aperture as A
from oracle import detect as D
from oracle import healpix_ref as hp

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


@pytest.mark.parametrize("nside", [1, 2, 8, 64, 512])
def test_detect_whole_sphere_and_cap(ctx, nside):
    rng = np.random.default_rng(nside)
    allp = np.arange(hp.npix(nside))
    for pix in (allp, allp[hp.pix2vec(nside, allp)[:, 0] > math.cos(1.0)]):
        if pix.size == 0:
            continue
        # a smooth field plus noise: peaks of every kind, ties broken by the noise
        v = hp.pix2vec(nside, pix)
        val = np.sin(3 * v[:, 0]) * np.cos(2 * v[:, 1]) + 0.3 * rng.normal(size=pix.size)
        sd = rng.uniform(0.2, 1.0, size=pix.size)
        for thr, noise in ((-np.inf, None), (0.5, None), (1.5, sd)):
            got = ctx.detect_peaks(nside, pix, val, thr, noise).cpu().numpy()
            want = D.detect_peaks(nside, pix, val, thr, noise)
            assert np.array_equal(got, want), (nside, pix.size, thr)
    # a plateau has no peak
    assert ctx.detect_peaks(nside, allp, np.ones(allp.size)).numel() == 0


def test_detect_rejects_bad_maps(ctx):
    from paper_2609_11181_amd import lib as L

    with pytest.raises(L.SmartError):
        ctx.detect_peaks(16, np.array([5, 3]), np.array([1.0, 2.0]))
    with pytest.raises(L.SmartError):
        ctx.detect_peaks(16, np.array([12 * 256]), np.array([1.0]))
    assert ctx.detect_peaks(16, np.zeros(0, np.int64), np.zeros(0)).numel() == 0


def test_detect_on_the_nside4096_workload_map(ctx):
    """The 5' M_E map of the 15000 deg^2 NSIDE-4096 workload (double maps),
    detections on all of it, and as a signal-to-noise cut with the sigma
    channel; the oracle decides the pixels of three 1-degree patches (inside
    the field, at its edge, in the polar rings) from the same values."""
    import synth
    import torch
    from paper_2609_11181_amd import lib as L

    pm, R = synth.config3_pixelmap()
    data = ctx.pixel_map(4096, pm["pix"], pm["W"], pm["G1"], pm["G2"], pm["E2"])
    plan = ctx.plan(data, L.VAR_PIXEL, 4096, pm["pix"], [5 * ARCMIN], [ctx.filter(L.FILTER_TANH)],
                    precision=L.PREC_FP32_OUT64)
    out = plan.run(L.NORM_SUMMED_PIXCOUNT)
    pix_d = torch.from_numpy(pm["pix"]).cuda()
    me, sg = out[0, 0].contiguous(), out[0, 2].contiguous()
    peaks = ctx.detect_peaks(4096, pix_d, me).cpu().numpy()
    snr = ctx.detect_peaks(4096, pix_d, me, 4.0, sg).cpu().numpy()
    assert peaks.size > 1e5 and 0 < snr.size < peaks.size
    me_h, sg_h = me.cpu().numpy(), sg.cpu().numpy()
    vp = hp.pix2vec(4096, pm["pix"])
    for anchor in (A.radec2vec(-0.3, 0.2), A.radec2vec(R - 0.3 * DEG, 0.0), A.radec2vec(0.0, math.asin(0.93))):
        sel = np.nonzero(vp @ anchor > math.cos(1 * DEG))[0]
        p = pm["pix"][sel]
        nb = hp.neighbours(4096, p)
        interior = np.isin(np.where(nb >= 0, nb, p[:, None]), p).all(axis=1)
        inner = p[interior]
        for got, want in ((peaks, D.detect_peaks(4096, p, me_h[sel])),
                          (snr, D.detect_peaks(4096, p, me_h[sel], 4.0, sg_h[sel]))):
            assert np.array_equal(np.intersect1d(got, inner), want)
