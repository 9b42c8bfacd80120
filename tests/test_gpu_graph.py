"""Capture of smart_run and of the batched noise maps in a HIP graph (through
torch.cuda.CUDAGraph on the capture stream): after one eager call has built
the plan's schedules, both entry points only launch kernels, so they can be
captured; every replay, with eager work and synchronisations in between,
reproduces the eager maps bit for bit."""
import math

import numpy as np
import pytest

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


def test_graph_capture_of_run_and_noise_batch(ctx):
    import torch
    from paper_2609_11181_amd import lib as L

    nside = 256
    rng = np.random.default_rng(31)
    pix = np.arange(hp.npix(nside))
    v = hp.pix2vec(nside, pix)
    pix = pix[v[:, 0] > math.cos(12 * DEG)]
    W = rng.poisson(20, pix.size).astype(np.float32)
    G1 = (rng.normal(0, 0.26, pix.size) * np.sqrt(W)).astype(np.float32)
    G2 = (rng.normal(0, 0.26, pix.size) * np.sqrt(W)).astype(np.float32)
    E2 = (G1.astype(np.float64) ** 2 + G2.astype(np.float64) ** 2).astype(np.float32)
    data = ctx.pixel_map(nside, pix, W, G1, G2, E2)
    ths = [30 * ARCMIN, 60 * ARCMIN]
    fid = ctx.filter(L.FILTER_TANH)
    plan = ctx.plan(data, L.VAR_PIXEL, nside, pix, ths, [fid, fid])
    n_real = 40
    u = torch.from_numpy(noise_angles(5, 0, n_real, pix.size)).cuda()
    # eager calls (they also build the schedules)
    ref_run = plan.run(L.NORM_SUMMED_PIXCOUNT).clone()
    ref_noise = plan.noise_batch(u, n_real, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3).clone()
    torch.cuda.synchronize()
    out_run = torch.empty_like(ref_run)
    out_noise = torch.empty_like(ref_noise)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(L.NORM_SUMMED_PIXCOUNT, out_run)
        plan.noise_batch(u, n_real, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3, out_noise)
    for rep in range(3):
        out_run.fill_(float("nan"))
        out_noise.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_run, ref_run), rep
        assert torch.equal(out_noise, ref_noise), rep
        del junk
