"""smart_mixed_batch_noalloc (fixed per-device workspace, no device
allocation) through the C ABI: the same maps as smart_mixed_batch, bit for
bit, on two calls in a row (the second with fewer and smaller plans, so it
reuses the workspace the first one left), with the averaged normalisation
once the records exist, and a clean refusal beyond the workspace's job
limit."""
import math

import numpy as np
import pytest

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


def _map(nside, cap, seed):
    rng = np.random.default_rng(seed)
    pix = np.arange(hp.npix(nside))
    pix = pix[hp.pix2vec(nside, pix)[:, 0] > math.cos(cap)]
    W = rng.poisson(15, pix.size).astype(np.float32)
    G1 = (rng.normal(0, 0.26, pix.size) * np.sqrt(W)).astype(np.float32)
    G2 = (rng.normal(0, 0.26, pix.size) * np.sqrt(W)).astype(np.float32)
    return pix, W, G1, G2, (W * 0.1352).astype(np.float32)


def _plans(ctx, specs):
    from paper_2609_11181_amd import lib as L

    plans, keep = [], []
    for nside, cap, ths, seed in specs:
        pix, W, G1, G2, E2 = _map(nside, cap, seed)
        d = ctx.pixel_map(nside, pix, W, G1, G2, E2)
        fids = [ctx.filter(L.FILTER_TANH if k % 2 == 0 else L.FILTER_POLY) for k in range(len(ths))]
        prec = L.PREC_FP32_OUT64 if seed % 2 else L.PREC_FP32_GEO64
        plans.append(ctx.plan(d, L.VAR_PIXEL, nside, pix, ths, fids, precision=prec))
        keep.append(d)
    return plans, keep


def _both(ctx, plans, norms):
    import torch

    ref = [p.empty_out() for p in plans]
    ctx.mixed_batch(plans, norms, ref)
    got = [torch.full_like(r, float("nan")) for r in ref]
    ctx.mixed_batch(plans, norms, got, noalloc=True)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    return got


def test_noalloc_matches_mixed_batch_twice(ctx):
    from paper_2609_11181_amd import lib as L

    big, keep1 = _plans(ctx, [(256, 12 * DEG, [20 * ARCMIN, 60 * ARCMIN], 1), (512, 6 * DEG, [8 * ARCMIN], 2),
                              (128, 30 * DEG, [2 * DEG, 40 * ARCMIN, 3 * DEG], 3)])
    _both(ctx, big, [L.NORM_SUMMED_PIXCOUNT, L.NORM_SUMMED_CAP, L.NORM_RAW])
    small, keep2 = _plans(ctx, [(64, 20 * DEG, [3 * DEG], 4)])
    _both(ctx, small, [L.NORM_SUMMED_PIXCOUNT])
    # averaged normalisation: refused until an allocating call built the records
    import torch

    out = small[0].empty_out()
    with pytest.raises(L.SmartError):
        ctx.mixed_batch(small, [L.NORM_AVERAGED], [out], noalloc=True)
    small[0].run(L.NORM_AVERAGED)
    _both(ctx, small, [L.NORM_AVERAGED])
    torch.cuda.synchronize()


def test_noalloc_rejects_beyond_its_workspace(ctx):
    """513 jobs (plan-scale pairs) exceed the 512 the workspace holds."""
    import torch
    from paper_2609_11181_amd import lib as L

    pix, W, G1, G2, E2 = _map(16, 40 * DEG, 9)
    d = ctx.pixel_map(16, pix, W, G1, G2, E2)
    fid = ctx.filter(L.FILTER_TANH)
    plans = [ctx.plan(d, L.VAR_PIXEL, 16, pix, [5 * DEG + 0.001 * k for k in range(57)], [fid] * 57)
             for _ in range(9)]
    outs = [p.empty_out() for p in plans]
    with pytest.raises(L.SmartError, match="exceed the fixed workspace"):
        ctx.mixed_batch(plans, [L.NORM_RAW] * 9, outs, noalloc=True)
    ctx.mixed_batch(plans[:8], [L.NORM_RAW] * 8, outs[:8], noalloc=True)  # 456 jobs fit
    torch.cuda.synchronize()
