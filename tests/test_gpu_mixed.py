"""Mixed batches (smart_mixed_batch): many plans with different NSIDE, field
sizes, apertures and filters in one persistent launch give exactly the maps
of the single-plan runs, and those match the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import aperture as A
from oracle import filters as F
from synth import ARCMIN, DEG, PixelMapSpec, pixel_level_map
from synth.generators import cap_radius_from_area

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


INSTANCES = [
    # nside, area deg2, theta_ap arcmin (one or two scales), filter
    (128, 400.0, [60.0, 150.0], F.TANH),
    (256, 150.0, [20.0], F.POLY),
    (64, 3000.0, [240.0], F.TANH),
    (256, 40.0, [45.0, 10.0], F.TANH),
    (128, 900.0, [90.0], F.POLY),
    (512, 30.0, [8.0], F.TANH),
    (1024, 200.0, [10.0], F.TANH),
    (512, 600.0, [20.0, 40.0], F.POLY),
    # belt windows of about 65 members per ring: the belt kernels' wider LDS spans
    (256, 3000.0, [660.0], F.TANH),
]


def test_mixed_batch_equals_single_runs_and_oracle(ctx):
    import torch
    from paper_2609_11181_amd import lib as L

    plans, outs_single, maps = [], [], []
    for k, (nside, area, ths, kind) in enumerate(INSTANCES):
        m = pixel_level_map(PixelMapSpec(nside=nside, cap_radius=cap_radius_from_area(area), density_arcmin2=14.0,
                                         halos_per_deg2=0.5, seed=100 + k))
        data = ctx.pixel_map(nside, m["pix"], m["W"], m["G1"], m["G2"], m["E2"])
        th = [t * ARCMIN for t in ths]
        plan = ctx.plan(data, L.VAR_PIXEL, nside, m["pix"], th, [ctx.filter(kind)] * len(th))
        outs_single.append(plan.run(L.NORM_SUMMED_PIXCOUNT).cpu().numpy())
        if ths == [660.0]:  # the wide-window instance runs on the belt path
            assert plan.tiles(0)[0].shape[0] > 0
        plans.append(plan)
        maps.append((m, th, kind))
    outs = [p.empty_out().fill_(np.nan) for p in plans]
    ctx.mixed_batch(plans, [L.NORM_SUMMED_PIXCOUNT] * len(plans), outs)
    torch.cuda.synchronize()
    for k, (o, s) in enumerate(zip(outs, outs_single)):
        assert np.array_equal(o.cpu().numpy(), s), k
    # oracle on a sample of every instance
    rng = np.random.default_rng(0)
    for k, (m, th, kind) in enumerate(maps):
        pick = np.sort(rng.choice(m["pix"].size, min(400, m["pix"].size), replace=False))
        for si, t in enumerate(th):
            ref = A.aperture_mass_pixel(m, m["pix"][pick], t, kind)
            ok = ~ref["tie"]
            rms = math.sqrt(np.mean(ref["M_E"][ok] ** 2))
            diff = np.max(np.abs(outs_single[k][si, 0][pick][ok] - ref["M_E"][ok]))
            if rms == 0.0:  # aperture inside one pixel: only the coincident centre, no shear term
                assert diff == 0.0, (k, si)
                continue
            assert diff / rms <= 1e-6, (k, si, diff / rms)
