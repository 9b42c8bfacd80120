"""Benchmark of the spherical aperture-mass hot path on one MI355X.

Workload (default): the pixel-based variant at NSIDE 4096 over a 15000 deg^2
field centred on the equator, 30 galaxies/arcmin^2 binned per pixel with
shape noise 0.26 and SIS signal from 20000 halos; maps at every field pixel
for theta_ap = 5', 10', 20' with the NFW-like (tanh) filter, FP32 filter and
weight sums with FP64 geometry.

One step = the whole path on the resident input: pixel-map ingest into the
ring-range layout, plan creation (output list copy and validation) and the
pair-sum kernels of the three scales (disc windows, geometry, filter,
accumulation, normalisation). Inputs sit in HBM before the timed region.

Prints one JSON line. `value` = pair evaluations per second (pairs of an
aperture centre and an occupied source pixel inside the aperture, summed
over the three scales). `roofline` reports the dominant kernel (the 20'
scale) against the plain-ALU peak; `cpu_baseline` times the FP64 oracle on a
bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

ARCMIN = math.pi / 10800.0
# algorithmic work of one pair evaluation, in lane operations: FP64 chord and
# test (7), FP32 rotation, filter and accumulation (24)
OPS_PER_PAIR = 31
# belt items: the pair coefficients come from per-ring tables, so a pair costs
# its contraction only (4 FP64 FMA for E/B, 1 FP32 FMA for V)
BELT_OPS_PER_PAIR = 5
# plain-ALU peak: 256 CUs x 64 lanes x 2.4 GHz, one lane op per clock
ALU_PEAK = 256 * 64 * 2.4e9


def belt_pairs_of(plan, n_out_ch, scale=0):
    """Pairs of a plan scale's belt items: its N channel (n_out_ch, a device
    tensor of the scale's outputs) summed over the list positions that the
    belt items cover; the rest of the scale's pairs are general-tile pairs."""
    import torch

    belt, _ = plan.tiles(scale)
    n = n_out_ch.shape[0]
    mark = torch.zeros(n + 1, dtype=torch.int32, device=n_out_ch.device)
    if belt.shape[0]:
        b = belt.long()
        mark.index_add_(0, b[:, 0], torch.ones_like(b[:, 0], dtype=torch.int32))
        mark.index_add_(0, b[:, 0] + b[:, 1], -torch.ones_like(b[:, 0], dtype=torch.int32))
    sel = torch.cumsum(mark[:n], 0) > 0
    return float(n_out_ch.double()[sel].sum())
# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE (x2.0) and WRITE_SIZE (x1.0)
# counter runs of the default workload, double maps (profiles/pixel_kernels_nside4096_15000deg2_3scales.md,
# which names the source version it was measured on); valid for that kernel version and workload only
TRAFFIC_BYTES = {"k_pixel_f32 (20 arcmin)": 1.689e10}
TRAFFIC_SOURCE = "profiles/pixel_kernels_nside4096_15000deg2_3scales.md"
# counter-measured utilisation of the same kernel versions (rocprofv3 SQ counters of the committed profiles,
# which name the source version): VALU issue share = SQ_INSTS_VALU / (duration x 256 CU x 2.4 GHz); MFMA busy =
# SQ_VALU_MFMA_BUSY_CYCLES / (4 x CU-cycles). Valid for those kernel versions and workloads only.
COUNTERS = {
    "k_pixel_f32 (20 arcmin)": {"valu_issue_share": 0.88, "source": TRAFFIC_SOURCE},
    "k_galaxy_f32": {"valu_issue_share": 0.66, "fetch_bytes": 4.4e10,
                     "source": "profiles/galaxy_kernel_5e7gal_1000deg2_nside2048_10arcmin.md"},
    "k_noise_stack": {"mfma_busy_5_10_20_arcmin": [0.21, 0.31, 0.37], "valu_per_mfma_5_10_20_arcmin": [10.8, 7.6, 6.2],
                      "source": "profiles/noise_stack_nside2048_5000deg2_256real.md"},
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-outputs", type=int, default=32000)
    p.add_argument("--area", type=float, default=15000.0, help="field area in deg^2")
    p.add_argument("--nside", type=int, default=4096)
    p.add_argument("--no-batched", action="store_true", help="skip the batched noise-realisation leg")
    p.add_argument("--only-batched", action="store_true", help="run only the batched noise-realisation leg")
    p.add_argument("--n-real", type=int, default=256, help="realisations of the batched leg")
    p.add_argument("--plain-real", type=int, default=8, help="realisations timed on the plain FP32 path")
    p.add_argument("--no-tune", action="store_true", help="keep the default launch choices (no autotuning)")
    p.add_argument("--no-mixed", action="store_true", help="skip the uneven mixed-batch leg")
    p.add_argument("--no-averaged", action="store_true", help="skip the averaged-normalisation leg")
    p.add_argument("--only-mixed", action="store_true", help="run only the uneven mixed-batch leg")
    p.add_argument("--no-config2", action="store_true", help="skip the brute-force galaxy-variant leg")
    p.add_argument("--only-config2", action="store_true", help="run only the brute-force galaxy-variant leg")
    p.add_argument("--mixed-area-scale", type=float, default=1.0, help="scale of the mixed-batch cap areas")
    p.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                   help="only run a plain device copy of GIB GiB three times (HBM counter calibration)")
    return p.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_CPU_SUB = None  # sub-map shared with the forked oracle workers


def _oracle_chunk(task):
    from oracle import aperture as A
    from oracle import filters as F

    out_pix, th = task
    r = A.aperture_mass_pixel(_CPU_SUB, out_pix, th, F.TANH)
    return {k: r[k] for k in ("M_E", "M_B", "sigma", "W", "N", "tie")}


def cpu_baseline(pm, R, scales, n_out, workers, seed=11):
    """FP64 oracle on a patch of the same map: n_out apertures drawn in a
    2-degree disc at a random point of the field, with the input pixels that
    can reach them; the apertures are split over `workers` forked processes
    (the oracle itself is unchanged). Runs before the GPU is touched."""
    import multiprocessing as mp

    from oracle import healpix_ref as hp

    global _CPU_SUB
    nside = pm["nside"]
    rng = np.random.default_rng(seed)
    # patch centre: inside the field, away from its edge
    while True:
        ra0 = rng.uniform(-0.8 * R, 0.8 * R)
        dec0 = rng.uniform(-0.8 * R, 0.8 * R)
        if math.cos(dec0) * math.cos(ra0) > math.cos(0.8 * R):
            break
    c = np.array([math.cos(dec0) * math.cos(ra0), math.cos(dec0) * math.sin(ra0), math.sin(dec0)])
    # candidate pixels: rings within the patch band, then exact distance
    rt = hp.ring_table(nside)
    colat0 = math.pi / 2 - dec0
    patch = 2.0 * math.pi / 180
    reach = patch + max(scales) + 0.01
    colat = np.arctan2(rt["sin"], rt["z"])
    rings = np.nonzero(np.abs(colat - colat0) < reach)[0]
    lo = rt["first"][rings[0]]
    hi = rt["first"][rings[-1]] + rt["n"][rings[-1]]
    sel = (pm["pix"] >= lo) & (pm["pix"] < hi)
    pix = pm["pix"][sel]
    v = hp.pix2vec(nside, pix)
    d = np.arccos(np.clip(v @ c, -1, 1))
    keep = d < reach
    sub = {"nside": nside, "pix": pix[keep]}
    for k in ("W", "G1", "G2", "E2"):
        sub[k] = pm[k][sel][keep]
    inner = sub["pix"][d[keep] < patch]
    out_pix = np.sort(rng.choice(inner, min(n_out, inner.size), replace=False))
    _CPU_SUB = sub
    chunks = np.array_split(out_pix, workers)
    tasks = [(ch, th) for th in scales for ch in chunks]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_oracle_chunk, tasks, chunksize=1)
    dt = time.perf_counter() - t0
    refs, pairs = [], 0
    for k in range(len(scales)):
        ps = parts[k * workers:(k + 1) * workers]
        r = {key: np.concatenate([q[key] for q in ps]) for key in ps[0]}
        refs.append(r)
        pairs += int(r["N"].sum())
    _CPU_SUB = None
    # reference of the averaged-normalisation leg (not timed): the first
    # apertures of the sample at the smallest scale
    from oracle import aperture as A
    from oracle import filters as F

    avg_pix = out_pix[:1000]
    avg_ref = A.aperture_mass_pixel(sub, avg_pix, scales[0], F.TANH, norm=A.NORM_AVERAGED)
    return out_pix, refs, pairs, dt, (avg_pix, avg_ref)


def config2_leg(ctx, args):
    """Brute-force galaxy variant (Sect. 3.1): 5e7 galaxies in a 1000 deg^2
    cap (about 14 galaxies/arcmin^2, 500 SIS halos), maps at every NSIDE-2048
    pixel centre in the cap, theta_ap = 10', tanh filter, FP32 pair sums with
    FP64 geometry and double maps; catalogue partitioned at NSIDE 4096 (the
    partition only selects candidates; every galaxy gets the exact test).
    Also the sphS_posB / sphS_pos ratio on an NSIDE-2048 partition (posB
    selects the binning pixels centred in the aperture, Sect. 3.4)."""
    import torch

    from oracle import healpix_ref as hp
    from paper_2609_11181_amd import lib as L
    from synth import config2_catalogue

    t = time.perf_counter()
    cat, R = config2_catalogue()
    log(f"config-2 leg: generated {cat['ra'].size} galaxies in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda", 0)
    cols = [torch.from_numpy(cat[k]).to(dev) for k in ("ra", "dec", "g1", "g2", "w")]
    nside = 2048
    rt = hp.ring_table(nside)
    rings = np.nonzero(np.abs(np.arcsin(rt["z"])) < R)[0]
    pix = np.arange(rt["first"][rings[0]], rt["first"][rings[-1]] + rt["n"][rings[-1]])
    v = hp.pix2vec(nside, pix)
    out_pix = pix[v[:, 0] > math.cos(R)]
    th = 10 * ARCMIN
    fid = ctx.filter(L.FILTER_TANH)
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"workload": f"sphS_pos brute force, {cat['ra'].size:.3g} galaxies in a 1000 deg2 cap, "
                       f"{out_pix.size} NSIDE-2048 centres, theta_ap 10 arcmin, tanh filter, double maps"}

    def timed(plan, out, n=3):
        plan.run(L.NORM_SUMMED_CAP, out)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(n):
            plan.run(L.NORM_SUMMED_CAP, out)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / n

    data = ctx.bin_galaxies(*cols, nside_bin=4096)
    plan = ctx.plan(data, L.VAR_GALAXY, nside, out_pix, [th], [fid], precision=L.PREC_FP32_OUT64)
    out = plan.empty_out()
    ms = timed(plan, out)
    pairs = plan.last_pairs()
    achieved = pairs * OPS_PER_PAIR / (ms / 1e3)
    res.update({"run_ms": ms, "pairs": pairs, "pair_evals_per_s": pairs / (ms / 1e3),
                "roofline": {"bound": "alu", "kernel": "k_galaxy_f32", "achieved": achieved / 1e12,
                             "peak": ALU_PEAK / 1e12, "unit": "Tlane-op/s", "frac": achieved / ALU_PEAK,
                             "ops_per_pair": OPS_PER_PAIR, "counters": COUNTERS["k_galaxy_f32"]}})
    log(f"config-2: {ms:.2f} ms, {pairs:.4e} pairs, {pairs / (ms / 1e3):.3e} pair-evals/s")
    if not args.no_cpu:
        res.update(config2_accuracy(cat, R, out_pix, out[0].cpu().numpy(), th))
    del out
    plan.free()
    data.free()
    # posB against the brute force on the map's own NSIDE partition
    data2 = ctx.bin_galaxies(*cols, nside_bin=nside)
    for name, var in (("pos", L.VAR_GALAXY), ("posB", L.VAR_GALAXY_POSB)):
        p2 = ctx.plan(data2, var, nside, out_pix, [th], [fid], precision=L.PREC_FP32_OUT64)
        o2 = p2.empty_out()
        res[f"{name}_nside2048_partition_ms"] = timed(p2, o2)
        p2.free()
    res["posB_speedup_vs_pos"] = res["pos_nside2048_partition_ms"] / res["posB_nside2048_partition_ms"]
    res["posB_note"] = "the paper reports about 2x for posB over pos on its CPU (Table 2)"
    data2.free()
    del cols
    return res


def config2_accuracy(cat, R, out_pix, out, th, n_check=1024, seed=21):
    """Oracle on 768 apertures in a 1-degree patch inside the field and 256
    at its edge: max error over the whole-map RMS and the paper's relative
    difference (Sect. 5.1) per channel."""
    from oracle import aperture as A
    from oracle import filters as F
    from oracle import healpix_ref as hp

    rng = np.random.default_rng(seed)
    vo = hp.pix2vec(2048, out_pix)
    gv = A.radec2vec(cat["ra"], cat["dec"])
    sels, refs = [], []
    for anchor, n in ((A.radec2vec(0.1, -0.05), 3 * n_check // 4), (A.radec2vec(R - 0.2 * math.pi / 180, 0.0),
                                                                     n_check // 4)):
        near = np.nonzero(vo @ anchor > math.cos(math.pi / 180))[0]
        sel = np.sort(rng.choice(near, n, replace=False))
        keep = gv @ anchor > math.cos(math.pi / 180 + th + 0.002)
        sub = {k: cat[k][keep] for k in ("ra", "dec", "g1", "g2", "w")}
        ra, dec = hp.pix2radec(2048, out_pix[sel])
        sels.append(sel)
        refs.append(A.aperture_mass_galaxy(sub, ra, dec, th, F.TANH))
    sel = np.concatenate(sels)
    errs, eps = {}, {}
    for ch, key in enumerate(("M_E", "M_B", "sigma")):
        ref = np.concatenate([r[key] for r in refs])
        ok = ~np.concatenate([r["tie"] for r in refs])
        full = out[ch]
        d = out[ch][sel][ok] - ref[ok]
        errs[key] = float(np.max(np.abs(d)) / math.sqrt(np.mean(full * full)))
        eps[key] = {"mean": float(np.mean(d / np.std(full))), "std": float(np.std(d / np.std(full)))}
    return {"max_rel_err_vs_oracle": errs, "epsilon_vs_oracle": eps,
            "accuracy_sample": f"{sel.size} apertures (768 in a 1-degree patch, 256 at the field edge), "
                               "error over the whole-map RMS"}


def batched_leg(ctx, args):
    """Shape-noise realisations: galaxies of a 5000 deg^2 field (config-2
    statistics, about 2.5e8 galaxies) binned at NSIDE 2048, 256 realisations
    x 3 scales (5', 10', 20') = 768 noise maps, split-BF16 MFMA path against
    the plain FP32 path (timed on a few realisations)."""
    import torch

    from paper_2609_11181_amd import lib as L
    from synth import config4_catalogue

    t = time.perf_counter()
    cat, R4 = config4_catalogue()
    log(f"batched leg: generated {cat['ra'].size} galaxies in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda", 0)
    cols = [torch.from_numpy(cat[k]).to(dev) for k in ("ra", "dec", "g1", "g2")]
    del cat
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream(dev)
    # the first call also allocates the handle's and the sort's device
    # blocks; the second reuses them from the library's block cache (a
    # pipeline that bins one catalogue after another)
    t = time.perf_counter()
    data = ctx.bin_galaxies(*cols, None, nside_bin=2048, pixel_sums=True)
    torch.cuda.synchronize()
    bin_cold_ms = (time.perf_counter() - t) * 1e3
    data.free()
    ev0.record(stream)
    data = ctx.bin_galaxies(*cols, None, nside_bin=2048, pixel_sums=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    bin_ms = ev0.elapsed_time(ev1)
    n_gal = cols[0].numel()
    src = data.sources()
    n_src = src.numel()
    scales = [5 * ARCMIN, 10 * ARCMIN, 20 * ARCMIN]
    fid = ctx.filter(L.FILTER_TANH)
    plan = ctx.plan(data, L.VAR_PIXEL, 2048, src, scales, [fid] * 3)
    gen = torch.Generator(device=dev)
    gen.manual_seed(4)
    R = args.n_real
    u = torch.rand((R, n_src), generator=gen, device=dev, dtype=torch.float32)
    out = torch.empty(3, R, 2, n_src, dtype=torch.float32, device=dev)
    plan.noise_batch(u, R, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3, out)  # warm-up
    torch.cuda.synchronize()
    ev0.record(stream)
    plan.noise_batch(u, R, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_b = ev0.elapsed_time(ev1) / 1e3
    # the same batch captured once in a HIP graph and replayed (the schedule
    # was built by the first call; the launches allocate nothing)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.noise_batch(u, R, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3, out)
    graph.replay()
    torch.cuda.synchronize()
    ev0.record(stream)
    graph.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_graph = ev0.elapsed_time(ev1) / 1e3
    del graph
    # pairs of one realisation set (N summed over centres and scales)
    main = plan.run(L.NORM_SUMMED_PIXCOUNT)
    pairs1 = plan.last_pairs()
    Rp = args.plain_real
    outp = torch.empty(3, Rp, 2, n_src, dtype=torch.float32, device=dev)
    plan.noise_batch(u[:1], 1, L.NORM_SUMMED_PIXCOUNT, L.PREC_FP32_GEO64, torch.empty_like(outp[:, :1]))
    torch.cuda.synchronize()
    ev0.record(stream)
    plan.noise_batch(u[:Rp], Rp, L.NORM_SUMMED_PIXCOUNT, L.PREC_FP32_GEO64, outp)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_p = ev0.elapsed_time(ev1) / 1e3
    # galaxy-level realisations on the same plan: every galaxy rotated by its
    # own angle and the pixel sums re-formed, then the plain FP32 pair kernels
    ug = torch.rand((Rp, n_gal), generator=gen, device=dev, dtype=torch.float32)
    outg = torch.empty(3, Rp, 2, n_src, dtype=torch.float32, device=dev)
    plan.noise_galaxy_batch(ug[:1], 1, L.NORM_SUMMED_PIXCOUNT,
                            torch.empty_like(outg[:, :1]))  # allocates the rotation buffers
    torch.cuda.synchronize()
    ev0.record(stream)
    plan.noise_galaxy_batch(ug, Rp, L.NORM_SUMMED_PIXCOUNT, outg)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_g = ev0.elapsed_time(ev1) / 1e3
    del ug, outg
    # galaxy-level realisations on the matrix cores: per-galaxy angles drawn
    # on the device, the rotated pixel sums of each chunk of 32 realisations
    # contracted by the split-BF16x3 kernels (all R realisations)
    outs = torch.empty_like(out)  # `out` keeps the pixel-level maps for the accuracy check
    plan.noise_galaxy_seeded(11, 0, R, L.NORM_SUMMED_PIXCOUNT, out=outs)  # warm-up
    torch.cuda.synchronize()
    ev0.record(stream)
    plan.noise_galaxy_seeded(11, 0, R, L.NORM_SUMMED_PIXCOUNT, out=outs)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_gs = ev0.elapsed_time(ev1) / 1e3
    del outs
    # sphS_pixB: the same catalogue's occupied pixels at their barycentres,
    # galaxy-variant FP32 plan with the pixel centres as outputs
    ev0.record(stream)
    bdata = data.barycentre()
    ev1.record(stream)
    torch.cuda.synchronize()
    bary_build_ms = ev0.elapsed_time(ev1)
    bplan = ctx.plan(bdata, L.VAR_GALAXY, 2048, src, scales, [fid] * 3)
    bout = bplan.run(L.NORM_SUMMED_PIXCOUNT)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(3):
        bplan.run(L.NORM_SUMMED_PIXCOUNT, bout)
    ev1.record(stream)
    torch.cuda.synchronize()
    bary_ms = ev0.elapsed_time(ev1) / 3
    bary_pairs = bplan.last_pairs()
    barycentre = {
        "workload": f"sphS_pixB: {n_src} occupied pixels at their barycentres, outputs at the pixel centres, "
                    "3 scales (5/10/20 arcmin), tanh filter",
        "build_ms": bary_build_ms,
        "run_ms": bary_ms,
        "pairs": bary_pairs,
        "pair_evals_per_s": bary_pairs / (bary_ms / 1e3),
    }
    bplan.free()
    bdata.free()
    del bout
    # sphS_posB and the brute force on the same catalogue, for the first
    # 2^18 occupied pixels as outputs (the brute force over all 6.1e6 would
    # take seconds)
    sub = src[: 1 << 18]
    posb = {}
    for name, var in (("posB", L.VAR_GALAXY_POSB), ("pos", L.VAR_GALAXY)):
        gplan = ctx.plan(data, var, 2048, sub, scales, [fid] * 3)
        gout = gplan.run(L.NORM_SUMMED_CAP)
        torch.cuda.synchronize()
        ev0.record(stream)
        gplan.run(L.NORM_SUMMED_CAP, gout)
        ev1.record(stream)
        torch.cuda.synchronize()
        g_ms = ev0.elapsed_time(ev1)
        g_pairs = gplan.last_pairs()
        posb[name] = {"run_ms": g_ms, "members": g_pairs, "member_evals_per_s": g_pairs / (g_ms / 1e3)}
        gplan.free()
        del gout
    posb["workload"] = (f"galaxy-level variants over {n_gal:.3g} galaxies (NSIDE-2048 partition), "
                        f"{sub.numel()} output pixels, 3 scales (5/10/20 arcmin), tanh filter")
    table3 = table3_leg(ctx, cols, data, fid)
    log(f"table 3: {json.dumps({k: v for k, v in table3.items() if k.startswith('nside') or k == 'jarvis_4arcmin'})}")
    del cols
    maps_b = 3 * R / t_b
    maps_p = 3 * Rp / t_p
    flops = 8.0 * pairs1 * R  # one complex multiply-add per pair and realisation
    res = {
        "workload": f"{n_gal:.3g} galaxies in a 5000 deg2 field binned at NSIDE 2048 ({n_src} pixels), "
                    f"{R} realisations x 3 scales (5/10/20 arcmin), tanh filter",
        "maps": 3 * R,
        "bf16x3_s": t_b,
        "bf16x3_maps_per_s": maps_b,
        "bf16x3_graph_replay_s": t_graph,
        "bf16x3_graph_maps_per_s": 3 * R / t_graph,
        "plain_fp32_maps_per_s": maps_p,
        "plain_fp32_timed_realisations": Rp,
        "galaxy_level_fp32_maps_per_s": 3 * Rp / t_g,
        "galaxy_level_note": "smart_noise_galaxy_batch: per-galaxy rotation, re-binned pixel sums, plain FP32 "
                             "pair kernels; same realisation count as the plain pixel-level timing",
        "galaxy_level_bf16x3_s": t_gs,
        "galaxy_level_bf16x3_maps_per_s": 3 * R / t_gs,
        "galaxy_level_bf16x3_note": "smart_noise_galaxy_seeded: Philox4x32-10 angles per galaxy drawn on the "
                                    "device, rotated pixel sums per chunk of 32 realisations, split-BF16x3 "
                                    "stack; all realisations of the leg",
        "speedup_vs_plain": maps_b / maps_p,
        "realisation_pair_evals_per_s": pairs1 * R / t_b,
        "mfma": {"bound": "mfma", "achieved": flops / t_b / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                 "frac": flops / t_b / 2.5e15,
                 "note": "algorithmic 8 flop per (pair, realisation); split-BF16 issues 3 products per term",
                 "counters": COUNTERS["k_noise_stack"]},
        "binning_ms": bin_ms,
        "binning_first_call_ms": bin_cold_ms,
        "binning_gb_per_s": (n_gal * (28 + 56) + 12 * 2048 ** 2 * 8) / (bin_ms / 1e3) / 1e9,
        "binning_note": "algorithmic bytes: 28 read + 56 written per galaxy (sorted unit vector with right "
                        "ascension, shear and weight, catalogue order) + 8 per pixel of the offset table, over "
                        "the time of a second "
                        "smart_bin_galaxies call (device blocks from the library's cache; the first call, which "
                        "allocates them, is binning_first_call_ms, host clock)",
        "barycentre": barycentre,
        "galaxy_variants": posb,
        "table3_epsilon": table3,
    }
    if not args.no_cpu:
        res.update(batched_accuracy(data, src, u, out, outp, scales, R))
    return res


def jarvis_table(theta_s_over_ap, n=4097):
    """Samples of the aperture filter of Jarvis et al. (2004) (the Gaussian
    profile of Crittenden et al. 2002, Q(theta) proportional to
    theta^2 exp(-theta^2 / (2 theta_s^2))) at n uniform nodes of x =
    theta / theta_ap on [0, 1], for a table filter truncated at theta_ap; the
    overall factor cancels in Table 3's normalised differences."""
    x = np.linspace(0.0, 1.0, n) / theta_s_over_ap
    return (x * x * np.exp(-0.5 * x * x)).tolist()


def table3_leg(ctx, cols, data2048, fid, th=10 * ARCMIN):
    """The paper's Table 3 comparison (Sect. 5.1) on the synthetic catalogue:
    eps_X = (M_E^X - M_E^pos) / std(M_E^pos) for X = sphS_pix, sphS_pixB and
    sphS_posB against the brute force sphS_pos, mean and standard deviation
    over the map, at NSIDE 2048 (every occupied pixel within 8 degrees of the
    field centre) and NSIDE 4096 (within 4 degrees; the catalogue binned
    again), summed approach; with the tanh filter at 10' (the workloads'
    filter) and with the filter the paper uses for its table (Jarvis et al.
    2004 at a 4' scale, here truncated at 5 x 4' = 20' and passed as a table
    filter)."""
    import torch

    from oracle import healpix_ref as hp
    from paper_2609_11181_amd import lib as L

    theta_s = 4 * ARCMIN
    fid_j = ctx.filter(L.FILTER_TABLE, jarvis_table(0.2))
    filters = (("tanh_10arcmin", fid, th), ("jarvis_4arcmin", fid_j, 5 * theta_s))
    out = {name: {} for name, _, _ in filters}
    for nside, rad in ((2048, 8.0), (4096, 4.0)):
        data = data2048 if nside == 2048 else ctx.bin_galaxies(*cols, None, nside_bin=4096, pixel_sums=True)
        srcs = data.sources().cpu().numpy()
        sel = srcs[hp.pix2vec(nside, srcs)[:, 0] > math.cos(math.radians(rad))]
        bdata = data.barycentre()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        for fname, f, tha in filters:
            maps, ms = {}, {}
            for name, d, var, norm in (("pos", data, L.VAR_GALAXY, L.NORM_SUMMED_CAP),
                                       ("pix", data, L.VAR_PIXEL, L.NORM_SUMMED_PIXCOUNT),
                                       ("pixB", bdata, L.VAR_GALAXY, L.NORM_SUMMED_PIXCOUNT),
                                       ("posB", data, L.VAR_GALAXY_POSB, L.NORM_SUMMED_CAP)):
                plan = ctx.plan(d, var, nside, sel, [tha], [f], precision=L.PREC_FP32_OUT64)
                o = plan.run(norm)
                torch.cuda.synchronize()
                ev0.record(stream)
                plan.run(norm, o)
                ev1.record(stream)
                torch.cuda.synchronize()
                ms[name] = ev0.elapsed_time(ev1)
                maps[name] = o[0, 0].cpu().numpy()
                plan.free()
            ref = maps["pos"]
            sd = float(np.std(ref))
            out[fname][f"nside{nside}"] = {
                "outputs": int(sel.size),
                **{f"eps_{k}": {"mean": float(np.mean((maps[k] - ref) / sd)),
                                "std": float(np.std((maps[k] - ref) / sd))}
                   for k in ("pix", "pixB", "posB")},
                "run_ms": ms,
            }
        bdata.free()
        if nside != 2048:
            data.free()
    res = dict(out["tanh_10arcmin"])
    res["jarvis_4arcmin"] = out["jarvis_4arcmin"]
    res["workload"] = ("eps of sphS_pix / sphS_pixB / sphS_posB against sphS_pos (Table 3 definition) on the "
                       "2.5e8-galaxy catalogue (13.9 gal/arcmin2): tanh filter at 10 arcmin (top-level nside keys) "
                       "and the Jarvis et al. (2004) filter at theta_s = 4 arcmin truncated at 20 arcmin "
                       "(jarvis_4arcmin)")
    res["paper_table3"] = {"nside2048": {"pix": [2.00e-5, 3.30e-2], "pixB": [2.00e-5, 3.22e-2], "posB": [1.54e-6, 8.02e-3]},
                           "nside4096": {"pix": [4.29e-6, 8.58e-3], "pixB": [4.36e-6, 7.51e-3],
                                         "posB": [-3.62e-7, 3.53e-3]},
                           "note": "mean, std on the paper's mock (27 gal/arcmin2, Jarvis filter at 4 arcmin)"}
    return res


def batched_accuracy(data, src, u, out, outp, scales, R, n_check=512, seed=12):
    """Oracle check of realisations 0, 1 and R-1 on a random sample of
    centres inside a 1-degree patch."""
    from oracle import aperture as A
    from oracle import filters as F
    from oracle import healpix_ref as hp

    inf = data.info()
    _, _, sums = data.export(sums=True)
    srcs = src.cpu().numpy()
    s = sums.cpu().numpy()[srcs - inf["pix_first"]]
    rng = np.random.default_rng(seed)
    c_pix = srcs[rng.integers(0, srcs.size)]
    c = hp.pix2vec(2048, np.array([c_pix]))[0]
    v = hp.pix2vec(2048, srcs)
    d = np.arccos(np.clip(v @ c, -1, 1))
    near = d < math.radians(1.0) + max(scales) + 0.01
    inner = np.nonzero(d < math.radians(1.0))[0]
    pick = np.sort(rng.choice(inner, min(n_check, inner.size), replace=False))
    out_pix = srcs[pick]
    sub = {"nside": 2048, "pix": srcs[near], "W": s[near, 2], "G1": s[near, 0], "G2": s[near, 1], "E2": s[near, 3]}
    errs_b, errs_p = [], []
    ob = out.cpu().numpy()
    op = outp.cpu().numpy()
    for r in (0, 1, R - 1):
        ur = u[r].cpu().numpy()[near]
        G1, G2 = A.rotate_realisation(sub["G1"], sub["G2"], ur)
        mr = dict(sub, G1=G1, G2=G2)
        for k, th in enumerate(scales):
            ref = A.aperture_mass_pixel(mr, out_pix, th, F.TANH)
            ok = ~ref["tie"]
            for e, key in enumerate(("M_E", "M_B")):
                rms = math.sqrt(np.mean(ref[key][ok] ** 2))
                errs_b.append(float(np.max(np.abs(ob[k, r, e][pick][ok] - ref[key][ok])) / rms))
                if r < op.shape[1]:
                    errs_p.append(float(np.max(np.abs(op[k, r, e][pick][ok] - ref[key][ok])) / rms))
    return {"max_rel_err_bf16x3": max(errs_b), "max_rel_err_plain_fp32": max(errs_p) if errs_p else None,
            "accuracy_sample": f"{pick.size} centres x 3 scales x realisations (0, 1, {R - 1}), E and B"}


def mixed_leg(ctx, args):
    """Uneven mixed batch: the 64 instances of synth.config5_instances (NSIDE,
    cap area, aperture and filter drawn per instance; pixel-level maps with
    config-2 statistics, 13.9 gal/arcmin^2 and 0.5 halos/deg^2), all plans in
    one smart_mixed_batch launch, against the same plans run one by one."""
    import torch

    from paper_2609_11181_amd import lib as L
    from synth import PixelMapSpec, config5_instances, pixel_level_map
    from synth.generators import cap_radius_from_area

    dev = torch.device("cuda", 0)
    inst = config5_instances()
    t = time.perf_counter()
    maps, plans, outs = [], [], []
    for k, d in enumerate(inst):
        R = cap_radius_from_area(d["area_deg2"] * args.mixed_area_scale)
        m = pixel_level_map(PixelMapSpec(nside=d["nside"], cap_radius=R, density_arcmin2=13.9, halos_per_deg2=0.5,
                                         seed=d["seed"]))
        pix = torch.from_numpy(m["pix"]).to(dev)
        data = ctx.pixel_map(d["nside"], pix, *[torch.from_numpy(m[c]).to(dev) for c in ("W", "G1", "G2", "E2")])
        fid = ctx.filter(L.FILTER_POLY if d["filter"] == 0 else L.FILTER_TANH)
        plan = ctx.plan(data, L.VAR_PIXEL, d["nside"], pix, [d["theta_ap"]], [fid])
        plans.append(plan)
        outs.append(plan.empty_out())
        maps.append(m)
    log(f"mixed leg: {sum(m['pix'].size for m in maps)} pixels in 64 maps, generated and planned in "
        f"{time.perf_counter() - t:.1f}s")
    norms = [L.NORM_SUMMED_PIXCOUNT] * len(plans)
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.mixed_batch(plans, norms, outs)  # warm-up
    torch.cuda.synchronize()
    ev0.record(stream)
    ctx.mixed_batch(plans, norms, outs)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_mix = ev0.elapsed_time(ev1) / 1e3
    ev0.record(stream)
    for p, o in zip(plans, outs):
        p.run(L.NORM_SUMMED_PIXCOUNT, o)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_seq = ev0.elapsed_time(ev1) / 1e3
    ctx.mixed_batch(plans, norms, outs)
    pairs = float(sum(float(o[0, 4].double().sum()) for o in outs))
    # ideal work: each pair at the algorithmic lane-op count of the kernel form
    # that runs it (belt items 5, general tiles 31)
    belt = sum(belt_pairs_of(p, o[0, 4]) for p, o in zip(plans, outs))
    ideal_ops = belt * BELT_OPS_PER_PAIR + (pairs - belt) * OPS_PER_PAIR
    res = {
        "workload": f"64 pixel maps (NSIDE 512-4096, caps 100-15000 deg2 x {args.mixed_area_scale:g}, "
                    "theta_ap 2-40 arcmin, both filters), one persistent launch",
        "pixels": int(sum(m["pix"].size for m in maps)),
        "pairs": pairs,
        "mixed_ms": t_mix * 1e3,
        "pair_evals_per_s": pairs / t_mix,
        "one_by_one_ms": t_seq * 1e3,
        "belt_pairs": belt,
        "scheduler_efficiency": ideal_ops / (t_mix * ALU_PEAK),
        "scheduler_efficiency_note": "sum of the jobs' ideal times (belt-item pairs x 5 and general-tile pairs x 31 "
                                     "lane-ops at the ALU peak) over the launch's makespan",
    }
    if not args.no_cpu:
        res.update(mixed_accuracy(inst, maps, outs))
    return res


def mixed_accuracy(inst, maps, outs, n_check=256, seed=13):
    """Oracle check of every instance on n_check centres around a random
    pixel of its field (the oracle sees the pixels within reach)."""
    from oracle import aperture as A
    from oracle import filters as F
    from oracle import healpix_ref as hp

    rng = np.random.default_rng(seed)
    errs = []
    for d, m, o in zip(inst, maps, outs):
        nside = d["nside"]
        anchor = m["pix"][rng.integers(0, m["pix"].size)]
        a = hp.pix2vec(nside, np.array([anchor]))[0]
        # candidates: rings within reach of the anchor, then exact distance
        rt = hp.ring_table(nside)
        colat = np.arctan2(rt["sin"], rt["z"])
        reach = 0.5 * math.pi / 180 + d["theta_ap"] + 0.01
        rings = np.nonzero(np.abs(colat - math.acos(a[2])) < reach)[0]
        lo = rt["first"][rings[0]]
        hi = rt["first"][rings[-1]] + rt["n"][rings[-1]]
        sel = np.nonzero((m["pix"] >= lo) & (m["pix"] < hi))[0]
        v = hp.pix2vec(nside, m["pix"][sel])
        dist = np.arccos(np.clip(v @ a, -1, 1))
        near = sel[dist < reach]
        sub = {"nside": nside, "pix": m["pix"][near]}
        for c in ("W", "G1", "G2", "E2"):
            sub[c] = m[c][near]
        inner = sel[dist < 0.5 * math.pi / 180]
        pick = np.sort(rng.choice(inner, min(n_check, inner.size), replace=False))
        ref = A.aperture_mass_pixel(sub, m["pix"][pick], d["theta_ap"], F.POLY if d["filter"] == 0 else F.TANH)
        ok = ~ref["tie"]
        g = o[0, 0].cpu().numpy()[pick].astype(np.float64)
        rms = math.sqrt(np.mean(ref["M_E"][ok] ** 2))
        diff = float(np.max(np.abs(g[ok] - ref["M_E"][ok])))
        errs.append(diff / rms if rms > 0 else diff)
    return {"per_instance_max_rel_err": errs, "max_rel_err": max(errs),
            "accuracy_sample": f"{n_check} centres within 0.5 deg of a random pixel of each instance, M_E"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {n * 4} bytes x 3 (read {n * 4} B + write {n * 4} B per copy)")
        return

    from synth import config3_pixelmap

    if not (args.only_batched or args.only_mixed or args.only_config2):
        t = time.perf_counter()
        pm, R = config3_pixelmap(area_deg2=args.area, nside=args.nside)
        log(f"generated {pm['pix'].size} pixels in {time.perf_counter() - t:.1f}s")
        scales = [5 * ARCMIN, 10 * ARCMIN, 20 * ARCMIN]
        cpu = None
        if not args.no_cpu:  # on the host cores, before the GPU is touched (the workers are forked)
            workers = max(1, min(len(os.sched_getaffinity(0)), 16))  # the host CPU share of one GPU is 16 cores
            cpu = cpu_baseline(pm, R, scales, args.cpu_outputs, workers) + (workers,)
            log(f"oracle baseline: {cpu[2]} pairs in {cpu[3]:.1f}s on {workers} processes")

    from paper_2609_11181_amd import api
    from paper_2609_11181_amd import lib as L

    if args.only_batched:
        print(json.dumps({"batched": batched_leg(api.Context(0), args)}), flush=True)
        return
    if args.only_mixed:
        print(json.dumps({"mixed": mixed_leg(api.Context(0), args)}), flush=True)
        return
    if args.only_config2:
        print(json.dumps({"config2": config2_leg(api.Context(0), args)}), flush=True)
        return

    dev = torch.device("cuda", 0)
    ctx = api.Context(0)
    fid = ctx.filter(L.FILTER_TANH)
    pix = torch.from_numpy(pm["pix"]).to(dev)
    cols = [torch.from_numpy(pm[k]).to(dev) for k in ("W", "G1", "G2", "E2")]
    n_out = pix.numel()
    out3 = torch.empty(len(scales), 5, n_out, dtype=torch.float64, device=dev)  # maps in double (FP32_OUT64)
    outs = [out3[k:k + 1] for k in range(len(scales))]
    torch.cuda.synchronize()

    import tempfile

    tune_cache = os.path.join(tempfile.gettempdir(), f"smartap_tune_{os.getpid()}.txt")

    stream = torch.cuda.current_stream(dev)

    def step(keep, ev=None, tune_budget=0):
        data = ctx.pixel_map(args.nside, pix, *cols)
        plan = ctx.plan(data, L.VAR_PIXEL, args.nside, pix, scales, [fid] * len(scales),
                        precision=L.PREC_FP32_OUT64)  # one plan, three scales; FP32 pair sums, double maps
        if not args.no_tune:
            plan.autotune(tune_budget, tune_cache)  # budget 0: cached choices only
        plan.set_timing(True)
        if ev is not None:
            ev[0].record(stream)
        plan.run(L.NORM_SUMMED_PIXCOUNT, out3)
        if ev is not None:
            ev[1].record(stream)
        keep.append((data, plan))

    splits = []

    def retire(keep):
        """Kernel durations of the previous step's plan, then free its handles
        (a batch loop frees the previous batch's map and plan; the library
        keeps their device blocks for the next ones)."""
        for data, plan in keep:
            splits.append([plan.kernel_ms(k) for k in range(len(scales))])
            plan.free()
            data.free()
        keep.clear()

    keep = []
    t = time.perf_counter()
    for w in range(max(args.warmup, 1 if not args.no_tune else 0)):
        retire(keep)
        step(keep, tune_budget=20000 if w == 0 else 0)  # the first warm-up step measures the launch choices
    torch.cuda.synchronize()
    log(f"warm-up (with autotuning) {time.perf_counter() - t:.1f}s")
    retire(keep)
    splits.clear()
    events = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        retire(keep)
        step(keep, events[s])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    # per-kernel durations (HIP events recorded by the library on this stream around each pair kernel)
    last_plan = keep[-1][1]
    splits.append([last_plan.kernel_ms(k) for k in range(len(scales))])
    split_ms = np.mean(splits, axis=0)
    # pairs of each scale: its N channel summed over the centres (integer counts, exact in FP64)
    pairs_scale = [float(out3[k, 4].double().sum()) for k in range(len(scales))]
    pairs = last_plan.last_pairs()
    assert pairs == sum(pairs_scale), (pairs, pairs_scale)
    # pairs of the belt items (N channel summed over their centres); the rest are general-tile pairs
    pairs_belt = [belt_pairs_of(last_plan, outs[k][0, 4], k) for k in range(len(scales))]
    # the run call (all scales) from torch events; per scale the library's belt + general kernel times
    run_ms = float(np.mean([events[s][0].elapsed_time(events[s][1]) for s in range(args.steps)]))
    kern_ms = [float(split_ms[k][0] + split_ms[k][1]) for k in range(len(scales))]
    value = pairs / (ms_step / 1e3)
    # dominant kernel: the longest of the belt/general pair kernels over the scales
    cand = [(split_ms[k][j], k, j) for k in range(len(scales)) for j in range(2)]
    dom_ms, dom, dom_kind = max(cand)
    dom_pairs = pairs_belt[dom] if dom_kind == 0 else pairs_scale[dom] - pairs_belt[dom]
    dom_ops = BELT_OPS_PER_PAIR if dom_kind == 0 else OPS_PER_PAIR
    achieved = dom_pairs * dom_ops / (dom_ms / 1e3)
    log(f"step {ms_step:.2f} ms; run {run_ms:.2f} ms, pair kernels {['%.2f' % k for k in kern_ms]} ms; "
        f"belt/general {[['%.2f' % x for x in r] for r in split_ms]} ms; pairs {pairs:.4e}")
    res = {
        "metric": "pair-evals/s at NSIDE 4096 (pixel-based aperture mass, 3 scales)",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",  # FP32 filter/V sums, FP64 geometry and E/B sums, double maps
        "data": "synthetic",
        "config": {
            "workload": f"pixel-based sphS_pix, NSIDE {args.nside}, {args.area:g} deg2 cap, theta_ap 5/10/20 arcmin, "
                        "tanh filter, summed normalisation",
            "n_pixels": int(n_out),
            "pairs_per_step": pairs,
            "run_ms": run_ms,
            "pair_kernel_ms": kern_ms,
            "belt_general_kernel_ms": [[float(x) for x in r] for r in split_ms],
            "belt_pairs": pairs_belt,
            "general_pairs": [a - b for a, b in zip(pairs_scale, pairs_belt)],
        },
        "roofline": {
            "bound": "alu",
            "kernel": ("k_pixel_belt" if dom_kind == 0 else "k_pixel_f32") + f" ({scales[dom] / ARCMIN:g} arcmin)",
            "achieved": achieved / 1e12,
            "peak": ALU_PEAK / 1e12,
            "unit": "Tlane-op/s",
            "frac": achieved / ALU_PEAK,
            "traffic": None,
            "ops_per_pair": dom_ops,
            "kernel_ms": dom_ms,
            "pairs": dom_pairs,
        },
    }
    # averaged normalisation (Sect. 2.4) on the same plan: the first call also
    # builds the map's averaged records (untimed), then `steps` timed runs
    out_avg = None
    if not args.no_averaged:
        out_avg = torch.empty_like(out3)
        last_plan.run(L.NORM_AVERAGED, out_avg)
        ev_a = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
                for _ in range(args.steps)]
        torch.cuda.synchronize()
        for s in range(args.steps):
            ev_a[s][0].record(stream)
            last_plan.run(L.NORM_AVERAGED, out_avg)
            ev_a[s][1].record(stream)
        torch.cuda.synchronize()
        avg_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev_a]))
        res["averaged"] = {
            "run_ms": avg_ms,
            "summed_run_ms": run_ms,
            "pair_evals_per_s": pairs / (avg_ms / 1e3),
            "note": "smart_run with the averaged normalisation on the step's plan (three scales, maps resident); "
                    "the per-map averaged records are built by the first call, outside the timed runs",
        }
        log(f"averaged normalisation: run {avg_ms:.2f} ms (summed {run_ms:.2f} ms)")
    # detection step (Sect. 6.1) on the 5' M_E map of the last step: every
    # local maximum over the eight neighbours, and a signal-to-noise cut
    # (M_E / sigma >= 4) with the sigma channel
    me, sg = out3[0, 0].contiguous(), out3[0, 2].contiguous()
    ctx.detect_peaks(args.nside, pix, me)  # warm-up
    torch.cuda.synchronize()
    ev_d = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev_d[0].record(stream)
    n_peaks = ctx.detect_peaks(args.nside, pix, me).numel()
    ev_d[1].record(stream)
    n_snr = ctx.detect_peaks(args.nside, pix, me, 4.0, sg).numel()
    ev_d[2].record(stream)
    torch.cuda.synchronize()
    res["detection"] = {
        "workload": f"local maxima of the 5 arcmin M_E map ({n_out} pixels, NSIDE {args.nside})",
        "ms_per_map": ev_d[0].elapsed_time(ev_d[1]),
        "peaks": n_peaks,
        "snr4_ms_per_map": ev_d[1].elapsed_time(ev_d[2]),
        "snr4_peaks": n_snr,
        "note": "smart_detect_peaks: value above its 8 (7 at the 24 three-face corners) neighbours; the second cut "
                "also needs M_E / sigma >= 4; times include the pixel check and the dense scatter",
    }
    log(f"detection: {res['detection']['ms_per_map']:.2f} ms per map, {n_peaks} peaks, {n_snr} above S/N 4")
    # the single map through the split-BF16 MFMA path: one realisation with
    # zero angles (the identity rotation), E and B of the three scales
    zero_u = torch.zeros(1, n_out, dtype=torch.float32, device=dev)
    out_bf = torch.empty(len(scales), 1, 2, n_out, dtype=torch.float32, device=dev)
    last_plan.noise_batch(zero_u, 1, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3, out_bf)  # builds the noise schedule
    torch.cuda.synchronize()
    ev_b = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev_b[0].record(stream)
    last_plan.noise_batch(zero_u, 1, L.NORM_SUMMED_PIXCOUNT, L.PREC_BF16X3, out_bf)
    ev_b[1].record(stream)
    torch.cuda.synchronize()
    res["bf16x3_single_map"] = {
        "run_ms": ev_b[0].elapsed_time(ev_b[1]),
        "fp32_run_ms": run_ms,
        "note": "one zero-angle realisation through the batched split-BF16x3 MFMA kernels (E and B of the three "
                "scales); a single map is a sparse matrix-vector product, so the 32-wide realisation tile is 1/32 "
                "used and this path loses to the plain FP32 kernels",
    }
    del zero_u
    default_workload = args.nside == 4096 and args.area == 15000.0
    res["roofline"]["traffic"] = TRAFFIC_BYTES.get(res["roofline"]["kernel"]) if default_workload else None
    if res["roofline"]["traffic"] is not None:
        res["roofline"]["traffic_source"] = TRAFFIC_SOURCE
    if default_workload and res["roofline"]["kernel"] in COUNTERS:
        res["roofline"]["counters"] = COUNTERS[res["roofline"]["kernel"]]
    # accuracy on the oracle sample + CPU baseline
    if cpu is not None:
        out_pix, refs, cpairs, cdt, avg_check, workers = cpu
        idx = np.searchsorted(pm["pix"], out_pix)
        errs, errs_patch, floor, errs_f32, eps = [], [], [], [], []
        for k, r in enumerate(refs):
            full = outs[k][0, 0].double()
            map_rms = float(torch.sqrt(torch.mean(full * full)))  # RMS of the whole M_E map
            map_std = float(torch.std(full))
            g = full.cpu().numpy()[idx]
            ok = ~r["tie"]
            patch_rms = math.sqrt(np.mean(r["M_E"][ok] ** 2))
            d = float(np.max(np.abs(g[ok] - r["M_E"][ok])))
            errs.append(d / map_rms)
            errs_patch.append(d / patch_rms)
            # the FP32 output format alone: the oracle values rounded to float
            f32 = r["M_E"][ok].astype(np.float32).astype(np.float64)
            floor.append(float(np.max(np.abs(f32 - r["M_E"][ok]))) / map_rms)
            errs_f32.append(float(np.max(np.abs(g[ok] - f32))) / map_rms)
            # the paper's relative difference (Sect. 5.1): (M - M_ref) / std of the reference map
            e = (g[ok] - r["M_E"][ok]) / map_std
            eps.append({"mean": float(np.mean(e)), "std": float(np.std(e))})
        res["max_rel_err_vs_oracle"] = errs
        res["epsilon_vs_oracle"] = eps
        bf_errs = []
        for k, r in enumerate(refs):
            full = outs[k][0, 0].double()
            map_rms = float(torch.sqrt(torch.mean(full * full)))
            ok = ~r["tie"]
            g = out_bf[k, 0, 0].double().cpu().numpy()[idx]
            bf_errs.append(float(np.max(np.abs(g[ok] - r["M_E"][ok]))) / map_rms)
        res["bf16x3_single_map"]["max_rel_err_vs_oracle"] = bf_errs
        res["accuracy"] = {
            "metric": "max |M_E - oracle| over the sample / RMS of the whole M_E map, per scale",
            "max_err_over_patch_rms": errs_patch,
            "f32_output_rounding_floor": floor,
            "max_err_vs_oracle_rounded_to_f32": errs_f32,
            "sample": f"{out_pix.size} apertures in a 2-degree patch, 5/10/20 arcmin",
        }
        if out_avg is not None:
            avg_pix, avg_ref = avg_check
            full = out_avg[0, 0].double()
            map_rms = float(torch.sqrt(torch.mean(full * full)))
            g = full.cpu().numpy()[np.searchsorted(pm["pix"], avg_pix)]
            ok = ~avg_ref["tie"]
            res["averaged"]["max_rel_err_vs_oracle"] = float(np.max(np.abs(g[ok] - avg_ref["M_E"][ok]))) / map_rms
            res["averaged"]["sample"] = f"{avg_pix.size} apertures of the oracle patch, 5 arcmin, M_E"
        res["cpu_baseline"] = {
            "value": cpairs / cdt,
            "unit": "pair-evals/s",
            "cores": workers,
            "cpu_model": cpu_model(),
            "host_cpus_visible": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"{out_pix.size} apertures x 3 scales in a 2-degree patch of the same map "
                      f"({cpairs} pairs, {cdt:.1f} s wall, numpy FP64, apertures split over {workers} processes)",
        }
    if not args.no_config2:
        keep.clear()
        del outs, out3, cols, pix, out_avg, out_bf, me, sg
        outs = out3 = cols = pix = out_avg = out_bf = me = sg = None
        torch.cuda.empty_cache()
        res["config2"] = config2_leg(ctx, args)
    if not args.no_batched:
        keep.clear()
        del outs, out3, cols, pix, out_avg
        torch.cuda.empty_cache()
        res["batched"] = batched_leg(ctx, args)
    if not args.no_mixed:
        torch.cuda.empty_cache()
        res["mixed"] = mixed_leg(ctx, args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
