#!/usr/bin/env python3
"""Throughput of colorization (Algorithm 1, steps 1-6) on MI355X.

Default workload (`--workload relight`): the view-dependent relighting scene
-- 100k anisotropic Gaussians (20 blobs, log-scales N(-4, 0.5), random
rotations, opacity Beta(2,2)), 50 hemisphere cameras at 512x512, SH degree 3,
C = 3 FP32 channels, per-band Lambda (1e-5, 1e-4, 1e-3, 1e-2).  Targets are
the render of random ground-truth SH coefficients plus N(0, 0.01^2) noise,
resident in HBM before timing.  One step = one gsc_colorize call (project,
depth sort, binning, tile sort, fused blend + accumulate, FP64 fold +
Cholesky solve).

Other workloads (one JSON line each, same fields):
  features  500k isotropic Gaussians, 100 cameras 960x540, L=0, C=64 BF16
            feature targets (feature distillation).
  batched   32 segmentation scenes of uneven size (5k-400k Gaussians, 20-200
            cameras, 640x480 .. 1280x720), L=0, C=16 BF16 one-hot labels, as
            one plan captured into a graph; a step is one graph replay.
  diff      300k anisotropic Gaussians, 100 cameras 800x800, L=3, C=3: a step
            is colorize + render of the loss mean((render(colorize(y1)) - y2)^2)
            and its backward through both adjoints (targets and opacities).

`value` is accepted Gaussian-pixel contributions per second of the colorize
pass(es) in a step; `roofline` rates the dominant kernel (fused blend +
accumulate) by its algorithmic FP32 work against the MI355X vector peak,
timed with HIP events on the stream it runs on; `cpu_baseline` times the FP64
oracle on the host on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12  # MI355X FP32 vector FLOP/s
PEAK_HBM = 8.0e12            # MI355X HBM3E bytes/s
METRIC = "Gaussian-pixel contributions/sec (accumulate+solve)"


def algorithmic_flops_per_contribution(C: int) -> float:
    # weight: offsets, quadratic form, alpha, transmittance (12 FLOP) + 1 exp;
    # accumulation of V and S: 2 (C + 1) FLOP
    return 12.0 + 1.0 + 2.0 * (C + 1)


def host_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(sc, threads: int, what: str):
    """Time the FP64 oracle (as it stands) on `sc` on the host."""
    import oracle
    y = oracle.make_targets(sc, threads=threads)
    t0 = time.perf_counter()
    r = oracle.colorize(sc, y, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": r["count"] / dt, "unit": "contributions/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}: one colorize of {sc.N} Gaussians, {len(sc.cams)} views "
                      f"{sc.cams[0].width}x{sc.cams[0].height}, L={sc.sh_deg}, C={sc.C}; "
                      f"{r['count']} contributions in {dt:.3g} s (oracle-rendered targets)"}


def gpu_targets(gsc, sc, which=0, bf16=False):
    """Targets on the device: GPU render of ground-truth set `which` plus the
    seeded noise, cast to BF16 (round to nearest even) when asked."""
    import numpy as np
    import torch
    from paper_2604_17155_amd import synthetic as syn
    m, s, q, o = gsc.scene_tensors(sc)
    rctx = gsc.Context()
    gt = torch.from_numpy(sc.gt[which].astype(np.float32)).cuda()
    img = rctx.render(m, s, q, o, sc.cams, gt)
    if sc.noise_std:
        img += torch.from_numpy(syn.target_noise(sc, which)).cuda()
    return img.to(torch.bfloat16).contiguous() if bf16 else img.contiguous()


# HBM bytes per k_accumulate launch, from FETCH_SIZE (x2) and WRITE_SIZE counter
# runs (profiles/accumulate_*.md), valid only for the kernel sources they were
# taken on: the digest of those sources is kept beside each figure.
MEASURED_TRAFFIC = {
    "relight": {"bytes": 2.599e9, "sources": "32621809bd307686"},
}
ACCUMULATE_SOURCES = ("paper_2604_17155_amd/csrc/k_accum.hip", "paper_2604_17155_amd/csrc/wave_ops.h",
                      "paper_2604_17155_amd/csrc/k_sort.hip",    # the tile order
                      "paper_2604_17155_amd/csrc/gsc_api.hip")   # the launch shape


def accumulate_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ACCUMULATE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    m = MEASURED_TRAFFIC.get(workload)
    if m is None or m["sources"] != accumulate_sources_digest():
        return None
    return m["bytes"]


def roofline(C, contrib, blend_ms_total, launches, workload=None):
    flops = algorithmic_flops_per_contribution(C) * contrib
    achieved = flops / (blend_ms_total * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
            "traffic": measured_traffic(workload),
            "kernel": "k_accumulate", "kernel_ms": blend_ms_total / max(1, launches),
            "launches_per_step": launches,
            "flop_per_contribution": algorithmic_flops_per_contribution(C)}


def variant_name(v: int) -> str:
    """Readable accumulate variant code (see gsc_options.accumulate_variant)."""
    ch = v & 127
    base = ("mfma-packed" if ch == 1 else f"mfma{ch}") if v & 128 else f"vec{ch}"
    return base + ("/persistent" if v & 256 else "")


def variant_launches(C: int, v: int) -> int:
    ch = v & 127
    if v & 128 and ch == 1:
        return 1
    return (C + ch - 1) // ch


def hbm_view(target_bytes: float, kernel_ms_total: float):
    """The accumulate's algorithmic HBM traffic (the targets, read once per
    step) against the MI355X HBM peak."""
    gbs = target_bytes / (kernel_ms_total * 1e-3) / 1e9
    return {"target_bytes": target_bytes, "achieved_GBps": gbs, "peak_GBps": PEAK_HBM / 1e9,
            "frac": gbs * 1e9 / PEAK_HBM}


def line(args, value, ms_per_step, dtype, config, roof):
    return {"metric": METRIC, "value": value, "unit": "contributions/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config, "roofline": roof}


def run_single(args, gsc, sc, targets, label, dtype, traffic_key=None):
    """Time `steps` gsc_colorize calls on one scene."""
    import torch
    m, s, q, o = gsc.scene_tensors(sc)
    lam = list(sc.lam)
    # the timed steps record events around the blend only (the roofline's
    # kernel time); the other stages are timed in a separate pass below
    blend_bit = 1 << 5  # GSC_STAGE_BLEND
    ctx = gsc.Context(flags=gsc.GSC_FLAG_PROFILE, bin_size=args.bin, accumulate_variant=args.variant,
                      schedule=args.schedule, profile_stages=blend_bit)
    for _ in range(args.warmup):
        ctx.colorize(m, s, q, o, sc.cams, targets, sc.sh_deg, lam)
    torch.cuda.synchronize()
    contrib = int(ctx.stats().contributions)  # also drains the warm-up timings
    stream = torch.cuda.current_stream()
    coeffs = torch.empty((sc.N, sc.n_b, sc.C), dtype=torch.float32, device="cuda")
    status = torch.empty((sc.N,), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.colorize(m, s, q, o, sc.cams, targets, sc.sh_deg, lam, coeffs=coeffs, status=status,
                     stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ctx.stats()
    blend_ms = st.stage_dict()["blend"] / args.steps
    launches = max(1, int(st.stage_launches[5]) // args.steps)
    # per-stage breakdown: a few more calls with every stage timed, outside
    # the timed region
    pctx = gsc.Context(flags=gsc.GSC_FLAG_PROFILE, bin_size=args.bin, accumulate_variant=args.variant,
                       schedule=args.schedule)
    n_prof = min(args.steps, 5)
    pctx.colorize(m, s, q, o, sc.cams, targets, sc.sh_deg, lam, coeffs=coeffs, status=status, stream=stream)
    torch.cuda.synchronize()
    pctx.stats()
    for _ in range(n_prof):
        pctx.colorize(m, s, q, o, sc.cams, targets, sc.sh_deg, lam, coeffs=coeffs, status=status,
                      stream=stream)
    torch.cuda.synchronize()
    stages = {k: v / n_prof for k, v in pctx.stats().stage_dict().items() if v}
    tbytes = float(sum(c.width * c.height for c in sc.cams)) * sc.C * (2 if dtype == "bf16" else 4)
    config = {"workload": label, "contributions_per_step": contrib,
              "scenes_per_sec": args.steps / elapsed, "tile_pairs_per_step": int(st.pairs),
              "bin_size": int(st.bin_size), "stage_ms_per_step": stages,
              "tile_schedule": ["automatic", "grid", "longest first"][args.schedule],
              "accumulate_hbm": hbm_view(tbytes, blend_ms)}
    return line(args, contrib * args.steps / elapsed, 1e3 * elapsed / args.steps, dtype, config,
                roofline(sc.C, contrib, blend_ms, launches, traffic_key))


def workload_relight(args, gsc):
    from paper_2604_17155_amd import synthetic as syn
    sc = syn.make_relight(n=args.n or 100_000, n_cams=args.views or 50, res=args.res or 512)
    targets = gpu_targets(gsc, sc)
    label = (f"relighting: {sc.N} anisotropic Gaussians, {len(sc.cams)} hemisphere cameras "
             f"{sc.cams[0].width}x{sc.cams[0].height}, SH degree {sc.sh_deg}, C={sc.C}, FP32 targets")
    default_size = not (args.n or args.views or args.res or args.bin or args.variant or args.schedule)
    out = run_single(args, gsc, sc, targets, label, "f32", "relight" if default_size else None)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, host_threads(), "the full benchmark workload")
    return out


def workload_features(args, gsc):
    from paper_2604_17155_amd import synthetic as syn
    sc = syn.make_features(n=args.n or 500_000, n_cams=args.views or 100)
    targets = gpu_targets(gsc, sc, bf16=True)
    label = (f"feature distillation: {sc.N} isotropic Gaussians, {len(sc.cams)} hemisphere cameras "
             f"{sc.cams[0].width}x{sc.cams[0].height}, SH degree 0, C={sc.C}, BF16 targets")
    out = run_single(args, gsc, sc, targets, label, "bf16")
    if not args.no_cpu_baseline:
        sub = syn.make_features(n=sc.N, n_cams=len(sc.cams))
        sub.cams = sub.cams[:4]
        out["cpu_baseline"] = cpu_baseline(sub, host_threads(), "first 4 views of the workload")
    return out


def workload_batched(args, gsc):
    import numpy as np
    import torch
    from paper_2604_17155_amd import synthetic as syn
    n_scenes = args.scenes
    scenes = [syn.make_segment_scene(k) for k in range(n_scenes)]
    table, cams = [], []
    g0 = c0 = r0 = 0
    for sc in scenes:
        table.append((g0, sc.N, c0, len(sc.cams)))
        g0, c0, r0 = g0 + sc.N, c0 + len(sc.cams), r0 + sc.n_pixels
        cams += list(sc.cams)
    C = scenes[0].C
    targets = torch.empty((r0, C), dtype=torch.bfloat16, device="cuda")
    r = 0
    for sc in scenes:  # one scene at a time: its FP32 render is the only temporary
        targets[r:r + sc.n_pixels] = gpu_targets(gsc, sc, bf16=True)
        r += sc.n_pixels
    cat = lambda f: torch.from_numpy(np.ascontiguousarray(np.concatenate([getattr(sc, f) for sc in scenes]))).cuda()
    geo = [cat(f) for f in ("means", "scales", "quats", "opacities")]
    ctx = gsc.Context(bin_size=args.bin)
    plan = gsc.Plan(ctx, table, *geo, cams, C, 0)
    lam = list(scenes[0].lam)
    coeffs, status = plan.autotune(targets, lam)
    info = plan.info()
    contrib = int(info.contributions)
    variant = int(info.accumulate_variant)
    tuned = {variant_name(v): float(info.tuned_ms[i]) for i, v in enumerate(info.tuned_variant) if v}
    acc_ms = [float(info.tuned_ms[i]) for i, v in enumerate(info.tuned_variant) if v == variant][0]
    # capture one run and replay it
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(max(1, args.warmup)):
            plan.run(targets, lam, coeffs, status)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(targets, lam, coeffs, status)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info2 = plan.info()
    assert int(info2.dropped_pairs) == 0
    launches = variant_launches(C, variant) * int(info.batches)
    config = {"workload": f"multi-scene segmentation: {n_scenes} scenes, {g0} Gaussians in total "
                          f"(5k-400k per scene), {c0} cameras 640x480..1280x720, SH degree 0, "
                          f"C={C}, BF16 targets, one plan replayed as a graph",
              "contributions_per_step": contrib, "scenes_per_sec": n_scenes * args.steps / elapsed,
              "pixels": r0, "tile_pairs_per_step": int(info.pair_capacity),
              "view_batches": int(info.batches), "bin_size": int(info.bin_size),
              "autotune_accumulate_ms": tuned,
              "accumulate_variant": variant_name(variant),
              "accumulate_hbm": hbm_view(float(r0) * C * 2, acc_ms)}
    out = line(args, contrib * args.steps / elapsed, 1e3 * elapsed / args.steps, "bf16", config,
               roofline(C, contrib, acc_ms, launches))
    if not args.no_cpu_baseline:
        small = min(scenes, key=lambda sc: sc.N * len(sc.cams))
        out["cpu_baseline"] = cpu_baseline(small, host_threads(), "the smallest scene of the batch")
    return out


def workload_plain(args, gsc):
    """The plain 2k-Gaussian scene (8 views 64x64, L=0, C=3) as a one-scene
    plan captured into a graph: a step is one replay (scenes/s)."""
    import torch
    from paper_2604_17155_amd import synthetic as syn
    sc = syn.make_plain(n=args.n or 2000, n_cams=args.views or 8, res=args.res or 64)
    targets = gpu_targets(gsc, sc)
    m, s, q, o = gsc.scene_tensors(sc)
    ctx = gsc.Context(bin_size=args.bin, accumulate_variant=args.variant)
    plan = gsc.Plan(ctx, [(0, sc.N, 0, len(sc.cams))], m, s, q, o, list(sc.cams), sc.C, sc.sh_deg)
    lam = list(sc.lam)
    coeffs, status = plan.run(targets, lam)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(max(1, args.warmup)):
            plan.run(targets, lam, coeffs, status)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(targets, lam, coeffs, status)
    graph.replay()
    torch.cuda.synchronize()
    contrib = int(plan.info().contributions)
    steps = max(args.steps, 200)  # a replay takes tens of microseconds
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    config = {"workload": f"plain: {sc.N} isotropic Gaussians, {len(sc.cams)} circle cameras "
                          f"{sc.cams[0].width}x{sc.cams[0].height}, SH degree 0, C=3, FP32 targets, "
                          f"one-scene plan replayed as a graph",
              "contributions_per_step": contrib, "scenes_per_sec": steps / elapsed,
              "replays": steps}
    out = line(args, contrib * steps / elapsed, 1e3 * elapsed / steps, "f32", config, None)
    out["steps"] = steps
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, host_threads(), "the full workload")
    return out


def workload_diff(args, gsc):
    import torch
    from paper_2604_17155_amd import autograd as ag, synthetic as syn
    sc = syn.make_diff(n=args.n or 300_000, n_cams=args.views or 100, res=args.res or 800)
    y1 = gpu_targets(gsc, sc, 0)
    y2 = gpu_targets(gsc, sc, 1)
    m, s, q, o = gsc.scene_tensors(sc)
    lam = list(sc.lam)
    ctx = gsc.Context(bin_size=args.bin, schedule=args.schedule)
    o_p = o.clone().requires_grad_(True)
    y_p = y1.clone().requires_grad_(True)

    def step():
        c = ag.colorize(y_p, o_p, m, s, q, sc.cams, sc.sh_deg, lam, context=ctx)
        img = ag.render(c, o_p, m, s, q, sc.cams, context=ctx)
        loss = ((img - y2) ** 2).mean()
        y_p.grad = None
        o_p.grad = None
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    c, _ = ctx.colorize(m, s, q, o, sc.cams, y1, sc.sh_deg, lam)
    torch.cuda.synchronize()
    contrib = int(ctx.stats().contributions)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # kernel time of the forward accumulate, for the roofline
    pctx = gsc.Context(flags=gsc.GSC_FLAG_PROFILE, bin_size=args.bin)
    pctx.colorize(m, s, q, o, sc.cams, y1, sc.sh_deg, lam)
    torch.cuda.synchronize()
    st = pctx.stats()
    config = {"workload": f"differentiable re-render loss: {sc.N} anisotropic Gaussians, {len(sc.cams)} "
                          f"hemisphere cameras {sc.cams[0].width}x{sc.cams[0].height}, SH degree 3, C=3; "
                          f"step = colorize + render + both adjoints (targets, opacities)",
              "forward_contributions_per_step": contrib}
    out = line(args, contrib * args.steps / elapsed, 1e3 * elapsed / args.steps, "f32", config,
               roofline(sc.C, contrib, st.stage_dict()["blend"], max(1, int(st.stage_launches[5]))))
    out["metric"] = "forward colorize contributions/sec over full forward+backward steps"
    return out


def copy_calibration():
    """One plain device copy of a known size (256 MiB read, 256 MiB written):
    the reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copied_bytes": a.numel() * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device copy (counter calibration) and exit")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="relight",
                    choices=["relight", "features", "batched", "diff", "plain"])
    ap.add_argument("--n", type=int, default=0, help="Gaussians (0: the workload's size)")
    ap.add_argument("--views", type=int, default=0, help="cameras (0: the workload's count)")
    ap.add_argument("--res", type=int, default=0, help="square resolution (0: the workload's)")
    ap.add_argument("--scenes", type=int, default=32, help="scenes of the batched workload")
    ap.add_argument("--bin", type=int, default=0, help="screen bin size 16 or 32 (0: automatic)")
    ap.add_argument("--schedule", type=int, default=0,
                    help="tile schedule of the accumulate launch (0: automatic, 1: grid, 2: longest first)")
    ap.add_argument("--variant", type=int, default=0,
                    help="accumulate variant code (0: automatic; see gsc_options.accumulate_variant)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by views "
              "across GPUs as described in the design notes, but no multi-GPU run exists.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    import __graft_entry__
    __graft_entry__._ensure_built()
    from paper_2604_17155_amd import gsc

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    fn = {"relight": workload_relight, "features": workload_features, "batched": workload_batched,
          "plain": workload_plain,
          "diff": workload_diff}[args.workload]
    print(json.dumps(fn(args, gsc)), flush=True)


if __name__ == "__main__":
    main()
