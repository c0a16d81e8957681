#!/usr/bin/env python3
"""Throughput of colorization (Algorithm 1, steps 1-6) on MI355X.

Default workload (`--workload batched`), the largest one-GPU configuration:
32 segmentation scenes of uneven size (5k-400k isotropic Gaussians,
log-uniform; 20-200 hemisphere cameras each at 640x480 .. 1280x720), SH
degree 0, C = 16 one-hot label channels rendered from per-Gaussian labels
(nearest of 16 random seeds) to BF16 targets, lambda = 1e-4.  All scenes are
one plan (gsc_plan_create), autotuned once and captured into a graph; one
step is one graph replay that projects, bins, blends, accumulates and solves
every scene.  Targets (63 GB of BF16) are resident in HBM before timing.
The line also carries the relighting workload (100k anisotropic Gaussians,
50 cameras 512x512, L=3, C=3 FP32; one gsc_colorize per step) as a
secondary figure.

Other workloads (`--workload`, one JSON line each, same fields):
  relight   the relighting workload above as the headline.
  features  500k isotropic Gaussians, 100 cameras 960x540, L=0, C=64 BF16
            feature targets (feature distillation).
  diff      300k anisotropic Gaussians, 100 cameras 800x800, L=3, C=3: a step
            is colorize + render of the loss mean((render(colorize(y1)) - y2)^2)
            and its backward through both adjoints (targets and opacities).
  plain     2k Gaussians, 8 cameras 64x64, L=0, C=3, a one-scene plan replayed
            as a graph (scenes/s).

`value` is accepted Gaussian-pixel contributions per second; `roofline`
rates the dominant kernel (the fused blend + accumulate) against its roof,
with its launch times taken by HIP events on its own stream over the timed
steps; `cpu_baseline` times the FP64 oracle on the host on a bounded sample
of the same workload, and for the batched workload the same leg checks the
timed plan against the oracle on sampled Gaussians of the smallest, the
largest and two random scenes: the line is printed only if they pass.
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


def progress(msg: str):
    """One line per finished stage on stderr (the result line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
    # HBM bytes per accumulate launch: FETCH_SIZE x 2 + WRITE_SIZE x 1 (the
    # factors a plain 256 MiB device copy gives), averaged over the launches
    # of one step; valid while the accumulate's sources hash to "sources"
    "relight": {"bytes": 2.207e9, "sources": "4a382471bd57137b"},
    "features": {"bytes": 2.362e10, "sources": "4a382471bd57137b"},
    "batched": {"bytes": 7.689e9, "sources": "4a382471bd57137b"},
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


def secondary_relight(args, gsc):
    """The relighting workload (one gsc_colorize per step) as a secondary
    figure of the default line."""
    from paper_2604_17155_amd import synthetic as syn
    sc = syn.make_relight()
    targets = gpu_targets(gsc, sc)
    label = (f"relighting: {sc.N} anisotropic Gaussians, {len(sc.cams)} hemisphere cameras "
             f"{sc.cams[0].width}x{sc.cams[0].height}, SH degree {sc.sh_deg}, C={sc.C}, FP32 targets")
    r = run_single(args, gsc, sc, targets, label, "f32", "relight")
    progress(f"secondary relighting figure: {r['ms_per_step']:.3f} ms per step")
    return {"workload": label, "value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"],
            "dtype": r["dtype"], "stage_ms_per_step": r["config"]["stage_ms_per_step"],
            "roofline": r["roofline"]}


def workload_features(args, gsc):
    from paper_2604_17155_amd import synthetic as syn
    sc = syn.make_features(n=args.n or 500_000, n_cams=args.views or 100)
    targets = gpu_targets(gsc, sc, bf16=True)
    label = (f"feature distillation: {sc.N} isotropic Gaussians, {len(sc.cams)} hemisphere cameras "
             f"{sc.cams[0].width}x{sc.cams[0].height}, SH degree 0, C={sc.C}, BF16 targets")
    default_size = not (args.n or args.views or args.res or args.bin or args.variant or args.schedule)
    out = run_single(args, gsc, sc, targets, label, "bf16", "features" if default_size else None)
    if not args.no_cpu_baseline:
        sub = syn.make_features(n=sc.N, n_cams=len(sc.cams))
        sub.cams = sub.cams[:4]
        out["cpu_baseline"] = cpu_baseline(sub, host_threads(), "first 4 views of the workload")
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line_ in fh:
                if line_.startswith("model name"):
                    return line_.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def roofline_hbm(kernel, bytes_per_step, kernel_ms_per_step, launches, traffic=None):
    """The accumulate's algorithmic HBM traffic (each target read once per
    step) over its launch time, against the MI355X HBM peak."""
    gbs = bytes_per_step / (kernel_ms_per_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": gbs * 1e9 / PEAK_HBM, "traffic": traffic, "kernel": kernel,
            "kernel_ms": kernel_ms_per_step / max(1, launches), "launches_per_step": launches,
            "bytes_per_launch": bytes_per_step / max(1, launches)}


def accumulate_kernel_name(variant: int, C: int) -> str:
    if variant & 128:
        return "k_accumulate_mfma"
    return "k_accumulate"


def segment_subset(scenes, seed=20260417):
    """The scenes the oracle checks and times: the smallest and the largest
    (by Gaussian count) and two others drawn with a fixed seed."""
    import numpy as np
    order = sorted(range(len(scenes)), key=lambda k: scenes[k].N)
    rest = order[1:-1]
    rng = np.random.default_rng(seed)
    pick = [int(k) for k in rng.choice(rest, size=min(2, len(rest)), replace=False)]
    return [order[0], order[-1]] + pick


def segment_check(scenes, table, row0, targets, rerun, coeffs, status, threads):
    """Accuracy of the batched plan against the oracle on the smallest, the
    largest and two random scenes: sample Gaussians, render the target rows
    they read with the oracle, write those rows into the device targets, run
    the plan again (`rerun`) and compare the sampled Gaussians' coefficients
    with the oracle's (e_g <= 1e-4 + the bound of near-threshold decisions,
    as in tests/parity.py; the unobserved sets agree where no decision is in
    doubt).  Returns the accuracy record."""
    import numpy as np
    import torch
    import oracle
    subset = segment_subset(scenes)
    rng = np.random.default_rng(7)
    checks = []
    for k in subset:
        sc = scenes[k]
        # sampled among the top twentieth by height (the cameras look down from
        # the upper hemisphere, so these are rarely hidden) and, of those, the
        # smaller-scale half; as many as keep the target rows they read within
        # about two million
        top = np.argsort(-sc.means[:, 2], kind="stable")[:max(1, sc.N // 20)]
        small = top[np.argsort(sc.scales[top, 0], kind="stable")[:max(1, top.size // 2)]]
        n_want = 64
        while True:
            want = np.zeros(sc.N, np.uint8)
            want[rng.choice(small, min(n_want, small.size), replace=False)] = 1
            rows = oracle.wanted_rows(sc, want)
            if rows.size <= 2_000_000 or n_want <= 2:
                break
            n_want //= 2
        ysp, vals = oracle.sparse_targets(sc, rows, threads=threads)
        progress(f"check: scene {k}, {int(want.sum())} sampled Gaussians reading {rows.size} target rows")
        idx = torch.from_numpy(rows + row0[k]).cuda()
        targets[idx] = torch.from_numpy(vals.view(np.int16)).cuda().view(torch.bfloat16)
        checks.append((k, want, ysp))
    torch.cuda.synchronize()
    rerun()
    torch.cuda.synchronize()
    c_all, s_all = coeffs.cpu().numpy(), status.cpu().numpy()
    per_scene, ok, all_e = [], True, []
    t_check = time.perf_counter()
    for k, want, ysp in checks:
        sc = scenes[k]
        g0 = table[k][0]
        ref = oracle.colorize(sc, ysp, want=want, threads=threads)
        sel = want.astype(bool)
        c, st = c_all[g0:g0 + sc.N], s_all[g0:g0 + sc.N]
        nrm = np.linalg.norm(ref["coeffs"].reshape(sc.N, -1), axis=1)
        obs = sel & ((ref["status"] & 1) == 0)
        tau = 1e-3 * np.median(nrm[obs]) if obs.any() else 1.0
        scale = np.maximum(nrm, tau)
        e = np.linalg.norm((c.astype(np.float64) - ref["coeffs"]).reshape(sc.N, -1), axis=1) / scale
        b = ref["flip"] / scale
        inside = bool(np.all(e[obs] <= 1e-4 + b[obs]))
        sure = sel & (ref["ndec"] == 0)
        same_obs = bool(np.array_equal(st[sure] & 1, ref["status"][sure] & 1))
        fl = obs & (b > 0.5e-4)
        ok = ok and inside and same_obs and bool(obs.any())
        all_e.append(e[obs])
        per_scene.append({"scene": k, "gaussians": sc.N, "views": len(sc.cams), "sampled": int(sel.sum()),
                          "observed": int(obs.sum()), "flagged": int(fl.sum()),
                          "max_rel_err": float(e[obs & ~fl].max()) if (obs & ~fl).any() else 0.0,
                          "max_rel_err_flagged": float(e[fl].max()) if fl.any() else 0.0,
                          "within_bounds": inside, "unobserved_agree": same_obs})
        progress(f"check: scene {k} compared, within bounds: {inside}")
    observed = sum(p["observed"] for p in per_scene)
    accuracy = {"gate": "e_g <= 1e-4 + near-threshold bound on every sampled observed Gaussian",
                "passed": ok, "observed_compared": observed,
                "flagged_fraction": sum(p["flagged"] for p in per_scene) / max(1, observed),
                "max_rel_err": max(p["max_rel_err"] for p in per_scene),
                "scenes": per_scene, "check_seconds": time.perf_counter() - t_check}
    ea = np.concatenate(all_e) if all_e else np.zeros(1)
    accuracy["rel_err_all_compared"] = {"p50": float(np.median(ea)), "p99": float(np.percentile(ea, 99)),
                                        "max": float(ea.max())}
    return accuracy


def cpu_baseline_leg(args, gsc, scenes, table, row0, targets, graph, coeffs, status):
    """The oracle leg of the batched workload (the only place bench.py runs
    the oracle).  Two parts:
      check  -- segment_check() on the timed graph;
      timing -- the oracle's full colorize on a bounded sample of the same
                scenes (their first views), on all host threads and on one.
    Returns (accuracy, cpu_baseline)."""
    import oracle
    from paper_2604_17155_amd import synthetic as syn
    threads = host_threads()
    subset = segment_subset(scenes)
    accuracy = segment_check(scenes, table, row0, targets, graph.replay, coeffs, status, threads)
    # timing: full oracle colorize of each subset scene's first views (about
    # 3 M pixels per scene), on every host thread, and the smallest of these
    # samples on one thread
    samples = []
    for k in subset:
        sc = scenes[k]
        px = sc.cams[0].width * sc.cams[0].height
        sub = syn.make_segment_scene(k)
        sub.cams = sub.cams[:max(1, min(len(sub.cams), 3_000_000 // px))]
        samples.append((k, sub, oracle.make_targets(sub, threads=threads)))
        progress(f"baseline sample of scene {k}: {len(sub.cams)} views")
    count, dt = 0, 0.0
    for k, sub, y in samples:
        t0 = time.perf_counter()
        r = oracle.colorize(sub, y, threads=threads)
        dt += time.perf_counter() - t0
        count += r["count"]
    desc = "; ".join(f"scene {k} ({sub.N} Gaussians, first {len(sub.cams)} of {len(scenes[k].cams)} views "
                     f"{sub.cams[0].width}x{sub.cams[0].height})" for k, sub, _ in samples)
    # one thread: the smallest scene's sample, a third of its views
    k1, sub, y = min(samples, key=lambda t: t[1].N)
    sub1 = syn.make_segment_scene(k1)
    sub1.cams = sub.cams[:max(1, len(sub.cams) // 3)]
    y1 = y[:sub1.n_pixels]
    t0 = time.perf_counter()
    r1 = oracle.colorize(sub1, y1, threads=1)
    dt1 = time.perf_counter() - t0
    baseline = {"value": count / dt, "unit": "contributions/s", "cores": threads, "kind": "oracle",
                "sample": f"full FP64 oracle colorize of the first views of the smallest, the largest "
                          f"and two random scenes: {desc}; {count} contributions in {dt:.3g} s "
                          f"(oracle-rendered targets)",
                "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                "single_thread": {"value": r1["count"] / dt1, "unit": "contributions/s",
                                  "sample": f"scene {k1}, first {len(sub1.cams)} views, "
                                            f"{r1['count']} contributions in {dt1:.3g} s"},
                "check_seconds": accuracy["check_seconds"]}
    return accuracy, baseline


def build_segment_workload(gsc, n_scenes):
    """The multi-scene segmentation workload: scenes, the plan's scene table
    (Gaussian offset, count, camera offset, count), each scene's first target
    row, all cameras, the concatenated geometry on the device and the BF16
    targets (each scene's GPU render of its ground truth)."""
    import numpy as np
    import torch
    from paper_2604_17155_amd import synthetic as syn
    scenes = [syn.make_segment_scene(k) for k in range(n_scenes)]
    table, cams, row0 = [], [], []
    g0 = c0 = r0 = 0
    for sc in scenes:
        table.append((g0, sc.N, c0, len(sc.cams)))
        row0.append(r0)
        g0, c0, r0 = g0 + sc.N, c0 + len(sc.cams), r0 + sc.n_pixels
        cams += list(sc.cams)
    C = scenes[0].C
    targets = torch.empty((r0, C), dtype=torch.bfloat16, device="cuda")
    r = 0
    for sc in scenes:  # one scene at a time: its FP32 render is the only temporary
        targets[r:r + sc.n_pixels] = gpu_targets(gsc, sc, bf16=True)
        r += sc.n_pixels
    progress(f"targets of {n_scenes} scenes rendered ({r0} pixels)")
    cat = lambda f: torch.from_numpy(np.ascontiguousarray(np.concatenate([getattr(sc, f) for sc in scenes]))).cuda()
    geo = [cat(f) for f in ("means", "scales", "quats", "opacities")]
    return scenes, table, row0, cams, geo, targets


def workload_batched(args, gsc):
    import torch
    n_scenes = args.scenes
    scenes, table, row0, cams, geo, targets = build_segment_workload(gsc, n_scenes)
    C = scenes[0].C
    g0 = sum(sc.N for sc in scenes)
    c0 = len(cams)
    r0 = sum(sc.n_pixels for sc in scenes)
    blend_bit = 1 << 5  # GSC_STAGE_BLEND: events around each batch's accumulate
    ctx = gsc.Context(bin_size=args.bin, flags=gsc.GSC_FLAG_PROFILE, profile_stages=blend_bit)
    plan = gsc.Plan(ctx, table, *geo, cams, C, 0)
    lam = list(scenes[0].lam)
    coeffs, status = plan.autotune(targets, lam)
    info = plan.info()
    contrib = int(info.contributions)
    variant = int(info.accumulate_variant)
    progress(f"plan created and autotuned: {int(info.batches)} view batches, {variant_name(variant)}")
    tuned = {variant_name(v): float(info.tuned_ms[i]) for i, v in enumerate(info.tuned_variant) if v}
    # warm up on the capture stream, then capture one run (its stage events
    # become graph nodes, re-recorded by every replay) and replay it
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(max(1, args.warmup)):
            plan.run(targets, lam, coeffs, status)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ctx.stats()  # drain the eager runs' events
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
    progress(f"{args.steps} graph replays timed: {1e3 * elapsed / args.steps:.1f} ms each")
    st = ctx.stats()  # the accumulate events of the last timed replay
    acc_ms = float(st.stage_dict()["blend"])
    info2 = plan.info()
    assert int(info2.dropped_pairs) == 0 and int(info2.contributions) == contrib
    launches = variant_launches(C, variant) * int(info.batches)
    target_bytes = float(r0) * C * 2
    # the counters were read on the 32-scene plan, 32-pixel bins, 29 view
    # batches, the 16-channel matrix-core accumulate as a grid
    measured_shape = (n_scenes == 32 and int(info.bin_size) == 32 and int(info.batches) == 29
                      and variant_name(variant) == "mfma16")
    config = {"workload": f"multi-scene segmentation: {n_scenes} scenes, {g0} Gaussians in total "
                          f"(5k-400k per scene), {c0} cameras 640x480..1280x720, SH degree 0, "
                          f"C={C}, BF16 targets, one plan replayed as a graph",
              "arithmetic": "BF16 targets decoded exactly; blend weights FP32, split into BF16 high "
                            "and low parts for the matrix-core product (FP32 accumulation); "
                            "per-Gaussian sums FP32; fold and solve FP64",
              "contributions_per_step": contrib, "scenes_per_sec": n_scenes * args.steps / elapsed,
              "pixels": r0, "target_bytes": target_bytes, "tile_pairs_per_step": int(info.pair_capacity),
              "view_batches": int(info.batches), "bin_size": int(info.bin_size),
              "autotune_accumulate_ms": tuned,
              "accumulate_variant": variant_name(variant),
              "accumulate_ms_per_step": acc_ms,
              "accumulate_ms_source": "HIP event nodes around each batch's accumulate in the "
                                      "captured graph, read after the last timed replay"}
    out = line(args, contrib * args.steps / elapsed, 1e3 * elapsed / args.steps, "bf16", config,
               roofline_hbm(accumulate_kernel_name(variant, C), target_bytes, acc_ms, launches,
                            measured_traffic("batched") if measured_shape else None))
    out["roofline_valu"] = roofline(C, contrib, acc_ms, launches)
    if not args.no_cpu_baseline:
        acc, base = cpu_baseline_leg(args, gsc, scenes, table, row0, targets, graph, coeffs, status)
        out["accuracy"] = acc
        out["cpu_baseline"] = base
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

    def step():  # geometry and opacities stay fixed here, so the tile lists are reused
        c = ag.colorize(y_p, o_p, m, s, q, sc.cams, sc.sh_deg, lam, context=ctx, reuse_binning=True)
        img = ag.render(c, o_p, m, s, q, sc.cams, context=ctx, reuse_binning=True)
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
    ap.add_argument("--workload", default="batched",
                    choices=["relight", "features", "batched", "diff", "plain"])
    ap.add_argument("--no-secondary", action="store_true",
                    help="batched workload: skip the relighting figure carried as a secondary field")
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
    out = fn(args, gsc)
    if args.workload == "batched" and not args.no_secondary:
        out["config"]["secondary"] = secondary_relight(args, gsc)
    acc = out.get("accuracy")
    if acc is not None and not acc["passed"]:
        print("accuracy check against the oracle failed; no result line:\n" + json.dumps(acc),
              file=sys.stderr)
        sys.exit(1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
