"""GPU parity of the batched multi-scene colorize (plans): each scene of a
batch against the FP64 oracle on that scene alone and against the
single-scene GPU call, graph capture and replay, the autotuner, and the
capacity guard of a plan whose geometry changed after planning."""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_17155_amd import gsc
    import __graft_entry__
    __graft_entry__._ensure_built()
    gsc.load()
    return gsc


@pytest.fixture(scope="module")
def ctx(gsc_mod):
    return gsc_mod.Context()


def segment_scenes():
    """Five scenes of the multi-scene segmentation workload's kind (L=0,
    C=16 one-hot labels, BF16 targets), shrunk so the oracle finishes in
    seconds; sizes and resolutions deliberately uneven."""
    shapes = [(600, 3, 160, 120), (5000, 6, 200, 150), (1500, 4, 240, 136), (9000, 8, 320, 180),
              (300, 2, 160, 120)]
    out = []
    for k, (n, nc, w, h) in enumerate(shapes):
        sc = syn.make_segment_scene(k, n_override=n, cams_override=nc)
        sc.cams = syn.hemisphere_cams(nc, 3.0, w, h)
        out.append(sc)
    return out


def concat(scenes, targets):
    """Concatenated geometry, cameras (global pixel offsets), targets and the
    scene table."""
    table, cams = [], []
    g0 = c0 = 0
    for sc in scenes:
        table.append((g0, sc.N, c0, len(sc.cams)))
        g0 += sc.N
        c0 += len(sc.cams)
        cams += list(sc.cams)
    cat = lambda a: np.ascontiguousarray(np.concatenate(a, axis=0))
    geo = [cat([getattr(sc, f) for sc in scenes]) for f in ("means", "scales", "quats", "opacities")]
    return table, geo, cams, cat(targets)


def make_plan(gsc_mod, ctx, scenes, targets):
    import torch
    table, geo, cams, y = concat(scenes, targets)
    tens = [torch.from_numpy(a).cuda() for a in geo]
    plan = gsc_mod.Plan(ctx, table, *tens, cams, scenes[0].C, scenes[0].sh_deg)
    return plan, table, tens, cams, parity.to_device_targets(y)


def check_scenes(scenes, targets, table, coeffs, status, label):
    for k, (sc, y) in enumerate(zip(scenes, targets)):
        g0, n = table[k][0], table[k][1]
        ref = oracle.colorize(sc, y)
        msg = parity.check_colorize(coeffs[g0:g0 + n], status[g0:g0 + n], ref,
                                    label=f"{label} scene {k} (N={n}, cams={len(sc.cams)})")
        print(msg, flush=True)


def test_batched_segment_scenes(ctx, gsc_mod):
    import torch
    scenes = segment_scenes()
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    lam = list(scenes[0].lam)
    coeffs, status = plan.run(y, lam)
    torch.cuda.synchronize()
    info = plan.info()
    print(f"plan: batches={info.batches} views={info.views} items={info.items} "
          f"pairs={info.pair_capacity} contributions={info.contributions}", flush=True)
    assert info.dropped_pairs == 0
    c, st = coeffs.cpu().numpy(), status.cpu().numpy()
    check_scenes(scenes, targets, table, c, st, "batched L0 C16 bf16")
    # the single-scene call on each scene gives the same result
    for k, sc in enumerate(scenes):
        m, s, q, o = gsc_mod.scene_tensors(sc)
        c1, _ = ctx.colorize(m, s, q, o, sc.cams, parity.to_device_targets(targets[k]), 0, lam)
        g0, n = table[k][0], table[k][1]
        e, _ = parity.rel_errors(c[g0:g0 + n], dict(coeffs=c1.cpu().numpy().astype(np.float64),
                                                    status=st[g0:g0 + n]))
        assert e.max() < 1e-5, (k, e.max())


def test_batched_view_dependent(ctx, gsc_mod):
    """L=2, C=3 float32: the per-view fold runs per scene."""
    import torch
    scenes = []
    for k, (n, nc, r) in enumerate([(2500, 5, 96), (800, 3, 64), (4000, 6, 128)]):
        sc = syn.make_relight(seed_offset=20 + k, n=n, n_cams=nc, res=r, sh_deg=2)
        scenes.append(sc)
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    coeffs, status = plan.run(y, list(scenes[0].lam))
    torch.cuda.synchronize()
    check_scenes(scenes, targets, table, coeffs.cpu().numpy(), status.cpu().numpy(), "batched L2 C3")


def test_batched_graph_capture_and_replay(ctx, gsc_mod):
    """A run captured into a graph and replayed, with eager work between the
    replays, matches the eager run every time."""
    import torch
    scenes = segment_scenes()[:3]
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    lam = list(scenes[0].lam)
    ref_c, ref_s = plan.run(y, lam)
    torch.cuda.synchronize()
    ref_c, ref_s = ref_c.clone(), ref_s.clone()
    coeffs = torch.zeros_like(ref_c)
    status = torch.zeros_like(ref_s)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run(y, lam, coeffs, status)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        plan.run(y, lam, coeffs, status)
    other = scenes[0]
    m, s, q, o = gsc_mod.scene_tensors(other)
    for rep in range(3):
        coeffs.fill_(float("nan"))
        status.fill_(255)
        graph.replay()
        torch.cuda.synchronize()
        e, _ = parity.rel_errors(coeffs.cpu().numpy(), dict(coeffs=ref_c.cpu().numpy().astype(np.float64),
                                                            status=ref_s.cpu().numpy()))
        print(f"replay {rep}: max rel diff to eager {e.max():.2e}", flush=True)
        assert e.max() < 1e-5
        assert torch.equal(status, ref_s)
        # eager work between replays
        ctx.colorize(m, s, q, o, other.cams, parity.to_device_targets(targets[0]), 0, lam)
        torch.cuda.synchronize()


def test_profiled_plan_in_a_graph(gsc_mod):
    """A plan run with stage profiling captured into a graph: its events are
    graph nodes, so every replay re-times the stages, and the replays still
    match the eager run."""
    import torch
    scenes = segment_scenes()[:3]
    targets = [oracle.make_targets(sc) for sc in scenes]
    pctx = gsc_mod.Context(flags=gsc_mod.GSC_FLAG_PROFILE, profile_stages=1 << 5)
    plan, table, tens, cams, y = make_plan(gsc_mod, pctx, scenes, targets)
    lam = list(scenes[0].lam)
    ref_c, ref_s = plan.run(y, lam)
    torch.cuda.synchronize()
    ref_c = ref_c.clone()
    pctx.stats()  # drain the eager run's events
    coeffs = torch.zeros_like(ref_c)
    status = torch.zeros_like(ref_s)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run(y, lam, coeffs, status)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    pctx.stats()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(y, lam, coeffs, status)
    for rep in range(3):
        coeffs.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.allclose(coeffs, ref_c, rtol=1e-5, atol=1e-6)
    st = pctx.stats()
    blend = st.stage_dict()["blend"]
    print(f"profiled graph: blend {blend:.3f} ms over {plan.info().batches} batch(es), "
          f"{int(st.stage_launches[5])} launches", flush=True)
    assert blend > 0.0 and int(st.stage_launches[5]) >= 1


def test_colorize_refuses_capture(gsc_mod):
    """Entry points that read a count back return GSC_ERR_NOT_CAPTURABLE on a
    capturing stream and enqueue nothing; the capture stays usable."""
    import torch
    sc = syn.make_plain(n=500, n_cams=2, res=32)
    y = parity.to_device_targets(oracle.make_targets(sc))
    m, s, q, o = gsc_mod.scene_tensors(sc)
    ctx = gsc_mod.Context()
    lam = list(sc.lam)
    coeffs, status = ctx.colorize(m, s, q, o, sc.cams, y, 0, lam)
    torch.cuda.synchronize()
    buf = torch.zeros(4, device="cuda")
    graph = torch.cuda.CUDAGraph()
    errors = []
    with torch.cuda.graph(graph):
        for call in (lambda: ctx.colorize(m, s, q, o, sc.cams, y, 0, lam, coeffs=coeffs, status=status),
                     lambda: ctx.colorize_noalloc(m, s, q, o, sc.cams, y, 0, lam, coeffs, status),
                     lambda: ctx.render(m, s, q, o, sc.cams, coeffs)):
            try:
                call()
            except gsc_mod.GscError as e:
                errors.append(e.status)
        buf.add_(1.0)
    graph.replay()
    torch.cuda.synchronize()
    assert errors == [gsc_mod.GSC_ERR_NOT_CAPTURABLE] * 3, errors
    assert torch.equal(buf, torch.ones(4, device="cuda"))


def test_batched_autotune(ctx, gsc_mod):
    import torch
    scenes = segment_scenes()[1:4]
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    lam = list(scenes[0].lam)
    ref_c, _ = plan.run(y, lam)
    torch.cuda.synchronize()
    ref_c = ref_c.clone()
    c, _ = plan.autotune(y, lam)
    info = plan.info()
    cands = [info.tuned_variant[i] for i in range(8) if info.tuned_variant[i]]
    times = [info.tuned_ms[i] for i in range(len(cands))]
    names = [f"{v & 511}" for v in cands]
    print(f"autotune: {dict(zip(names, ['%.3f' % t for t in times]))} -> {info.accumulate_variant}",
          flush=True)
    assert len(cands) >= 4 and info.accumulate_variant in cands
    assert any(v >> 8 for v in cands)  # persistent shapes were timed
    assert all(t > 0 for t in times)
    # the fastest, or the plain grid within 3% of the persistent form
    chosen = times[cands.index(info.accumulate_variant)]
    assert chosen <= 1.03 * min(times) * (1 + 1e-6)
    if info.accumulate_variant >> 8:
        grid = info.accumulate_variant & 255
        assert grid not in cands or times[cands.index(grid)] > 1.03 * chosen
    e, _ = parity.rel_errors(c.cpu().numpy(), dict(coeffs=ref_c.cpu().numpy().astype(np.float64),
                                                   status=np.zeros(len(c), np.uint8)))
    assert e.max() < 1e-5
    c2, _ = plan.run(y, lam)
    torch.cuda.synchronize()
    e, _ = parity.rel_errors(c2.cpu().numpy(), dict(coeffs=ref_c.cpu().numpy().astype(np.float64),
                                                    status=np.zeros(len(c), np.uint8)))
    assert e.max() < 1e-5


def test_batched_capacity_guard(ctx, gsc_mod):
    """Geometry grown after planning: surplus tile pairs are dropped and
    reported, nothing is written out of bounds; restoring the geometry
    restores the result."""
    import torch
    scenes = segment_scenes()[:2]
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    lam = list(scenes[0].lam)
    ref_c, _ = plan.run(y, lam)
    torch.cuda.synchronize()
    ref_c = ref_c.clone()
    scales = tens[1]
    saved = scales.clone()
    scales.mul_(2.0)
    plan.run(y, lam)
    info = plan.info()
    print(f"grown geometry: dropped {info.dropped_pairs} items' pairs", flush=True)
    assert info.dropped_pairs > 0
    scales.copy_(saved)
    c, _ = plan.run(y, lam)
    info = plan.info()
    assert info.dropped_pairs == 0
    e, _ = parity.rel_errors(c.cpu().numpy(), dict(coeffs=ref_c.cpu().numpy().astype(np.float64),
                                                   status=np.zeros(len(c), np.uint8)))
    assert e.max() < 1e-5


def test_batched_bins_of_32_pixels(gsc_mod):
    import torch
    ctx = gsc_mod.Context(bin_size=32)
    scenes = segment_scenes()
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    coeffs, status = plan.run(y, list(scenes[0].lam))
    torch.cuda.synchronize()
    check_scenes(scenes, targets, table, coeffs.cpu().numpy(), status.cpu().numpy(), "batched bin32")


@pytest.mark.parametrize("bin_size", [32, 16])
def test_batched_bins_of_32_pixels_wide_splats(gsc_mod, bin_size):
    """Splats of two scenes grown sixteen- and three-fold.  With 32-pixel
    bins, blocks of items whose pairs exceed what the block-wide emission
    collects (2048 per 256 items) fall back to each item writing its own
    pairs, beside blocks that take the block-wide path; with 16-pixel bins
    the per-item emission's unstaged path runs beside its staged one.  Every
    scene still matches the oracle."""
    import torch
    ctx = gsc_mod.Context(bin_size=bin_size)
    scenes = segment_scenes()[:3]
    for sc, f in zip(scenes[:2], (16.0, 3.0)):
        sc.scales = np.ascontiguousarray(sc.scales * np.float32(f))
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    coeffs, status = plan.run(y, list(scenes[0].lam))
    torch.cuda.synchronize()
    info = plan.info()
    print(f"wide splats, bins of {bin_size}: pair capacity {info.pair_capacity} for {info.items} items",
          flush=True)
    check_scenes(scenes, targets, table, coeffs.cpu().numpy(), status.cpu().numpy(), f"bin{bin_size} wide")


def test_batched_bins_of_32_pixels_capacity_guard(gsc_mod):
    """The capacity guard with 32-pixel bins: pairs past the plan's capacity
    are dropped and reported by the block-wide emission as well."""
    import torch
    ctx = gsc_mod.Context(bin_size=32)
    scenes = segment_scenes()[:2]
    targets = [oracle.make_targets(sc) for sc in scenes]
    plan, table, tens, cams, y = make_plan(gsc_mod, ctx, scenes, targets)
    lam = list(scenes[0].lam)
    ref_c, _ = plan.run(y, lam)
    torch.cuda.synchronize()
    ref_c = ref_c.clone()
    scales = tens[1]
    saved = scales.clone()
    scales.mul_(2.0)
    plan.run(y, lam)
    info = plan.info()
    print(f"bins of 32, grown geometry: dropped {info.dropped_pairs} items' pairs", flush=True)
    assert info.dropped_pairs > 0
    scales.copy_(saved)
    c, _ = plan.run(y, lam)
    assert plan.info().dropped_pairs == 0
    e, _ = parity.rel_errors(c.cpu().numpy(), dict(coeffs=ref_c.cpu().numpy().astype(np.float64),
                                                   status=np.zeros(len(c), np.uint8)))
    assert e.max() < 1e-5
