"""Multi-batch paths against the FP64 oracle and the single-batch GPU path.

A call (or a plan) splits its views into batches of consecutive views: at
most `batch_items` (view, Gaussian) items per batch, and a batch of several
views whose (bin, item) pairs exceed `batch_pairs` is halved until it fits.
Each batch numbers its tiles, items and per-view sum slots locally.  The
limits are set low here so that small scenes take the multi-batch paths of
colorize (L = 0 sums straight into [N, C+1], L > 0 per-view sums), render,
both adjoints (the colorize adjoint re-bins each batch for its second pass)
and plans, including the pair-count halving, and every result is compared
with the oracle and with the same call in one batch.
"""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import parity
from tests.test_gpu_batched import concat, segment_scenes

pytestmark = pytest.mark.gpu

SMOOTH = dict(alpha_min=0.0, t_min=0.0, sigma_cut=6.0)


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


def _colorize(ctx, sc, y):
    """Coefficients, statuses, statistics and per-Gaussian counts."""
    import torch
    from paper_2604_17155_amd import gsc
    m, s, q, o = gsc.scene_tensors(sc)
    c, st, x = ctx.colorize(m, s, q, o, sc.cams, parity.to_device_targets(y), sc.sh_deg, list(sc.lam),
                            extras={"counts"})
    torch.cuda.synchronize()
    return c.cpu().numpy(), st.cpu().numpy(), ctx.stats(), x["counts"].cpu().numpy()


def _same(a, b, tol=1e-5):
    """Two GPU results of the same call up to the order of float atomics."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    scale = max(np.abs(b).max(), 1e-30)
    return float(np.abs(a - b).max() / scale) <= tol


@pytest.mark.parametrize("case", ["plain L0", "relight L3", "ragged L2 C5"])
def test_colorize_view_batches(gsc_mod, case):
    if case == "plain L0":
        sc = syn.make_plain()
    elif case == "relight L3":
        sc = syn.make_relight(n=3000, n_cams=8, res=96)
    else:
        rng = np.random.Generator(np.random.PCG64(7))
        sc = syn.make_relight(n=2500, n_cams=7, res=64, sh_deg=2,
                              lam=rng.uniform(1e-4, 1e-2, 9).astype(np.float32))
        sc.cams = syn.hemisphere_cams(7, 3.0, 120, 88)
        sc.C = 5
        sc.gt = [np.concatenate([sc.gt[0], sc.gt[0][:, :, :2] * 0.5], axis=2)]
    y = oracle.make_targets(sc)
    ref = oracle.colorize(sc, y)
    one = _colorize(gsc_mod.Context(), sc, y)
    assert one[2].view_batches == 1
    # two views per batch (the last batch ragged), then one view per batch
    for per in (2, 1):
        ctx = gsc_mod.Context(batch_items=per * sc.N)
        print(f"[case] {case}: N={sc.N} cams={len(sc.cams)}, {per} view(s) per batch", flush=True)
        c, st, stats, cnt = _colorize(ctx, sc, y)
        assert stats.view_batches == (len(sc.cams) + per - 1) // per
        print(parity.check_colorize(c, st, ref, count_gpu=stats.contributions, cnt_gpu=cnt,
                                    label=f"{case} {stats.view_batches} batches"), flush=True)
        assert stats.contributions == one[2].contributions
        assert np.array_equal(cnt, one[3])
        assert np.array_equal(st, one[1])
        assert _same(c, one[0])


def test_colorize_pair_halving(gsc_mod):
    """batch_pairs below the pair count of the whole call: the batch is halved
    (and halved again) until each part fits."""
    sc = syn.make_relight(n=3000, n_cams=8, res=96)
    y = oracle.make_targets(sc)
    ref = oracle.colorize(sc, y)
    one = _colorize(gsc_mod.Context(), sc, y)
    pairs = int(one[2].pairs)
    ctx = gsc_mod.Context(batch_pairs=max(1, pairs // 5))
    print(f"[case] pair halving: {pairs} pairs, limit {pairs // 5}", flush=True)
    c, st, stats, cnt = _colorize(ctx, sc, y)
    print(f"batches {stats.view_batches}, pairs {stats.pairs}", flush=True)
    assert stats.view_batches >= 5
    assert stats.pairs == pairs
    print(parity.check_colorize(c, st, ref, count_gpu=stats.contributions, cnt_gpu=cnt,
                                label="pair halving"), flush=True)
    assert np.array_equal(st, one[1]) and np.array_equal(cnt, one[3]) and _same(c, one[0])


def test_bf16_matrix_core_view_batches(gsc_mod):
    sc = syn.make_segment_scene(0, n_override=4000, cams_override=7)
    sc.cams = syn.hemisphere_cams(7, 3.0, 160, 120)
    y = oracle.make_targets(sc)
    ref = oracle.colorize(sc, y)
    for variant in (128 | 16, 16):
        ctx = gsc_mod.Context(batch_items=3 * sc.N, accumulate_variant=variant)
        print(f"[case] segment 4k C16 bf16 variant {variant}, 3 views per batch", flush=True)
        c, st, stats, cnt = _colorize(ctx, sc, y)
        assert stats.view_batches == 3
        print(parity.check_colorize(c, st, ref, count_gpu=stats.contributions, cnt_gpu=cnt,
                                    label=f"segment variant {variant} 3 batches"), flush=True)


def test_render_view_batches(gsc_mod):
    import torch
    sc = syn.make_relight(n=5000, n_cams=7, res=112)
    coeffs = torch.from_numpy(sc.gt[0].astype(np.float32)).cuda()
    m, s, q, o = gsc_mod.scene_tensors(sc)
    img1 = gsc_mod.Context().render(m, s, q, o, sc.cams, coeffs)
    ctx = gsc_mod.Context(batch_items=2 * sc.N)
    print(f"[case] render L3 N={sc.N} cams={len(sc.cams)}, 2 views per batch", flush=True)
    img = ctx.render(m, s, q, o, sc.cams, coeffs)
    torch.cuda.synchronize()
    assert ctx.stats().view_batches == 4
    img, img1 = img.cpu().numpy(), img1.cpu().numpy()
    assert np.array_equal(img, img1)  # render has no atomics: identical bits
    ref, pb = oracle.render(sc, sc.gt[0].astype(np.float32).astype(np.float64), with_bound=True)
    print(parity.check_render(img, ref, pb, label="render 4 batches"), flush=True)


def test_backward_view_batches(gsc_mod):
    import torch
    sc = syn.make_relight(n=3000, n_cams=7, res=96)
    opts = oracle.Options(alpha_min=0.0, t_min=0.0, sigma_cut=6.0)
    y = oracle.make_targets(sc, opts=opts)
    ref = oracle.colorize(sc, y, opts=opts)
    c32 = ref["coeffs"].astype(np.float32)
    rng = np.random.default_rng(5)
    G = rng.standard_normal(c32.shape).astype(np.float32)
    gi = rng.standard_normal((sc.n_pixels, 3)).astype(np.float32)
    gt_ref, go_ref = oracle.colorize_backward(sc, y, c32.astype(np.float64), G.astype(np.float64), opts=opts)
    gc_ref, gor_ref = oracle.render_backward(sc, c32.astype(np.float64), gi.astype(np.float64), opts=opts)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = {}
    for per in (0, 2):
        ctx = gsc_mod.Context(batch_items=per * sc.N, **SMOOTH)
        print(f"[case] adjoints L3 N={sc.N} cams={len(sc.cams)}, batch_items {per * sc.N}", flush=True)
        gt, go = ctx.colorize_backward(m, s, q, o, sc.cams, parity.to_device_targets(y), sc.sh_deg,
                                       list(sc.lam), dev(c32), dev(G))
        nb1 = ctx.stats().view_batches
        gc, gor = ctx.render_backward(m, s, q, o, sc.cams, dev(c32), dev(gi))
        torch.cuda.synchronize()
        nb2 = ctx.stats().view_batches
        assert (nb1, nb2) == ((1, 1) if per == 0 else (4, 4))
        out[per] = [a.cpu().numpy() for a in (gt, go, gc, gor)]
    for name, a, r in zip(("grad_targets", "grad_opacities", "render grad_coeffs", "render grad_opacities"),
                          out[2], (gt_ref, go_ref, gc_ref, gor_ref)):
        e = float(np.linalg.norm(a - r) / np.linalg.norm(r))
        print(f"multi-batch {name}: rel L2 vs oracle {e:.2e}", flush=True)
        assert e <= 1e-4, name
    for a, b in zip(out[2], out[0]):
        assert _same(a, b, 1e-4)


def test_plan_view_batches(gsc_mod):
    import torch
    scenes = segment_scenes()
    targets = [oracle.make_targets(sc) for sc in scenes]
    table, geo, cams, y = concat(scenes, targets)
    tens = [torch.from_numpy(a).cuda() for a in geo]
    yd = parity.to_device_targets(y)
    C = scenes[0].C
    base = gsc_mod.Plan(gsc_mod.Context(), table, *tens, cams, C, 0)
    c1, st1 = base.run(yd, [1e-4])
    torch.cuda.synchronize()
    b1 = base.info().batches
    results = {}
    for label, over in (("items", dict(batch_items=20000)),
                        ("pairs", dict(batch_pairs=max(1, int(base.info().pair_capacity) // 6)))):
        ctx = gsc_mod.Context(**over)
        plan = gsc_mod.Plan(ctx, table, *tens, cams, C, 0)
        info = plan.info()
        print(f"[case] plan {label}: {info.batches} batches (one-batch plan: {b1})", flush=True)
        assert info.batches >= 3 > b1 or info.batches >= b1 + 2
        c, st = plan.run(yd, [1e-4])
        torch.cuda.synchronize()
        info = plan.info()
        assert info.dropped_pairs == 0
        assert info.pair_capacity == base.info().pair_capacity
        assert info.contributions == base.info().contributions
        c, st = c.cpu().numpy(), st.cpu().numpy()
        assert np.array_equal(st, st1.cpu().numpy()) and _same(c, c1.cpu().numpy())
        results[label] = (c, st)
    for k, (sc, yk) in enumerate(zip(scenes, targets)):
        g0, n = table[k][0], table[k][1]
        ref = oracle.colorize(sc, yk)
        for label, (c, st) in results.items():
            print(parity.check_colorize(c[g0:g0 + n], st[g0:g0 + n], ref,
                                        label=f"plan {label} scene {k}"), flush=True)
