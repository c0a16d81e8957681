"""GPU parity of gsc_colorize / gsc_render against the FP64 oracle.

Inputs are the seeded synthetic workloads at sizes the oracle finishes in
seconds (several tiles, ragged image edges), plus the full 100k-Gaussian
relighting workload compared on a random sample of Gaussians.
"""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import parity, tiny

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


def run_gpu(ctx, sc, y, lam=None, counts=False):
    """GPU colorize; with counts=True also the per-Gaussian contribution
    counts (as a fourth element)."""
    import torch
    from paper_2604_17155_amd import gsc
    m, s, q, o = gsc.scene_tensors(sc)
    lam = list(sc.lam if lam is None else lam)
    out = ctx.colorize(m, s, q, o, sc.cams, parity.to_device_targets(y), sc.sh_deg, lam,
                       extras={"counts"} if counts else None)
    torch.cuda.synchronize()
    res = (out[0].cpu().numpy(), out[1].cpu().numpy(), ctx.stats())
    if counts:
        res = res + (out[2]["counts"].cpu().numpy(),)
    return res


def check(ctx, sc, y, ref, label, max_flagged=None):
    """Colorize on the GPU and gate against `ref`: coefficients, statuses, and
    per-Gaussian and total contribution counts."""
    c, st, stats, cnt = run_gpu(ctx, sc, y, counts=True)
    msg = parity.check_colorize(c, st, ref, count_gpu=stats.contributions, cnt_gpu=cnt, label=label,
                                max_flagged=max_flagged)
    print(msg, flush=True)
    return c, st, stats


def _case(ctx, sc, y, label, want=None, max_flagged=None):
    print(f"[case] {label}: N={sc.N} cams={len(sc.cams)} L={sc.sh_deg} C={sc.C} dtype={y.dtype}", flush=True)
    ref = oracle.colorize(sc, y, want=want)
    if want is None:
        c, st, stats = check(ctx, sc, y, ref, label, max_flagged=max_flagged)
        print(f"| contributions gpu={stats.contributions} oracle={ref['count']} decisions={ref['events']}",
              flush=True)
        return c, st, stats, ref
    c, st, stats = run_gpu(ctx, sc, y)
    msg = parity.check_colorize(c, st, ref, want=want, label=label, max_flagged=max_flagged)
    print(msg, f"| contributions gpu={stats.contributions} oracle={ref['count']} events={ref['events']}",
          flush=True)
    return c, st, stats, ref


def test_plain_workload(ctx):
    sc = syn.make_plain()
    y = oracle.make_targets(sc)
    _case(ctx, sc, y, "plain 2k L0 C3")


def test_relight_reduced(ctx):
    sc = syn.make_relight(n=20000, n_cams=16, res=256)
    y = oracle.make_targets(sc)
    _case(ctx, sc, y, "relight 20k L3 C3 256^2")


def test_ragged_sizes_and_channel_chunks(ctx):
    rng = np.random.Generator(np.random.PCG64(7))
    sc = syn.make_relight(n=4000, n_cams=6, res=64, sh_deg=2,
                          lam=rng.uniform(1e-4, 1e-2, 9).astype(np.float32))
    sc.cams = syn.hemisphere_cams(6, 3.0, 200, 120)
    sc.C = 5
    sc.gt = [np.concatenate([sc.gt[0], sc.gt[0][:, :, :2] * 0.5], axis=2)]
    y = oracle.make_targets(sc)
    _case(ctx, sc, y, "ragged 200x120 L2 C5 per-coefficient lambda")


def test_bf16_targets_l1(ctx):
    sc = syn.make_relight(n=3000, n_cams=6, res=96, sh_deg=1)
    sc.cams = syn.hemisphere_cams(6, 3.0, 96, 80)
    sc.target_dtype = "bf16"
    y = oracle.make_targets(sc)
    assert y.dtype == np.uint16
    _case(ctx, sc, y, "bf16 L1 C3 96x80")


def test_feature_channels_bf16(ctx):
    sc = syn.make_features(n=20000, n_cams=8, width=240, height=136, C=64)
    y = oracle.make_targets(sc)
    _case(ctx, sc, y, "features 20k L0 C64 bf16")


def test_segment_like_c16(ctx):
    sc = syn.make_segment_scene(0, n_override=8000, cams_override=10)
    sc.cams = syn.hemisphere_cams(10, 3.0, 160, 120)
    y = oracle.make_targets(sc)
    _case(ctx, sc, y, "segment 8k L0 C16 bf16")


# accumulate variants: vector lanes (16 channels per launch) and the
# matrix-core form with 16, 32 and 64 channels per launch
BF16_VARIANTS = [16, 128 | 16, 128 | 32, 128 | 64]


@pytest.fixture(scope="module")
def ragged_features():
    """C = 40 BF16 feature channels: the last block of 16 (or 32, 64) is
    partly outside C."""
    sc = syn.make_features(n=12000, n_cams=6, width=200, height=120, C=40)
    y = oracle.make_targets(sc)
    return sc, y, oracle.colorize(sc, y)


@pytest.mark.parametrize("bin_size", [16, 32])
@pytest.mark.parametrize("variant", BF16_VARIANTS)
def test_accumulate_variants_bf16(gsc_mod, ragged_features, variant, bin_size):
    sc, y, ref = ragged_features
    ctx = gsc_mod.Context(bin_size=bin_size, accumulate_variant=variant)
    c, st, stats = check(ctx, sc, y, ref, f"features L0 C40 bf16 variant {variant} bin {bin_size}")
    assert stats.bin_size == bin_size


@pytest.mark.parametrize("bin_size", [16, 32])
@pytest.mark.parametrize("schedule", [1, 2])
def test_tile_schedules(gsc_mod, schedule, bin_size):
    """Tiles in index order (one wave each) and longest lists first from a
    work queue: C = 5 over ragged 200x120 views, one and several channel
    launches."""
    rng = np.random.Generator(np.random.PCG64(11))
    sc = syn.make_relight(n=6000, n_cams=8, res=64, sh_deg=2,
                          lam=rng.uniform(1e-4, 1e-2, 9).astype(np.float32))
    sc.cams = syn.hemisphere_cams(8, 3.0, 200, 120)
    sc.C = 5
    sc.gt = [np.concatenate([sc.gt[0], sc.gt[0][:, :, :2] * 0.5], axis=2)]
    y = oracle.make_targets(sc)
    ref = oracle.colorize(sc, y)
    for variant in (0, 2):
        ctx = gsc_mod.Context(bin_size=bin_size, schedule=schedule, accumulate_variant=variant)
        check(ctx, sc, y, ref, f"schedule {schedule} bin {bin_size} variant {variant}")


@pytest.mark.parametrize("schedule", [1, 2])
def test_tile_schedules_matrix_core(gsc_mod, ragged_features, schedule):
    sc, y, ref = ragged_features
    ctx = gsc_mod.Context(bin_size=32, schedule=schedule, accumulate_variant=128 | 16)
    check(ctx, sc, y, ref, f"features C40 bf16 matrix core schedule {schedule}")


PACKED = 128 | 1  # all channels and a ones column in one matrix-core block


def _packed_scenes():
    out = []
    sc = syn.make_relight(n=12000, n_cams=10, res=160)
    out.append((sc, "relight 12k L3 C3 f32"))
    rng = np.random.Generator(np.random.PCG64(7))
    sc = syn.make_relight(n=4000, n_cams=6, res=64, sh_deg=2,
                          lam=rng.uniform(1e-4, 1e-2, 9).astype(np.float32))
    sc.cams = syn.hemisphere_cams(6, 3.0, 200, 120)
    sc.C = 7
    sc.gt = [np.concatenate([sc.gt[0], sc.gt[0] * 0.5, sc.gt[0][:, :, :1] * -0.7], axis=2)]
    out.append((sc, "ragged 200x120 L2 C7 f32"))
    sc = syn.make_features(n=8000, n_cams=6, width=176, height=112, C=12)
    out.append((sc, "features 8k L0 C12 bf16"))
    return out


@pytest.mark.parametrize("bin_size", [16, 32])
@pytest.mark.parametrize("idx", [0, 1, 2])
def test_packed_matrix_core(gsc_mod, idx, bin_size):
    """The packed matrix-core accumulate (FP32 targets split into BF16 high
    and low parts, or BF16 targets, with V from a ones column)."""
    sc, label = _packed_scenes()[idx]
    y = oracle.make_targets(sc)
    ctx = gsc_mod.Context(bin_size=bin_size, accumulate_variant=PACKED)
    print(f"[case] packed {label} bin {bin_size}", flush=True)
    ref = oracle.colorize(sc, y)
    check(ctx, sc, y, ref, f"packed {label} bin {bin_size}")


def test_matrix_core_per_view_l1(gsc_mod):
    """L = 1 with 16 BF16 channels: the matrix-core accumulate writes per-view
    sums that the FP64 fold consumes."""
    rng = np.random.default_rng(77)
    sc = syn.make_features(n=4000, n_cams=8, width=128, height=96, C=16)
    sc.sh_deg = 1
    sc.gt = [rng.normal(0.0, 1.0, (sc.N, 4, 16)) * np.array([1.0, 0.1, 0.1, 0.1])[None, :, None]]
    sc.lam = np.array([1e-4, 1e-3], dtype=np.float32)
    y = oracle.make_targets(sc)
    assert y.dtype == np.uint16
    for variant in (128 | 16, 16):
        ctx = gsc_mod.Context(accumulate_variant=variant)
        print(f"[case] L1 C16 bf16 variant {variant}", flush=True)
        ref = oracle.colorize(sc, y)
        check(ctx, sc, y, ref, f"L1 C16 bf16 variant {variant}")


def test_degenerate_inputs(ctx, gsc_mod):
    import torch
    # no Gaussians
    sc = tiny.random_scene(1, n=0, n_cams=2, res=16, sh_deg=1, C=2)
    y = np.zeros((sc.n_pixels, 2), np.float32)
    m = torch.zeros((0, 3), device="cuda")
    coeffs, st = ctx.colorize(m, m, torch.zeros((0, 4), device="cuda"), torch.zeros(0, device="cuda"),
                              sc.cams, parity.to_device_targets(y), 1, [1e-4, 1e-3])
    assert coeffs.shape == (0, 4, 2)
    # no cameras: everything unobserved
    sc = tiny.random_scene(2, n=50, n_cams=0, sh_deg=3, C=3)
    c, st, _ = run_gpu(ctx, sc, np.zeros((1, 3), np.float32))
    assert np.all(st == gsc_mod.GSC_G_UNOBSERVED) and np.all(c == 0)
    # Gaussians behind the camera or outside every view
    cam = tiny.axis_camera(32, 32, z=-4.0)
    sc = tiny.scene([[0, 0, 0], [0, 0, -6.0], [8.0, 0, 0], [0.05, 0.02, 0.3]], np.full((4, 3), 0.05),
                    tiny.identity_quats(4), [0.5, 0.5, 0.5, 0.7], [cam], sh_deg=1, C=1,
                    lam=[1e-4, 1e-3])
    y = np.random.default_rng(0).uniform(0, 1, (sc.n_pixels, 1)).astype(np.float32)
    ref = oracle.colorize(sc, y)
    c, st, stats = check(ctx, sc, y, ref, "tiny")
    assert list(st & 1) == list(ref["status"] & 1) == [0, 1, 1, 0]


def test_render_matches_oracle(ctx, gsc_mod):
    import torch
    sc = syn.make_relight(n=20000, n_cams=8, res=200)
    coeffs = sc.gt[0]
    m, s, q, o = gsc_mod.scene_tensors(sc)
    img = ctx.render(m, s, q, o, sc.cams, torch.from_numpy(coeffs.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    img = img.cpu().numpy()
    # the oracle renders the float32-rounded coefficients the GPU sees
    ref32, pb = oracle.render(sc, coeffs.astype(np.float32).astype(np.float64), with_bound=True)
    stats = ctx.stats()
    print(parity.check_render(img, ref32, pb, label="render L3 C3"), flush=True)
    ref_full = oracle.colorize(sc, np.zeros((sc.n_pixels, 3), np.float32))
    assert abs(int(stats.contributions) - ref_full["count"]) <= ref_full["events"]


def test_render_l2_six_channels_ragged(ctx, gsc_mod):
    """L = 2, C = 6 (two render launches of four channels, the second partly
    outside C), 200x120 views: the transposed coefficient reads for every
    (m, c) row."""
    import torch
    rng = np.random.default_rng(21)
    sc = syn.make_relight(n=6000, n_cams=5, res=64, sh_deg=2)
    sc.cams = syn.hemisphere_cams(5, 3.0, 200, 120)
    coeffs = rng.normal(0.0, 0.3, (sc.N, 9, 6))
    coeffs[:, 0, :] += 0.5
    m, s, q, o = gsc_mod.scene_tensors(sc)
    img = ctx.render(m, s, q, o, sc.cams, torch.from_numpy(coeffs.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    img = img.cpu().numpy()
    sc.C = 6
    ref32, pb = oracle.render(sc, coeffs.astype(np.float32).astype(np.float64), with_bound=True)
    assert img.shape == (sc.n_pixels, 6)
    print(parity.check_render(img, ref32, pb, label="render L2 C6"), flush=True)


def test_repeat_and_context_reuse(ctx):
    sc_big = syn.make_relight(n=20000, n_cams=10, res=160)
    y_big = oracle.make_targets(sc_big)
    sc_small = syn.make_plain()
    y_small = oracle.make_targets(sc_small)
    a1, _, s1 = run_gpu(ctx, sc_big, y_big)
    b, _, _ = run_gpu(ctx, sc_small, y_small)
    a2, _, s2 = run_gpu(ctx, sc_big, y_big)
    assert s1.contributions == s2.contributions
    e, obs = parity.rel_errors(a2, dict(coeffs=a1.astype(np.float64), status=np.zeros(len(a1), np.uint8)))
    assert e.max() < 1e-5  # only the order of float atomics differs
    ref = oracle.colorize(sc_small, y_small)
    e, obs = parity.rel_errors(b, ref)
    assert np.all(e[obs] <= parity.TOL_F32 + parity.bound(ref)[obs])


def test_relight_full_size(ctx):
    """The 100k-Gaussian, 50 x 512^2, L=3 workload in the benchmark's launch
    configuration, compared on every Gaussian."""
    sc = syn.make_relight()
    y = oracle.make_targets(sc)
    _case(ctx, sc, y, "relight full 100k L3 50x512^2", max_flagged=0.015)


@pytest.fixture(scope="module")
def ctx32(gsc_mod):
    return gsc_mod.Context(bin_size=32)


@pytest.mark.parametrize("case", ["plain", "relight", "ragged", "features", "segment"])
def test_bins_of_32_pixels(ctx32, case):
    """The same workloads binned at 32x32 pixels (four wave tiles per bin):
    the result does not depend on the binning."""
    if case == "plain":
        sc = syn.make_plain()
    elif case == "relight":
        sc = syn.make_relight(n=20000, n_cams=8, res=200)
    elif case == "ragged":
        sc = syn.make_relight(n=4000, n_cams=6, res=64, sh_deg=2)
        sc.cams = syn.hemisphere_cams(6, 3.0, 200, 120)
    elif case == "features":
        sc = syn.make_features(n=20000, n_cams=6, width=240, height=136, C=64)
    else:
        sc = syn.make_segment_scene(0, n_override=8000, cams_override=10)
        sc.cams = syn.hemisphere_cams(10, 3.0, 170, 110)
    y = oracle.make_targets(sc)
    _case(ctx32, sc, y, f"bin32 {case}")


def test_render_bins_of_32_pixels(ctx32, gsc_mod):
    import torch
    sc = syn.make_relight(n=20000, n_cams=6, res=176)
    coeffs = sc.gt[0]
    m, s, q, o = gsc_mod.scene_tensors(sc)
    img = ctx32.render(m, s, q, o, sc.cams, torch.from_numpy(coeffs.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    ref32, pb = oracle.render(sc, coeffs.astype(np.float32).astype(np.float64), with_bound=True)
    print(parity.check_render(img.cpu().numpy(), ref32, pb, label="render bin32"), flush=True)
