"""GPU parity of the adjoints (gsc_colorize_backward, gsc_render_backward and
the autograd wrappers) against the FP64 oracle's adjoints.

Gate.  Per output tensor the relative L2 error ||g_gpu - g_ref|| / ||g_ref||
must stay within 1e-4.  Pixel decisions whose inputs sit within rounding of a
threshold (footprint edge, alpha floor, early stop) may go either way in the
FP32 kernel and the FP64 oracle; each such pixel perturbs the gradients at
that pixel by up to O(alpha_min) relative, so several results are correct
there.  Most cases therefore use blending options under which no decision
can move a weight by more than ~1e-8: no alpha floor, no early stop, and a
6-sigma footprint (exp(-18) ~ 1.5e-8 at its edge).  The production options
(alpha floor 1/255, early stop 1e-4, 3-sigma footprint) are compared too; on
these seeded inputs their near-threshold decisions are rare enough that the
same 1e-4 gate holds, and the median element error must stay below 1e-5 of
the largest gradient.

At full size the adjoint identities are checked on the GPU alone:
<dL/dy, dy> = <dL/dc, colorize(dy)> (colorize is linear in the targets) and
<dL/dc, dc> = <dL/dimages, render(dc)> (render is linear in the coefficients).
With random test vectors each inner product <a, b> cancels down to about
||a|| ||b|| / sqrt(n), so its rounding is stated relative to ||a|| ||b||: the
two sides must agree to 1e-6 of that scale (FP32 accumulation in both).
"""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import parity

pytestmark = pytest.mark.gpu

SMOOTH = dict(alpha_min=0.0, t_min=0.0, sigma_cut=6.0)
TOL_GRAD = 1e-4
TOL_GRAD_PRODUCTION = 1e-4


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
def ctx_smooth(gsc_mod):
    return gsc_mod.Context(**SMOOTH)


@pytest.fixture(scope="module")
def ctx_prod(gsc_mod):
    return gsc_mod.Context()


def smooth_opts():
    return oracle.Options(alpha_min=0.0, t_min=0.0, sigma_cut=6.0)


def rel_l2(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def colorize_backward_case(ctx, sc, y, opts, label, seed=0):
    """GPU and oracle adjoints of colorize at the same (float32) coefficients and
    upstream gradient.  Returns the relative L2 errors (targets, opacities)."""
    import torch
    from paper_2604_17155_amd import gsc
    print(f"[case] {label}: N={sc.N} cams={len(sc.cams)} L={sc.sh_deg} C={sc.C} dtype={y.dtype}", flush=True)
    ref = oracle.colorize(sc, y, opts=opts)
    c32 = ref["coeffs"].astype(np.float32)
    G = np.random.default_rng(seed).standard_normal(c32.shape).astype(np.float32)
    gt_ref, go_ref = oracle.colorize_backward(sc, y, c32.astype(np.float64), G.astype(np.float64),
                                              opts=opts)
    m, s, q, o = gsc.scene_tensors(sc)
    gt, go = ctx.colorize_backward(m, s, q, o, sc.cams, parity.to_device_targets(y), sc.sh_deg,
                                   list(sc.lam), _dev(c32), _dev(G))
    torch.cuda.synchronize()
    gt, go = gt.cpu().numpy(), go.cpu().numpy()
    et, eo = rel_l2(gt, gt_ref), rel_l2(go, go_ref)
    med_t = float(np.median(np.abs(gt - gt_ref)) / max(np.abs(gt_ref).max(), 1e-300))
    med_o = float(np.median(np.abs(go - go_ref)) / max(np.abs(go_ref).max(), 1e-300))
    print(f"{label}: grad_targets rel L2 {et:.2e} (median |d|/max {med_t:.1e}); "
          f"grad_opacities rel L2 {eo:.2e} (median |d|/max {med_o:.1e})", flush=True)
    # unobserved Gaussians get exactly zero
    un = (ref["status"] & 1) == 1
    assert np.all(go[un] == 0.0)
    return et, eo, med_t, med_o


def test_colorize_backward_smooth_l3(ctx_smooth):
    sc = syn.make_relight(n=6000, n_cams=8, res=128)
    y = oracle.make_targets(sc)
    et, eo, _, _ = colorize_backward_case(ctx_smooth, sc, y, smooth_opts(), "colorize adjoint L3 C3 smooth")
    assert et <= TOL_GRAD and eo <= TOL_GRAD


def test_colorize_backward_production_options(ctx_prod):
    sc = syn.make_relight(n=6000, n_cams=8, res=128)
    y = oracle.make_targets(sc)
    et, eo, mt, mo = colorize_backward_case(ctx_prod, sc, y, oracle.Options(),
                                            "colorize adjoint L3 C3 production options")
    assert et <= TOL_GRAD_PRODUCTION and eo <= TOL_GRAD_PRODUCTION
    assert mt <= 1e-5 and mo <= 1e-5


def test_colorize_backward_bf16_channel_chunks(ctx_smooth):
    """L=0, C=20 BF16 targets: two channel chunks (16 + 4) share dL/do."""
    sc = syn.make_segment_scene(1, n_override=5000, cams_override=6, C=20)
    sc.cams = syn.hemisphere_cams(6, 3.0, 120, 96)
    y = oracle.make_targets(sc)
    assert y.dtype == np.uint16
    et, eo, _, _ = colorize_backward_case(ctx_smooth, sc, y, smooth_opts(),
                                          "colorize adjoint L0 C20 bf16 smooth", seed=1)
    assert et <= TOL_GRAD and eo <= TOL_GRAD


def test_colorize_backward_l2_c5_ragged(ctx_smooth):
    rng = np.random.Generator(np.random.PCG64(11))
    sc = syn.make_relight(n=3000, n_cams=5, res=64, sh_deg=2,
                          lam=rng.uniform(1e-4, 1e-2, 9).astype(np.float32))
    sc.cams = syn.hemisphere_cams(5, 3.0, 150, 90)
    sc.C = 5
    sc.gt = [np.concatenate([sc.gt[0], sc.gt[0][:, :, :2] * 0.5], axis=2)]
    y = oracle.make_targets(sc)
    et, eo, _, _ = colorize_backward_case(ctx_smooth, sc, y, smooth_opts(),
                                          "colorize adjoint L2 C5 ragged smooth", seed=2)
    assert et <= TOL_GRAD and eo <= TOL_GRAD


def test_render_backward_smooth(ctx_smooth, gsc_mod):
    import torch
    sc = syn.make_relight(n=6000, n_cams=8, res=128)
    opts = smooth_opts()
    c32 = sc.gt[0].astype(np.float32)
    gi = np.random.default_rng(3).standard_normal((sc.n_pixels, 3)).astype(np.float32)
    gc_ref, go_ref = oracle.render_backward(sc, c32.astype(np.float64), gi.astype(np.float64), opts=opts)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    gc, go = ctx_smooth.render_backward(m, s, q, o, sc.cams, _dev(c32), _dev(gi))
    torch.cuda.synchronize()
    ec, eo = rel_l2(gc.cpu().numpy(), gc_ref), rel_l2(go.cpu().numpy(), go_ref)
    print(f"render adjoint L3 C3 smooth: grad_coeffs rel L2 {ec:.2e}; grad_opacities rel L2 {eo:.2e}",
          flush=True)
    assert ec <= TOL_GRAD and eo <= TOL_GRAD


def test_render_backward_l1_five_channels(ctx_smooth, gsc_mod):
    """L = 1, C = 5 on 150x90 views: transposed coefficient reads for every
    (m, c) row in the render adjoint."""
    import torch
    rng = np.random.default_rng(5)
    sc = syn.make_relight(n=3000, n_cams=5, res=64, sh_deg=1)
    sc.cams = syn.hemisphere_cams(5, 3.0, 150, 90)
    sc.C = 5
    c32 = (rng.normal(0.0, 0.3, (sc.N, 4, 5)) + np.array([0.5, 0, 0, 0])[None, :, None]).astype(np.float32)
    gi = rng.standard_normal((sc.n_pixels, 5)).astype(np.float32)
    gc_ref, go_ref = oracle.render_backward(sc, c32.astype(np.float64), gi.astype(np.float64),
                                            opts=smooth_opts())
    m, s, q, o = gsc_mod.scene_tensors(sc)
    gc, go = ctx_smooth.render_backward(m, s, q, o, sc.cams, _dev(c32), _dev(gi))
    torch.cuda.synchronize()
    ec, eo = rel_l2(gc.cpu().numpy(), gc_ref), rel_l2(go.cpu().numpy(), go_ref)
    print(f"render adjoint L1 C5 smooth: grad_coeffs {ec:.2e}; grad_opacities {eo:.2e}", flush=True)
    assert ec <= TOL_GRAD and eo <= TOL_GRAD


def test_render_backward_l0_production(ctx_prod, gsc_mod):
    import torch
    sc = syn.make_plain()
    c32 = sc.gt[0].astype(np.float32)
    gi = np.random.default_rng(4).standard_normal((sc.n_pixels, 3)).astype(np.float32)
    gc_ref, go_ref = oracle.render_backward(sc, c32.astype(np.float64), gi.astype(np.float64))
    m, s, q, o = gsc_mod.scene_tensors(sc)
    gc, go = ctx_prod.render_backward(m, s, q, o, sc.cams, _dev(c32), _dev(gi))
    torch.cuda.synchronize()
    ec, eo = rel_l2(gc.cpu().numpy(), gc_ref), rel_l2(go.cpu().numpy(), go_ref)
    print(f"render adjoint L0 plain production: grad_coeffs {ec:.2e}; grad_opacities {eo:.2e}", flush=True)
    assert ec <= TOL_GRAD_PRODUCTION and eo <= TOL_GRAD_PRODUCTION


def test_autograd_rerender_loss(ctx_smooth, gsc_mod):
    """L = mean((render(colorize(y1, o), o) - y2)^2) through the autograd
    wrappers against the oracle's composed adjoints."""
    import torch
    from paper_2604_17155_amd import autograd as ag
    sc = syn.make_diff(n=5000, n_cams=8, res=128)
    opts = smooth_opts()
    y1 = oracle.make_targets(sc, 0)
    y2 = oracle.make_targets(sc, 1)
    # oracle chain
    c = oracle.colorize(sc, y1, opts=opts)["coeffs"]
    img = oracle.render(sc, c, opts=opts)
    ibar = 2.0 * (img - y2) / img.size
    gc, go_r = oracle.render_backward(sc, c, ibar, opts=opts)
    gy_ref, go_c = oracle.colorize_backward(sc, y1, c, gc, opts=opts)
    go_ref = go_r + go_c
    # GPU chain
    m, s, q, o = gsc_mod.scene_tensors(sc)
    y1_t = _dev(y1).requires_grad_(True)
    o_t = o.clone().requires_grad_(True)
    coeffs = ag.colorize(y1_t, o_t, m, s, q, sc.cams, sc.sh_deg, list(sc.lam), context=ctx_smooth)
    images = ag.render(coeffs, o_t, m, s, q, sc.cams, context=ctx_smooth)
    loss = ((images - _dev(y2)) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    ey = rel_l2(y1_t.grad.cpu().numpy(), gy_ref)
    eo = rel_l2(o_t.grad.cpu().numpy(), go_ref)
    print(f"autograd rerender loss: dL/dy1 rel L2 {ey:.2e}; dL/do rel L2 {eo:.2e}; "
          f"loss gpu {float(loss):.6e} oracle {((img - y2) ** 2).mean():.6e}", flush=True)
    assert ey <= TOL_GRAD and eo <= TOL_GRAD


def test_binning_reuse(gsc_mod):
    """Calls on the same, unmodified geometry tensors reuse the previous call's
    tile lists (no projection launched) with the same result as a fresh
    binning; an in-place change of the opacities, other cameras, or a call
    that does not allow reuse bin anew."""
    import torch
    sc = syn.make_relight(seed_offset=31, n=6000, n_cams=6, res=128)
    y = _dev(oracle.make_targets(sc))
    m, s, q, o = gsc_mod.scene_tensors(sc)
    lam = list(sc.lam)
    ctx = gsc_mod.Context(flags=gsc_mod.GSC_FLAG_PROFILE)
    fresh = gsc_mod.Context()

    def projected(c):
        return int(c.stats().stage_launches[0])

    c1, _ = ctx.colorize(m, s, q, o, sc.cams, y, sc.sh_deg, lam, reuse_binning=True)
    torch.cuda.synchronize()
    assert projected(ctx) > 0  # nothing to reuse yet
    c2, _ = ctx.colorize(m, s, q, o, sc.cams, y, sc.sh_deg, lam, reuse_binning=True)
    torch.cuda.synchronize()
    assert projected(ctx) == 0  # reused
    img = ctx.render(m, s, q, o, sc.cams, c2, reuse_binning=True)
    torch.cuda.synchronize()
    assert projected(ctx) == 0
    ref, _ = fresh.colorize(m, s, q, o, sc.cams, y, sc.sh_deg, lam)
    img_ref = fresh.render(m, s, q, o, sc.cams, ref)
    torch.cuda.synchronize()
    assert torch.allclose(c2, ref, rtol=1e-5, atol=1e-6)
    assert torch.allclose(img, img_ref, rtol=1e-5, atol=1e-6)
    # an in-place change of the opacities: new binning, new result
    o.mul_(0.8)
    c3, _ = ctx.colorize(m, s, q, o, sc.cams, y, sc.sh_deg, lam, reuse_binning=True)
    torch.cuda.synchronize()
    assert projected(ctx) > 0
    ref3, _ = fresh.colorize(m, s, q, o, sc.cams, y, sc.sh_deg, lam)
    torch.cuda.synchronize()
    assert torch.allclose(c3, ref3, rtol=1e-5, atol=1e-6)
    assert not torch.allclose(c3, ref, rtol=1e-3, atol=1e-4)
    # other cameras
    ctx.colorize(m, s, q, o, sc.cams[:4], y, sc.sh_deg, lam, reuse_binning=True)
    torch.cuda.synchronize()
    assert projected(ctx) > 0
    # reuse not allowed by the caller
    ctx.colorize(m, s, q, o, sc.cams[:4], y, sc.sh_deg, lam)
    torch.cuda.synchronize()
    assert projected(ctx) > 0


def test_autograd_sees_data_edits(gsc_mod):
    """The autograd wrappers bin anew on every call unless asked not to, so an
    opacity update written through `.data` (which leaves torch's version
    counter alone) reaches the next call's coefficients."""
    import torch
    from paper_2604_17155_amd import autograd as ag
    sc = syn.make_relight(seed_offset=37, n=5000, n_cams=6, res=128)
    y = _dev(oracle.make_targets(sc))
    m, s, q, o = gsc_mod.scene_tensors(sc)
    lam = list(sc.lam)
    ctx = gsc_mod.Context(flags=gsc_mod.GSC_FLAG_PROFILE)
    fresh = gsc_mod.Context()
    o_p = o.clone().requires_grad_(True)
    ag.colorize(y, o_p, m, s, q, sc.cams, sc.sh_deg, lam, context=ctx)
    v0 = o_p._version
    o_p.data.mul_(0.7)
    assert o_p._version == v0  # the write is invisible to the version guard
    c2 = ag.colorize(y, o_p, m, s, q, sc.cams, sc.sh_deg, lam, context=ctx)
    torch.cuda.synchronize()
    assert int(ctx.stats().stage_launches[0]) > 0  # projected again
    ref, _ = fresh.colorize(m, s, q, o_p.detach(), sc.cams, y, sc.sh_deg, lam)
    torch.cuda.synchronize()
    assert torch.allclose(c2.detach(), ref, rtol=1e-5, atol=1e-6)
    # opting in reuses the lists when nothing changed
    ag.colorize(y, o_p, m, s, q, sc.cams, sc.sh_deg, lam, context=ctx, reuse_binning=True)
    torch.cuda.synchronize()
    assert int(ctx.stats().stage_launches[0]) == 0


def test_backward_degenerate(ctx_prod, gsc_mod):
    import torch
    from tests import tiny
    # no cameras: every gradient is zero
    sc = tiny.random_scene(3, n=20, n_cams=0, sh_deg=1, C=2)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    y = torch.zeros((1, 2), device="cuda")
    c = torch.ones((20, 4, 2), device="cuda")
    gt, go = ctx_prod.colorize_backward(m, s, q, o, sc.cams, y, 1, [1e-4, 1e-3], c, c)
    assert torch.all(go == 0) and torch.all(gt == 0)
    gc, go = ctx_prod.render_backward(m, s, q, o, sc.cams, c, y)
    assert torch.all(gc == 0) and torch.all(go == 0)


def test_adjoint_identities_full_size(ctx_prod, gsc_mod):
    """The differentiable workload at full size (300k Gaussians, 100 x 800^2,
    L=3, C=3): <dL/dy, dy> = <G, colorize(dy)> and <dL/dc, dc> = <gi, render(dc)>."""
    import torch
    sc = syn.make_diff()
    print(f"[case] adjoint identities: N={sc.N} cams={len(sc.cams)} rows={sc.n_pixels}", flush=True)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    gen = torch.Generator(device="cuda").manual_seed(5)
    rows = sc.n_pixels
    nb = (sc.sh_deg + 1) ** 2
    dy = torch.randn((rows, 3), device="cuda", generator=gen)
    G = torch.randn((sc.N, nb, 3), device="cuda", generator=gen)
    lam = list(sc.lam)
    c_dy, _ = ctx_prod.colorize(m, s, q, o, sc.cams, dy, sc.sh_deg, lam)
    gt, _ = ctx_prod.colorize_backward(m, s, q, o, sc.cams, dy, sc.sh_deg, lam, c_dy, G,
                                       want_opacities=False)
    lhs = float((gt.double() * dy.double()).sum())
    rhs = float((G.double() * c_dy.double()).sum())
    scale = float(G.double().norm() * c_dy.double().norm())
    print(f"colorize adjoint identity: {lhs:.9e} vs {rhs:.9e} (|d|/||G|| ||c|| = "
          f"{abs(lhs - rhs) / scale:.1e}, |d|/|rhs| = {abs(lhs - rhs) / abs(rhs):.1e})", flush=True)
    assert abs(lhs - rhs) <= 1e-6 * scale
    dc = torch.randn((sc.N, nb, 3), device="cuda", generator=gen)
    gi = torch.randn((rows, 3), device="cuda", generator=gen)
    img = ctx_prod.render(m, s, q, o, sc.cams, dc)
    gc, _ = ctx_prod.render_backward(m, s, q, o, sc.cams, dc, gi, want_opacities=False)
    lhs = float((gc.double() * dc.double()).sum())
    rhs = float((gi.double() * img.double()).sum())
    scale = float(gi.double().norm() * img.double().norm())
    print(f"render adjoint identity: {lhs:.9e} vs {rhs:.9e} (|d|/||gi|| ||img|| = "
          f"{abs(lhs - rhs) / scale:.1e}, |d|/|rhs| = {abs(lhs - rhs) / abs(rhs):.1e})", flush=True)
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_colorize_backward_bins_of_32_pixels(gsc_mod):
    ctx = gsc_mod.Context(bin_size=32, **SMOOTH)
    sc = syn.make_relight(n=6000, n_cams=8, res=128)
    y = oracle.make_targets(sc)
    et, eo, _, _ = colorize_backward_case(ctx, sc, y, smooth_opts(), "colorize adjoint L3 C3 smooth bin32")
    assert et <= TOL_GRAD and eo <= TOL_GRAD


@pytest.mark.parametrize("schedule", [1, 2])
def test_backward_tile_schedules(gsc_mod, schedule):
    """Colorize and render adjoints with tiles in index order (grid) and
    longest lists first."""
    import torch
    ctx = gsc_mod.Context(schedule=schedule, **SMOOTH)
    sc = syn.make_relight(n=6000, n_cams=8, res=128)
    y = oracle.make_targets(sc)
    et, eo, _, _ = colorize_backward_case(ctx, sc, y, smooth_opts(), f"colorize adjoint schedule {schedule}")
    assert et <= TOL_GRAD and eo <= TOL_GRAD
    c32 = sc.gt[0].astype(np.float32)
    gi = np.random.default_rng(3).standard_normal((sc.n_pixels, 3)).astype(np.float32)
    gc_ref, go_ref = oracle.render_backward(sc, c32.astype(np.float64), gi.astype(np.float64),
                                            opts=smooth_opts())
    m, s, q, o = gsc_mod.scene_tensors(sc)
    gc, go = ctx.render_backward(m, s, q, o, sc.cams, _dev(c32), _dev(gi))
    torch.cuda.synchronize()
    ec, eo2 = rel_l2(gc.cpu().numpy(), gc_ref), rel_l2(go.cpu().numpy(), go_ref)
    print(f"render adjoint schedule {schedule}: grad_coeffs {ec:.2e}; grad_opacities {eo2:.2e}", flush=True)
    assert ec <= TOL_GRAD and eo2 <= TOL_GRAD
