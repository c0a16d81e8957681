"""Gradients of the re-render loss at the differentiation workload's full
size against the FP64 oracle (spec item: colorize + render + both
adjoints on 300k Gaussians).

    L = mean over (view, pixel, channel) of (render(colorize(y1, o), o) - y2)^2

The oracle takes about ten minutes of host time at this size, more than the
round of GPU tests allows, so these run only with GSC_FULL_SIZE=1.

test_full_size_production: 300k Gaussians, 100 views of 800x800, production
  options (t_min = 1e-4).  Relative L2 of dL/dy1 and dL/do <= 1e-4 against
  the oracle's composed adjoints, and 32 target entries on covered pixels
  within 1e-3 of their central difference (exact for targets: L is
  quadratic in y1 and no decision depends on it; tests/fdcheck.py).

test_opacity_fd_entries: the same geometry and image size seen from 8 of the
  views, t_min = 0 (then no decision depends on an opacity in [0.40, 0.98]:
  the footprint is bounded by q <= 9 before alpha_min, and o G < 0.99).
  Relative L2 of both gradients <= 1e-4, and 32 opacity entries within 1e-3
  of their incremental central difference (h = 1e-3).  The entries are drawn
  among observed Gaussians with o in [0.40, 0.98], a gradient above 1e-3 of
  the largest (smaller ones are below the resolution of the loss) and a
  scale at most the median (the difference walks every pixel of the
  Gaussian's footprint in every view)."""
import os

import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import fdcheck

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("GSC_FULL_SIZE") != "1",
                                 reason="full differentiation size: the oracle takes ~10 minutes "
                                        "(run with GSC_FULL_SIZE=1)")]


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


def _threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _gpu_grads(gsc_mod, sc, y1, y2, **opts):
    import torch
    from paper_2604_17155_amd import autograd as ag
    ctx = gsc_mod.Context(**opts)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    y1_t = torch.from_numpy(np.ascontiguousarray(y1, np.float32)).cuda().requires_grad_(True)
    y2_t = torch.from_numpy(np.ascontiguousarray(y2, np.float32)).cuda()
    o_t = o.clone().requires_grad_(True)
    c = ag.colorize(y1_t, o_t, m, s, q, sc.cams, sc.sh_deg, list(sc.lam), context=ctx, reuse_binning=True)
    img = ag.render(c, o_t, m, s, q, sc.cams, context=ctx, reuse_binning=True)
    loss = ((img - y2_t) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    return y1_t.grad.cpu().numpy().astype(np.float64), o_t.grad.cpu().numpy().astype(np.float64), \
        float(loss.detach())


def _rel_l2(a, ref):
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def test_full_size_production(gsc_mod):
    sc = syn.make_diff()
    opts = oracle.Options()
    print(f"[case] gradients at full size: {sc.N} Gaussians, {len(sc.cams)} views, "
          f"{sc.n_pixels} pixels, t_min = 1e-4", flush=True)
    y1 = oracle.make_targets(sc, 0, opts=opts, threads=_threads())
    y2 = oracle.make_targets(sc, 1, opts=opts, threads=_threads())
    print("oracle targets done", flush=True)
    base = fdcheck.loss_and_parts(sc, y1, y2, opts, threads=_threads())
    print(f"oracle loss and adjoints done: L = {base.loss:.6e}", flush=True)
    gy, go, loss = _gpu_grads(gsc_mod, sc, y1, y2)
    ey, eo = _rel_l2(gy, base.grad_y), _rel_l2(go, base.grad_o)
    print(f"GPU L = {loss:.6e}; rel L2: dL/dy1 {ey:.2e}, dL/do {eo:.2e}", flush=True)
    assert ey <= 1e-4 and eo <= 1e-4
    # 32 target entries on covered pixels
    rng = np.random.default_rng(11)
    worst = 0.0
    covered = np.flatnonzero(np.abs(base.img).sum(axis=1) > 0)
    for row in rng.choice(covered, 32, replace=False):
        ch = int(rng.integers(0, sc.C))
        fd = fdcheck.fd_target(base, int(row), ch, threads=_threads())
        err = abs(gy[row, ch] - fd) / max(abs(fd), 1e-30)
        worst = max(worst, err)
        assert err <= 1e-3, (row, ch, gy[row, ch], fd)
    print(f"32 target entries: largest relative difference to the central difference {worst:.2e}", flush=True)


def test_opacity_fd_entries(gsc_mod):
    sc = syn.make_diff()
    sc.cams = sc.cams[:8]
    opts = oracle.Options(t_min=0.0)
    print(f"[case] opacity FD: {sc.N} Gaussians, {len(sc.cams)} views of 800x800, t_min = 0", flush=True)
    y1 = oracle.make_targets(sc, 0, opts=opts, threads=_threads())
    y2 = oracle.make_targets(sc, 1, opts=opts, threads=_threads())
    base = fdcheck.loss_and_parts(sc, y1, y2, opts, threads=_threads())
    print(f"oracle loss and adjoints done: L = {base.loss:.6e}", flush=True)
    gy, go, loss = _gpu_grads(gsc_mod, sc, y1, y2, t_min=0.0)
    ey, eo = _rel_l2(gy, base.grad_y), _rel_l2(go, base.grad_o)
    print(f"GPU L = {loss:.6e}; rel L2: dL/dy1 {ey:.2e}, dL/do {eo:.2e}", flush=True)
    assert ey <= 1e-4 and eo <= 1e-4
    o = sc.opacities
    ok = (base.w > 0) & (o >= 0.40) & (o <= 0.98)
    ok &= np.abs(base.grad_o) >= 1e-3 * np.abs(base.grad_o[ok]).max()
    ok &= sc.scales.max(axis=1) <= np.median(sc.scales.max(axis=1))
    picks = np.random.default_rng(12).choice(np.flatnonzero(ok), 32, replace=False)
    worst = 0.0
    for k, g in enumerate(picks):
        fd = fdcheck.fd_opacity(base, int(g), 1e-3, threads=_threads())
        err = abs(go[g] - fd) / abs(fd)
        worst = max(worst, err)
        print(f"  opacity {k + 1}/32 (g {g}): GPU {go[g]:.6e} FD {fd:.6e} ({err:.1e})", flush=True)
        assert err <= 1e-3
    print(f"32 opacity entries: largest relative difference {worst:.2e}", flush=True)
