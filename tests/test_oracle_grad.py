"""Pins of the oracle's adjoints: dot-product tests for the linear maps and
central finite differences for the opacities.

colorize is linear in the targets, so <dL/dy, dy> must equal the change of L
exactly.  Opacity derivatives are compared with central differences with the
early stop disabled (T_min = 0) and opacities in [0.4, 0.98]: there no pixel
decision depends on the perturbed opacity (alpha stays above alpha_min inside
the 3-sigma footprint and below alpha_max), so L is smooth in o.
"""
import numpy as np
import pytest

import oracle
from tests import tiny

H = 2.0 ** -10  # exact in float32 around the chosen opacities


def _smooth_scene(seed, sh_deg, C, n=30):
    sc = tiny.random_scene(seed, n=n, n_cams=5, res=20, sh_deg=sh_deg, C=C, aniso=True,
                           opac_range=(0.45, 0.9), log_scale=-2.4)
    # opacities on a 2^-10 grid so that o +- H is exact
    sc.opacities = (np.round(sc.opacities * 1024) / 1024).astype(np.float32)
    return sc


def test_target_adjoint_dot_product(oracle_lib):
    sc = _smooth_scene(60, 3, 3)
    rng = np.random.default_rng(0)
    y = rng.uniform(0, 1, (sc.n_pixels, 3)).astype(np.float32)
    r = oracle.colorize(sc, y)
    G = rng.standard_normal(r["coeffs"].shape)
    gy, _ = oracle.colorize_backward(sc, y, r["coeffs"], G)
    dy = rng.standard_normal(y.shape).astype(np.float32)
    lhs = (gy * dy.astype(np.float64)).sum()
    rhs = (G * oracle.colorize(sc, dy)["coeffs"]).sum()
    assert abs(lhs - rhs) <= 1e-11 * abs(rhs)


@pytest.mark.parametrize("sh_deg", [0, 3])
def test_opacity_adjoint_of_colorize_fd(oracle_lib, sh_deg):
    sc = _smooth_scene(61 + sh_deg, sh_deg, 2)
    opts = oracle.Options(t_min=0.0)
    rng = np.random.default_rng(1)
    y = rng.uniform(0, 1, (sc.n_pixels, 2)).astype(np.float32)
    r = oracle.colorize(sc, y, opts=opts)
    G = rng.standard_normal(r["coeffs"].shape)
    _, go = oracle.colorize_backward(sc, y, r["coeffs"], G, opts=opts)
    obs = np.nonzero((r["status"] & 1) == 0)[0]
    base = sc.opacities.copy()
    for g in obs[:12]:
        vals = []
        for s in (+1, -1):
            sc.opacities = base.copy()
            sc.opacities[g] = np.float32(base[g] + s * H)
            vals.append((G * oracle.colorize(sc, y, opts=opts)["coeffs"]).sum())
        sc.opacities = base
        fd = (vals[0] - vals[1]) / (2 * H)
        assert abs(go[g] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.abs(go).max()), (g, go[g], fd)


def test_render_adjoints(oracle_lib):
    sc = _smooth_scene(64, 3, 3)
    opts = oracle.Options(t_min=0.0)
    rng = np.random.default_rng(2)
    c = rng.standard_normal((sc.N, 16, 3))
    gi = rng.standard_normal((sc.n_pixels, 3))
    gc, go = oracle.render_backward(sc, c, gi, opts=opts)
    dc = rng.standard_normal(c.shape)
    lhs = (gc * dc).sum()
    rhs = (gi * oracle.render(sc, dc, opts=opts)).sum()
    assert abs(lhs - rhs) <= 1e-11 * abs(rhs)
    base = sc.opacities.copy()
    for g in range(0, sc.N, 3):
        vals = []
        for s in (+1, -1):
            sc.opacities = base.copy()
            sc.opacities[g] = np.float32(base[g] + s * H)
            vals.append((gi * oracle.render(sc, c, opts=opts)).sum())
        sc.opacities = base
        fd = (vals[0] - vals[1]) / (2 * H)
        assert abs(go[g] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.abs(go).max()), (g, go[g], fd)


def test_rerender_loss_gradients(oracle_lib):
    """L = mean((render(colorize(y1, o), o) - y2)^2): gradients with respect to
    y1 and o composed from the two adjoints, checked by central differences."""
    sc = _smooth_scene(65, 3, 3)
    opts = oracle.Options(t_min=0.0)
    rng = np.random.default_rng(3)
    y1 = rng.uniform(0, 1, (sc.n_pixels, 3)).astype(np.float32)
    y2 = rng.uniform(0, 1, (sc.n_pixels, 3)).astype(np.float32)

    def loss(y1_, scene):
        c = oracle.colorize(scene, y1_, opts=opts)["coeffs"]
        img = oracle.render(scene, c, opts=opts)
        return ((img - y2) ** 2).mean(), c, img

    L0, c, img = loss(y1, sc)
    ibar = 2.0 * (img - y2) / img.size
    gc, go_r = oracle.render_backward(sc, c, ibar, opts=opts)
    gy, go_c = oracle.colorize_backward(sc, y1, c, gc, opts=opts)
    go = go_r + go_c
    # targets: pick covered entries; steps on a 2^-10 grid keep y1 +- h exact
    covered = np.nonzero(np.abs(gy).sum(1) > 0)[0]
    for row in rng.choice(covered, 8, replace=False):
        for ch in range(3):
            vals = []
            for s in (+1, -1):
                yy = y1.copy()
                yy[row, ch] = np.float32(y1[row, ch] + s * H)
                vals.append(loss(yy, sc)[0])
            hh = (np.float64(np.float32(y1[row, ch] + H)) - np.float64(np.float32(y1[row, ch] - H)))
            fd = (vals[0] - vals[1]) / hh
            assert abs(gy[row, ch] - fd) <= 1e-6 * np.abs(gy).max() + 1e-4 * abs(fd)
    base = sc.opacities.copy()
    for g in range(0, sc.N, 4):
        vals = []
        for s in (+1, -1):
            sc.opacities = base.copy()
            sc.opacities[g] = np.float32(base[g] + s * H)
            vals.append(loss(y1, sc)[0])
        sc.opacities = base
        fd = (vals[0] - vals[1]) / (2 * H)
        assert abs(go[g] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.abs(go).max()), (g, go[g], fd)
