"""Pin of the oracle's weight-error bound `werr` (the relative error that
binary32 evaluation of the pixel weights w = alpha T may put into a
Gaussian's per-view sum V_gj = sum_p w).

An independent binary32 blend, written here in numpy, evaluates the same
pixels: the conic and centre rounded once to binary32, q = a dx^2 + 2 b dx dy +
c dy^2, alpha = min(0.99, o exp(-q/2)) and T <- T (1 - alpha), all in binary32
(one implementation within the margin model).  On scenes where the oracle
records no near-threshold decision (so both walks accept the same Gaussians at
the same pixels), every per-view sum of the binary32 walk lies within
1 +- werr_g of the oracle's exact one."""
import numpy as np
import pytest

import oracle
from tests import tiny

F = np.float32


def _binary32_view_sums(sc, j, opts):
    P = oracle.project(sc, j, opts)
    cam = sc.cams[j]
    W, H = cam.width, cam.height
    vis = np.flatnonzero(P[:, 0] > 0)
    order = vis[np.lexsort((vis, P[vis, 1].astype(F)))]  # binary32 key, then index
    u, v = P[:, 2].astype(F), P[:, 3].astype(F)
    a, b, c = P[:, 4].astype(F), P[:, 5].astype(F), P[:, 6].astype(F)
    o = sc.opacities.astype(F)
    xs = (np.arange(W, dtype=F) + F(0.5))[None, :].repeat(H, 0)
    ys = (np.arange(H, dtype=F) + F(0.5))[:, None].repeat(W, 1)
    T = np.ones((H, W), F)
    live = np.ones((H, W), bool)
    V = np.zeros(sc.N)
    s2, amin, amax, tmin = F(opts.sigma_cut) ** 2, F(opts.alpha_min), F(opts.alpha_max), F(opts.t_min)
    for g in order:
        dx, dy = xs - u[g], ys - v[g]
        q = a[g] * dx * dx + F(2) * b[g] * dx * dy + c[g] * dy * dy
        al = np.minimum(amax, o[g] * np.exp(F(-0.5) * q))
        take = live & (q <= s2) & (al >= amin)
        test = T * (F(1) - al)
        stop = take & (test < tmin)
        live &= ~stop
        take &= ~stop
        V[g] += float((al * T)[take].astype(np.float64).sum())
        T = np.where(take, test, T)
    return V


@pytest.mark.parametrize("seed", [81, 82, 83])
def test_binary32_view_sums_within_werr(oracle_lib, seed):
    opts = oracle.Options()
    sc = tiny.random_scene(seed, n=25, n_cams=3, res=20, sh_deg=0, C=1, aniso=True,
                           opac_range=(0.3, 0.98))
    y = np.zeros((sc.n_pixels, 1), np.float32)
    ref = oracle.colorize(sc, y, opts=opts)
    if ref["events"] != 0:
        pytest.skip("scene has near-threshold decisions")
    idx, w = oracle.contributions(sc, opts)
    checked = 0
    for j in range(len(sc.cams)):
        V64 = np.zeros(sc.N)
        sel = idx[:, 0] == j
        np.add.at(V64, idx[sel, 2], w[sel])
        V32 = _binary32_view_sums(sc, j, opts)
        seen = V64 > 0
        assert np.array_equal(seen, V32 > 0)
        rel = np.abs(V32[seen] / V64[seen] - 1)
        bound = ref["werr"][seen] + 1e-12
        assert np.all(rel <= bound), (rel / bound).max()
        checked += int(seen.sum())
    assert checked > 20
    # the bound is not vacuous: it is a few hundred roundings at most here
    obs = (ref["status"] & 1) == 0
    assert ref["werr"][obs].max() < 3e-4


def test_werr_grows_behind_dense_layers(oracle_lib):
    """A Gaussian seen behind nearly opaque unclamped layers inherits their
    alpha error amplified by alpha / (1 - alpha)."""
    means = np.array([[0, 0, -0.4], [0, 0, 0.0]], np.float32)
    # a wide front layer at alpha ~ 0.97 over the whole of a small splat behind it
    scales = np.array([[1.0] * 3, [0.03] * 3])
    sc = tiny.scene(means, scales, tiny.identity_quats(2), [0.97, 0.5], [tiny.axis_camera(16, 16)], C=1)
    ref = oracle.colorize(sc, np.zeros((sc.n_pixels, 1), np.float32))
    assert ref["werr"][1] > 5 * ref["werr"][0] > 0
