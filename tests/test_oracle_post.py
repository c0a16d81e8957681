"""Pins of the oracle's post-processing (Sec. 4.1 qualitative results: light
fields are linear, so coefficient sets combine and filter; Sec. 4.3: Gaussians
whose mask value falls below 0.6 are removed).

- combine: a combination of coefficient sets equals the colorization of the
  same combination of the targets (colorize is linear in the targets), and a
  per-channel filter equals colorizing filtered targets.
- mask value: equals the colour averaged over the sphere, computed by an
  exact product quadrature of the SH basis; at L = 0 it is the colour in every
  direction.
- segmentation: on disjoint splats with a constant mask value v_g on each
  splat's pixels, the L = 0 solve gives the value Y0^2/(Y0^2+lambda) v_g in
  closed form, so which splats the 0.6 threshold keeps is known in advance.
"""
import math

import numpy as np
import pytest

import oracle
from tests import tiny


def test_combine_equals_colorize_of_combined_targets(oracle_lib):
    sc = tiny.random_scene(61, n=40, n_cams=5, res=20, sh_deg=2, C=3, aniso=True)
    rng = np.random.default_rng(61)
    y1 = rng.uniform(0, 1, (sc.n_pixels, 3))
    y2 = rng.uniform(-1, 1, (sc.n_pixels, 3))
    y3 = rng.uniform(0, 2, (sc.n_pixels, 3))
    w = np.array([0.75, -1.25, 0.5], np.float32)
    filt = np.array([1.0, 0.5, 0.25], np.float32)
    cs = [oracle.colorize(sc, y)["coeffs"] for y in (y1, y2, y3)]  # FP64 targets
    mixed = w[0] * y1 + w[1] * y2 + w[2] * y3
    ref = oracle.colorize(sc, mixed)["coeffs"]
    got = oracle.combine(cs, w)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)
    # a colour filter is the colorization of filtered targets
    ref_f = oracle.colorize(sc, mixed * filt.astype(np.float64))["coeffs"]
    np.testing.assert_allclose(oracle.combine(cs, w, filt), ref_f, rtol=0, atol=1e-12 * scale)
    # a filter acts on channels (the last axis), not on coefficients
    assert not np.allclose(oracle.combine(cs, w, filt), oracle.combine(cs, w) * filt[0])


def _sphere_average(L, c):
    """Exact mean over the unit sphere of phi(d)^T c: Gauss-Legendre in
    z = cos(theta) (exact to degree 2n-1) times uniform nodes in the azimuth
    (exact for trigonometric degree < n_phi)."""
    z, wz = np.polynomial.legendre.leggauss(L + 2)
    n_phi = 2 * L + 3
    ph = 2 * math.pi * np.arange(n_phi) / n_phi
    zz, pp = np.meshgrid(z, ph, indexing="ij")
    r = np.sqrt(1 - zz ** 2)
    dirs = np.stack([r * np.cos(pp), r * np.sin(pp), zz], -1).reshape(-1, 3)
    wts = (np.repeat(wz, n_phi) / 2.0 / n_phi)  # weights sum to 1
    phi = oracle.sh_basis(L, dirs)  # [n_dirs, nb]
    return np.einsum("d,dm,gmc->gc", wts, phi, c)


@pytest.mark.parametrize("L", [0, 1, 3])
def test_mask_value_is_the_direction_average(oracle_lib, L):
    rng = np.random.default_rng(62 + L)
    c = rng.normal(0, 1, (200, (L + 1) ** 2, 2))
    avg = _sphere_average(L, c)
    for ch in range(2):
        v = oracle.mask_value(c, ch).astype(np.float64)
        np.testing.assert_allclose(v, avg[:, ch], rtol=3e-7, atol=1e-7)  # three binary32 roundings
    if L == 0:
        # the colour itself, in any direction
        d = rng.normal(size=(5, 3))
        col = oracle.sh_basis(0, d)[:, 0]
        np.testing.assert_allclose(oracle.mask_value(c, 1), col[0] * c[:, 0, 1], rtol=3e-7)
        assert np.allclose(col, col[0])


def test_mask_filter_decisions(oracle_lib):
    """>= keeps ties; status drops unobserved and failed but not ill-conditioned."""
    y0 = np.float32(oracle.sh_basis(0, np.array([[0.0, 0.0, 1.0]]))[0, 0])
    thr = np.float32(0.6)
    # the smallest binary32 coefficient whose binary32 mask value reaches the
    # threshold, and its neighbours
    c = np.float32(thr / y0)
    while np.float32(y0 * c) >= thr:
        c = np.nextafter(c, np.float32(0))
    while np.float32(y0 * c) < thr:
        c = np.nextafter(c, np.float32(4))
    cands = [np.nextafter(c, np.float32(0)), c, np.nextafter(c, np.float32(4))]
    coeffs = np.zeros((6, 1, 1), np.float32)
    coeffs[:3, 0, 0] = cands
    coeffs[3:, 0, 0] = 5.0
    keep, idx = oracle.mask_filter(coeffs, 0, 0.6)
    assert list(keep[:3]) == [False, True, True]
    status = np.array([0, 0, 0, oracle.UNOBSERVED, oracle.FAILED, oracle.ILL_COND], np.uint8)
    keep_s, idx_s = oracle.mask_filter(coeffs, 0, 0.6, status)
    assert list(keep_s[3:]) == [False, False, True]
    assert list(idx_s) == [i for i in range(6) if keep_s[i]]


def test_segmentation_closed_form_on_disjoint_splats(oracle_lib):
    rng = np.random.default_rng(64)
    g = np.stack(np.meshgrid(np.arange(4), np.arange(3), indexing="ij"), -1).reshape(-1, 2)
    n = g.shape[0]
    means = np.zeros((n, 3), np.float32)
    means[:, 0] = (g[:, 0] - 1.5) * 0.45
    means[:, 1] = (g[:, 1] - 1.0) * 0.45
    cams = [tiny.axis_camera(64, 64, z=-3.0), tiny.axis_camera(48, 48, z=-2.5)]
    lam = 1e-4
    sc = tiny.scene(means, np.full((n, 3), 0.04), tiny.identity_quats(n),
                    rng.uniform(0.4, 0.9, n), cams, sh_deg=0, C=2, lam=[lam])
    idx, w = oracle.contributions(sc)
    _, counts = np.unique(idx[:, 1], return_counts=True)
    assert counts.max() == 1  # no pixel sees two splats
    assert set(idx[:, 2].tolist()) == set(range(n))
    # mask values around the threshold, one per splat; channel 1 is 1 - channel 0
    y0sq = 1.0 / (4 * math.pi)
    shrink = y0sq / (y0sq + lam)
    v = np.array([1.0, 0.0, 0.7, 0.55, 0.6 / shrink * (1 + 1e-4), 0.6 / shrink * (1 - 1e-4),
                  0.9, 0.3, 0.61, 0.59, 1.0, 0.0])
    y = np.zeros((sc.n_pixels, 2))
    for (_, row, gg) in idx:
        y[row] = [v[gg], 1.0 - v[gg]]
    r = oracle.colorize(sc, y)
    value = shrink * v
    np.testing.assert_allclose(oracle.mask_value(r["coeffs"], 0), value, rtol=1e-6, atol=1e-7)
    keep, kept = oracle.mask_filter(r["coeffs"], 0, 0.6, r["status"])
    assert list(keep) == list(value >= 0.6)
    keep1, _ = oracle.mask_filter(r["coeffs"], 1, 0.6, r["status"])
    assert list(keep1) == list(shrink * (1 - v) >= 0.6)
