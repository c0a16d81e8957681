"""Pins of the oracle's accumulate + solve (eqs. 10-15, Algorithm 1 steps 1-6).

The per-Gaussian result is compared with a dense least-squares solve
(numpy.linalg.lstsq) of the explicitly built weighted system, in both the
per-pixel form (eq. 10/11) and the per-view form (eq. 12), plus the L=0
closed form (eq. 7), linearity in the targets, constant targets, exact-fit
recovery on disjoint footprints and invariance under reordering.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import tiny


def _expanded_lambda(lam, L):
    nb = (L + 1) ** 2
    lam = np.asarray(lam, np.float64)
    if lam.size == 1:
        return np.full(nb, lam[0])
    if lam.size == L + 1:
        return np.concatenate([[lam[l]] * (2 * l + 1) for l in range(L + 1)])
    return lam


def _phi(sc, g, j):
    cam = sc.cams[j]
    centre = -cam.R.astype(np.float64).T @ cam.t.astype(np.float64)
    return oracle.sh_basis(sc.sh_deg, (sc.means[g].astype(np.float64) - centre)[None])[0]


def _lstsq_pixel_form(sc, y, idx, w):
    """min_c sum_{j,p} w (y_p - phi^T c)^2 + w_g sum_m lambda_m c_m^2, per g."""
    nb, C = sc.n_b, sc.C
    lamx = _expanded_lambda(sc.lam.astype(np.float64), sc.sh_deg)
    out = np.zeros((sc.N, nb, C))
    obs = np.zeros(sc.N, bool)
    for g in range(sc.N):
        sel = idx[:, 2] == g
        if not sel.any():
            continue
        obs[g] = True
        rows, rhs = [], []
        wg = w[sel].sum()
        for (j, row, _), ww in zip(idx[sel], w[sel]):
            rows.append(math.sqrt(ww) * _phi(sc, g, j))
            rhs.append(math.sqrt(ww) * y[row].astype(np.float64))
        for m in range(nb):
            e = np.zeros(nb)
            e[m] = math.sqrt(wg * lamx[m])
            rows.append(e)
            rhs.append(np.zeros(C))
        out[g] = np.linalg.lstsq(np.asarray(rows), np.asarray(rhs), rcond=None)[0]
    return out, obs


@pytest.mark.parametrize("sh_deg,C,aniso", [(0, 3, False), (2, 2, True), (3, 3, True)])
def test_matches_dense_lstsq_pixel_form(oracle_lib, sh_deg, C, aniso):
    sc = tiny.random_scene(20 + sh_deg, n=24, n_cams=7, res=20, sh_deg=sh_deg, C=C, aniso=aniso,
                           log_scale=-2.3)
    y = np.random.default_rng(5).uniform(0, 1, (sc.n_pixels, C)).astype(np.float32)
    r = oracle.colorize(sc, y)
    idx, w = oracle.contributions(sc)
    ref, obs = _lstsq_pixel_form(sc, y, idx, w)
    assert obs.sum() >= 10
    np.testing.assert_allclose(r["coeffs"][obs], ref[obs], rtol=1e-8, atol=1e-9)
    assert np.all(r["coeffs"][~obs] == 0) and np.all(r["status"][~obs] & 1)
    assert r["count"] == len(w)


def test_per_view_form_same_minimiser(oracle_lib):
    """Eq. 12: the per-view weighted averages C_hat_j with weights V_j give the
    same minimiser as the per-pixel sum of eq. 10."""
    sc = tiny.random_scene(31, n=24, n_cams=7, res=20, sh_deg=3, C=2, aniso=True, log_scale=-2.3)
    y = np.random.default_rng(6).uniform(0, 1, (sc.n_pixels, 2)).astype(np.float32)
    r = oracle.colorize(sc, y)
    idx, w = oracle.contributions(sc)
    lamx = _expanded_lambda(sc.lam, 3)
    n_ok = 0
    for g in range(sc.N):
        rows, rhs, wg = [], [], 0.0
        for j in range(len(sc.cams)):
            sel = (idx[:, 2] == g) & (idx[:, 0] == j)
            V = w[sel].sum()
            if V == 0:
                continue
            Chat = (w[sel][:, None] * y[idx[sel, 1]].astype(np.float64)).sum(0) / V
            rows.append(math.sqrt(V) * _phi(sc, g, j))
            rhs.append(math.sqrt(V) * Chat)
            wg += V
        if not rows:
            continue
        for m in range(16):
            e = np.zeros(16)
            e[m] = math.sqrt(wg * lamx[m])
            rows.append(e)
            rhs.append(np.zeros(2))
        ref = np.linalg.lstsq(np.asarray(rows), np.asarray(rhs), rcond=None)[0]
        np.testing.assert_allclose(r["coeffs"][g], ref, rtol=1e-8, atol=1e-9)
        n_ok += 1
    assert n_ok >= 10


def test_dc_closed_form(oracle_lib):
    """L = 0: c = Y1 sum w y / (w (Y1^2 + lambda)); with lambda -> 0 this is the
    visibility-weighted colour average of eq. 7 divided by Y1."""
    sc = tiny.random_scene(40, n=50, n_cams=5, res=24, sh_deg=0, C=3)
    y = np.random.default_rng(7).uniform(0, 1, (sc.n_pixels, 3)).astype(np.float32)
    r = oracle.colorize(sc, y)
    idx, w = oracle.contributions(sc)
    Y1 = 1 / math.sqrt(4 * math.pi)
    lam = float(sc.lam[0])
    for g in range(sc.N):
        sel = idx[:, 2] == g
        if not sel.any():
            continue
        wg = w[sel].sum()
        avg = (w[sel][:, None] * y[idx[sel, 1]].astype(np.float64)).sum(0) / wg
        np.testing.assert_allclose(r["coeffs"][g, 0], Y1 * avg / (Y1 ** 2 + lam), rtol=1e-11)


def test_linear_in_targets(oracle_lib):
    """Light fields are linear (Sec. 4.1 combined lighting): colorize(a y1 + b y2)
    = a colorize(y1) + b colorize(y2).  Targets on a 2^-8 grid keep a y1 + b y2
    exact in float32, so the identity holds to double rounding."""
    sc = tiny.random_scene(41, n=40, n_cams=5, res=20, sh_deg=3, C=3, aniso=True)
    rng = np.random.default_rng(8)
    y1 = (rng.integers(0, 256, (sc.n_pixels, 3)) / 256.0).astype(np.float32)
    y2 = (rng.integers(-256, 256, (sc.n_pixels, 3)) / 256.0).astype(np.float32)
    a, b = 0.75, -1.5
    y3 = (a * y1.astype(np.float64) + b * y2.astype(np.float64))
    assert np.all(y3.astype(np.float32).astype(np.float64) == y3)
    c1 = oracle.colorize(sc, y1)["coeffs"]
    c2 = oracle.colorize(sc, y2)["coeffs"]
    c3 = oracle.colorize(sc, y3.astype(np.float32))["coeffs"]
    np.testing.assert_allclose(c3, a * c1 + b * c2, rtol=0, atol=1e-12 * np.abs(c3).max())


@pytest.mark.parametrize("sh_deg", [0, 3])
def test_constant_target_gives_dc_only(oracle_lib, sh_deg):
    """A constant target y fits exactly with c = (y / Y1) e_1 when lambda_1 = 0
    (phi_1 = Y1 everywhere); higher bands stay at zero."""
    lam = [0.0] + [1e-3] * sh_deg if sh_deg > 0 else [0.0]
    sc = tiny.random_scene(42, n=40, n_cams=6, res=20, sh_deg=sh_deg, C=2, aniso=True, lam=lam)
    yv = np.array([0.25, 0.8], np.float32)
    y = np.tile(yv, (sc.n_pixels, 1))
    r = oracle.colorize(sc, y)
    obs = (r["status"] & 1) == 0
    Y1 = 1 / math.sqrt(4 * math.pi)
    np.testing.assert_allclose(r["coeffs"][obs, 0, :], np.tile(yv.astype(np.float64) / Y1, (obs.sum(), 1)), rtol=1e-10)
    if sh_deg > 0:
        assert np.abs(r["coeffs"][obs, 1:, :]).max() < 1e-10


def test_exact_fit_on_disjoint_footprints(oracle_lib):
    """Well separated splats seen from many directions, targets equal to the
    view-dependent colour phi_gj^T C_true on each splat's own pixels: with
    negligible regularisation the solve recovers C_true (eq. 13)."""
    rng = np.random.default_rng(9)
    means = np.array([[0.6, 0, 0], [-0.6, 0, 0], [0, 0.6, 0.2], [0, -0.5, -0.3]], np.float32)
    n = 4
    cams = tiny.sphere_cams(40, radius=3.0, res=48)
    sc = tiny.scene(means, np.full((n, 3), 0.04), tiny.identity_quats(n), np.full(n, 0.6), cams,
                    sh_deg=3, C=2, lam=[1e-12])
    idx, w = oracle.contributions(sc)
    # keep only the views in which no pixel has two contributors
    rows, counts = np.unique(idx[:, 1], return_counts=True)
    shared = set(idx[np.isin(idx[:, 1], rows[counts > 1]), 0].tolist())
    keep = [c for j, c in enumerate(cams) if j not in shared]
    assert len(keep) >= 24
    sc = tiny.scene(means, np.full((n, 3), 0.04), tiny.identity_quats(n), np.full(n, 0.6), keep,
                    sh_deg=3, C=2, lam=[1e-12])
    idx, w = oracle.contributions(sc)
    _, counts = np.unique(idx[:, 1], return_counts=True)
    assert counts.max() == 1
    Ct = rng.normal(0, 1, (n, 16, 2))
    y = np.zeros((sc.n_pixels, 2), np.float64)
    for (j, row, g) in idx:
        y[row] = _phi(sc, g, j) @ Ct[g]
    r = oracle.colorize(sc, y.astype(np.float32))
    # float32 targets limit the recovery; the system is well conditioned
    np.testing.assert_allclose(r["coeffs"], Ct, atol=2e-4)


def test_permutation_invariance(oracle_lib):
    sc = tiny.random_scene(43, n=50, n_cams=5, res=20, sh_deg=2, C=2, aniso=True)
    y = np.random.default_rng(10).uniform(0, 1, (sc.n_pixels, 2)).astype(np.float32)
    r = oracle.colorize(sc, y)
    perm = np.random.default_rng(11).permutation(sc.N)
    sc2 = tiny.scene(sc.means[perm], sc.scales[perm], sc.quats[perm], sc.opacities[perm], sc.cams,
                     sh_deg=2, C=2, lam=sc.lam)
    r2 = oracle.colorize(sc2, y)
    np.testing.assert_allclose(r2["coeffs"], r["coeffs"][perm], rtol=1e-10, atol=1e-12)
    # reversing the camera order (targets move with their cameras)
    offs = sc.pixel_offsets()
    yr = np.concatenate([y[offs[j]:offs[j + 1]] for j in reversed(range(len(sc.cams)))])
    sc3 = tiny.scene(sc.means, sc.scales, sc.quats, sc.opacities, list(reversed(sc.cams)),
                     sh_deg=2, C=2, lam=sc.lam)
    r3 = oracle.colorize(sc3, yr)
    np.testing.assert_allclose(r3["coeffs"], r["coeffs"], rtol=1e-10, atol=1e-12)


def test_unobserved_and_culled(oracle_lib):
    cam = tiny.axis_camera(16, 16, z=-4.0)
    sc = tiny.scene([[0, 0, 0], [0, 0, -6.0], [5.0, 0, 0]], np.full((3, 3), 0.05),
                    tiny.identity_quats(3), [0.5, 0.5, 0.5], [cam], sh_deg=1, C=1, lam=[1e-4, 1e-3])
    y = np.ones((sc.n_pixels, 1), np.float32)
    r = oracle.colorize(sc, y)
    assert list(r["status"]) == [0, 1, 1]
    assert np.all(r["coeffs"][1:] == 0) and r["w"][1] == 0


def test_solver_matches_numpy(oracle_lib):
    rng = np.random.default_rng(12)
    for n in [1, 4, 9, 16]:
        M = rng.standard_normal((n, n))
        A = M @ M.T + n * np.eye(n)
        B = rng.standard_normal((n, 5))
        np.testing.assert_allclose(oracle.solve(A, B), np.linalg.solve(A, B), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(oracle.cond(A), np.linalg.cond(A), rtol=1e-9)


def test_regularised_gradient_vanishes(oracle_lib):
    """Eq. 15: at the solution the gradient of
    sum_j V_j ((C_hat_j - phi^T c)^2 + sum_m lambda_m c_m^2) is zero."""
    sc = tiny.random_scene(44, n=30, n_cams=6, res=20, sh_deg=3, C=1, aniso=True)
    y = np.random.default_rng(13).uniform(0, 1, (sc.n_pixels, 1)).astype(np.float32)
    r = oracle.colorize(sc, y)
    idx, w = oracle.contributions(sc)
    lamx = _expanded_lambda(sc.lam, 3)
    for g in np.nonzero((r["status"] & 1) == 0)[0][:10]:
        c = r["coeffs"][g, :, 0]
        grad = np.zeros(16)
        sel = idx[:, 2] == g
        for (j, row, _), ww in zip(idx[sel], w[sel]):
            ph = _phi(sc, g, j)
            grad += -2 * ww * (float(y[row, 0]) - ph @ c) * ph + 2 * ww * lamx * c
        assert np.abs(grad).max() < 1e-10 * max(1.0, w[sel].sum())
