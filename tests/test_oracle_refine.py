"""Pins of the oracle's iterative refinement (Algorithm 1, steps 8-10).

With w_gp the blend weights and phi_g the SH values of a fixed geometry, the
refinement's fixed point  sum_p w_gp phi_g (y_p - img_p)^T = w_g Lambda c_g,
img_p = sum_h w_hp phi_h^T c_h,  is the normal equation of the coupled
regularised least-squares problem
    min_c  sum_p |y_p - sum_g w_gp phi_g^T c_g|^2 + sum_g w_g c_g^T Lambda c_g,
i.e.  M c = b  with  M = X^T X + R, b = X^T y  (X: rows w_gp phi_g^T).  One
refinement step is the preconditioned step
    c <- c + D^{-1} (b - M c),  D_g = sum_p w_gp phi_g phi_g^T + w_g Lambda,
D_g being the per-Gaussian regularised normal matrix of eq. 14 (linear in the
weights, where M's diagonal blocks are quadratic), and the first pass is
c = D^{-1} b.  The dense system is built here from the oracle's list of
accepted contributions and its SH basis and solved with numpy, independently
of the oracle's per-Gaussian accumulate, render and solve."""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import tiny


def dense_system(sc, lam_full):
    """X [rows, N*nb] (rows: pixels with contributions), regularisation R
    (diagonal), the pixel rows, the visibilities w_g and the blocks D_g."""
    idx, w = oracle.contributions(sc)
    nb, N = sc.n_b, sc.N
    phis = []
    for cam in sc.cams:
        R = np.asarray(cam.R, np.float64)
        centre = -R.T @ np.asarray(cam.t, np.float64)
        phis.append(oracle.sh_basis(sc.sh_deg, sc.means.astype(np.float64) - centre))
    rows = np.unique(idx[:, 1])
    rmap = {r: k for k, r in enumerate(rows)}
    X = np.zeros((rows.size, N * nb))
    wg = np.zeros(N)
    D = np.zeros((N, nb, nb))
    for (j, r, g), ww in zip(idx, w):
        X[rmap[r], g * nb:(g + 1) * nb] += ww * phis[j][g]
        wg[g] += ww
        D[g] += ww * np.outer(phis[j][g], phis[j][g])
    Rdiag = np.repeat(wg, nb) * np.tile(lam_full, N)
    D += wg[:, None, None] * np.diag(lam_full)[None]
    return X, Rdiag, rows, wg, D


def _scene(seed=4):
    return tiny.random_scene(seed, n=40, n_cams=6, res=32, sh_deg=1, C=2, aniso=True,
                             log_scale=-2.4, lam=[1e-3, 1e-2])


def test_one_step_is_the_preconditioned_step():
    sc = _scene()
    y = oracle.make_targets(sc)
    lam_full = oracle.expand_lambda(sc.lam, sc.sh_deg)
    X, Rd, rows, wg, D = dense_system(sc, lam_full)
    nb, N, C = sc.n_b, sc.N, sc.C
    M = X.T @ X + np.diag(Rd)
    b = X.T @ y[rows].astype(np.float64)
    first = oracle.colorize(sc, y)
    c0 = first["coeffs"].reshape(N * nb, C)
    c1 = oracle.refine_step(sc, y, first["coeffs"], first).reshape(N * nb, C)
    expect = c0.copy()
    for g in np.flatnonzero(wg > 0):
        s = slice(g * nb, (g + 1) * nb)
        expect[s] = c0[s] + np.linalg.solve(D[g], b[s] - M[s] @ c0)
    assert np.allclose(c1, expect, rtol=1e-9, atol=1e-11 * np.abs(expect).max())
    # and the first pass is the same step from c = 0
    c00 = np.zeros_like(c0)
    for g in np.flatnonzero(wg > 0):
        s = slice(g * nb, (g + 1) * nb)
        c00[s] = np.linalg.solve(D[g], b[s])
    assert np.allclose(c0, c00, rtol=1e-9, atol=1e-11 * np.abs(c00).max())
    # a step is not block Jacobi: M's diagonal blocks weigh phi phi^T by w^2
    g = int(np.flatnonzero(wg > 0)[0])
    s = slice(g * nb, (g + 1) * nb)
    assert not np.allclose(D[g], M[s, s], rtol=1e-3)


def test_global_solution_is_the_fixed_point():
    sc = _scene(3)
    y = oracle.make_targets(sc)
    lam_full = oracle.expand_lambda(sc.lam, sc.sh_deg)
    X, Rd, rows, wg, D = dense_system(sc, lam_full)
    nb, N, C = sc.n_b, sc.N, sc.C
    obs = np.repeat(wg > 0, nb)
    Xa = np.vstack([X[:, obs], np.diag(np.sqrt(Rd[obs]))])
    Ya = np.vstack([y[rows].astype(np.float64), np.zeros((int(obs.sum()), C))])
    sol, *_ = np.linalg.lstsq(Xa, Ya, rcond=None)
    cstar = np.zeros((N * nb, C))
    cstar[obs] = sol
    cstar = cstar.reshape(N, nb, C)
    first = oracle.colorize(sc, y)
    step = oracle.refine_step(sc, y, cstar, first)
    assert np.linalg.norm(step - cstar) <= 1e-9 * np.linalg.norm(cstar)
    # the iterates approach it, the error shrinking every step
    r = oracle.refine(sc, y, 8, return_all=True)
    errs = [np.linalg.norm(c - cstar) for c in r["history"]]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.6 * errs[0]


def test_disjoint_footprints_l0_closed_form():
    """Gaussians that never share a pixel, L = 0: per Gaussian the system is
    scalar.  With W1 = sum_p w_p, W2 = sum_p w_p^2, Wy = sum_p w_p y_p and
    Y0 = 1/sqrt(4 pi): the first pass is c0 = Y0 Wy / (W1 (Y0^2 + lam)), one
    step gives c1 = c0 + (Y0 Wy - Y0^2 W2 c0 - lam W1 c0) / (W1 (Y0^2 + lam)),
    and the fixed point is c* = Y0 Wy / (Y0^2 W2 + lam W1) (the alpha dimming
    of the render compensated, which the first pass does not do)."""
    cams = [tiny.axis_camera(48, 48, z=-4.0)]
    means = [[-0.6, -0.6, 0.0], [0.6, 0.6, 0.0], [-0.6, 0.6, 0.0], [0.6, -0.6, 0.0]]
    lam = 1e-3
    sc = tiny.scene(means, np.full((4, 3), 0.05), tiny.identity_quats(4), [0.6, 0.8, 0.5, 0.9],
                    cams, sh_deg=0, C=2, lam=[lam])
    rng = np.random.default_rng(2)
    y = rng.uniform(0, 1, (sc.n_pixels, 2)).astype(np.float32)
    idx, w = oracle.contributions(sc)
    assert len(np.unique(idx[:, 1])) == len(idx)  # no pixel holds two Gaussians
    Y0 = 1.0 / np.sqrt(4 * np.pi)
    W1 = np.bincount(idx[:, 2], w, minlength=4)
    W2 = np.bincount(idx[:, 2], w * w, minlength=4)
    Wy = np.stack([np.bincount(idx[:, 2], w * y[idx[:, 1], k].astype(np.float64), minlength=4)
                   for k in range(2)], axis=1)
    den = (W1 * (Y0 ** 2 + lam))[:, None]
    c0 = Y0 * Wy / den
    c1 = c0 + (Y0 * Wy - Y0 ** 2 * W2[:, None] * c0 - lam * W1[:, None] * c0) / den
    cstar = Y0 * Wy / (Y0 ** 2 * W2 + lam * W1)[:, None]
    first = oracle.colorize(sc, y)
    assert np.allclose(first["coeffs"][:, 0, :], c0, rtol=1e-12)
    step = oracle.refine_step(sc, y, first["coeffs"], first)
    assert np.allclose(step[:, 0, :], c1, rtol=1e-12)
    fix = oracle.refine_step(sc, y, cstar[:, None, :], first)
    assert np.allclose(fix[:, 0, :], cstar, rtol=1e-12)
    assert np.abs(c1 - c0).max() > 1e-3  # refinement does change the coefficients


def test_refinement_recovers_exact_fit_with_overlap():
    """Targets rendered from known coefficients (no noise), tiny Lambda,
    overlapping transparent Gaussians: the first pass is biased by colour
    mixing, and the known coefficients are (up to the tiny Lambda) the
    refinement's fixed point."""
    sc = _scene(5)
    sc.lam = np.asarray([1e-9, 1e-9], np.float32)
    sc.noise_std = 0.0
    y = oracle.render(sc, sc.gt[0])  # FP64 targets
    first = oracle.colorize(sc, y)
    obs = (first["status"] & 1) == 0
    ct = sc.gt[0]
    e_first = np.linalg.norm((first["coeffs"] - ct)[obs]) / np.linalg.norm(ct[obs])
    step = oracle.refine_step(sc, y, ct, first)
    e_fix = np.linalg.norm((step - ct)[obs]) / np.linalg.norm(ct[obs])
    assert e_first > 1e-2, e_first
    assert e_fix < 1e-6, e_fix
