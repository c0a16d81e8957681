"""Pins of the oracle's geometry: SH basis, projection, depth key.

Each check compares the oracle with something independent of it: scipy's
complex spherical harmonics, quadrature, Unsoeld's addition theorem, scipy's
quaternion rotations with a numerical Jacobian of the pinhole projection, and
exact rational arithmetic for the single-precision depth key.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
from tests import tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _real_sh_scipy(L, d):
    """Real orthonormal SH from scipy's complex ones (with Condon-Shortley
    phase): m>0 -> sqrt2 (-1)^m Re Y_l^m, m<0 -> sqrt2 (-1)^m Im Y_l^|m|."""
    d = d / np.linalg.norm(d)
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    out = []
    for l in range(L + 1):
        for m in range(-l, l + 1):
            if m == 0:
                v = sph_harm_y(l, 0, theta, phi).real
            elif m > 0:
                v = math.sqrt(2) * (-1) ** m * sph_harm_y(l, m, theta, phi).real
            else:
                v = math.sqrt(2) * (-1) ** m * sph_harm_y(l, -m, theta, phi).imag
            out.append(v)
    return np.asarray(out)


def test_sh_matches_scipy(oracle_lib):
    rng = np.random.default_rng(0)
    dirs = rng.standard_normal((200, 3))
    dirs[0] = [0, 0, 1]
    dirs[1] = [0, 0, -1]
    dirs[2] = [1, 0, 0]
    got = oracle.sh_basis(3, dirs)
    for i, d in enumerate(dirs):
        np.testing.assert_allclose(got[i], _real_sh_scipy(3, d), rtol=0, atol=1e-13)


def test_sh_constant_band_is_paper_value(oracle_lib):
    """The first basis function is the constant 1/sqrt(4 pi) (Sec. 3, visibility)."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        consts = json.load(f)
    y1 = consts["Y1"]["value"]
    got = oracle.sh_basis(3, np.random.default_rng(1).standard_normal((50, 3)))
    np.testing.assert_allclose(got[:, 0], y1, rtol=1e-15)
    assert abs(y1 - 1.0 / math.sqrt(4 * math.pi)) < 1e-15


def test_sh_orthonormal_by_quadrature(oracle_lib):
    # Gauss-Legendre in cos(theta) (exact to degree 2n-1) x uniform azimuth.
    zs, wz = np.polynomial.legendre.leggauss(10)
    nphi = 24
    phis = 2 * np.pi * np.arange(nphi) / nphi
    dirs, wts = [], []
    for z, w in zip(zs, wz):
        s = math.sqrt(1 - z * z)
        for p in phis:
            dirs.append([s * math.cos(p), s * math.sin(p), z])
            wts.append(w * 2 * np.pi / nphi)
    Y = oracle.sh_basis(3, np.asarray(dirs))
    G = (Y * np.asarray(wts)[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_unsold_sum(oracle_lib):
    Y = oracle.sh_basis(3, np.random.default_rng(2).standard_normal((500, 3)))
    for L in range(4):
        nb = (L + 1) ** 2
        np.testing.assert_allclose((Y[:, :nb] ** 2).sum(1), nb / (4 * np.pi), rtol=1e-13)


def test_projection_on_axis_closed_form(oracle_lib):
    cam = tiny.axis_camera(32, 32, z=-4.0)
    sig = 0.05
    sc = tiny.scene([[0, 0, 0]], [[sig] * 3], tiny.identity_quats(1), [0.5], [cam])
    r = oracle.project(sc, 0)[0]
    assert r[0] == 1 and r[1] == 4.0
    f = cam.fx
    s2 = (f * sig / 4.0) ** 2 + np.float32(0.3)
    np.testing.assert_allclose(r[2:4], [16.0, 16.0], atol=1e-12)
    np.testing.assert_allclose(r[7:10], [s2, 0.0, s2], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(r[4:7], [1 / s2, 0.0, 1 / s2], rtol=1e-6, atol=1e-12)


def test_projection_matches_numerical_jacobian(oracle_lib):
    """Sigma_2D - dilation = J Sigma_cam J^T with J the Jacobian of the
    pinhole projection at the mean, Sigma from scipy's quaternion rotation."""
    rng = np.random.default_rng(3)
    cams = tiny.sphere_cams(4, res=64)
    n = 12
    means = rng.uniform(-0.5, 0.5, (n, 3)).astype(np.float32)
    scales = np.exp(rng.normal(-3, 0.5, (n, 3))).astype(np.float32)
    q = rng.standard_normal((n, 4)).astype(np.float32)
    sc = tiny.scene(means, scales, q, np.full(n, 0.5), cams)
    for j, cam in enumerate(cams):
        out = oracle.project(sc, j)
        W = cam.R.astype(np.float64)
        t = cam.t.astype(np.float64)
        for g in range(n):
            qq = q[g].astype(np.float64)
            rot = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
            S = rot @ np.diag(scales[g].astype(np.float64) ** 2) @ rot.T
            pc = W @ means[g].astype(np.float64) + t

            def proj(p):
                return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])

            h = 1e-6
            J = np.stack([(proj(pc + h * e) - proj(pc - h * e)) / (2 * h) for e in np.eye(3)], 1)
            S2 = J @ (W @ S @ W.T) @ J.T
            got = out[g]
            np.testing.assert_allclose(got[2:4], proj(pc), rtol=1e-10)
            dil = float(np.float32(0.3))
            ref = np.array([S2[0, 0] + dil, S2[0, 1], S2[1, 1] + dil])
            np.testing.assert_allclose(got[7:10], ref, rtol=1e-6, atol=1e-9 * abs(ref).max())
            Sm = np.array([[got[7], got[8]], [got[8], got[9]]])
            np.testing.assert_allclose(np.array([[got[4], got[5]], [got[5], got[6]]]),
                                       np.linalg.inv(Sm), rtol=1e-9, atol=1e-12)


def _round_f32(fr: Fraction) -> np.float32:
    """Correctly rounded (nearest, ties to even) float32 of an exact rational."""
    f = np.float32(float(fr))
    best = f
    for cand in (np.nextafter(f, np.float32(-np.inf)), np.nextafter(f, np.float32(np.inf))):
        d_c, d_b = abs(Fraction(float(cand)) - fr), abs(Fraction(float(best)) - fr)
        if d_c < d_b or (d_c == d_b and (cand.view(np.uint32) & 1) == 0):
            best = cand
    return best


def test_depth_key_is_single_precision_fma_chain(oracle_lib):
    rng = np.random.default_rng(4)
    cams = tiny.sphere_cams(3, res=16)
    means = rng.uniform(-1, 1, (40, 3)).astype(np.float32)
    sc = tiny.scene(means, np.full((40, 3), 0.01), tiny.identity_quats(40), np.full(40, 0.5), cams)
    for j, cam in enumerate(cams):
        out = oracle.project(sc, j)
        R, t = cam.R, cam.t
        for g in range(40):
            m = means[g]
            inner = _round_f32(Fraction(float(R[2, 2])) * Fraction(float(m[2])) + Fraction(float(t[2])))
            mid = _round_f32(Fraction(float(R[2, 1])) * Fraction(float(m[1])) + Fraction(float(inner)))
            key = _round_f32(Fraction(float(R[2, 0])) * Fraction(float(m[0])) + Fraction(float(mid)))
            assert np.float32(out[g, 1]) == key


def test_behind_camera_is_culled(oracle_lib):
    cam = tiny.axis_camera(16, 16, z=-4.0)
    sc = tiny.scene([[0, 0, -5.0], [0, 0, 0]], np.full((2, 3), 0.05), tiny.identity_quats(2),
                    [0.5, 0.5], [cam])
    r = oracle.project(sc, 0)
    assert r[0, 0] == 0 and r[1, 0] == 1
