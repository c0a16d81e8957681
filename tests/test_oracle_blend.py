"""Pins of the oracle's front-to-back blend (eq. 2) and of the identities the
paper derives from it (eq. 4 visibility, eq. 9 SH values).

Hand-computed cases use closed-form footprints of isotropic Gaussians on the
optical axis, where the projected covariance is (f*sigma/z)^2 + dilation.
"""
import math

import numpy as np

import oracle
from tests import tiny

AMIN = float(np.float32(1 / 255))
AMAX = float(np.float32(0.99))
TMIN = float(np.float32(1e-4))
DIL = float(np.float32(0.3))


def _pix_weights(sc, cam_idx=0):
    idx, w = oracle.contributions(sc)
    cam = sc.cams[cam_idx]
    out = {}
    for (j, row, g), ww in zip(idx, w):
        if j != cam_idx:
            continue
        out.setdefault((int(row % cam.width), int(row // cam.width)), []).append((int(g), ww))
    return out


def _axis_q(cam, sigma, z, x, y):
    sigma = float(np.float32(sigma))
    s2 = (cam.fx * sigma / z) ** 2 + DIL
    dx, dy = x + 0.5 - cam.cx, y + 0.5 - cam.cy
    return (dx * dx + dy * dy) / s2


def test_single_gaussian_weights_are_alpha(oracle_lib):
    cam = tiny.axis_camera(20, 20, z=-4.0)
    sig, o = 0.04, 0.7
    sc = tiny.scene([[0, 0, 0]], [[sig] * 3], tiny.identity_quats(1), [o], [cam])
    got = _pix_weights(sc)
    expect = {}
    for y in range(20):
        for x in range(20):
            q = _axis_q(cam, sig, 4.0, x, y)
            a = min(AMAX, float(np.float32(o)) * math.exp(-q / 2))
            if q <= 9 and a >= AMIN:
                expect[(x, y)] = a
    assert set(got) == set(expect)
    for k, a in expect.items():
        assert got[k][0][0] == 0
        assert abs(got[k][0][1] - a) < 1e-14


def test_three_stacked_gaussians_front_to_back(oracle_lib):
    """w1 = a1, w2 = a2 (1-a1), w3 = a3 (1-a1)(1-a2), regardless of storage order."""
    cam = tiny.axis_camera(16, 16, z=-4.0)
    zs = [0.5, -0.5, 0.0]       # depths 4.5, 3.5, 4.0 -> front-to-back order 1, 2, 0
    sig = [0.05, 0.03, 0.04]
    op = [0.6, 0.45, 0.8]
    sc = tiny.scene([[0, 0, z] for z in zs], [[s] * 3 for s in sig], tiny.identity_quats(3), op, [cam])
    got = _pix_weights(sc)
    order = [1, 2, 0]
    n_checked = 0
    for (x, y), lst in got.items():
        T = 1.0
        exp_list = []
        for g in order:
            q = _axis_q(cam, sig[g], 4.0 + float(np.float32(zs[g])), x, y)
            a = min(AMAX, float(np.float32(op[g])) * math.exp(-q / 2))
            if q > 9 or a < AMIN:
                continue
            assert T * (1 - a) >= TMIN
            exp_list.append((g, a * T))
            T *= 1 - a
        assert [g for g, _ in lst] == [g for g, _ in exp_list]
        np.testing.assert_allclose([w for _, w in lst], [w for _, w in exp_list], rtol=1e-13)
        n_checked += len(lst)
    assert n_checked > 20


def test_early_stop_at_transmittance_floor(oracle_lib):
    """Twenty stacked splats covering the four centre pixels: the
    k-th is accepted while (1-a)^k >= T_min; the first that would cross stops."""
    cam = tiny.axis_camera(16, 16, z=-4.0)
    n = 20
    sig = 0.1
    zs = np.linspace(-0.5, 0.5, n)
    sc = tiny.scene([[0, 0, z] for z in zs], np.full((n, 3), sig), tiny.identity_quats(n),
                    np.full(n, 0.9), [cam])
    got = _pix_weights(sc)
    for (x, y) in [(7, 7), (8, 8), (7, 8), (8, 7)]:
        lst = got[(x, y)]
        T = 1.0
        k = 0
        for g in range(n):
            q = _axis_q(cam, sig, 4.0 + float(np.float32(zs[g])), x, y)
            a = min(AMAX, float(np.float32(0.9)) * math.exp(-q / 2))
            if T * (1 - a) < TMIN:
                break
            assert lst[k][0] == g
            assert abs(lst[k][1] - a * T) < 1e-14
            T *= 1 - a
            k += 1
        assert len(lst) == k and 10 <= k < n
        # telescoping identity: accepted weights sum to 1 - T_end
        assert abs(sum(w for _, w in lst) - (1 - T)) < 1e-13


def test_alpha_floor_skips(oracle_lib):
    cam = tiny.axis_camera(16, 16, z=-4.0)
    sc = tiny.scene([[0, 0, 0], [0, 0, 0.3]], np.full((2, 3), 0.05), tiny.identity_quats(2),
                    [0.003, 0.5], [cam])
    got = _pix_weights(sc)
    assert all(g == 1 for lst in got.values() for g, _ in lst)
    assert len(got) > 0


def test_anisotropic_footprint_uses_full_conic(oracle_lib):
    """A rotated elongated splat: weight at each pixel equals o*exp(-q/2) with
    q from the eigen-decomposition of the projected covariance."""
    cam = tiny.axis_camera(40, 40, z=-4.0)
    ang = math.radians(30.0)
    quat = [math.cos(ang / 2), 0, 0, math.sin(ang / 2)]   # rotation about the optical axis
    s = [0.5, 0.12, 0.2]
    sc = tiny.scene([[0, 0, 0]], [s], [quat], [0.9], [cam])
    got = _pix_weights(sc)
    f = cam.fx / 4.0
    s32 = [float(np.float32(v)) for v in s]
    ev = np.array([(f * s32[0]) ** 2 + DIL, (f * s32[1]) ** 2 + DIL])
    e0 = np.array([math.cos(ang), math.sin(ang)])
    e1 = np.array([-math.sin(ang), math.cos(ang)])
    n = 0
    for y in range(40):
        for x in range(40):
            d = np.array([x + 0.5 - cam.cx, y + 0.5 - cam.cy])
            q = (d @ e0) ** 2 / ev[0] + (d @ e1) ** 2 / ev[1]
            a = min(AMAX, float(np.float32(0.9)) * math.exp(-q / 2))
            # float32 inputs perturb the rotation by ~1e-8 relative
            if q <= 9 * (1 - 1e-6) and a >= AMIN * (1 + 1e-6):
                assert abs(got[(x, y)][0][1] - a) < 1e-6 * a
                n += 1
            elif q > 9 * (1 + 1e-6):
                assert (x, y) not in got
    assert n > 50


def test_visibility_is_scaled_dc_derivative(oracle_lib):
    """Eq. 4: V_{g,p} = sqrt(4 pi) d img_p / d c_g^1.  Render is linear in the
    coefficients, so rendering a unit DC coefficient is an exact derivative."""
    sc = tiny.random_scene(11, n=40, n_cams=3, res=20, sh_deg=0, C=1)
    idx, w = oracle.contributions(sc)
    for g in [0, 5, 17, 33]:
        c = np.zeros((sc.N, 1, 1))
        c[g, 0, 0] = 1.0
        img = oracle.render(sc, c)[:, 0]
        vis = np.zeros(sc.n_pixels)
        sel = idx[:, 2] == g
        vis[idx[sel, 1]] = w[sel]
        np.testing.assert_allclose(img * math.sqrt(4 * math.pi), vis, rtol=1e-13, atol=1e-15)


def test_sh_values_from_derivative_ratio(oracle_lib):
    """Eq. 9: (d sum img / d c_g^m) / V_g^j is the SH basis at the direction
    camera -> Gaussian mean, for every m."""
    sc = tiny.random_scene(12, n=30, n_cams=4, res=20, sh_deg=3, C=1)
    offs = sc.pixel_offsets()
    for g in [1, 9, 22]:
        c1 = np.zeros((sc.N, 16, 1))
        c1[g, 0, 0] = 1.0
        v = oracle.render(sc, c1)[:, 0] * math.sqrt(4 * math.pi)
        for j, cam in enumerate(sc.cams):
            Vj = v[offs[j]:offs[j + 1]].sum()
            if Vj == 0:
                continue
            centre = -cam.R.astype(np.float64).T @ cam.t.astype(np.float64)
            d = sc.means[g].astype(np.float64) - centre
            phi = oracle.sh_basis(3, d[None])[0]
            for m in range(16):
                cm = np.zeros((sc.N, 16, 1))
                cm[g, m, 0] = 1.0
                dm = oracle.render(sc, cm)[offs[j]:offs[j + 1], 0].sum()
                assert abs(dm / Vj - phi[m]) < 1e-12
