"""Hand-built tiny scenes for the oracle pins and small parity cases."""
import math

import numpy as np

from paper_2604_17155_amd import synthetic as syn


def axis_camera(width=16, height=16, z=-4.0, fov=60.0):
    """Camera on the -z axis looking along +z (x right, y down)."""
    R = np.eye(3, dtype=np.float32)
    t = np.array([0.0, 0.0, -z], np.float32)  # x_cam = x - (0,0,z)
    fx = (width / 2.0) / math.tan(math.radians(fov) / 2.0)
    return syn.Camera(R=R, t=t, fx=float(np.float32(fx)), fy=float(np.float32(fx)),
                      cx=width / 2.0, cy=height / 2.0, width=width, height=height)


def scene(means, scales, quats, opac, cams, sh_deg=0, C=1, lam=(1e-4,), gt=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    scales = np.asarray(scales, np.float32).reshape(n, 3)
    quats = np.asarray(quats, np.float32).reshape(n, 4)
    opac = np.asarray(opac, np.float32).reshape(n)
    nb = (sh_deg + 1) ** 2
    if gt is None:
        gt = np.zeros((n, nb, C))
    return syn.Scene(means, scales, quats, opac, list(cams), sh_deg, C,
                     np.asarray(lam, np.float32), [gt], 0.0, "f32", 0)


def identity_quats(n):
    q = np.zeros((n, 4), np.float32)
    q[:, 0] = 1
    return q


def sphere_cams(n, radius=3.0, res=32, fov=60.0):
    """Cameras on a full sphere (Fibonacci), looking at the origin."""
    out = []
    for k in range(n):
        z = 1.0 - 2.0 * (k + 0.5) / n
        s = math.sqrt(max(0.0, 1 - z * z))
        a = math.radians(137.50776) * k
        up = (0.0, 0.0, 1.0) if abs(z) < 0.95 else (1.0, 0.0, 0.0)
        out.append(syn.look_at((radius * s * math.cos(a), radius * s * math.sin(a), radius * z),
                               res, res, fov, up=up))
    return out


def random_scene(seed, n=60, n_cams=6, res=24, sh_deg=0, C=3, lam=None, opac_range=(0.1, 0.9),
                 log_scale=-2.6, aniso=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-0.6, 0.6, size=(n, 3)).astype(np.float32)
    if aniso:
        scales = np.exp(rng.normal(log_scale, 0.4, size=(n, 3))).astype(np.float32)
        q = rng.standard_normal((n, 4))
        quats = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    else:
        scales = np.repeat(np.exp(rng.normal(log_scale, 0.2, size=(n, 1))), 3, 1).astype(np.float32)
        quats = identity_quats(n)
    opac = rng.uniform(*opac_range, size=n).astype(np.float32)
    cams = syn.hemisphere_cams(n_cams, 3.0, res, res) if n_cams > 0 else []
    nb = (sh_deg + 1) ** 2
    gt = np.zeros((n, nb, C))
    gt[:, 0, :] = rng.uniform(0, 1, size=(n, C)) / syn.Y00
    if nb > 1:
        gt[:, 1:, :] = rng.normal(0, 0.1, size=(n, nb - 1, C))
    if lam is None:
        lam = syn.paper_lambda(sh_deg) if sh_deg > 0 else np.asarray([1e-4], np.float32)
    s = syn.Scene(means, scales, quats, opac, cams, sh_deg, C, np.asarray(lam, np.float32),
                  [gt], 0.01, "f32", seed)
    return s
