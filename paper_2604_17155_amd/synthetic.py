"""Seeded synthetic scenes, cameras and ground-truth coefficients.

This module only draws inputs: Gaussian geometry, opacities, pinhole
cameras, ground-truth coefficient sets, labels and noise.  It holds none of
the colorization method's arithmetic (no projection, blending, accumulation,
solve or rendering); the targets a workload needs are produced by rendering
the ground-truth coefficients with whichever renderer the caller trusts and
then adding the noise drawn here.

The paper measures on captured photo sets, DINOv2 feature maps and SAM2
masks (relighting, feature enrichment and segmentation experiments, Sec. 4).
None of those are available, so these recipes stand in for them with the
shapes, sizes and value distributions of five workloads:

* ``plain``        2,000 isotropic Gaussians, 8 cameras 64x64, L=0, C=3
* ``relight``      100k anisotropic blob-clustered Gaussians, 50 cameras
                   512x512 on a hemisphere, L=3, C=3, FP32
* ``features``     500k Gaussians, 100 cameras 960x540, L=0, C=64, BF16
* ``diff``         300k Gaussians, 100 cameras 800x800, L=3, C=3, two
                   independent target sets
* ``segment``      32 scenes of 5k-400k Gaussians, 20-200 cameras each at
                   640x480..1280x720, L=0, C=16 one-hot labels, BF16

Random draws use ``numpy.random.Generator(PCG64(seed))`` with a fixed draw
order: means, scales, quaternions, opacities, ground-truth coefficients,
labels, noise.

Camera convention (shared by every consumer): world-to-camera
``x_cam = R x + t`` with ``R`` row-major, OpenCV axes (x right, y down,
z forward), world +z up; pinhole intrinsics ``fx = fy = (W/2)/tan(fov_x/2)``,
``cx = W/2``, ``cy = H/2``; the centre of pixel (x, y) is (x+0.5, y+0.5).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 20260417

# Normalisation of the constant real spherical harmonic, 1/sqrt(4 pi): only
# used to turn a ground-truth colour into its DC coefficient.
Y00 = 0.28209479177387814


@dataclasses.dataclass
class Camera:
    R: np.ndarray          # (3, 3) float32, world -> camera rotation
    t: np.ndarray          # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


@dataclasses.dataclass
class Scene:
    means: np.ndarray      # (N, 3) float32
    scales: np.ndarray     # (N, 3) float32, linear standard deviations
    quats: np.ndarray      # (N, 4) float32, (w, x, y, z), not necessarily unit
    opacities: np.ndarray  # (N,) float32 in (0, 1)
    cams: List[Camera]
    sh_deg: int
    C: int
    lam: np.ndarray        # (n_lambda,) float32
    gt: List[np.ndarray]   # ground-truth coefficient sets, each (N, (L+1)^2, C) float64
    noise_std: float
    target_dtype: str      # "f32" or "bf16"
    seed: int
    labels: Optional[np.ndarray] = None

    @property
    def N(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_b(self) -> int:
        return (self.sh_deg + 1) ** 2

    def pixel_offsets(self) -> np.ndarray:
        off = [0]
        for c in self.cams:
            off.append(off[-1] + c.width * c.height)
        return np.asarray(off, dtype=np.int64)

    @property
    def n_pixels(self) -> int:
        return int(sum(c.width * c.height for c in self.cams))


def look_at(position, width: int, height: int, fov_x_deg: float = 60.0,
            target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> Camera:
    """Pinhole camera at ``position`` looking at ``target`` (OpenCV axes)."""
    p = np.asarray(position, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - p
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f]).astype(np.float32)
    t = (-(R.astype(np.float64) @ p)).astype(np.float32)
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R=R, t=t, fx=float(np.float32(fx)), fy=float(np.float32(fx)),
                  cx=width / 2.0, cy=height / 2.0, width=int(width), height=int(height))


def circle_cams(n: int, radius: float, width: int, height: int, fov: float = 60.0) -> List[Camera]:
    out = []
    for k in range(n):
        a = 2.0 * math.pi * k / n
        out.append(look_at((radius * math.cos(a), radius * math.sin(a), 0.0), width, height, fov))
    return out


def hemisphere_cams(n: int, radius: float, width: int, height: int, fov: float = 60.0) -> List[Camera]:
    """Fibonacci directions on the upper hemisphere: z_k = 1-(k+1/2)/n, azimuth k*137.5 deg."""
    out = []
    for k in range(n):
        z = 1.0 - (k + 0.5) / n
        s = math.sqrt(max(0.0, 1.0 - z * z))
        a = math.radians(137.5) * k
        out.append(look_at((radius * s * math.cos(a), radius * s * math.sin(a), radius * z),
                           width, height, fov))
    return out


def paper_lambda(sh_deg: int) -> np.ndarray:
    """Per-band regularisation weights reported in the implementation details (Sec. 4)."""
    return np.asarray([1e-5, 1e-4, 1e-3, 1e-2][: sh_deg + 1], dtype=np.float32)


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _gt_sh(rng, n, sh_deg, C, hi_std=0.1):
    nb = (sh_deg + 1) ** 2
    gt = np.zeros((n, nb, C), dtype=np.float64)
    gt[:, 0, :] = rng.uniform(0.0, 1.0, size=(n, C)) / Y00
    if nb > 1:
        gt[:, 1:, :] = rng.normal(0.0, hi_std, size=(n, nb - 1, C))
    return gt


def isotropic_geometry(rng, n):
    means = rng.uniform(-1.0, 1.0, size=(n, 3)).astype(np.float32)
    ls = rng.normal(-3.5, 0.3, size=(n, 1))
    scales = np.exp(np.repeat(ls, 3, axis=1)).astype(np.float32)
    quats = np.zeros((n, 4), dtype=np.float32)
    quats[:, 0] = 1.0
    opac = rng.uniform(0.1, 0.9, size=n).astype(np.float32)
    return means, scales, quats, opac


def blob_geometry(rng, n, n_blobs=20):
    centres = rng.uniform(-0.7, 0.7, size=(n_blobs, 3))
    pick = rng.integers(0, n_blobs, size=n)
    means = (centres[pick] + rng.normal(0.0, 0.2, size=(n, 3))).astype(np.float32)
    scales = np.exp(rng.normal(-4.0, 0.5, size=(n, 3))).astype(np.float32)
    quats = _unit_quats(rng, n)
    opac = rng.beta(2.0, 2.0, size=n).astype(np.float32)
    opac = np.clip(opac, 1e-4, 1.0 - 1e-4).astype(np.float32)
    return means, scales, quats, opac


def make_plain(seed_offset: int = 1, n: int = 2000, n_cams: int = 8, res: int = 64) -> Scene:
    seed = SEED_BASE + seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    means, scales, quats, opac = isotropic_geometry(rng, n)
    gt = _gt_sh(rng, n, 0, 3)
    return Scene(means, scales, quats, opac, circle_cams(n_cams, 3.0, res, res), 0, 3,
                 np.asarray([1e-4], np.float32), [gt], 0.01, "f32", seed)


def make_relight(seed_offset: int = 2, n: int = 100_000, n_cams: int = 50, res: int = 512,
                 sh_deg: int = 3, lam: Optional[np.ndarray] = None) -> Scene:
    seed = SEED_BASE + seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    means, scales, quats, opac = blob_geometry(rng, n)
    gt = _gt_sh(rng, n, sh_deg, 3)
    return Scene(means, scales, quats, opac, hemisphere_cams(n_cams, 3.0, res, res), sh_deg, 3,
                 paper_lambda(sh_deg) if lam is None else np.asarray(lam, np.float32),
                 [gt], 0.01, "f32", seed)


def make_features(seed_offset: int = 3, n: int = 500_000, n_cams: int = 100,
                  width: int = 960, height: int = 540, C: int = 64) -> Scene:
    seed = SEED_BASE + seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    means, scales, quats, opac = isotropic_geometry(rng, n)
    gt = np.zeros((n, 1, C), dtype=np.float64)
    gt[:, 0, :] = rng.standard_normal((n, C)) / Y00
    return Scene(means, scales, quats, opac, hemisphere_cams(n_cams, 3.0, width, height), 0, C,
                 np.asarray([1e-4], np.float32), [gt], 0.0, "bf16", seed)


def make_diff(seed_offset: int = 4, n: int = 300_000, n_cams: int = 100, res: int = 800) -> Scene:
    seed = SEED_BASE + seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    means, scales, quats, opac = blob_geometry(rng, n)
    gt_a = _gt_sh(rng, n, 3, 3)
    gt_b = _gt_sh(rng, n, 3, 3)
    return Scene(means, scales, quats, opac, hemisphere_cams(n_cams, 3.0, res, res), 3, 3,
                 paper_lambda(3), [gt_a, gt_b], 0.01, "f32", seed)


SEGMENT_RESOLUTIONS = [(640, 480), (800, 600), (960, 540), (1280, 720)]


def make_segment_scene(scene_idx: int, seed_offset: int = 5, n_override: Optional[int] = None,
                       cams_override: Optional[int] = None, C: int = 16) -> Scene:
    seed = SEED_BASE + seed_offset + 100 * scene_idx
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(round(math.exp(rng.uniform(math.log(5e3), math.log(4e5)))))
    n_cams = int(rng.integers(20, 201))
    w, h = SEGMENT_RESOLUTIONS[int(rng.integers(0, len(SEGMENT_RESOLUTIONS)))]
    if n_override is not None:
        n = n_override
    if cams_override is not None:
        n_cams = cams_override
    means, scales, quats, opac = isotropic_geometry(rng, n)
    seeds = rng.uniform(-1.0, 1.0, size=(C, 3))
    d2 = ((means[:, None, :].astype(np.float64) - seeds[None]) ** 2).sum(-1)
    labels = np.argmin(d2, axis=1)  # lowest index wins ties
    gt = np.zeros((n, 1, C), dtype=np.float64)
    gt[np.arange(n), 0, labels] = 1.0 / Y00
    return Scene(means, scales, quats, opac, hemisphere_cams(n_cams, 3.0, w, h), 0, C,
                 np.asarray([1e-4], np.float32), [gt], 0.0, "bf16", seed, labels=labels)


def target_noise(scene: Scene, which: int = 0) -> np.ndarray:
    """Additive N(0, noise_std^2) noise for target set ``which`` (drawn last)."""
    rng = np.random.Generator(np.random.PCG64(scene.seed * 7 + 1000 + which))
    if scene.noise_std == 0.0:
        return np.zeros((scene.n_pixels, scene.C), dtype=np.float32)
    return rng.normal(0.0, scene.noise_std, size=(scene.n_pixels, scene.C)).astype(np.float32)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16) with round-to-nearest-even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(x)
    if nan.any():
        r[nan] = 0x7FC0
    return r


def bf16_to_f32(b: np.ndarray) -> np.ndarray:
    """Exact decode of bfloat16 bit patterns to float32."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def cams_to_array(cams: List[Camera]) -> np.ndarray:
    """Pack cameras as rows of 16 float32 (R[9], t[3], fx, fy, cx, cy) plus sizes."""
    a = np.zeros((len(cams), 16), dtype=np.float32)
    for i, c in enumerate(cams):
        a[i, 0:9] = c.R.reshape(-1)
        a[i, 9:12] = c.t
        a[i, 12:16] = (c.fx, c.fy, c.cx, c.cy)
    return a
