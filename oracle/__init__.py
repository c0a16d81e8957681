"""FP64 CPU oracle for Gaussian-splat colorization -- test infrastructure only.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never touches it, and the two share no code: the only common module
is the seeded input generator, which holds none of the method's arithmetic.

The arithmetic lives in ``gsc_oracle.c`` (plain C, double precision, OpenMP
over views).  This module compiles it with gcc, loads it with ctypes and
marshals numpy arrays.  See the C file for what each function computes and
which part of the paper it follows.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

from paper_2604_17155_amd import synthetic as syn

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OcCamera(ct.Structure):
    _fields_ = [("R", ct.c_float * 9), ("t", ct.c_float * 3), ("fx", ct.c_float),
                ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float),
                ("width", ct.c_int32), ("height", ct.c_int32), ("pixel_offset", ct.c_int64)]


class OcOptions(ct.Structure):
    _fields_ = [("alpha_min", ct.c_float), ("alpha_max", ct.c_float), ("t_min", ct.c_float),
                ("sigma_cut", ct.c_float), ("dilation", ct.c_float), ("znear", ct.c_float),
                ("eps_q", ct.c_double), ("eps_a", ct.c_double), ("eps_t", ct.c_double),
                ("eps_p", ct.c_double), ("p_span", ct.c_double), ("eps_cov", ct.c_double)]


# unit roundoff of binary32 (round to nearest)
U32 = 2.0 ** -24


@dataclasses.dataclass
class Options:
    """Blending constants (3DGS conventions) and the event margins.

    Thresholds are single-precision numbers so that both sides compare against
    the identical threshold value.

    The margins model an implementation that evaluates the pixel decisions in
    binary32 from a projection computed in binary64 (see gsc_oracle.c,
    oc_options).  Each is the worst-case count of roundings it covers, in
    units of u = 2^-24 (a rounding moves a value by at most u of it), times
    a safety factor of about 1.5:
      eps_q    6u  q: conic rounded once, a*dx*dx (two), b*dx (one), two fused
                   adds: at most 4u of the sum of the terms' magnitudes (a
                   binary32 emulation without fused adds peaked at 4.3u);
      eps_p  4.5u  pixel offsets (tile centre point - centre_hi) - centre_lo
                   + (pixel - centre point): three roundings per axis of
                   quantities of at most |d| + 7.5 pixels, so at most
                   u (3 |d| + 15), taken as eps_p (|d| + p_span), p_span = 5;
      eps_cov 1e-14  the 3D covariance R diag(s^2) R^T is formed in binary64
                   (its error is then a few units of 2^-53), against the bound
                   s_max sqrt(q) |v| + sum_k s_k^2 ((|R|^T|v|)_k)^2 of
                   gsc_oracle.c.  (A binary32 covariance would need about
                   20u: a binary32 emulation on the reduced relighting scene
                   peaked at 9.3u of that bound.);
      eps_a    4u  alpha beyond q: exp2 within one ulp (2u) and the product
                   with the opacity (u);
      eps_t  1.5u  one fused T (1 - alpha) update (u).
    """
    alpha_min: float = float(np.float32(1.0 / 255.0))
    alpha_max: float = float(np.float32(0.99))
    t_min: float = float(np.float32(1e-4))
    sigma_cut: float = 3.0
    dilation: float = float(np.float32(0.3))
    znear: float = float(np.float32(0.01))
    eps_q: float = 6 * U32
    eps_a: float = 4 * U32
    eps_t: float = 1.5 * U32
    eps_p: float = 4.5 * U32
    p_span: float = 5.0
    eps_cov: float = 1e-14

    def c(self) -> OcOptions:
        return OcOptions(self.alpha_min, self.alpha_max, self.t_min, self.sigma_cut,
                         self.dilation, self.znear, self.eps_q, self.eps_a, self.eps_t,
                         self.eps_p, self.p_span, self.eps_cov)

    def scaled_margins(self, k: float) -> "Options":
        """The same options with every margin multiplied by k."""
        return dataclasses.replace(self, eps_q=self.eps_q * k, eps_a=self.eps_a * k,
                                   eps_t=self.eps_t * k, eps_p=self.eps_p * k,
                                   eps_cov=self.eps_cov * k)


def _f(a):
    return a.ctypes.data_as(ct.c_void_p)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ct.CDLL(_LIB)
    P = ct.c_void_p
    i64, i32 = ct.c_int64, ct.c_int
    lib.oc_sh_basis.argtypes = [i32, P, i64, P]
    lib.oc_colorize.argtypes = [P, P, P, P, i64, P, i32, P, i32, i32, i32, P, i32, P, P, P, P, P,
                                P, P, P, P, P, P, P, P, i32]
    lib.oc_render.argtypes = [P, P, P, P, i64, P, i32, P, i32, i32, P, P, P, P, i32]
    lib.oc_colorize_backward.argtypes = [P, P, P, P, i64, P, i32, P, i32, i32, i32, P, i32, P, P,
                                         P, P, P, i32]
    lib.oc_render_backward.argtypes = [P, P, P, P, i64, P, i32, P, i32, i32, P, P, P, P, i32]
    lib.oc_project.argtypes = [P, P, P, P, i64, P, P, P]
    lib.oc_contributions.argtypes = [P, P, P, P, i64, P, i32, P, P, P, i64]
    lib.oc_contributions.restype = ct.c_int64
    lib.oc_contributions_rows.argtypes = [P, P, P, P, i64, P, i32, P, P, i64, P, P, i64, i32]
    lib.oc_contributions_rows.restype = ct.c_int64
    lib.oc_wanted_rows.argtypes = [P, P, P, P, i64, P, i32, P, P, P, i64]
    lib.oc_wanted_rows.restype = ct.c_int64
    lib.oc_render_rows.argtypes = [P, P, P, P, i64, P, i32, P, i32, i32, P, P, i64, P, i32]
    lib.oc_solve.argtypes = [i32, i32, P, P, P]
    lib.oc_cond.argtypes = [i32, P]
    lib.oc_cond.restype = ct.c_double
    _lib = lib
    return lib


def cameras(cams, offsets=None):
    arr = (OcCamera * max(1, len(cams)))()
    off = 0
    for i, c in enumerate(cams):
        arr[i].R[:] = [float(v) for v in np.asarray(c.R, np.float32).reshape(-1)]
        arr[i].t[:] = [float(v) for v in np.asarray(c.t, np.float32)]
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = c.fx, c.fy, c.cx, c.cy
        arr[i].width, arr[i].height = c.width, c.height
        arr[i].pixel_offset = off if offsets is None else int(offsets[i])
        off += c.width * c.height
    return arr


def _geom(scene):
    m = np.ascontiguousarray(scene.means, np.float32)
    s = np.ascontiguousarray(scene.scales, np.float32)
    q = np.ascontiguousarray(scene.quats, np.float32)
    o = np.ascontiguousarray(scene.opacities, np.float32)
    return m, s, q, o


def _targets(targets):
    t = np.ascontiguousarray(targets)
    if t.dtype == np.uint16:
        return t, 1
    if t.dtype == np.float64:
        return t, 2
    return np.ascontiguousarray(t, np.float32), 0


def _threads(n):
    if n is not None:
        return int(n)
    return int(os.environ.get("GSC_ORACLE_THREADS", "0"))


def colorize(scene, targets, want: Optional[np.ndarray] = None, opts: Optional[Options] = None,
             lam=None, with_kappa: bool = False, threads=None):
    """Oracle colorization (Algorithm 1, steps 1-6).  Returns a dict with
    coeffs [N,nb,C], status, A (regularised), B, w, flip (bound on the
    coefficient change near-threshold decisions could cause), kappa, cnt
    (accepted contributions per Gaussian), ndec (near-threshold decisions on
    each Gaussian's own acceptance), werr (bound on the relative error of
    each Gaussian's per-view weight sums from binary32 weights), count
    (accepted contributions) and events (near-threshold decisions)."""
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    t, td = _targets(targets)
    N, nb, C = scene.N, scene.n_b, scene.C
    lam = np.ascontiguousarray(scene.lam if lam is None else lam, np.float32)
    cams = cameras(scene.cams)
    coeffs = np.zeros((N, nb, C), np.float64)
    status = np.zeros(N, np.uint8)
    A = np.zeros((N, nb, nb), np.float64)
    B = np.zeros((N, nb, C), np.float64)
    w = np.zeros(N, np.float64)
    flip = np.zeros(N, np.float64)
    kappa = np.zeros(N, np.float64) if with_kappa else None
    cnt = np.zeros(N, np.int64)
    ndec = np.zeros(N, np.int64)
    werr = np.zeros(N, np.float64)
    stats = np.zeros(2, np.int64)
    wp = None
    if want is not None:
        wp = np.ascontiguousarray(want, np.uint8)
    oo = opts.c()
    rc = lib.oc_colorize(_f(m), _f(s), _f(q), _f(o), N, ct.cast(cams, ct.c_void_p),
                         len(scene.cams), _f(t), td, C, scene.sh_deg, _f(lam), lam.size,
                         ct.byref(oo), None if wp is None else _f(wp), _f(coeffs), _f(status),
                         _f(A), _f(B), _f(w), _f(flip), None if kappa is None else _f(kappa),
                         _f(cnt), _f(ndec), _f(werr), _f(stats), _threads(threads))
    if rc != 0:
        raise ValueError("oracle colorize rejected its arguments")
    return dict(coeffs=coeffs, status=status, A=A, B=B, w=w, flip=flip, kappa=kappa, cnt=cnt,
                ndec=ndec, werr=werr, count=int(stats[0]), events=int(stats[1]))


def expand_lambda(lam, L: int) -> np.ndarray:
    """Lambda per coefficient (l*l + l + m) from 1, L+1 or (L+1)^2 values."""
    lam = np.asarray(lam, np.float64).reshape(-1)
    nb = (L + 1) ** 2
    if lam.size == 1:
        return np.full(nb, lam[0])
    if lam.size == L + 1:
        return np.concatenate([np.full(2 * l + 1, lam[l]) for l in range(L + 1)])
    return lam.copy()


def refine_step(scene, targets, coeffs, first, opts: Optional[Options] = None, lam=None,
                threads=None):
    """One refinement pass (Algorithm 1, steps 8-10) from coefficients
    `coeffs`: render them, take the residual targets (decoded targets minus
    the render, FP64), accumulate the right-hand side B_g of the residual and
    update c_g <- c_g + (A_g + w_g Lambda)^{-1} (B_g - w_g Lambda c_g) with
    the regularised normal matrix A and visibilities w of the first pass
    (`first`, an oracle colorize of the same scene).  Unobserved Gaussians and
    failed factorisations keep their coefficients."""
    lam = scene.lam if lam is None else lam
    lam_full = expand_lambda(lam, scene.sh_deg)
    y = decode_targets(targets).astype(np.float64)
    c = np.array(coeffs, np.float64, copy=True)
    img = render(scene, c, opts=opts, threads=threads)
    res = colorize(scene, y - img, opts=opts, lam=lam, threads=threads)
    for g in np.flatnonzero((first["status"] & 5) == 0):
        rhs = res["B"][g] - first["w"][g] * lam_full[:, None] * c[g]
        c[g] = c[g] + solve(first["A"][g], rhs)
    return c


def refine(scene, targets, n_steps: int, opts: Optional[Options] = None, lam=None, threads=None,
           return_all: bool = False):
    """Colorization with iterative refinement (Algorithm 1: steps 1-6, then
    n_steps refinement passes, refine_step).  Returns the colorize dict of the
    first pass with coeffs replaced by the refined ones (and, with return_all,
    `history`: the coefficients after every pass, the first one included)."""
    first = colorize(scene, targets, opts=opts, lam=lam, threads=threads)
    c = first["coeffs"]
    history = [c.copy()]
    for _ in range(n_steps):
        c = refine_step(scene, targets, c, first, opts=opts, lam=lam, threads=threads)
        history.append(c.copy())
    out = dict(first)
    out["coeffs"] = c
    if return_all:
        out["history"] = history
    return out


def render(scene, coeffs, opts: Optional[Options] = None, threads=None, with_bound: bool = False):
    """Oracle render (eq. 1-3) of coefficients [N,nb,C] -> images [rows, C] float64.
    with_bound: also return, per pixel, a bound on how far an implementation
    within the event margins may render it away from the result (max over
    channels)."""
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    coeffs = np.ascontiguousarray(coeffs, np.float64)
    C = coeffs.shape[2]
    L = int(round(np.sqrt(coeffs.shape[1]))) - 1
    cams = cameras(scene.cams)
    img = np.zeros((scene.n_pixels, C), np.float64)
    bound = np.zeros(scene.n_pixels, np.float64) if with_bound else None
    stats = np.zeros(2, np.int64)
    oo = opts.c()
    rc = lib.oc_render(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                       len(scene.cams), _f(coeffs), C, L, ct.byref(oo), _f(img),
                       None if bound is None else _f(bound), _f(stats), _threads(threads))
    if rc != 0:
        raise ValueError("oracle render rejected its arguments")
    return (img, bound) if with_bound else img


def colorize_backward(scene, targets, coeffs, grad_coeffs, opts: Optional[Options] = None,
                      lam=None, threads=None):
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    t, td = _targets(targets)
    lam = np.ascontiguousarray(scene.lam if lam is None else lam, np.float32)
    coeffs = np.ascontiguousarray(coeffs, np.float64)
    gc = np.ascontiguousarray(grad_coeffs, np.float64)
    cams = cameras(scene.cams)
    gt = np.zeros((scene.n_pixels, scene.C), np.float64)
    go = np.zeros(scene.N, np.float64)
    oo = opts.c()
    rc = lib.oc_colorize_backward(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                                  len(scene.cams), _f(t), td, scene.C, scene.sh_deg, _f(lam),
                                  lam.size, ct.byref(oo), _f(coeffs), _f(gc), _f(gt), _f(go),
                                  _threads(threads))
    if rc != 0:
        raise ValueError("oracle colorize_backward rejected its arguments")
    return gt, go


def render_backward(scene, coeffs, grad_images, opts: Optional[Options] = None, threads=None):
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    coeffs = np.ascontiguousarray(coeffs, np.float64)
    gi = np.ascontiguousarray(grad_images, np.float64)
    C = coeffs.shape[2]
    L = int(round(np.sqrt(coeffs.shape[1]))) - 1
    cams = cameras(scene.cams)
    gc = np.zeros_like(coeffs)
    go = np.zeros(scene.N, np.float64)
    oo = opts.c()
    rc = lib.oc_render_backward(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                                len(scene.cams), _f(coeffs), C, L, ct.byref(oo), _f(gi), _f(gc),
                                _f(go), _threads(threads))
    if rc != 0:
        raise ValueError("oracle render_backward rejected its arguments")
    return gc, go


def project(scene, cam_index: int, opts: Optional[Options] = None):
    """Per Gaussian [visible, key, u, v, ca, cb, cc, sxx, sxy, syy] for one camera."""
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    cams = cameras(scene.cams)
    out = np.zeros((scene.N, 10), np.float64)
    oo = opts.c()
    lib.oc_project(_f(m), _f(s), _f(q), _f(o), scene.N,
                   ct.byref(cams[cam_index]), ct.byref(oo), _f(out))
    return out


def contributions(scene, opts: Optional[Options] = None, cap: int = 5_000_000):
    """All accepted contributions: (view, target row, g) int64 [n,3] and w [n]."""
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    cams = cameras(scene.cams)
    idx = np.zeros((cap, 3), np.int64)
    w = np.zeros(cap, np.float64)
    oo = opts.c()
    n = lib.oc_contributions(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                             len(scene.cams), ct.byref(oo), _f(idx), _f(w), cap)
    if n > cap:
        raise ValueError("contribution buffer too small")
    return idx[:n].copy(), w[:n].copy()


def contributions_rows(scene, rows: np.ndarray, opts: Optional[Options] = None, threads=None):
    """Accepted contributions at the given target rows only (each pixel's full
    front-to-back walk): (view, row, g) int64 [n,3] and w [n], in view order."""
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    cams = cameras(scene.cams)
    r = np.ascontiguousarray(np.unique(np.asarray(rows, np.int64)))
    cap = max(1024, 64 * r.size)
    while True:
        idx = np.zeros((cap, 3), np.int64)
        w = np.zeros(cap, np.float64)
        oo = opts.c()
        n = lib.oc_contributions_rows(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                                      len(scene.cams), ct.byref(oo), _f(r), r.size, _f(idx), _f(w), cap,
                                      _threads(threads))
        if n <= cap:
            return idx[:n].copy(), w[:n].copy()
        cap = int(n)


def wanted_rows(scene, want: np.ndarray, opts: Optional[Options] = None) -> np.ndarray:
    """Target rows a colorize restricted to the Gaussians with want[g] != 0
    reads (their pixel ranges in every view), ascending."""
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    cams = cameras(scene.cams)
    w = np.ascontiguousarray(want, np.uint8)
    oo = opts.c()
    n = lib.oc_wanted_rows(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                           len(scene.cams), ct.byref(oo), _f(w), None, 0)
    rows = np.zeros(max(1, n), np.int64)
    lib.oc_wanted_rows(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                       len(scene.cams), ct.byref(oo), _f(w), _f(rows), n)
    return np.sort(rows[:n])


def render_rows(scene, coeffs, rows: np.ndarray, opts: Optional[Options] = None, threads=None):
    """Oracle render (eqs. 1-3) of the listed target rows only -> [len(rows), C]."""
    lib = load()
    opts = opts or Options()
    m, s, q, o = _geom(scene)
    coeffs = np.ascontiguousarray(coeffs, np.float64)
    C = coeffs.shape[2]
    L = int(round(np.sqrt(coeffs.shape[1]))) - 1
    rows = np.ascontiguousarray(rows, np.int64)
    out = np.zeros((rows.size, C), np.float64)
    cams = cameras(scene.cams)
    oo = opts.c()
    rc = lib.oc_render_rows(_f(m), _f(s), _f(q), _f(o), scene.N, ct.cast(cams, ct.c_void_p),
                            len(scene.cams), _f(coeffs), C, L, ct.byref(oo), _f(rows), rows.size,
                            _f(out), _threads(threads))
    if rc != 0:
        raise ValueError("oracle render_rows rejected its arguments")
    return out


def sparse_targets(scene, rows: np.ndarray, which: int = 0, opts: Optional[Options] = None,
                   threads=None):
    """Targets of a synthetic workload at the listed rows only (the oracle's
    render of ground-truth set `which` plus the seeded noise, cast to the
    workload's target dtype), returned as (full-size array that holds them at
    those rows and zeros elsewhere, the values at the rows).  The full array
    is allocated lazily, so only the pages of the listed rows use memory."""
    vals = render_rows(scene, scene.gt[which], rows, opts, threads)
    if scene.noise_std:
        vals = vals + syn.target_noise(scene, which)[rows]
    vals = vals.astype(np.float32)
    if scene.target_dtype == "bf16":
        vals = syn.round_bf16(vals)
    full = np.zeros((scene.n_pixels, scene.C), vals.dtype)
    full[rows] = vals
    return full, vals


def sh_basis(L: int, dirs: np.ndarray) -> np.ndarray:
    lib = load()
    d = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    out = np.zeros((d.shape[0], (L + 1) ** 2), np.float64)
    if lib.oc_sh_basis(L, _f(d), d.shape[0], _f(out)) != 0:
        raise ValueError("bad degree")
    return out


def solve(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    lib = load()
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    X = np.zeros_like(B)
    if lib.oc_solve(A.shape[0], B.shape[1], _f(A), _f(B), _f(X)) != 0:
        raise ValueError("not positive definite")
    return X


def cond(A: np.ndarray) -> float:
    lib = load()
    A = np.ascontiguousarray(A, np.float64)
    return float(lib.oc_cond(A.shape[0], _f(A)))


def make_targets(scene, which: int = 0, opts: Optional[Options] = None, threads=None):
    """Targets of a synthetic workload: the oracle's render of ground-truth set
    ``which`` plus the seeded noise, cast to the workload's target dtype
    (float32, or bfloat16 bit patterns as uint16)."""
    img = render(scene, scene.gt[which], opts, threads)
    y = (img + syn.target_noise(scene, which)).astype(np.float32)
    if scene.target_dtype == "bf16":
        return syn.round_bf16(y)
    return y


def decode_targets(t: np.ndarray) -> np.ndarray:
    if t.dtype == np.uint16:
        return syn.bf16_to_f32(t)
    return np.asarray(t, np.float32)


# --- post-processing (Sec. 4.1 qualitative results; Sec. 4.3) ----------------
# Plain definitions in numpy.

UNOBSERVED, ILL_COND, FAILED = 1, 2, 4


def combine(sets, weights, filt=None) -> np.ndarray:
    """A new lighting from solved coefficient sets (Sec. 4.1, qualitative
    results: light fields are linear, so colorizations can be combined and
    filtered): filt[c] * sum_k weights[k] * sets[k], in FP64.  The weights and
    the filter are taken as the binary32 values a caller hands over."""
    acc = np.zeros(np.shape(sets[0]), np.float64)
    for s, w in zip(sets, weights):
        acc += float(np.float32(w)) * np.asarray(s, np.float64)
    if filt is not None:
        acc *= np.asarray(filt, np.float32).astype(np.float64)  # last axis: channels
    return acc


def mask_value(coeffs, channel: int) -> np.ndarray:
    """Mask value of every Gaussian in one channel (Sec. 4.3): its colour
    averaged over all view directions.  Only the l = 0 harmonic has a non-zero
    mean over the sphere, so the average is Y_0 c[g][0][channel], with Y_0
    taken from the basis routine; at L = 0 it is the colour itself.  Returned
    in binary32, the precision the keep decision is taken in."""
    y0 = np.float32(sh_basis(0, np.array([[0.0, 0.0, 1.0]]))[0, 0])
    return y0 * np.asarray(coeffs, np.float32)[:, 0, channel]


def mask_filter(coeffs, channel: int = 0, threshold: float = 0.6, status=None):
    """Segmentation filter (Sec. 4.3): a Gaussian stays when its mask value
    reaches the threshold (0.6 in the paper), and, when status bits are given,
    it was observed and solved.  Returns (keep [N] bool, kept indices in
    increasing order)."""
    keep = mask_value(coeffs, channel) >= np.float32(threshold)
    if status is not None:
        keep &= (np.asarray(status) & (UNOBSERVED | FAILED)) == 0
    return keep, np.nonzero(keep)[0].astype(np.int64)


# --- view selection (Sec. 5: fewer camera images) ----------------------------

def observed_pairs(scene, opts: Optional[Options] = None) -> np.ndarray:
    """[n_views, N] bool: view j observes Gaussian g (some pixel of j gives g
    weight), from the oracle's contributions."""
    idx, _ = contributions(scene, opts, cap=max(5_000_000, 4 * scene.n_pixels))
    seen = np.zeros((len(scene.cams), scene.N), bool)
    seen[idx[:, 0], idx[:, 2]] = True
    return seen


def coverage(seen: np.ndarray, views, multiplicity: int) -> int:
    """sum_g min(number of the given views that observe g, multiplicity)."""
    if len(views) == 0:
        return 0
    return int(np.minimum(seen[list(views)].sum(axis=0), multiplicity).sum())


def select_views(seen: np.ndarray, k: int, multiplicity: int = 1):
    """Greedy maximum coverage: k times, take the view whose addition raises
    coverage() the most (lowest index on ties).  Returns (views in pick
    order, objective)."""
    chosen = []
    for _ in range(k):
        base = coverage(seen, chosen, multiplicity)
        best, best_gain = -1, -1
        for j in range(seen.shape[0]):
            if j in chosen:
                continue
            gain = coverage(seen, chosen + [j], multiplicity) - base
            if gain > best_gain:
                best, best_gain = j, gain
        chosen.append(best)
    return chosen, coverage(seen, chosen, multiplicity)
