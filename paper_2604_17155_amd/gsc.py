"""Python binding of libgsc (ctypes).  Argument marshalling only: every step
of colorize and render runs in the HIP library.  PyTorch supplies device
memory and the current stream.

Importing this module does not need a GPU; calling into the library does.
If libgsc.so has not been built the loader raises instead of falling back to
anything else.
"""
from __future__ import annotations

import ctypes as ct
import weakref
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsc.so")

GSC_OK = 0
GSC_ERR_INVALID_ARG = -1
GSC_ERR_HIP = -2
GSC_ERR_CAPACITY = -3
GSC_ERR_UNSUPPORTED = -4
GSC_ERR_NOT_CAPTURABLE = -5
GSC_F32 = 0
GSC_BF16 = 1
GSC_G_UNOBSERVED = 1
GSC_G_ILL_COND = 2
GSC_G_FAILED = 4
GSC_FLAG_VALIDATE_ONLY = 1


class GscCamera(ct.Structure):
    _fields_ = [("R", ct.c_float * 9), ("t", ct.c_float * 3), ("fx", ct.c_float),
                ("fy", ct.c_float), ("cx", ct.c_float), ("cy", ct.c_float),
                ("width", ct.c_int32), ("height", ct.c_int32), ("pixel_offset", ct.c_int64)]


class GscOptions(ct.Structure):
    _fields_ = [("alpha_min", ct.c_float), ("alpha_max", ct.c_float), ("t_min", ct.c_float),
                ("sigma_cut", ct.c_float), ("dilation", ct.c_float), ("znear", ct.c_float),
                ("kappa_max", ct.c_float), ("flags", ct.c_int32), ("bin_size", ct.c_int32),
                ("accumulate_variant", ct.c_int32), ("schedule", ct.c_int32),
                ("profile_stages", ct.c_uint32), ("batch_items", ct.c_uint32),
                ("batch_pairs", ct.c_uint32)]


GSC_SCHEDULE_AUTO, GSC_SCHEDULE_GRID, GSC_SCHEDULE_LONGEST_FIRST = 0, 1, 2
GSC_FLAG_PROFILE = 2
GSC_FLAG_REUSE_BINNING = 4
GSC_FLAG_DETERMINISTIC = 8
GSC_FLAG_CHECK_FINITE = 16
STAGES = ["project", "depth_sort", "scan", "emit", "tile_sort", "blend", "solve", "blend_adjoint"]


class GscStats(ct.Structure):
    _fields_ = [("contributions", ct.c_uint64), ("pairs", ct.c_uint64), ("items", ct.c_uint64),
                ("view_batches", ct.c_uint32), ("ill_conditioned", ct.c_uint32),
                ("bin_size", ct.c_uint32),
                ("stage_ms", ct.c_float * 8), ("stage_launches", ct.c_uint32 * 8)]

    def stage_dict(self):
        return {n: float(self.stage_ms[i]) for i, n in enumerate(STAGES)}


class GscExtras(ct.Structure):
    _fields_ = [("view_sums", ct.c_void_p), ("visibility", ct.c_void_p), ("counts", ct.c_void_p)]


class GscScene(ct.Structure):
    _fields_ = [("gaussian_offset", ct.c_int64), ("n_gaussians", ct.c_int64),
                ("camera_offset", ct.c_int32), ("n_cameras", ct.c_int32)]


class GscPlanInfo(ct.Structure):
    _fields_ = [("contributions", ct.c_uint64), ("items", ct.c_uint64),
                ("pair_capacity", ct.c_uint64), ("dropped_pairs", ct.c_uint32),
                ("ill_conditioned", ct.c_uint32), ("batches", ct.c_uint32), ("views", ct.c_uint32),
                ("bin_size", ct.c_int32), ("accumulate_variant", ct.c_int32), ("tuned_variant", ct.c_int32 * 8),
                ("tuned_ms", ct.c_float * 8)]


class GscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gsc error {status}: {msg}")
        self.status = status


_lib = None


def load(path: Optional[str] = None):
    """Load libgsc.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libgsc.so not found at {p}; build it with __graft_entry__.build()")
    lib = ct.CDLL(p)
    P, i64, i32 = ct.c_void_p, ct.c_int64, ct.c_int32
    lib.gsc_default_options.argtypes = [ct.POINTER(GscOptions)]
    lib.gsc_default_options.restype = ct.c_int
    lib.gsc_ctx_create.argtypes = [ct.POINTER(P), ct.POINTER(GscOptions)]
    lib.gsc_ctx_create.restype = ct.c_int
    lib.gsc_ctx_destroy.argtypes = [P]
    lib.gsc_ctx_destroy.restype = None
    lib.gsc_ctx_set_options.argtypes = [P, ct.POINTER(GscOptions)]
    lib.gsc_ctx_set_options.restype = ct.c_int
    lib.gsc_colorize.argtypes = [P, P, P, P, P, i64, P, i32, P, i32, i32, i32, P, i32, P, P, P]
    lib.gsc_colorize.restype = ct.c_int
    lib.gsc_colorize_ex.argtypes = [P, P, P, P, P, i64, P, i32, P, i32, i32, i32, P, i32, P, P,
                                    ct.POINTER(GscExtras), P]
    lib.gsc_colorize_ex.restype = ct.c_int
    lib.gsc_colorize_refine.argtypes = [P, P, P, P, P, i64, P, i32, P, i32, i32, i32, P, i32, i32, P, P, P]
    lib.gsc_colorize_refine.restype = ct.c_int
    lib.gsc_colorize_noalloc.argtypes = [P, P, P, P, P, i64, P, i32, P, i32, i32, i32, P, i32, P, P, P]
    lib.gsc_colorize_noalloc.restype = ct.c_int
    lib.gsc_render.argtypes = [P, P, P, P, P, i64, P, i32, P, i32, i32, P, P]
    lib.gsc_render.restype = ct.c_int
    lib.gsc_colorize_backward.argtypes = [P, P, P, P, P, i64, P, i32, P, i32, i32, i32, P, i32, P, P,
                                          P, P, P]
    lib.gsc_colorize_backward.restype = ct.c_int
    lib.gsc_render_backward.argtypes = [P, P, P, P, P, i64, P, i32, P, i32, i32, P, P, P, P]
    lib.gsc_render_backward.restype = ct.c_int
    lib.gsc_plan_create.argtypes = [P, P, i32, P, P, P, P, P, i32, i32, i32, ct.POINTER(P), P]
    lib.gsc_plan_create.restype = ct.c_int
    lib.gsc_plan_destroy.argtypes = [P]
    lib.gsc_plan_destroy.restype = None
    lib.gsc_colorize_batched.argtypes = [P, P, i32, P, i32, P, P, P]
    lib.gsc_colorize_batched.restype = ct.c_int
    lib.gsc_plan_autotune.argtypes = [P, P, i32, P, i32, P, P, P]
    lib.gsc_plan_autotune.restype = ct.c_int
    lib.gsc_plan_get_info.argtypes = [P, ct.POINTER(GscPlanInfo)]
    lib.gsc_plan_get_info.restype = ct.c_int
    lib.gsc_combine_coeffs.argtypes = [P, P, i32, P, i64, i32, i32, P, P]
    lib.gsc_combine_coeffs.restype = ct.c_int
    lib.gsc_mask_filter.argtypes = [P, P, i64, i32, i32, i32, ct.c_float, P, P, P, P, P]
    lib.gsc_mask_filter.restype = ct.c_int
    lib.gsc_select_views.argtypes = [P, P, P, P, P, i64, P, i32, i32, i32, P, P, P]
    lib.gsc_select_views.restype = ct.c_int
    lib.gsc_get_stats.argtypes = [P, ct.POINTER(GscStats)]
    lib.gsc_get_stats.restype = ct.c_int
    lib.gsc_last_error.argtypes = []
    lib.gsc_last_error.restype = ct.c_char_p
    if path is None:
        _lib = lib
    return lib


def _check(lib, st: int):
    if st != GSC_OK:
        raise GscError(st, lib.gsc_last_error().decode())


def default_options() -> GscOptions:
    lib = load()
    o = GscOptions()
    _check(lib, lib.gsc_default_options(ct.byref(o)))
    return o


def make_cameras(cams: Sequence, offsets: Optional[Sequence[int]] = None):
    """ctypes array of gsc_camera from objects with R, t, fx, fy, cx, cy,
    width, height.  Pixel offsets default to the cameras' cumulative sizes."""
    arr = (GscCamera * max(1, len(cams)))()
    off = 0
    for i, c in enumerate(cams):
        arr[i].R[:] = [float(v) for v in np.asarray(c.R, dtype=np.float32).reshape(-1)]
        arr[i].t[:] = [float(v) for v in c.t]
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[i].width, arr[i].height = int(c.width), int(c.height)
        arr[i].pixel_offset = off if offsets is None else int(offsets[i])
        off += int(c.width) * int(c.height)
    return arr


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """Owns a gsc_ctx (device scratch reused across calls)."""

    def __init__(self, options: Optional[GscOptions] = None, **overrides):
        self.lib = load()
        o = options or default_options()
        for k, v in overrides.items():
            setattr(o, k, v)
        h = ct.c_void_p()
        _check(self.lib, self.lib.gsc_ctx_create(ct.byref(h), ct.byref(o)))
        self.handle = h
        self.options = o

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gsc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, **overrides):
        for k, v in overrides.items():
            setattr(self.options, k, v)
        _check(self.lib, self.lib.gsc_ctx_set_options(self.handle, ct.byref(self.options)))


    # --- binning reuse -------------------------------------------------------
    # The library may reuse the tile lists of the previous call on this context
    # (GSC_FLAG_REUSE_BINNING) when the geometry is unchanged.  That is only
    # asked for when the caller allows it (reuse_binning=True) and the
    # geometry tensors are the very objects of the previous call, unmodified
    # since (same version counters), with the same cameras.
    def _reuse_begin(self, tensors, cam_arr, allow: bool) -> bool:
        last = getattr(self, "_last_geo", None)
        ok = False
        if allow and last is not None:
            refs, vers, cb = last
            ok = (all(r() is t for r, t in zip(refs, tensors)) and
                  vers == tuple(int(t._version) for t in tensors) and cb == bytes(cam_arr))
        if ok:
            self.options.flags |= GSC_FLAG_REUSE_BINNING
            _check(self.lib, self.lib.gsc_ctx_set_options(self.handle, ct.byref(self.options)))
        self._last_geo = None
        return ok

    def _reuse_end(self, tensors, cam_arr, used: bool, succeeded: bool):
        if used:
            self.options.flags &= ~GSC_FLAG_REUSE_BINNING
            _check(self.lib, self.lib.gsc_ctx_set_options(self.handle, ct.byref(self.options)))
        if succeeded:
            self._last_geo = ([weakref.ref(t) for t in tensors],
                              tuple(int(t._version) for t in tensors), bytes(cam_arr))

    def stats(self) -> GscStats:
        out = GscStats()
        _check(self.lib, self.lib.gsc_get_stats(self.handle, ct.byref(out)))
        return out

    def colorize(self, means, scales, quats, opacities, cams, targets, sh_deg: int, lam,
                 coeffs=None, status=None, offsets=None, stream=None, with_status: bool = True,
                 extras=None, reuse_binning: bool = False):
        """Solve the per-Gaussian regularised normal equations.  Returns
        (coeffs [N,(L+1)^2,C] float32, status [N] uint8 or None).

        extras: optional set of names among {"view_sums", "visibility",
        "counts"}; when given, a third element is returned: a dict of device
        tensors (view_sums [n_cams,N,C+1], visibility [N], counts [N] int32)."""
        import torch
        N = int(means.shape[0])
        C = int(targets.shape[1]) if targets.dim() == 2 else 1
        nb = (sh_deg + 1) ** 2
        if targets.dtype == torch.float32:
            td = GSC_F32
        elif targets.dtype == torch.bfloat16:
            td = GSC_BF16
        else:
            raise ValueError("targets must be float32 or bfloat16")
        dev = means.device
        if coeffs is None:
            coeffs = torch.empty((N, nb, C), dtype=torch.float32, device=dev)
        if status is None and with_status:
            status = torch.empty((N,), dtype=torch.uint8, device=dev)
        lam_a = (ct.c_float * len(lam))(*[float(v) for v in lam])
        cam_arr = make_cameras(cams, offsets)
        xd = None
        xs = None
        if extras:
            xd = {}
            if "view_sums" in extras:
                xd["view_sums"] = torch.zeros((len(cams), N, C + 1), dtype=torch.float32, device=dev)
            if "visibility" in extras:
                xd["visibility"] = torch.zeros((N,), dtype=torch.float32, device=dev)
            if "counts" in extras:
                xd["counts"] = torch.zeros((N,), dtype=torch.int32, device=dev)
            xs = GscExtras(_ptr(xd.get("view_sums")), _ptr(xd.get("visibility")),
                           _ptr(xd.get("counts")))
        geo = (means, scales, quats, opacities)
        used = self._reuse_begin(geo, cam_arr, reuse_binning)
        st = self.lib.gsc_colorize_ex(self.handle, _ptr(means), _ptr(scales), _ptr(quats),
                                      _ptr(opacities), N, cam_arr, len(cams), _ptr(targets), td, C,
                                      sh_deg, lam_a, len(lam), _ptr(coeffs), _ptr(status),
                                      None if xs is None else ct.byref(xs), _stream_ptr(stream))
        self._reuse_end(geo, cam_arr, used, st == GSC_OK)
        _check(self.lib, st)
        if xd is not None:
            return coeffs, status, xd
        return coeffs, status

    def colorize_refine(self, means, scales, quats, opacities, cams, targets, sh_deg: int, lam,
                        n_refine: int, coeffs=None, status=None, offsets=None, stream=None):
        """Colorize, then n_refine refinement passes (gsc_colorize_refine).
        Returns (coeffs [N,(L+1)^2,C] float32, status [N] uint8)."""
        import torch
        N = int(means.shape[0])
        C = int(targets.shape[1])
        nb = (sh_deg + 1) ** 2
        if coeffs is None:
            coeffs = torch.empty((N, nb, C), dtype=torch.float32, device=means.device)
        if status is None:
            status = torch.empty((N,), dtype=torch.uint8, device=means.device)
        lam_a = (ct.c_float * len(lam))(*[float(v) for v in lam])
        cam_arr = make_cameras(cams, offsets)
        st = self.lib.gsc_colorize_refine(self.handle, _ptr(means), _ptr(scales), _ptr(quats),
                                          _ptr(opacities), N, cam_arr, len(cams), _ptr(targets),
                                          _tdtype(targets), C, sh_deg, lam_a, len(lam), int(n_refine),
                                          _ptr(coeffs), _ptr(status), _stream_ptr(stream))
        _check(self.lib, st)
        return coeffs, status

    def colorize_noalloc(self, means, scales, quats, opacities, cams, targets, sh_deg: int, lam,
                         coeffs, status=None, offsets=None, stream=None):
        """gsc_colorize_noalloc: colorize with the library's fixed scratch
        (no allocation inside the call).  coeffs [N,(L+1)^2,C] float32 and
        status [N] uint8 (optional) are caller-allocated outputs."""
        N = int(means.shape[0])
        C = int(targets.shape[1])
        lam_a = (ct.c_float * len(lam))(*[float(v) for v in lam])
        cam_arr = make_cameras(cams, offsets)
        st = self.lib.gsc_colorize_noalloc(self.handle, _ptr(means), _ptr(scales), _ptr(quats),
                                           _ptr(opacities), N, cam_arr, len(cams), _ptr(targets),
                                           _tdtype(targets), C, sh_deg, lam_a, len(lam),
                                           _ptr(coeffs), _ptr(status), _stream_ptr(stream))
        _check(self.lib, st)
        return coeffs, status

    def select_views(self, means, scales, quats, opacities, cams, k: int, multiplicity: int = 1,
                     offsets=None, stream=None):
        """gsc_select_views: k view indices picked greedily for coverage
        (in pick order) and the coverage objective they reach."""
        cam_arr = make_cameras(cams, offsets)
        out = (ct.c_int32 * max(1, int(k)))()
        obj = ct.c_int64(0)
        st = self.lib.gsc_select_views(self.handle, _ptr(means), _ptr(scales), _ptr(quats),
                                       _ptr(opacities), int(means.shape[0]), cam_arr, len(cams), int(k),
                                       int(multiplicity), out, ct.byref(obj), _stream_ptr(stream))
        _check(self.lib, st)
        return [int(out[i]) for i in range(int(k))], int(obj.value)

    def mask_filter(self, coeffs, channel: int = 0, threshold: float = 0.6, status=None,
                    want_keep: bool = True, stream=None):
        """Segmentation filter (gsc_mask_filter) of coefficients [N,(L+1)^2,C].
        Returns (keep [N] uint8 or None, kept indices [n_kept] int64); reads
        the count back, so it synchronises."""
        import torch
        N, nb, C = (int(v) for v in coeffs.shape)
        sh_deg = int(round(nb ** 0.5)) - 1
        dev = coeffs.device
        keep = torch.empty((N,), dtype=torch.uint8, device=dev) if want_keep else None
        idx = torch.empty((max(N, 1),), dtype=torch.int64, device=dev)
        cnt = torch.zeros((1,), dtype=torch.int64, device=dev)
        st = self.lib.gsc_mask_filter(self.handle, _ptr(coeffs), N, sh_deg, C, int(channel),
                                      float(threshold), _ptr(status), _ptr(keep), _ptr(idx),
                                      _ptr(cnt), _stream_ptr(stream))
        _check(self.lib, st)
        return keep, idx[:int(cnt.item())]

    def render(self, means, scales, quats, opacities, cams, coeffs, images=None, offsets=None,
               stream=None, reuse_binning: bool = False):
        """Render coefficients [N,(L+1)^2,C] to images [sum HW, C] float32."""
        import torch
        N = int(means.shape[0])
        nb, C = int(coeffs.shape[1]), int(coeffs.shape[2])
        sh_deg = int(round(nb ** 0.5)) - 1
        rows = _rows(cams, offsets)
        if images is None:
            images = torch.empty((rows, C), dtype=torch.float32, device=means.device)
        cam_arr = make_cameras(cams, offsets)
        geo = (means, scales, quats, opacities)
        used = self._reuse_begin(geo, cam_arr, reuse_binning)
        st = self.lib.gsc_render(self.handle, _ptr(means), _ptr(scales), _ptr(quats),
                                 _ptr(opacities), N, cam_arr, len(cams), _ptr(coeffs), C, sh_deg,
                                 _ptr(images), _stream_ptr(stream))
        self._reuse_end(geo, cam_arr, used, st == GSC_OK)
        _check(self.lib, st)
        return images


    def colorize_backward(self, means, scales, quats, opacities, cams, targets, sh_deg: int, lam,
                          coeffs, grad_coeffs, want_targets: bool = True, want_opacities: bool = True,
                          offsets=None, stream=None, reuse_binning: bool = False):
        """Adjoint of colorize at `coeffs` for dL/dcoeffs = grad_coeffs.  Returns
        (grad_targets [rows, C] float32 or None, grad_opacities [N] float32 or None)."""
        import torch
        N = int(means.shape[0])
        C = int(targets.shape[1])
        td = _tdtype(targets)
        dev = means.device
        gt = None
        if want_targets:
            # the library writes the camera rows; rows past the last camera stay zero
            gt = torch.empty((int(targets.shape[0]), C), dtype=torch.float32, device=dev)
            used = _rows(cams, offsets)
            if used < gt.shape[0]:
                gt[used:].zero_()
        go = torch.empty((N,), dtype=torch.float32, device=dev) if want_opacities else None
        lam_a = (ct.c_float * len(lam))(*[float(v) for v in lam])
        cam_arr = make_cameras(cams, offsets)
        geo = (means, scales, quats, opacities)
        used = self._reuse_begin(geo, cam_arr, reuse_binning)
        st = self.lib.gsc_colorize_backward(self.handle, _ptr(means), _ptr(scales), _ptr(quats),
                                            _ptr(opacities), N, cam_arr, len(cams), _ptr(targets), td,
                                            C, sh_deg, lam_a, len(lam), _ptr(coeffs),
                                            _ptr(grad_coeffs), _ptr(gt), _ptr(go), _stream_ptr(stream))
        self._reuse_end(geo, cam_arr, used, st == GSC_OK)
        _check(self.lib, st)
        return gt, go

    def render_backward(self, means, scales, quats, opacities, cams, coeffs, grad_images,
                        want_coeffs: bool = True, want_opacities: bool = True, offsets=None,
                        stream=None, reuse_binning: bool = False):
        """Adjoint of render for dL/dimages = grad_images.  Returns
        (grad_coeffs [N,(L+1)^2,C] or None, grad_opacities [N] or None)."""
        import torch
        N = int(means.shape[0])
        nb, C = int(coeffs.shape[1]), int(coeffs.shape[2])
        sh_deg = int(round(nb ** 0.5)) - 1
        dev = means.device
        gc = torch.empty((N, nb, C), dtype=torch.float32, device=dev) if want_coeffs else None
        go = torch.empty((N,), dtype=torch.float32, device=dev) if want_opacities else None
        cam_arr = make_cameras(cams, offsets)
        geo = (means, scales, quats, opacities)
        used = self._reuse_begin(geo, cam_arr, reuse_binning)
        st = self.lib.gsc_render_backward(self.handle, _ptr(means), _ptr(scales), _ptr(quats),
                                          _ptr(opacities), N, cam_arr, len(cams), _ptr(coeffs), C,
                                          sh_deg, _ptr(grad_images), _ptr(gc), _ptr(go),
                                          _stream_ptr(stream))
        self._reuse_end(geo, cam_arr, used, st == GSC_OK)
        _check(self.lib, st)
        return gc, go


class Plan:
    """A batched multi-scene colorize with all sizes fixed at creation.

    scenes: sequence of (gaussian_offset, n_gaussians, camera_offset, n_cameras);
    means/scales/quats/opacities: concatenated device tensors; cams: all cameras
    (their pixel offsets index one concatenated target array; by default the
    cameras' cumulative sizes).  run() allocates nothing when coeffs/status
    are passed in, never synchronises, and may be captured into a graph."""

    def __init__(self, context: Context, scenes, means, scales, quats, opacities, cams, C: int,
                 sh_deg: int, offsets=None, stream=None):
        self.context = context
        self.lib = context.lib
        self.C, self.sh_deg = int(C), int(sh_deg)
        self._keep = (means, scales, quats, opacities)
        tab = (GscScene * max(1, len(scenes)))()
        for i, sc in enumerate(scenes):
            tab[i].gaussian_offset, tab[i].n_gaussians = int(sc[0]), int(sc[1])
            tab[i].camera_offset, tab[i].n_cameras = int(sc[2]), int(sc[3])
        self.n_total = max([int(sc[0]) + int(sc[1]) for sc in scenes] or [0])
        self.cam_arr = make_cameras(cams, offsets)
        h = ct.c_void_p()
        st = self.lib.gsc_plan_create(context.handle, tab, len(scenes), _ptr(means), _ptr(scales),
                                      _ptr(quats), _ptr(opacities), self.cam_arr, len(cams), self.C,
                                      self.sh_deg, ct.byref(h), _stream_ptr(stream))
        _check(self.lib, st)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gsc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _outputs(self, coeffs, status, device):
        import torch
        nb = (self.sh_deg + 1) ** 2
        if coeffs is None:
            coeffs = torch.zeros((self.n_total, nb, self.C), dtype=torch.float32, device=device)
        if status is None:
            status = torch.zeros((self.n_total,), dtype=torch.uint8, device=device)
        return coeffs, status

    def run(self, targets, lam, coeffs=None, status=None, stream=None):
        coeffs, status = self._outputs(coeffs, status, targets.device)
        lam_a = (ct.c_float * len(lam))(*[float(v) for v in lam])
        st = self.lib.gsc_colorize_batched(self.handle, _ptr(targets), _tdtype(targets), lam_a,
                                           len(lam), _ptr(coeffs), _ptr(status), _stream_ptr(stream))
        _check(self.lib, st)
        return coeffs, status

    def autotune(self, targets, lam, coeffs=None, status=None, stream=None):
        coeffs, status = self._outputs(coeffs, status, targets.device)
        lam_a = (ct.c_float * len(lam))(*[float(v) for v in lam])
        st = self.lib.gsc_plan_autotune(self.handle, _ptr(targets), _tdtype(targets), lam_a,
                                        len(lam), _ptr(coeffs), _ptr(status), _stream_ptr(stream))
        _check(self.lib, st)
        return coeffs, status

    def info(self) -> GscPlanInfo:
        out = GscPlanInfo()
        _check(self.lib, self.lib.gsc_plan_get_info(self.handle, ct.byref(out)))
        return out


def combine_coeffs(sets, weights, filt=None, out=None, stream=None):
    """Linear combination of coefficient sets (gsc_combine_coeffs):
    out = filt[c] * sum_k weights[k] * sets[k], each [N,(L+1)^2,C] float32."""
    import torch
    lib = load()
    sets = list(sets)
    N, nb, C = (int(v) for v in sets[0].shape)
    for t in sets:
        if tuple(t.shape) != (N, nb, C) or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("every set must be a contiguous float32 tensor of one shape")
    sh_deg = int(round(nb ** 0.5)) - 1
    if out is None:
        out = torch.empty_like(sets[0])
    ptrs = (ct.c_void_p * len(sets))(*[_ptr(t) for t in sets])
    w = (ct.c_float * len(sets))(*[float(v) for v in weights])
    if len(weights) != len(sets):
        raise ValueError("one weight per set")
    f = None if filt is None else (ct.c_float * C)(*[float(v) for v in filt])
    st = lib.gsc_combine_coeffs(ptrs, w, len(sets), f, N, sh_deg, C, _ptr(out), _stream_ptr(stream))
    _check(lib, st)
    return out


def _rows(cams, offsets=None) -> int:
    if not len(cams):
        return 0
    if offsets is None:
        return sum(int(c.width) * int(c.height) for c in cams)
    return max(int(o) + int(c.width) * int(c.height) for o, c in zip(offsets, cams))


def _tdtype(targets) -> int:
    import torch
    if targets.dtype == torch.float32:
        return GSC_F32
    if targets.dtype == torch.bfloat16:
        return GSC_BF16
    raise ValueError("targets must be float32 or bfloat16")


def scene_tensors(scene, device="cuda"):
    """Device tensors (means, scales, quats, opacities) of a synthetic scene."""
    import torch
    f = lambda a: torch.from_numpy(a).to(device).contiguous()
    return f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacities)
