"""Host-side checks of the C ABI (no GPU needed): every symbol declared in
include/gsc.h is exported, and argument validation rejects bad input before
any device work (GSC_FLAG_VALIDATE_ONLY makes valid calls return without
touching the GPU)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2604_17155_amd import gsc, synthetic as syn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsc.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gsc.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return gsc.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:gsc_status|void|const char\*)\s+(gsc_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["gsc_colorize", "gsc_render", "gsc_ctx_create", "gsc_ctx_destroy",
                     "gsc_get_stats", "gsc_last_error", "gsc_default_options"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _vctx(**over):
    o = gsc.default_options()
    o.flags = gsc.GSC_FLAG_VALIDATE_ONLY
    for k, v in over.items():
        setattr(o, k, v)
    return gsc.Context(o)


FAKE = 4096  # never dereferenced in validate-only mode


def _call(ctx, N=10, cams=None, tdtype=0, C=3, sh_deg=0, lam=(1e-4,), means=FAKE, coeffs=FAKE,
          targets=FAKE):
    cams = cams if cams is not None else syn.circle_cams(2, 3.0, 16, 16)
    arr = gsc.make_cameras(cams)
    lam_a = (ct.c_float * max(1, len(lam)))(*lam)
    return ctx.lib.gsc_colorize(ctx.handle, means, FAKE, FAKE, FAKE, N, arr, len(cams), targets,
                                tdtype, C, sh_deg, lam_a, len(lam), coeffs, None, None)


def test_validate_only_accepts_valid(lib):
    ctx = _vctx()
    assert _call(ctx) == gsc.GSC_OK
    assert _call(ctx, sh_deg=3, lam=(1e-5, 1e-4, 1e-3, 1e-2)) == gsc.GSC_OK
    assert _call(ctx, sh_deg=3, lam=tuple([1e-3] * 16)) == gsc.GSC_OK
    assert _call(ctx, C=64, tdtype=1) == gsc.GSC_OK
    assert _call(ctx, N=0, means=None, coeffs=None) == gsc.GSC_OK
    assert _call(ctx, cams=[], targets=None) == gsc.GSC_OK


@pytest.mark.parametrize("kw,needle", [
    (dict(N=-1), "N must be"),
    (dict(C=0), "C must be"),
    (dict(C=65), "C must be"),
    (dict(sh_deg=4), "sh_deg"),
    (dict(sh_deg=-1), "sh_deg"),
    (dict(sh_deg=3, lam=(1e-4, 1e-4)), "n_lambda"),
    (dict(lam=(-1.0,)), "lambda[0]"),
    (dict(lam=(float("nan"),)), "lambda[0]"),
    (dict(tdtype=7), "tdtype"),
    (dict(means=None), "null Gaussian"),
    (dict(coeffs=None), "coeffs is null"),
    (dict(targets=None), "targets is null"),
])
def test_validate_rejects(lib, kw, needle):
    ctx = _vctx()
    st = _call(ctx, **kw)
    assert st == gsc.GSC_ERR_INVALID_ARG
    assert needle in lib.gsc_last_error().decode()


def test_bad_camera_rejected(lib):
    ctx = _vctx()
    cams = syn.circle_cams(2, 3.0, 16, 16)
    cams[1].width = 0
    assert _call(ctx, cams=cams) == gsc.GSC_ERR_INVALID_ARG
    assert "camera 1" in lib.gsc_last_error().decode()
    cams = syn.circle_cams(2, 3.0, 16, 16)
    cams[0].fx = -1.0
    assert _call(ctx, cams=cams) == gsc.GSC_ERR_INVALID_ARG


def test_bad_options_rejected(lib):
    for over in [dict(alpha_max=1.5), dict(t_min=-1.0), dict(znear=0.0), dict(sigma_cut=0.0),
                 dict(bin_size=8), dict(bin_size=64), dict(accumulate_variant=5),
                 dict(accumulate_variant=128 | 48), dict(accumulate_variant=128 | 8),
                 dict(accumulate_variant=256 | 16), dict(schedule=3), dict(schedule=-1)]:
        o = gsc.default_options()
        for k, v in over.items():
            setattr(o, k, v)
        h = ct.c_void_p()
        st = lib.gsc_ctx_create(ct.byref(h), ct.byref(o))
        assert st == gsc.GSC_ERR_INVALID_ARG


def test_accumulate_variants_accepted(lib):
    for v in [0, 1, 2, 3, 4, 8, 16, 128 | 1, 128 | 16, 128 | 32, 128 | 64]:
        o = gsc.default_options()
        o.accumulate_variant = v
        h = ct.c_void_p()
        assert lib.gsc_ctx_create(ct.byref(h), ct.byref(o)) == gsc.GSC_OK, v
        lib.gsc_ctx_destroy(h)


def test_default_options_values(lib):
    o = gsc.default_options()
    assert o.accumulate_variant == 0 and o.bin_size == 0
    assert o.schedule == gsc.GSC_SCHEDULE_AUTO
    assert o.profile_stages == 0
    assert o.alpha_min == np.float32(1 / 255)
    assert o.alpha_max == np.float32(0.99)
    assert o.t_min == np.float32(1e-4)
    assert o.sigma_cut == 3.0 and o.dilation == np.float32(0.3)


def test_render_validation(lib):
    ctx = _vctx()
    cams = syn.circle_cams(2, 3.0, 16, 16)
    arr = gsc.make_cameras(cams)
    st = lib.gsc_render(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 0, 0, FAKE, None)
    assert st == gsc.GSC_ERR_INVALID_ARG
    st = lib.gsc_render(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 3, 0, FAKE, None)
    assert st == gsc.GSC_OK


def test_binding_has_no_fallback(tmp_path):
    with pytest.raises(ImportError):
        gsc.load(str(tmp_path / "missing.so"))


def test_backward_validation(lib):
    ctx = _vctx()
    cams = syn.circle_cams(2, 3.0, 16, 16)
    arr = gsc.make_cameras(cams)
    lam = (ct.c_float * 1)(1e-4)
    cb = lib.gsc_colorize_backward
    # valid: both outputs, or only one of them
    assert cb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 0, 3, 0, lam, 1, FAKE, FAKE,
              FAKE, FAKE, None) == gsc.GSC_OK
    assert cb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, None, 0, 3, 0, lam, 1, FAKE, FAKE,
              FAKE, None, None) == gsc.GSC_OK
    # missing upstream gradient, missing targets when dL/do is wanted, bad channel count
    assert cb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 0, 3, 0, lam, 1, FAKE, None,
              FAKE, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert "grad_coeffs" in lib.gsc_last_error().decode()
    assert cb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, None, 0, 3, 0, lam, 1, FAKE, FAKE,
              None, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert cb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 0, 0, 0, lam, 1, FAKE, FAKE,
              FAKE, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    rb = lib.gsc_render_backward
    assert rb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 3, 0, FAKE, FAKE, FAKE,
              None) == gsc.GSC_OK
    assert rb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 3, 0, None, FAKE, FAKE,
              None) == gsc.GSC_ERR_INVALID_ARG
    assert "grad_images" in lib.gsc_last_error().decode()
    assert rb(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, None, 3, 0, FAKE, FAKE, FAKE,
              None) == gsc.GSC_ERR_INVALID_ARG


def test_plan_validation(lib):
    ctx = _vctx()
    cams = syn.circle_cams(4, 3.0, 16, 16)
    arr = gsc.make_cameras(cams)

    def create(scenes, C=16, sh_deg=0):
        tab = (gsc.GscScene * max(1, len(scenes)))()
        for i, sc in enumerate(scenes):
            tab[i].gaussian_offset, tab[i].n_gaussians = sc[0], sc[1]
            tab[i].camera_offset, tab[i].n_cameras = sc[2], sc[3]
        h = ct.c_void_p()
        return lib.gsc_plan_create(ctx.handle, tab, len(scenes), FAKE, FAKE, FAKE, FAKE, arr, 4, C,
                                   sh_deg, ct.byref(h), None)

    assert create([(0, 100, 0, 2), (100, 50, 2, 2)]) == gsc.GSC_OK
    assert create([]) == gsc.GSC_OK
    assert create([(0, 100, 0, 2), (50, 100, 2, 2)]) == gsc.GSC_ERR_INVALID_ARG
    assert "share" in lib.gsc_last_error().decode()
    assert create([(0, 100, 3, 2)]) == gsc.GSC_ERR_INVALID_ARG
    assert "cameras out of range" in lib.gsc_last_error().decode()
    assert create([(0, -1, 0, 2)]) == gsc.GSC_ERR_INVALID_ARG
    assert create([(0, 1 << 26, 0, 2)]) == gsc.GSC_ERR_INVALID_ARG
    assert create([(0, 10, 0, 2)], C=65) == gsc.GSC_ERR_INVALID_ARG
    assert create([(0, 10, 0, 2)], sh_deg=4) == gsc.GSC_ERR_INVALID_ARG
    assert lib.gsc_colorize_batched(None, FAKE, 0, None, 1, FAKE, None, None) == gsc.GSC_ERR_INVALID_ARG


def _call_noalloc(ctx, N=10, n_cams=2, C=3, sh_deg=0, lam=(1e-4,), res=16):
    cams = syn.circle_cams(n_cams, 3.0, res, res) if n_cams <= 64 else syn.hemisphere_cams(n_cams, 3.0, res, res)
    arr = gsc.make_cameras(cams)
    lam_a = (ct.c_float * max(1, len(lam)))(*lam)
    return ctx.lib.gsc_colorize_noalloc(ctx.handle, FAKE, FAKE, FAKE, FAKE, N, arr, len(cams), FAKE,
                                        0, C, sh_deg, lam_a, len(lam), FAKE, None, None)


def test_noalloc_validation(lib):
    """The allocation-free colorize validates like gsc_colorize and rejects,
    before any device work, calls whose known sizes exceed its fixed scratch."""
    ctx = _vctx()
    assert _call_noalloc(ctx) == gsc.GSC_OK
    assert _call_noalloc(ctx, N=2000, n_cams=8, res=64) == gsc.GSC_OK
    assert _call_noalloc(ctx, C=0) == gsc.GSC_ERR_INVALID_ARG
    st = _call_noalloc(ctx, N=300_000, n_cams=100, sh_deg=3, lam=(1e-4,))
    assert st == gsc.GSC_ERR_CAPACITY
    assert "static scratch" in lib.gsc_last_error().decode()
    st = _call_noalloc(ctx, N=10, n_cams=1025)
    assert st == gsc.GSC_ERR_CAPACITY
    assert "1024 cameras" in lib.gsc_last_error().decode()


def test_batch_limit_options(lib):
    o = gsc.default_options()
    assert o.batch_items == 0 and o.batch_pairs == 0
    for over, ok in [(dict(batch_items=1), True), (dict(batch_items=1 << 26), True),
                     (dict(batch_items=(1 << 26) + 1), False), (dict(batch_pairs=5), True),
                     (dict(batch_pairs=(1 << 31) - 1), True), (dict(batch_pairs=1 << 31), False)]:
        o = gsc.default_options()
        for k, v in over.items():
            setattr(o, k, v)
        h = ct.c_void_p()
        st = lib.gsc_ctx_create(ct.byref(h), ct.byref(o))
        assert (st == gsc.GSC_OK) == ok, over
        if st == gsc.GSC_OK:
            lib.gsc_ctx_destroy(h)


def test_refine_validation(lib):
    ctx = _vctx()
    cams = syn.circle_cams(2, 3.0, 16, 16)
    arr = gsc.make_cameras(cams)
    lam_a = (ct.c_float * 1)(1e-4)

    def call(n_refine, C=3):
        return lib.gsc_colorize_refine(ctx.handle, FAKE, FAKE, FAKE, FAKE, 10, arr, 2, FAKE, 0, C, 0,
                                       lam_a, 1, n_refine, FAKE, None, None)
    assert call(0) == gsc.GSC_OK and call(5) == gsc.GSC_OK
    assert call(-1) == gsc.GSC_ERR_INVALID_ARG and "n_refine" in lib.gsc_last_error().decode()
    assert call(3, C=0) == gsc.GSC_ERR_INVALID_ARG


def test_post_processing_validation(lib):
    """gsc_combine_coeffs and gsc_mask_filter reject bad arguments before any
    device work."""
    ptrs = (ct.c_void_p * 17)(*([FAKE] * 17))
    w = (ct.c_float * 17)(*([1.0] * 17))
    comb = lib.gsc_combine_coeffs
    assert comb(ptrs, w, 0, None, 10, 0, 3, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert "n_sets" in lib.gsc_last_error().decode()
    assert comb(ptrs, w, 2, None, 10, 4, 3, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert comb(ptrs, w, 2, None, 10, 0, 65, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert comb(ptrs, w, 2, None, -1, 0, 3, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert comb(ptrs, w, 2, None, 10, 0, 3, None, None) == gsc.GSC_ERR_INVALID_ARG
    bad_w = (ct.c_float * 2)(1.0, float("nan"))
    assert comb(ptrs, bad_w, 2, None, 10, 0, 3, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert "weights[1]" in lib.gsc_last_error().decode()
    bad_f = (ct.c_float * 3)(1.0, float("inf"), 1.0)
    assert comb(ptrs, w, 2, bad_f, 10, 0, 3, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    # out aliasing a set is allowed up to 16 sets only
    assert comb(ptrs, w, 17, None, 10, 0, 3, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    assert "alias" in lib.gsc_last_error().decode()
    null_set = (ct.c_void_p * 2)(FAKE, None)
    assert comb(null_set, w, 2, None, 10, 0, 3, FAKE, None) == gsc.GSC_ERR_INVALID_ARG
    # nothing to do: no device work, success
    assert comb(ptrs, w, 2, None, 0, 0, 3, FAKE, None) == gsc.GSC_OK

    ctx = _vctx()
    mf = lib.gsc_mask_filter
    assert mf(ctx.handle, FAKE, 10, 0, 3, 0, 0.6, None, FAKE, None, None, None) == gsc.GSC_OK
    assert mf(ctx.handle, FAKE, 10, 0, 3, 3, 0.6, None, FAKE, None, None, None) == gsc.GSC_ERR_INVALID_ARG
    assert "channel" in lib.gsc_last_error().decode()
    assert mf(ctx.handle, FAKE, 10, 0, 3, 0, float("nan"), None, FAKE, None, None, None) == gsc.GSC_ERR_INVALID_ARG
    assert mf(ctx.handle, FAKE, 10, 0, 3, 0, 0.6, None, None, None, None, None) == gsc.GSC_ERR_INVALID_ARG
    assert "no output" in lib.gsc_last_error().decode()
    assert mf(ctx.handle, None, 10, 0, 3, 0, 0.6, None, FAKE, None, None, None) == gsc.GSC_ERR_INVALID_ARG
    assert mf(None, FAKE, 10, 0, 3, 0, 0.6, None, FAKE, None, None, None) == gsc.GSC_ERR_INVALID_ARG
    assert mf(ctx.handle, FAKE, 1 << 26, 0, 3, 0, 0.6, None, FAKE, None, None, None) == gsc.GSC_ERR_UNSUPPORTED
