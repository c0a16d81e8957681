"""GPU parity of gsc_colorize_refine (Algorithm 1 with refinement passes)
against the oracle's refinement (oracle.refine), pass by pass."""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_17155_amd import gsc
    import __graft_entry__
    __graft_entry__._ensure_built()
    gsc.load()
    return gsc


def _refine_case(gsc_mod, sc, y, label, passes=(1, 2, 3), **ctx_opts):
    import torch
    print(f"[case] refine {label}: N={sc.N} cams={len(sc.cams)} L={sc.sh_deg} C={sc.C}", flush=True)
    ref = oracle.refine(sc, y, max(passes), return_all=True)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    t = parity.to_device_targets(y)
    ctx = gsc_mod.Context(**ctx_opts)
    out = {}
    for k in (0,) + tuple(passes):
        c, st = ctx.colorize_refine(m, s, q, o, sc.cams, t, sc.sh_deg, list(sc.lam), k)
        torch.cuda.synchronize()
        c = c.cpu().numpy()
        rk = dict(ref)
        rk["coeffs"] = ref["history"][k]
        msg = parity.check_colorize(c, st.cpu().numpy(), rk, label=f"{label} after {k} pass(es)")
        print(msg, flush=True)
        out[k] = c
    # refinement moves the coefficients (colour mixing of overlapping splats)
    e1, obs = parity.rel_errors(out[max(passes)], dict(coeffs=ref["history"][0], status=ref["status"]))
    assert np.median(e1[obs]) > 1e-3
    return ctx


def test_refine_relight_l3(gsc_mod):
    sc = syn.make_relight(n=6000, n_cams=8, res=128)
    y = oracle.make_targets(sc)
    ctx = _refine_case(gsc_mod, sc, y, "relight 6k L3 C3")
    assert ctx.stats().view_batches == 1


def test_refine_plain_l0(gsc_mod):
    sc = syn.make_plain()
    y = oracle.make_targets(sc)
    _refine_case(gsc_mod, sc, y, "plain 2k L0 C3")


def test_refine_bf16_segment(gsc_mod):
    sc = syn.make_segment_scene(0, n_override=4000, cams_override=6)
    sc.cams = syn.hemisphere_cams(6, 3.0, 160, 120)
    y = oracle.make_targets(sc)
    _refine_case(gsc_mod, sc, y, "segment 4k L0 C16 bf16", passes=(1, 2))


def test_refine_view_batches(gsc_mod):
    """Three view batches: every pass bins each batch again."""
    sc = syn.make_relight(n=3000, n_cams=7, res=96, sh_deg=2)
    y = oracle.make_targets(sc)
    ctx = _refine_case(gsc_mod, sc, y, "relight 3k L2 C3, 3 view batches", passes=(1, 2),
                       batch_items=3 * 3000)
    assert ctx.stats().view_batches == 3
