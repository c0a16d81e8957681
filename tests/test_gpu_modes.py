"""GPU checks of the deterministic accumulate mode (GSC_FLAG_DETERMINISTIC)
and of the input check (GSC_FLAG_CHECK_FINITE).

Deterministic mode: the per-view sums are exact 64-bit fixed-point integers,
so a result is bit-identical across runs, tile schedules and view-batch
splits.  It still passes the oracle gate, and it agrees with the float-atomic
mode within the atomic mode's own rounding."""
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


def _scene(case):
    if case == "relight":
        return syn.make_relight(seed_offset=51, n=6000, n_cams=8, res=128), "relight 6k L3 C3 f32"
    if case == "plain":
        return syn.make_plain(), "plain 2k L0 C3 f32"
    return syn.make_segment_scene(3, n_override=6000, cams_override=8), "segment 6k L0 C16 bf16"


def _run(gsc_mod, sc, t, flags, **opts):
    import torch
    ctx = gsc_mod.Context(flags=flags, **opts)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    c, st, x = ctx.colorize(m, s, q, o, sc.cams, t, sc.sh_deg, list(sc.lam), extras={"view_sums"})
    torch.cuda.synchronize()
    return c.cpu().numpy(), st.cpu().numpy(), x["view_sums"].cpu().numpy()


@pytest.mark.parametrize("case", ["relight", "plain", "segment"])
def test_deterministic_bit_identical(gsc_mod, case):
    sc, label = _scene(case)
    print(f"[case] deterministic {label}", flush=True)
    y = oracle.make_targets(sc)
    t = parity.to_device_targets(y)
    DET = gsc_mod.GSC_FLAG_DETERMINISTIC
    base = _run(gsc_mod, sc, t, DET)
    variants = [dict(schedule=gsc_mod.GSC_SCHEDULE_GRID), dict(schedule=gsc_mod.GSC_SCHEDULE_LONGEST_FIRST),
                dict(batch_items=max(1, sc.N * len(sc.cams) // 3))]
    for v in variants + [dict()]:
        got = _run(gsc_mod, sc, t, DET, **v)
        for a, b, name in zip(base, got, ("coeffs", "status", "view_sums")):
            assert np.array_equal(a, b), f"{label}: {name} differs under {v}"
    ref = oracle.colorize(sc, y)
    msg = parity.check_colorize(base[0], base[1], ref, label=f"{label} deterministic")
    # against the float-atomic mode: both carry the per-view sums' rounding only
    c_at, st_at, vs_at = _run(gsc_mod, sc, t, 0)
    e, obs = parity.rel_errors(base[0], dict(coeffs=c_at.astype(np.float64), status=st_at))
    vs_scale = np.abs(vs_at).max()
    vs_diff = np.abs(base[2].astype(np.float64) - vs_at).max() / vs_scale
    print(msg + f"; vs atomic mode: coeff max {e[obs].max():.2e}, view sums {vs_diff:.2e}", flush=True)
    assert vs_diff <= 1e-5
    assert np.all(e[obs & ~parity.flagged(ref)] <= parity.TOL_F32)


def test_check_finite(gsc_mod):
    import torch
    sc = syn.make_plain()
    y = oracle.make_targets(sc)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    ctx = gsc_mod.Context(flags=gsc_mod.GSC_FLAG_CHECK_FINITE)
    plain = gsc_mod.Context()
    t = parity.to_device_targets(y)
    c_ok, _ = ctx.colorize(m, s, q, o, sc.cams, t, sc.sh_deg, list(sc.lam))
    c_ref, _ = plain.colorize(m, s, q, o, sc.cams, t, sc.sh_deg, list(sc.lam))
    torch.cuda.synchronize()
    assert torch.allclose(c_ok, c_ref, rtol=1e-5, atol=1e-6)
    # a NaN target: rejected, and the message names the array and the row
    bad = t.clone()
    row, ch = 12345, 2
    bad[row, ch] = float("nan")
    with pytest.raises(gsc_mod.GscError) as ei:
        ctx.colorize(m, s, q, o, sc.cams, bad, sc.sh_deg, list(sc.lam))
    assert ei.value.status == gsc_mod.GSC_ERR_INVALID_ARG
    assert "targets" in str(ei.value) and f"element {row * sc.C + ch} " in str(ei.value), str(ei.value)
    assert f"(entry {row})" in str(ei.value)
    # the first of several
    bad[row + 10, 0] = float("inf")
    bad[77, 1] = float("-inf")
    with pytest.raises(gsc_mod.GscError) as ei:
        ctx.colorize(m, s, q, o, sc.cams, bad, sc.sh_deg, list(sc.lam))
    assert "(entry 77)" in str(ei.value)
    # an infinite opacity
    o_bad = o.clone()
    o_bad[5] = float("inf")
    with pytest.raises(gsc_mod.GscError) as ei:
        ctx.colorize(m, s, q, o_bad, sc.cams, t, sc.sh_deg, list(sc.lam))
    assert "opacities" in str(ei.value) and "(entry 5)" in str(ei.value)
    # BF16 targets
    sb = syn.make_segment_scene(0, n_override=3000, cams_override=4)
    yb = parity.to_device_targets(oracle.make_targets(sb))
    yb[9, 4] = float("nan")
    mb, sbb, qb, ob = gsc_mod.scene_tensors(sb)
    with pytest.raises(gsc_mod.GscError) as ei:
        ctx.colorize(mb, sbb, qb, ob, sb.cams, yb, sb.sh_deg, list(sb.lam))
    assert "targets" in str(ei.value) and "(entry 9)" in str(ei.value)
    # without the flag the call goes through (no check is made)
    plain.colorize(m, s, q, o, sc.cams, bad, sc.sh_deg, list(sc.lam))
    torch.cuda.synchronize()
