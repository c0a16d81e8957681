"""gsc_colorize_noalloc against gsc_colorize: the allocation-free entry point
runs the same kernels with every scratch buffer taken from the library's
fixed device array, so its results must match the allocating entry point's
(coefficients within the parity tolerance, statuses and contribution counts
exactly), on two calls in a row, the second with a smaller input."""
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


def _both(gsc, sc, y):
    import torch
    m, s, q, o = gsc.scene_tensors(sc)
    t = parity.to_device_targets(y)
    lam = list(sc.lam)
    ref_ctx = gsc.Context()
    c_ref, st_ref = ref_ctx.colorize(m, s, q, o, sc.cams, t, sc.sh_deg, lam)
    torch.cuda.synchronize()
    n_ref = ref_ctx.stats().contributions
    ctx = gsc.Context()
    nb = (sc.sh_deg + 1) ** 2
    # outputs pre-filled with garbage: the call must overwrite every entry
    c = torch.full((sc.N, nb, sc.C), 7.0, dtype=torch.float32, device="cuda")
    st = torch.full((sc.N,), 0xFF, dtype=torch.uint8, device="cuda")
    ctx.colorize_noalloc(m, s, q, o, sc.cams, t, sc.sh_deg, lam, c, st)
    torch.cuda.synchronize()
    n = ctx.stats().contributions
    return (c_ref.cpu().numpy(), st_ref.cpu().numpy(), n_ref), (c.cpu().numpy(), st.cpu().numpy(), n)


def _compare(ref, got, label):
    c_ref, st_ref, n_ref = ref
    c, st, n = got
    N = c_ref.shape[0]
    nrm = np.linalg.norm(c_ref.reshape(N, -1).astype(np.float64), axis=1)
    obs = (st_ref & 1) == 0
    tau = 1e-3 * np.median(nrm[obs]) if obs.any() else 1.0
    e = np.linalg.norm((c.astype(np.float64) - c_ref).reshape(N, -1), axis=1) / np.maximum(nrm, tau)
    print(f"{label}: N={N} observed={int(obs.sum())} max e={e.max():.2e} "
          f"contributions {n} vs {n_ref}", flush=True)
    assert np.array_equal(st, st_ref), label + ": statuses differ"
    assert n == n_ref, label + ": contribution counts differ"
    assert e.max() <= parity.TOL_F32, label


def test_noalloc_matches_colorize_twice(gsc_mod):
    big = syn.make_relight(n=6000, n_cams=8, res=128)
    big.cams = syn.hemisphere_cams(8, 3.0, 136, 120)
    y_big = oracle.make_targets(big)
    small = syn.make_plain()
    y_small = oracle.make_targets(small)
    print("[case] noalloc relight 6k L3 C3 136x120 then plain 2k L0 C3", flush=True)
    ref, got = _both(gsc_mod, big, y_big)
    _compare(ref, got, "relight 6k L3")
    ref, got = _both(gsc_mod, small, y_small)
    _compare(ref, got, "plain 2k L0")


def test_noalloc_bf16_channels(gsc_mod):
    sc = syn.make_segment_scene(0, n_override=5000, cams_override=6)
    sc.cams = syn.hemisphere_cams(6, 3.0, 160, 120)
    y = oracle.make_targets(sc)
    print("[case] noalloc segment 5k L0 C16 bf16", flush=True)
    ref, got = _both(gsc_mod, sc, y)
    _compare(ref, got, "segment 5k L0 C16")


def test_noalloc_rejects_oversize(gsc_mod):
    import torch
    gsc = gsc_mod
    cams = syn.hemisphere_cams(100, 3.0, 64, 64)
    N = 300_000
    ctx = gsc.Context()
    f = lambda *shape: torch.zeros(shape, dtype=torch.float32, device="cuda")
    with pytest.raises(gsc.GscError) as ei:
        ctx.colorize_noalloc(f(N, 3), f(N, 3), f(N, 4), f(N), cams, f(100 * 64 * 64, 3), 3,
                             [1e-4], f(N, 16, 3))
    assert ei.value.status == gsc.GSC_ERR_CAPACITY
    assert "static scratch" in str(ei.value)
