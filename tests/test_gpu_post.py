"""GPU parity of the post-processing entry points against the oracle:
gsc_combine_coeffs (Sec. 4.1 qualitative results: coefficient sets combine
and filter linearly) and gsc_mask_filter (Sec. 4.3: Gaussians whose mask value
is below 0.6 are removed).

The combination is compared element by element within the rounding bound of
its binary32 arithmetic: an fma chain over n sets and one product with the
filter make at most n + 1 roundings, so
    |out - exact| <= (n + 2) u |f_c| sum_k |w_k x_k|,   u = 2^-24.
The mask filter is an integer result whose decision is taken in binary32 on
both sides: keep bytes, kept indices and count are compared bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import parity

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


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


def _combine_case(gsc_mod, N, L, C, n_sets, filt, seed, alias=False):
    import torch
    print(f"[case] combine N={N} L={L} C={C} sets={n_sets} filter={filt is not None} alias={alias}",
          flush=True)
    rng = np.random.default_rng(seed)
    nb = (L + 1) ** 2
    sets = [rng.normal(0, 1, (N, nb, C)).astype(np.float32) for _ in range(n_sets)]
    w = rng.uniform(-2, 2, n_sets).astype(np.float32)
    f = None if filt is None else np.asarray(filt, np.float32)
    ref = oracle.combine(sets, w, f)
    mag = sum(np.abs(float(wk) * s.astype(np.float64)) for wk, s in zip(w, sets))
    if f is not None:
        mag = mag * np.abs(f.astype(np.float64))
    dev = [torch.from_numpy(s).cuda() for s in sets]
    out = dev[0] if alias else None
    got = gsc_mod.combine_coeffs(dev, w, f, out=out)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    lim = (n_sets + 2) * U * mag + 1e-45
    assert np.all(err <= lim), f"max err {err.max():.3e}, worst ratio {(err / lim).max():.2f}"
    print(f"combine: max err {err.max():.2e}, at most {(err / lim).max():.2f} of the bound", flush=True)


@pytest.mark.parametrize("N,L,C,n_sets,filt,alias", [
    (5000, 3, 3, 3, (1.0, 0.5, 0.25), False),   # float4 path
    (5000, 3, 3, 20, (0.8, 1.0, 1.2), False),   # two launches, the second continuing the sum
    (1001, 0, 3, 4, None, False),               # 3003 floats: scalar path
    (777, 2, 5, 2, (1, 2, 3, 4, 5), True),      # out is the first set
    (3000, 1, 64, 17, None, False),             # widest channel count, two launches
])
def test_combine_parity(gsc_mod, N, L, C, n_sets, filt, alias):
    _combine_case(gsc_mod, N, L, C, n_sets, filt, seed=N + n_sets, alias=alias)


def test_combined_lighting_end_to_end(gsc_mod):
    """Two colorizations on the GPU, combined and filtered on the GPU, against
    the oracle's colorization of the combined, filtered targets (one solve):
    the two agree because colorize is linear in the targets."""
    import torch
    sc = syn.make_relight(seed_offset=41, n=6000, n_cams=8, res=128)
    y1 = oracle.make_targets(sc, 0)
    y2 = np.random.default_rng(41).uniform(0, 1, y1.shape).astype(np.float32)  # a second lighting
    w = np.array([0.6, 0.4], np.float32)
    f = np.array([1.0, 0.7, 0.4], np.float32)
    mixed = (w[0] * y1.astype(np.float64) + w[1] * y2.astype(np.float64)) * f.astype(np.float64)
    ref = oracle.colorize(sc, mixed)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    ctx = gsc_mod.Context()
    c1, st = ctx.colorize(m, s, q, o, sc.cams, parity.to_device_targets(y1), sc.sh_deg, list(sc.lam))
    c2, _ = ctx.colorize(m, s, q, o, sc.cams, parity.to_device_targets(y2), sc.sh_deg, list(sc.lam))
    out = gsc_mod.combine_coeffs([c1, c2], w, f)
    torch.cuda.synchronize()
    msg = parity.check_colorize(out.cpu().numpy(), st.cpu().numpy(), ref,
                                label="relight 6k L3: 0.6 y1 + 0.4 y2, filter (1, 0.7, 0.4)")
    print(msg, flush=True)


def _near_threshold_coeffs(rng, N, L, C, channel, thr):
    """Coefficients whose mask values cluster at the threshold: a third are the
    binary32 neighbours of the smallest kept value, the rest spread widely."""
    y0 = np.float32(oracle.sh_basis(0, np.array([[0.0, 0.0, 1.0]]))[0, 0])
    t = np.float32(thr)
    c = np.float32(t / y0)
    while np.float32(y0 * c) >= t:
        c = np.nextafter(c, np.float32(-np.inf))
    while np.float32(y0 * c) < t:
        c = np.nextafter(c, np.float32(np.inf))
    near = np.array([np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))],
                    np.float32)
    nb = (L + 1) ** 2
    out = rng.normal(0, 2, (N, nb, C)).astype(np.float32)
    pick = rng.random(N) < 1 / 3
    out[pick, 0, channel] = near[rng.integers(0, 3, int(pick.sum()))]
    return out


@pytest.mark.parametrize("N,L,C,channel,with_status", [
    (5000, 0, 16, 3, True),
    (1023, 2, 3, 2, False),
    (1025, 0, 1, 0, True),
    ((1 << 20) + 3, 0, 2, 1, True),
    (1, 3, 3, 0, False),
    (0, 0, 3, 0, True),
])
def test_mask_filter_bit_exact(gsc_mod, N, L, C, channel, with_status):
    import torch
    print(f"[case] mask filter N={N} L={L} C={C} channel={channel} status={with_status}", flush=True)
    rng = np.random.default_rng(N + C)
    thr = 0.6
    coeffs = _near_threshold_coeffs(rng, N, L, C, channel, thr)
    status = rng.choice(np.array([0, 0, 0, 1, 2, 4], np.uint8), N) if with_status else None
    keep_ref, idx_ref = oracle.mask_filter(coeffs, channel, thr, status)
    ctx = gsc_mod.Context()
    st_t = None if status is None else torch.from_numpy(status).cuda()
    keep, idx = ctx.mask_filter(torch.from_numpy(coeffs).cuda(), channel, thr, st_t)
    torch.cuda.synchronize()
    assert np.array_equal(keep.cpu().numpy().astype(bool), keep_ref)
    assert np.array_equal(idx.cpu().numpy(), idx_ref)
    print(f"mask filter: {idx_ref.size} of {N} kept, identical", flush=True)


def test_segmentation_end_to_end(gsc_mod):
    """Masks colorized at L = 0 (the multi-scene segmentation workload's kind,
    16 mask channels, BF16 targets) and filtered at 0.6 on the GPU, against
    the oracle's colorize + filter.  The keep decisions agree for every
    Gaussian whose oracle mask value lies farther from the threshold than the
    coefficient parity gate allows it to move; the rest may go either way."""
    import torch
    sc = syn.make_segment_scene(2, n_override=20000, cams_override=10)
    print(f"[case] segmentation N={sc.N} cams={len(sc.cams)} {sc.cams[0].width}x{sc.cams[0].height}",
          flush=True)
    y = oracle.make_targets(sc)
    ref = oracle.colorize(sc, y)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    ctx = gsc_mod.Context()
    c, st = ctx.colorize(m, s, q, o, sc.cams, parity.to_device_targets(y), sc.sh_deg, list(sc.lam))
    torch.cuda.synchronize()
    cg, sg = c.cpu().numpy(), st.cpu().numpy()
    parity.check_colorize(cg, sg, ref, label="segment 20k L0 C16")
    y0 = float(oracle.sh_basis(0, np.array([[0.0, 0.0, 1.0]]))[0, 0])
    scale, _ = parity.norms(ref)
    slack = y0 * (parity.TOL_F32 + parity.bound(ref)) * scale + 1e-6
    sure = ref["ndec"] == 0
    n_amb = 0
    for ch in range(sc.C):
        keep, idx = ctx.mask_filter(c, ch, 0.6, st)
        torch.cuda.synchronize()
        keep = keep.cpu().numpy().astype(bool)
        keep_ref, _ = oracle.mask_filter(ref["coeffs"], ch, 0.6, ref["status"])
        v = oracle.mask_value(ref["coeffs"], ch).astype(np.float64)
        clear = (np.abs(v - 0.6) > slack) & sure
        n_amb += int((~clear).sum())
        assert np.array_equal(keep[clear], keep_ref[clear]), f"channel {ch}"
        assert np.array_equal(idx.cpu().numpy(), np.flatnonzero(keep))
    print(f"segmentation: keep sets identical on all clear decisions ({n_amb} of "
          f"{sc.N * sc.C} (Gaussian, channel) pairs left open)", flush=True)
