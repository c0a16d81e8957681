"""View selection on the GPU (gsc_select_views; Sec. 5: fewer camera images,
chosen by visibility).

Parity: the chosen views against the oracle's greedy on the oracle's own
observation sets.  Observation is an integer decision per (view, Gaussian);
only Gaussians with near-threshold decisions (ndec > 0) may be observed
differently, so the lists agree when there are none, and otherwise the
objectives differ by at most multiplicity times their number.

Measurement (printed): the relighting workload (100k Gaussians, 50 views
512^2, L = 3) colorized from selected subsets against all views."""
import time

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


def _wide_scene():
    """Gaussians spread over a box wider than any one view sees, twelve
    narrow cameras around it: every view observes a different part."""
    from tests import tiny
    rng = np.random.default_rng(95)
    n = 3000
    means = rng.uniform(-2.0, 2.0, (n, 3)).astype(np.float32)
    scales = np.repeat(np.exp(rng.normal(-3.0, 0.2, (n, 1))), 3, 1)
    cams = tiny.sphere_cams(12, radius=3.5, res=64, fov=35.0)
    return tiny.scene(means, scales, tiny.identity_quats(n), rng.uniform(0.3, 0.9, n), cams, sh_deg=0, C=3)


@pytest.mark.parametrize("k,R", [(1, 1), (4, 1), (6, 2), (8, 3)])
def test_select_views_parity(gsc_mod, k, R):
    sc = _wide_scene()
    print(f"[case] select views k={k} R={R}", flush=True)
    seen = oracle.observed_pairs(sc)
    ref_views, ref_obj = oracle.select_views(seen, k, R)
    ndec = oracle.colorize(sc, np.zeros((sc.n_pixels, 3), np.float32))["ndec"]
    m, s, q, o = gsc_mod.scene_tensors(sc)
    views, obj = gsc_mod.Context().select_views(m, s, q, o, sc.cams, k, R)
    amb = int((ndec > 0).sum())
    print(f"gpu {views} ({obj}), oracle {ref_views} ({ref_obj}); Gaussians with decisions in doubt: {amb}",
          flush=True)
    assert len(set(views)) == k
    if amb == 0:
        assert views == ref_views and obj == ref_obj
    else:
        assert abs(obj - ref_obj) <= R * amb
        assert oracle.coverage(seen, views, R) >= ref_obj - R * amb


def test_select_views_degenerate(gsc_mod):
    sc = syn.make_relight(seed_offset=96, n=500, n_cams=5, res=64)
    m, s, q, o = gsc_mod.scene_tensors(sc)
    ctx = gsc_mod.Context()
    assert ctx.select_views(m, s, q, o, sc.cams, 0) == ([], 0)
    views, obj = ctx.select_views(m, s, q, o, sc.cams, 5, 64)
    assert sorted(views) == list(range(5))
    seen = oracle.observed_pairs(sc)
    assert abs(obj - int(seen.sum())) <= 64 * int((oracle.colorize(
        sc, np.zeros((sc.n_pixels, 3), np.float32))["ndec"] > 0).sum())


def test_subset_colorize_measurement(gsc_mod):
    """Relighting from k selected views against all 50: time per colorize and
    the coefficient difference to the all-view solution (printed)."""
    import torch
    sc = syn.make_relight()
    m, s, q, o = gsc_mod.scene_tensors(sc)
    ctx = gsc_mod.Context()
    gt = torch.from_numpy(sc.gt[0].astype(np.float32)).cuda()
    y = ctx.render(m, s, q, o, sc.cams, gt)  # noise-free targets from the ground truth
    lam = list(sc.lam)

    def timed(cams, reps=5):
        ctx.colorize(m, s, q, o, cams, y, sc.sh_deg, lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c, st = ctx.colorize(m, s, q, o, cams, y, sc.sh_deg, lam)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3, c.cpu().numpy(), st.cpu().numpy()

    y_rms = float(torch.sqrt((y * y).mean()))

    def image_err(c):  # relative RMS error of the render over all 50 views
        img = ctx.render(m, s, q, o, sc.cams, torch.from_numpy(c).cuda())
        return float(torch.sqrt(((img - y) ** 2).mean())) / y_rms

    t_all, c_all, st_all = timed(sc.cams)
    obs_all = (st_all & 1) == 0
    nrm = np.linalg.norm(c_all.reshape(sc.N, -1), axis=1)
    print(f"all 50 views: {t_all:.2f} ms, {int(obs_all.sum())} observed, image error "
          f"{image_err(c_all):.4f}", flush=True)
    for k, R in [(25, 8), (12, 4), (6, 2), (-12, 0)]:
        if k < 0:  # every fourth view, for comparison with the greedy choice
            k = -k
            views = list(range(0, 50, 50 // k))[:k]
        else:
            views, obj = ctx.select_views(m, s, q, o, sc.cams, k, R)
        cams_k = [sc.cams[j] for j in sorted(views)]
        offsets = [int(np.sum([c.width * c.height for c in sc.cams[:j]])) for j in sorted(views)]
        ctx.colorize(m, s, q, o, cams_k, y, sc.sh_deg, lam, offsets=offsets)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            c, st = ctx.colorize(m, s, q, o, cams_k, y, sc.sh_deg, lam, offsets=offsets)
        torch.cuda.synchronize()
        t_k = (time.perf_counter() - t0) / 5 * 1e3
        c, st = c.cpu().numpy(), st.cpu().numpy()
        obs = obs_all & ((st & 1) == 0)
        e = np.linalg.norm((c - c_all).reshape(sc.N, -1), axis=1) / np.maximum(nrm, 1e-3 * np.median(nrm[obs_all]))
        print(f"k={k} R={R}: {t_k:.2f} ms ({t_all / t_k:.1f}x); observed {int(obs.sum())} of "
              f"{int(obs_all.sum())}; image error over all 50 views {image_err(c):.4f}; "
              f"coefficients vs all views p50 {np.median(e[obs]):.2e}", flush=True)
        assert t_k < t_all
