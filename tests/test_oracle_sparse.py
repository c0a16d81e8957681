"""The oracle's restricted forms used at full workload sizes: a render of
listed target rows and a colorize restricted to sampled Gaussians, fed with
targets known only at the rows those Gaussians read.  Both must reproduce
the unrestricted oracle exactly (same arithmetic in the same order)."""
import numpy as np

import oracle
from paper_2604_17155_amd import synthetic as syn


def _scene():
    sc = syn.make_segment_scene(2, n_override=3000, cams_override=5)
    sc.cams = syn.hemisphere_cams(5, 3.0, 96, 72)
    return sc


def test_render_rows_equals_full_render():
    sc = syn.make_relight(n=2000, n_cams=4, res=64)
    full = oracle.render(sc, sc.gt[0])
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(sc.n_pixels, 3000, replace=False))
    part = oracle.render_rows(sc, sc.gt[0], rows)
    assert np.array_equal(part, full[rows])


def test_restricted_colorize_on_sparse_targets():
    sc = _scene()
    y = oracle.make_targets(sc)
    rng = np.random.default_rng(1)
    want = np.zeros(sc.N, np.uint8)
    want[rng.choice(sc.N, 40, replace=False)] = 1
    rows = oracle.wanted_rows(sc, want)
    assert 0 < rows.size < sc.n_pixels and np.all(np.diff(rows) > 0)
    ysp, vals = oracle.sparse_targets(sc, rows)
    assert np.array_equal(vals, y[rows])        # the same targets where they are read
    a = oracle.colorize(sc, y, want=want)
    b = oracle.colorize(sc, ysp, want=want)
    sel = want.astype(bool)
    for k in ("coeffs", "w", "flip"):
        assert np.array_equal(a[k][sel], b[k][sel]), k
    assert np.array_equal(a["cnt"][sel], b["cnt"][sel]) and a["count"] == b["count"]
    # and the restricted colorize equals the unrestricted one on the sample
    c = oracle.colorize(sc, y)
    assert np.allclose(c["coeffs"][sel], a["coeffs"][sel], rtol=1e-12, atol=1e-14)
    assert np.array_equal(c["cnt"][sel], a["cnt"][sel])
