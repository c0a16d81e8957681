"""Pin of the incremental finite differences (tests/fdcheck.py) used at the
differentiation workload's full size: on a small scene of the same kind,
every incremental entry equals the brute-force central difference (full
oracle colorize + render at y1 +- h e and o_g +- h), and both equal the
oracle's adjoint gradient (itself pinned by dot-product and FD tests)."""
import numpy as np
import pytest

import oracle
from paper_2604_17155_amd import synthetic as syn
from tests import fdcheck

H = 1e-3


@pytest.fixture(scope="module")
def case(oracle_lib):
    sc = syn.make_diff(n=2000, n_cams=5, res=64)
    opts = oracle.Options(t_min=0.0)
    y1 = oracle.make_targets(sc, 0, opts=opts)
    y2 = oracle.make_targets(sc, 1, opts=opts)
    base = fdcheck.loss_and_parts(sc, y1, y2, opts)
    return sc, opts, y1, y2, base


def _loss(sc, y1, y2, opts):
    c = oracle.colorize(sc, y1, opts=opts)["coeffs"]
    img = oracle.render(sc, c, opts=opts)
    return float(((img - oracle.decode_targets(y2).astype(np.float64)) ** 2).mean())


def test_target_entries(case):
    sc, opts, y1, y2, base = case
    idx, _ = oracle.contributions(sc, opts)
    rng = np.random.default_rng(3)
    for row in rng.choice(np.unique(idx[:, 1]), 4, replace=False):
        ch = int(rng.integers(0, sc.C))
        inc = fdcheck.fd_target(base, int(row), ch, H)
        yp = y1.astype(np.float64).copy()
        ym = y1.astype(np.float64).copy()
        yp[row, ch] += H
        ym[row, ch] -= H
        brute = (_loss(sc, yp, y2, opts) - _loss(sc, ym, y2, opts)) / (2 * H)
        adj = float(base.grad_y[row, ch])
        assert abs(inc - brute) <= 1e-7 * abs(brute) + 1e-13, (row, inc, brute)
        assert abs(inc - adj) <= 1e-6 * abs(adj) + 1e-13, (row, inc, adj)


def test_opacity_entries(case):
    sc, opts, y1, y2, base = case
    obs = np.flatnonzero((base.w > 0) & (sc.opacities >= 0.40) & (sc.opacities <= 0.98))
    obs = obs[np.abs(base.grad_o[obs]) >= 1e-3 * np.abs(base.grad_o[obs]).max()]
    for g in np.random.default_rng(4).choice(obs, 6, replace=False):
        inc = fdcheck.fd_opacity(base, int(g), H)
        o0 = sc.opacities[g]
        op, om = np.float32(float(o0) + H), np.float32(float(o0) - H)
        sc.opacities[g] = op
        lp = _loss(sc, y1, y2, opts)
        sc.opacities[g] = om
        lm = _loss(sc, y1, y2, opts)
        sc.opacities[g] = o0
        brute = (lp - lm) / (float(op) - float(om))
        adj = float(base.grad_o[g])
        assert abs(inc - brute) <= 1e-6 * abs(brute) + 1e-12, (g, inc, brute)
        assert abs(inc - adj) <= 2e-5 * abs(adj) + 1e-12, (g, inc, adj)
