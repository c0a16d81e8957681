"""Pins of the oracle's near-threshold bounds.

The oracle records every footprint, alpha-floor and stop decision that an
implementation evaluating q, alpha and T in binary32 might take the other way
(margins derived from the arithmetic, oracle.Options), and bounds per
Gaussian the coefficient change such decisions can cause (`flip`), counts the
decisions on each Gaussian's own acceptance (`ndec`), and bounds per pixel
the change of a render.

An implementation that decides differently within the margins is emulated by
the oracle itself with its thresholds moved inside them: alpha_min,
sigma_cut^2 and t_min scaled by (1 +- 0.9 eps) flip exactly the decisions
whose relative distance to the threshold is below 0.9 eps, all of which the
margins cover.  The margins are scaled up here so that a small scene has
hundreds of such decisions.  Every combination of signs must then move
  - every Gaussian's coefficients by at most its `flip` bound,
  - its contribution count by at most `ndec`, and not at all where ndec = 0,
  - every render pixel by at most its bound.
A bound that dropped a term (the rescaling of later weights, the
continuation past a stop, the second-order factor) fails these checks.
"""
import dataclasses
import itertools

import numpy as np
import pytest

import oracle
from tests import tiny

SCALE = 2000.0  # margins x SCALE: decisions within ~1e-3 relative of a threshold


def _scene(sh_deg=2, seed=3):
    sc = tiny.random_scene(seed, n=160, n_cams=5, res=40, sh_deg=sh_deg, C=3, aniso=True,
                           log_scale=-2.4)
    return sc


def _nudged(base: oracle.Options, sa, sq, st):
    """Thresholds moved by 0.9 of their smallest margins, in the given directions;
    returns the options and the relative moves actually made (binary32)."""
    f32 = np.float32
    da = 0.9 * base.eps_a
    dq = 0.9 * base.eps_q
    dt = 0.9 * base.eps_t
    amin = float(f32(base.alpha_min * (1 + sa * da)))
    cut = float(f32(base.sigma_cut * np.sqrt(1 + sq * dq)))
    tmin = float(f32(base.t_min * (1 + st * dt)))
    moves = (abs(amin / base.alpha_min - 1), abs((cut / base.sigma_cut) ** 2 - 1), abs(tmin / base.t_min - 1))
    return dataclasses.replace(base, alpha_min=amin, sigma_cut=cut, t_min=tmin), moves, (da, dq, dt)


@pytest.mark.parametrize("sh_deg", [0, 2])
def test_flip_bounds_threshold_moves(sh_deg):
    sc = _scene(sh_deg)
    y = oracle.make_targets(sc)
    base = oracle.Options().scaled_margins(SCALE)
    ref = oracle.colorize(sc, y, opts=base)
    obs = (ref["status"] & 1) == 0
    assert ref["events"] > 50, ref["events"]
    nrm = np.linalg.norm(ref["coeffs"].reshape(sc.N, -1), axis=1)
    changed = 0
    for sa, sq, st in itertools.product((-1, 1), repeat=3):
        opts, moves, lim = _nudged(base, sa, sq, st)
        assert all(m <= l * 1.0001 for m, l in zip(moves, lim)), (moves, lim)
        alt = oracle.colorize(sc, y, opts=opts)
        d = np.linalg.norm((alt["coeffs"] - ref["coeffs"]).reshape(sc.N, -1), axis=1)
        changed += int((d > 1e-12 * np.maximum(nrm, 1e-12)).sum())
        # coefficient change within the bound (FP64 summation-order slack)
        slack = 1e-10 * np.maximum(nrm, 1.0)
        bad = obs & ~(d <= ref["flip"] + slack)
        assert not bad.any(), (sa, sq, st, np.flatnonzero(bad)[:5], d[bad][:5], ref["flip"][bad][:5])
        # the unobserved set can only change where a decision was recorded
        un_b, un_a = (ref["status"] & 1) == 1, (alt["status"] & 1) == 1
        assert np.all((un_b == un_a) | (ref["ndec"] > 0))
        # contribution counts: exact without decisions, within ndec otherwise
        dc = np.abs(alt["cnt"] - ref["cnt"])
        assert np.all(dc <= ref["ndec"]), np.flatnonzero(dc > ref["ndec"])[:5]
        assert abs(alt["count"] - ref["count"]) <= ref["events"]
    assert changed > 20, "the threshold moves flipped too few decisions to test the bound"


def test_render_pixel_bound_threshold_moves():
    sc = _scene(2, seed=5)
    base = oracle.Options().scaled_margins(SCALE)
    coeffs = sc.gt[0]
    img, bound = oracle.render(sc, coeffs, opts=base, with_bound=True)
    assert (bound > 0).sum() > 50
    moved = 0
    for sa, sq, st in itertools.product((-1, 1), repeat=3):
        opts, _, _ = _nudged(base, sa, sq, st)
        alt = oracle.render(sc, coeffs, opts=opts)
        d = np.abs(alt - img).max(axis=1)
        moved += int((d > 1e-13).sum())
        assert np.all(d <= bound + 1e-12), np.flatnonzero(d > bound + 1e-12)[:5]
        # pixels without events render identically
        assert np.all(d[bound == 0] <= 1e-13)
    assert moved > 20


def test_no_events_without_margins():
    """With zero margins no decision is recorded: the bound vanishes and the
    result is the unique one."""
    sc = _scene(2, seed=7)
    y = oracle.make_targets(sc)
    z = dataclasses.replace(oracle.Options(), eps_q=0, eps_a=0, eps_t=0, eps_p=0, eps_cov=0)
    ref = oracle.colorize(sc, y, opts=z)
    assert ref["events"] == 0 and np.all(ref["flip"] == 0) and np.all(ref["ndec"] == 0)
    img, bound = oracle.render(sc, sc.gt[0], opts=z, with_bound=True)
    assert np.all(bound == 0)


def test_default_margins_are_small():
    """The default (binary32) margins flag few decisions: on the reduced
    relighting workload fewer than 1% of the observed Gaussians have a bound
    above half the 1e-4 gate."""
    from paper_2604_17155_amd import synthetic as syn
    sc = syn.make_relight(n=20000, n_cams=16, res=256)
    y = oracle.make_targets(sc)
    ref = oracle.colorize(sc, y)
    obs = (ref["status"] & 1) == 0
    nrm = np.linalg.norm(ref["coeffs"].reshape(sc.N, -1), axis=1)
    tau = 1e-3 * np.median(nrm[obs])
    frac = float((obs & (ref["flip"] > 0.5e-4 * np.maximum(nrm, tau))).sum() / obs.sum())
    assert frac < 0.01, frac
