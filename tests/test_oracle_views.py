"""Pins of the oracle's view selection (Sec. 5: fewer camera images, chosen
by visibility): the greedy maximum-coverage rule against brute force over
every k-subset on tiny cases (greedy reaches at least (1 - 1/e) of the optimum,
and the optimum exactly where sets nest), and the objective's special cases."""
import itertools
import math

import numpy as np
import pytest

import oracle
from tests import tiny


def _brute(seen, k, R):
    return max(oracle.coverage(seen, list(c), R) for c in itertools.combinations(range(seen.shape[0]), k))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("R", [1, 2, 3])
def test_greedy_against_brute_force(seed, R):
    rng = np.random.default_rng(seed)
    seen = rng.random((7, 40)) < rng.uniform(0.1, 0.6, size=(7, 1))
    for k in (1, 2, 3, 4):
        views, obj = oracle.select_views(seen, k, R)
        assert len(set(views)) == k
        assert obj == oracle.coverage(seen, views, R)
        opt = _brute(seen, k, R)
        assert obj >= (1 - 1 / math.e) * opt - 1e-9
        if k == 1:
            assert obj == opt  # one pick is the best single view


def test_greedy_special_cases():
    # nested sets: the greedy picks the largest first and is optimal
    seen = np.zeros((4, 10), bool)
    for j, n in enumerate([3, 10, 6, 1]):
        seen[j, :n] = True
    views, obj = oracle.select_views(seen, 2, 1)
    assert views[0] == 1 and obj == 10
    # disjoint sets: picks in order of size, ties to the lower index
    seen = np.zeros((4, 12), bool)
    seen[0, 0:3] = seen[1, 3:8] = seen[2, 8:11] = seen[3, 11:12] = True
    views, obj = oracle.select_views(seen, 3, 1)
    assert views == [1, 0, 2] and obj == 11
    # every view, multiplicity above the view count: the objective counts every observed pair
    rng = np.random.default_rng(9)
    seen = rng.random((5, 30)) < 0.4
    views, obj = oracle.select_views(seen, 5, 99)
    assert sorted(views) == list(range(5)) and obj == int(seen.sum())


def test_observed_pairs_match_visibility(oracle_lib):
    """A view observes exactly the Gaussians to which it gives weight."""
    sc = tiny.random_scene(91, n=30, n_cams=4, res=20, sh_deg=0, C=1)
    seen = oracle.observed_pairs(sc)
    idx, w = oracle.contributions(sc)
    for j in range(len(sc.cams)):
        V = np.zeros(sc.N)
        sel = idx[:, 0] == j
        np.add.at(V, idx[sel, 2], w[sel])
        assert np.array_equal(seen[j], V > 0)
