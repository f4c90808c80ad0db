"""Pins for the oracle's Gibbs-simplex projection (Gibbs-constraint section).

The oracle follows the paper's correction loop.  It is checked here against two
independent textbook routes to the same Euclidean projection:
  * the sort-based threshold of Held, Wolfe & Crowder (1974) / Duchi et al. (2008);
  * bisection on the threshold theta of x = max(y - theta, 0), sum x = 1;
and against the KKT conditions, idempotence, shift invariance, permutation
equivariance, the N = 2 closed form and the round bound of the paper (<= N).
"""
import numpy as np
import pytest


def proj_sort(y):
    """Held-Wolfe-Crowder: sort descending, find the largest k with a positive gap."""
    u = np.sort(y)[::-1]
    css = np.cumsum(u)
    k = np.arange(1, len(y) + 1)
    rho = np.nonzero(u - (css - 1.0) / k > 0)[0][-1]
    theta = (css[rho] - 1.0) / (rho + 1)
    return np.maximum(y - theta, 0.0)


def proj_bisect(y, iters=200):
    lo, hi = y.min() - 1.0, y.max()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.maximum(y - mid, 0.0).sum() > 1.0:
            lo = mid
        else:
            hi = mid
    return np.maximum(y - 0.5 * (lo + hi), 0.0)


def _cases(rng, count=3000):
    for _ in range(count):
        N = int(rng.integers(2, 9))
        scale = 10.0 ** rng.uniform(-2, 2)
        y = rng.normal(0.0, scale, N) + rng.uniform(-3, 3)
        yield y


def test_matches_sort_and_bisection(orc):
    rng = np.random.default_rng(1)
    worst = 0.0
    for y in _cases(rng):
        x, rounds = orc.project(y)
        xs = proj_sort(y)
        xb = proj_bisect(y)
        worst = max(worst, np.abs(x - xs).max())
        assert np.abs(x - xs).max() < 1e-12 * max(1.0, np.abs(y).max())
        assert np.abs(x - xb).max() < 1e-9 * max(1.0, np.abs(y).max())
        assert 1 <= rounds <= len(y)
    assert worst < 1e-10


def test_kkt_and_feasibility(orc):
    rng = np.random.default_rng(2)
    for y in _cases(rng, 1000):
        x, _ = orc.project(y)
        assert abs(x.sum() - 1.0) < 1e-12 * max(1.0, np.abs(y).max())
        assert (x >= 0).all()
        free = x > 0
        theta = (y[free] - x[free]).mean()
        # free components are shifted by one common theta, clamped ones lie below it
        assert np.allclose(y[free] - x[free], theta, atol=1e-11 * max(1.0, np.abs(y).max()))
        assert (y[~free] <= theta + 1e-11 * max(1.0, np.abs(y).max())).all()


def test_idempotent_and_shift_invariant(orc):
    rng = np.random.default_rng(3)
    for y in _cases(rng, 500):
        x, _ = orc.project(y)
        x2, r2 = orc.project(x)
        assert np.abs(x2 - x).max() < 1e-13
        assert r2 <= 2  # at most a round-off clean-up of exact zeros
        t = rng.normal() * 5
        xt, _ = orc.project(y + t)
        assert np.abs(xt - x).max() < 1e-11 * max(1.0, np.abs(y).max() + abs(t))


def test_permutation_equivariant(orc):
    rng = np.random.default_rng(4)
    for y in _cases(rng, 500):
        perm = rng.permutation(len(y))
        x, _ = orc.project(y)
        xp, _ = orc.project(y[perm])
        assert np.abs(xp - x[perm]).max() < 1e-13 * max(1.0, np.abs(y).max())


def test_two_phase_closed_form(orc):
    # on G^2 the projection of (y1, y2) is u1 = clamp((y1 - y2 + 1)/2, 0, 1)
    rng = np.random.default_rng(5)
    for _ in range(500):
        y = rng.normal(0, 2, 2)
        x, _ = orc.project(y)
        u1 = min(max((y[0] - y[1] + 1.0) / 2.0, 0.0), 1.0)
        assert abs(x[0] - u1) < 1e-14 and abs(x[1] - (1 - u1)) < 1e-14


def test_vertex_and_barycentre(orc):
    x, r = orc.project([10.0, 0.0, 0.0, 0.0])
    assert np.array_equal(x, [1.0, 0.0, 0.0, 0.0])
    x, r = orc.project([0.3, 0.3, 0.3])
    assert np.allclose(x, 1.0 / 3.0)
    assert r == 1


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_worst_case_round_count(orc, N):
    # a staircase forces one component out per round: N - 1 removals + the final check
    y = -np.arange(N, dtype=float) * 10.0
    x, r = orc.project(y)
    assert np.allclose(x, np.eye(N)[0], atol=1e-14)
    assert r <= N
