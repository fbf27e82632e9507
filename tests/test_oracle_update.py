"""Pins of the oracle's weight recursion and flatness test.

Paper Sec. 2: the simple recursion W^{i+1}(E) = W^i(E) / H^i(E), and the
recursive scheme used by the authors (reading: Berg's error-weighted
recursion, in which the slope of lnW between neighbouring bins is the
p-weighted mean of the estimates of all iterations so far,
p = H(b) H(b+1) / (H(b) + H(b+1))).
"""
import math

import numpy as np
import pytest

import oracle as O


def _ctx_bins(nb):
    # one walker, 32 particles on a 64 x 64 lattice, window [-(nb-1), 0]
    return O.RefContext([(2, 64, 32, 1, -(nb - 1), 0)], seed=1)


def test_one_step_from_exact_histogram_gives_inverse_dos():
    # H = Omega (the expected histogram of lnW = 0 up to a factor) must give
    # lnW = -ln Omega + const, by both rules (W = 1/Omega, Sec. 2).
    om = O.brute_dos(2, 4, 6)
    E_lo = min(om)
    H = np.array([om[E] for E in range(E_lo, 1)], dtype=np.int32)
    ctx = O.RefContext([(2, 4, 6, 1, E_lo, 0)], seed=1)
    want = -np.log(H.astype(np.float64))
    want -= want[-1]
    for rule in (0, 1):
        lnW = np.zeros(len(H))
        P = np.zeros(len(H))
        ctx.update(H, lnW, P, rule=rule)
        assert lnW[-1] == 0.0
        np.testing.assert_allclose(lnW, want, rtol=0, atol=1e-12)


def test_constant_histogram_is_a_fixed_point():
    ctx = _ctx_bins(30)
    rng = np.random.default_rng(5)
    lnW0 = np.cumsum(rng.normal(0, 2, 30))
    lnW0 -= lnW0[-1]
    for rule in (0, 1):
        lnW = lnW0.copy()
        P = np.zeros(30)
        ctx.update(np.full(30, 777, dtype=np.int32), lnW, P, rule=rule)
        np.testing.assert_allclose(lnW, lnW0, rtol=0, atol=1e-12)


def test_simple_rule_definition():
    ctx = _ctx_bins(20)
    rng = np.random.default_rng(6)
    lnW = rng.normal(0, 3, 20)
    H = rng.integers(0, 5000, 20).astype(np.int32)
    H[[0, 7]] = 0
    want = lnW - np.log(np.maximum(H, 1))
    want -= want[-1]
    P = np.zeros(20)
    ctx.update(H, lnW, P, rule=1)
    np.testing.assert_allclose(lnW, want, rtol=0, atol=1e-12)


def test_berg_first_step_equals_simple_rule_when_all_bins_visited():
    ctx = _ctx_bins(25)
    rng = np.random.default_rng(7)
    H = rng.integers(1, 10**6, 25).astype(np.int32)
    lnW0 = rng.normal(0, 3, 25)
    a, b = lnW0.copy(), lnW0.copy()
    ctx.update(H, a, np.zeros(25), rule=0)
    ctx.update(H, b, np.zeros(25), rule=1)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)


def test_berg_two_steps_is_weighted_mean_of_estimates():
    nb = 18
    ctx = _ctx_bins(nb)
    rng = np.random.default_rng(8)
    H1 = rng.integers(1, 5000, nb).astype(np.int32)
    H2 = rng.integers(1, 5000, nb).astype(np.int32)
    lnW = rng.normal(0, 1, nb)
    d0 = np.diff(lnW)
    P = np.zeros(nb)
    ctx.update(H1, lnW, P, rule=0)
    d1 = np.diff(lnW)
    ctx.update(H2, lnW, P, rule=0)
    d2 = np.diff(lnW)
    h1, h2 = H1.astype(float), H2.astype(float)
    p1 = h1[:-1] * h1[1:] / (h1[:-1] + h1[1:])
    p2 = h2[:-1] * h2[1:] / (h2[:-1] + h2[1:])
    e1 = d0 + np.log(h1[:-1] / h1[1:])
    e2 = d1 + np.log(h2[:-1] / h2[1:])
    np.testing.assert_allclose(d1, e1, atol=1e-10)
    np.testing.assert_allclose(d2, (p1 * e1 + p2 * e2) / (p1 + p2), atol=1e-10)
    np.testing.assert_allclose(P[:-1], p1 + p2, rtol=1e-15)


def test_berg_frontier_slopes_are_copied():
    # reading: never-estimated pairs beyond the estimated range take the
    # slope of the nearest estimated pair, so the walk is pushed outward.
    nb = 16
    ctx = _ctx_bins(nb)
    H = np.zeros(nb, dtype=np.int32)
    H[5:11] = [10, 40, 90, 160, 250, 360]
    lnW = np.zeros(nb)
    P = np.zeros(nb)
    ctx.update(H, lnW, P, rule=0)
    d = np.diff(lnW)
    for b in range(5, 10):
        assert d[b] == pytest.approx(math.log(H[b] / H[b + 1]), abs=1e-12)
    assert np.all(d[:5] == d[5])
    assert np.all(d[10:] == d[9])
    assert np.all(P[:5] == 0) and np.all(P[10:] == 0) and np.all(P[5:10] > 0)


def test_berg_interior_gap_keeps_slope():
    nb = 12
    ctx = _ctx_bins(nb)
    H = np.array([5, 6, 7, 0, 9, 10, 11, 12, 13, 14, 15, 16], dtype=np.int32)
    lnW = np.linspace(3.0, 0.0, nb)
    d_before = np.diff(lnW)
    P = np.zeros(nb)
    ctx.update(H, lnW, P, rule=0)
    d = np.diff(lnW)
    assert d[2] == pytest.approx(d_before[2], abs=1e-12)
    assert d[3] == pytest.approx(d_before[3], abs=1e-12)
    assert P[2] == 0 and P[3] == 0


@pytest.mark.parametrize("H,flat", [
    ([5, 5, 5, 5], 1),
    ([5, 9, 5, 5], 1),
    ([5, 10, 5, 5], 0),     # 2 min == max is not flat
    ([0, 5, 5, 5], 0),      # lower end unvisited
    ([5, 5, 5, 0], 0),      # upper end unvisited
    ([5, 0, 6, 5], 1),      # interior gap ignored
    ([1, 0, 0, 1], 1),
])
def test_flatness(H, flat):
    ctx = _ctx_bins(4)
    assert ctx.flat(np.array(H, dtype=np.int32))[0] == flat
