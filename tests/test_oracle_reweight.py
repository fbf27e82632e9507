"""Pins of the oracle's canonical reweighting (the step after the weight
iteration: Sec. 3 reweights the multicanonical data to the temperatures of
interest).

* Against canonical averages summed directly over every configuration of
  small lattices (energies counted here with an adjacency built from
  np.roll; no density of states involved), from a flat multicanonical
  histogram H = const with lnW = -ln Omega: ln Z, <E>, <E^2> and the
  specific heat at several beta.
* Closed form: two particles on the 4 x 4 torus at beta = 0 have
  <E> = -32/120 (32 of the 120 pairs of sites are neighbours).
* Limits: large beta gives the ground-state energy and C -> 0; unvisited
  bins carry no weight; no visited bin gives NaN.
* From a converged oracle run with a production histogram, <E> at beta = 0.5
  is within the statistical error of the exact value.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle.droplet_ref import largest_cluster
from oracle.reweight_ref import reweight, reweight_observable


def _config_energies(d, L, N):
    V = L ** d
    idx = np.arange(V).reshape((L,) * d)
    pairs = set()
    for a in range(d):
        nb = np.roll(idx, -1, axis=a).ravel()
        for s, t in zip(idx.ravel(), nb):
            pairs.add((min(s, t), max(s, t)))
    adj = np.zeros((V, V), dtype=np.int64)
    for s, t in pairs:
        adj[s, t] = adj[t, s] = 1
    out = []
    for c in itertools.combinations(range(V), N):
        c = np.array(c)
        out.append(-int(adj[np.ix_(c, c)].sum()) // 2)
    return np.array(out, dtype=np.float64)


def _direct(Es, beta):
    a = -beta * Es
    m = a.max()
    w = np.exp(a - m)
    z = w.sum()
    mean = (w * Es).sum() / z
    return (m + math.log(z), mean, (w * Es * Es).sum() / z,
            beta * beta * (w * (Es - mean) ** 2).sum() / z)


@pytest.mark.parametrize("d,L,N", [(2, 4, 3), (2, 4, 5), (3, 3, 4)])
def test_flat_histogram_gives_direct_canonical_sums(d, L, N):
    Es = _config_energies(d, L, N)
    e_lo = int(Es.min())
    counts = np.array([(Es == e).sum() for e in range(e_lo, 1)], dtype=np.float64)
    lnW = np.where(counts > 0, -np.log(np.maximum(counts, 1)), 0.0)
    H = np.where(counts > 0, 1000, 0)
    betas = [0.0, 0.5, 1.0, 2.0, 4.0]
    out = reweight(lnW, H, e_lo, betas)
    for k, beta in enumerate(betas):
        lz, mean, sq, c = _direct(Es, beta)
        assert out[k, 0] - math.log(1000) == pytest.approx(lz, rel=1e-12, abs=1e-12)
        assert out[k, 1] == pytest.approx(mean, rel=1e-12, abs=1e-12)
        assert out[k, 2] == pytest.approx(sq, rel=1e-12, abs=1e-12)
        assert out[k, 3] == pytest.approx(c, rel=1e-10, abs=1e-12)


def test_two_particles_infinite_temperature():
    # lnW = 0 and H proportional to Omega: Omega(-1) = 32, Omega(0) = 88
    out = reweight([0.0, 0.0], [32, 88], -1, [0.0])
    assert out[0, 1] == pytest.approx(-32 / 120, rel=1e-15)
    assert out[0, 0] == pytest.approx(math.log(120), rel=1e-15)


def test_limits_and_unvisited_bins():
    H = np.array([5, 0, 7, 9, 0, 11])
    lnW = np.array([0.3, 9.0, -1.2, 0.4, -7.0, 0.0])
    out = reweight(lnW, H, -5, [50.0, 0.0])
    assert out[0, 1] == pytest.approx(-5.0, abs=1e-12) and out[0, 3] < 1e-12
    # the unvisited bins (E = -4, -1) must not count, whatever their lnW
    w = H[[0, 2, 3, 5]] * np.exp(-lnW[[0, 2, 3, 5]])
    E = np.array([-5, -3, -2, 0])
    assert out[1, 1] == pytest.approx((w * E).sum() / w.sum(), rel=1e-14)
    assert np.isnan(reweight(lnW, np.zeros(6, dtype=int), -5, [1.0])).all()


def test_reweighted_iteration_matches_exact():
    d, L, N = 2, 4, 5
    Es = _config_energies(d, L, N)
    e_lo = int(Es.min())
    ctx = O.RefContext([(d, L, N, 64, e_lo, 0)], seed=21)
    lnW, P = np.zeros(-e_lo + 1), np.zeros(-e_lo + 1)
    status, H, iters, flat = ctx.run(lnW, P, sweeps=200, max_iters=60, rule=0, stop_on_flat=True)
    assert status == 0
    H = ctx.sweep(lnW, 6000)
    out = reweight(lnW, H, e_lo, [0.5])
    exact = _direct(Es, 0.5)[1]
    assert abs(out[0, 1] - exact) < 0.02 * abs(e_lo), (out[0, 1], exact)


def test_observable_reweighting_against_direct_sums():
    """<largest droplet>_beta over every configuration of 2D L = 4, N = 5
    (direct canonical sums) equals the reweighting of a flat histogram whose
    per-bin observable sums hold the exact microcanonical means."""
    d, L, N = 2, 4, 5
    V = L ** d
    Ls = []
    for c in itertools.combinations(range(V), N):
        occ = np.zeros(V, dtype=np.uint8)
        occ[list(c)] = 1
        Ls.append(largest_cluster(occ, d, L))
    Es = _config_energies(d, L, N)
    Ls = np.array(Ls, dtype=np.float64)
    e_lo = int(Es.min())
    bins = np.arange(e_lo, 1)
    counts = np.array([(Es == e).sum() for e in bins], dtype=np.float64)
    micro = np.array([Ls[Es == e].mean() if (Es == e).any() else 0.0 for e in bins])
    H = np.where(counts > 0, 500, 0)
    lnW = np.where(counts > 0, -np.log(np.maximum(counts, 1)), 0.0)
    Osum = micro * H
    betas = [0.0, 0.7, 1.5, 3.0]
    got = reweight_observable(lnW, H, Osum, e_lo, betas)
    for k, beta in enumerate(betas):
        w = np.exp(-beta * (Es - Es.min()))
        assert got[k] == pytest.approx((w * Ls).sum() / w.sum(), rel=1e-12)
    # O = E reproduces <E> of reweight()
    np.testing.assert_allclose(reweight_observable(lnW, H, bins * H, e_lo, betas),
                               reweight(lnW, H, e_lo, betas)[:, 1], rtol=1e-13)
