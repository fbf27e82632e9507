"""Statistical and invariant pins of the oracle's equilibrium runs.

* With lnW = 0 the energy histogram samples Omega(E) (Sec. 2, eq. (1) with
  W = 1).
* With lnW = -beta E the run is canonical; <E> matches the exact value
  from the enumerated Omega (the micromagnetic comparison of Sec. 4 in
  miniature: fixed particle number Metropolis at one temperature).
* With W = 1/Omega the histogram is flat (Sec. 2).
* The whole iteration (Sec. 2), started from flat weights, estimates
  ln Omega within 0.02 of the exact enumeration on L = 4 lattices.
* Invariants: particle number, particle list, incremental energy,
  histogram total = walkers x sweeps; splitting the walkers over two
  contexts (the paper's processes) sums to the same histogram (eq. (2)).
"""
import math

import numpy as np
import pytest

import oracle as O


def _exact(d, L, N):
    om = O.brute_dos(d, L, N)
    lo = min(om)
    return lo, np.array([om.get(E, 0) for E in range(lo, 1)], dtype=np.float64)


def _grouped(d, L, N, lo, ngroups, walkers, seed):
    return O.RefContext([(d, L, N, walkers, lo, 0)] * ngroups, seed=seed)


def _group_fractions(ctx, H, nb):
    return np.array([H[ctx.bin_offset(g):ctx.bin_offset(g) + nb] for g in range(ctx.ngroups)],
                    dtype=np.float64)


@pytest.mark.parametrize("d,L,N", [(2, 4, 5), (2, 4, 7), (3, 4, 3)])
def test_flat_weights_sample_density_of_states(d, L, N):
    lo, om = _exact(d, L, N)
    nb = len(om)
    ctx = _grouped(d, L, N, lo, 16, 4, seed=11)
    H = ctx.sweep(np.zeros(ctx.total_bins), 1500)
    f = _group_fractions(ctx, H, nb)
    f /= f.sum(axis=1, keepdims=True)
    mean, se = f.mean(axis=0), f.std(axis=0, ddof=1) / math.sqrt(f.shape[0])
    p = om / om.sum()
    assert np.all(np.abs(mean - p) <= 5 * se + 1e-12), (mean, p, se)
    assert np.all(mean[om == 0] == 0)  # unreachable energies never appear


@pytest.mark.parametrize("d,L,N,beta", [(2, 4, 6, 0.8), (3, 4, 4, 1.2), (2, 5, 6, 1.5)])
def test_canonical_weights_mean_energy(d, L, N, beta):
    lo, om = _exact(d, L, N)
    E = np.arange(lo, 1, dtype=np.float64)
    w = om * np.exp(-beta * (E - E.max()))
    exact = (E * w).sum() / w.sum()
    nb = len(om)
    ctx = _grouped(d, L, N, lo, 16, 4, seed=12)
    lnW = np.tile(-beta * E, ctx.ngroups)
    H = ctx.sweep(lnW, 1500)
    f = _group_fractions(ctx, H, nb)
    means = (f * E).sum(axis=1) / f.sum(axis=1)
    se = means.std(ddof=1) / math.sqrt(len(means))
    assert abs(means.mean() - exact) <= 5 * se, (means.mean(), exact, se)


def test_inverse_dos_weights_give_flat_histogram():
    lo, om = _exact(2, 4, 6)
    nb = len(om)
    ctx = _grouped(2, 4, 6, lo, 16, 4, seed=13)
    lnW = np.tile(-np.log(om), ctx.ngroups)
    H = ctx.sweep(lnW, 1500)
    f = _group_fractions(ctx, H, nb)
    f /= f.sum(axis=1, keepdims=True)
    mean, se = f.mean(axis=0), f.std(axis=0, ddof=1) / math.sqrt(f.shape[0])
    assert np.all(np.abs(mean - 1.0 / nb) <= 5 * se), (mean, se)
    assert ctx.flat(H).all()


CASES_L4 = [(2, 2, 0), (2, 3, 0), (2, 4, 0), (2, 5, 0), (2, 6, 0), (2, 7, 1), (2, 8, 1),
            (3, 2, 0), (3, 3, 0), (3, 4, 0), (3, 5, 0)]


@pytest.mark.slow
@pytest.mark.parametrize("d,N,rule", CASES_L4)
def test_muca_iteration_recovers_exact_dos_L4(d, N, rule):
    # rule 1 (simple) where the spectrum has gaps: the pair recursion cannot
    # bridge an unreachable energy.
    lo, om = _exact(d, 4, N)
    nb = len(om)
    ctx = O.RefContext([(d, 4, N, 64, lo, 0)], seed=21)
    lnW = np.zeros(nb)
    P = np.zeros(nb)
    status, H, iters, flat = ctx.run(lnW, P, sweeps=200, max_iters=60, rule=rule,
                                     stop_on_flat=True)
    assert status == 0 and flat[0] == 1
    # production run with the converged weights
    sweeps = 12000 if d == 2 else 3000
    H = ctx.sweep(lnW, sweeps)
    assert H.sum() == 64 * sweeps
    seen = H > 0
    assert np.array_equal(seen, om > 0)
    ln_est = np.log(H[seen]) - lnW[seen]
    ln_est += math.log(math.comb(4 ** d, N)) - np.logaddexp.reduce(ln_est)
    err = np.abs(ln_est - np.log(om[seen]))
    assert err.max() < 0.02, (err, iters)


@pytest.mark.parametrize("groups", [
    [(2, 8, 16, 8)],
    [(3, 5, 12, 4), (2, 6, 3, 3)],
    [(2, 9, 20, 5, -30, -2)],
])
def test_invariants_under_random_weights(groups):
    ctx = O.RefContext(groups, seed=3)
    rng = np.random.default_rng(4)
    lnW = rng.normal(0.0, 2.0, ctx.total_bins)
    sweeps = 37
    H = ctx.sweep(lnW, sweeps)
    w = 0
    for gi, g in enumerate(groups):
        d, L, N, walkers = g[:4]
        lo, hi = ctx.window(gi)
        off, nb = ctx.bin_offset(gi), hi - lo + 1
        assert H[off:off + nb].sum() == walkers * sweeps
        for _ in range(walkers):
            n, pos, E, t = ctx.walker(w)
            assert n.sum() == N
            assert len(set(pos.tolist())) == N and np.all(n[pos] == 1)
            assert E == ctx.recount(w)
            assert lo <= E <= hi
            assert t == sweeps * L ** d
            w += 1


def test_single_particle_has_zero_energy():
    ctx = O.RefContext([(3, 5, 1, 3)], seed=9)
    assert ctx.window(0) == (0, 0)
    H = ctx.sweep(np.zeros(1), 10)
    assert H.tolist() == [30]


def test_walkers_split_over_processes_sum_to_same_histogram():
    # eq. (2): H^i = sum_j H^i_j over independent processes with identical W^i
    rng = np.random.default_rng(10)
    full = O.RefContext([(2, 8, 16, 12)], seed=5)
    a = O.RefContext([(2, 8, 16, 5)], seed=5, first_id=0)
    b = O.RefContext([(2, 8, 16, 7)], seed=5, first_id=5)
    lnW = rng.normal(0, 1.5, full.total_bins)
    Hf = full.sweep(lnW, 50)
    Ha = a.sweep(lnW, 50)
    Hb = b.sweep(lnW, 50)
    assert np.array_equal(Hf, Ha + Hb)
    for w in range(12):
        src, j = (a, w) if w < 5 else (b, w - 5)
        for x, y in zip(full.walker(w), src.walker(j)):
            assert np.array_equal(x, y)


def test_invalid_groups_are_rejected():
    for g in [(1, 8, 4, 1), (2, 2, 2, 1), (2, 8, 0, 1), (2, 8, 4, 0), (2, 8, 40, 1),
              (2, 8, 4, 1, -9, 0), (2, 8, 4, 1, -2, 1), (2, 8, 4, 1, -1, -2)]:
        with pytest.raises(ValueError):
            O.RefContext([g], seed=1)
