"""Pins of the oracle's tunnelling count (the convergence measure of Sec. 4:
trips of a walker from the top of the energy range to its bottom or back).

The count is restated here from its definition and applied to the energy
sequence at sweep ends, read one sweep at a time from a second oracle
context: a walker's first visit to a window end starts it, every later
visit to the other end completes one trip.  Also: invariants (trips never
exceed sweeps, a window of one bin never tunnels), and the run that stops
at a target number of tunnelling events stops at the first iteration that
reaches it.
"""
import numpy as np
import pytest

import oracle as O


def trips_from_energies(seq, lo, hi):
    """(last end, trips) of one walker from its energies at sweep ends."""
    last, trips = 0, 0
    for E in seq:
        end = 1 if E == lo else (2 if E == hi else 0)
        if end and end != last:
            trips += last != 0
            last = end
    return last, trips


@pytest.mark.parametrize("groups,sweeps", [
    ([(2, 4, 2, 6, -1, 0)], 40),            # two energies: every change is a trip
    ([(2, 4, 3, 5), (3, 3, 3, 4)], 30),     # default windows, 2D and 3D
    ([(2, 6, 5, 4, -4, -1)], 25),           # an explicit window inside the range
])
def test_trips_match_the_definition(groups, sweeps):
    lnW_rng = np.random.default_rng(3)
    a = O.RefContext(groups, seed=7)
    b = O.RefContext(groups, seed=7)
    lnW = lnW_rng.normal(0.0, 0.5, a.total_bins)
    a.sweep(lnW, sweeps)
    seqs = [[] for _ in range(b.nwalkers)]
    for _ in range(sweeps):
        b.sweep(lnW, 1)
        for w in range(b.nwalkers):
            seqs[w].append(b.walker(w)[2])
    last, trips = a.tunnel()
    first = 0
    for g, grp in enumerate(groups):
        lo, hi = a.window(g)
        for w in range(first, first + grp[3]):
            assert (last[w], trips[w]) == trips_from_energies(seqs[w], lo, hi), w
        first += grp[3]
    assert np.array_equal(b.tunnel()[1], trips)
    assert trips.max() <= sweeps - 1
    assert trips.sum() > 0  # the cases do tunnel


def test_two_energy_window_counts_changes():
    """Window [-1, 0] of two particles: every energy change between sweep
    ends is one trip."""
    a = O.RefContext([(2, 4, 2, 3, -1, 0)], seed=2)
    b = O.RefContext([(2, 4, 2, 3, -1, 0)], seed=2)
    a.sweep(np.zeros(2), 60)
    seq = [[] for _ in range(3)]
    for _ in range(60):
        b.sweep(np.zeros(2), 1)
        for w in range(3):
            seq[w].append(b.walker(w)[2])
    for w in range(3):
        changes = sum(1 for x, y in zip(seq[w], seq[w][1:]) if x != y)
        assert a.tunnel()[1][w] == changes


def test_single_bin_window_never_tunnels():
    a = O.RefContext([(2, 5, 1, 4)], seed=1)  # N = 1: E = 0 always
    assert a.window(0) == (0, 0)
    a.sweep(np.zeros(1), 20)
    last, trips = a.tunnel()
    assert (trips == 0).all() and (last == 1).all()


def test_run_stops_at_the_tunnelling_target():
    groups = [(2, 4, 3, 4), (2, 5, 4, 3)]
    target = 6
    a = O.RefContext(groups, seed=11)
    lnW, P = a.zeros_lnW(), a.zeros_lnW()
    rc, H, it, fl = a.run(lnW, P, 5, 200, 0, tunnel_target=target)
    assert rc == 0
    trips = a.tunnel()[1]
    first = 0
    for g, grp in enumerate(groups):
        assert trips[first:first + grp[3]].sum() >= target
        first += grp[3]
    # one iteration fewer (same weights up to then) has not reached it
    for g in range(len(groups)):
        if it[g] < 2:
            continue
        b = O.RefContext(groups, seed=11)
        lw, Pb = b.zeros_lnW(), b.zeros_lnW()
        b.run(lw, Pb, 5, int(it[g]) - 1, 0)
        tb = b.tunnel()[1]
        first = sum(x[3] for x in groups[:g])
        assert tb[first:first + groups[g][3]].sum() < target, g
