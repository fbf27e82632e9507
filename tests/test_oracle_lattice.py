"""Pins of the oracle's lattice gas: energies, densities of states, windows.

The lattice gas of the paper (Sec. 3, eq. (5)) with J = 1 has
E = -(number of occupied nearest-neighbour pairs) on a periodic square or
simple-cubic lattice.  The exact densities of states Omega_N(E) from the
oracle's enumeration are checked against an independent transfer-matrix
computation (2D), an enumeration over an adjacency matrix built with np.roll
(3D), closed forms for N <= 3 and particle-hole symmetry.  The default
window floor is checked against the Harary-Harborth maximum edge count in 2D,
the cube in 3D, and reachability by enumeration.
"""
import math

import numpy as np
import pytest

import oracle as O


# ---------------------------------------------------------------- transfer matrix
def _ring_bonds(mask, L):
    rot = ((mask << 1) | (mask >> (L - 1))) & ((1 << L) - 1)
    return bin(mask & rot).count("1")


def _layer_bonds_2d(mask, L):
    """Bonds inside an L x L periodic layer stored as L*L bits, x fastest."""
    b = 0
    for y in range(L):
        row = (mask >> (y * L)) & ((1 << L) - 1)
        b += _ring_bonds(row, L)
        nxt = (mask >> (((y + 1) % L) * L)) & ((1 << L) - 1)
        b += bin(row & nxt).count("1")
    return b


def transfer_dos(d, L):
    """Omega[N][P] (P = number of bonds) for all N by stacking slices along the
    last axis with periodic closure.  Slices are rows (2D) or layers (3D)."""
    ns = L ** (d - 1)
    S = 1 << ns
    inner = np.array([_ring_bonds(m, L) if d == 2 else _layer_bonds_2d(m, L)
                      for m in range(S)])
    pop = np.array([bin(m).count("1") for m in range(S)])
    V = L ** d
    maxP = d * V
    omega = np.zeros((V + 1, maxP + 1), dtype=object)
    for first in range(S):
        # dp[state] = dict (n, p) -> count, after placing slices 0..k
        dp = {first: {(pop[first], inner[first]): 1}}
        for _ in range(L - 1):
            nd = {}
            for st, poly in dp.items():
                for nx in range(S):
                    vb = bin(st & nx).count("1")
                    tgt = nd.setdefault(nx, {})
                    for (n, p), c in poly.items():
                        key = (n + pop[nx], p + inner[nx] + vb)
                        tgt[key] = tgt.get(key, 0) + c
            dp = nd
        for st, poly in dp.items():
            vb = bin(st & first).count("1")
            for (n, p), c in poly.items():
                omega[n, p + vb] += c
    return omega


@pytest.fixture(scope="module")
def tm_2d_L4():
    return transfer_dos(2, 4)


@pytest.mark.parametrize("N", range(0, 17))
def test_brute_dos_matches_transfer_matrix_2d_L4(tm_2d_L4, N):
    got = O.brute_dos(2, 4, N)
    want = {-p: int(c) for p, c in enumerate(tm_2d_L4[N]) if c}
    assert got == want


def test_brute_dos_matches_transfer_matrix_2d_L5():
    tm = transfer_dos(2, 5)
    for N in range(0, 7):
        got = O.brute_dos(2, 5, N)
        assert got == {-p: int(c) for p, c in enumerate(tm[N]) if c}


def _adjacency_by_roll(d, L):
    """Site adjacency of the periodic lattice built with np.roll of the index
    grid (independent of the oracle's coordinate arithmetic)."""
    idx = np.arange(L ** d).reshape((L,) * d)
    A = np.zeros((L ** d, L ** d), dtype=np.int64)
    for axis in range(d):
        nb = np.roll(idx, -1, axis=axis)
        A[idx.ravel(), nb.ravel()] = 1
        A[nb.ravel(), idx.ravel()] = 1
    return A


@pytest.mark.parametrize("L,Ns", [(3, range(0, 6)), (4, range(0, 4))])
def test_brute_dos_matches_numpy_enumeration_3d(L, Ns):
    import itertools
    A = _adjacency_by_roll(3, L)
    V = L ** 3
    for N in Ns:
        want = {}
        if N == 0:
            want = {0: 1}
        else:
            combos = np.array(list(itertools.combinations(range(V), N)), dtype=np.int64)
            pairs = np.zeros(len(combos), dtype=np.int64)
            for i in range(N):
                for j in range(i + 1, N):
                    pairs += A[combos[:, i], combos[:, j]]
            for p, c in zip(*np.unique(pairs, return_counts=True)):
                want[-int(p)] = int(c)
        assert O.brute_dos(3, L, N) == want


@pytest.mark.parametrize("d,L", [(2, 4), (2, 5), (2, 7), (3, 4), (3, 5)])
def test_closed_forms_small_N(d, L):
    V = L ** d
    assert O.brute_dos(d, L, 1) == {0: V}
    # N = 2: d V adjacent pairs
    assert O.brute_dos(d, L, 2) == {-1: d * V, 0: math.comb(V, 2) - d * V}
    # N = 3 (L >= 4, no triangles): paths of two bonds V C(2d,2); one bond
    # plus an isolated site d V (V - 2 - 2(2d-1))
    two = V * math.comb(2 * d, 2)
    one = d * V * (V - 2 - 2 * (2 * d - 1))
    assert O.brute_dos(d, L, 3) == {-2: two, -1: one, 0: math.comb(V, 3) - two - one}


@pytest.mark.parametrize("N", range(0, 17))
def test_total_and_particle_hole_symmetry_2d_L4(N):
    V, d = 16, 2
    om = O.brute_dos(d, 4, N)
    assert sum(om.values()) == math.comb(V, N)
    # holes: P_hh = P_nn + d (V - 2N), so Omega_{V-N}(E - d(V-2N)) = Omega_N(E)
    hole = O.brute_dos(d, 4, V - N)
    shift = d * (V - 2 * N)
    assert hole == {E - shift: c for E, c in om.items()}


# ---------------------------------------------------------------- window floor
@pytest.mark.parametrize("N", list(range(1, 400)))
def test_energy_floor_2d_harary_harborth(N):
    # max bonds of N unit squares: 2N - ceil(2 sqrt N)
    assert O.energy_floor(2, 64, N) == -(2 * N - math.isqrt(4 * N - 1) - 1)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_energy_floor_3d_cube(m):
    # m^3 sites: the cube has 3 m^2 (m - 1) bonds, the maximum for m^3 cubes
    assert O.energy_floor(3, 16, m ** 3) == -3 * m * m * (m - 1)


@pytest.mark.parametrize("d,L,Ns", [(2, 4, range(1, 9)), (2, 5, range(1, 8)),
                                    (3, 4, range(1, 6))])
def test_energy_floor_is_reachable(d, L, Ns):
    for N in Ns:
        om = O.brute_dos(d, L, N)
        f = O.energy_floor(d, L, N)
        assert f in om and f >= min(om)


def test_energy_floor_values_of_workloads():
    assert O.energy_floor(2, 8, 16) == -24    # 4 x 4 square
    assert O.energy_floor(3, 16, 205) == -509
