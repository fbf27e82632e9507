"""Pins of the oracle's largest-droplet measurement (Sec. 3: the largest
cluster of nearest-neighbour-connected particles).

* Hand-made configurations with known cluster sizes, including clusters
  that close through the periodic boundary in x, y and z.
* An independent algorithm in the test (union-find over the particles with
  neighbours found by coordinate arithmetic on an occupancy grid built with
  np.roll) agrees on seeded random configurations of every density.
* Limits: isolated particles give 1, one compact block gives N, an empty
  lattice gives 0.
"""
import numpy as np
import pytest

from oracle.droplet_ref import largest_cluster


def _occ(d, L, coords):
    occ = np.zeros(L ** d, dtype=np.uint8)
    for c in coords:
        occ[sum(c[a] * L ** a for a in range(d))] = 1
    return occ


def _union_find(occ, d, L):
    # site s = x + L y + L^2 z: as a C-ordered array the last axis is x
    grid = np.asarray(occ).reshape((L,) * d)
    idx = -np.ones(grid.shape, dtype=np.int64)
    pts = np.argwhere(grid)
    idx[tuple(pts.T)] = np.arange(len(pts))
    parent = list(range(len(pts)))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for ax in range(d):
        nb = np.roll(idx, -1, axis=ax)
        both = (idx >= 0) & (nb >= 0)
        for a, b in zip(idx[both], nb[both]):
            ra, rb = find(int(a)), find(int(b))
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    if not len(pts):
        return 0
    roots = [find(i) for i in range(len(pts))]
    return int(np.bincount(roots).max())


def test_hand_made_2d():
    L = 6
    # a 2x2 square, a bar of 3 closing through x = 5 -> 0, and a single site
    coords = [(1, 1), (2, 1), (1, 2), (2, 2), (5, 4), (0, 4), (1, 4), (3, 5)]
    assert largest_cluster(_occ(2, L, coords), 2, L) == 4
    # join the bar to the square through y: (1, 3)
    assert largest_cluster(_occ(2, L, coords + [(1, 3)]), 2, L) == 8
    # a column wrapping through y = 5 -> 0
    col = [(4, y) for y in (4, 5, 0, 1)]
    assert largest_cluster(_occ(2, L, col), 2, L) == 4


def test_hand_made_3d():
    L = 4
    # a line closing through z = 3 -> 0 and a diagonal pair (not bonded)
    coords = [(0, 0, 3), (0, 0, 0), (0, 0, 1), (2, 2, 2), (3, 3, 2)]
    assert largest_cluster(_occ(3, L, coords), 3, L) == 3
    # a full plane z = 1 wraps in x and y: 16 sites
    plane = [(x, y, 1) for x in range(L) for y in range(L)]
    assert largest_cluster(_occ(3, L, plane), 3, L) == 16


def test_limits():
    L = 8
    iso = [(x, y) for x in range(0, L, 2) for y in range(0, L, 2)]
    assert largest_cluster(_occ(2, L, iso), 2, L) == 1
    block = [(x, y) for x in range(3) for y in range(5)]
    assert largest_cluster(_occ(2, L, block), 2, L) == 15
    assert largest_cluster(np.zeros(L * L), 2, L) == 0


@pytest.mark.parametrize("d,L", [(2, 7), (2, 16), (3, 5), (3, 8)])
@pytest.mark.parametrize("rho", [0.05, 0.2, 0.45, 0.7])
def test_matches_union_find(d, L, rho):
    rng = np.random.default_rng(int(rho * 100) + 10 * d + L)
    for _ in range(5):
        occ = (rng.random(L ** d) < rho).astype(np.uint8)
        assert largest_cluster(occ, d, L) == _union_find(occ, d, L)
