"""Reference of the largest-droplet measurement (test infrastructure).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Plain Python/numpy, written from
the definition.  Sec. 3 studies condensation through the largest droplet:
the largest set of particles connected through nearest-neighbour bonds of
the lattice (periodic boundaries, sites s = x + L y + L^2 z).  The size of
that set is measured on a walker's configuration by a breadth-first search
over the occupied sites.
"""
import numpy as np


def neighbours(s, d, L):
    """The 2d nearest neighbours of site s on the periodic lattice."""
    c = [(s // L ** a) % L for a in range(d)]
    out = []
    for a in range(d):
        for step in (1, -1):
            cc = list(c)
            cc[a] = (cc[a] + step) % L
            out.append(sum(cc[b] * L ** b for b in range(d)))
    return out


def largest_cluster(occ, d, L):
    """Size of the largest nearest-neighbour cluster of occupied sites
    (0 for an empty lattice)."""
    occ = np.asarray(occ).astype(bool)
    seen = np.zeros(occ.size, dtype=bool)
    best = 0
    for s in np.flatnonzero(occ):
        if seen[s]:
            continue
        seen[s] = True
        stack, n = [int(s)], 0
        while stack:
            u = stack.pop()
            n += 1
            for v in neighbours(u, d, L):
                if occ[v] and not seen[v]:
                    seen[v] = True
                    stack.append(v)
        best = max(best, n)
    return best
