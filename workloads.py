"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module holds the workload definitions (lattice sizes, densities, walker
counts, schedules) and seeded random weight tables.  It holds none of the
method's arithmetic and imports neither the oracle nor the GPU library.

Workloads (synthetic lattice-gas states; the paper uses no dataset):
  plain_2d      2D L=8, N=16, 64 walkers, 10 iterations x 1e4 sweeps
  batched_2d    6 groups (L, rho) in {32,48,64} x {0.05,0.10}, 4096 walkers,
                20 iterations x 1e4 sweeps
  cubic_3d      3D L=16, rho=0.05 (N=205), 8192 walkers, until flat, S=1e3
  batched_3d    8 groups L in {24,32} x rho in {.02,.04,.06,.10},
                16384 walkers split in proportion to N, until flat, S=1e2
  large_3d      3D L=48, rho=0.03 (N=3318), 16384 walkers, until flat, S=1e2
  held_out_3d   3D L=24, rho=0.03 (N=415), 4096 walkers, until flat, S=1e2: the
                large lattice's density at a size both weight arms can flatten
                within minutes (a held-out target of the learned weights)
"""
from fractions import Fraction

import numpy as np


def particles(d, L, rho):
    """N = rho L^d rounded half up, with rho taken as an exact decimal."""
    x = Fraction(str(rho)) * L ** d
    return int(x + Fraction(1, 2))  # floor(x + 1/2)


def split_even(total, n):
    base, rem = divmod(total, n)
    return [base + (1 if i < rem else 0) for i in range(n)]


def split_proportional(total, weights):
    """Largest-remainder split of `total` in proportion to `weights`."""
    s = sum(weights)
    exact = [Fraction(total * w, s) for w in weights]
    out = [int(e) for e in exact]
    order = sorted(range(len(weights)), key=lambda i: (-(exact[i] - out[i]), i))
    for i in order[:total - sum(out)]:
        out[i] += 1
    return out


def _batched_2d():
    shapes = [(L, r) for L in (32, 48, 64) for r in (0.05, 0.10)]
    walkers = split_even(4096, len(shapes))
    return [(2, L, particles(2, L, r), w) for (L, r), w in zip(shapes, walkers)]


def _batched_3d():
    shapes = [(L, r) for L in (24, 32) for r in (0.02, 0.04, 0.06, 0.10)]
    Ns = [particles(3, L, r) for L, r in shapes]
    walkers = split_proportional(16384, Ns)
    return [(3, L, N, w) for (L, _), N, w in zip(shapes, Ns, walkers)]


WORKLOADS = {
    "plain_2d": dict(groups=[(2, 8, 16, 64)], seed=1, sweeps=10_000, iters=10,
                     stop_on_flat=False),
    "batched_2d": dict(groups=_batched_2d(), seed=1, sweeps=10_000, iters=20,
                       stop_on_flat=False),
    "cubic_3d": dict(groups=[(3, 16, particles(3, 16, 0.05), 8192)], seed=1, sweeps=1_000,
                     iters=None, stop_on_flat=True),
    "batched_3d": dict(groups=_batched_3d(), seed=1, sweeps=100, iters=None, stop_on_flat=True),
    "large_3d": dict(groups=[(3, 48, particles(3, 48, 0.03), 16384)], seed=1, sweeps=100,
                     iters=None, stop_on_flat=True),
    "held_out_3d": dict(groups=[(3, 24, particles(3, 24, 0.03), 4096)], seed=1, sweeps=100,
                        iters=None, stop_on_flat=True),
}


def scaled(name, walkers_per_group=None, sweeps=None):
    """A reduced copy of a workload: same lattices and densities, fewer
    walkers per group and/or sweeps (for parity runs the oracle finishes)."""
    w = dict(WORKLOADS[name])
    if walkers_per_group is not None:
        w["groups"] = [g[:3] + (min(g[3], walkers_per_group),) + tuple(g[4:]) for g in w["groups"]]
    if sweeps is not None:
        w["sweeps"] = sweeps
    return w


def random_lnW(total_bins, seed, scale=2.0):
    """Seeded random weights (standard normal steps, a random walk)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.normal(0.0, scale, total_bins))


def random_histogram(total_bins, seed, high=10_000, zero_frac=0.1):
    rng = np.random.default_rng(seed)
    h = rng.integers(1, high, total_bins).astype(np.int32)
    h[rng.random(total_bins) < zero_frac] = 0
    return h


# Learned-initial-weights network: 4 -> 128 -> 128 -> 128 -> 1 (flat FP32
# parameter vector W1[128][4] b1 W2[128][128] b2 W3[128][128] b3 W4[128] b4).
MLP_SIZES = (4, 128, 128, 128, 1)


def mlp_init_params(seed):
    """Seeded initial parameters: weights N(0, 1/fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in zip(MLP_SIZES[:-1], MLP_SIZES[1:]):
        parts.append(rng.normal(0.0, 1.0 / np.sqrt(fan_in), (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def mlp_synthetic_rows(n, seed):
    """Seeded feature rows in the ranges the features take, and a smooth target."""
    rng = np.random.default_rng(seed)
    X = np.stack([rng.choice([-1.0, 1.0], n), rng.uniform(0.1, 1.0, n), rng.uniform(0.2, 2.5, n),
                  rng.uniform(0.0, 1.0, n)], axis=1).astype(np.float32)
    T = (np.sin(3 * X[:, 3]) * X[:, 2] - 0.5 * X[:, 1] + 0.2 * X[:, 0]).astype(np.float32)
    return X, T
