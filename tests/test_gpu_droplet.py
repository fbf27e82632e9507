"""GPU parity of the largest-droplet measurement (mucaLargestCluster, through
the C ABI) against the oracle's breadth-first search on the same walker
configurations (integer result: exact), from small lattices to the large 3D
workload (V = 110592 sites)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.droplet_ref import largest_cluster

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def _bits_to_occ(bits, V):
    b = np.array(bits, dtype=np.uint32)
    return ((b[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.uint8).ravel()[:V]


def test_largest_cluster_matches_oracle():
    # 2D and 3D, dense and sparse, a bricked 3D group, V = 32768, N = 1, and
    # particle counts at and next to powers of two (the LDS of the sorted
    # sites is padded to one)
    groups = [(2, 8, 16, 4), (3, 5, 30, 3), (2, 32, 300, 3), (3, 16, 1300, 2),
              (3, 24, 1100, 2), (3, 32, 655, 1), (2, 6, 1, 2), (2, 16, 128, 3),
              (2, 16, 127, 2), (2, 64, 1024, 1), (3, 16, 1025, 1), (3, 48, 3318, 1)]
    say("droplets", groups)
    ctx = M.Context(groups, seed=7)
    ref = O.RefContext(groups, seed=7)
    lnW = W.random_lnW(ctx.total_bins, seed=3, scale=0.2)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    ctx.sweep(torch.tensor(lnW, device=DEV), 2, H)
    ref.sweep(lnW, 2)
    out = torch.full((ctx.nwalkers,), -7, dtype=torch.int32, device=DEV)
    ctx.largest_cluster(out)
    got = out.cpu().numpy()
    w = 0
    for d, L, N, walkers, *_ in groups:
        for _ in range(walkers):
            n = ref.walker(w)[0]
            assert got[w] == largest_cluster(n, d, L), (w, d, L, N)
            assert 1 <= got[w] <= N
            w += 1


def test_full_size_batched_2d_sampled():
    wl = W.WORKLOADS["batched_2d"]
    ctx = M.Context(wl["groups"], wl["seed"])
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    ctx.sweep(torch.zeros(ctx.total_bins, dtype=torch.float64, device=DEV), 3, H)
    out = torch.empty(ctx.nwalkers, dtype=torch.int32, device=DEV)
    ctx.largest_cluster(out)  # warm
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    ctx.largest_cluster(out)
    b.record()
    torch.cuda.synchronize()
    say(f"largest cluster: {ctx.nwalkers} walkers in {a.elapsed_time(b):.3f} ms")
    got = out.cpu().numpy()
    rng = np.random.default_rng(2)
    first = 0
    for d, L, N, walkers in wl["groups"]:
        assert ((got[first:first + walkers] >= 1) & (got[first:first + walkers] <= N)).all()
        for w in first + rng.choice(walkers, 8, replace=False):
            bits, pos, E, t = ctx.read_walker(int(w))
            assert got[w] == largest_cluster(_bits_to_occ(bits, L ** d), d, L), w
        first += walkers


def test_full_size_large_3d_sampled():
    """The large 3D workload (V = 110592 sites, N = 3318, bricked state in
    device memory): every walker measured, sampled walkers replayed by the
    oracle's search."""
    wl = W.WORKLOADS["large_3d"]
    ctx = M.Context(wl["groups"], wl["seed"])
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    ctx.sweep(torch.zeros(ctx.total_bins, dtype=torch.float64, device=DEV), 1, H)
    out = torch.full((ctx.nwalkers,), -7, dtype=torch.int32, device=DEV)
    ctx.largest_cluster(out)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    ctx.largest_cluster(out)
    b.record()
    torch.cuda.synchronize()
    say(f"largest cluster: {ctx.nwalkers} walkers of V = 110592 in {a.elapsed_time(b):.3f} ms")
    got = out.cpu().numpy()
    d, L, N, walkers = wl["groups"][0]
    assert ((got >= 1) & (got <= N)).all()
    rng = np.random.default_rng(5)
    for w in rng.choice(walkers, 6, replace=False):
        bits, pos, E, t = ctx.read_walker(int(w))
        assert got[w] == largest_cluster(_bits_to_occ(bits, L ** d), d, L), w
    ctx.close()


def test_too_many_particles_are_refused():
    # N = 16500 sorted sites (padded to 32768) and parents exceed the LDS
    ctx = M.Context([(3, 32, 16500, 1, -49500, 0)], seed=1)
    out = torch.full((1,), -7, dtype=torch.int32, device=DEV)
    with pytest.raises(M.MucaError) as e:
        ctx.largest_cluster(out)
    assert e.value.code == M.MUCA_EINVAL
    torch.cuda.synchronize()
    assert out.item() == -7
