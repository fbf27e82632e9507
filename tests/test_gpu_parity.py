"""GPU parity: every call of libmuca (through its C ABI) against the CPU
oracle on the same seeded inputs.  Histograms, walker states, thresholds and
weights must agree bit for bit (integer work is exact; the binary64 steps use
the same IEEE operation sequence on both sides)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def dev_f64(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device=DEV)


def dev_i32(a):
    return torch.tensor(np.asarray(a, dtype=np.int32), device=DEV)


def bits_to_occ(bits, V):
    b = np.array(bits, dtype=np.uint32)
    occ = ((b[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.uint8).ravel()
    return occ[:V]


def assert_walkers_equal(ctx, ref, walkers):
    for w in walkers:
        bits, pos, E, t = ctx.read_walker(w)
        n, rpos, rE, rt = ref.walker(w)
        assert E == rE and t == rt, (w, E, rE, t, rt)
        assert np.array_equal(bits_to_occ(bits, len(n)), n), w
        assert np.array_equal(np.array(pos, dtype=np.uint32), rpos), w
    assert_tunnel_equal(ctx, ref)


def assert_tunnel_equal(ctx, ref):
    """Tunnelling state of every walker (last window end, trips), bit-exact."""
    last, trips = ctx.tunnel()
    rlast, rtrips = ref.tunnel()
    assert np.array_equal(np.array(last, dtype=np.uint32), rlast)
    assert np.array_equal(np.array(trips, dtype=np.uint32), rtrips)


def same_f64(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return np.array_equal(a.view(np.int64), b.view(np.int64))


MIXED = [(2, 8, 16, 5), (3, 5, 12, 3), (2, 9, 7, 70), (3, 4, 3, 2), (2, 32, 51, 3)]


def test_initial_placement_matches_oracle():
    say("placement", MIXED)
    ctx = M.Context(MIXED, seed=7)
    ref = O.RefContext(MIXED, seed=7)
    assert ctx.total_bins == ref.total_bins
    for g in range(len(MIXED)):
        lo, hi, off = ctx.window(g)
        assert (lo, hi) == ref.window(g) and off == ref.bin_offset(g)
    assert_walkers_equal(ctx, ref, range(ctx.nwalkers))


def test_bricked_placement_matches_oracle():
    # 3D groups whose 16-walker state exceeds 160 KiB keep 8x8x8-bricked bits;
    # mucaReadWalker returns the linear layout
    groups = [(3, 16, 1300, 3), (3, 24, 1100, 2), (3, 16, 205, 2)]
    say("bricked placement", groups)
    ctx = M.Context(groups, seed=5)
    ref = O.RefContext(groups, seed=5)
    assert_walkers_equal(ctx, ref, range(ctx.nwalkers))


def test_first_id_offsets_streams():
    say("first_id")
    ctx = M.Context([(2, 8, 16, 4)], seed=3, first_id=1000)
    ref = O.RefContext([(2, 8, 16, 4)], seed=3, first_id=1000)
    assert_walkers_equal(ctx, ref, range(4))


def test_thresholds_match_oracle_decision():
    groups = [(2, 8, 16, 1), (3, 5, 12, 1), (2, 6, 5, 1, -6, -1)]
    say("thresholds", groups)
    ctx = M.Context(groups, seed=1)
    ref = O.RefContext(groups, seed=1)
    rng = np.random.default_rng(0)
    lnW = rng.normal(0.0, 6.0, ctx.total_bins)
    lnW[::7] += rng.normal(0.0, 1e-12, len(lnW[::7]))  # near-zero differences
    out = torch.zeros(ctx.threshold_entries, dtype=torch.int32, device=DEV)
    ctx.build_thresholds(dev_f64(lnW), out)
    T = out.cpu().numpy().view(np.uint32)
    i = 0
    checked = 0
    for g, grp in enumerate(groups):
        d = grp[0]
        lo, hi, off = ctx.window(g)
        nb = hi - lo + 1
        for bo in range(nb):
            for dE in range(-2 * d, 2 * d + 1):
                t = int(T[i])
                i += 1
                bn = bo + dE
                if bn < 0 or bn >= nb:
                    assert t == 0
                    continue
                x = lnW[off + bn] - lnW[off + bo]
                if t == 0xFFFFFFFF:
                    assert O.accept(x, 0xFFFFFFFF), x
                elif t == 0:
                    assert not O.accept(x, 0), x
                else:
                    assert O.accept(x, t - 1) and not O.accept(x, t), (x, t)
                checked += 1
    assert i == ctx.threshold_entries and checked > 200


@pytest.mark.parametrize("rule", [0, 1])
def test_update_matches_oracle_bitwise(rule):
    groups = [(2, 32, 230, 1, -429, 0), (3, 6, 40, 1, -80, 0), (2, 5, 3, 1, -2, 0)]
    say("update rule", rule)
    ctx = M.Context(groups, seed=1)
    ref = O.RefContext(groups, seed=1)
    nb = ctx.total_bins
    lnW = W.random_lnW(nb, seed=5)
    P = np.zeros(nb)
    glnW, gP = dev_f64(lnW), dev_f64(P)
    for step in range(4):
        H = W.random_histogram(nb, seed=10 + step, zero_frac=0.05 + 0.1 * step)
        if step == 3:
            H[:] = 0
            H[200:260] = 1000  # visited band in the middle of group 0: frontier
        ctx.update_weights(dev_i32(H), glnW, gP, rule)
        ref.update(H, lnW, P, rule)
        torch.cuda.synchronize()
        assert same_f64(glnW.cpu().numpy(), lnW), (rule, step)
        assert same_f64(gP.cpu().numpy(), P), (rule, step)
    assert ctx.status() == 0


def test_flatness_matches_oracle():
    groups = [(2, 8, 16, 1), (3, 5, 12, 1), (2, 9, 7, 1)]
    ctx = M.Context(groups, seed=1)
    ref = O.RefContext(groups, seed=1)
    flags = torch.zeros(3, dtype=torch.int32, device=DEV)
    rng = np.random.default_rng(3)
    for trial in range(40):
        H = rng.integers(0, 40, ctx.total_bins).astype(np.int32) + (trial % 3) * 30
        if trial % 5 == 0:
            H[rng.integers(0, ctx.total_bins)] = 0
        ctx.is_flat(dev_i32(H), flags)
        assert np.array_equal(flags.cpu().numpy(), ref.flat(H)), trial


# (layout, LDS limit): every kernel variant, with walker state in LDS and in
# device memory
VARIANTS = [(M.MUCA_LAYOUT_LANE, 163840), (M.MUCA_LAYOUT_SUB16, 163840),
            (M.MUCA_LAYOUT_SUB16, 0), (M.MUCA_LAYOUT_SUB64, 163840), (M.MUCA_LAYOUT_SUB64, 0),
            (M.MUCA_LAYOUT_SUB16, 24576), (M.MUCA_LAYOUT_LOOK4, 163840),
            (M.MUCA_LAYOUT_LOOK4, 24576), (M.MUCA_LAYOUT_SUB16X2, 163840),
            (M.MUCA_LAYOUT_SUB16X2, 0), (M.MUCA_LAYOUT_SUB16X1, 163840),
            (M.MUCA_LAYOUT_SUB16MIX, 163840), (M.MUCA_LAYOUT_SUB16MIX, 0)]
VARIANT_IDS = ["lane", "sub16-lds", "sub16-hbm", "sub64-lds", "sub64-hbm", "sub16-lds24k",
               "look4", "look4-lds24k", "sub16x2-lds", "sub16x2-hbm", "sub16x1-lds",
               "sub16mix-lds", "sub16mix-hbm"]


def make_ctx(groups, seed, variant=None, first_id=0):
    ctx = M.Context(groups, seed, first_id)
    if variant is not None:
        ctx.set_layout(variant[0])
        ctx.set_lds_limit(variant[1])
    return ctx


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
@pytest.mark.parametrize("groups,sweeps", [
    (MIXED, 7),
    ([(2, 8, 16, 64)], 30),
    ([(3, 3, 5, 10), (3, 16, 205, 3)], 3),
    ([(2, 9, 20, 5, -30, -2)], 11),
    ([(2, 4, 8, 17, -12, 0), (3, 4, 30, 6, -80, 0)], 9),   # dense: many rejected candidates
    # bricked occupation bits (3D, L % 8 == 0, state too large for LDS) beside a
    # linear group; L = 24 has an odd number of bricks per axis
    ([(3, 16, 1300, 3), (2, 8, 16, 2)], 2),
    ([(3, 24, 1100, 2)], 1),
])
def test_sweep_matches_oracle(groups, sweeps, variant):
    say("sweep", groups, sweeps, variant)
    ctx = make_ctx(groups, 2, variant)
    ref = O.RefContext(groups, seed=2)
    lnW = W.random_lnW(ctx.total_bins, seed=9, scale=1.5)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    for call in range(2):  # walker state carries over between calls
        ctx.sweep(dev_f64(lnW), sweeps, H)
        rH = ref.sweep(lnW, sweeps)
        torch.cuda.synchronize()
        assert np.array_equal(H.cpu().numpy(), rH), call
    assert_walkers_equal(ctx, ref, range(ctx.nwalkers))


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_packed_blocks_match_oracle(variant):
    # more walker sets than CUs, not a whole multiple: sets are packed longest
    # first into whole rounds of blocks, some blocks running two sets
    groups = [(2, 4, 5, 2056), (2, 6, 10, 2056), (3, 4, 9, 20, -20, 0)]
    say("packed", groups, variant)
    ctx = make_ctx(groups, 6, variant)
    ref = O.RefContext(groups, seed=6)
    lnW = W.random_lnW(ctx.total_bins, seed=7, scale=1.0)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    for call in range(2):
        ctx.sweep(dev_f64(lnW), 3, H)
        rH = ref.sweep(lnW, 3)
        torch.cuda.synchronize()
        assert np.array_equal(H.cpu().numpy(), rH), call
    rng = np.random.default_rng(0)
    assert_walkers_equal(ctx, ref, sorted(rng.choice(ctx.nwalkers, 150, replace=False)))


def test_sweep_active_mask():
    groups = [(2, 8, 16, 4), (3, 4, 5, 3), (2, 6, 4, 5)]
    ctx = M.Context(groups, seed=4)
    ref = O.RefContext(groups, seed=4)
    lnW = W.random_lnW(ctx.total_bins, seed=2, scale=1.0)
    active = np.array([1, 0, 1], dtype=np.int32)
    H = torch.full((ctx.total_bins,), -7, dtype=torch.int32, device=DEV)
    rH = np.full(ctx.total_bins, -7, dtype=np.int32)
    ctx.sweep(dev_f64(lnW), 5, H, active=dev_i32(active))
    r = ref.sweep(lnW, 5, active=active)
    lo, hi, off = ctx.window(1)
    mask = np.zeros(ctx.total_bins, bool)
    mask[off:off + hi - lo + 1] = True
    rH[~mask] = r[~mask]
    assert np.array_equal(H.cpu().numpy(), rH)
    assert_walkers_equal(ctx, ref, range(ctx.nwalkers))


def _run_both(groups, seed, sweeps, iters, rule=0, stop_on_flat=False, lnW0=None,
              check_walkers=True, variant=None, tunnel_target=None, graph=True):
    say("run", groups, "sweeps", sweeps, "iters", iters, "rule", rule, "flat", stop_on_flat,
        "tunnel", tunnel_target, "variant", variant)
    ctx = make_ctx(groups, seed, variant)
    ctx.set_graph(graph)
    stop = None
    if tunnel_target is not None:
        ctx.set_tunnel_target(tunnel_target)
        stop = M.MUCA_STOP_TUNNEL
    ref = O.RefContext(groups, seed)
    lnW = np.zeros(ctx.total_bins) if lnW0 is None else np.array(lnW0, dtype=np.float64)
    P = np.full(ctx.total_bins, 123.0)  # mucaRun zeroes P itself
    glnW, gP = dev_f64(lnW), dev_f64(P)
    gH = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    rc, it, fl = ctx.run(glnW, gP, gH, sweeps, iters, rule, stop_on_flat, stop=stop)
    P[:] = 0.0
    rrc, rH, rit, rfl = ref.run(lnW, P, sweeps, iters, rule, stop_on_flat,
                                tunnel_target=tunnel_target)
    assert rc == rrc
    assert list(it) == list(rit) and list(fl) == list(rfl)
    assert np.array_equal(gH.cpu().numpy(), rH)
    assert same_f64(glnW.cpu().numpy(), lnW)
    assert same_f64(gP.cpu().numpy(), P)
    if check_walkers:
        n = ctx.nwalkers
        assert_walkers_equal(ctx, ref, sorted(set([0, n - 1] + list(range(0, n, max(1, n // 16))))))
    else:
        assert_tunnel_equal(ctx, ref)
    return rc, it, fl


@pytest.mark.parametrize("variant", [VARIANTS[0], VARIANTS[1], VARIANTS[6]],
                         ids=[VARIANT_IDS[0], VARIANT_IDS[1], VARIANT_IDS[6]])
def test_run_plain_2d_full_schedule(variant):
    # 2D L=8, N=16, 64 walkers, 10 iterations x 1e4 sweeps from lnW = 0
    wl = W.WORKLOADS["plain_2d"]
    _run_both(wl["groups"], wl["seed"], wl["sweeps"], wl["iters"], variant=variant)


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
@pytest.mark.parametrize("name,walkers,sweeps,iters", [
    ("batched_2d", 8, 40, 3),
    ("cubic_3d", 16, 20, 3),
    ("batched_3d", 2, 2, 2),
    ("large_3d", 2, 1, 2),
])
def test_run_reduced_workloads(name, walkers, sweeps, iters, variant):
    wl = W.scaled(name, walkers_per_group=walkers, sweeps=sweeps)
    _run_both(wl["groups"], wl["seed"], wl["sweeps"], iters, stop_on_flat=wl["stop_on_flat"],
              variant=variant)


@pytest.mark.parametrize("variant", [VARIANTS[1], VARIANTS[2], VARIANTS[8], VARIANTS[9]],
                         ids=[VARIANT_IDS[1], VARIANT_IDS[2], VARIANT_IDS[8], VARIANT_IDS[9]])
def test_run_with_packed_blocks_until_flat(variant):
    # more walker sets than CUs (packed blocks) inside the captured iteration
    # loop, groups stopping at different iterations
    groups = [(2, 4, 5, 2056), (2, 6, 10, 2056), (3, 4, 9, 20, -20, 0)]
    rc, it, fl = _run_both(groups, 3, 20, 30, rule=0, stop_on_flat=True, variant=variant)
    assert list(fl) == [1, 1, 0] and list(it) == [2, 3, 30]  # as the oracle (checked above)


FLAT_GROUPS = [(2, 4, 5, 64, -5, 0), (2, 6, 10, 16, 0, 0), (3, 4, 4, 16, -4, 0),
               (2, 8, 12, 16, 0, 0), (2, 7, 9, 8, 0, 0)]


@pytest.mark.parametrize("variant", VARIANTS[:2] + VARIANTS[6:7], ids=VARIANT_IDS[:2] + ["look4"])
def test_run_until_flat_per_group(variant):
    # the groups go flat at different iterations (2, 4, 3, 7, 10 for this seed)
    rc, it, fl = _run_both(FLAT_GROUPS, 5, 50, 80, rule=0, stop_on_flat=True, variant=variant)
    assert rc == 0 and all(fl) and len(set(it)) >= 4


TUNNEL_GROUPS = [(2, 4, 2, 6, -1, 0), (2, 4, 3, 5), (3, 3, 3, 4), (2, 6, 5, 4, -3, 0),
                 (3, 6, 12, 3, -10, 0)]


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_tunnelling_matches_oracle(variant):
    """Tunnelling state after sweeps with small windows (every layout):
    last window end and trips of every walker, bit-exact."""
    say("tunnel", variant)
    ctx = make_ctx(TUNNEL_GROUPS, 4, variant)
    ref = O.RefContext(TUNNEL_GROUPS, seed=4)
    lnW = W.random_lnW(ctx.total_bins, seed=6, scale=0.3)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    for call in range(2):  # the state carries over between calls
        ctx.sweep(dev_f64(lnW), 25, H)
        rH = ref.sweep(lnW, 25)
        torch.cuda.synchronize()
        assert np.array_equal(H.cpu().numpy(), rH), call
        assert_tunnel_equal(ctx, ref)
    assert sum(ctx.tunnel()[1]) > 0


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
@pytest.mark.parametrize("variant", [None, VARIANTS[0], VARIANTS[2], VARIANTS[6], VARIANTS[8]],
                         ids=["auto", VARIANT_IDS[0], VARIANT_IDS[2], VARIANT_IDS[6],
                              VARIANT_IDS[8]])
def test_run_until_tunnelling_target(variant, graph):
    """The convergence criterion of Sec. 4: each group stops after the first
    iteration at whose end its walkers made the target number of trips."""
    rc, it, fl = _run_both(TUNNEL_GROUPS[1:], 9, 10, 200, rule=0, variant=variant,
                           tunnel_target=12, graph=graph)
    assert rc == M.MUCA_OK and min(it) >= 1 and len(set(it)) > 1


def test_run_until_flat_some_groups_not_converged():
    rc, it, fl = _run_both(FLAT_GROUPS, 5, 20, 80, rule=0, stop_on_flat=True)
    assert rc == M.MUCA_NOT_CONVERGED and not all(fl)


def test_run_simple_rule_and_not_converged():
    groups = [(2, 4, 8, 16, -12, 0), (2, 6, 9, 8)]
    rc, it, fl = _run_both(groups, 6, 30, 4, rule=1, stop_on_flat=True)
    assert rc == M.MUCA_NOT_CONVERGED


def test_run_from_nonzero_weights():
    groups = [(2, 8, 16, 16)]
    lnW0 = W.random_lnW(25, seed=3, scale=0.7)
    _run_both(groups, 8, 50, 3, lnW0=lnW0)


@pytest.mark.parametrize("variant", VARIANTS, ids=VARIANT_IDS)
def test_edge_single_particle_and_small_lattices(variant):
    # N = 1; V = 9 and 27 (sweeps shorter than a 16- or 64-attempt batch);
    # N = V - 1 (every candidate but one occupied)
    groups = [(3, 5, 1, 3), (2, 3, 4, 2, -4, 0), (3, 3, 13, 2, -30, 0), (2, 4, 15, 2, -28, 0)]
    say("edge", groups, variant)
    ctx = make_ctx(groups, 1, variant)
    ref = O.RefContext(groups, seed=1)
    assert ctx.window(0)[:2] == (0, 0)
    lnW = W.random_lnW(ctx.total_bins, seed=4, scale=1.0)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    ctx.sweep(dev_f64(lnW), 9, H)
    rH = ref.sweep(lnW, 9)
    assert np.array_equal(H.cpu().numpy(), rH)
    assert H[0].item() == 27  # N = 1: E = 0 always
    assert_walkers_equal(ctx, ref, range(ctx.nwalkers))


@pytest.mark.parametrize("variant", [None] + VARIANTS[1:], ids=["auto"] + VARIANT_IDS[1:])
@pytest.mark.parametrize("name,sample", [("batched_2d", 12), ("large_3d", 4),
                                         ("batched_3d", 8), ("cubic_3d", 6)])
def test_full_size_sampled_walkers(name, sample, variant):
    """Full walker populations: every walker sweeps on the GPU; sampled
    walkers are replayed one by one by the oracle (same global id)."""
    wl = W.WORKLOADS[name]
    groups = wl["groups"]
    sweeps = 1
    say("full size", name, groups, variant)
    ctx = make_ctx(groups, wl["seed"], variant)
    lnW = W.random_lnW(ctx.total_bins, seed=12, scale=0.5)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    ctx.sweep(dev_f64(lnW), sweeps, H)
    Hn = H.cpu().numpy()
    glast, gtrips = ctx.tunnel()
    rng = np.random.default_rng(1)
    first = 0
    picks = []
    for g, grp in enumerate(groups):
        lo, hi, off = ctx.window(g)
        assert Hn[off:off + hi - lo + 1].sum() == grp[3] * sweeps
        picks += [(g, first + int(j)) for j in rng.choice(grp[3], size=min(grp[3], max(
            1, sample // len(groups))), replace=False)]
        first += grp[3]
    for g, w in picks:
        grp = groups[g]
        lo, hi, off = ctx.window(g)
        ref = O.RefContext([grp[:3] + (1, lo, hi)], wl["seed"], first_id=w)
        ref.sweep(lnW[off:off + hi - lo + 1], sweeps)
        bits, pos, E, t = ctx.read_walker(w)
        n, rpos, rE, rt = ref.walker(0)
        assert (E, t) == (rE, rt), (name, w)
        rlast, rtrips = ref.tunnel()
        assert (glast[w], gtrips[w]) == (rlast[0], rtrips[0]), (name, w)
        assert np.array_equal(np.array(pos, dtype=np.uint32), rpos)
        assert np.array_equal(bits_to_occ(bits, len(n)), n)


def recount_energy(occ, d, L):
    """E = -(occupied nearest-neighbour pairs), periodic (site s = x + L y + L^2 z)."""
    n = occ.reshape((L,) * d).astype(np.int64)
    return -int(sum((n * np.roll(n, 1, axis=a)).sum() for a in range(d)))


@pytest.mark.parametrize("variant", [None, VARIANTS[1], VARIANTS[2], VARIANTS[8]],
                         ids=["auto", VARIANT_IDS[1], VARIANT_IDS[2], VARIANT_IDS[8]])
@pytest.mark.parametrize("name", ["batched_2d", "cubic_3d", "batched_3d", "large_3d"])
def test_full_size_invariants(name, variant):
    """Invariants of the walker state after a sweep of the full population:
    N occupied sites, the particle list on occupied sites and distinct, the
    incremental energy equal to a recount, inside the window; sum of H equal
    to walkers x sweeps per group."""
    wl = W.WORKLOADS[name]
    groups = wl["groups"]
    say("invariants", name, variant)
    ctx = make_ctx(groups, wl["seed"], variant)
    lnW = W.random_lnW(ctx.total_bins, seed=21, scale=0.3)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    ctx.sweep(dev_f64(lnW), 2, H)
    Hn = H.cpu().numpy()
    rng = np.random.default_rng(5)
    first = 0
    for g, (d, L, N, walkers, *_r) in enumerate(groups):
        lo, hi, off = ctx.window(g)
        assert Hn[off:off + hi - lo + 1].sum() == walkers * 2
        for w in first + rng.choice(walkers, size=min(walkers, 3), replace=False):
            bits, pos, E, t = ctx.read_walker(int(w))
            occ = bits_to_occ(bits, L ** d)
            pos = np.array(pos, dtype=np.int64)
            assert occ.sum() == N and len(np.unique(pos)) == N
            assert occ[pos].all()
            assert E == recount_energy(occ, d, L) and lo <= E <= hi
            assert t == 2 * L ** d
        first += walkers


def test_errors():
    ctx = M.Context([(2, 8, 16, 4)], seed=1)
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=DEV)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    with pytest.raises(M.MucaError) as e:
        ctx.sweep(lnW, 2**30, H)
    assert e.value.code == M.MUCA_EOVERFLOW
    with pytest.raises(M.MucaError) as e:
        ctx.sweep(lnW, 0, H)
    assert e.value.code == M.MUCA_EINVAL
    bad = lnW.clone()
    bad[3] = float("nan")
    ctx.sweep(bad, 1, H)
    with pytest.raises(M.MucaError) as e:
        ctx.status()
    assert e.value.code == M.MUCA_ENONFINITE
    assert ctx.status() == 0  # cleared
    P = torch.zeros_like(lnW)
    with pytest.raises(M.MucaError) as e:
        ctx.run(bad, P, H, 1, 2)
    assert e.value.code == M.MUCA_ENONFINITE
    with pytest.raises(M.MucaError) as e:
        ctx.run(lnW, P, H, 1, 2, stop=3)
    assert e.value.code == M.MUCA_EINVAL
    with pytest.raises(M.MucaError) as e:
        ctx.set_tunnel_target(0)
    assert e.value.code == M.MUCA_EINVAL


def test_determinism_two_contexts():
    groups = W.scaled("batched_2d", walkers_per_group=64)["groups"]
    outs = []
    for _ in range(2):
        ctx = M.Context(groups, seed=1)
        lnW = dev_f64(W.random_lnW(ctx.total_bins, seed=1, scale=0.3))
        H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
        ctx.sweep(lnW, 5, H)
        outs.append(H.cpu().numpy())
        ctx.close()
    assert np.array_equal(outs[0], outs[1])


def test_layouts_and_autotune_give_identical_results():
    groups = W.scaled("batched_2d", walkers_per_group=40)["groups"] + [(3, 16, 205, 20)]
    outs = []
    for variant in VARIANTS + [None]:
        ctx = make_ctx(groups, 3, variant)
        lnW = dev_f64(W.random_lnW(ctx.total_bins, seed=21, scale=0.4))
        H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
        if variant is None:
            chosen, ms = ctx.autotune(lnW, probe_sweeps=2)
            say("autotune chose", chosen, ms)
            assert chosen in M.LAYOUTS and ctx.layout() == chosen
        ctx.sweep(lnW, 6, H)
        states = [ctx.read_walker(w) for w in range(0, ctx.nwalkers, 7)]
        outs.append((H.cpu().numpy(), states))
        ctx.close()
    for H, st in outs[1:]:
        assert np.array_equal(H, outs[0][0])
        assert st == outs[0][1]


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
def test_run_graph_and_eager_match_oracle_across_calls(graph):
    """mucaRun replays a captured iteration; several calls in a row (with
    the caller's own work in between) must equal the eager path and the
    oracle every time."""
    groups = [(2, 8, 16, 24), (3, 5, 12, 9)]
    ctx = make_ctx(groups, 13)
    ctx.set_graph(graph)
    ref = O.RefContext(groups, 13)
    glnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=DEV)
    gP = torch.zeros_like(glnW)
    gH = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    lnW = np.zeros(ctx.total_bins)
    for call in range(3):
        scratch = torch.ones(1 << 20, device=DEV) * 2.0  # unrelated eager work
        rc, it, fl = ctx.run(glnW, gP, gH, 20, 3, 0, False)
        P = np.zeros(ctx.total_bins)  # mucaRun restarts the accumulator
        rrc, rH, rit, rfl = ref.run(lnW, P, 20, 3, 0, False)
        torch.cuda.synchronize()
        assert float(scratch.sum()) == 2.0 * (1 << 20)
        assert rc == rrc and list(it) == list(rit)
        assert np.array_equal(gH.cpu().numpy(), rH), call
        assert same_f64(glnW.cpu().numpy(), lnW), call
        assert same_f64(gP.cpu().numpy(), P), call


def test_run_resumed_in_chunks_equals_one_run():
    """Splitting a flat-terminated run into several resumed calls gives the
    same weights, histograms and iteration counts as one call (and the
    oracle)."""
    rc1, it1, fl1 = _run_both(FLAT_GROUPS, 5, 50, 80, rule=0, stop_on_flat=True)
    ctx = make_ctx(FLAT_GROUPS, 5)
    glnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=DEV)
    gP = torch.zeros_like(glnW)
    gH = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    ref = O.RefContext(FLAT_GROUPS, 5)
    lnW, P = np.zeros(ctx.total_bins), np.zeros(ctx.total_bins)
    rrc, rH, rit, rfl = ref.run(lnW, P, 50, 80, 0, True)
    done = 0
    rc = None
    while done < 80:
        rc, it, fl = ctx.run(glnW, gP, gH, 50, 3, 0, True, resume=done > 0)
        done += 3
        if rc == 0:
            break
    assert rc == rrc == 0
    assert list(it) == list(rit) == list(it1) and list(fl) == list(rfl)
    assert np.array_equal(gH.cpu().numpy(), rH)
    assert same_f64(glnW.cpu().numpy(), lnW) and same_f64(gP.cpu().numpy(), P)


@pytest.mark.parametrize("layout", [M.MUCA_LAYOUT_SUB16, M.MUCA_LAYOUT_SUB16X2])
def test_resident_cap_rounds_match_oracle(layout):
    """Walker state in device memory with more than two sets per CU: a
    resident cap of one byte leaves one block per CU (the sets run in rounds,
    two or more per block), no cap and the default cap two or more blocks per
    CU; all equal the oracle."""
    groups = [(2, 8, 16, 8300), (3, 8, 30, 300)]  # 538 sets of 16 (SUB16)
    ref = O.RefContext(groups, seed=12)
    lnW = W.random_lnW(ref.total_bins, seed=13, scale=0.8)
    rH = ref.sweep(lnW, 4)
    for cap in (1, 0, 234881024):
        say("resident cap", cap, "layout", layout)
        ctx = make_ctx(groups, 12, (layout, 0))
        ctx.set_resident_limit(cap)
        assert ctx.resident_limit() == cap
        assert ctx.placement() == (False, False)
        H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
        ctx.sweep(dev_f64(lnW), 4, H)
        torch.cuda.synchronize()
        assert np.array_equal(H.cpu().numpy(), rH), cap
        assert_walkers_equal(ctx, ref, list(range(0, ctx.nwalkers, 97)) + [ctx.nwalkers - 1])
        ctx.close()


def test_placement_reports_where_state_lives():
    ctx = M.Context([(2, 8, 16, 40)], seed=1)
    ctx.set_layout(M.MUCA_LAYOUT_SUB16)
    assert ctx.placement() == (True, True)
    ctx.set_lds_limit(0)
    assert ctx.placement() == (False, False)
    ctx.set_layout(M.MUCA_LAYOUT_LANE)
    assert ctx.placement() == (False, False)
    ctx.close()
    big = M.Context([(3, 48, 3318, 16)], seed=1)  # bricked: device memory in every layout
    for lay in (M.MUCA_LAYOUT_SUB16, M.MUCA_LAYOUT_SUB16X2, M.MUCA_LAYOUT_SUB64):
        big.set_layout(lay)
        assert big.placement() == (False, False)
    big.close()


def test_random_line_calibration_reads_every_line_it_counts():
    """mucaCalibrateRandomLines on a table of ones: every lane folds 8 loads
    per round, so each sink word is 8 x rounds; bad arguments are refused."""
    table = torch.ones((1 << 20) // 4, dtype=torch.int32, device=DEV)  # 8192 lines
    sink = torch.zeros(512 * 256, dtype=torch.int32, device=DEV)
    lines, sec = M.calibrate_random_lines(table, sink, 5)
    assert lines == 512 * 256 * 8 * 5 and sec > 0
    assert int((sink != 40).sum().item()) == 0
    with pytest.raises(M.MucaError):
        M.calibrate_random_lines(table[:8], sink, 5)  # less than one 128-byte line
    with pytest.raises(M.MucaError):
        M.calibrate_random_lines(table, sink[:100], 5)
