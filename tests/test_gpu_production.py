"""GPU parity of the production run with the energy-binned droplet
measurement (mucaProduction, mucaMeasureDroplets) and of the canonical
reweighting of the measured observable (mucaReweightObservable), through the
C ABI, against the oracle: the oracle sweeps the same walkers with the same
weights, measures each walker's largest droplet by its own search at every
measurement sweep and bins it by the walker's energy (integer sums: exact);
oracle/reweight_ref.reweight_observable reweights the same sums.

Reweighting tolerance (binary64 on both sides, different exp/log and
summation order): each weight exp(a - m) carries a relative error of a few
ulp and the average is a ratio of sums of positive terms, so its relative
error stays below bins x ulp ~ 1e4 x 1.1e-16: rtol 1e-11."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.droplet_ref import largest_cluster
from oracle.reweight_ref import reweight_observable

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")

pytestmark = pytest.mark.gpu

DEV = "cuda"
BETAS = [0.0, 0.3, 1 / 0.6995, 2.0, 1 / 0.375, 6.0]


def say(*a):
    print(*a, flush=True)


def oracle_production(ref, groups, lnW, between, rounds):
    H = np.zeros(ref.total_bins, dtype=np.int64)
    osum = np.zeros(ref.total_bins, dtype=np.int64)
    cnt = np.zeros(ref.total_bins, dtype=np.int64)
    for _ in range(rounds):
        H += ref.sweep(lnW, between)
        w = 0
        for gi, (d, L, N, walkers, *_r) in enumerate(groups):
            lo, hi = ref.window(gi)
            off = ref.bin_offset(gi)
            for _j in range(walkers):
                n, pos, E, t = ref.walker(w)
                osum[off + E - lo] += largest_cluster(n, d, L)
                cnt[off + E - lo] += 1
                w += 1
    return H, osum, cnt


@pytest.mark.parametrize("layout", [M.MUCA_LAYOUT_SUB16, M.MUCA_LAYOUT_LANE,
                                    M.MUCA_LAYOUT_SUB16X2])
def test_production_droplet_sums_match_oracle(layout):
    groups = [(2, 8, 16, 6), (3, 5, 12, 4), (2, 12, 30, 5), (3, 16, 1300, 2)]
    say(f"production, layout {layout}: {groups}")
    ctx = M.Context(groups, seed=9)
    ref = O.RefContext(groups, seed=9)
    ctx.set_layout(layout)
    lnW = W.random_lnW(ctx.total_bins, seed=10, scale=0.3)
    gl = torch.tensor(lnW, device=DEV)
    H = torch.full((ctx.total_bins,), -7, dtype=torch.int32, device=DEV)
    osum = torch.full((ctx.total_bins,), -7, dtype=torch.int64, device=DEV)
    cnt = torch.full((ctx.total_bins,), -7, dtype=torch.int32, device=DEV)
    ctx.production(gl, 3, 5, H, osum, cnt)
    rH, rosum, rcnt = oracle_production(ref, groups, lnW, 3, 5)
    assert np.array_equal(H.cpu().numpy(), rH)
    assert np.array_equal(osum.cpu().numpy(), rosum)
    assert np.array_equal(cnt.cpu().numpy(), rcnt)
    assert int(cnt.sum().item()) == 5 * ctx.nwalkers
    # the walker states carried on exactly as in the oracle
    for w in range(ctx.nwalkers):
        bits, pos, E, t = ctx.read_walker(w)
        n, rpos, rE, rt = ref.walker(w)
        assert (E, t) == (rE, rt) and np.array_equal(np.array(pos, np.uint32), rpos), w
    # reweighting of the measured droplet sizes
    gb = torch.tensor(np.asarray(BETAS, dtype=np.float64), device=DEV)
    out = torch.full((ctx.ngroups * len(BETAS),), -1.0, dtype=torch.float64, device=DEV)
    ctx.reweight_observable(gl, cnt, osum, gb, out)
    got = out.cpu().numpy().reshape(ctx.ngroups, len(BETAS))
    for gi in range(ctx.ngroups):
        lo, hi, off = ctx.window(gi)
        sl = slice(off, off + hi - lo + 1)
        want = reweight_observable(lnW[sl], rcnt[sl], rosum[sl], lo, BETAS)
        np.testing.assert_allclose(got[gi], want, rtol=1e-11, err_msg=f"group {gi}")
    ctx.close()


def test_reweight_observable_on_seeded_sums():
    """Seeded sums over long windows, a group without measurements (NaN)."""
    groups = [(2, 32, 102, 2), (3, 24, 415, 1), (2, 6, 4, 2, -3, 0), (3, 48, 3318, 1)]
    ctx = M.Context(groups, seed=3)
    lnW = W.random_lnW(ctx.total_bins, seed=4, scale=0.7)
    cnt = W.random_histogram(ctx.total_bins, seed=5)
    rng = np.random.default_rng(6)
    osum = (cnt.astype(np.int64) * rng.integers(1, 400, ctx.total_bins)).astype(np.int64)
    lo, hi, off = ctx.window(2)
    cnt[off:off + hi - lo + 1] = 0
    osum[off:off + hi - lo + 1] = 0
    out = torch.full((ctx.ngroups * len(BETAS),), -1.0, dtype=torch.float64, device=DEV)
    ctx.reweight_observable(torch.tensor(lnW, device=DEV),
                            torch.tensor(cnt, dtype=torch.int32, device=DEV),
                            torch.tensor(osum, device=DEV),
                            torch.tensor(np.asarray(BETAS), device=DEV), out)
    got = out.cpu().numpy().reshape(ctx.ngroups, len(BETAS))
    for gi in range(ctx.ngroups):
        lo, hi, off = ctx.window(gi)
        sl = slice(off, off + hi - lo + 1)
        want = reweight_observable(lnW[sl], cnt[sl], osum[sl], lo, BETAS)
        if np.isnan(want).all():
            assert np.isnan(got[gi]).all()
            continue
        np.testing.assert_allclose(got[gi], want, rtol=1e-11, err_msg=f"group {gi}")
    ctx.close()
