"""GPU parity of the canonical reweighting (mucaReweight, through the C ABI)
against the oracle's reweighting on the same seeded weights and histograms.

Tolerance (binary64 on both sides, different exp/log implementations and
summation orders): each weight exp(a - m) carries a relative error of a few
ulp, and the sums, means and ln Z are sums of positive terms, so their
relative error stays below (bins x ulp) ~ 1e4 x 1.1e-16; rtol 1e-11 (with an
absolute floor of 1e-11 x the largest |E| for values near zero).  The
specific heat is a weighted sum of (E - <E>)^2 about a mean that carries
that error itself: rtol 1e-9.
"""
import numpy as np
import pytest

import workloads as W
from oracle.reweight_ref import reweight

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")

pytestmark = pytest.mark.gpu

DEV = "cuda"
BETAS = [0.0, 0.1, 0.5, 1.0, 1 / 0.6995, 2.0, 5.0, 40.0]


def say(*a):
    print(*a, flush=True)


def _check(ctx, lnW, H, betas):
    gl = torch.tensor(lnW, device=DEV)
    gH = torch.tensor(H, dtype=torch.int32, device=DEV)
    gb = torch.tensor(np.asarray(betas, dtype=np.float64), device=DEV)
    out = torch.full((ctx.ngroups * len(betas) * 4,), -1.0, dtype=torch.float64, device=DEV)
    ctx.reweight(gl, gH, gb, out)
    got = out.cpu().numpy().reshape(ctx.ngroups, len(betas), 4)
    for g in range(ctx.ngroups):
        lo, hi, off = ctx.window(g)
        sl = slice(off, off + hi - lo + 1)
        ref = reweight(lnW[sl], H[sl], lo, betas)
        if np.isnan(ref).all():
            assert np.isnan(got[g]).all(), g
            continue
        scale = max(1.0, abs(lo))
        for j, rtol in enumerate((1e-11, 1e-11, 1e-11, 1e-9)):
            np.testing.assert_allclose(got[g, :, j], ref[:, j], rtol=rtol,
                                       atol=1e-11 * scale ** (2 if j >= 2 else 1),
                                       err_msg=f"group {g} column {j}")
    return got


def test_reweight_matches_oracle():
    groups = [(2, 8, 16, 4), (3, 5, 12, 3), (2, 6, 4, 2, -3, 0), (2, 32, 102, 2),
              (3, 24, 415, 1)]
    ctx = M.Context(groups, seed=3)
    lnW = W.random_lnW(ctx.total_bins, seed=4, scale=0.7)
    H = W.random_histogram(ctx.total_bins, seed=5)
    lo, hi, off = ctx.window(2)
    H[off:off + hi - lo + 1] = 0  # a group without visited bins
    say("reweight groups", groups, "bins", ctx.total_bins)
    _check(ctx, lnW, H, BETAS)


def test_reweight_after_production_run():
    """The intended use: a flat run's weights, a production histogram, then
    canonical averages; <E> falls from 0 toward the window bottom as beta
    grows and C stays non-negative."""
    groups = [(2, 8, 16, 64)]
    ctx = M.Context(groups, seed=5)
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=DEV)
    P = torch.zeros_like(lnW)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=DEV)
    rc, it, fl = ctx.run(lnW, P, H, 200, 100, M.MUCA_RULE_BERG, True)
    assert rc == M.MUCA_OK
    ctx.sweep(lnW, 2000, H)
    got = _check(ctx, lnW.cpu().numpy(), H.cpu().numpy().astype(np.int64), BETAS)
    mean = got[0, :, 1]
    assert (np.diff(mean) < 0).all() and (got[0, :, 3] >= 0).all()
    assert mean[-1] == pytest.approx(ctx.window(0)[0], abs=0.05)


def test_reweight_errors_and_timing():
    ctx = M.Context([(3, 48, 3318, 1)], seed=1)  # the large 3D window (~9300 bins)
    nb = 1000
    lnW = torch.tensor(W.random_lnW(ctx.total_bins, seed=1, scale=0.5), device=DEV)
    H = torch.tensor(W.random_histogram(ctx.total_bins, seed=2), device=DEV)
    beta = torch.linspace(0.0, 3.0, nb, dtype=torch.float64, device=DEV)
    out = torch.empty(4 * nb, dtype=torch.float64, device=DEV)
    with pytest.raises(M.MucaError) as e:
        M._check(M.lib().mucaReweight(ctx._h, None, None, None, 1, None, None))
    assert e.value.code == M.MUCA_EINVAL
    with pytest.raises(M.MucaError) as e:
        ctx.reweight(lnW, H, beta[:0], out)
    assert e.value.code == M.MUCA_EINVAL
    ctx.reweight(lnW, H, beta, out)  # warm
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        ctx.reweight(lnW, H, beta, out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / 10
    say(f"reweight: {ctx.total_bins} bins x {nb} beta in {ms:.3f} ms")
    ref = reweight(lnW.cpu().numpy(), H.cpu().numpy(), ctx.window(0)[0], beta[::97].cpu().numpy())
    got = out.cpu().numpy().reshape(nb, 4)[::97]
    np.testing.assert_allclose(got[:, :3], ref[:, :3], rtol=1e-11, atol=1e-7)
