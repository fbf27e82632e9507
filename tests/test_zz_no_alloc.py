"""GPU test of mucaSweepNoAlloc, the sweep whose threshold and task tables
live in the library's static device workspace: through the C ABI, its
histograms and walker states equal those of mucaSweep on a twin context (same
groups, seed and weights), bit for bit, on two calls in a row (the second
with a smaller context, so stale workspace contents would show), in every
layout and with bricked device-memory state; a context whose tables exceed
the workspace is refused before any device work."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1401_4076_amd.muca")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def twins(groups, seed):
    return M.Context(groups, seed), M.Context(groups, seed)


def compare(a, b, H_a, H_b):
    torch.cuda.synchronize()
    assert np.array_equal(H_a.cpu().numpy(), H_b.cpu().numpy())
    for w in range(a.nwalkers):
        assert a.read_walker(w) == b.read_walker(w), w
    assert a.tunnel() == b.tunnel()


def sweep_pair(groups, seed, layout, sweeps, lnW_seed):
    a, b = twins(groups, seed)
    for c in (a, b):
        c.set_layout(layout)
    lnW = torch.tensor(W.random_lnW(a.total_bins, lnW_seed, scale=0.5), dtype=torch.float64,
                       device=DEV)
    H_a = torch.full((a.total_bins,), -7, dtype=torch.int32, device=DEV)
    H_b = torch.full((a.total_bins,), -7, dtype=torch.int32, device=DEV)
    a.sweep(lnW, sweeps, H_a)
    b.sweep_noalloc(lnW, sweeps, H_b)
    compare(a, b, H_a, H_b)
    assert int(H_b.sum().item()) == a.nwalkers * sweeps
    # the state carries over: a second sweep of both continues identically
    a.sweep(lnW, 3, H_a)
    b.sweep_noalloc(lnW, 3, H_b)
    compare(a, b, H_a, H_b)
    a.close()
    b.close()


BIG = [(2, 16, 40, 37), (3, 8, 30, 21), (2, 12, 20, 9), (3, 6, 11, 40)]
SMALL = [(2, 8, 16, 5)]


@pytest.mark.parametrize("layout", M.LAYOUTS)
def test_noalloc_sweep_matches_sweep_on_two_calls(layout):
    say(f"no-alloc sweep, layout {layout}: larger context, then a smaller one")
    sweep_pair(BIG, 1, layout, 20, 3)
    sweep_pair(SMALL, 2, layout, 7, 4)


@pytest.mark.parametrize("layout", [M.MUCA_LAYOUT_SUB16, M.MUCA_LAYOUT_SUB16X2,
                                    M.MUCA_LAYOUT_SUB64])
def test_noalloc_sweep_with_bricked_device_state(layout):
    say(f"no-alloc sweep, bricked state, layout {layout}")
    sweep_pair([(3, 16, 1300, 6), (2, 10, 12, 7)], 5, layout, 2, 6)
    sweep_pair(SMALL, 2, layout, 3, 4)


def test_noalloc_sweep_refuses_tables_beyond_the_workspace():
    # 90001 bins x 13 entries x 4 bytes > 4 MiB of workspace
    ctx = M.Context([(3, 64, 30000, 1, -90000, 0)], 1)
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=DEV)
    H = torch.full((ctx.total_bins,), -7, dtype=torch.int32, device=DEV)
    with pytest.raises(M.MucaError) as e:
        ctx.sweep_noalloc(lnW, 1, H)
    assert e.value.code == M.MUCA_EINVAL
    assert "workspace" in str(e.value)
    torch.cuda.synchronize()
    assert int((H != -7).sum().item()) == 0  # refused before any device work
    ctx.close()
