"""Host logic of bench.py: the --gpus contract and the walker split of the
all-cores oracle baseline (each range keeps its global ids, so the summed
histograms equal one context's, as when the paper's processes each run a
share of the walkers)."""
import subprocess
import sys
import os

import numpy as np

import bench
import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_split_walkers_covers_every_id_once():
    groups = [(2, 32, 51, 683), (2, 64, 410, 682), (3, 8, 20, 5, -40, 0)]
    for parts in (1, 2, 3, 7, 16):
        ranges = bench.split_walkers(groups, parts)
        ids = []
        for sub, first in ranges:
            ids += list(range(first, first + sum(g[3] for g in sub)))
        assert ids == list(range(sum(g[3] for g in groups)))
        # the groups of a range keep (d, L, N) and any explicit window
        for sub, _ in ranges:
            for g in sub:
                assert any(g[:3] == h[:3] and g[4:] == h[4:] for h in groups)


def test_split_walkers_balances_work():
    groups = [(2, 32, 51, 600), (2, 64, 410, 600)]
    ranges = bench.split_walkers(groups, 4)
    work = [sum(g[3] * g[1] ** g[0] for g in sub) for sub, _ in ranges]
    assert max(work) <= 1.05 * min(work)


def test_split_runs_sum_to_one_context():
    groups = [(2, 8, 16, 5), (3, 4, 6, 3), (2, 6, 9, 4)]
    whole = O.RefContext(groups, seed=3)
    H = whole.sweep(np.zeros(whole.total_bins), 4)
    parts = bench.split_walkers(groups, 3)
    Hs = np.zeros_like(H)
    for sub, first in parts:
        r = O.RefContext(sub, seed=3, first_id=first)
        h = r.sweep(np.zeros(r.total_bins), 4)
        # scatter the range's groups back into the whole context's bins
        for gi, g in enumerate(sub):
            j = next(k for k, x in enumerate(groups) if x[:3] == g[:3])
            lo, hi = r.window(gi)
            Hs[whole.bin_offset(j):whole.bin_offset(j) + hi - lo + 1] += \
                h[r.bin_offset(gi):r.bin_offset(gi) + hi - lo + 1]
    assert np.array_equal(Hs, H)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
