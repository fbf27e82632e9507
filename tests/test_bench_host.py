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


def test_cpu_sample_is_a_prefix_of_the_walkers():
    groups = [(3, 48, 3318, 16384)]
    n = bench.sample_walkers(groups, 1e8)
    assert n == 905  # ceil(1e8 / 48^3)
    assert bench.first_walkers(groups, n) == [(3, 48, 3318, 905)]
    mixed = [(2, 8, 16, 3), (3, 4, 6, 2, -10, 0), (2, 6, 9, 4)]
    assert bench.first_walkers(mixed, 4) == [(2, 8, 16, 3), (3, 4, 6, 1, -10, 0)]
    assert bench.sample_walkers(mixed, 1) == 1
    assert bench.sample_walkers(mixed, 1e12) == 9


def test_per_attempt_counts_follow_the_algorithm():
    # 3D at rho = 0.03: Philox block (110), 3 draws (12), 12 neighbour indices
    # (36), 12 bit tests (24), two 3D coordinate splits (24), decision (8)
    assert abs(bench.valu_ops_per_attempt(3, 0.0) - 214.0) < 1e-9
    assert abs(bench.valu_ops_per_attempt(2, 0.0) - 182.0) < 1e-9
    # pos[k], candidate word, 2 x 2d neighbour words, threshold entry
    assert abs(bench.state_bytes_per_attempt(3, 0.0) - 60.0) < 1e-9
    assert abs(bench.state_bytes_per_attempt(2, 0.5) - 48.0) < 1e-9
    g = [(3, 48, 3318, 10), (2, 8, 16, 10)]
    mean = bench._weighted(g, bench.valu_ops_per_attempt)
    lo, hi = bench.valu_ops_per_attempt(2, 0.25), bench.valu_ops_per_attempt(3, 0.03)
    assert min(lo, hi) < mean < max(lo, hi)


def test_bench_record_of_a_large_3d_run():
    """The JSON record of a timed run, from the figures of a driver-style run
    on the large 3D workload (20 steps of 2388.83 ms, sweep launch 2387.30 ms,
    456.20 counter bytes per attempt): the contract's keys, the value, the
    roofline against HBM and the moved bytes against the random-line ceiling."""
    import json
    groups = [(3, 48, 3318, 16384)]
    per_step = 16384 * 16 * 48 ** 3
    r = bench.bench_record("large_3d", groups, 16, 20, 5, 20 * 2.38883436185, 2387.30303955,
                           2, False, False, 234881024, None, 456.2014152849162 * per_step)
    json.dumps(r)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in r, k
    assert r["config"]["workload"] == "large_3d" and r["config"]["attempts_per_step"] == per_step
    assert abs(r["value"] / 1.2136056694e10 - 1) < 1e-9
    assert abs(r["ms_per_step"] - 2388.83436185) < 1e-6
    roof = r["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - 0.0912666) < 1e-6
    assert abs(roof["achieved"] / roof["peak"] - roof["frac"]) < 1e-12
    assert abs(roof["traffic_per_attempt"] - 456.2014152849162) < 1e-9
    assert abs(roof["moved"]["frac_of_random_line_peak"] - 0.84195) < 1e-4
    assert roof["lds"]["frac"] == 0.0 and abs(roof["valu"]["frac"] - 0.0661220) < 1e-6
    assert abs(r["sweep_attempts_per_s"] * 2.38730303955 - per_step) < 1.0


def test_bench_record_with_state_in_lds():
    """LDS-resident walker state: bound by the VALU, no HBM or moved entry."""
    groups = [(2, 64, 205, 4096)]
    r = bench.bench_record("x", groups, 100, 3, 1, 3.0, 900.0, 5, True, True, 0, [0.0], None)
    roof = r["roofline"]
    assert roof["bound"] == "alu" and roof["traffic"] is None and "moved" not in roof
    assert roof["hbm"]["frac"] == 0.0 and roof["lds"]["frac"] > 0.0
    assert abs(roof["frac"] - roof["valu"]["frac"]) < 1e-15
