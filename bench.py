"""Benchmark of the MUCA iteration on one MI355X.

One step = one iteration of the parallel multicanonical method (paper
Sec. 2) over the whole batch of walkers: acceptance thresholds from lnW,
`sweeps` sweeps of every walker (histogram fill and sum, eq. (2)), flatness
test and the binary64 weight recursion.  The default workload is the large
3D lattice gas: L = 48, rho = 0.03 (N = 3318), 16384 walkers, starting from
flat weights, 16 sweeps per walker per iteration (the rate does not depend on
the sweep count: the per-iteration work outside the sweep takes well under a
millisecond); inputs are synthetic and resident in device memory when timing
starts.

Prints one JSON line: move attempts/s (attempts = sum over walkers of
sweeps x L^d, accepted or not), the roofline of the sweep kernel (device
memory when the walker state lives there, else the VALU), with the VALU, HBM
and LDS fractions from per-attempt algorithmic counts, and the CPU oracle's
rate on a bounded sample of the same workload, on one core and on all the
host cores the process may use.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

# MI355X peaks: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz full-rate 32-bit VALU
# lane-ops/s; HBM3E 8 TB/s; LDS 128 bytes per clock per CU.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12
LDS_PEAK = 256 * 128 * 2.4e9
# Measured rate of random whole 128-byte line reads from HBM on MI355X
# (bench.py --calibrate-random-lines 4294967296): the ceiling of the sweeps
# whose walker state lives in device memory.
RANDOM_LINE_PEAK = 6.58e12

# One Philox4x32-10 block: 10 rounds of two 32x32->64 products (quarter rate:
# 4 full-rate lane-op equivalents each), two three-input XORs and the key
# schedule.
PHILOX_OPS = 10 * (2 * 4 + 2 + 1)

BENCH_SWEEPS = {"large_3d": 16, "batched_3d": 16}


def attempts_per_sweep(groups):
    return sum(g[3] * g[1] ** g[0] for g in groups)


def _weighted(groups, f):
    """Walker-and-site weighted mean of f(d, rho) over the groups."""
    tot = attempts_per_sweep(groups)
    return sum(g[3] * g[1] ** g[0] * f(g[0], g[2] / g[1] ** g[0]) for g in groups) / tot


def valu_ops_per_attempt(d, rho):
    """Algorithmic full-rate 32-bit lane-ops of one attempt: Philox blocks
    (block 0 always, further blocks when both candidate sites are occupied,
    a geometric number with mean rho^2/(1 - rho)), three multiply-shift draws
    (quarter-rate products), 3 ops per neighbour index of s_o and s_n (edge
    compare, select, add: 4d sites), 2 per bit test (word index, bit extract:
    4d sites), 6 per site-to-coordinate division for two sites (d - 1 each),
    and 8 for the energy change, window check and threshold compare."""
    return (PHILOX_OPS * (1.0 + rho * rho / (1.0 - rho)) + 3 * 4 + 3 * 4 * d + 2 * 4 * d +
            6 * (d - 1) * 2 + 8)


def state_bytes_per_attempt(d, rho):
    """Algorithmic bytes of walker state an attempt reads: the particle's site
    pos[k] (4), the occupation words of the candidate sites until an empty one
    (4 / (1 - rho)), one word per neighbour of s_o and of s_n (2 x 2d x 4) and
    the threshold entry (4).  Writes of accepted moves (two words and pos[k])
    are not counted: a lower bound."""
    return 4 + 4.0 / (1.0 - rho) + 2 * 2 * d * 4 + 4


def measured_traffic(workload, kernel_layout, attempts):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs
    (profiles/sweep_traffic.json: bytes per attempt), or None when the kernel
    source has changed since the counters were taken or another kernel ran."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(workload)
    if not rec:
        return None
    csrc = os.path.join(ROOT, "paper_1401_4076_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, n), "rb").read()
                   for n in ("muca_sweep_sub.hip", "muca_device.h"))
    if hashlib.sha256(src).hexdigest() != rec["kernel_source_sha256"]:
        return None
    if rec.get("layout") != kernel_layout:
        return None
    return rec["bytes_per_attempt"] * attempts


def bench_record(workload, groups, sweeps, steps, warmup, seconds, sweep_ms, layout, state_lds,
                 table_lds, resident_limit, tune_ms, traffic):
    """The JSON record of a timed run (host arithmetic only): `steps`
    iterations took `seconds` in all and the sweep launch `sweep_ms` on
    average; traffic = counter bytes per launch or None."""
    per_step = attempts_per_sweep(groups) * sweeps
    value = per_step * steps / seconds
    kernel_rate = per_step / (sweep_ms * 1e-3)  # attempts/s inside the sweep launch
    ops = _weighted(groups, valu_ops_per_attempt)
    sbytes = _weighted(groups, state_bytes_per_attempt)
    valu = {"achieved": ops * kernel_rate, "peak": VALU_PEAK_OPS, "unit": "int32 lane-op/s",
            "frac": ops * kernel_rate / VALU_PEAK_OPS, "per_attempt": ops}
    # the walker state is read from device memory or from LDS, not both
    state_rate = sbytes * kernel_rate
    hbm = {"achieved": 0.0 if state_lds else state_rate, "peak": HBM_PEAK, "unit": "B/s",
           "per_attempt": 0.0 if state_lds else sbytes}
    hbm["frac"] = hbm["achieved"] / HBM_PEAK
    lds = {"achieved": state_rate if state_lds else 0.0, "peak": LDS_PEAK, "unit": "B/s",
           "per_attempt": sbytes if state_lds else 0.0}
    lds["frac"] = lds["achieved"] / LDS_PEAK
    if state_lds:
        roof = {"bound": "alu", "achieved": valu["achieved"], "peak": VALU_PEAK_OPS,
                "unit": "int32 lane-op/s", "frac": valu["frac"], "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": hbm["achieved"] / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": hbm["frac"], "traffic": traffic}
    roof.update({"valu": valu, "hbm": hbm, "lds": lds,
                 "traffic_per_attempt": None if traffic is None else traffic / per_step})
    if traffic is not None and not state_lds:
        moved = traffic / (sweep_ms * 1e-3)  # counter bytes per second of the launch
        roof["moved"] = {"achieved": moved, "unit": "B/s",
                         "random_line_peak": RANDOM_LINE_PEAK,
                         "frac_of_random_line_peak": moved / RANDOM_LINE_PEAK}
    return {
        "metric": "move attempts/s on 1 GPU",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": seconds * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": workload, "groups": [list(g) for g in groups],
                   "walkers": sum(g[3] for g in groups), "sweeps_per_iter": sweeps,
                   "attempts_per_step": per_step, "rule": "berg", "layout": layout,
                   "state_in_lds": state_lds, "table_in_lds": table_lds,
                   "resident_limit_bytes": resident_limit,
                   "autotune_probe_ms": tune_ms},
        "sweep_kernel_ms": sweep_ms,
        "sweep_attempts_per_s": kernel_rate,  # attempts / sweep-phase time (value: whole steps)
        "roofline": roof,
    }


def cpu_threads():
    """Host cores for the oracle: the process's CPU set, at most 16 (one
    GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def split_walkers(groups, parts):
    """Split the global walker ids into `parts` contiguous ranges of about
    equal work (walkers x L^d); returns (groups of the range, first id) per
    non-empty range, ids and therefore random streams unchanged."""
    total = sum(g[3] for g in groups)
    work = np.concatenate([np.full(g[3], g[1] ** g[0], dtype=np.float64) for g in groups])
    cum = np.concatenate([[0.0], np.cumsum(work)])
    cuts = [int(np.searchsorted(cum, cum[-1] * i / parts)) for i in range(parts)] + [total]
    out = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        sub, first = [], 0
        for g in groups:
            lo, hi = max(a, first), min(b, first + g[3])
            if lo < hi:
                sub.append(tuple(g[:3]) + (hi - lo,) + tuple(g[4:]))
            first += g[3]
        if sub:
            out.append((sub, a))
    return out


def first_walkers(groups, n):
    """The groups restricted to global walker ids [0, n)."""
    out, left = [], n
    for g in groups:
        if left <= 0:
            break
        k = min(left, g[3])
        out.append(tuple(g[:3]) + (k,) + tuple(g[4:]))
        left -= k
    return out


def sample_walkers(groups, target_attempts):
    """Walkers (a prefix of the global ids, at least one) whose single sweep
    makes about target_attempts attempts."""
    total = sum(g[3] for g in groups)
    n = 0
    acc = 0
    for g in groups:
        for _ in range(g[3]):
            if n > 0 and acc >= target_attempts:
                return n
            acc += g[1] ** g[0]
            n += 1
    return total


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(groups, seed, threads, per_thread_attempts=6.0e7):
    """The oracle on the host: one sweep of a prefix of the walkers on one
    core, then one sweep of a larger prefix split over `threads` threads, one
    oracle instance per thread over disjoint ranges of global walker ids (the
    paper's one-process-per-core scheme).  The oracle is C called through
    ctypes, which releases the GIL, so the instances run in parallel."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor

    n1 = sample_walkers(groups, per_thread_attempts)
    one = first_walkers(groups, n1)
    r = O.RefContext(one, seed)
    t0 = time.perf_counter()
    H = r.sweep(np.zeros(r.total_bins), 1)
    dt1 = time.perf_counter() - t0
    assert int(H.sum()) == n1
    a1 = attempts_per_sweep(one)
    r.close()

    nall = sample_walkers(groups, per_thread_attempts * threads)
    allg = first_walkers(groups, nall)
    refs = [O.RefContext(sub, seed, first_id=a) for sub, a in split_walkers(allg, threads)]
    lnWs = [np.zeros(x.total_bins) for x in refs]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(len(refs)) as ex:
        Hs = list(ex.map(lambda i: refs[i].sweep(lnWs[i], 1), range(len(refs))))
    dt = time.perf_counter() - t0
    assert sum(int(h.sum()) for h in Hs) == nall
    a = attempts_per_sweep(allg)
    for x in refs:
        x.close()
    return {"value": a / dt, "unit": "attempts/s", "cores": len(refs), "kind": "oracle",
            "single_core_value": a1 / dt1,
            "sample": f"one sweep of walkers 0..{nall - 1} ({a:.3g} attempts, flat weights) "
                      f"in {dt:.1f} s on {len(refs)} threads, one oracle instance per thread "
                      f"over disjoint walker ranges; single core: one sweep of walkers "
                      f"0..{n1 - 1} ({a1:.3g} attempts) in {dt1:.1f} s ({cpu_model()})"}


def calibrate_copy(nbytes):
    """A plain device copy of known size (for scaling HBM byte counters)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def calibrate_random_lines(table_bytes, rounds=256):
    """The device's rate of random whole-line reads (mucaCalibrateRandomLines):
    8 independent random 128-byte lines per lane and round, 2048 blocks of
    256 lanes.  Prints lines/s and the bytes of those lines per second."""
    import torch
    from paper_1401_4076_amd import muca as M
    table = torch.ones(table_bytes // 4, dtype=torch.int32, device="cuda")
    sink = torch.zeros(2048 * 256, dtype=torch.int32, device="cuda")
    lines, sec = M.calibrate_random_lines(table, sink, rounds)
    print(json.dumps({"table_bytes": table_bytes, "lines": lines, "seconds": sec,
                      "lines_per_s": lines / sec, "line_GBps": lines * 128 / sec / 1e9}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large_3d", choices=sorted(W.WORKLOADS))
    ap.add_argument("--sweeps", type=int, default=None, help="sweeps per iteration")
    ap.add_argument("--layout", type=int, default=0,
                    help="0: autotune, else a MUCA_LAYOUT_* index (1 lane, 2 16 lanes/walker, "
                         "3 64 lanes/walker, 4 lookahead, 5/6 16 lanes with 2/1 walkers "
                         "per wavefront)")
    ap.add_argument("--probe-sweeps", type=int, default=1, help="autotune probe length")
    ap.add_argument("--resident-mib", type=int, default=None,
                    help="with --layout: cap of the walker state in flight when it lives in "
                         "device memory (MiB, 0 = none; default: the library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES")
    ap.add_argument("--calibrate-random-lines", type=int, default=0, metavar="TABLE_BYTES",
                    help="time random 128-byte row gathers from a table of this size")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of walkers is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.calibrate_random_lines:
        calibrate_random_lines(args.calibrate_random_lines)
        return

    import torch
    from paper_1401_4076_amd import muca as M

    wl = W.WORKLOADS[args.workload]
    groups, seed = wl["groups"], wl["seed"]
    sweeps = args.sweeps or BENCH_SWEEPS.get(args.workload, wl["sweeps"])
    print(f"bench: workload={args.workload} groups={groups} sweeps={sweeps} "
          f"steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    ctx = M.Context(groups, seed)
    dev = torch.device("cuda")
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=dev)
    tune_ms = None
    if args.layout == 0:
        # state-preserving: the probes do not change any later result
        chosen, tune_ms = ctx.autotune(lnW, probe_sweeps=min(args.probe_sweeps, sweeps))
        print(f"bench: autotune chose layout {chosen} (probe ms per layout {tune_ms[1:]})",
              file=sys.stderr, flush=True)
    else:
        ctx.set_layout(args.layout)
        if args.resident_mib is not None:
            ctx.set_resident_limit(args.resident_mib << 20)
    state_lds, table_lds = ctx.placement()
    P = torch.zeros_like(lnW)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=dev)
    flags = torch.zeros(ctx.ngroups, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    ev = []

    def step(timed):
        if timed:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
        ctx.sweep(lnW, sweeps, H, stream=stream)  # thresholds + sweep kernel
        if timed:
            b.record(stream)
            ev.append((a, b))
        ctx.is_flat(H, flags, stream=stream)
        ctx.update_weights(H, lnW, P, M.MUCA_RULE_BERG, stream=stream)

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        print(f"bench: warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        if args.steps > 1:
            torch.cuda.synchronize()  # progress line per step (steps last seconds)
            print(f"bench: step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.status(stream)

    sweep_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    traffic = measured_traffic(args.workload, ctx.layout(), attempts_per_sweep(groups) * sweeps)
    out = bench_record(args.workload, groups, sweeps, args.steps, args.warmup, t1 - t0, sweep_ms,
                       ctx.layout(), state_lds, table_lds, ctx.resident_limit(), tune_ms, traffic)
    if not args.no_cpu_baseline:
        nt = cpu_threads()
        print(f"bench: CPU oracle sample on 1 and {nt} threads", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(groups, seed, nt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
