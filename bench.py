"""Benchmark of the MUCA iteration on one MI355X.

One step = one iteration of the parallel multicanonical method (paper
Sec. 2) over the whole batch of walkers: acceptance thresholds from lnW,
`sweeps` sweeps of every walker (histogram fill and sum, eq. (2)), flatness
test and the binary64 weight recursion.  The default workload is the batched
2D lattice gas: 6 groups (L, rho) in {32, 48, 64} x {0.05, 0.10}, 4096
walkers, 1e4 sweeps per iteration, starting from flat weights; inputs are
synthetic and resident in device memory when timing starts.

Prints one JSON line: move attempts/s (attempts = sum over walkers of
sweeps x L^d, accepted or not), the VALU roofline of the sweep kernel and
the CPU oracle's rate on a bounded sample of the same workload.
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

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz full-rate 32-bit VALU lane-ops/s
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# One Philox4x32-10 block: 10 rounds of two 32x32->64 products (quarter rate,
# 4 full-rate equivalents each) and two three-input XORs.
PHILOX_OPS = 10 * (2 * 4 + 2)


def attempts_per_sweep(groups):
    return sum(g[3] * g[1] ** g[0] for g in groups)


def philox_blocks_per_attempt(groups):
    """Expected Philox blocks per attempt (weighted over walkers): block 0
    always; block 1 when the first two candidate sites are occupied (~rho^2)."""
    tot = sum(g[3] * g[1] ** g[0] for g in groups)
    acc = 0.0
    for d, L, N, w, *_ in groups:
        rho = N / L ** d
        acc += w * L ** d * (1.0 + rho * rho / (1.0 - rho))
    return acc / tot


def measured_traffic(workload, kernel_layout):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs
    (profiles/sweep_traffic.json), or None when the kernel source has changed
    since the counters were taken or another kernel ran."""
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
    want = {2: "k_sweep_sub<16", 3: "k_sweep_sub<64", 5: "k_sweep_sub<16",
            6: "k_sweep_sub<16"}.get(kernel_layout)
    if want is None or want not in rec["kernel"]:
        return None
    return rec["traffic_bytes_per_launch"]


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(groups, seed, sample_sweeps, threads):
    """The oracle on the host, one instance per thread over disjoint ranges of
    global walker ids (the paper's one-process-per-core scheme).  The oracle
    is C called through ctypes, which releases the GIL, so the instances run
    in parallel."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    total = sum(g[3] for g in groups)
    refs = [O.RefContext(sub, seed, first_id=a) for sub, a in split_walkers(groups, threads)]
    lnWs = [np.zeros(r.total_bins) for r in refs]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(len(refs)) as ex:
        Hs = list(ex.map(lambda i: refs[i].sweep(lnWs[i], sample_sweeps), range(len(refs))))
    dt = time.perf_counter() - t0
    n = attempts_per_sweep(groups) * sample_sweeps
    assert sum(int(H.sum()) for H in Hs) == total * sample_sweeps
    return {"value": n / dt, "unit": "attempts/s", "cores": len(refs), "kind": "oracle",
            "sample": f"all {total} walkers x {sample_sweeps} sweeps ({n:.3g} attempts, flat "
                      f"weights) in {dt:.1f} s on {len(refs)} threads ({cpu_model()}), one "
                      f"oracle instance per thread over disjoint walker ranges"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched_2d", choices=sorted(W.WORKLOADS))
    ap.add_argument("--sweeps", type=int, default=None, help="sweeps per iteration")
    ap.add_argument("--layout", type=int, default=0,
                    help="0: autotune, else a MUCA_LAYOUT_* index (1 lane, 2 16 lanes/walker, "
                         "3 64 lanes/walker, 4 lookahead, 5/6 16 lanes with 2/1 walkers "
                         "per wavefront)")
    ap.add_argument("--probe-sweeps", type=int, default=20, help="autotune probe length")
    ap.add_argument("--cpu-sweeps", type=int, default=None,
                    help="sweeps of the CPU oracle sample (default: ~4e8 attempts)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of walkers is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import torch
    from paper_1401_4076_amd import muca as M

    wl = W.WORKLOADS[args.workload]
    groups, seed = wl["groups"], wl["seed"]
    sweeps = args.sweeps or wl["sweeps"]
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

    per_step = attempts_per_sweep(groups) * sweeps
    dt = t1 - t0
    value = per_step * args.steps / dt
    sweep_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ops = per_step * philox_blocks_per_attempt(groups) * PHILOX_OPS
    achieved = ops / (sweep_ms * 1e-3)
    out = {
        "metric": "move attempts/s on 1 GPU",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "groups": [list(g) for g in groups],
                   "walkers": sum(g[3] for g in groups), "sweeps_per_iter": sweeps,
                   "attempts_per_step": per_step, "rule": "berg", "layout": ctx.layout(),
                   "autotune_probe_ms": tune_ms},
        "sweep_kernel_ms": sweep_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_OPS,
                     "unit": "int32 lane-op/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": measured_traffic(args.workload, ctx.layout())},
    }
    if not args.no_cpu_baseline:
        cs = args.cpu_sweeps
        if cs is None:  # ~4e8 attempts: ~15-20 s of single-core oracle work
            cs = max(1, int(round(4e8 / attempts_per_sweep(groups))))
        nt = cpu_threads()
        print(f"bench: CPU oracle sample, {cs} sweeps of all walkers on {nt} threads",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(groups, seed, cs, nt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
