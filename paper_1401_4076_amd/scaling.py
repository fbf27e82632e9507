"""Speed-up of the parallel iteration with the number of walkers (Sec. 4).

The paper's protocol: a fixed total of 25600 sweeps per iteration shared by
the p processes (25600/p sweeps each), the recursion started from flat
weights, a run converged once its processes made 30 tunnelling events in
total (trips from the top of the energy range to the bottom or back), 32
independent runs per p.  Here a process is a walker and the 32 runs of one
p are the groups of one context: the same lattice, disjoint walker ids
(independent random streams), all advanced together on the GPU, each group
stopping on its own (mucaRun with MUCA_STOP_TUNNEL).

Speed-up S_p = t_1 / t_p with t_p the time of one run to convergence.  The
p walkers of a run sweep in parallel and exchange data only at the end of
an iteration, so t_p is proportional to iterations x 25600 / p sweeps of one
walker and S_p = p x (mean iterations at p = 1) / (mean iterations at p).
The GPU wall time of each batch of runs is reported beside it.

Prints progress to stderr and one JSON line.

    python -m paper_1401_4076_amd.scaling --d 2 --L 16 --N 20 --p 1,2,4,8,16,32,64,128
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402

from paper_1401_4076_amd import muca as M  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def speedups(results):
    """S_p = p x (mean iterations at p = 1) / (mean iterations at p) per result,
    or None for all when p = 1 was not run."""
    base = next((r for r in results if r["p"] == 1), None)
    if base is None:
        return [None] * len(results)
    return [r["p"] * base["iters_mean"] / r["iters_mean"] for r in results]


def runs_for(d, L, N, p, runs, seed, total_sweeps, target, max_iters, chunk, rule,
             max_seconds=None):
    """The runs of one p, all in one context; returns a summary dict."""
    if total_sweeps % p:
        raise ValueError(f"{total_sweeps} sweeps per iteration do not split over {p} walkers")
    sweeps = total_sweeps // p
    groups = [(d, L, N, p)] * runs
    ctx = M.Context(groups, seed)
    ctx.set_tunnel_target(target)
    dev = torch.device("cuda")
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=dev)
    P = torch.zeros_like(lnW)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, rc, it = 0, None, []
    while done < max_iters:
        n = min(chunk, max_iters - done)
        rc, it, fl = ctx.run(lnW, P, H, sweeps, n, rule, stop=M.MUCA_STOP_TUNNEL,
                             resume=done > 0)
        done += n
        trips = ctx.tunnel()[1]
        per_run = [sum(trips[r * p:(r + 1) * p]) for r in range(runs)]
        ok = sum(1 for x in per_run if x >= target)
        log(f"  p={p}: {done} iterations, {ok}/{runs} runs converged, "
            f"{time.perf_counter() - t0:.1f} s")
        if rc == M.MUCA_OK:
            break
        if max_seconds is not None and time.perf_counter() - t0 > max_seconds:
            break
    seconds = time.perf_counter() - t0
    trips = ctx.tunnel()[1]
    per_run = [sum(trips[r * p:(r + 1) * p]) for r in range(runs)]
    conv = [x >= target for x in per_run]
    its = [it[r] for r in range(runs) if conv[r]]
    ctx.close()
    mean = sum(its) / len(its) if its else float("nan")
    sem = (math.sqrt(sum((x - mean) ** 2 for x in its) / (len(its) - 1) / len(its))
           if len(its) > 1 else float("nan"))
    return {"p": p, "sweeps_per_walker": sweeps, "runs": runs, "converged": sum(conv),
            "iters": list(it), "iters_mean": mean, "iters_sem": sem, "trips": per_run,
            "gpu_seconds": seconds}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--L", type=int, default=16)
    ap.add_argument("--N", type=int, default=20)
    ap.add_argument("--p", default="1,2,4,8,16,32,64,128", help="walkers per run, comma list")
    ap.add_argument("--runs", type=int, default=32, help="independent runs per p")
    ap.add_argument("--total-sweeps", type=int, default=25600, help="sweeps per iteration, shared")
    ap.add_argument("--target", type=int, default=30, help="tunnelling events to convergence")
    ap.add_argument("--max-iters", type=int, default=400)
    ap.add_argument("--chunk", type=int, default=10, help="iterations per mucaRun call")
    ap.add_argument("--rule", type=int, default=M.MUCA_RULE_BERG)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--max-seconds", type=float, default=None, help="per p, between chunks")
    args = ap.parse_args()

    ps = [int(x) for x in args.p.split(",")]
    lo, hi = M.mucaDefaultWindow(args.d, args.L, args.N)
    out = {"d": args.d, "L": args.L, "N": args.N, "window": [lo, hi], "runs": args.runs,
           "total_sweeps": args.total_sweeps, "target": args.target, "rule": args.rule,
           "seed": args.seed, "results": []}
    log(f"scaling: d={args.d} L={args.L} N={args.N} window [{lo}, {hi}], runs {args.runs}, "
        f"{args.total_sweeps} sweeps per iteration, target {args.target}")
    for p in ps:
        res = runs_for(args.d, args.L, args.N, p, args.runs, args.seed, args.total_sweeps,
                       args.target, args.max_iters, args.chunk, args.rule, args.max_seconds)
        out["results"].append(res)
        log(f"p={p}: {res['converged']}/{args.runs} converged, mean iterations "
            f"{res['iters_mean']:.2f} +- {res['iters_sem']:.2f}, {res['gpu_seconds']:.1f} s")
    for r, sp in zip(out["results"], speedups(out["results"])):
        if sp is not None:
            r["speedup"] = sp
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
