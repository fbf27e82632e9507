"""Speed-up of the parallel iteration with the number of walkers (Sec. 4).

The paper's protocol: a fixed total of 25600 sweeps per iteration shared by
the p processes (25600/p sweeps each), the recursion started from flat
weights, a run converged once its processes made 30 tunnelling events in
total (trips from the top of the energy range to the bottom or back), 32
independent runs per p.  Here a process is a walker and the 32 runs of one
p are the groups of one context: the same lattice, disjoint walker ids
(independent random streams), all advanced together on the GPU, each group
stopping on its own (mucaRun with MUCA_STOP_TUNNEL).

Speed-up S_p = t_1 / t_p with t_p the time of one run to convergence
(Sec. 4, eq. (S_p)).  Each run's time is measured: the iteration is stepped
one iteration per call and a run's time is the wall time at the end of the
iteration in which it converged; t_p is the mean over the converged runs.
Beside it the iteration model: the p walkers of a run sweep in parallel and
exchange data only at the end of an iteration, so t_p is proportional to
iterations x 25600 / p sweeps of one walker and
S_p = p x (mean iterations at p = 1) / (mean iterations at p).  When p = 1
is not run, both are given relative to the smallest p that was
(S_p / S_p0, which is p / p0 for a linear speed-up).

Every p gets its own range of global walker ids (first id = the number of
walkers of the runs of all p before it), so no two runs of the whole study
share a random stream or an initial placement.

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
    """Per result: (iteration model, measured) speed-ups relative to the
    smallest p run, p0: S = (p / p0) x iters(p0) / iters(p) and
    S = t(p0) / t(p), each times S_p0 = p0 (normalised so that the linear
    speed-up is p)."""
    if not results:
        return []
    base = min(results, key=lambda r: r["p"])
    p0 = base["p"]
    out = []
    for r in results:
        model = r["p"] * base["iters_mean"] / r["iters_mean"]
        meas = p0 * base["seconds_mean"] / r["seconds_mean"]
        out.append((model, meas))
    return out


def runs_for(d, L, N, p, runs, seed, total_sweeps, target, max_iters, rule, first_id=0,
             max_seconds=None):
    """The runs of one p, all in one context (walker ids from first_id);
    returns a summary dict with each run's iterations and wall time to
    convergence."""
    if total_sweeps % p:
        raise ValueError(f"{total_sweeps} sweeps per iteration do not split over {p} walkers")
    sweeps = total_sweeps // p
    groups = [(d, L, N, p)] * runs
    ctx = M.Context(groups, seed, first_id=first_id)
    ctx.set_tunnel_target(target)
    dev = torch.device("cuda")
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=dev)
    P = torch.zeros_like(lnW)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, rc, it = 0, None, []
    run_seconds = [None] * runs
    while done < max_iters:
        rc, it, fl = ctx.run(lnW, P, H, sweeps, 1, rule, stop=M.MUCA_STOP_TUNNEL,
                             resume=done > 0)
        done += 1
        now = time.perf_counter() - t0
        trips = ctx.tunnel()[1]
        per_run = [sum(trips[r * p:(r + 1) * p]) for r in range(runs)]
        for r in range(runs):
            if run_seconds[r] is None and per_run[r] >= target:
                run_seconds[r] = now
        ok = sum(1 for x in run_seconds if x is not None)
        if done % 10 == 0 or rc == M.MUCA_OK:
            log(f"  p={p}: {done} iterations, {ok}/{runs} runs converged, {now:.1f} s")
        if rc == M.MUCA_OK:
            break
        if max_seconds is not None and now > max_seconds:
            break
    seconds = time.perf_counter() - t0
    trips = ctx.tunnel()[1]
    per_run = [sum(trips[r * p:(r + 1) * p]) for r in range(runs)]
    conv = [x >= target for x in per_run]
    its = [it[r] for r in range(runs) if conv[r]]
    secs = [run_seconds[r] for r in range(runs) if conv[r]]
    ctx.close()

    def mean_sem(v):
        if not v:
            return float("nan"), float("nan")
        m = sum(v) / len(v)
        e = math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v)) if len(v) > 1 \
            else float("nan")
        return m, e

    im, ie = mean_sem(its)
    sm, se = mean_sem(secs)
    return {"p": p, "sweeps_per_walker": sweeps, "runs": runs, "first_id": first_id,
            "converged": sum(conv), "iters": list(it), "iters_mean": im, "iters_sem": ie,
            "run_seconds": secs, "seconds_mean": sm, "seconds_sem": se, "trips": per_run,
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
    ap.add_argument("--rule", type=int, default=M.MUCA_RULE_BERG)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--max-seconds", type=float, default=None, help="per p, between iterations")
    ap.add_argument("--out", default=None, help="JSON file rewritten after every p")
    ap.add_argument("--first-id", type=int, default=0,
                    help="first global walker id of the first p (a study split over several "
                         "invocations continues the ranges of the earlier ones)")
    args = ap.parse_args()

    ps = [int(x) for x in args.p.split(",")]
    lo, hi = M.mucaDefaultWindow(args.d, args.L, args.N)
    out = {"d": args.d, "L": args.L, "N": args.N, "window": [lo, hi], "runs": args.runs,
           "total_sweeps": args.total_sweeps, "target": args.target, "rule": args.rule,
           "seed": args.seed, "results": []}
    log(f"scaling: d={args.d} L={args.L} N={args.N} window [{lo}, {hi}], runs {args.runs}, "
        f"{args.total_sweeps} sweeps per iteration, target {args.target}")
    first = args.first_id
    for p in ps:
        res = runs_for(args.d, args.L, args.N, p, args.runs, args.seed, args.total_sweeps,
                       args.target, args.max_iters, args.rule, first_id=first,
                       max_seconds=args.max_seconds)
        first += p * args.runs
        out["results"].append(res)
        log(f"p={p}: {res['converged']}/{args.runs} converged, mean iterations "
            f"{res['iters_mean']:.2f} +- {res['iters_sem']:.2f}, mean run time "
            f"{res['seconds_mean']:.2f} s, {res['gpu_seconds']:.1f} s in all")
        if args.out:
            json.dump(out, open(args.out, "w"))
    for r, (model, meas) in zip(out["results"], speedups(out["results"])):
        r["speedup_model"] = model
        r["speedup_measured"] = meas
    if args.out:
        json.dump(out, open(args.out, "w"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
