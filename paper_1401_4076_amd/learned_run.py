"""Learned vs plain initial weights on a target lattice (command line).

Trains the network on converged weight tables the iteration produces for
the training workloads (default: plain_2d, batched_2d, cubic_3d, each with
the given walkers per group and sweeps), proposes initial weights for the
target (default large_3d: 3D L=48, rho=0.03, N=3318) and runs the iteration
from the proposal and from flat weights until the histogram is flat.
Prints progress to stderr and one JSON line: iterations and wall time to a
flat histogram per arm (the learned arm includes inference), and the largest
difference of the two ln Omega estimates after a production run.  The two
stages can run apart: --stage train --net FILE saves the trained parameters
(float32 .npy), --stage eval --net FILE loads them.

    python -m paper_1401_4076_amd.learned_run --target-walkers 1024 --target-sweeps 10
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import workloads as W  # noqa: E402
from paper_1401_4076_amd import learned as LR  # noqa: E402
from paper_1401_4076_amd import muca as M  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", default="plain_2d,batched_2d,cubic_3d")
    ap.add_argument("--train-walkers", type=int, default=None, help="walkers per group cap (default: full)")
    ap.add_argument("--train-sweeps", type=int, default=1000)
    ap.add_argument("--train-max-iters", type=int, default=400)
    ap.add_argument("--steps", type=int, default=4000, help="Adam steps")
    ap.add_argument("--extra", default="",
                    help="additional training lattices d:L:rho:walkers[,...], converged in one "
                         "context with --extra-sweeps sweeps per iteration")
    ap.add_argument("--extra-sweeps", type=int, default=200)
    ap.add_argument("--target", default="large_3d")
    ap.add_argument("--target-walkers", type=int, default=None)
    ap.add_argument("--target-sweeps", type=int, default=None)
    ap.add_argument("--target-max-iters", type=int, default=400)
    ap.add_argument("--prod-sweeps", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--stage", choices=("all", "train", "eval"), default="all")
    ap.add_argument("--arms", default="learned,plain", help="arms of the comparison, in order")
    ap.add_argument("--net", default=None, help="parameter file (.npy) to save or load")
    ap.add_argument("--max-seconds", type=float, default=None,
                    help="wall-time budget of each iteration run (stops between chunks)")
    ap.add_argument("--race", action="store_true",
                    help="eval: step the iteration one at a time under a shared cap and note "
                         "when the tunnelling target and flatness are first met (see learned.race)")
    ap.add_argument("--tunnel-target", type=int, default=30)
    ap.add_argument("--out", default=None, help="eval --race: JSON file rewritten every iteration")
    args = ap.parse_args()
    if args.stage != "all" and not args.net:
        ap.error("--stage train/eval needs --net")

    out = {"stage": args.stage}
    if args.stage == "eval":
        net = M.Mlp(16384)
        net.set_params(np.load(args.net).astype(np.float32))
    else:
        net = train_stage(args, out)
        if net is not None and args.net:
            np.save(args.net, net.get_params())
    if args.stage != "train" and net is not None:
        eval_stage(args, net, out)
    print(json.dumps(out), flush=True)


def train_stage(args, out):
    out["train"] = []
    Xs, Ts = [], []
    for name in args.train.split(","):
        wl = W.scaled(name, walkers_per_group=args.train_walkers, sweeps=args.train_sweeps)
        log(f"train table {name}: groups {wl['groups']} sweeps {wl['sweeps']}")
        run = LR.converge(wl["groups"], wl["seed"], wl["sweeps"], args.train_max_iters,
                          chunk=args.chunk, max_seconds=args.max_seconds,
                          progress=lambda n, f, s, d, nm=name: log(
                              f"  {nm}: {n} iterations, flat {list(f)}, {s:.1f} s, "
                              f"(bottom, top visited, min/max, lowest E, visited) {d}"))
        done = [g for g, f in enumerate(run["flat"]) if f]
        out["train"].append({"workload": name, "groups": [list(g) for g in wl["groups"]],
                             "sweeps": wl["sweeps"], "iters": list(run["iters"]),
                             "flat": list(run["flat"]), "seconds": run["seconds"]})
        if done:
            X, T = LR.table_rows(run["ctx"], run["lnW"], done)
            Xs.append(X)
            Ts.append(T)
        run["ctx"].close()
    if args.extra:
        groups = []
        for spec in args.extra.split(","):
            d, L, rho, walkers = spec.split(":")
            d, L, walkers = int(d), int(L), int(walkers)
            groups.append((d, L, W.particles(d, L, float(rho)), walkers))
        log(f"extra tables: groups {groups} sweeps {args.extra_sweeps}")
        run = LR.converge(groups, args.seed, args.extra_sweeps, args.train_max_iters,
                          chunk=args.chunk, max_seconds=args.max_seconds,
                          progress=lambda n, f, s, d: log(f"  extra: {n} iterations, flat {list(f)}, "
                                                          f"{s:.1f} s"))
        done = [g for g, f in enumerate(run["flat"]) if f]
        out["train"].append({"workload": "extra", "groups": [list(g) for g in groups],
                             "sweeps": args.extra_sweeps, "iters": list(run["iters"]),
                             "flat": list(run["flat"]), "seconds": run["seconds"]})
        if done:
            X, T = LR.table_rows(run["ctx"], run["lnW"], done)
            Xs.append(X)
            Ts.append(T)
        run["ctx"].close()
    if not Xs:
        out["train_rows"] = 0
        log("no training table converged: nothing to train")
        return None
    X, T = torch.cat(Xs), torch.cat(Ts)
    out["train_rows"] = int(X.shape[0])
    net = M.Mlp(max(X.shape[0], 16384))
    net.set_params(W.mlp_init_params(args.seed))
    t0 = time.perf_counter()
    hist = LR.train(net, X, T, args.steps, log_every=max(1, args.steps // 8))
    out["train_seconds"] = time.perf_counter() - t0
    out["loss"] = hist
    log(f"trained {args.steps} steps on {X.shape[0]} rows: loss {hist}")
    return net


def race_stage(args, net, out):
    """Each arm on the target under the same seeds, sweeps and caps."""
    wl = W.scaled(args.target, walkers_per_group=args.target_walkers, sweeps=args.target_sweeps)
    out.update({"target": args.target, "target_groups": [list(g) for g in wl["groups"]],
                "target_sweeps": wl["sweeps"], "cap_iterations": args.target_max_iters,
                "cap_seconds": args.max_seconds, "tunnel_target": args.tunnel_target,
                "seed": wl["seed"], "arms": {}})
    log(f"race on {args.target}: groups {wl['groups']} sweeps {wl['sweeps']}")

    def dump():
        if args.out:
            with open(args.out + ".tmp", "w") as f:
                json.dump(out, f)
            os.replace(args.out + ".tmp", args.out)

    for arm in args.arms.split(","):
        t0 = time.perf_counter()
        lnW0 = None
        if arm == "learned":
            probe = M.Context(wl["groups"], wl["seed"])
            lnW0 = LR.predict(net, probe)
            probe.close()
        infer = time.perf_counter() - t0  # the learned arm includes the network's inference
        rec = out["arms"].setdefault(arm, {"inference_seconds": infer, "trajectory": []})

        def progress(r, _rec=rec, _arm=arm):
            _rec["trajectory"].append(r)
            d = r["detail"][0]
            log(f"  {_arm}: iteration {r['iter']}, {r['seconds']:.1f} s, tunnelling "
                f"{r['tunnelling']}, flat {r['flat']}, (bottom, top visited, min/max, lowest E, "
                f"visited) {d}")
            dump()

        res = LR.race(wl["groups"], wl["seed"], wl["sweeps"], args.target_max_iters, lnW0=lnW0,
                      tunnel_target=args.tunnel_target, max_seconds=args.max_seconds,
                      progress=progress, extra_seconds=infer)
        rec.update({k: res[k] for k in ("first_flat", "first_tunnel", "iterations")})
        rec["ln_omega"] = [[None if np.isnan(x) else float(x) for x in v]
                           for v in res["ln_omega"]]
        dump()


def eval_stage(args, net, out):
    if args.race:
        race_stage(args, net, out)
        return
    out["target"] = args.target
    wl = W.scaled(args.target, walkers_per_group=args.target_walkers, sweeps=args.target_sweeps)
    out["target_groups"] = [list(g) for g in wl["groups"]]
    out["target_sweeps"] = wl["sweeps"]
    log(f"target {args.target}: groups {wl['groups']} sweeps {wl['sweeps']}")
    history = out.setdefault("history", {})

    def progress(arm, n, f, s, d):
        history.setdefault(arm, []).append({"iters": n, "seconds": round(s, 1), "detail": d})
        log(f"  {arm}: {n} iterations, flat {list(f)}, {s:.1f} s, "
            f"(bottom, top visited, min/max, lowest E, visited) {d}")

    res = LR.compare(net, wl["groups"], wl["seed"], wl["sweeps"], args.target_max_iters,
                     prod_sweeps=args.prod_sweeps, chunk=args.chunk,
                     max_seconds=args.max_seconds, arms=tuple(args.arms.split(",")),
                     progress=progress)
    out.update(res)


if __name__ == "__main__":
    main()
