"""The MUCA iteration on a workload, one iteration per call of mucaRun, with
per-iteration metrics and checkpoint files (command line).

Each iteration (Sec. 2: sweeps with fixed weights, summed histogram, weight
recursion) runs in libmuca; this module sequences the calls, copies the
histogram and the tunnelling counts to the host after each iteration and
writes one JSON line per iteration: per group the iterations done, whether
it has stopped, its flatness flag and tunnelling events (Sec. 4), the
visited part of its window (lowest and highest visited energy, fraction of
the bins) and min/max of H over the visited bins; for the whole iteration
its wall time, the move attempts it made and their rate.

--net starts from the learned network's proposal (its inference time is
reported apart) instead of flat weights.

A checkpoint file (.npz: the library's state image from mucaSaveState, the
caller-owned lnW, P and H, and the run's parameters as JSON) is written
every --checkpoint-every iterations and at the end; --resume continues from
it in a new process, bit-identically to a run that was never interrupted
(the random streams are counter-based).  --max-iters counts the iterations
of the whole run, across resumes.

    python -m paper_1401_4076_amd.run --workload large_3d --max-iters 1000 \\
        --log large_3d.jsonl --checkpoint large_3d.npz --checkpoint-every 20 --max-seconds 900
    python -m paper_1401_4076_amd.run --workload large_3d --max-iters 1000 \\
        --log large_3d.jsonl --checkpoint large_3d.npz --resume
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

import workloads as W  # noqa: E402

STOPS = {"none": 0, "flat": 1, "tunnel": 2}  # MUCA_STOP_NONE, _FLAT, _TUNNEL
RULES = {"berg": 0, "simple": 1}  # MUCA_RULE_BERG, _SIMPLE
CHECKPOINT_VERSION = 1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse_groups(spec):
    """'d:L:N:walkers[,...]' -> [(d, L, N, walkers), ...]."""
    groups = []
    for part in spec.split(","):
        f = part.split(":")
        if len(f) != 4:
            raise ValueError(f"group {part!r} is not d:L:N:walkers")
        groups.append(tuple(int(x) for x in f))
    return groups


def group_metrics(h, e_lo):
    """Visited part of one group's window from its histogram h (host array
    over the bins e_lo, e_lo + 1, ...)."""
    seen = np.flatnonzero(h > 0)
    if seen.size == 0:
        return {"visited": 0.0, "lowest_e": None, "highest_e": None, "bottom": False,
                "top": False, "min_over_max": 0.0}
    hv = h[seen]
    return {"visited": round(float(seen.size / h.size), 6),
            "lowest_e": int(e_lo + seen[0]), "highest_e": int(e_lo + seen[-1]),
            "bottom": bool(seen[0] == 0), "top": bool(seen[-1] == h.size - 1),
            "min_over_max": round(float(hv.min() / hv.max()), 6)}


def save_checkpoint(path, image, lnW, P, H, meta):
    """Write the checkpoint atomically (a temporary file, then a rename)."""
    tmp = path + ".tmp.npz"
    np.savez(tmp, image=np.frombuffer(bytes(image), dtype=np.uint8),
             lnW=np.asarray(lnW, dtype=np.float64), P=np.asarray(P, dtype=np.float64),
             H=np.asarray(H, dtype=np.int32), meta=np.array(json.dumps(meta)))
    os.replace(tmp, path)


def load_checkpoint(path):
    """(image bytes, lnW, P, H, meta dict); no pickled objects are read."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        if meta.get("version") != CHECKPOINT_VERSION:
            raise ValueError(f"{path}: checkpoint version {meta.get('version')} is not "
                             f"{CHECKPOINT_VERSION}")
        return z["image"].tobytes(), z["lnW"].copy(), z["P"].copy(), z["H"].copy(), meta


RUN_KEYS = ("groups", "seed", "sweeps", "rule", "stop", "tunnel_target")


def check_meta(saved, expected):
    """Raise ValueError unless the saved run has the parameters of this one."""
    bad = [k for k in RUN_KEYS if saved.get(k) != expected.get(k)]
    if bad:
        raise ValueError("checkpoint is of another run: " + ", ".join(
            f"{k} {saved.get(k)!r} (this run: {expected.get(k)!r})" for k in bad))


def build_parser():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="large_3d", help="a workload of workloads.py")
    ap.add_argument("--groups", default=None,
                    help="d:L:N:walkers[,...] instead of the workload's groups")
    ap.add_argument("--walkers", type=int, default=None, help="walkers per group cap")
    ap.add_argument("--sweeps", type=int, default=None, help="sweeps per iteration")
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--rule", choices=tuple(RULES), default="berg")
    ap.add_argument("--stop", choices=tuple(STOPS), default="flat",
                    help="a group stops at its first flat histogram, at the tunnelling "
                         "target of its walkers (Sec. 4), or never")
    ap.add_argument("--tunnel-target", type=int, default=30)
    ap.add_argument("--max-iters", type=int, default=100,
                    help="iterations of the whole run, counted across resumes")
    ap.add_argument("--max-seconds", type=float, default=None,
                    help="stop this process after the iteration that passes it")
    ap.add_argument("--log", default=None, help="JSON lines, one per iteration")
    ap.add_argument("--checkpoint", default=None, help=".npz checkpoint file")
    ap.add_argument("--checkpoint-every", type=int, default=0,
                    help="also write the checkpoint every K iterations")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint")
    ap.add_argument("--net", default=None,
                    help="start from the learned network's proposal (float32 parameter .npy) "
                         "instead of flat weights")
    return ap


def run_config(args):
    wl = W.scaled(args.workload, walkers_per_group=args.walkers, sweeps=args.sweeps)
    groups = parse_groups(args.groups) if args.groups else [tuple(g) for g in wl["groups"]]
    if args.groups and args.walkers is not None:
        groups = [g[:3] + (min(g[3], args.walkers),) for g in groups]
    return {"version": CHECKPOINT_VERSION,
            "workload": None if args.groups else args.workload,
            "groups": [list(g) for g in groups],
            "seed": int(wl["seed"] if args.seed is None else args.seed),
            "sweeps": int(wl["sweeps"]), "rule": args.rule, "stop": args.stop,
            "tunnel_target": int(args.tunnel_target),
            "init": "flat" if not args.net else "learned:" + os.path.basename(args.net)}


def main(argv=None):
    """Run; returns the summary dict (also printed as one JSON line)."""
    ap = build_parser()
    args = ap.parse_args(argv)
    if args.resume and not args.checkpoint:
        ap.error("--resume needs --checkpoint")
    if args.max_iters < 1 or args.checkpoint_every < 0:
        ap.error("--max-iters must be >= 1 and --checkpoint-every >= 0")

    import torch
    from paper_1401_4076_amd import muca as M

    cfg = run_config(args)
    groups = [tuple(g) for g in cfg["groups"]]
    stop, rule, S = STOPS[args.stop], RULES[args.rule], cfg["sweeps"]
    ctx = M.Context(groups, cfg["seed"])
    ctx.set_tunnel_target(cfg["tunnel_target"])
    dev = torch.device("cuda")
    done, iters_before, all_stopped, flat = 0, [0] * ctx.ngroups, False, [0] * ctx.ngroups
    inference = 0.0
    if args.resume:
        image, lnW_h, P_h, H_h, saved = load_checkpoint(args.checkpoint)
        check_meta(saved, cfg)
        ctx.load_state(image)
        lnW = torch.tensor(lnW_h, device=dev)
        P = torch.tensor(P_h, device=dev)
        H = torch.tensor(H_h, device=dev)
        done, iters_before = saved["iterations"], list(saved["iters"])
        all_stopped, flat = bool(saved["stopped"]), list(saved["flat"])
        log(f"resumed {args.checkpoint} after {done} iterations")
    elif args.net:
        from paper_1401_4076_amd import learned as LR
        t0 = time.perf_counter()
        rows = max(hi - lo + 1 for lo, hi, _ in (ctx.window(g) for g in range(ctx.ngroups)))
        net = M.Mlp(max(16384, rows))
        net.set_params(np.load(args.net, allow_pickle=False).astype(np.float32))
        lnW = LR.predict(net, ctx)  # synchronised
        net.close()
        inference = time.perf_counter() - t0
        log(f"initial weights from {args.net}: {inference:.3f} s")
        P = torch.zeros_like(lnW)
        H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=dev)
    else:
        lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device=dev)
        P = torch.zeros_like(lnW)
        H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=dev)
    windows = [ctx.window(g) for g in range(ctx.ngroups)]
    sizes = [g[1] ** g[0] for g in groups]
    first = np.cumsum([0] + [g[3] for g in groups])
    logf = open(args.log, "a" if args.resume else "w") if args.log else None

    def checkpoint():
        if args.checkpoint:
            meta = dict(cfg, iterations=done, iters=[int(x) for x in iters_before],
                        flat=[int(x) for x in flat], stopped=all_stopped)
            save_checkpoint(args.checkpoint, ctx.save_state(), lnW.cpu().numpy(),
                            P.cpu().numpy(), H.cpu().numpy(), meta)

    t_start = time.perf_counter()
    while done < args.max_iters and not all_stopped:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, iters, flat = ctx.run(lnW, P, H, S, 1, rule, stop=stop, resume=done > 0)
        sec = time.perf_counter() - t0  # mucaRun returns after the iteration
        done += 1
        swept = [a > b for a, b in zip(iters, iters_before)]
        attempts = sum(g[3] * S * v for g, v, s in zip(groups, sizes, swept) if s)
        h = H.cpu().numpy()
        trips = np.asarray(ctx.tunnel()[1], dtype=np.int64)
        rec = {"iteration": done, "seconds": round(sec, 6), "attempts": int(attempts),
               "attempts_per_s": attempts / sec if sec > 0 else None, "groups": []}
        for g, (lo, hi, off) in enumerate(windows):
            m = group_metrics(h[off:off + hi - lo + 1], lo)
            rec["groups"].append(dict(group=g, iters=int(iters[g]), swept=bool(swept[g]),
                                      flat=bool(flat[g]),
                                      trips=int(trips[first[g]:first[g + 1]].sum()), **m))
        if logf:
            logf.write(json.dumps(rec) + "\n")
            logf.flush()
        iters_before = list(iters)
        log(f"iteration {done}: {sec:.3f} s, {attempts / max(sec, 1e-9):.3g} attempts/s, "
            f"flat {list(flat)}, trips {[r['trips'] for r in rec['groups']]}, visited "
            f"{[r['visited'] for r in rec['groups']]}")
        all_stopped = stop != 0 and rc == M.MUCA_OK
        if all_stopped:
            break
        if args.checkpoint_every and done % args.checkpoint_every == 0:
            checkpoint()
        if args.max_seconds is not None and time.perf_counter() - t_start > args.max_seconds:
            break
    checkpoint()
    if logf:
        logf.close()
    out = dict(cfg, iterations=done, iters=[int(x) for x in iters_before],
               flat=[int(x) for x in flat], stopped=all_stopped,
               seconds=round(time.perf_counter() - t_start, 3), checkpoint=args.checkpoint,
               inference_seconds=round(inference, 3))
    print(json.dumps(out), flush=True)
    out["lnW"], out["P"], out["H"] = lnW.cpu().numpy(), P.cpu().numpy(), H.cpu().numpy()
    ctx.close()
    return out


if __name__ == "__main__":
    main()
