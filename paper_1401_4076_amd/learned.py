"""Learned initial weights: orchestration of the mucaMlp* calls.

1. converge weight tables with the MUCA iteration itself (mucaRun until flat);
2. build training rows from them (mucaMlpTableRows, one row per bin);
3. train the network with full-batch Adam steps (mucaMlpTrainStep);
4. propose lnW for a new lattice (mucaMlpPredictWeights) and compare the
   iteration started there with the plain recursion from flat weights:
   iterations and wall time to a flat histogram, and the ln Omega estimates.
All arithmetic runs in the HIP kernels of libmuca; this module only sequences
calls and moves small results to the host for reporting.
"""
import time

import numpy as np
import torch

from . import muca as M


def converge(groups, seed, sweeps, max_iters, rule=M.MUCA_RULE_BERG, lnW0=None, layout=None,
             stream=None, chunk=0, progress=None, max_seconds=None):
    """Run the iteration until every group is flat (at most max_iters).
    chunk > 0 splits the run into resumed calls of `chunk` iterations (same
    result), calls progress(done_iterations, flat_flags, seconds, detail)
    after each (detail: flat_detail of the last histogram) and stops early once max_seconds have passed (status not converged).
    Returns a dict with the context, weights, histogram, per-group
    iterations, flags, status and wall time."""
    ctx = M.Context(groups, seed)
    if layout is not None:
        ctx.set_layout(layout)
    dev = torch.device("cuda")
    lnW = (torch.zeros(ctx.total_bins, dtype=torch.float64, device=dev) if lnW0 is None
           else lnW0.clone())
    P = torch.zeros_like(lnW)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = chunk if chunk > 0 else max_iters
    done = 0
    while True:
        n = min(step, max_iters - done)
        rc, iters, flat = ctx.run(lnW, P, H, sweeps, n, rule, True, stream=stream,
                                  resume=done > 0)
        done += n
        if progress:
            progress(done, flat, time.perf_counter() - t0, flat_detail(ctx, H))
        if rc == M.MUCA_OK or done >= max_iters:
            break
        if max_seconds is not None and time.perf_counter() - t0 > max_seconds:
            break
    torch.cuda.synchronize()
    return {"ctx": ctx, "lnW": lnW, "H": H, "iters": iters, "flat": flat,
            "status": rc, "seconds": time.perf_counter() - t0}


def flat_detail(ctx, H):
    """Per group, for progress reports: (window bottom visited, window top
    visited, min/max of H over visited bins, lowest visited energy, fraction
    of the window's bins visited) of a histogram."""
    h = H.cpu().numpy()
    out = []
    for g in range(ctx.ngroups):
        lo, hi, off = ctx.window(g)
        hg = h[off:off + hi - lo + 1]
        seen = hg > 0
        if not seen.any():
            out.append((False, False, 0.0, None, 0.0))
            continue
        out.append((bool(seen[0]), bool(seen[-1]), round(float(hg[seen].min() / hg[seen].max()), 3),
                    int(lo + np.argmax(seen)), round(float(seen.mean()), 4)))
    return out


def race(groups, seed, sweeps, max_iters, lnW0=None, tunnel_target=30, rule=M.MUCA_RULE_BERG,
         max_seconds=None, progress=None, extra_seconds=0.0):
    """The iteration one step at a time (fixed schedule, mucaRun resumed per
    iteration), noting when each stop criterion is first met: the paper's
    convergence at `tunnel_target` tunnelling events in total (Sec. 4) and a
    flat histogram (every group).  Stops when both are met, after max_iters
    iterations or once max_seconds have passed.  Per iteration: elapsed
    seconds (plus extra_seconds, e.g. the network's inference), tunnelling
    events, flatness and flat_detail of H^i.  Returns the trajectory, the
    first iteration and time of each criterion (None if not met) and
    ln Omega = ln H^i - ln W^i of the last iteration (host arrays per group)."""
    ctx = M.Context(groups, seed)
    ctx.set_tunnel_target(tunnel_target)
    dev = torch.device("cuda")
    lnW = (torch.zeros(ctx.total_bins, dtype=torch.float64, device=dev) if lnW0 is None
           else lnW0.clone())
    P = torch.zeros_like(lnW)
    H = torch.zeros(ctx.total_bins, dtype=torch.int32, device=dev)
    prev = torch.empty_like(lnW)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    traj, first_flat, first_tunnel = [], None, None
    for i in range(max_iters):
        prev.copy_(lnW)  # the weights that produce H^i
        _, _, fl = ctx.run(lnW, P, H, sweeps, 1, rule, stop=M.MUCA_STOP_NONE, resume=i > 0)
        sec = time.perf_counter() - t0 + extra_seconds
        trips = int(sum(ctx.tunnel()[1]))
        flat = all(fl)
        rec = {"iter": i + 1, "seconds": round(sec, 2), "tunnelling": trips, "flat": flat,
               "detail": flat_detail(ctx, H)}
        traj.append(rec)
        if flat and first_flat is None:
            first_flat = {"iter": i + 1, "seconds": sec}
        if trips >= tunnel_target and first_tunnel is None:
            first_tunnel = {"iter": i + 1, "seconds": sec}
        if progress:
            progress(rec)
        if first_flat and first_tunnel:
            break
        if max_seconds is not None and sec > max_seconds:
            break
    lo = ln_omega(ctx, prev, H)
    ctx.close()
    return {"trajectory": traj, "first_flat": first_flat, "first_tunnel": first_tunnel,
            "iterations": len(traj), "ln_omega": lo}


def ln_omega_difference(a, b):
    """Largest |difference| of two ln Omega estimates of one group over the
    bins both visited, after removing the mean offset; and the bin count."""
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    both = ~np.isnan(a) & ~np.isnan(b)
    if not both.any():
        return float("nan"), 0
    d = a[both] - b[both]
    return float(np.max(np.abs(d - d.mean()))), int(both.sum())


def table_rows(ctx, lnW, groups=None):
    """Features and targets of every bin of the chosen groups (all by default)."""
    sel = range(ctx.ngroups) if groups is None else groups
    Xs, Ts = [], []
    for g in sel:
        lo, hi, _ = ctx.window(g)
        nb = hi - lo + 1
        X = torch.empty((nb, 4), dtype=torch.float32, device="cuda")
        T = torch.empty(nb, dtype=torch.float32, device="cuda")
        M.mucaMlpTableRows(ctx, g, lnW, X, T)
        Xs.append(X)
        Ts.append(T)
    return torch.cat(Xs), torch.cat(Ts)


def train(net, X, T, steps, lr=2e-3, lr_end=2e-4, log_every=0):
    """Full-batch Adam with a geometric learning-rate decay; returns losses
    at the logged steps (device values read back at the end)."""
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for s in range(steps):
        lr_s = lr * (lr_end / lr) ** (s / max(1, steps - 1))
        if log_every and (s % log_every == 0 or s == steps - 1):
            net.train_step(X, T, lr_s, loss)
            hist.append((s, loss.clone()))
        else:
            net.train_step(X, T, lr_s)
    torch.cuda.synchronize()
    return [(s, float(v.item())) for s, v in hist]


def predict(net, ctx):
    """Initial weights for every group of ctx from the network."""
    lnW = torch.zeros(ctx.total_bins, dtype=torch.float64, device="cuda")
    for g in range(ctx.ngroups):
        net.predict_weights(ctx, g, lnW)
    torch.cuda.synchronize()
    return lnW


def ln_omega(ctx, lnW, H):
    """ln Omega(E) = ln H(E) - lnW(E) over visited bins of each group, shifted
    so that the largest value is 0 (host arrays, for reporting)."""
    lw = lnW.cpu().numpy()
    h = H.cpu().numpy()
    out = []
    for g in range(ctx.ngroups):
        lo, hi, off = ctx.window(g)
        sl = slice(off, off + hi - lo + 1)
        v = np.full(hi - lo + 1, np.nan)
        seen = h[sl] > 0
        v[seen] = np.log(h[sl][seen]) - lw[sl][seen]
        v -= np.nanmax(v)
        out.append(v)
    return out


def production(run, sweeps):
    """One equilibrium run with the converged weights (more statistics for
    the ln Omega estimate); returns the histogram."""
    H = torch.zeros_like(run["H"])
    run["ctx"].sweep(run["lnW"], sweeps, H)
    torch.cuda.synchronize()
    return H


def compare(net, groups, seed, sweeps, max_iters, layout=None, prod_sweeps=0, chunk=0,
            progress=None, max_seconds=None, arms=("learned", "plain")):
    """Iteration from the network's proposal ("learned") and from flat weights
    ("plain"), same seeds and schedule.  With prod_sweeps > 0 the ln Omega
    estimates come from a production run with each arm's final weights, else
    from the last histogram; their largest difference (after removing the
    mean offset, over bins both arms visited) is reported when both ran."""
    runs = {}
    for arm in arms:
        t0 = time.perf_counter()
        lnW0 = None
        if arm == "learned":
            probe = M.Context(groups, seed)
            lnW0 = predict(net, probe)
            probe.close()
        infer_s = time.perf_counter() - t0  # the learned arm includes the network's inference
        run = converge(groups, seed, sweeps, max_iters, lnW0=lnW0, layout=layout, chunk=chunk,
                       progress=(lambda *a, _arm=arm: progress(_arm, *a)) if progress else None,
                       max_seconds=max_seconds)
        run["seconds"] += infer_s
        runs[arm] = run
    out = {arm: {k: r[k] for k in ("iters", "flat", "status", "seconds")}
           for arm, r in runs.items()}
    if len(runs) == 2:
        lo = []
        for arm in arms:
            r = runs[arm]
            Hx = production(r, prod_sweeps) if prod_sweeps else r["H"]
            lo.append(ln_omega(r["ctx"], r["lnW"], Hx))
        diffs = []
        for a, b in zip(*lo):
            both = ~np.isnan(a) & ~np.isnan(b)
            d = a[both] - b[both]
            diffs.append(float(np.max(np.abs(d - d.mean()))) if both.any() else float("nan"))
        out["ln_omega_max_abs_diff"] = diffs
    for r in runs.values():
        r["ctx"].close()
    return out
