"""Serving run for a stream of SL1M deconvolution requests (config 5).

Requests arrive as a Poisson process; each asks for a full solve (30 power
steps for L, 200 FISTA iterations, objective terms).  Two ways to serve them
on one GPU are timed on the same stream:

* batched   -- the library's continuous-batching server (sl1m_server_*):
               requests are admitted by HBM footprint as slots free up and the
               work of all active requests shares each round of launches;
* unbatched -- one request at a time in arrival order, each with its own plan
               and sl1m_solve.

Inputs (pixel lists, uvw, data) are placed in HBM before the clock starts;
latency = completion - arrival.  Usage:

    python -m paper_1310_2078_amd.serve --requests 256 --out result.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import sl1m
from . import workloads as W


def request_evals(wl, power_iters=30) -> float:
    """Operator evaluations of one request: (power steps + iterations) forward
    and adjoint applications plus the final objective forward."""
    return float(wl.n_pix) * wl.n_vis * (2 * (power_iters + wl.n_iter) + 1)


def make_stream(n: int, time_scale: float = 1.0):
    arrivals = W.config5_arrivals(n_req=n) * time_scale
    reqs = [W.config5_request(r) for r in range(n)]
    return arrivals, reqs


def prepare(reqs, device):
    """Device copies of every request's inputs and its data V = M x_true + noise
    (formed with the library's forward operator)."""
    out = []
    for wl in reqs:
        plan = sl1m.Plan.from_workload(wl, device=device)
        V = plan.forward(wl.x_true) + torch.as_tensor(wl.noise, dtype=torch.complex64,
                                                      device=device)
        dev = W.Workload(wl.name,
                         torch.as_tensor(wl.l, device=device), torch.as_tensor(wl.m, device=device),
                         wl.sigma, wl.kind,
                         torch.as_tensor(wl.u, device=device), torch.as_tensor(wl.v, device=device),
                         torch.as_tensor(wl.w, device=device),
                         lam=wl.lam, n_iter=wl.n_iter, power_iters=wl.power_iters)
        out.append((dev, V))
        plan.close()
    torch.cuda.synchronize(device)
    return out


def _summary(lat, total_s, evals):
    lat = np.asarray(lat)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "makespan_s": total_s,
            "evals": evals, "evals_per_s": evals / total_s}


def run_batched(arrivals, reqs, data, device, arena_bytes=48 << 30, max_slots=32,
                round_budget=3e10, policy="oldest", tile_blocks=0, log=None):
    srv = sl1m.Server(arena_bytes, max_slots=max_slots, round_budget=round_budget, device=device,
                      policy=policy)
    n = len(reqs)
    lat = [None] * n
    open_t = {}
    nxt = 0
    done = 0
    t0 = time.perf_counter()
    last_log = t0
    while done < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            dev, V = data[nxt]
            t = srv.submit(dev, V, dev.lam, dev.n_iter, L=0.0, power_iters=dev.power_iters,
                           tile_blocks=tile_blocks)
            open_t[t] = nxt
            nxt += 1
        active, pending = srv.step()
        for t in list(open_t):
            ok, info, _ = srv.poll(t)
            if ok:
                i = open_t.pop(t)
                lat[i] = time.perf_counter() - t0 - arrivals[i]
                if info["status"] != 0:
                    raise RuntimeError(f"request {i} failed: {info}")
                srv.release(t)
                done += 1
        if active == 0 and pending == 0 and nxt < n:
            time.sleep(max(0.0, min(0.01, arrivals[nxt] - (time.perf_counter() - t0))))
        if log and time.perf_counter() - last_log > 10:
            last_log = time.perf_counter()
            print(f"[serve batched] t={last_log - t0:.1f}s done={done}/{n} active={active} "
                  f"pending={pending}", file=log, flush=True)
    total = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    evals = sum(request_evals(r) for r in reqs)
    out = _summary(lat, total, evals)
    out["rounds"] = st["rounds"]
    return out, lat


def run_unbatched(arrivals, reqs, data, device, log=None):
    n = len(reqs)
    lat = [None] * n
    t0 = time.perf_counter()
    last_log = t0
    for i in range(n):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        dev, V = data[i]
        plan = sl1m.Plan(dev.l, dev.m, dev.u, dev.v, dev.w,
                         sigma=reqs[i].sigma if np.any(reqs[i].kind) else None,
                         kind=reqs[i].kind if np.any(reqs[i].kind) else None, device=device)
        _, info = plan.solve(V, dev.lam, dev.n_iter, L=0.0, power_iters=dev.power_iters)
        plan.close()
        lat[i] = time.perf_counter() - t0 - arrivals[i]
        if log and time.perf_counter() - last_log > 10:
            last_log = time.perf_counter()
            print(f"[serve unbatched] t={last_log - t0:.1f}s done={i + 1}/{n}", file=log,
                  flush=True)
    total = time.perf_counter() - t0
    evals = sum(request_evals(r) for r in reqs)
    return _summary(lat, total, evals), lat


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--time-scale", type=float, default=1.0,
                    help="multiply the arrival times (1 = 4 requests/s on average)")
    ap.add_argument("--mode", choices=["both", "batched", "unbatched"], default="both")
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--budget", type=float, default=3e10)
    ap.add_argument("--tile-blocks", type=int, default=0,
                    help="per-request operator split target in the server (0: its default)")
    ap.add_argument("--policy", choices=["fair", "oldest"], default="oldest",
                    help="how the batched server shares each round")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    arrivals, reqs = make_stream(args.requests, args.time_scale)
    print(f"[serve] preparing {len(reqs)} requests", file=sys.stderr, flush=True)
    data = prepare(reqs, dev)
    res = {"requests": len(reqs), "arrival_rate_per_s": len(reqs) / float(arrivals[-1]),
           "offered_evals": sum(request_evals(r) for r in reqs)}
    if args.mode in ("both", "batched"):
        res["batched"], _ = run_batched(arrivals, reqs, data, dev, max_slots=args.slots,
                                        round_budget=args.budget, policy=args.policy,
                                        tile_blocks=args.tile_blocks,
                                        log=sys.stderr)
        res["batched"].update(policy=args.policy, slots=args.slots, budget=args.budget,
                              tile_blocks=args.tile_blocks)
        print(f"[serve] batched {res['batched']}", file=sys.stderr, flush=True)
    if args.mode in ("both", "unbatched"):
        res["unbatched"], _ = run_unbatched(arrivals, reqs, data, dev, log=sys.stderr)
        print(f"[serve] unbatched {res['unbatched']}", file=sys.stderr, flush=True)
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
