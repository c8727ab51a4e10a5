"""Benchmark of the SL1M hot path on one MI355X.

Workload: config 2 of the measurement plan -- a 256x256 wide-field delta grid
over l, m in +-0.3 (65,536 pixels) against 97,536 visibilities of a
128-antenna array (12 snapshots over 6 h, 150 MHz), FP32 operator with FP64
phase.  A step is one FISTA iteration: forward operator, residual, adjoint,
threshold and momentum update, i.e. 2 x 65,536 x 97,536 pixel-visibility
evaluations.  The timed region is exactly `--steps` iterations of one L1 solve
(100 by default, the workload's solve length) with L fixed beforehand.

Prints one JSON line with the throughput, the dominant kernel's roofline
fraction (kernel durations from HIP events recorded by the library around
each launch on the launch stream) and the FP64 CPU oracle's rate on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3            # MI355X FP32 vector peak (published)
FLOP_PER_EVAL_DELTA = 14            # phase 3 FMA, reduction 2, sin+cos 2, accumulate 2 FMA


def _function_text(src: str, name: str) -> str:
    """The definition of kernel `name` (signature through its closing brace)."""
    i = src.find(f"void {name}(")
    if i < 0:
        return ""
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        depth += {"{": 1, "}": -1}.get(src[k], 0)
        if depth == 0:
            return src[i:k + 1]
    return src[i:]


def kernel_source_hash(kernel: str) -> str:
    """Hash of the device code `kernel` is compiled from: its own definition,
    the tile and device headers, and the records and constants that precede
    the plan struct in sl1m_internal.h (its counters go stale when any of them
    changes; host code in the same files does not count)."""
    csrc = os.path.join(ROOT, "paper_1310_2078_amd", "csrc")

    def read(f):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            return fh.read()

    base = kernel.split("<")[0]
    grid = kernel.startswith("k_grid")
    parts = [_function_text(read("sl1m_grid.hip" if grid else "sl1m_kernels.hip"), base)]
    if grid:
        parts.append(read("sl1m_grid.h"))
    parts.append(read("sl1m_device.h"))
    internal = read("sl1m_internal.h")
    parts.append(internal[:internal.find("struct sl1m_plan {")])
    h = hashlib.sha256()
    for t in parts:
        h.update(t.encode())
    return h.hexdigest()[:16]


# Inner-loop instruction mix of the kernels that can dominate the iteration
# (counted in their gfx950 assembly): entries per wavefront unit of work, then
# FP32-rate (FP32 arithmetic, bit operations, integer), FP64 and sin/cos
# wave64 instructions per unit.  The pair adjoint's unit is a wavefront and a
# visibility (64 lanes x 32 entries), the pair forward's a wavefront and a
# (pair record, visibility) (64 lanes x 8 entries, with the per-|l| phasors
# spread over the 8 records), the direct kernels' a wavefront and an entry.
SLOT_MIX = {
    "k_grid_adj_delta_square": (2048, 76, 6, 12),
    "k_grid_fwd_delta_pairs": (512, 21.25, 1.25, 2.5),
    "k_adj_delta<float,4>": (64, 3, 3, 2),
    "k_fwd_delta<float,4>": (64, 3, 3, 2),
}

HBM_PEAK_BPS = 8.0e12  # MI355X HBM3E, published

PLAN_KEYS = ("n_fchunks_grid", "n_achunks", "fwd_vpl", "adj_ppl")


def load_traffic(kernel: str, plan_shape=None):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source and (when recorded) with the same
    operator split as the timed plan; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = d.get(kernel)
    if not rec or rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    rec_plan = rec.get("plan")
    if plan_shape is not None and rec_plan is not None:
        # the fields of the kernel's own operator (the adjoint's traffic does
        # not depend on the forward split, and the other way round)
        keys = ("n_achunks", "adj_ppl") if "adj" in kernel else ("n_fchunks_grid", "fwd_vpl")
        if any(rec_plan.get(k) != plan_shape.get(k) for k in keys):
            return None
    return rec.get("bytes_per_launch")


CALIB_BYTES = 256 << 20


def _counter_rows(path):
    """(kernel name, counter value in bytes) per dispatch from a rocprofv3
    counter_collection CSV (one row per dispatch and counter)."""
    import csv
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("kernel_name") or ""
            val = r.get("Counter_Value") or r.get("Counter-Value") or r.get("counter_value")
            if val is None:
                continue
            rows.append((name, float(val) * 1024.0))   # FETCH_SIZE / WRITE_SIZE are in KiB
    return rows


def ingest_counters(fetch_csv, write_csv, bench_log=None):
    """Per-launch HBM bytes of the operator kernels, scaled by what the same
    counters read for the calibration copy of CALIB_BYTES (read once, written
    once); with the counted runs' bench output, the plan's split is recorded."""
    out = {}
    shape = None
    if bench_log:
        with open(bench_log) as fh:
            last = [ln for ln in fh if ln.startswith("{")][-1]
        shape = json.loads(last)["config"].get("plan")
    for counter, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _counter_rows(path)
        copy = [v for n, v in rows if "copy" in n.lower() or "elementwise" in n.lower()]
        big = [v for v in copy if v > 0.5 * CALIB_BYTES]
        if not big:
            raise SystemExit(f"no calibration copy found in {path}")
        scale = CALIB_BYTES / (sum(big) / len(big))
        for key, pat in (("k_fwd_delta<float,4>", "k_fwd_delta<float, 4, false, 1>"),
                         ("k_adj_delta<float,4>", "k_adj_delta<float, 4, false, 1>"),
                         ("k_grid_fwd_delta_pairs", "k_grid_fwd_delta_pairs"),
                         ("k_grid_adj_delta_square", "k_grid_adj_delta_square"),
                         ("k_grid_fwd_delta", "k_grid_fwd_delta("),
                         ("k_grid_adj_delta", "k_grid_adj_delta(")):
            vals = [v for n, v in rows if pat in n]
            if vals:
                rec = out.setdefault(key, {"source_hash": kernel_source_hash(key)})
                if shape is not None:
                    rec["plan"] = shape
                rec[counter + "_bytes_per_launch"] = scale * sum(vals) / len(vals)
                rec[counter + "_scale"] = scale
                rec["launches"] = len(vals)
    for rec in out.values():
        rec["bytes_per_launch"] = rec.get("fetch_bytes_per_launch", 0.0) + \
            rec.get("write_bytes_per_launch", 0.0)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def cpu_baseline(wl, threads: int):
    """The FP64 oracle, untuned, on a bounded sample of the workload: the
    forward for the first 512*threads visibilities (all pixels) and the adjoint
    for the first 2048*threads pixels against the first quarter of the
    visibilities."""
    import oracle as O
    p = O.Problem.from_workload(wl, threads=threads)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(wl.n_pix)
    nf = min(wl.n_vis, 512 * threads)
    t0 = time.perf_counter()
    O.forward_rows(p, x, np.arange(nf))
    tf = time.perf_counter() - t0
    nvq = wl.n_vis // 4
    pq = O.Problem(l=wl.l, m=wl.m, u=wl.u[:nvq], v=wl.v[:nvq], w=wl.w[:nvq], threads=threads)
    na = min(wl.n_pix, 2048 * threads)
    r = rng.standard_normal(nvq) + 1j * rng.standard_normal(nvq)
    t0 = time.perf_counter()
    O.adjoint_cols(pq, r, np.arange(na))
    ta = time.perf_counter() - t0
    evals = nf * wl.n_pix + na * nvq
    return {
        "value": evals / (tf + ta),
        "unit": "evals/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"forward rows 0..{nf - 1} x {wl.n_pix} pixels + adjoint pixels 0..{na - 1} "
                  f"x {nvq} visibilities ({evals:.3e} evals, {tf + ta:.1f} s)",
    }


def _time_ops(plan, fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def extras(plan2, wl2, dev):
    """Secondary workloads, reported beside the headline line (not in `value`)."""
    import torch
    from paper_1310_2078_amd import sl1m
    from paper_1310_2078_amd import workloads as W
    ex = {}
    # the same FISTA iteration with every entry evaluated directly (no grid
    # factorisation), for comparison with the headline evaluation
    pdir = sl1m.Plan.from_workload(wl2, device=dev, grid="off")
    Vd = pdir.forward(wl2.x_true)
    Ld = 1.01 * pdir.estimate_L(10, seed=0)
    pdir.solve(Vd, wl2.lam, 3, L=Ld)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pdir.solve(Vd, wl2.lam, 20, L=Ld)
    torch.cuda.synchronize()
    td = time.perf_counter() - t0
    ex["config2_direct_evaluation"] = {
        "iterations": 20, "time_s": td,
        "evals_per_s": 2.0 * wl2.n_pix * wl2.n_vis * 20 / td}
    pdir.close()
    del pdir, Vd
    # warm start from the dirty image (Section "Acceleration strategies"):
    # relative objective gap after k iterations, cold against warm, with F*
    # from a 400-iteration cold solve
    V2 = plan2.forward(wl2.x_true) + torch.as_tensor(wl2.noise, dtype=torch.complex64, device=dev)
    L2 = 1.01 * plan2.estimate_L(wl2.power_iters, seed=0)
    _, ref = plan2.solve(V2, wl2.lam, 400, L=L2)
    D = plan2.dirty_image(V2)
    gaps = {}
    for k in (10, 30, 100):
        _, c = plan2.solve(V2, wl2.lam, k, L=L2)
        _, w = plan2.solve(V2, wl2.lam, k, L=L2, x0=D)
        gaps[str(k)] = {"cold": (c["F"] - ref["F"]) / ref["F"],
                        "dirty_start": (w["F"] - ref["F"]) / ref["F"]}
    ex["config2_warm_start"] = {"F_star_400_iterations": ref["F"], "relative_gap": gaps}
    # MFISTA (one more forward per iteration, monotone objective) against FISTA
    mf = {}
    for k in (10, 30, 100):
        _, c = plan2.solve(V2, wl2.lam, k, L=L2, method="mfista")
        mf[str(k)] = (c["F"] - ref["F"]) / ref["F"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan2.solve(V2, wl2.lam, 50, L=L2, method="mfista")
    torch.cuda.synchronize()
    t_m = (time.perf_counter() - t0) / 50
    ex["config2_mfista"] = {"relative_gap": mf, "ms_per_iteration": t_m * 1e3}
    del V2, D
    # multi-RHS: 4 right-hand sides (Stokes I, Q, U, V) at config 2's shape
    rng = np.random.default_rng(5)
    X = torch.as_tensor(rng.standard_normal((4, wl2.n_pix)), dtype=torch.float32, device=dev)
    ev = wl2.n_pix * wl2.n_vis
    for grid in ("auto", "off"):
        pm = sl1m.Plan.from_workload(wl2, device=dev, max_rhs=4, grid=grid)
        Vm = pm.forward_multi(X)
        tf = _time_ops(pm, lambda: pm.forward_multi(X, out=Vm), 5)
        G = torch.empty((4, wl2.n_pix), dtype=torch.float32, device=dev)
        ta = _time_ops(pm, lambda: pm.adjoint_multi(Vm, out=G), 5)
        rec = {"evaluation": "grid" if pm.info()["grid_multi"] >= 4 else "direct",
               "forward_ms": tf * 1e3, "adjoint_ms": ta * 1e3,
               "phasor_evals_per_s": 2 * ev / (tf + ta),
               "rhs_products_per_s": 8 * ev / (tf + ta)}
        ex["config2_shape_multi_rhs4" if grid == "auto" else
           "config2_shape_multi_rhs4_direct"] = rec
        pm.close()
        del pm, Vm, G
    # eight sides: grid evaluation (FP32) against the matrix cores (FP16)
    X8 = torch.as_tensor(np.random.default_rng(8).standard_normal((8, wl2.n_pix)),
                         dtype=torch.float32, device=dev)
    rec8 = {}
    for label, kw in (("grid", {}), ("mfma_f16", {"precision": "mfma_f16"})):
        pm = sl1m.Plan.from_workload(wl2, device=dev, max_rhs=8, **kw)
        Vm = pm.forward_multi(X8)
        tf = _time_ops(pm, lambda: pm.forward_multi(X8, out=Vm), 5)
        G = torch.empty((8, wl2.n_pix), dtype=torch.float32, device=dev)
        ta = _time_ops(pm, lambda: pm.adjoint_multi(Vm, out=G), 5)
        rec8[label] = {"forward_ms": tf * 1e3, "adjoint_ms": ta * 1e3,
                       "rhs_products_per_s": 16 * ev / (tf + ta)}
        pm.close()
        del pm, Vm, G
    ex["config2_shape_multi_rhs8"] = rec8
    del X8
    # the same four sides on the matrix cores (float16 / bfloat16 operands)
    for prec in ("mfma_f16", "mfma_bf16"):
        pm = sl1m.Plan.from_workload(wl2, device=dev, max_rhs=4, precision=prec)
        Vm = pm.forward_multi(X)
        tf = _time_ops(pm, lambda: pm.forward_multi(X, out=Vm), 5)
        G = torch.empty((4, wl2.n_pix), dtype=torch.float32, device=dev)
        ta = _time_ops(pm, lambda: pm.adjoint_multi(Vm, out=G), 5)
        ex[f"config2_shape_multi_rhs4_{prec}"] = {
            "evaluation": "direct, MFMA 4x4x4", "forward_ms": tf * 1e3, "adjoint_ms": ta * 1e3,
            "phasor_evals_per_s": 2 * ev / (tf + ta), "rhs_products_per_s": 8 * ev / (tf + ta)}
        pm.close()
        del pm, Vm, G
    del X
    # config 4: multiscale Gaussian pixels with direction-dependent gains
    wl4 = W.config4()
    t0 = time.perf_counter()
    p4 = sl1m.Plan.from_workload(wl4, device=dev)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    x4 = torch.as_tensor(rng.standard_normal(wl4.n_pix), dtype=torch.float32, device=dev)
    V4 = p4.forward(x4)
    g4 = torch.empty(wl4.n_pix, dtype=torch.float32, device=dev)
    p4.timing_begin(16)
    tf = _time_ops(p4, lambda: p4.forward(x4, out=V4), 2)
    ta = _time_ops(p4, lambda: p4.adjoint(V4, out=g4), 2)
    t4 = p4.timing_end()
    n_delta = 1024 * 1024
    n_gauss = wl4.n_pix - n_delta
    flops = (14 * n_delta + 26 * n_gauss) * wl4.n_vis
    ex["config4"] = {
        "n_pix": wl4.n_pix, "n_vis": wl4.n_vis, "plan_s": t_plan,
        "evaluation": "grid" if p4.info()["grid"] else "direct",
        "forward_ms": tf * 1e3, "adjoint_ms": ta * 1e3,
        "forward_kernel_ms": t4["forward"][1] / max(t4["forward"][0], 1),
        "adjoint_kernel_ms": t4["adjoint"][1] / max(t4["adjoint"][0], 1),
        "evals_per_s": 2 * wl4.n_pix * wl4.n_vis / (tf + ta),
        "fista_iteration_s_est": tf + ta,
        "canonical_tflops": 2 * flops / (tf + ta) / 1e12}
    # one GPU's share of config 4 split over 8 GPUs by visibilities (every 8th
    # record, all pixels: the grid evaluation keeps its square pixel grid)
    ws = dataclasses.replace(wl4, u=wl4.u[::8], v=wl4.v[::8], w=wl4.w[::8],
                             ant_p=wl4.ant_p[::8], ant_q=wl4.ant_q[::8], noise=None)
    ps = sl1m.Plan.from_workload(ws, device=dev)
    Vs = ps.forward(x4)
    gsh = torch.empty(wl4.n_pix, dtype=torch.float32, device=dev)
    ps.timing_begin(16)
    tfs = _time_ops(ps, lambda: ps.forward(x4, out=Vs), 3)
    tas = _time_ops(ps, lambda: ps.adjoint(Vs, out=gsh), 3)
    tsh = ps.timing_end()
    rate_s = 2 * ws.n_pix * ws.n_vis / (tfs + tas)
    ex["config4_shard_1_of_8_by_visibilities"] = {
        "n_pix": ws.n_pix, "n_vis": ws.n_vis, "forward_ms": tfs * 1e3, "adjoint_ms": tas * 1e3,
        "forward_kernel_ms": tsh["forward"][1] / max(tsh["forward"][0], 1),
        "adjoint_kernel_ms": tsh["adjoint"][1] / max(tsh["adjoint"][0], 1),
        "evals_per_s": rate_s, "rate_vs_full_config4": rate_s / ex["config4"]["evals_per_s"]}
    ps.close()
    del ps, Vs, gsh
    # the config 4 L1 solve: data = the point sources through the operator plus
    # the 50 extended sources as a fine FP64 sum of delta points (not the
    # Gaussian-pixel model) plus noise; L from 30 power steps; 100 iterations
    pe = sl1m.Plan(wl4.extra_l, wl4.extra_m, wl4.u, wl4.v, wl4.w, ant_p=wl4.ant_p,
                   ant_q=wl4.ant_q, ant_gain=wl4.ant_gain, ant_fwhm=wl4.ant_fwhm,
                   precision="fp64", device=dev)
    Ve = pe.forward(wl4.extra_flux)
    pe.close()
    Ve32 = Ve.to(torch.complex64)
    V4d = p4.forward(wl4.x_true) + Ve32 + \
        torch.as_tensor(wl4.noise, dtype=torch.complex64, device=dev)
    del Ve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    img4, info4 = p4.solve(V4d, wl4.lam, wl4.n_iter, L=0.0, power_iters=wl4.power_iters)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    ex["config4"]["solve"] = {
        "time_s": ts, "iterations": wl4.n_iter, "power_iterations": wl4.power_iters,
        "L": info4["L"], "F": info4["F"], "nnz": info4["nnz"],
        "evals_per_s": 2 * wl4.n_pix * wl4.n_vis * (wl4.n_iter + wl4.power_iters) / ts}
    del p4, x4, V4, g4, img4
    # adaptive quad-tree refinement (Section "Acceleration strategies"): 32 x 32
    # cells over the field, six levels down to the 1024^2 grid's spacing, 100
    # iterations per level, against the full 1024^2 delta grid solved with the
    # same iterations; on config 4's data, and on its 50 extended sources alone
    # (the kind of sky the paper refined: one HI channel of a galaxy)
    from paper_1310_2078_amd import refine as R
    gkw = dict(ant_p=wl4.ant_p, ant_q=wl4.ant_q, ant_gain=wl4.ant_gain, ant_fwhm=wl4.ant_fwhm)
    half4 = 0.35
    h_min4 = 2 * half4 / 1024
    delta = wl4.kind == 0
    noise4 = torch.as_tensor(wl4.noise, dtype=torch.complex64, device=dev)
    for key, data in (("config4_quadtree", V4d), ("config4_quadtree_extended_only", Ve32 + noise4)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lv = R.quadtree_solve(wl4.u, wl4.v, wl4.w, data, wl4.lam, 32, half4, 6, wl4.n_iter,
                              h_min4, power_iters=wl4.power_iters, device=dev,
                              max_cells=400_000, **gkw)
        tq = time.perf_counter() - t0
        pf = sl1m.Plan(wl4.l[delta], wl4.m[delta], wl4.u, wl4.v, wl4.w, device=dev, **gkw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infof = pf.solve(data, wl4.lam, wl4.n_iter, L=0.0, power_iters=wl4.power_iters)
        torch.cuda.synchronize()
        tf_ = time.perf_counter() - t0
        pf.close()
        ex[key] = {
            "levels": [{"cells": int(x.l.size),
                        "delta_cells": int(np.sum(x.h <= h_min4 * (1 + 1e-9))),
                        "seconds": x.seconds, "F": x.info["F"], "nnz": x.info["nnz"]} for x in lv],
            "time_s": tq, "final_F": lv[-1].info["F"],
            "full_grid_1024sq_delta": {"time_s": tf_, "F": infof["F"], "nnz": infof["nnz"]},
            "time_ratio_full_over_quadtree": tf_ / tq,
            "F_ratio_quadtree_over_full": lv[-1].info["F"] / infof["F"]}
    del V4d, Ve32
    # config 1: plain SL1M in FP64 (100 iterations + 30 power steps)
    wl1 = W.config1()
    p1 = sl1m.Plan.from_workload(wl1, device=dev, precision="fp64")
    V1 = p1.forward(wl1.x_true) + torch.as_tensor(wl1.noise, device=dev)
    p1.solve(V1, wl1.lam, 5, L=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = p1.solve(V1, wl1.lam, wl1.n_iter, L=0.0, power_iters=wl1.power_iters)
    torch.cuda.synchronize()
    ex["config1_fp64_solve"] = {"time_s": time.perf_counter() - t0, "iterations": wl1.n_iter,
                                "power_iterations": wl1.power_iters, "F": info["F"],
                                "nnz": info["nnz"]}
    return ex


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workloads (config 4, multi-RHS, FP64 config 1)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM counters)")
    ap.add_argument("--ingest-counters", nargs="+", metavar="PATH",
                    help="FETCH_CSV WRITE_CSV [BENCH_OUT]: turn two rocprofv3 --pmc counter CSVs "
                         "(FETCH_SIZE, WRITE_SIZE) of a --calib-copy run into "
                         "profiles/traffic.json (with the run's plan split, read from its "
                         "output line) and exit")
    ap.add_argument("--grid", choices=["auto", "off", "require"], default="auto",
                    help="evaluation of the delta pixels: grid factorisation when the pixels "
                         "qualify (auto), always direct (off)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the plan's default launch shapes instead of tuning them first")
    ap.add_argument("--tuning", default=None,
                    help="JSON of a tuning choice (the config.tuning of an earlier line): use it "
                         "instead of tuning")
    ap.add_argument("--profile-ops", type=int, default=0,
                    help="after the timed region, run this many extra forward+adjoint pairs "
                         "(for profiler runs)")
    args = ap.parse_args()
    if args.ingest_counters:
        if len(args.ingest_counters) not in (2, 3):
            ap.error("--ingest-counters takes FETCH_CSV WRITE_CSV [BENCH_OUT]")
        ingest_counters(*args.ingest_counters)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(sharding over several GPUs, by visibilities for grid plans and by pixels otherwise, is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1310_2078_amd import sl1m
    from paper_1310_2078_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    wl = W.config2()
    n_pix, n_vis = wl.n_pix, wl.n_vis
    print(f"[bench] config2 n_pix={n_pix} n_vis={n_vis} steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)
    plan = sl1m.Plan.from_workload(wl, device=dev, grid=args.grid)
    tuning = None
    if args.tuning:
        # a fixed choice (e.g. the one a timed run printed), for profiler runs
        tuning = json.loads(args.tuning)
        plan.close()
        plan = sl1m.Plan.from_workload(wl, device=dev, tuning=tuning)
    elif not args.no_tune:
        # launch shapes from the autotuner (sl1m_tune), restricted to the
        # requested evaluation
        tuning = plan.tune(reps=7)
        if args.grid != "auto" and tuning["grid"] != args.grid:
            tuning = None
        else:
            plan.close()
            plan = sl1m.Plan.from_workload(wl, device=dev, tuning=tuning)
        print(f"[bench] tuning {tuning}", file=sys.stderr, flush=True)
    noise = torch.as_tensor(wl.noise, dtype=torch.complex64, device=dev)
    V = plan.forward(wl.x_true) + noise            # synthetic data, not timed

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rq = plan.estimate_L(wl.power_iters, seed=0)
    torch.cuda.synchronize()
    t_power = time.perf_counter() - t0
    L = 1.01 * rq

    if args.warmup > 0:
        plan.solve(V, wl.lam, args.warmup, L=L)
    torch.cuda.synchronize()
    plan.timing_begin(max(16, 2 * args.steps + 8))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    img, info = plan.solve(V, wl.lam, args.steps, L=L)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = plan.timing_end()
    elapsed = t1 - t0
    evals = 2.0 * n_pix * n_vis * args.steps
    print(f"[bench] solve {args.steps} it in {elapsed:.4f} s; timing {tim}; info {info}",
          file=sys.stderr, flush=True)

    for _ in range(args.profile_ops):
        plan.adjoint(plan.forward(img))
    if args.calib_copy:
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # an elementwise kernel: reads and writes CALIB_BYTES
    torch.cuda.synchronize()

    fwd_n, fwd_ms = tim["forward"]
    adj_n, adj_ms = tim["adjoint"]
    fis_n, fis_ms = tim["fista"]
    fwd_avg = fwd_ms / max(fwd_n, 1)
    adj_avg = adj_ms / max(adj_n, 1)
    pinfo = plan.info()
    plan_shape = {k: pinfo[k] for k in PLAN_KEYS}
    grid = bool(pinfo["grid"])
    if grid and pinfo["grid_pairs"]:
        names = ("k_grid_adj_delta_square", "k_grid_fwd_delta_pairs")
    elif grid:
        names = ("k_grid_adj_delta", "k_grid_fwd_delta")
    else:
        names = ("k_adj_delta<float,4>", "k_fwd_delta<float,4>")
    if adj_avg >= fwd_avg:
        dom, dom_ms, dom_name = "adjoint", adj_avg, names[0]
    else:
        dom, dom_ms, dom_name = "forward", fwd_avg, names[1]
    exec_flop = 4.5 if (grid and pinfo["grid_pairs"]) else 6.0 if grid else float(FLOP_PER_EVAL_DELTA)
    flops = FLOP_PER_EVAL_DELTA * n_pix * n_vis
    achieved = flops / (dom_ms * 1e-3) / 1e12
    out = {
        "metric": "pixel x visibility evals/s (forward + adjoint), FISTA iteration on config 2",
        "value": evals / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 phase)",
        "data": "synthetic",
        "config": {
            "workload": "config2: 256x256 wide-field delta pixels over +-0.3, 97,536 visibilities "
                        "(128 antennas, 12 snapshots, 150 MHz), FISTA lambda=3*sigma*sqrt(N_v)",
            "n_pix": n_pix,
            "n_vis": n_vis,
            "evals_per_step": 2 * n_pix * n_vis,
            "evaluation": "grid" if grid else "direct",
            "tuning": tuning,
            "plan": plan_shape,
        },
        "l1_solve_time_s": elapsed,
        "solve": {
            "iterations": args.steps,
            "time_s": elapsed,
            "power_iteration_s": t_power,
            "power_iterations": wl.power_iters,
            "L": L,
            "F": info["F"],
            "nnz": info["nnz"],
        },
        "kernels": {
            "forward_avg_ms": fwd_avg,
            "adjoint_avg_ms": adj_avg,
            "fista_update_avg_ms": fis_ms / max(fis_n, 1),
            # the update reads the adjoint's split-K rows (n_achunks x 4 B per
            # pixel) plus scale, y and I, and writes y and I: algorithmic HBM
            # bytes per launch over its measured time, against 8 TB/s
            "fista_update_hbm_gbs": n_pix * (4 * pinfo["n_achunks"] + 20)
                                    / (fis_ms / max(fis_n, 1) * 1e-3) / 1e9,
            "fista_update_hbm_frac": n_pix * (4 * pinfo["n_achunks"] + 20)
                                     / (fis_ms / max(fis_n, 1) * 1e-3) / HBM_PEAK_BPS,
            "forward_evals_per_s": n_pix * n_vis / (fwd_avg * 1e-3),
            "adjoint_evals_per_s": n_pix * n_vis / (adj_avg * 1e-3),
        },
        "roofline": {
            "bound": "alu",
            "kernel": dom_name,
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": load_traffic(dom_name, plan_shape),
            "flop_per_eval": FLOP_PER_EVAL_DELTA,
            "evals_per_launch": n_pix * n_vis,
            # the same counting rules applied to the work the kernel executes:
            # a mirrored pair of cells (8 entries) takes 36 FLOP, a single cell
            # (4 entries) 24, a direct entry 14
            "executed_flop_per_eval": exec_flop,
            "executed_achieved": exec_flop * n_pix * n_vis / (dom_ms * 1e-3) / 1e12,
            "executed_frac": exec_flop * n_pix * n_vis / (dom_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "accounting": "achieved/frac: canonical delta-eval FLOPs (14 per entry, the "
                          "direct evaluation); executed_*: the grid evaluation's own count "
                          "(one sincos per 4 entries, per 8 for mirrored pairs)" if grid else
                          "canonical delta-eval FLOPs (14 per entry)",
        },
    }
    # issue-slot roofline of the dominant kernel: its inner loop's instruction
    # mix (from its gfx950 assembly) priced at the issue rates measured now
    if dom_name in SLOT_MIX:
        rates = sl1m.issue_rates(dev)
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        per_unit, n32, n64, ntr = SLOT_MIX[dom_name]
        t_model = (n_pix * n_vis / per_unit) / cus * (
            n32 / rates["fp32_fma"] + n64 / rates["fp64_fma"] + ntr / rates["sin_cos"])
        out["roofline"]["slots"] = {
            "unit": "wave64 instructions per s per CU", "rates": rates, "cus": cus,
            "mix_per_unit": {"entries": per_unit, "fp32_rate": n32, "fp64": n64,
                             "sin_cos": ntr},
            "model_ms": t_model * 1e3, "frac": t_model * 1e3 / dom_ms}
    if not args.no_extras:
        out["extras"] = extras(plan, wl, dev)
    if not args.no_cpu_baseline:
        try:
            threads = max(1, min(16, len(os.sched_getaffinity(0))))
        except AttributeError:
            threads = 1
        out["cpu_baseline"] = cpu_baseline(wl, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
