"""Benchmark of the SL1M hot path on one MI355X.

Headline workload: config 4 of the measurement plan, the NGC2403-size
problem -- a 1024x1024 wide-field delta grid over l, m in +-0.35 plus
wide-field Gaussian-pixel layers with sigma = 2, 4, 8 grid spacings on 512^2,
256^2 and 128^2 grids (1,392,640 pixels), 409,600 visibilities of a
256-antenna array (13 snapshots, 150 MHz) with per-antenna complex gains and
Gaussian primary beams, FP32 operator with FP64 phase, lambda = 3 sigma
sqrt(N_v).  A step is one FISTA iteration of the L1 solve: forward operator,
residual, adjoint, threshold and momentum update (2 x N_p x N_v
pixel-visibility evaluations).  The timed region is one sl1m_solve call of
exactly `--steps` iterations with L fixed beforehand; it ends with the
objective's forward (counted: evals = (2 steps + 1) N_p N_v).

Reported beside it, in the same JSON line:
* the full L1 solve of the workload (30 power-iteration steps for L, 100
  FISTA iterations, objective), timed once: `l1_solve_time_s`;
* per-kernel durations of the grid evaluation (HIP events recorded by the
  library around each launch, on the launch stream) and the dominant
  kernel's roofline: its executed FLOPs against the FP32 vector peak, and
  its issue-slot model priced at the issue rates measured on this GPU;
* the served-latency part of the metric: config 5's stream of 256 requests
  (Poisson arrivals at 4/s, 200 FISTA iterations each), batched by the
  library's continuous-batching server and one at a time, p50/p99/mean
  latency and evals/s; plus a saturated stream (the first 64 requests at
  4x the arrival rate);
* config 2's FISTA iteration (256^2 delta grid, 97,536 visibilities) as a
  secondary operator figure, and at its shape 1, 2, 4 and 8 right-hand
  sides through the FP32 grid evaluation and the float16 / bfloat16
  matrix-core plans (`config2_shape_multi_rhs`);
* the FP64 CPU oracle's rate on a bounded sample of config 4
  (`cpu_baseline`).
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
FLOP_PER_EVAL_GAUSS_WIDE = 26       # + taper 9, amplitude 1, kappa FMA 2
# The same counting rules (FMA = 2, sin, cos, exp2 = 1) applied to what the
# grid kernels execute: a mirrored pair of delta cells (8 entries) costs one
# FP64 phase FMA, one sin/cos pair and about 20 FP32 operations, 36 FLOP; a
# single delta cell (4 entries) 24; a Gaussian cell (4 entries) one sin/cos
# pair, two exp2 and about 26 FP32 operations, at most 32.
EXEC_FLOP_PER_EVAL = {
    "k_grid_fwd_delta_pairs": 4.5,
    "k_grid_adj_delta_square": 4.5,
    "k_grid_fwd_delta": 6.0,
    "k_grid_adj_delta": 6.0,
    "k_grid_fwd_gauss_pairs": 8.0,
    "k_grid_adj_gauss_multi": 8.0,
    "k_fwd_delta<float,4>": 14.0,
    "k_adj_delta<float,4>": 14.0,
}


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


# Inner-loop instruction mix of the grid kernels (counted in their gfx950
# assembly): entries per wavefront unit of work, then FP32-rate (FP32
# arithmetic, bit operations, integer), FP64, sin/cos and exp2 wave64
# instructions per unit.  Units: the pair adjoints' a wavefront and a
# visibility (64 lanes x 32 entries); the delta pair forward's a wavefront
# and a (pair record, visibility) (64 lanes x 8 entries, with the per-|l|
# phasors spread over the 8 records); the Gaussian pair forward's a wavefront
# and an |l| value (64 lanes x 8 pair records x 8 entries); the direct
# kernels' a wavefront and an entry.
SLOT_MIX = {
    "k_grid_adj_delta_square": (2048, 72, 6, 12, 0),
    "k_grid_fwd_delta_pairs": (512, 21.25, 1.25, 2.5, 0),
    "k_grid_adj_gauss_multi": (2048, 158, 10, 12, 4),
    "k_grid_fwd_gauss_pairs": (4096, 319, 18, 20, 4),
    "k_adj_delta<float,4>": (64, 3, 3, 2, 0),
    "k_fwd_delta<float,4>": (64, 3, 3, 2, 0),
}


def slot_model_s(name, evals, rates, cus):
    """Issue-slot time of `evals` entries of kernel `name` at the measured
    per-CU issue rates."""
    per_unit, n32, n64, ntr, nexp = SLOT_MIX[name]
    return (evals / per_unit) / cus * (n32 / rates["fp32_fma"] + n64 / rates["fp64_fma"]
                                       + ntr / rates["sin_cos"] + nexp / rates["exp"])


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
                         ("k_grid_adj_delta", "k_grid_adj_delta("),
                         ("k_grid_fwd_gauss_pairs", "k_grid_fwd_gauss_pairs"),
                         ("k_grid_adj_gauss_multi", "k_grid_adj_gauss_multi")):
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


def _time_ops(plan, fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def multi_rhs_table(wl2, dev, reps: int = 5):
    """1, 2, 4 and 8 right-hand sides (the paper's polarisations, or stacked
    iterates) through one plan at config 2's shape: the FP32 grid plan
    against the float16 and bfloat16 matrix-core plans, forward and adjoint
    times and side-products per second (2 R N_p N_v per operator pair)."""
    import torch
    from paper_1310_2078_amd import sl1m
    ev = wl2.n_pix * wl2.n_vis
    out = {}
    for R in (1, 2, 4, 8):
        X = torch.as_tensor(np.random.default_rng(5).standard_normal((R, wl2.n_pix)),
                            dtype=torch.float32, device=dev)
        for label, kw in (("fp32_grid", {}), ("mfma_f16", {"precision": "mfma_f16"}),
                          ("mfma_bf16", {"precision": "mfma_bf16"})):
            pm = sl1m.Plan.from_workload(wl2, device=dev, max_rhs=R, **kw)
            if R == 1:
                Vm = pm.forward(X[0])
                G = torch.empty(wl2.n_pix, dtype=torch.float32, device=dev)
                tf = _time_ops(pm, lambda: pm.forward(X[0], out=Vm), reps)
                ta = _time_ops(pm, lambda: pm.adjoint(Vm, out=G), reps)
            else:
                Vm = pm.forward_multi(X)
                G = torch.empty((R, wl2.n_pix), dtype=torch.float32, device=dev)
                tf = _time_ops(pm, lambda: pm.forward_multi(X, out=Vm), reps)
                ta = _time_ops(pm, lambda: pm.adjoint_multi(Vm, out=G), reps)
            out[f"R{R}_{label}"] = {"forward_ms": tf * 1e3, "adjoint_ms": ta * 1e3,
                                    "side_products_per_s": 2 * R * ev / (tf + ta),
                                    "grid_mfma": pm.info()["grid_mfma"]}
            print(f"[bench] multi-RHS R={R} {label}: {out[f'R{R}_{label}']}", file=sys.stderr,
                  flush=True)
            pm.close()
            del pm, Vm, G
    return out


def extras(plan2, wl2, dev, c4):
    """More workloads (`--extras`), reported beside the headline line (not in
    `value`): direct evaluation, warm starts, MFISTA, several right-hand
    sides, one GPU's share of config 4, the quad-tree refinement and the FP64
    config 1 solve."""
    import torch
    from paper_1310_2078_amd import sl1m
    from paper_1310_2078_amd import workloads as W
    ex = {}
    # the same FISTA iteration with every entry evaluated directly (no grid
    # factorisation), for comparison with the headline evaluation
    # (FP64 phase), and with the phase formed in float32 hi/lo arithmetic
    for key, kw in (("config2_direct_evaluation", dict(grid="off")),
                    ("config2_direct_hilo_phase", dict(precision="fp32_hilo"))):
        pdir = sl1m.Plan.from_workload(wl2, device=dev, **kw)
        Vd = pdir.forward(wl2.x_true)
        Ld = 1.01 * pdir.estimate_L(10, seed=0)
        pdir.solve(Vd, wl2.lam, 3, L=Ld)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pdir.solve(Vd, wl2.lam, 20, L=Ld)
        torch.cuda.synchronize()
        td = time.perf_counter() - t0
        ex[key] = {"iterations": 20, "time_s": td,
                   "evals_per_s": 2.0 * wl2.n_pix * wl2.n_vis * 20 / td}
        print(f"[bench] {key}: {ex[key]}", file=sys.stderr, flush=True)
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
    # several right-hand sides at config 2's shape: FP32 grid evaluation
    # against the matrix-core plans (float16, bfloat16)
    ex["config2_shape_multi_rhs"] = multi_rhs_table(wl2, dev)
    # config 4 (the headline workload): one GPU's share of it split over 8
    # GPUs by visibilities (every 8th record, all pixels: the grid evaluation
    # keeps its square pixel grid)
    wl4, V4d, Ve32, rate4 = c4["wl"], c4["data"], c4["extended_data"], c4["evals_per_s"]
    rng = np.random.default_rng(5)
    x4 = torch.as_tensor(rng.standard_normal(wl4.n_pix), dtype=torch.float32, device=dev)
    ws = dataclasses.replace(wl4, u=wl4.u[::8], v=wl4.v[::8], w=wl4.w[::8],
                             ant_p=wl4.ant_p[::8], ant_q=wl4.ant_q[::8], noise=None)
    ps = sl1m.Plan.from_workload(ws, device=dev)
    Vs = ps.forward(x4)
    gsh = torch.empty(wl4.n_pix, dtype=torch.float32, device=dev)
    tfs = _time_ops(ps, lambda: ps.forward(x4, out=Vs), 3)
    tas = _time_ops(ps, lambda: ps.adjoint(Vs, out=gsh), 3)
    rate_s = 2 * ws.n_pix * ws.n_vis / (tfs + tas)
    ex["config4_shard_1_of_8_by_visibilities"] = {
        "n_pix": ws.n_pix, "n_vis": ws.n_vis, "forward_ms": tfs * 1e3, "adjoint_ms": tas * 1e3,
        "evals_per_s": rate_s, "rate_vs_full_config4": rate_s / rate4}
    ps.close()
    del ps, Vs, gsh, x4
    # warm starts on config 4 (Section "Acceleration strategies"): relative
    # objective gap after k iterations from a zero image, from the dirty
    # image, and coarse-to-fine (the 512^2 delta grid with the same Gaussian
    # layers solved for 50 iterations, upscaled to the 1024^2 grid), with F*
    # from a 200-iteration cold solve; seconds include every level
    from paper_1310_2078_amd import coarse as CF
    p4 = sl1m.Plan.from_workload(wl4, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, ref4 = p4.solve(V4d, wl4.lam, 200, L=0.0, power_iters=wl4.power_iters)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    L4 = ref4["L"]
    D4 = p4.dirty_image(V4d)
    gk = wl4.kind != 0
    extra = (wl4.l[gk], wl4.m[gk], wl4.sigma[gk], wl4.kind[gk])
    ws = {}
    for k in (10, 30, 100):
        rec = {}
        for label, x0 in (("cold", None), ("dirty_start", D4)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, inf = p4.solve(V4d, wl4.lam, k, L=L4, x0=x0)
            torch.cuda.synchronize()
            rec[label] = {"gap": (inf["F"] - ref4["F"]) / ref4["F"],
                          "seconds": time.perf_counter() - t0}
        t0 = time.perf_counter()
        lv = CF.coarse_to_fine(1024, 0.35, 2, wl4.u, wl4.v, wl4.w, V4d, wl4.lam, [50, k],
                               power_iters=wl4.power_iters, extra=extra, device=dev,
                               ant_p=wl4.ant_p, ant_q=wl4.ant_q, ant_gain=wl4.ant_gain,
                               ant_fwhm=wl4.ant_fwhm, L_per_level=[0.0, L4])
        rec["coarse_to_fine"] = {"gap": (lv[-1].info["F"] - ref4["F"]) / ref4["F"],
                                 "seconds": time.perf_counter() - t0,
                                 "coarse_level_seconds": lv[0].seconds}
        ws[str(k)] = rec
    ex["config4_warm_starts"] = {"F_star_200_iterations": ref4["F"], "F_star_seconds": t_ref,
                                 "after_k_iterations": ws}
    p4.close()
    del p4, D4
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




def cpu_baseline(wl, threads: int):
    """The FP64 oracle, untuned, on a bounded sample of config 4: the forward
    of every 32nd pixel of each pixel kind and layer (its mix of delta and
    Gaussian pixels, gains included) for the first 512 x threads
    visibilities, and the adjoint of 2048 x threads pixels spread evenly over
    the image against every 32nd visibility.  Returns evals/s over both."""
    import oracle as O
    sub = np.arange(0, wl.n_pix, 32)
    nf = min(wl.n_vis, 512 * threads)
    pf = O.Problem(l=wl.l[sub], m=wl.m[sub], u=wl.u[:nf], v=wl.v[:nf], w=wl.w[:nf],
                   sigma=wl.sigma[sub], kind=wl.kind[sub], ant_p=wl.ant_p[:nf],
                   ant_q=wl.ant_q[:nf], ant_gain=wl.ant_gain, ant_fwhm=wl.ant_fwhm,
                   threads=threads)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(sub.size)
    t0 = time.perf_counter()
    O.forward(pf, x)
    tf = time.perf_counter() - t0
    ks = np.arange(0, wl.n_vis, 32)
    na = min(wl.n_pix, 2048 * threads)
    js = np.linspace(0, wl.n_pix - 1, na).astype(np.int64)
    pa = O.Problem(l=wl.l, m=wl.m, u=wl.u[ks], v=wl.v[ks], w=wl.w[ks], sigma=wl.sigma,
                   kind=wl.kind, ant_p=wl.ant_p[ks], ant_q=wl.ant_q[ks], ant_gain=wl.ant_gain,
                   ant_fwhm=wl.ant_fwhm, threads=threads)
    r = rng.standard_normal(ks.size) + 1j * rng.standard_normal(ks.size)
    t0 = time.perf_counter()
    O.adjoint_cols(pa, r, js)
    ta = time.perf_counter() - t0
    evals = sub.size * nf + na * ks.size
    return {
        "value": evals / (tf + ta),
        "unit": "evals/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"config 4: forward of every 32nd pixel ({sub.size}, all kinds and layers) x "
                  f"the first {nf} visibilities + adjoint of {na} pixels spread over the image x "
                  f"every 32nd visibility ({ks.size}); gains and beams included "
                  f"({evals:.3e} evals, {tf + ta:.1f} s)",
    }


def config4_data(wl4, plan, dev):
    """Config 4's data (not timed): the point sources through the operator,
    the 50 extended sources as a fine FP64 sum of delta points (not the
    Gaussian-pixel model), and noise."""
    import torch
    from paper_1310_2078_amd import sl1m
    pe = sl1m.Plan(wl4.extra_l, wl4.extra_m, wl4.u, wl4.v, wl4.w, ant_p=wl4.ant_p,
                   ant_q=wl4.ant_q, ant_gain=wl4.ant_gain, ant_fwhm=wl4.ant_fwhm,
                   precision="fp64", device=dev)
    Ve32 = pe.forward(wl4.extra_flux).to(torch.complex64)
    pe.close()
    noise = torch.as_tensor(wl4.noise, dtype=torch.complex64, device=dev)
    return plan.forward(wl4.x_true) + Ve32 + noise, Ve32 + noise


def dominant_kernel(pinfo, tim, n_delta, n_gauss, n_vis, n_layers):
    """The grid kernel with the longest average launch in the timed region:
    (name, average ms, evals per launch)."""
    pairs = bool(pinfo["grid_pairs"])
    cands = [
        ("k_grid_fwd_delta_pairs" if pairs else "k_grid_fwd_delta", "grid_fwd_delta",
         n_delta * n_vis),
        ("k_grid_adj_delta_square" if pairs else "k_grid_adj_delta", "grid_adj_delta",
         n_delta * n_vis),
        ("k_grid_adj_gauss_multi", "grid_adj_gauss", n_gauss * n_vis),
        # one launch per layer: evals per launch on average
        ("k_grid_fwd_gauss_pairs", "grid_fwd_gauss", n_gauss * n_vis / max(n_layers, 1)),
    ]
    best = None
    for name, key, ev in cands:
        n, ms = tim.get(key, (0, 0.0))
        if n == 0:
            continue
        avg = ms / n
        if best is None or avg > best[1]:
            best = (name, avg, ev)
    return best


def headline(args, dev):
    import torch
    from paper_1310_2078_amd import sl1m
    from paper_1310_2078_amd import workloads as W

    wl4 = W.config4()
    n_pix, n_vis = wl4.n_pix, wl4.n_vis
    n_delta = int(np.sum(wl4.kind == W.PIX_DELTA))
    n_gauss = n_pix - n_delta
    n_layers = len(np.unique(wl4.sigma[wl4.kind != W.PIX_DELTA]))
    print(f"[bench] config4 n_pix={n_pix} n_vis={n_vis} steps={args.steps} "
          f"warmup={args.warmup}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plan = sl1m.Plan.from_workload(wl4, device=dev)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    tuning = None
    if args.tune:
        tuning = plan.tune(reps=3)
        plan.close()
        plan = sl1m.Plan.from_workload(wl4, device=dev, tuning=tuning)
        print(f"[bench] tuning {tuning}", file=sys.stderr, flush=True)
    V, V_ext = config4_data(wl4, plan, dev)
    torch.cuda.synchronize()

    # the full L1 solve: 30 power steps, 100 iterations, objective
    t0 = time.perf_counter()
    img, info = plan.solve(V, wl4.lam, wl4.n_iter, L=0.0, power_iters=wl4.power_iters)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    L = info["L"]
    solve_evals = float(n_pix) * n_vis * (2 * (wl4.power_iters + wl4.n_iter) + 1)
    print(f"[bench] full solve {t_solve:.3f} s; info {info}", file=sys.stderr, flush=True)

    if args.warmup > 0:
        plan.solve(V, wl4.lam, args.warmup, L=L)
    torch.cuda.synchronize()
    plan.timing_begin(max(16, 4 * args.steps + 16))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    img, info_k = plan.solve(V, wl4.lam, args.steps, L=L)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tim = plan.timing_end()
    evals = float(n_pix) * n_vis * (2 * args.steps + 1)
    print(f"[bench] {args.steps} iterations in {elapsed:.4f} s; timing {tim}",
          file=sys.stderr, flush=True)
    for _ in range(args.profile_ops):
        plan.adjoint(plan.forward(img))
    torch.cuda.synchronize()

    pinfo = plan.info()
    plan_shape = {k: pinfo[k] for k in PLAN_KEYS}
    avg = {k: (ms / n if n else 0.0) for k, (n, ms) in tim.items()}
    dom_name, dom_ms, dom_evals = dominant_kernel(pinfo, tim, n_delta, n_gauss, n_vis, n_layers)
    exec_flop = EXEC_FLOP_PER_EVAL[dom_name]
    achieved = exec_flop * dom_evals / (dom_ms * 1e-3) / 1e12
    canonical = (FLOP_PER_EVAL_DELTA if "delta" in dom_name else FLOP_PER_EVAL_GAUSS_WIDE)
    # executed FLOPs of one iteration (both operators) over the time of a step
    exec_step = 2 * n_vis * (n_delta * EXEC_FLOP_PER_EVAL["k_grid_adj_delta_square"]
                             + n_gauss * EXEC_FLOP_PER_EVAL["k_grid_adj_gauss_multi"])
    canon_step = 2 * n_vis * (n_delta * FLOP_PER_EVAL_DELTA + n_gauss * FLOP_PER_EVAL_GAUSS_WIDE)
    step_s = elapsed / args.steps
    roof = {
        "bound": "alu",
        "kernel": dom_name,
        "achieved": achieved,
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_TFLOPS,
        "traffic": load_traffic(dom_name, plan_shape),
        "kernel_avg_ms": dom_ms,
        "evals_per_launch": dom_evals,
        "executed_flop_per_eval": exec_flop,
        "accounting": "achieved/frac: the FLOPs the kernel executes (FMA = 2; sin, cos, exp2 = "
                      "1; the grid factorisation shares one sincos among 4 or 8 entries) over "
                      "its average launch duration (HIP events on the launch stream); "
                      "effective_*: the direct evaluation's count per entry at the same rate",
        "effective_flop_per_eval": canonical,
        "effective_tflops": canonical * dom_evals / (dom_ms * 1e-3) / 1e12,
    }
    rates = sl1m.issue_rates(dev)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    if dom_name in SLOT_MIX:
        per_unit, n32, n64, ntr, nexp = SLOT_MIX[dom_name]
        t_model = slot_model_s(dom_name, dom_evals, rates, cus)
        roof["slots"] = {
            "unit": "wave64 instructions per s per CU", "rates": rates, "cus": cus,
            "mix_per_unit": {"entries": per_unit, "fp32_rate": n32, "fp64": n64, "sin_cos": ntr,
                             "exp": nexp},
            "model_ms": t_model * 1e3, "frac": t_model * 1e3 / dom_ms}
    out = {
        "metric": "pixel x visibility evals/s (forward + adjoint) of the L1 solve on config 4; "
                  "L1 solve time; p50/p99 served latency (config 5)",
        "value": evals / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * step_s,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 phase)",
        "data": "synthetic",
        "config": {
            "workload": "config4: 1024^2 wide-field delta grid over +-0.35 plus wide-field "
                        "Gaussian layers sigma = 2, 4, 8 spacings (512^2, 256^2, 128^2), "
                        "1,392,640 pixels; 409,600 visibilities (256 antennas, 13 snapshots, "
                        "150 MHz); per-antenna gains and 0.4 rad primary beams; FISTA "
                        "lambda = 3 sigma sqrt(N_v)",
            "n_pix": n_pix,
            "n_vis": n_vis,
            "evals_per_step": 2 * n_pix * n_vis,
            "evaluation": "grid" if pinfo["grid"] else "direct",
            "tuning": tuning,
            "plan": plan_shape,
        },
        "l1_solve_time_s": t_solve,
        "solve": {
            "power_iterations": wl4.power_iters, "iterations": wl4.n_iter,
            "time_s": t_solve, "evals": solve_evals, "evals_per_s": solve_evals / t_solve,
            "L": L, "F": info["F"], "l2_term": info["l2_term"], "l1_term": info["l1_term"],
            "nnz": info["nnz"], "plan_s": t_plan},
        "kernels": {
            "forward_avg_ms": avg["forward"],
            "adjoint_avg_ms": avg["adjoint"],
            "fista_update_avg_ms": avg["fista"],
            "grid_fwd_delta_avg_ms": avg["grid_fwd_delta"],
            "grid_adj_delta_avg_ms": avg["grid_adj_delta"],
            "grid_fwd_gauss_avg_ms_per_layer": avg["grid_fwd_gauss"],
            "grid_adj_gauss_avg_ms": avg["grid_adj_gauss"],
            # the update's algorithmic bytes: read the gradient (adjoint
            # output), scale, y and I, write y and I -- 20 B per pixel
            "fista_update_hbm_gbs": 20.0 * n_pix / (avg["fista"] * 1e-3) / 1e9
                                    if avg["fista"] else None,
            "fista_update_hbm_frac": 20.0 * n_pix / (avg["fista"] * 1e-3) / HBM_PEAK_BPS
                                     if avg["fista"] else None,
            "fista_update_rows_read": pinfo["n_achunks"],
            "executed_tflops_per_step": exec_step / step_s / 1e12,
            "effective_tflops_per_step": canon_step / step_s / 1e12,
        },
        "roofline": roof,
    }
    # every grid kernel against its issue-slot model (per launch)
    pairs = bool(pinfo["grid_pairs"])
    slot = {}
    for name, key, ev in (("k_grid_fwd_delta_pairs", "grid_fwd_delta", n_delta * n_vis),
                          ("k_grid_adj_delta_square", "grid_adj_delta", n_delta * n_vis),
                          ("k_grid_adj_gauss_multi", "grid_adj_gauss", n_gauss * n_vis),
                          ("k_grid_fwd_gauss_pairs", "grid_fwd_gauss", n_gauss * n_vis / n_layers)):
        if pairs and avg.get(key) and name in SLOT_MIX:
            slot[name] = slot_model_s(name, ev, rates, cus) * 1e3 / avg[key]
    out["kernels"]["slot_frac"] = slot
    ctx = {"wl": wl4, "plan": plan, "data": V, "extended_data": V_ext,
           "evals_per_s": evals / elapsed}
    return out, ctx


def config2_secondary(dev, steps=20):
    """Config 2's FISTA iteration (a 256^2 delta grid over +-0.3, 97,536
    visibilities): evals/s and kernel durations."""
    import torch
    from paper_1310_2078_amd import sl1m
    from paper_1310_2078_amd import workloads as W
    wl = W.config2()
    plan = sl1m.Plan.from_workload(wl, device=dev)
    V = plan.forward(wl.x_true) + torch.as_tensor(wl.noise, dtype=torch.complex64, device=dev)
    L = 1.01 * plan.estimate_L(wl.power_iters, seed=0)
    plan.solve(V, wl.lam, 3, L=L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.solve(V, wl.lam, steps, L=L)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.timing_begin(4 * steps + 16)
    plan.solve(V, wl.lam, steps, L=L)
    tim = plan.timing_end()
    avg = {k: (ms / n if n else 0.0) for k, (n, ms) in tim.items()}
    pinfo = plan.info()
    out = {"n_pix": wl.n_pix, "n_vis": wl.n_vis, "iterations": steps,
           "ms_per_iteration": 1e3 * el / steps,
           "evals_per_s": float(wl.n_pix) * wl.n_vis * (2 * steps + 1) / el,
           "forward_avg_ms": avg["forward"], "adjoint_avg_ms": avg["adjoint"],
           "fista_update_avg_ms": avg["fista"],
           "grid_adj_delta_avg_ms": avg["grid_adj_delta"],
           "grid_fwd_delta_avg_ms": avg["grid_fwd_delta"],
           "plan": {k: pinfo[k] for k in PLAN_KEYS}}
    name = "k_grid_adj_delta_square"
    if avg["grid_adj_delta"] and name in SLOT_MIX:
        rates = sl1m.issue_rates(dev)
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        t_model = slot_model_s(name, wl.n_pix * wl.n_vis, rates, cus)
        out["adjoint_slot_frac"] = t_model * 1e3 / avg["grid_adj_delta"]
        out["adjoint_executed_frac"] = (EXEC_FLOP_PER_EVAL[name] * wl.n_pix * wl.n_vis
                                        / (avg["grid_adj_delta"] * 1e-3) / 1e12
                                        / PEAK_FP32_TFLOPS)
        out["adjoint_traffic"] = load_traffic(name, out["plan"])
    return plan, wl, out


def serving(dev, n_req: int, n_sat: int):
    """Config 5: the 256-request stream batched and one at a time, and a
    saturated stream of its first `n_sat` requests at 4x the arrival rate."""
    from paper_1310_2078_amd import serve as S
    res = {}
    runs = [("stream", n_req, 1.0)]
    if n_sat > 0:
        runs.append(("saturated", n_sat, 0.25))
    for key, n, scale in runs:
        arrivals, reqs = S.make_stream(n, scale)
        print(f"[bench] serving {key}: preparing {n} requests", file=sys.stderr, flush=True)
        data = S.prepare(reqs, dev)
        rec = {"requests": n, "arrival_rate_per_s": n / float(arrivals[-1]),
               "offered_evals": sum(S.request_evals(r) for r in reqs)}
        rec["batched"], _ = S.run_batched(arrivals, reqs, data, dev, log=sys.stderr)
        print(f"[bench] serving {key} batched {rec['batched']}", file=sys.stderr, flush=True)
        rec["unbatched"], _ = S.run_unbatched(arrivals, reqs, data, dev, log=sys.stderr)
        print(f"[bench] serving {key} unbatched {rec['unbatched']}", file=sys.stderr, flush=True)
        res[key] = rec
        del data
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the config 5 request streams")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-saturated", type=int, default=64,
                    help="requests in the saturated stream (4x arrival rate); 0 skips it")
    ap.add_argument("--no-config2", action="store_true")
    ap.add_argument("--extras", action="store_true",
                    help="also run the secondary workloads (direct evaluation, warm starts, "
                         "MFISTA, several right-hand sides, quad-tree, FP64 config 1)")
    ap.add_argument("--multi-rhs-only", action="store_true",
                    help="only the several-right-hand-sides table at config 2's shape "
                         "(FP32 grid against the matrix-core plans), as one JSON line")
    ap.add_argument("--tune", action="store_true",
                    help="tune the headline plan's launch shapes (sl1m_tune) first")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM counters)")
    ap.add_argument("--ingest-counters", nargs="+", metavar="PATH",
                    help="FETCH_CSV WRITE_CSV [BENCH_OUT]: turn two rocprofv3 --pmc counter CSVs "
                         "(FETCH_SIZE, WRITE_SIZE) of a --calib-copy run into "
                         "profiles/traffic.json (with the run's plan split, read from its "
                         "output line) and exit")
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
              "(sharding over several GPUs, by visibilities for grid plans and by pixels "
              "otherwise, is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.multi_rhs_only:
        from paper_1310_2078_amd import workloads as W
        print(json.dumps({"config2_shape_multi_rhs": multi_rhs_table(W.config2(), dev)}),
              flush=True)
        return
    out, c4 = headline(args, dev)
    c4.pop("plan").close()
    if args.calib_copy:
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # an elementwise kernel: reads and writes CALIB_BYTES
        torch.cuda.synchronize()
        del src, dst
    if not args.no_serving:
        out["serving"] = serving(dev, args.serve_requests, args.serve_saturated)
        st = out["serving"]["stream"]
        out["p50_s"] = st["batched"]["p50_s"]
        out["p99_s"] = st["batched"]["p99_s"]
    plan2 = wl2 = None
    if not args.no_config2 or args.extras:
        plan2, wl2, out["config2"] = config2_secondary(dev)
        print(f"[bench] config2 {out['config2']}", file=sys.stderr, flush=True)
        if not args.extras:
            # several right-hand sides (Stokes images) at config 2's shape:
            # FP32 grid against the matrix-core plans (also in --extras)
            out["config2_shape_multi_rhs"] = multi_rhs_table(wl2, dev)
    if args.extras:
        out["extras"] = extras(plan2, wl2, dev, c4)
    if not args.no_cpu_baseline:
        try:
            threads = max(1, min(16, len(os.sched_getaffinity(0))))
        except AttributeError:
            threads = 1
        print(f"[bench] cpu baseline on {threads} threads", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(c4["wl"], threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
