"""Autotuning of launch shapes (sl1m_tune) and explicit lane counts, through
the C ABI.  A tuned plan computes the same operator (oracle tolerance); the
tuner's choice is never slower than the default it timed beside it."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1310_2078_amd import sl1m
from paper_1310_2078_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("name", ["config1", "irregular", "config1_gauss_layers"])
def test_tuned_plan_matches_oracle(name):
    if name == "config1":
        wl = W.config1()
    elif name == "irregular":
        wl = W.small_random(31, 3001, 2503, kind=W.PIX_GAUSS_WIDE, sigma=2e-3, with_gains=True)
    else:
        wl = W.config1()
        wl.kind = np.full(wl.n_pix, W.PIX_GAUSS_WIDE, np.uint8)
        wl.sigma = np.full(wl.n_pix, 2e-3)
    say(f"[case] tune {name} n_pix={wl.n_pix} n_vis={wl.n_vis}")
    base = sl1m.Plan.from_workload(wl)
    t = base.tune(reps=3)
    base.close()
    say(f"    tuning {t}")
    assert t["candidates"] >= 2
    assert t["forward_ms"] + t["adjoint_ms"] <= t["default_forward_ms"] + t["default_adjoint_ms"]
    plan = sl1m.Plan.from_workload(wl, tuning=t)
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    ef = rel(plan.forward(x).cpu().numpy(), O.forward(p, x))
    ea = rel(plan.adjoint(r).cpu().numpy(), O.adjoint(p, r))
    say(f"    tuned plan forward {ef:.3e} adjoint {ea:.3e}")
    assert ef <= 1e-5 and ea <= 1e-5


@pytest.mark.parametrize("vpl,ppl", [(1, 1), (2, 4), (4, 2)])
def test_explicit_lane_counts(vpl, ppl):
    """Direct kernels with every lane count the tuner may pick, on irregular
    pixels of two kinds with gains (ragged sizes)."""
    wl = W.small_random(32, 2777, 3101, with_gains=True)
    rng = np.random.default_rng(2)
    wl.kind = rng.choice([W.PIX_DELTA, W.PIX_GAUSS_WIDE], wl.n_pix).astype(np.uint8)
    wl.sigma = np.where(wl.kind == W.PIX_DELTA, 0.0, 2.5e-3)
    say(f"[case] lanes vpl={vpl} ppl={ppl}")
    plan = sl1m.Plan(wl.l, wl.m, wl.u, wl.v, wl.w, sigma=wl.sigma, kind=wl.kind, ant_p=wl.ant_p,
                     ant_q=wl.ant_q, ant_gain=wl.ant_gain, ant_fwhm=wl.ant_fwhm, grid="off",
                     fwd_vpl=vpl, adj_ppl=ppl)
    info = plan.info()
    assert info["fwd_vpl"] == vpl and info["adj_ppl"] == ppl
    p = O.Problem.from_workload(wl)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    ef = rel(plan.forward(x).cpu().numpy(), O.forward(p, x))
    ea = rel(plan.adjoint(r).cpu().numpy(), O.adjoint(p, r))
    say(f"    forward {ef:.3e} adjoint {ea:.3e}")
    assert ef <= 1e-5 and ea <= 1e-5
