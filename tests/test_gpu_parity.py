"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

FP32 mode: norm-relative error <= 1e-5 for both operators and every output
within its element-wise bound (tests/elementwise.py: the FP32 entry error
plus the probabilistic summation bound, times sum_j |M_kj| |x_j|); image
error of the FISTA solve <= 1e-4 of the peak.  FP64 mode: <= 1e-11 and the
FP64 element-wise bound.  Every case prints its name first so a failing GPU
step can be identified from the log.
"""
import math
import sys

import numpy as np
import pytest
import torch

import elementwise as E
import oracle as O
from paper_1310_2078_amd import sl1m
from paper_1310_2078_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-11, "fp32_hilo": 1e-5}
# element-wise bound of each precision (the hi/lo phase plan accumulates in
# float32 and its phase is off by about three roundings of 2^-24 turn, as the
# FP32 plan's)
EPREC = {"fp32": "fp32", "fp64": "fp64", "fp32_hilo": "fp32"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _rand(seed, n_pix, n_vis):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n_pix)
    r = rng.standard_normal(n_vis) + 1j * rng.standard_normal(n_vis)
    return x, r


def _check_ops(wl, prec, tag, x=None, r=None):
    say(f"[case] {tag} prec={prec} n_pix={wl.n_pix} n_vis={wl.n_vis}")
    plan = sl1m.Plan.from_workload(wl, precision=prec)
    p = O.Problem.from_workload(wl)
    xs, rs = _rand(99, wl.n_pix, wl.n_vis)
    x = xs if x is None else x
    r = rs if r is None else r
    Vg = plan.forward(x).cpu().numpy()
    Vo = O.forward(p, x)
    gg = plan.adjoint(r).cpu().numpy()
    go = O.adjoint(p, r)
    ef, ea = rel(Vg, Vo), rel(gg, go)
    wf = E.worst_ratio(Vg, Vo, E.abs_forward_rows(p, x), wl.n_pix, EPREC[prec])
    wa = E.worst_ratio(gg, go, E.abs_adjoint_cols(p, r), wl.n_vis, EPREC[prec])
    say(f"    forward rel err {ef:.3e}  adjoint rel err {ea:.3e}  "
        f"element-wise (fraction of bound) forward {wf:.3e} adjoint {wa:.3e}")
    assert ef <= TOL[prec] and ea <= TOL[prec]
    assert wf <= 1.0 and wa <= 1.0
    return plan


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp32_hilo"])
def test_config1_operators(prec):
    _check_ops(W.config1(), prec, "config1")


@pytest.mark.parametrize("kind,sigma,gains,distinct", [
    (W.PIX_DELTA, 0.0, False, False),
    (W.PIX_GAUSS_PARAXIAL, 3e-3, False, False),
    (W.PIX_GAUSS_WIDE, 3e-3, False, False),
    (W.PIX_DELTA, 0.0, True, False),
    (W.PIX_GAUSS_WIDE, 2e-3, True, False),
    (W.PIX_DELTA, 0.0, True, True),
    (W.PIX_GAUSS_WIDE, 2e-3, True, True),
])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_irregular_ragged_operators(kind, sigma, gains, distinct, prec):
    """Off-grid pixels over +-0.2, sizes that span several tiles and end in a
    ragged tail, every pixel kind, separable and per-pair gains."""
    wl = W.small_random(5, 2537, 3001, kind=kind, sigma=sigma, with_gains=gains,
                        distinct_fwhm=distinct, uv_radius=1200.0, w_sigma=300.0)
    _check_ops(wl, prec, f"irregular kind={kind} sigma={sigma} gains={gains} distinct={distinct}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mixed_kinds_and_layers(prec):
    """Delta, paraxial and wide-field pixels with several sigmas in one plan,
    interleaved in the caller's order (exercises grouping and permutation)."""
    rng = np.random.default_rng(8)
    wl = W.small_random(6, 3000, 1500, half_extent=0.3, with_gains=True)
    kinds = rng.integers(0, 3, wl.n_pix).astype(np.uint8)
    sig = rng.choice([1.5e-3, 3e-3, 6e-3], wl.n_pix)
    sig[kinds == 0] = 0.0
    wl.kind, wl.sigma = kinds, sig
    _check_ops(wl, prec, "mixed kinds/layers")


@pytest.mark.parametrize("tile_blocks", [0, 4096, 8192])
def test_config2_full_size_sampled(tile_blocks):
    """Config 2 at full size in the benchmark's launch configurations (the
    default split and the splits its tuner picks from): sampled visibilities
    (every 97th) and pixels (every 61st) against the oracle, and the adjoint
    identity on the full GPU vectors."""
    wl = W.config2()
    say(f"[case] config2 full n_pix={wl.n_pix} n_vis={wl.n_vis} tile_blocks={tile_blocks}")
    plan = sl1m.Plan.from_workload(wl, tile_blocks=tile_blocks)
    say(f"    info {plan.info()}")
    p = O.Problem.from_workload(wl)
    x, r = _rand(7, wl.n_pix, wl.n_vis)
    Vg = plan.forward(x).cpu().numpy()
    gg = plan.adjoint(r).cpu().numpy()
    ks = np.arange(0, wl.n_vis, 97)
    js = np.arange(0, wl.n_pix, 61)
    Vo, go = O.forward_rows(p, x, ks), O.adjoint_cols(p, r, js)
    ef = rel(Vg[ks], Vo)
    ea = rel(gg[js], go)
    wf = E.worst_ratio(Vg[ks], Vo, E.abs_forward_rows(p, x, ks), wl.n_pix)
    wa = E.worst_ratio(gg[js], go, E.abs_adjoint_cols(p, r, js), wl.n_vis)
    lhs = np.vdot(Vg.astype(np.complex128), r).real
    rhs = float(np.dot(x, gg.astype(np.float64)))
    ident = abs(lhs - rhs) / (np.linalg.norm(Vg) * np.linalg.norm(r))
    say(f"    sampled forward {ef:.3e} adjoint {ea:.3e} identity {ident:.3e}; "
        f"element-wise forward {wf:.3e} adjoint {wa:.3e}")
    assert ef <= 1e-5 and ea <= 1e-5 and ident <= 1e-5
    assert wf <= 1.0 and wa <= 1.0


def test_config2_long_baseline_precision_stress():
    """Radius-3 km array (phases ~1e4 rad): the FP64 phase with exact
    reduction keeps the FP32 operator within tolerance."""
    wl = W.config2(diameter_m=6000.0)
    sub = np.arange(0, wl.n_vis, 8)
    pix = np.arange(0, wl.n_pix, 16)
    wl2 = W.Workload("stress", wl.l[pix], wl.m[pix], wl.sigma[pix], wl.kind[pix],
                     wl.u[sub], wl.v[sub], wl.w[sub])
    assert np.max(np.abs(wl2.u)) > 2500
    _check_ops(wl2, "fp32", "config2 6km stress")


@pytest.mark.parametrize("gains", [False, True])
def test_hilo_phase_irregular_ragged(gains):
    """The FP32 hi/lo phase plan on off-grid delta pixels with a ragged tail
    (and separable gains with one beam width): within the FP32 bounds."""
    wl = W.small_random(5, 2537, 3001, with_gains=gains, uv_radius=1200.0, w_sigma=300.0)
    plan = _check_ops(wl, "fp32_hilo", f"hilo irregular gains={gains}")
    assert plan.info()["grid"] == 0


def test_hilo_phase_long_baseline_stress():
    """The radius-3 km array of the FP64-phase stress test (phases ~1e4 rad)
    with the phase formed in float32 hi/lo: the same tolerance holds."""
    wl = W.config2(diameter_m=6000.0)
    sub = np.arange(0, wl.n_vis, 8)
    pix = np.arange(0, wl.n_pix, 16)
    wl2 = W.Workload("stress", wl.l[pix], wl.m[pix], wl.sigma[pix], wl.kind[pix],
                     wl.u[sub], wl.v[sub], wl.w[sub])
    _check_ops(wl2, "fp32_hilo", "config2 6km stress, hi/lo phase")


def test_hilo_phase_rejects_gaussian_and_pair_beams():
    say("[case] hilo rejects")
    wl = W.small_random(9, 300, 200, kind=W.PIX_GAUSS_WIDE, sigma=2e-3)
    with pytest.raises(sl1m.SL1MError):
        sl1m.Plan.from_workload(wl, precision="fp32_hilo")
    wl = W.small_random(9, 300, 200, with_gains=True, distinct_fwhm=True)
    with pytest.raises(sl1m.SL1MError):
        sl1m.Plan.from_workload(wl, precision="fp32_hilo")


def test_empty_inputs():
    say("[case] empty inputs")
    wl = W.small_random(1, 10, 20)
    e1 = W.Workload("np0", wl.l[:0], wl.m[:0], wl.sigma[:0], wl.kind[:0], wl.u, wl.v, wl.w)
    plan = sl1m.Plan.from_workload(e1)
    V = plan.forward(np.zeros(0)).cpu().numpy()
    assert V.shape == (20,) and np.all(V == 0)
    e2 = W.Workload("nv0", wl.l, wl.m, wl.sigma, wl.kind, wl.u[:0], wl.v[:0], wl.w[:0])
    plan = sl1m.Plan.from_workload(e2)
    g = plan.adjoint(np.zeros(0, complex)).cpu().numpy()
    assert g.shape == (10,) and np.all(g == 0)
    V = plan.forward(np.ones(10)).cpu().numpy()
    assert V.shape == (0,)


def test_single_pixel_single_visibility():
    say("[case] 1x1")
    p = sl1m.Plan([0.6], [0.0], [5 / 12], [0.0], [0.0], precision="fp64")
    V = p.forward(np.ones(1)).cpu().numpy()
    np.testing.assert_allclose(V, [-1.25j], atol=1e-14)


def test_unit_delta_at_phase_centre():
    say("[case] unit delta at phase centre")
    wl = W.config1()
    plan = sl1m.Plan.from_workload(wl)
    x = np.zeros(wl.n_pix)
    x[16 + 32 * 16] = 1.0
    V = plan.forward(x).cpu().numpy()
    assert np.max(np.abs(V - 1.0)) < 2e-6


def test_determinism_and_permutation_invariance():
    say("[case] determinism / permutation")
    wl = W.small_random(4, 4000, 5000, half_extent=0.3)
    x, r = _rand(3, wl.n_pix, wl.n_vis)
    plan = sl1m.Plan.from_workload(wl)
    a = plan.forward(x).cpu().numpy()
    b = plan.forward(x).cpu().numpy()
    assert np.array_equal(a, b)
    ga = plan.adjoint(r).cpu().numpy()
    gb = plan.adjoint(r).cpu().numpy()
    assert np.array_equal(ga, gb)
    perm = np.random.default_rng(0).permutation(wl.n_pix)
    plan2 = sl1m.Plan(wl.l[perm], wl.m[perm], wl.u, wl.v, wl.w)
    c = plan2.forward(x[perm]).cpu().numpy()
    assert rel(c, a) < 2e-6
    gc = plan2.adjoint(r).cpu().numpy()
    assert rel(gc, ga[perm]) < 1e-12


def test_domain_and_argument_errors():
    say("[case] errors")
    with pytest.raises(sl1m.SL1MError) as e:
        sl1m.Plan([0.8, 0.7], [0.7, 0.0], [1.0], [1.0], [1.0])
    assert e.value.status == sl1m.EDOMAIN
    with pytest.raises(sl1m.SL1MError) as e:
        sl1m.Plan([0.1], [0.0], [1.0], [1.0], [float("nan")])
    assert e.value.status == sl1m.EDOMAIN
    with pytest.raises(sl1m.SL1MError) as e:
        sl1m.Plan([0.1], [0.0], [1.0, 2.0], [1.0, 2.0], [1.0, 2.0], ant_p=[0, 5], ant_q=[1, 1],
                  ant_gain=np.ones(2, complex))
    assert e.value.status == sl1m.EINVAL
    with pytest.raises(sl1m.SL1MError) as e:
        sl1m.Plan([0.1], [0.0], [1.0], [1.0], [1.0], sigma=[-1.0])
    assert e.value.status == sl1m.EDOMAIN


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp32_hilo"])
def test_estimate_L_matches_oracle(prec):
    say(f"[case] estimate_L {prec}")
    wl = W.config1()
    plan = sl1m.Plan.from_workload(wl, precision=prec)
    op = O.Operator(O.Problem.from_workload(wl))
    _, rq_o = O.power_iteration(op, 30, seed=0)
    rq_g = plan.estimate_L(30, seed=0)
    say(f"    oracle {rq_o:.10g} gpu {rq_g:.10g}")
    assert abs(rq_g - rq_o) <= (1e-11 if prec == "fp64" else 1e-5) * rq_o


def _config1_data():
    wl = W.config1()
    op = O.Operator(O.Problem.from_workload(wl))
    V = op.forward(wl.x_true) + wl.noise
    L, _ = O.power_iteration(op, 30, seed=0)
    return wl, op, V, L


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp32_hilo"])
def test_config1_solve_matches_oracle(prec):
    """Config 1: 100 FISTA iterations with the same L; image error relative to
    the peak, plus the reported objective terms."""
    say(f"[case] config1 solve {prec}")
    wl, op, V, L = _config1_data()
    ref = O.fista(op, V, L, wl.lam, wl.n_iter)
    plan = sl1m.Plan.from_workload(wl, precision=prec)
    img, info = plan.solve(V, wl.lam, wl.n_iter, L=L)
    img = img.cpu().numpy()
    err = np.max(np.abs(img - ref.image)) / np.max(ref.image)
    say(f"    image err/peak {err:.3e}  F gpu {info['F']:.8g} oracle {ref.F:.8g}  nnz {info['nnz']} {ref.nnz}")
    tol = 1e-10 if prec == "fp64" else 1e-4
    assert err <= tol
    assert info["iters"] == wl.n_iter and info["status"] == 0
    assert abs(info["F"] - ref.F) <= tol * ref.F
    assert abs(info["l1_term"] - ref.l1_term) <= 1e-4 * ref.l1_term


def test_solve_with_estimated_L_and_termination():
    say("[case] solve eps / estimated L")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl)
    img, info = plan.solve(V, wl.lam, 100, L=0.0, power_iters=30, seed=0)
    assert abs(info["L"] - L) <= 1e-5 * L
    _, loose = plan.solve(V, wl.lam, 2000, L=L, eps=1e-3, check_every=5)
    _, tight = plan.solve(V, wl.lam, 2000, L=L, eps=1e-7, check_every=5)
    say(f"    loose {loose['iters']} tight {tight['iters']}")
    assert loose["converged"] == 1 and loose["iters"] <= tight["iters"]


def test_solve_diverges_with_tiny_L():
    """A step constant far below lambda_max makes the iteration blow up: the
    solve reports SL1M_EDIVERGED (condition forced from the host)."""
    say("[case] divergence")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl)
    with pytest.raises(sl1m.SL1MError) as e:
        plan.solve(V, wl.lam, 80, L=0.01 * L)
    assert e.value.status == sl1m.EDIVERGED


def test_kernel_timing_counts_launches():
    say("[case] timing")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl)
    plan.timing_begin(64)
    plan.solve(V, wl.lam, 5, L=L)
    t = plan.timing_end()
    assert t["forward"][0] == 6 and t["adjoint"][0] == 5 and t["fista"][0] == 5
    assert t["forward"][1] > 0


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp32_hilo"])
def test_config3_multi_rhs_stokes(prec):
    """Config 3: Stokes I, Q, U, V of config 1's sky through one operator pass;
    error reported per product (forward and adjoint, per right-hand side)."""
    wl = W.config3()
    say(f"[case] config3 multi-RHS {prec}")
    plan = sl1m.Plan.from_workload(wl, precision=prec, max_rhs=4)
    p = O.Problem.from_workload(wl)
    Vg = plan.forward_multi(wl.x_true).cpu().numpy()
    Vo = O.forward(p, wl.x_true)
    rng = np.random.default_rng(3)
    rr = rng.standard_normal((4, wl.n_vis)) + 1j * rng.standard_normal((4, wl.n_vis))
    gg = plan.adjoint_multi(rr).cpu().numpy()
    go = O.adjoint(p, rr)
    for r, name in enumerate("IQUV"):
        ef, ea = rel(Vg[r], Vo[r]), rel(gg[r], go[r])
        say(f"    Stokes {name}: forward {ef:.3e} adjoint {ea:.3e}")
        assert ef <= TOL[prec] and ea <= TOL[prec]
    # the multi-RHS path gives the same numbers as single-RHS calls
    V1 = plan.forward(wl.x_true[1]).cpu().numpy()
    assert rel(V1, Vg[1]) <= (1e-6 if prec == "fp32" else 1e-13)


@pytest.mark.parametrize("nr", [2, 8])
def test_multi_rhs_mixed_layers_with_gains(nr):
    say(f"[case] multi-RHS nr={nr} mixed layers, per-pair beams")
    rng = np.random.default_rng(12)
    wl = W.small_random(14, 2100, 1300, half_extent=0.3, with_gains=True, distinct_fwhm=(nr == 8))
    kinds = rng.integers(0, 3, wl.n_pix).astype(np.uint8)
    sig = rng.choice([2e-3, 4e-3], wl.n_pix)
    sig[kinds == 0] = 0.0
    wl.kind, wl.sigma = kinds, sig
    plan = sl1m.Plan.from_workload(wl, max_rhs=8)
    p = O.Problem.from_workload(wl)
    X = rng.standard_normal((nr, wl.n_pix))
    rr = rng.standard_normal((nr, wl.n_vis)) + 1j * rng.standard_normal((nr, wl.n_vis))
    ef = rel(plan.forward_multi(X).cpu().numpy(), O.forward(p, X))
    ea = rel(plan.adjoint_multi(rr).cpu().numpy(), O.adjoint(p, rr))
    say(f"    forward {ef:.3e} adjoint {ea:.3e}")
    assert ef <= 1e-5 and ea <= 1e-5
    with pytest.raises(sl1m.SL1MError):
        small = sl1m.Plan.from_workload(wl, max_rhs=2)
        small.forward_multi(np.zeros((4, wl.n_pix)))


def test_config4_full_size_sampled():
    """Config 4 at full size (1,392,640 delta + Gaussian pixels in 4 segments,
    409,600 visibilities, separable per-antenna gains): sampled visibilities
    and pixels of both kinds against the oracle, plus the adjoint identity."""
    wl = W.config4()
    say(f"[case] config4 full n_pix={wl.n_pix} n_vis={wl.n_vis}")
    plan = sl1m.Plan.from_workload(wl)
    p = O.Problem.from_workload(wl)
    x, r = _rand(17, wl.n_pix, wl.n_vis)
    Vg = plan.forward(x).cpu().numpy()
    gg = plan.adjoint(r).cpu().numpy()
    ks = np.arange(0, wl.n_vis, 800)
    nd = 1024 * 1024
    js = np.concatenate([np.arange(0, nd, 8191)[:64], nd + np.arange(0, wl.n_pix - nd, 2687)[:64]])
    Vo, go = O.forward_rows(p, x, ks), O.adjoint_cols(p, r, js)
    ef = rel(Vg[ks], Vo)
    ea = rel(gg[js], go)
    wf = E.worst_ratio(Vg[ks], Vo, E.abs_forward_rows(p, x, ks), wl.n_pix)
    wa = E.worst_ratio(gg[js], go, E.abs_adjoint_cols(p, r, js), wl.n_vis)
    lhs = np.vdot(Vg.astype(np.complex128), r).real
    rhs = float(np.dot(x, gg.astype(np.float64)))
    ident = abs(lhs - rhs) / (np.linalg.norm(Vg) * np.linalg.norm(r))
    say(f"    sampled forward {ef:.3e} adjoint {ea:.3e} identity {ident:.3e}; "
        f"element-wise forward {wf:.3e} adjoint {wa:.3e}")
    assert ef <= 1e-5 and ea <= 1e-5 and ident <= 1e-5
    assert wf <= 1.0 and wa <= 1.0


def test_graph_replayed_iteration_equals_direct_launches():
    """The solve replays a captured graph of one iteration; with kernel timing
    on it launches the kernels directly. Both give the same image bitwise,
    also across repeated replays with host work in between."""
    say("[case] graph vs direct")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl)
    a, ia = plan.solve(V, wl.lam, 60, L=L)
    a = a.cpu().numpy().copy()
    b, ib = plan.solve(V, wl.lam, 60, L=L)
    assert np.array_equal(b.cpu().numpy(), a)
    plan.timing_begin(256)
    c, ic = plan.solve(V, wl.lam, 60, L=L)
    plan.timing_end()
    assert np.array_equal(c.cpu().numpy(), a)
    assert ia["F"] == ib["F"] == ic["F"]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_dirty_image_and_warm_start_match_oracle(prec):
    """Warm starts (Section "Acceleration strategies"): the dirty image
    max(0, Re(M^H V) / N_v) against the oracle's, then 30 FISTA iterations
    from it and from a positive random image against the oracle's warm-started
    iteration (same L).  Config 1 runs on the grid evaluation in FP32."""
    say(f"[case] dirty image and warm start {prec}")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl, precision=prec)
    Dg = plan.dirty_image(V).cpu().numpy()
    Do = O.dirty_image(op, V)
    ed = rel(Dg, Do)
    say(f"    dirty image rel err {ed:.3e}")
    assert ed <= TOL[prec] and np.all(Dg >= 0)
    starts = {"dirty": Do, "random": np.abs(np.random.default_rng(8).standard_normal(wl.n_pix)) * 0.1}
    for name, I0 in starts.items():
        ref = O.fista_from(op, V, L, wl.lam, 30, I0)
        img, info = plan.solve(V, wl.lam, 30, L=L, x0=I0)
        err = np.max(np.abs(img.cpu().numpy() - ref.image)) / np.max(ref.image)
        say(f"    from {name}: image err/peak {err:.3e}  F gpu {info['F']:.8g} oracle {ref.F:.8g}")
        assert err <= (1e-4 if prec == "fp32" else 1e-10)
        assert abs(info["F"] - ref.F) <= (1e-4 if prec == "fp32" else 1e-10) * ref.F
    # x0 is required for a warm start (NULL through the C call)
    import ctypes
    with pytest.raises(sl1m.SL1MError):
        info = sl1m.SolveInfo()
        prm = sl1m.SolveParams(lam=wl.lam, eps=0.0, max_iter=2, check_every=1, L=L,
                               L_safety=1.01, power_iters=30, method=0,
                               seed=ctypes.c_uint64(0))
        out = torch.empty(wl.n_pix, dtype=plan.rdtype, device=plan.device)
        Vt = torch.as_tensor(V, dtype=plan.cdtype, device=plan.device)
        sl1m._check(sl1m.lib().sl1m_solve_from(plan._h, Vt.data_ptr(), None, ctypes.byref(prm),
                                               out.data_ptr(), ctypes.byref(info), None))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mfista_matches_oracle_and_is_monotone(prec):
    """MFISTA (the monotone variant): 60 iterations against the oracle's, cold
    and from the dirty image; the objective after 5, 10, 20 and 40 iterations
    never increases."""
    say(f"[case] mfista {prec}")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl, precision=prec)
    tol = 1e-4 if prec == "fp32" else 1e-10
    for name, I0 in (("cold", None), ("dirty", O.dirty_image(op, V))):
        ref = O.mfista(op, V, L, wl.lam, 60, I0=I0)
        img, info = plan.solve(V, wl.lam, 60, L=L, x0=I0, method="mfista")
        err = np.max(np.abs(img.cpu().numpy() - ref.image)) / np.max(ref.image)
        say(f"    {name}: image err/peak {err:.3e}  F gpu {info['F']:.8g} oracle {ref.F:.8g}")
        assert err <= tol and abs(info["F"] - ref.F) <= tol * ref.F
    Fs = [plan.solve(V, wl.lam, k, L=L, method="mfista")[1]["F"] for k in (5, 10, 20, 40)]
    say(f"    F after 5/10/20/40: {Fs}")
    assert all(b <= a * (1 + 1e-6) for a, b in zip(Fs, Fs[1:]))


def test_config2_solve_against_oracle_checked_fp64_plan():
    """Config 2's L1 solve at full size (65,536 pixels x 97,536 visibilities,
    100 iterations with a fixed L): the FP32 grid-evaluated solve against the
    same solve on an FP64 plan, within 1e-4 of the peak.  The FP64 plan's
    operators are first checked against the oracle on sampled outputs
    (1e-11 norm-relative and the FP64 element-wise bound), so the chain
    GPU FP32 -> GPU FP64 -> oracle pins the full-size solve."""
    wl = W.config2()
    say(f"[case] config2 solve FP32 grid vs FP64 plan n_pix={wl.n_pix} n_vis={wl.n_vis}")
    p64 = sl1m.Plan.from_workload(wl, precision="fp64")
    p = O.Problem.from_workload(wl)
    x, r = _rand(21, wl.n_pix, wl.n_vis)
    ks = np.arange(0, wl.n_vis, 487)
    js = np.arange(0, wl.n_pix, 331)
    Vs = p64.forward(x).cpu().numpy()[ks]
    gs = p64.adjoint(r).cpu().numpy()[js]
    Vo, go = O.forward_rows(p, x, ks), O.adjoint_cols(p, r, js)
    ef, ea = rel(Vs, Vo), rel(gs, go)
    wf = E.worst_ratio(Vs, Vo, E.abs_forward_rows(p, x, ks), wl.n_pix, "fp64")
    wa = E.worst_ratio(gs, go, E.abs_adjoint_cols(p, r, js), wl.n_vis, "fp64")
    say(f"    FP64 plan vs oracle sampled forward {ef:.3e} adjoint {ea:.3e} "
        f"element-wise {wf:.3e} {wa:.3e}")
    assert ef <= 1e-11 and ea <= 1e-11 and wf <= 1.0 and wa <= 1.0
    V = p64.forward(wl.x_true) + torch.as_tensor(wl.noise, dtype=torch.complex128,
                                                 device=p64.device)
    L = 1.01 * p64.estimate_L(wl.power_iters, seed=0)
    img64, info64 = p64.solve(V, wl.lam, wl.n_iter, L=L)
    img64 = img64.cpu().numpy()
    p64.close()
    p32 = sl1m.Plan.from_workload(wl)
    assert p32.info()["grid"] >= 1
    img32, info32 = p32.solve(V.to(torch.complex64), wl.lam, wl.n_iter, L=L)
    img32 = img32.cpu().numpy()
    peak = float(np.max(img64))
    err = float(np.max(np.abs(img32 - img64))) / peak
    say(f"    image err/peak {err:.3e}  F fp32 {info32['F']:.9g} fp64 {info64['F']:.9g}  "
        f"nnz {info32['nnz']} {info64['nnz']}")
    assert err <= 1e-4
    assert abs(info32["F"] - info64["F"]) <= 1e-4 * info64["F"]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_solve_resume_exact_and_state_matches_oracle(prec):
    """Checkpoint and resume (sl1m_solve_resume): 25 + 35 iterations equal a
    60-iteration solve bit for bit, and the exported state after 25
    iterations (I_25, y_26, t_26) matches the oracle's state."""
    say(f"[case] solve resume {prec}")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl, precision=prec)
    img, info = plan.solve(V, wl.lam, 60, L=L)
    img = img.cpu().numpy()
    _, i1, st = plan.solve_resume(V, wl.lam, 25, L)
    ref = O.fista(op, V, L, wl.lam, 25)
    k, t, I_k, y = ref.state
    peak = float(np.max(I_k))
    tol = 1e-4 if prec == "fp32" else 1e-10
    e_img = float(np.max(np.abs(st["img"].cpu().numpy() - I_k))) / peak
    e_y = float(np.max(np.abs(st["y"].cpu().numpy() - y))) / peak
    say(f"    state after 25: k {st['k']} vs {k}, t {st['t']!r} vs {t!r}, "
        f"image err/peak {e_img:.2e}, y err/peak {e_y:.2e}")
    assert st["k"] == k == 25 and abs(st["t"] - t) <= 1e-15 * t
    assert e_img <= tol and e_y <= tol
    img2, i2, st2 = plan.solve_resume(V, wl.lam, 35, L, state=st)
    assert st2["k"] == 60 and i2["iters"] == 35
    assert np.array_equal(img2.cpu().numpy(), img)
    assert i2["F"] == info["F"] and i2["nnz"] == info["nnz"]


def test_solve_stops_on_nonzero_count():
    """The non-zero-count stopping rule: the FP64 plan stops at the same
    check as the oracle, with the same image to 1e-10 of the peak; with both
    rules off the solve runs to the cap."""
    say("[case] solve nnz stop")
    wl, op, V, L = _config1_data()
    plan = sl1m.Plan.from_workload(wl, precision="fp64")
    for nnz_eps in (1e-9, 0.02):
        ref = O.fista(op, V, L, wl.lam, 500, check_every=5, nnz_eps=nnz_eps)
        img, info = plan.solve(V, wl.lam, 500, L=L, check_every=5, nnz_eps=nnz_eps)
        err = float(np.max(np.abs(img.cpu().numpy() - ref.image))) / float(np.max(ref.image))
        say(f"    nnz_eps {nnz_eps}: gpu {info['iters']} iterations ({info['converged']}), "
            f"oracle {ref.iters} ({ref.converged}); err/peak {err:.2e}")
        assert ref.converged == 2 and info["converged"] == 2
        assert info["iters"] == ref.iters and err <= 1e-10
    _, off = plan.solve(V, wl.lam, 40, L=L, check_every=5)
    assert off["iters"] == 40 and off["converged"] == 0


def test_config4_solve_against_oracle_checked_fp64_plan():
    """Config 4 at full size (1,392,640 pixels x 409,600 visibilities, gains
    and beams) in the benchmark's launch configuration: 5 FISTA iterations
    of the FP32 grid-evaluated plan against the same iterations on an FP64
    plan (direct evaluation), within 1e-4 of the peak, with the FP64 plan's
    forward and adjoint first checked against the oracle on sampled outputs
    (1e-11 norm-relative and the FP64 element-wise bound)."""
    wl = W.config4()
    say(f"[case] config4 solve FP32 grid vs FP64 plan n_pix={wl.n_pix} n_vis={wl.n_vis}")
    p64 = sl1m.Plan.from_workload(wl, precision="fp64")
    p = O.Problem.from_workload(wl)
    x, r = _rand(23, wl.n_pix, wl.n_vis)
    ks = np.arange(0, wl.n_vis, 8191)
    js = np.concatenate([np.arange(0, 1024 * 1024, 20011), np.arange(1024 * 1024, wl.n_pix, 4001)])
    Vs = p64.forward(x).cpu().numpy()[ks]
    gs = p64.adjoint(r).cpu().numpy()[js]
    Vo, go = O.forward_rows(p, x, ks), O.adjoint_cols(p, r, js)
    ef, ea = rel(Vs, Vo), rel(gs, go)
    wf = E.worst_ratio(Vs, Vo, E.abs_forward_rows(p, x, ks), wl.n_pix, "fp64")
    wa = E.worst_ratio(gs, go, E.abs_adjoint_cols(p, r, js), wl.n_vis, "fp64")
    say(f"    FP64 plan vs oracle sampled forward {ef:.3e} adjoint {ea:.3e} "
        f"element-wise {wf:.3e} {wa:.3e}")
    assert ef <= 1e-11 and ea <= 1e-11 and wf <= 1.0 and wa <= 1.0
    V = p64.forward(wl.x_true) + torch.as_tensor(wl.noise, dtype=torch.complex128,
                                                 device=p64.device)
    L = 1.01 * p64.estimate_L(5, seed=0)
    img64, info64 = p64.solve(V, wl.lam, 5, L=L)
    img64 = img64.cpu().numpy()
    p64.close()
    p32 = sl1m.Plan.from_workload(wl)
    assert p32.info()["grid"] == 4
    img32, info32 = p32.solve(V.to(torch.complex64), wl.lam, 5, L=L)
    img32 = img32.cpu().numpy()
    peak = float(np.max(img64))
    err = float(np.max(np.abs(img32 - img64))) / peak
    say(f"    image err/peak {err:.3e}  F fp32 {info32['F']:.9g} fp64 {info64['F']:.9g}  "
        f"nnz {info32['nnz']} {info64['nnz']}")
    assert err <= 1e-4
    assert abs(info32["F"] - info64["F"]) <= 1e-4 * info64["F"]
