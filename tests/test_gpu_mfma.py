"""Matrix-core precisions (SL1M_PREC_MFMA_F16 / _BF16) through the C ABI.

The forward and adjoint of these plans contract the FP32 matrix entries and
the images / residual records rounded to float16 or bfloat16 on the MFMA
units, accumulating in float32.  Two checks against the FP64 oracle:

* the error bound of that arithmetic, element by element:
      forward  |V_gpu - V|_k <= c sum_j |M_kj| |x_j|
      adjoint  |g_gpu - g|_j <= c sum_k |M_kj| (|Re r_k| + |Im r_k|)
  plus N 2^-37 max|operand| max|M| (float16 operands left subnormal by the
  power-of-two scaling), with c = 2u + u^2 + N 2^-24 + 2^-17: u the operand
  type's unit roundoff (2^-11 float16, 2^-8 bfloat16; an entry and the value
  it multiplies are each rounded once, so a product is off by at most
  2u + u^2 of |M_kj x_j| -- for the complex entry, |dM| <= u |M| when its
  real and imaginary parts are rounded separately), N the number of float32
  accumulations, 2^-17 the float32 entry itself (phase reduction, v_sin and
  v_cos);
* for results of at least 256 elements, the norm-relative error at most 4u:
  independent roundings of the terms add up like a random walk, so the error
  relative to the result stays near u (the element bound above allows for
  full cancellation and is loose; a handful of elements can cancel by
  chance, so short results get the bound alone).
The norm-relative errors are printed for the precision table.

Plans whose pixels form one square delta grid run the forward on the grid
evaluation (`grid_mfma`): a mirrored pair of cells is sixteen basis values
(products of the A, B and C phasors) against eight sign combinations of the
pair's amplitudes.  Since the two basis values that share a combination have
magnitudes summing to at most |C| <= 1 per component, a pair's error is at
most 2 e sum_j |M_kj| |x_j| (the factor 2 from the real and imaginary parts
together), e the relative error of one basis value times one combination:
* bfloat16: the basis is formed in float32 and rounded once, and the
  combination once: e = 2u + u^2; a basis value left subnormal adds at most
  2^-25 per product: n 2^-23 max|x| max|M|;
* float16: the basis is formed in packed float16 arithmetic (the two phasor
  components, their product, C and the product with C each rounded), so
  e = (1 + u)^6 - 1; each of the five roundings of a value below float16's
  normal range adds at most 2^-25 absolute, so a basis value is off by at
  most 5 2^-25 beyond e, i.e. 320 2^-25 max|x| per pair over its 16 values
  and combinations of four amplitudes; with at most n/8 + n/16 pairs this is
  below n 2^-19 max|x| max|M|.
The adjoint of float16 plans on such a grid (4 and 8 sides) contracts the
same basis, as (p_a cc, -p_a cs) or (p_a cs, p_a cc) per visibility, with
the scaled residual records (conj(G) r): a pixel's value adds four sums
whose products p_a have magnitudes summing to at most 2, and |Re r'| +
|Im r'| <= sqrt 2 |G| (|Re r| + |Im r|), so its error is at most
2 sqrt 2 ((1 + u)^6 - 1) sum_k |M_kj| (|Re r_k| + |Im r_k|) plus the
float32 terms above, and the subnormal basis values add at most
4 x 5 2^-25 sqrt 2 per visibility: below n 2^-21 max(|Re r| + |Im r|) max|M|
with n = 2 N_v.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1310_2078_amd import sl1m
from paper_1310_2078_amd import workloads as W

pytestmark = pytest.mark.gpu

UNIT = {"mfma_f16": 2.0 ** -11, "mfma_bf16": 2.0 ** -8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _coef(prec, n):
    u = UNIT[prec]
    return 2 * u + u * u + n * 2.0 ** -24 + 2.0 ** -17


def _check_forward(prec, p, Vg, X, ks=None, grid=False):
    """Vg[r][i] against the oracle at visibilities ks (all when None); grid:
    the plan's forward runs on the grid evaluation."""
    ks = np.arange(p.u.shape[0]) if ks is None else np.asarray(ks)
    M = O.matrix_block(p, ks, np.arange(p.l.shape[0]))
    absM = np.abs(M)
    n = X.shape[1]
    worst = 0.0
    u = UNIT[prec]
    for r in range(X.shape[0]):
        Vo = M @ X[r]
        ax = np.abs(X[r])
        if grid and prec == "mfma_f16":
            c = 2 * ((1 + u) ** 6 - 1) + n * 2.0 ** -24 + 2.0 ** -17
            b = c * (absM @ ax) + n * 2.0 ** -19 * ax.max() * absM.max()
        elif grid:
            c = 2 * (2 * u + u * u) + n * 2.0 ** -24 + 2.0 ** -17
            b = c * (absM @ ax) + n * 2.0 ** -23 * ax.max() * absM.max()
        else:
            b = _coef(prec, n) * (absM @ ax) + n * 2.0 ** -37 * ax.max() * absM.max()
        err = np.abs(Vg[r] - Vo)
        worst = max(worst, float((err / b).max()))
        assert np.all(err <= b), f"side {r}: error above the bound at {np.argmax(err / b)}"
        if Vo.size >= 256:
            assert rel(Vg[r], Vo) <= 4 * UNIT[prec], f"side {r}: norm-relative {rel(Vg[r], Vo):.3e}"
    return worst


def _check_adjoint(prec, p, gg, Rr, js=None, grid=False):
    """gg[r][i] against the oracle at pixels js (all when None); grid: the
    plan's pixels form one square delta grid."""
    js = np.arange(p.l.shape[0]) if js is None else np.asarray(js)
    M = O.matrix_block(p, np.arange(p.u.shape[0]), js)
    absMT = np.abs(M).T
    n = 2 * Rr.shape[1]  # the real and the imaginary product of each visibility
    u = UNIT[prec]
    worst = 0.0
    for r in range(Rr.shape[0]):
        go = np.real(M.conj().T @ Rr[r])
        ar = np.abs(Rr[r].real) + np.abs(Rr[r].imag)
        if grid and prec == "mfma_f16":
            c = 2 * np.sqrt(2.0) * ((1 + u) ** 6 - 1) + n * 2.0 ** -24 + 2.0 ** -17
            b = c * (absMT @ ar) + n * 2.0 ** -21 * ar.max() * absMT.max()
        else:
            b = _coef(prec, n) * (absMT @ ar) + n * 2.0 ** -37 * ar.max() * absMT.max()
        err = np.abs(gg[r] - go)
        worst = max(worst, float((err / b).max()))
        assert np.all(err <= b), f"side {r}: error above the bound at {np.argmax(err / b)}"
        if go.size >= 256:
            assert rel(gg[r], go) <= 4 * UNIT[prec], f"side {r}: norm-relative {rel(gg[r], go):.3e}"
    return worst


@pytest.mark.parametrize("prec", ["mfma_f16", "mfma_bf16"])
def test_config3_stokes_mfma(prec):
    """Config 3 (Stokes I, Q, U, V of config 1's sky, R = 4) on the matrix
    cores: every side within the bound, norm-relative errors printed."""
    wl = W.config3()
    say(f"[case] config3 {prec}")
    plan = sl1m.Plan.from_workload(wl, precision=prec, max_rhs=4)
    p = O.Problem.from_workload(wl)
    X = np.asarray(wl.x_true)
    Vg = plan.forward_multi(X).cpu().numpy()
    rng = np.random.default_rng(3)
    Rr = rng.standard_normal((4, wl.n_vis)) + 1j * rng.standard_normal((4, wl.n_vis))
    gg = plan.adjoint_multi(Rr).cpu().numpy()
    Vo, go = O.forward(p, X), O.adjoint(p, Rr)
    for r, name in enumerate("IQUV"):
        say(f"    Stokes {name}: forward {rel(Vg[r], Vo[r]):.3e} adjoint {rel(gg[r], go[r]):.3e}")
    grid = plan.info()["grid_mfma"] == 1
    assert grid  # config 3's 32 x 32 image is a square delta grid
    wf = _check_forward(prec, p, Vg, X, grid=grid)
    wa = _check_adjoint(prec, p, gg, Rr, grid=grid)
    say(f"    largest error / bound: forward {wf:.3f} adjoint {wa:.3f}")
    # a side alone equals that side of the multi-RHS call (same operand scale
    # only when it holds the largest magnitude: compare within the bound)
    V1 = plan.forward(X[0]).cpu().numpy()
    _check_forward(prec, p, V1[None], X[:1], grid=grid)


@pytest.mark.parametrize("prec", ["mfma_f16", "mfma_bf16"])
@pytest.mark.parametrize("nr", [1, 2, 4, 8])
def test_mfma_ragged_gains(prec, nr):
    """Irregular pixels, ragged sizes (1000 pixels, 1999 visibilities: neither
    a multiple of 32), antenna gains with one beam width, 1 to 8 sides."""
    say(f"[case] mfma ragged {prec} nr={nr}")
    wl = W.small_random(21, 1000, 1999, half_extent=0.25, with_gains=True)
    plan = sl1m.Plan.from_workload(wl, precision=prec, max_rhs=8)
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(22 + nr)
    X = rng.standard_normal((nr, wl.n_pix))
    Rr = rng.standard_normal((nr, wl.n_vis)) + 1j * rng.standard_normal((nr, wl.n_vis))
    if nr == 1:
        Vg = plan.forward(X[0]).cpu().numpy()[None]
        gg = plan.adjoint(Rr[0]).cpu().numpy()[None]
    else:
        Vg = plan.forward_multi(X).cpu().numpy()
        gg = plan.adjoint_multi(Rr).cpu().numpy()
    say(f"    forward {rel(Vg, O.forward(p, X)):.3e} adjoint {rel(gg, O.adjoint(p, Rr)):.3e}")
    wf = _check_forward(prec, p, Vg, X)
    wa = _check_adjoint(prec, p, gg, Rr)
    say(f"    largest error / bound: forward {wf:.3f} adjoint {wa:.3f}")


@pytest.mark.parametrize("prec", ["mfma_f16", "mfma_bf16"])
@pytest.mark.parametrize("lanes", [(2, 2), (4, 4), (1, 4)])
def test_mfma_lanes_per_thread(prec, lanes):
    """Two and four visibilities (forward) / pixels (adjoint) per lane, with
    ragged sizes and 8 sides (two groups of four)."""
    vpl, ppl = lanes
    say(f"[case] mfma {prec} fwd_vpl={vpl} adj_ppl={ppl}")
    wl = W.small_random(23, 2900, 3001, half_extent=0.25, with_gains=True)
    plan = sl1m.Plan.from_workload(wl, precision=prec, max_rhs=8, fwd_vpl=vpl, adj_ppl=ppl)
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(24)
    X = rng.standard_normal((8, wl.n_pix))
    Rr = rng.standard_normal((8, wl.n_vis)) + 1j * rng.standard_normal((8, wl.n_vis))
    wf = _check_forward(prec, p, plan.forward_multi(X).cpu().numpy(), X)
    wa = _check_adjoint(prec, p, plan.adjoint_multi(Rr).cpu().numpy(), Rr)
    say(f"    largest error / bound: forward {wf:.3f} adjoint {wa:.3f}")


@pytest.mark.parametrize("prec", ["mfma_f16", "mfma_bf16"])
def test_grid_mfma_side_counts(prec):
    """A square delta grid (48 x 48 pixels: 1,152 mirrored pairs over several
    pair chunks) with 3,001 visibilities (a ragged last tile) and antenna
    gains, one plan called with 1, 2, 4 and 8 sides: the grid forward on the
    matrix cores (float16 from 4 sides, bfloat16 at 8), the FP32 grid
    evaluation below that, and each adjoint path, all within their bounds."""
    say(f"[case] grid mfma {prec} 48x48 x 3001, sides 1/2/4/8")
    rng = np.random.default_rng(41)
    l, m, _ = W.grid_pixels(48, 0.1)
    u, v, w = W.disk_uvw(rng, 3001, 400.0, 60.0)
    n = l.shape[0]
    wl = W.Workload("grid48", l, m, np.zeros(n), np.zeros(n, np.uint8), u, v, w)
    wl.ant_p = rng.integers(0, 12, 3001).astype(np.int32)
    wl.ant_q = ((wl.ant_p + rng.integers(1, 12, 3001)) % 12).astype(np.int32)
    wl.ant_gain = (1.0 + 0.05 * rng.standard_normal(12)) * np.exp(1j * 0.05 * rng.standard_normal(12))
    wl.ant_fwhm = np.full(12, 0.5)
    plan = sl1m.Plan.from_workload(wl, precision=prec, max_rhs=8)
    assert plan.info()["grid_mfma"] == 1
    p = O.Problem.from_workload(wl)
    for nr in (1, 2, 4, 8):
        X = rng.standard_normal((nr, n))
        Rr = rng.standard_normal((nr, 3001)) + 1j * rng.standard_normal((nr, 3001))
        if nr == 1:
            Vg = plan.forward(X[0]).cpu().numpy()[None]
            gg = plan.adjoint(Rr[0]).cpu().numpy()[None]
        else:
            Vg = plan.forward_multi(X).cpu().numpy()
            gg = plan.adjoint_multi(Rr).cpu().numpy()
        wf = _check_forward(prec, p, Vg, X, grid=True)
        wa = _check_adjoint(prec, p, gg, Rr, grid=True)
        say(f"    sides {nr}: largest error / bound forward {wf:.3f} adjoint {wa:.3f}")
    plan.close()


@pytest.mark.parametrize("shape", [(5, 3), (33, 31), (1, 64)])
def test_mfma_tiny_shapes(shape):
    """Fewer pixels / visibilities than one 32-step, one lane, one block."""
    n_pix, n_vis = shape
    say(f"[case] mfma tiny n_pix={n_pix} n_vis={n_vis}")
    wl = W.small_random(30 + n_pix, n_pix, n_vis)
    plan = sl1m.Plan.from_workload(wl, precision="mfma_f16", max_rhs=4)
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(31)
    X = rng.standard_normal((4, n_pix))
    Rr = rng.standard_normal((4, n_vis)) + 1j * rng.standard_normal((4, n_vis))
    _check_forward("mfma_f16", p, plan.forward_multi(X).cpu().numpy(), X)
    _check_adjoint("mfma_f16", p, plan.adjoint_multi(Rr).cpu().numpy(), Rr)


def test_mfma_full_size_sampled():
    """Config 2's shape (65,536 pixels x 97,536 visibilities), four sides, as
    the bench times it: 64 visibilities of the forward and 64 pixels of the
    adjoint (the last of each included) against the oracle's rows and
    columns, within the bound; the norm-relative error over the 256 sampled
    values of each operator at most 4u."""
    wl = W.config2()
    say("[case] mfma f16 config2 shape sampled")
    plan = sl1m.Plan.from_workload(wl, precision="mfma_f16", max_rhs=4)
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, wl.n_pix))
    Rr = rng.standard_normal((4, wl.n_vis)) + 1j * rng.standard_normal((4, wl.n_vis))
    Vg = plan.forward_multi(X).cpu().numpy()
    gg = plan.adjoint_multi(Rr).cpu().numpy()
    ks = np.sort(rng.choice(wl.n_vis - 1, 63, replace=False))
    ks = np.append(ks, wl.n_vis - 1)
    js = np.sort(rng.choice(wl.n_pix - 1, 63, replace=False))
    js = np.append(js, wl.n_pix - 1)
    assert plan.info()["grid_mfma"] == 1
    wf = _check_forward("mfma_f16", p, Vg[:, ks], X, ks, grid=True)
    wa = _check_adjoint("mfma_f16", p, gg[:, js], Rr, js, grid=True)
    Vo = O.matrix_block(p, ks, np.arange(wl.n_pix)) @ X.T
    go = np.real(O.matrix_block(p, np.arange(wl.n_vis), js).conj().T @ Rr.T)
    ef, ea = rel(Vg[:, ks].T, Vo), rel(gg[:, js].T, go)
    say(f"    largest error / bound: forward {wf:.3f} adjoint {wa:.3f}; "
        f"norm-relative forward {ef:.3e} adjoint {ea:.3e}")
    assert ef <= 4 * UNIT["mfma_f16"] and ea <= 4 * UNIT["mfma_f16"]


def test_mfma_solve_config1():
    """FISTA on a float16 matrix-core plan (config 1, 100 iterations, the
    oracle's L).  The operator's error, about 3e-4 of |M I| ~ 6 per
    visibility, is a tenth of the noise (0.014 per visibility) that the
    objective's L2 term measures, so the iterate solves a perturbed problem:
    the reported objective and the oracle's objective of the returned image
    are both within 1e-2 of the oracle's iterate (measured 2.5e-3)."""
    wl = W.config1()
    say("[case] mfma f16 config1 solve")
    op = O.Operator(O.Problem.from_workload(wl))
    V = op.forward(wl.x_true) + wl.noise
    L, _ = O.power_iteration(op, 30, seed=0)
    ref = O.fista(op, V, L, wl.lam, wl.n_iter)
    plan = sl1m.Plan.from_workload(wl, precision="mfma_f16")
    img, info = plan.solve(V, wl.lam, wl.n_iter, L=L)
    F_img = O.objective(op, V, img.cpu().numpy().astype(np.float64), wl.lam)[0]
    say(f"    F gpu {info['F']:.8g}, oracle F of the gpu image {F_img:.8g}, oracle {ref.F:.8g}; "
        f"nnz {info['nnz']} {ref.nnz}")
    assert info["iters"] == wl.n_iter and info["status"] == 0
    assert abs(info["F"] - ref.F) <= 1e-2 * ref.F
    assert abs(F_img - ref.F) <= 1e-2 * ref.F


def test_mfma_rejects():
    """Gaussian pixels, per-pair beam widths and tuning are refused."""
    wl = W.small_random(40, 300, 200, kind=W.PIX_GAUSS_WIDE, sigma=2e-3)
    with pytest.raises(sl1m.SL1MError):
        sl1m.Plan.from_workload(wl, precision="mfma_f16")
    wl = W.small_random(41, 300, 200, with_gains=True, distinct_fwhm=True)
    with pytest.raises(sl1m.SL1MError):
        sl1m.Plan.from_workload(wl, precision="mfma_bf16")
    wl = W.small_random(42, 300, 200)
    plan = sl1m.Plan.from_workload(wl, precision="mfma_f16", max_rhs=2)
    with pytest.raises(sl1m.SL1MError):
        plan.forward_multi(np.zeros((4, 300)))


@pytest.mark.parametrize("prec", ["mfma_f16", "mfma_bf16"])
def test_mfma_empty_inputs(prec):
    """No pixels: the forward is all zeros; no visibilities: the adjoint is all
    zeros and the forward empty (no packing or matrix-core launch runs)."""
    say(f"[case] mfma empty inputs {prec}")
    wl = W.small_random(1, 10, 20)
    e1 = W.Workload("np0", wl.l[:0], wl.m[:0], wl.sigma[:0], wl.kind[:0], wl.u, wl.v, wl.w)
    plan = sl1m.Plan.from_workload(e1, precision=prec, max_rhs=4)
    V = plan.forward_multi(np.zeros((4, 0))).cpu().numpy()
    assert V.shape == (4, 20) and np.all(V == 0)
    e2 = W.Workload("nv0", wl.l, wl.m, wl.sigma, wl.kind, wl.u[:0], wl.v[:0], wl.w[:0])
    plan = sl1m.Plan.from_workload(e2, precision=prec, max_rhs=4)
    g = plan.adjoint_multi(np.zeros((4, 0), complex)).cpu().numpy()
    assert g.shape == (4, 10) and np.all(g == 0)
    V = plan.forward(np.ones(10)).cpu().numpy()
    assert V.shape == (0,)
