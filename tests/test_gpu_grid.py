"""Grid evaluation of the delta-pixel operators (through the C ABI).

The grid evaluation computes the same operator as the direct one (the
element of eq. (deltam) factorised into per-|l|, per-|m| and per-radius
phasors).  Each case checks both evaluations against the FP64 oracle at the
FP32 operator tolerance (norm-relative 1e-5, and every output within its
element-wise bound, tests/elementwise.py) and that the plan took the path
the case is about.  Sizes span several tiles, end in ragged tails (|m| groups
of 8 that do not divide the |m| count, visibility counts that are not
multiples of the tile) and cover the degenerate cells (the l = 0 and m = 0
rows, cells with missing sign slots, empty cells).
"""
import sys

import numpy as np
import pytest

import elementwise as E
import oracle as O
from paper_1310_2078_amd import sl1m
from paper_1310_2078_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _with_pixels(wl, l, m, sigma=None, kind=None):
    n = l.shape[0]
    wl.l, wl.m = l, m
    wl.sigma = np.zeros(n) if sigma is None else sigma
    wl.kind = np.zeros(n, np.uint8) if kind is None else kind
    wl.x_true = None
    return wl


def _odd_grid(n_side, half_extent):
    """Centred odd grid: offsets -(n-1)/2 .. (n-1)/2, so every position has
    all four sign mirrors and the l = 0 and m = 0 rows are present."""
    d = 2.0 * half_extent / n_side
    k = np.arange(n_side) - n_side // 2
    L, M = np.meshgrid(k * d, k * d)
    return L.ravel(), M.ravel()


SEEDS = {"config1": 0, "odd45": 1, "disk64": 2, "rect80x24_gains": 3, "grid_plus_gauss": 4,
         "gauss_wide48_gains": 5, "gauss_parax_odd41": 6, "layers_mixed": 7,
         "gauss_truncated50": 8, "gauss_rect72x30": 9}


def _case(name):
    """Gaussian cases take sigma so that pi sigma^2 |(u,v)|^2 is of order 1-10
    over their visibilities (the taper neither flat nor vanishing)."""
    rng = np.random.default_rng(SEEDS[name])
    if name == "config1":
        return W.config1()
    if name == "odd45":
        wl = W.small_random(11, 10, 3001, uv_radius=900.0, w_sigma=250.0)
        return _with_pixels(wl, *_odd_grid(45, 0.25))
    if name == "disk64":
        wl = W.small_random(12, 10, 2777, uv_radius=1200.0, w_sigma=300.0)
        l, m, d = W.grid_pixels(64, 0.3)
        keep = l * l + m * m < (0.27) ** 2
        return _with_pixels(wl, l[keep], m[keep])
    if name == "rect80x24_gains":
        wl = W.small_random(13, 10, 4099, uv_radius=1000.0, w_sigma=200.0, with_gains=True)
        d = 0.004
        kl = np.arange(80) - 40
        km = np.arange(24) - 12
        L, M = np.meshgrid(kl * d, km * d)
        return _with_pixels(wl, L.ravel(), M.ravel())
    if name == "grid_plus_gauss":
        wl = W.small_random(14, 10, 2500, uv_radius=800.0, w_sigma=200.0, with_gains=True)
        l, m, d = W.grid_pixels(48, 0.2)
        ng = 700
        lg = rng.uniform(-0.2, 0.2, ng)
        mg = rng.uniform(-0.2, 0.2, ng)
        kinds = np.concatenate([np.zeros(l.size, np.uint8),
                                rng.choice([W.PIX_GAUSS_PARAXIAL, W.PIX_GAUSS_WIDE], ng)
                                .astype(np.uint8)])
        sig = np.concatenate([np.zeros(l.size), rng.choice([2e-3, 5e-3], ng)])
        perm = rng.permutation(l.size + ng)   # interleave the kinds in caller order
        return _with_pixels(wl, np.concatenate([l, lg])[perm], np.concatenate([m, mg])[perm],
                            sig[perm], kinds[perm])
    if name == "gauss_wide48_gains":
        wl = W.small_random(15, 10, 2600, uv_radius=900.0, w_sigma=250.0, with_gains=True)
        l, m, d = W.grid_pixels(48, 0.2)
        return _with_pixels(wl, l, m, np.full(l.size, 1.5e-3),
                            np.full(l.size, W.PIX_GAUSS_WIDE, np.uint8))
    if name == "gauss_parax_odd41":
        wl = W.small_random(16, 10, 2111, uv_radius=700.0, w_sigma=200.0)
        l, m = _odd_grid(41, 0.15)
        return _with_pixels(wl, l, m, np.full(l.size, 1.2e-3),
                            np.full(l.size, W.PIX_GAUSS_PARAXIAL, np.uint8))
    if name == "layers_mixed":
        # delta 64^2 and wide-field 32^2 grids qualify; the paraxial 16^2 grid
        # is too small and stays direct; caller order interleaves all three
        wl = W.small_random(17, 10, 1800, uv_radius=800.0, w_sigma=200.0, with_gains=True)
        parts = []
        for n_side, kind, sig in ((64, W.PIX_DELTA, 0.0), (32, W.PIX_GAUSS_WIDE, 2e-3),
                                  (16, W.PIX_GAUSS_PARAXIAL, 3e-3)):
            l, m, d = W.grid_pixels(n_side, 0.2)
            sg = np.full(l.size, sig)
            parts.append((l, m, sg, np.full(l.size, kind, np.uint8)))
        l, m, sg, kd = (np.concatenate([q[i] for q in parts]) for i in range(4))
        perm = rng.permutation(l.size)
        return _with_pixels(wl, l[perm], m[perm], sg[perm], kd[perm])
    if name == "gauss_truncated50":
        # a serving-stream-like request: row-major grid truncated mid-row
        wl = W.small_random(18, 10, 2900, uv_radius=500.0, w_sigma=50.0)
        l, m, d = W.grid_pixels(50, 0.05)
        n = 2321
        return _with_pixels(wl, l[:n], m[:n], np.full(n, 2.0 * d),
                            np.full(n, W.PIX_GAUSS_WIDE, np.uint8))
    if name == "gauss_rect72x30":
        # rectangular: the |l| and |m| sets differ, so cells are not paired
        wl = W.small_random(19, 10, 2333, uv_radius=800.0, w_sigma=150.0, with_gains=True)
        d = 0.005
        L, M = np.meshgrid((np.arange(72) - 36) * d, (np.arange(30) - 15) * d)
        n = L.size
        return _with_pixels(wl, L.ravel(), M.ravel(), np.full(n, 1.5e-3),
                            np.full(n, W.PIX_GAUSS_WIDE, np.uint8))
    raise KeyError(name)


# case -> number of segments on the grid path
CASES = {"config1": 1, "odd45": 1, "disk64": 1, "rect80x24_gains": 1, "grid_plus_gauss": 1,
         "gauss_wide48_gains": 1, "gauss_parax_odd41": 1, "layers_mixed": 2,
         "gauss_truncated50": 1, "gauss_rect72x30": 1}
# cases whose grid segments are all square (evaluated as mirrored pairs)
SQUARE = {"config1", "odd45", "disk64", "grid_plus_gauss", "gauss_wide48_gains",
          "gauss_parax_odd41", "layers_mixed", "gauss_truncated50"}


@pytest.mark.parametrize("name", list(CASES))
def test_grid_and_direct_match_oracle(name):
    wl = _case(name)
    say(f"[case] grid {name} n_pix={wl.n_pix} n_vis={wl.n_vis}")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    p = O.Problem.from_workload(wl)
    Vo = O.forward(p, x)
    go = O.adjoint(p, r)
    mf, ma = E.abs_forward_rows(p, x), E.abs_adjoint_cols(p, r)
    out = {}
    for mode in ("require", "off"):
        plan = sl1m.Plan.from_workload(wl, grid=mode)
        info = plan.info()
        assert info["grid"] == (CASES[name] if mode == "require" else 0)
        if mode == "require":
            assert info["grid_pairs"] == (info["grid"] if name in SQUARE else 0)
        V = plan.forward(x).cpu().numpy()
        g = plan.adjoint(r).cpu().numpy()
        ef, ea = rel(V, Vo), rel(g, go)
        wf = E.worst_ratio(V, Vo, mf, wl.n_pix)
        wa = E.worst_ratio(g, go, ma, wl.n_vis)
        say(f"    {mode:8s} forward {ef:.3e} adjoint {ea:.3e} element-wise {wf:.3e} {wa:.3e} "
            f"info {info}")
        assert ef <= TOL and ea <= TOL
        assert wf <= 1.0 and wa <= 1.0
        out[mode] = (V, g)
        plan.close()
    say(f"    grid vs direct forward {rel(out['require'][0], out['off'][0]):.3e} "
        f"adjoint {rel(out['require'][1], out['off'][1]):.3e}")


def test_grid_solve_matches_direct_solve():
    """FISTA on config 1 with a given L: the grid and direct evaluations give
    images within the image tolerance of each other and of the oracle."""
    wl = W.config1()
    say(f"[case] grid solve config1")
    p = O.Problem.from_workload(wl)
    V = O.forward(p, wl.x_true) + wl.noise
    L = O.power_iteration(O.Operator(p), iters=50, seed=0)[0]
    ref = O.fista(O.Operator(p), V, L, wl.lam, 50).image
    peak = float(np.max(np.abs(ref)))
    for mode in ("require", "off"):
        plan = sl1m.Plan.from_workload(wl, grid=mode)
        img, info = plan.solve(V, wl.lam, 50, L=L)
        err = float(np.max(np.abs(img.cpu().numpy() - ref))) / peak
        say(f"    {mode:8s} image err/peak {err:.3e} iters {info['iters']}")
        assert err <= 1e-4
        plan.close()


def test_grid_rejections_and_fallbacks():
    say("[case] grid rejections")
    wl = W.small_random(21, 3000, 500)
    with pytest.raises(sl1m.SL1MError) as e:
        sl1m.Plan.from_workload(wl, grid="require")
    assert "grid evaluation required" in str(e.value)
    assert sl1m.Plan.from_workload(wl).info()["grid"] == 0      # auto falls back
    wl1 = W.config1()
    with pytest.raises(sl1m.SL1MError):
        sl1m.Plan.from_workload(wl1, precision="fp64", grid="require")
    assert sl1m.Plan.from_workload(wl1, precision="fp64").info()["grid"] == 0
    # a repeated position cannot be one sign slot: auto uses the direct path
    # and the duplicated pixels both get the column they share
    l = np.concatenate([wl1.l, wl1.l[:3]])
    m = np.concatenate([wl1.m, wl1.m[:3]])
    wld = _with_pixels(W.config1(), l, m)
    with pytest.raises(sl1m.SL1MError):
        sl1m.Plan.from_workload(wld, grid="require")
    plan = sl1m.Plan.from_workload(wld)
    assert plan.info()["grid"] == 0
    p = O.Problem.from_workload(wld)
    x = np.random.default_rng(2).standard_normal(wld.n_pix)
    assert rel(plan.forward(x).cpu().numpy(), O.forward(p, x)) <= TOL


def test_grid_config2_full_size_against_direct():
    """Config 2 at full size: every visibility and pixel of the grid
    evaluation against the direct evaluation (both FP32; the direct one is
    pinned to the oracle on samples elsewhere), plus sampled oracle checks."""
    wl = W.config2()
    say(f"[case] grid config2 full n_pix={wl.n_pix} n_vis={wl.n_vis}")
    rng = np.random.default_rng(3)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    pg = sl1m.Plan.from_workload(wl, grid="require")
    say(f"    info {pg.info()}")
    Vg = pg.forward(x).cpu().numpy()
    gg = pg.adjoint(r).cpu().numpy()
    pg.close()
    pd = sl1m.Plan.from_workload(wl, grid="off")
    Vd = pd.forward(x).cpu().numpy()
    gd = pd.adjoint(r).cpu().numpy()
    pd.close()
    p = O.Problem.from_workload(wl)
    ks = np.arange(0, wl.n_vis, 211)
    js = np.arange(0, wl.n_pix, 127)
    Vo, go = O.forward_rows(p, x, ks), O.adjoint_cols(p, r, js)
    ef = rel(Vg[ks], Vo)
    ea = rel(gg[js], go)
    wf = E.worst_ratio(Vg[ks], Vo, E.abs_forward_rows(p, x, ks), wl.n_pix)
    wa = E.worst_ratio(gg[js], go, E.abs_adjoint_cols(p, r, js), wl.n_vis)
    say(f"    grid vs direct forward {rel(Vg, Vd):.3e} adjoint {rel(gg, gd):.3e}; "
        f"grid vs oracle sampled forward {ef:.3e} adjoint {ea:.3e}; "
        f"element-wise {wf:.3e} {wa:.3e}")
    assert rel(Vg, Vd) <= TOL and rel(gg, gd) <= TOL
    assert ef <= TOL and ea <= TOL
    assert wf <= 1.0 and wa <= 1.0


def test_grid_config4_full_size_against_direct():
    """Config 4 at full size (1024^2 delta grid and 512^2, 256^2, 128^2
    Gaussian layers, direction-dependent gains): all four segments on the grid
    path; every output against the direct evaluation, sampled outputs against
    the oracle."""
    wl = W.config4()
    say(f"[case] grid config4 full n_pix={wl.n_pix} n_vis={wl.n_vis}")
    rng = np.random.default_rng(4)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    pg = sl1m.Plan.from_workload(wl, grid="require")
    info = pg.info()
    say(f"    info {info}")
    assert info["grid"] == 4
    Vg = pg.forward(x).cpu().numpy()
    gg = pg.adjoint(r).cpu().numpy()
    pg.close()
    pd = sl1m.Plan.from_workload(wl, grid="off")
    Vd = pd.forward(x).cpu().numpy()
    gd = pd.adjoint(r).cpu().numpy()
    pd.close()
    p = O.Problem.from_workload(wl)
    ks = np.arange(0, wl.n_vis, 4099)
    js = np.concatenate([np.arange(0, 1024 * 1024, 10007), np.arange(1024 * 1024, wl.n_pix, 2003)])
    Vo, go = O.forward_rows(p, x, ks), O.adjoint_cols(p, r, js)
    ef = rel(Vg[ks], Vo)
    ea = rel(gg[js], go)
    wf = E.worst_ratio(Vg[ks], Vo, E.abs_forward_rows(p, x, ks), wl.n_pix)
    wa = E.worst_ratio(gg[js], go, E.abs_adjoint_cols(p, r, js), wl.n_vis)
    say(f"    grid vs direct forward {rel(Vg, Vd):.3e} adjoint {rel(gg, gd):.3e}; "
        f"grid vs oracle sampled forward {ef:.3e} adjoint {ea:.3e}; "
        f"element-wise {wf:.3e} {wa:.3e}")
    assert rel(Vg, Vd) <= TOL and rel(gg, gd) <= TOL
    assert ef <= TOL and ea <= TOL
    assert wf <= 1.0 and wa <= 1.0


# case -> whether multi-RHS calls of 2 and 4 sides take the grid evaluation
# (every grid segment a square delta grid; the Gaussian pixels of
# grid_plus_gauss stay direct in the same call)
MULTI = {"config1": 8, "odd45": 8, "disk64": 8, "grid_plus_gauss": 8, "rect80x24_gains": 0,
         "layers_mixed": 0}


@pytest.mark.parametrize("name", list(MULTI))
def test_grid_multi_rhs(name):
    """Multi-RHS calls (2, 4 and 8 sides, as the paper's polarisations through one
    matrix): every side against the oracle, and equal to the plan's
    single-side call of that side.  The forward is bitwise equal where every
    pixel is on the grid (the same tiles, rows and summation order), within
    1e-6 where direct tiles of other pixels take part (their multi-RHS
    instantiations may round differently).  The adjoint's shared-phasor tile
    forms C r in Cartesian form where the single-side tile folds the
    residual's phase into C, so the two agree to FP32 rounding of each
    entry: within 1e-6 (norm-relative)."""
    wl = _case(name)
    say(f"[case] grid multi-RHS {name} n_pix={wl.l.size} n_vis={wl.u.size}")
    plan = sl1m.Plan.from_workload(wl, max_rhs=8)
    info = plan.info()
    say(f"    info {info}")
    assert info["grid_multi"] == MULTI[name]
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(SEEDS[name] + 50)
    X = rng.standard_normal((8, wl.l.size))
    Rr = rng.standard_normal((8, wl.u.size)) + 1j * rng.standard_normal((8, wl.u.size))
    mags = ([E.abs_forward_rows(p, X[r]) for r in range(8)],
            [E.abs_adjoint_cols(p, Rr[r]) for r in range(8)])
    for nr in (2, 4, 8):
        Vg = plan.forward_multi(X[:nr]).cpu().numpy()
        gg = plan.adjoint_multi(Rr[:nr]).cpu().numpy()
        Vo = O.forward(p, X[:nr])
        go = O.adjoint(p, Rr[:nr])
        for r in range(nr):
            ef, ea = rel(Vg[r], Vo[r]), rel(gg[r], go[r])
            wf = E.worst_ratio(Vg[r], Vo[r], mags[0][r], wl.l.size)
            wa = E.worst_ratio(gg[r], go[r], mags[1][r], wl.u.size)
            say(f"    nr={nr} side {r}: forward {ef:.3e} adjoint {ea:.3e} "
                f"element-wise {wf:.3e} {wa:.3e}")
            assert ef <= TOL and ea <= TOL
            assert wf <= 1.0 and wa <= 1.0
            V1 = plan.forward(X[r]).cpu().numpy()
            g1 = plan.adjoint(Rr[r]).cpu().numpy()
            say(f"    nr={nr} side {r}: multi vs single forward {rel(Vg[r], V1):.3e} "
                f"adjoint {rel(gg[r], g1):.3e}")
            if MULTI[name] and name != "grid_plus_gauss":
                assert np.array_equal(V1, Vg[r])
            else:
                assert rel(Vg[r], V1) <= 1e-6
            assert rel(gg[r], g1) <= 1e-6
