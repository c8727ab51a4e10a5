"""Grid evaluation of the delta-pixel operators (through the C ABI).

The grid evaluation computes the same operator as the direct one (the
element of eq. (deltam) factorised into per-|l|, per-|m| and per-radius
phasors).  Each case checks both evaluations against the FP64 oracle at the
FP32 operator tolerance (norm-relative 1e-5) and that the plan took the path
the case is about.  Sizes span several tiles, end in ragged tails (|m| groups
of 8 that do not divide the |m| count, visibility counts that are not
multiples of the tile) and cover the degenerate cells (the l = 0 and m = 0
rows, cells with missing sign slots, empty cells).
"""
import sys

import numpy as np
import pytest

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


SEEDS = {"config1": 0, "odd45": 1, "disk64": 2, "rect80x24_gains": 3, "grid_plus_gauss": 4}


def _case(name):
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
    raise KeyError(name)


CASES = ["config1", "odd45", "disk64", "rect80x24_gains", "grid_plus_gauss"]


@pytest.mark.parametrize("name", CASES)
def test_grid_and_direct_match_oracle(name):
    wl = _case(name)
    say(f"[case] grid {name} n_pix={wl.n_pix} n_vis={wl.n_vis}")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    p = O.Problem.from_workload(wl)
    Vo = O.forward(p, x)
    go = O.adjoint(p, r)
    out = {}
    for mode in ("require", "off"):
        plan = sl1m.Plan.from_workload(wl, grid=mode)
        info = plan.info()
        assert info["grid"] == (1 if mode == "require" else 0)
        V = plan.forward(x).cpu().numpy()
        g = plan.adjoint(r).cpu().numpy()
        ef, ea = rel(V, Vo), rel(g, go)
        say(f"    {mode:8s} forward {ef:.3e} adjoint {ea:.3e} info {info}")
        assert ef <= TOL and ea <= TOL
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
    ef = rel(Vg[ks], O.forward_rows(p, x, ks))
    ea = rel(gg[js], O.adjoint_cols(p, r, js))
    say(f"    grid vs direct forward {rel(Vg, Vd):.3e} adjoint {rel(gg, gd):.3e}; "
        f"grid vs oracle sampled forward {ef:.3e} adjoint {ea:.3e}")
    assert rel(Vg, Vd) <= TOL and rel(gg, gd) <= TOL
    assert ef <= TOL and ea <= TOL
