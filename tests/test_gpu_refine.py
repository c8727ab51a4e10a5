"""Adaptive quad-tree refinement on the GPU (Section "Acceleration
strategies", reading R17) against the oracle, level by level: each level's
start image, solution and next cell list, with mixed-sigma Gaussian pixels
and delta pixels in one irregular pixel set."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1310_2078_amd import refine as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_quadtree_levels_match_oracle():
    say("[case] quad-tree refinement, 3 levels")
    rng = np.random.default_rng(11)
    half, n0, levels, iters, lam = 0.02, 4, 3, 100, 20.0
    n_vis = 700
    r = 250.0 * np.sqrt(rng.random(n_vis))
    th = 2 * np.pi * rng.random(n_vis)
    u, v = r * np.cos(th), r * np.sin(th)
    w = rng.normal(0, 20, n_vis)
    ls = np.array([0.0025, -0.011, 0.013])
    ms = np.array([-0.0046, 0.007, 0.012])
    S = np.array([2.0, 1.2, 0.7])
    V = O.forward(O.Problem(l=ls, m=ms, u=u, v=v, w=w), S)
    V = V + 0.01 * (rng.standard_normal(n_vis) + 1j * rng.standard_normal(n_vis))
    h_min = 2 * half / n0 / 2 ** (levels - 1)
    got = R.quadtree_solve(u, v, w, V, lam, n0, half, levels, iters, h_min)
    assert len(got) == levels
    for i, lev in enumerate(got):
        sigma, kind = O.quadtree.cell_pixels(lev.h, h_min)
        op = O.Operator(O.Problem(l=lev.l, m=lev.m, sigma=sigma, kind=kind, u=u, v=v, w=w))
        if i == 0:
            es = rel(lev.start, O.dirty_image(op, V))
            say(f"    level 0 dirty image rel err {es:.3e}")
            assert es <= 1e-5
        ref = O.fista_from(op, V, lev.info["L"], lam, iters, lev.start)
        err = np.max(np.abs(lev.image - ref.image)) / np.max(ref.image)
        say(f"    level {i}: {lev.l.size} cells ({int(np.sum(kind == 0))} delta), "
            f"image err/peak {err:.3e}, F {lev.info['F']:.6g} / {ref.F:.6g}")
        assert err <= 1e-4
        if i + 1 < levels:
            nxt = got[i + 1]
            nl, nm, nh, x0, split = O.quadtree.refine(lev.l, lev.m, lev.h, lev.image, 0.01, h_min)
            assert np.array_equal(nl, nxt.l) and np.array_equal(nm, nxt.m)
            assert np.array_equal(nh, nxt.h)
            np.testing.assert_allclose(nxt.start, x0, rtol=1e-6, atol=1e-7)
            # the oracle's own image takes the same decisions away from the threshold
            _, _, _, _, split_o = O.quadtree.refine(lev.l, lev.m, lev.h, ref.image, 0.01, h_min)
            near = np.abs(lev.image - 0.01 * lev.image.max()) <= 1e-3 * lev.image.max()
            assert np.array_equal(split[~near], split_o[~near])
