"""Pins of the oracle's adaptive quad-tree refinement (Section "Acceleration
strategies", reading R17): the cells tile the field, refinement conserves the
start image's flux, the decision rule is the stated one, and on a single
point source the refinement follows the source down the tree."""
import math

import numpy as np

import oracle as O

Q = O.quadtree


def _covering_cells(l, m, h, pl, pm):
    """Indices of the cells containing point (pl, pm) (brute force)."""
    return np.nonzero((np.abs(pl - l) <= h / 2 + 1e-15) & (np.abs(pm - m) <= h / 2 + 1e-15))[0]


def test_refinement_tiles_the_field_and_conserves_flux():
    rng = np.random.default_rng(3)
    half, n0 = 0.2, 4
    l, m, h = Q.level0_cells(n0, half)
    h_min = h[0] / 8
    for _ in range(3):
        img = np.where(rng.random(l.size) < 0.3, rng.uniform(0, 1, l.size), 0.0)
        nl, nm, nh, x0, split = Q.refine(l, m, h, img, 0.01, h_min)
        # decision rule, brute force
        thr = 0.01 * img.max()
        for j in range(l.size):
            assert split[j] == (img[j] > thr and img[j] > 0 and h[j] > h_min * (1 + 1e-9))
        assert nl.size == l.size + 3 * int(split.sum())
        assert math.isclose(x0.sum(), img.sum(), rel_tol=1e-13)
        assert math.isclose(float(np.sum(nh ** 2)), (2 * half) ** 2, rel_tol=1e-12)
        # every point of a lattice inside the field lies in exactly one cell
        pts = (np.arange(64) + 0.37) / 64 * 2 * half - half
        for pl in pts[::5]:
            for pm in pts[::7]:
                assert _covering_cells(nl, nm, nh, pl, pm).size == 1
        l, m, h = nl, nm, nh


def test_refinement_follows_a_point_source():
    """A noiseless off-centre point source, uv coverage uniform over a disk of
    radius 250 wavelengths, level-0 cells 2.5 beams wide: at every level but
    the last the cell containing the source holds the image maximum and is
    refined, and at the last level it holds at least half the maximum."""
    rng = np.random.default_rng(5)
    half, n0, levels = 0.02, 4, 3
    r = 250.0 * np.sqrt(rng.random(500))
    th = 2 * np.pi * rng.random(500)
    u, v = r * np.cos(th), r * np.sin(th)
    w = rng.normal(0, 20, 500)
    ls, ms, S = 0.3 * half * 0.41, -0.3 * half * 0.77, 2.0
    src = O.Problem(l=[ls], m=[ms], u=u, v=v, w=w, threads=2)
    V = O.forward(src, np.array([S]))
    h_min = 2 * half / n0 / 2 ** (levels - 1)

    def problem_of(l, m, sigma, kind):
        return O.Problem(l=l, m=m, sigma=sigma, kind=kind, u=u, v=v, w=w, threads=2)

    res = Q.quadtree_solve(problem_of, V, 20.0, n0, half, levels, 300, h_min)
    for a, b in zip(res[:-1], res[1:]):
        j = _covering_cells(a["l"], a["m"], a["h"], ls, ms)
        assert j.size == 1 and np.argmax(a["image"]) == j[0]
        k = _covering_cells(b["l"], b["m"], b["h"], ls, ms)[0]
        assert b["h"][k] == a["h"][j[0]] / 2          # the source's cell was refined
    last = res[-1]
    k = _covering_cells(last["l"], last["m"], last["h"], ls, ms)[0]
    assert last["h"][k] == h_min and last["image"][k] >= 0.5 * last["image"].max()


def test_certificate_split_threshold_on_a_source_at_the_phase_centre():
    """`certificate_split` against a closed form: a unit-gain point source of
    flux S at the phase centre has V_k = S for every visibility (n = 1, zero
    phase), so with a zero image the delta child at the phase centre has
    Re(M^H (V - M I)) = S N_v exactly and every other child less.  A cell of
    side 2 h_min centred at (h_min/2, h_min/2) has that child; it is marked
    just below the threshold lam (1 + tol) = S N_v and not just above, and
    not at all once the image explains V (residual zero)."""
    rng = np.random.default_rng(11)
    n_v, S, h_min, tol = 300, 1.5, 0.01, 1e-3
    r = 250.0 * np.sqrt(rng.random(n_v))
    th = 2 * np.pi * rng.random(n_v)
    u, v, w = r * np.cos(th), r * np.sin(th), rng.normal(0, 20, n_v)
    V = np.full(n_v, S, np.complex128)  # closed form, not the oracle's forward

    def problem_of(l, m, sigma, kind):
        return O.Problem(l=l, m=m, sigma=sigma, kind=kind, u=u, v=v, w=w, threads=2)

    # a coarse cell (split candidate) and a fine delta cell at the phase centre
    l = np.array([h_min / 2, 0.0])
    m = np.array([h_min / 2, 0.0])
    h = np.array([2 * h_min, h_min])
    sigma, kind = Q.cell_pixels(h, h_min)
    op = O.Operator(problem_of(l, m, sigma, kind))
    thr = S * n_v / (1 + tol)
    zero = np.zeros(2)
    below = Q.certificate_split(problem_of, V, thr * (1 - 1e-6), l, m, h, zero, op, h_min, tol=tol)
    above = Q.certificate_split(problem_of, V, thr * (1 + 1e-6), l, m, h, zero, op, h_min, tol=tol)
    assert below.tolist() == [True, False]
    assert above.tolist() == [False, False]
    explained = Q.certificate_split(problem_of, V, 1e-9, l, m, h, np.array([0.0, S]), op, h_min,
                                    tol=tol)
    assert explained.tolist() == [False, False]
