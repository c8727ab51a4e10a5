"""Adaptive quad-tree refinement of the pixel set, oracle version.

TEST INFRASTRUCTURE ONLY (like sl1m_oracle): plain NumPy on the FP64 oracle
operators; the GPU library never calls it.

Section "Acceleration strategies" of the paper: solve on a coarse pixel grid,
subdivide the pixels where emission is detected (above 1 % of the maximum),
solve again, and repeat down to the resolution limit, with the same lambda at
every level.  Reading R17 fixes what the paper leaves open:

* a pixel is a square cell of side h centred at (l, m); it enters the operator
  as a wide-field Gaussian pixel with sigma = h / 2 (eq. samlm5), and cells of
  the finest side h_min as delta pixels (eq. deltam);
* level 0 is an n0 x n0 grid of cells over [-a, a]^2 shifted by -h_min / 2
  in l and m, cell centres at (i + 1/2) h0 - a - h_min / 2, so that the finest
  cells are centred on the pixel grid (i - N/2) h_min of reading R8 (N h_min =
  2a); it starts from the dirty image (reading R16);
* a level runs a fixed number of FISTA iterations from its start image, with
  L from power iteration on that level's operator;
* after a level, every cell whose image value exceeds frac * max(image) and
  whose side exceeds h_min is replaced, in place in the pixel list, by its
  four children (side h / 2, centres offset by (-h/4, -h/4), (+h/4, -h/4),
  (-h/4, +h/4), (+h/4, +h/4), in that order); the decision is taken in FP64;
* the next level starts from the previous image with a refined cell's value
  split equally among its children (flux conservation of the coarse-to-fine
  upscaling).

`certificate_split` (an extra refinement rule used only by the study in
`quadtree_study.py`, never compared with the GPU library) is pinned against
the closed form of a point source at the phase centre
(`tests/test_quadtree_oracle.py`).
"""
from __future__ import annotations

import numpy as np

from . import sl1m_oracle as O


def level0_cells(n0: int, half: float, shift: float = 0.0):
    """Cell centres and sides of the level-0 grid over [-half, half]^2, moved
    by -shift in l and m."""
    h = 2.0 * half / n0
    c = (np.arange(n0) + 0.5) * h - half - shift
    L, M = np.meshgrid(c, c, indexing="xy")
    return L.ravel(), M.ravel(), np.full(n0 * n0, h)


def cell_pixels(h, h_min: float):
    """sigma and kind of each cell's pixel (reading R17)."""
    fine = h <= h_min * (1.0 + 1e-9)
    sigma = np.where(fine, 0.0, h / 2.0)
    kind = np.where(fine, O.PIX_DELTA, O.PIX_GAUSS_WIDE).astype(np.uint8)
    return sigma, kind


def refine(l, m, h, image, frac: float, h_min: float):
    """The next level's cells and start image (reading R17)."""
    image = np.asarray(image, np.float64)
    thr = frac * float(np.max(image)) if image.size else 0.0
    split = (image > thr) & (h > h_min * (1.0 + 1e-9)) & (image > 0.0)
    return refine_mask(l, m, h, image, split)


def refine_mask(l, m, h, image, split):
    """Replaces the cells marked in `split` by their four children (reading
    R17's order and start values)."""
    image = np.asarray(image, np.float64)
    nl, nm, nh, x0 = [], [], [], []
    for j in range(l.shape[0]):
        if not split[j]:
            nl.append(l[j]); nm.append(m[j]); nh.append(h[j]); x0.append(image[j])
            continue
        q = h[j] / 4.0
        for dl, dm in ((-q, -q), (q, -q), (-q, q), (q, q)):
            nl.append(l[j] + dl); nm.append(m[j] + dm); nh.append(h[j] / 2.0)
            x0.append(image[j] / 4.0)
    return np.array(nl), np.array(nm), np.array(nh), np.array(x0), split


def certificate_split(problem_of, V, lam, l, m, h, image, op, h_min: float,
                      sigma_factor: float = 0.5, tol: float = 1e-3):
    """Cells whose refinement would lower the objective by the optimality
    conditions (Section "Implementation of SL1M"): a cell with side > h_min is
    marked when one of its four children, as a pixel of the next level, has
    Re(M^H (V - M I))_child > lam (1 + tol), i.e. would leave zero in the
    next solve.  Used by the refinement study beside the paper's
    emission-detected rule."""
    coarse = np.where(h > h_min * (1.0 + 1e-9))[0]
    mark = np.zeros(l.shape[0], bool)
    if coarse.size == 0:
        return mark
    res = np.asarray(V, np.complex128) - op.forward(image)
    q = h[coarse] / 4.0
    cl = np.concatenate([l[coarse] - q, l[coarse] + q, l[coarse] - q, l[coarse] + q])
    cm = np.concatenate([m[coarse] - q, m[coarse] - q, m[coarse] + q, m[coarse] + q])
    ch = np.concatenate([h[coarse] / 2.0] * 4)
    fine = ch <= h_min * (1.0 + 1e-9)
    cs = np.where(fine, 0.0, sigma_factor * ch)
    ck = np.where(fine, O.PIX_DELTA, O.PIX_GAUSS_WIDE).astype(np.uint8)
    G = O.adjoint(problem_of(cl, cm, cs, ck), res)
    mark[coarse] = (G.reshape(4, -1) > lam * (1.0 + tol)).any(axis=0)
    return mark


def quadtree_solve(problem_of, V, lam: float, n0: int, half: float, levels: int, iters: int,
                   h_min: float, frac: float = 0.01, power_iters: int = 30, eps: float = 0.0,
                   check_every: int = 5):
    """Runs `levels` levels; problem_of(l, m, sigma, kind) gives the oracle
    Problem of a pixel set against the observation's visibilities.  Each level
    runs at most `iters` iterations, fewer with eps > 0 (the relative-change
    rule, reading R6).  Returns a list with, per level, the cells, the start
    image, L and the image."""
    l, m, h = level0_cells(n0, half, h_min / 2.0)
    out = []
    x0 = None
    for lev in range(levels):
        sigma, kind = cell_pixels(h, h_min)
        op = O.Operator(problem_of(l, m, sigma, kind))
        L, _ = O.power_iteration(op, power_iters)
        start = O.dirty_image(op, V) if x0 is None else x0
        res = O.fista_from(op, V, L, lam, iters, start, eps=eps, check_every=check_every)
        out.append({"l": l, "m": m, "h": h, "start": start, "L": L, "image": res.image,
                    "F": res.F})
        if lev + 1 < levels:
            l, m, h, x0, _ = refine(l, m, h, res.image, frac, h_min)
    return out
