"""Adaptive quad-tree refinement of the pixel set on the GPU library
(Section "Acceleration strategies" of the paper: solve on a coarse grid,
subdivide the pixels where emission is detected, repeat to the resolution
limit, with the same lambda at every level).

Each level is one plan and one warm-started solve through the C ABI
(sl1m_dirty_image, sl1m_solve_from); this module only keeps the cell lists
and takes the refinement decisions on the host.  Conventions (reading R17):

* a cell of side h centred at (l, m) is a wide-field Gaussian pixel with
  sigma = h / 2 (eq. samlm5); cells of the finest side h_min are delta pixels;
* level 0: n0 x n0 cells over [-half, half]^2 moved by -h_min / 2 in l and m
  (centres (i + 1/2) h0 - half - h_min / 2, so that the finest cells sit on
  the pixel grid (i - N/2) h_min), started from the dirty image;
* after a level, every cell whose value exceeds frac * max (decided in FP64
  from the returned image) and whose side exceeds h_min is replaced in place by
  its four children (side h / 2, offsets (-h/4, -h/4), (+h/4, -h/4),
  (-h/4, +h/4), (+h/4, +h/4)), each starting from a quarter of its value.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np
import torch

from . import sl1m

_CHILD_DL = np.array([-1.0, 1.0, -1.0, 1.0])
_CHILD_DM = np.array([-1.0, -1.0, 1.0, 1.0])


@dataclass
class Level:
    l: np.ndarray
    m: np.ndarray
    h: np.ndarray
    start: np.ndarray      # the level's start image (FP64 copy)
    image: np.ndarray      # the level's solution (FP64 copy of the FP32/FP64 result)
    info: dict             # sl1m_solve_info of the level
    seconds: float         # plan creation + solve


def first_cells(n0: int, half: float, shift: float = 0.0):
    h = 2.0 * half / n0
    c = (np.arange(n0, dtype=np.float64) + 0.5) * h - half - shift
    m, l = np.divmod(np.arange(n0 * n0), n0)
    return c[l], c[m], np.full(n0 * n0, h)


def pixel_model(h: np.ndarray, h_min: float):
    finest = h <= h_min * (1.0 + 1e-9)
    sigma = np.where(finest, 0.0, 0.5 * h)
    kind = np.where(finest, sl1m.PIX_DELTA, sl1m.PIX_GAUSS_WIDE).astype(np.uint8)
    return sigma, kind


def split_cells(l, m, h, image, frac: float, h_min: float):
    """Next cells, their start values and the refined mask."""
    image = np.asarray(image, np.float64)
    peak = float(image.max()) if image.size else 0.0
    refine = (image > frac * peak) & (image > 0.0) & (h > h_min * (1.0 + 1e-9))
    count = np.where(refine, 4, 1)
    src = np.repeat(np.arange(l.shape[0]), count)
    # position of each new cell among its parent's children (0 for a kept cell)
    first = np.cumsum(count) - count
    child = np.arange(src.shape[0]) - first[src]
    q = np.where(refine[src], 0.25 * h[src], 0.0)
    nl = l[src] + q * _CHILD_DL[child]
    nm = m[src] + q * _CHILD_DM[child]
    nh = np.where(refine[src], 0.5 * h[src], h[src])
    x0 = np.where(refine[src], 0.25 * image[src], image[src])
    return nl, nm, nh, x0, refine


def quadtree_solve(u, v, w, vis, lam: float, n0: int, half: float, levels: int, iters: int,
                   h_min: float, frac: float = 0.01, power_iters: int = 30, ant_p=None,
                   ant_q=None, ant_gain=None, ant_fwhm=None, precision: str = "fp32",
                   device="cuda", max_cells: Optional[int] = None,
                   on_level: Optional[Callable[[Level], None]] = None, eps: float = 0.0,
                   check_every: int = 5) -> List[Level]:
    """Runs up to `levels` levels (fewer when a level would exceed max_cells).
    Each level runs at most `iters` iterations; with eps > 0 it stops earlier
    on a relative change of the objective of at most eps between checks every
    `check_every` iterations (the rule of Section "Implementation of SL1M")."""
    dev = torch.device(device)
    V = sl1m._dev(vis, torch.complex64 if precision == "fp32" else torch.complex128, dev)
    l, m, h = first_cells(n0, half, 0.5 * h_min)
    x0: Optional[np.ndarray] = None
    out: List[Level] = []
    for lev in range(levels):
        t0 = time.perf_counter()
        sigma, kind = pixel_model(h, h_min)
        plan = sl1m.Plan(l, m, u, v, w, sigma=sigma, kind=kind, ant_p=ant_p, ant_q=ant_q,
                         ant_gain=ant_gain, ant_fwhm=ant_fwhm, precision=precision, device=dev)
        start = plan.dirty_image(V) if x0 is None else \
            torch.as_tensor(x0, dtype=plan.rdtype, device=dev)
        img, info = plan.solve(V, lam, iters, L=0.0, power_iters=power_iters, x0=start,
                               eps=eps, check_every=check_every)
        image = img.double().cpu().numpy()
        start_np = start.double().cpu().numpy()
        plan.close()
        level = Level(l, m, h, start_np, image, info, time.perf_counter() - t0)
        out.append(level)
        if on_level:
            on_level(level)
        if lev + 1 == levels:
            break
        nl, nm, nh, nx0, _ = split_cells(l, m, h, image, frac, h_min)
        if max_cells is not None and nl.shape[0] > max_cells:
            break
        l, m, h, x0 = nl, nm, nh, nx0
    return out
