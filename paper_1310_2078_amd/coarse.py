"""Coarse-to-fine warm start on the GPU library (Section "Acceleration
strategies" of the paper: solve on a coarse pixel grid, double the
resolution, upscale the solution and use it to start the finer solve).

Each level is one plan (a square delta grid over the field, plus optional
pixels carried unchanged through every level, e.g. Gaussian layers) and one
solve through the C ABI (sl1m_solve, or sl1m_solve_from from the upscaled
previous level).  Conventions (reading R18):

* the grids follow the pixel-grid convention of Section "Delta function
  pixels" (offsets -N/2 .. N/2-1 of spacing 2 half / N), so pixel i of the
  N/2 grid sits on pixel 2i of the N grid;
* upscaling spreads each coarse pixel's flux over the fine pixels within one
  coarse spacing with weights 1/4, 1/2, 1/4 per axis (centred on the coarse
  position; at the border the outer weight folds onto the edge pixel), so the
  total flux and its centroid are kept and the start stays positive;
* the same lambda at every level (the L1 term is the total flux, which the
  upscaling keeps); L by power iteration per level.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import sl1m

_TENT = ((-1, 0.25), (0, 0.5), (1, 0.25))


def grid_positions(n_side: int, half: float):
    """(l, m) of an n_side^2 grid over +-half, row-major (j = col + n row)."""
    d = 2.0 * half / n_side
    idx = np.arange(n_side * n_side, dtype=np.int64)
    return (idx % n_side - n_side // 2) * d, (idx // n_side - n_side // 2) * d


def upscale2(img: np.ndarray, n: int) -> np.ndarray:
    """An n^2 image to the 2n^2 grid (flux-conserving tent spreading)."""
    c = np.asarray(img, np.float64).reshape(n, n)
    # along the columns, then the rows
    wide = np.zeros((n, 2 * n))
    for off, wt in _TENT:
        cols = np.clip(2 * np.arange(n) + off, 0, 2 * n - 1)
        np.add.at(wide, (slice(None), cols), wt * c)
    out = np.zeros((2 * n, 2 * n))
    for off, wt in _TENT:
        rows = np.clip(2 * np.arange(n) + off, 0, 2 * n - 1)
        np.add.at(out, (rows, slice(None)), wt * wide)
    return out.ravel()


@dataclass
class Level:
    n_side: int
    image: np.ndarray      # the level's grid image (FP64 copy), row-major
    extra: Optional[np.ndarray]
    info: dict
    seconds: float         # plan creation + solve


def coarse_to_fine(n_side: int, half: float, levels: int, u, v, w, vis, lam: float,
                   n_iter, power_iters: int = 30, extra=None, device="cuda",
                   ant_p=None, ant_q=None, ant_gain=None, ant_fwhm=None,
                   first_start: str = "cold", L_per_level=None) -> List[Level]:
    """Solves the grid at n_side / 2^(levels-1), ..., n_side, each level
    started from the upscaled previous one.  n_iter: iterations per level
    (an int, or one per level).  extra: optional (l, m, sigma, kind) pixels in
    every level's plan after the grid, started from the previous level's
    values.  first_start: "cold" (zero image) or "dirty" (the dirty image).
    L_per_level: the step constants to use (default: power iteration per
    level)."""
    dev = torch.device(device)
    iters = [int(n_iter)] * levels if np.isscalar(n_iter) else [int(k) for k in n_iter]
    vis_d = torch.as_tensor(vis, device=dev)
    out: List[Level] = []
    img_prev = extra_prev = None
    for i in range(levels):
        n = n_side >> (levels - 1 - i)
        t0 = time.perf_counter()
        l, m = grid_positions(n, half)
        sigma = np.zeros(l.size)
        kind = np.zeros(l.size, np.uint8)
        if extra is not None:
            el, em, es, ek = extra
            l, m = np.concatenate([l, el]), np.concatenate([m, em])
            sigma, kind = np.concatenate([sigma, es]), np.concatenate([kind, ek])
        has_kind = bool(np.any(kind != 0))
        plan = sl1m.Plan(l, m, u, v, w, sigma=sigma if has_kind else None,
                         kind=kind if has_kind else None, ant_p=ant_p, ant_q=ant_q,
                         ant_gain=ant_gain, ant_fwhm=ant_fwhm, device=dev)
        if i == 0:
            x0 = plan.dirty_image(vis_d) if first_start == "dirty" else None
        else:
            parts = [upscale2(img_prev, n // 2)]
            if extra is not None:
                parts.append(extra_prev)
            x0 = torch.as_tensor(np.concatenate(parts), dtype=torch.float32, device=dev)
        L = 0.0 if L_per_level is None else float(L_per_level[i])
        img, info = plan.solve(vis_d, lam, iters[i], L=L, power_iters=power_iters, x0=x0)
        torch.cuda.synchronize(dev)
        secs = time.perf_counter() - t0
        h = img.cpu().numpy().astype(np.float64)
        img_prev, extra_prev = h[:n * n], (h[n * n:] if extra is not None else None)
        out.append(Level(n, img_prev, extra_prev, info, secs))
        plan.close()
    return out
