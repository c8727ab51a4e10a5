"""The oracle's coarse-to-fine warm start (Section "Acceleration strategies":
solve on a coarse grid, double the resolution, upscale, continue).

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: written independently
of the GPU library's driver, from the same reading (R18):

* square grids with the pixel-grid convention of Section "Delta function
  pixels" (offsets -N/2 .. N/2-1 of spacing 2 half / N), so coarse pixel
  (i, j) of the N/2 grid lies on fine pixel (2i, 2j);
* upscaling: coarse pixel (i, j) gives fine pixel (2i + a, 2j + b),
  a, b in {-1, 0, 1}, the share w_a w_b of its flux with w_0 = 1/2 and
  w_-1 = w_1 = 1/4; a share that would fall outside the grid goes to the
  nearest border pixel;
* every level is the printed iteration started from the previous level's
  upscaled image (the warm start of `fista_from`).
"""
from __future__ import annotations

import numpy as np

from . import sl1m_oracle as O


def grid(n: int, half: float):
    """(l, m) of the n x n grid, row-major j = col + n row."""
    d = 2.0 * half / n
    l = np.empty(n * n)
    m = np.empty(n * n)
    for row in range(n):
        for col in range(n):
            l[col + n * row] = (col - n // 2) * d
            m[col + n * row] = (row - n // 2) * d
    return l, m


def upscale(img, n: int):
    """An n x n image onto the 2n x 2n grid (pure-Python loops)."""
    w = {-1: 0.25, 0: 0.5, 1: 0.25}
    out = np.zeros(4 * n * n)
    for row in range(n):
        for col in range(n):
            c = float(img[col + n * row])
            for a in (-1, 0, 1):
                for b in (-1, 0, 1):
                    fc = min(max(2 * col + a, 0), 2 * n - 1)
                    fr = min(max(2 * row + b, 0), 2 * n - 1)
                    out[fc + 2 * n * fr] += w[a] * w[b] * c
    return out


def coarse_to_fine(n: int, half: float, levels: int, u, v, w, V, lam: float, n_iter: int,
                   L_per_level, **gains):
    """Images of every level (coarsest first) with the given L per level."""
    images = []
    prev = None
    for i in range(levels):
        ni = n >> (levels - 1 - i)
        l, m = grid(ni, half)
        op = O.Operator(O.Problem(l=l, m=m, u=u, v=v, w=w, **gains))
        if prev is None:
            res = O.fista(op, V, L_per_level[i], lam, n_iter)
        else:
            res = O.fista_from(op, V, L_per_level[i], lam, n_iter, upscale(prev, ni // 2))
        prev = res.image
        images.append(res.image)
    return images
