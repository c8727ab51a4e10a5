"""CPU study of the quad-tree refinement (Section "Acceleration strategies")
on the oracle: how close the refined solution comes to the objective of the
full-grid solve, under the paper's rule (refine cells above 1 % of the
maximum) with two Gaussian cell widths, and with an added rule that also
refines cells whose children violate the optimality conditions
(`certificate_split`).  Test infrastructure: only the oracle is used.

Workload (seeded): a 64 x 64 grid over +-0.05 as the finest level, 3,000
visibilities with u, v uniform in a 400-wavelength disk and w ~ N(0, 50^2),
four extended Gaussian sources (paper sigma 3..8 grid spacings, fluxes
U[1, 4], given as fine delta sums) and six point sources (U[0.2, 1]), noise
0.01 per component; lambda = k * 3 sigma sqrt(N_v), k = 1 and 10.  Every
solve runs to a relative change of the objective of 1e-6 (checked every 5
iterations, at most 3,000).  Quad-tree: 8 x 8 cells at level 0, four levels
to the 64 x 64 spacing (more when the certificate rule keeps refining).

    python -m oracle.quadtree_study
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import quadtree as Q
from . import sl1m_oracle as O

N, HALF, N_VIS, EPS, CAP = 64, 0.05, 3000, 1e-6, 3000


def _workload():
    from paper_1310_2078_amd import workloads as W
    rng = np.random.default_rng(7)
    d = 2 * HALF / N
    u, v, w = W.disk_uvw(rng, N_VIS, 400.0, 50.0)
    L0, M0, _ = W.grid_pixels(N, HALF)
    inner = W.inner_pixel_indices(N)
    el, em, ef = [], [], []
    for c in rng.choice(inner, 4, replace=False):
        s = rng.uniform(3 * d, 8 * d)
        fl = rng.uniform(1, 4)
        offs = np.arange(-12, 13) * s / 4
        dl, dm = np.meshgrid(offs, offs)
        prof = np.exp(-np.pi * (dl ** 2 + dm ** 2) / s ** 2)
        el.append((L0[c] + dl).ravel())
        em.append((M0[c] + dm).ravel())
        ef.append((fl * prof / prof.sum()).ravel())
    for c in rng.choice(inner, 6, replace=False):
        el.append(np.array([L0[c]]))
        em.append(np.array([M0[c]]))
        ef.append(np.array([rng.uniform(0.2, 1.0)]))
    el, em, ef = map(np.concatenate, (el, em, ef))
    col = np.clip(np.rint(el / d).astype(int) + N // 2, 0, N - 1)
    row = np.clip(np.rint(em / d).astype(int) + N // 2, 0, N - 1)
    truth = np.zeros(N * N)
    np.add.at(truth, col + N * row, ef)
    V = O.forward(O.Problem(l=el, m=em, u=u, v=v, w=w), ef)
    V = V + 0.01 * (rng.standard_normal(N_VIS) + 1j * rng.standard_normal(N_VIS))
    return u, v, w, V, truth, L0, M0, d


def _on_grid(l, m, h, img, d):
    """Cell fluxes spread evenly over the finest pixels each cell covers."""
    out = np.zeros(N * N)
    for j in range(l.size):
        k = int(round(h[j] / d))
        c0 = int(round((l[j] - h[j] / 2 + d / 2) / d)) + N // 2
        r0 = int(round((m[j] - h[j] / 2 + d / 2) / d)) + N // 2
        for a in range(k):
            for b in range(k):
                if 0 <= c0 + a < N and 0 <= r0 + b < N:
                    out[c0 + a + N * (r0 + b)] += img[j] / (k * k)
    return out


def quadtree(problem_of, V, lam, d, sigma_factor, certificate, n0=8, levels=4):
    h_min = d
    l, m, h = Q.level0_cells(n0, HALF, h_min / 2)
    x0, cost, lev = None, 0.0, 0
    while True:
        fine = h <= h_min * (1 + 1e-9)
        sigma = np.where(fine, 0.0, sigma_factor * h)
        kind = np.where(fine, O.PIX_DELTA, O.PIX_GAUSS_WIDE).astype(np.uint8)
        op = O.Operator(problem_of(l, m, sigma, kind), dense=True)
        if x0 is None:
            x0 = O.dirty_image(op, V)
        L, _ = O.power_iteration(op, 30)
        res = O.fista_from(op, V, L, lam, CAP, x0, eps=EPS, check_every=5)
        cost += res.iters * l.size
        lev += 1
        img = res.image
        split = (img > 0.01 * img.max()) & (h > h_min * (1 + 1e-9)) & (img > 0)
        if lev >= levels and not certificate:
            break
        if certificate:
            split |= Q.certificate_split(problem_of, V, lam, l, m, h, img, op, h_min,
                                         sigma_factor)
            cost += 4 * np.count_nonzero(h > h_min * (1 + 1e-9))
        if not split.any():
            break
        l, m, h, x0, _ = Q.refine_mask(l, m, h, img, split)
    return res, l, m, h, cost, lev


def main():
    u, v, w, V, truth, L0, M0, d = _workload()

    def problem_of(l, m, sigma, kind):
        return O.Problem(l=l, m=m, u=u, v=v, w=w, sigma=sigma, kind=kind)

    def rms(x):
        return float(np.sqrt(np.mean((x - truth) ** 2)))

    print("| lambda | solve | cells | levels | F / F(full grid) | cost / full grid | RMS vs sky |")
    print("|---|---|---:|---:|---:|---:|---:|")
    for k in (1.0, 10.0):
        lam = 3 * 0.01 * math.sqrt(N_VIS) * k
        op = O.Operator(problem_of(L0, M0, np.zeros(N * N), np.zeros(N * N, np.uint8)), dense=True)
        L, _ = O.power_iteration(op, 30)
        full = O.fista(op, V, L, lam, CAP, eps=EPS, check_every=5)
        print(f"| {k:g} x | full 64x64 grid ({full.nnz} non-zero) | {N * N} | 1 | 1 | 1 | "
              f"{rms(full.image):.4g} |", flush=True)
        for sf, cert in ((0.5, False), (1.0, False), (0.5, True), (1.0, True)):
            t0 = time.time()
            res, l, m, h, cost, lev = quadtree(problem_of, V, lam, d, sf, cert)
            name = f"quad-tree, sigma = {sf:g} h, " + ("1 % + certificate" if cert else "1 %")
            print(f"| {k:g} x | {name} | {l.size} | {lev} | {res.F / full.F:.4f} | "
                  f"{cost / (full.iters * N * N):.3f} | {rms(_on_grid(l, m, h, res.image, d)):.4g} |",
                  flush=True)


if __name__ == "__main__":
    main()
