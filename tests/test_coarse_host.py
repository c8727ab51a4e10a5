"""Coarse-to-fine warm start (Section "Acceleration strategies", reading
R18), host parts on the CPU: the oracle's upscaling pinned by what the
reading fixes (total flux, centroid, positivity, the weights of one pixel,
the grid alignment), and the library driver's upscaling equal to it."""
import numpy as np

import oracle as O
from paper_1310_2078_amd import coarse as C
from paper_1310_2078_amd import workloads as W


def test_oracle_upscale_of_one_interior_pixel():
    n = 6
    img = np.zeros(n * n)
    img[2 + n * 3] = 8.0                      # col 2, row 3
    up = O.coarse.upscale(img, n).reshape(2 * n, 2 * n)   # [row, col]
    expect = np.zeros((2 * n, 2 * n))
    for b, wb in ((-1, 0.25), (0, 0.5), (1, 0.25)):
        for a, wa in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            expect[6 + b, 4 + a] = 8.0 * wa * wb
    np.testing.assert_array_equal(up, expect)


def test_oracle_upscale_keeps_flux_centroid_and_sign():
    rng = np.random.default_rng(0)
    n = 8
    half = 0.05
    img = np.maximum(rng.standard_normal(n * n), 0.0)
    img[0] = 3.0                              # a corner pixel: shares fold inwards
    up = O.coarse.upscale(img, n)
    assert np.all(up >= 0.0)
    assert abs(up.sum() - img.sum()) <= 1e-12 * img.sum()
    lc, mc = O.coarse.grid(n, half)
    lf, mf = O.coarse.grid(2 * n, half)
    inner = np.zeros(n * n)
    inner[3 + n * 4] = 1.0                    # away from the border: centroid kept
    ui = O.coarse.upscale(inner, n)
    assert abs(np.dot(ui, lf) - lc[3 + n * 4]) <= 1e-15
    assert abs(np.dot(ui, mf) - mc[3 + n * 4]) <= 1e-15


def test_grid_alignment_coarse_on_fine():
    """Coarse pixel (i, j) lies on fine pixel (2i, 2j), and both grids follow
    the workload grid convention (phase centre a pixel)."""
    n, half = 16, 0.3
    lc, mc = O.coarse.grid(n, half)
    lf, mf = O.coarse.grid(2 * n, half)
    for col, row in ((0, 0), (5, 9), (15, 15)):
        j, jf = col + n * row, 2 * col + 2 * n * 2 * row
        assert lc[j] == lf[jf] and mc[j] == mf[jf]
    lw, mw, _ = W.grid_pixels(n, half)
    np.testing.assert_array_equal(lc, lw)
    np.testing.assert_array_equal(mc, mw)


def test_library_upscale_equals_oracle():
    rng = np.random.default_rng(1)
    for n in (4, 9, 32):
        img = np.maximum(rng.standard_normal(n * n), 0.0)
        np.testing.assert_allclose(C.upscale2(img, n), O.coarse.upscale(img, n),
                                   rtol=0, atol=1e-15)
        lc, mc = C.grid_positions(n, 0.2)
        lo, mo = O.coarse.grid(n, 0.2)
        np.testing.assert_array_equal(lc, lo)
        np.testing.assert_array_equal(mc, mo)
