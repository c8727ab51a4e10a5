"""The element-wise parity bound (tests/elementwise.py) on the CPU: its
magnitude sums equal the dense |M| products, an FP32 rounding of the exact
result stays inside it, and planted mistakes of one term (a dropped pixel, a
conjugated entry) are outside it."""
import numpy as np

import oracle as O
from paper_1310_2078_amd import workloads as W

import elementwise as E


def _problem():
    wl = W.small_random(3, 300, 400, kind=W.PIX_GAUSS_WIDE, sigma=2e-3, with_gains=True)
    return O.Problem.from_workload(wl, threads=2), wl


def test_magnitude_sums_equal_dense_products():
    p, wl = _problem()
    rng = np.random.default_rng(0)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    M = O.matrix_block(p, np.arange(wl.n_vis), np.arange(wl.n_pix))
    ks = np.arange(0, wl.n_vis, 7)
    js = np.arange(0, wl.n_pix, 5)
    assert np.allclose(E.abs_forward_rows(p, x, ks, workers=3), np.abs(M[ks]) @ np.abs(x),
                       rtol=1e-13)
    assert np.allclose(E.abs_adjoint_cols(p, r, js, workers=3), np.abs(r) @ np.abs(M[:, js]),
                       rtol=1e-13)


def test_bound_accepts_rounding_and_rejects_one_wrong_term():
    p, wl = _problem()
    rng = np.random.default_rng(1)
    x = rng.standard_normal(wl.n_pix)
    M = O.matrix_block(p, np.arange(wl.n_vis), np.arange(wl.n_pix))
    V = M @ x
    mag = E.abs_forward_rows(p, x, workers=2)
    # the exact result rounded to complex64, and an FP32 evaluation
    V32 = (M.astype(np.complex64) @ x.astype(np.float32)).astype(np.complex128)
    assert E.worst_ratio(V.astype(np.complex64), V, mag, wl.n_pix) <= 1.0
    assert E.worst_ratio(V32, V, mag, wl.n_pix) <= 1.0
    # one pixel left out of visibility 17's sum
    j = int(np.argmax(np.abs(M[17]) * np.abs(x)))
    bad = V.copy()
    bad[17] -= M[17, j] * x[j]
    assert E.worst_ratio(bad, V, mag, wl.n_pix) > 1.0
    # one entry conjugated
    bad = V.copy()
    bad[5] += (np.conj(M[5, j]) - M[5, j]) * x[j]
    assert E.worst_ratio(bad, V, mag, wl.n_pix) > 1.0
