"""Seeded workload generators: sizes, determinism and domain."""
import json
import os

import numpy as np

from paper_1310_2078_amd import workloads as W


def test_point_source_record_count_matches_paper(golden_dir):
    """36 dishes sampled 60 times give the paper's 37,800 records: one record
    per antenna pair p < q per sample."""
    g = json.load(open(os.path.join(golden_dir, "point_source_record_count.json")))
    p, q = W.baseline_pairs(g["n_antennas"])
    assert p.shape[0] * g["n_samples"] == g["n_records"]
    assert np.all(p < q)


def test_config1_shapes_and_determinism():
    a, b = W.config1(), W.config1()
    assert a.n_pix == 1024 and a.n_vis == 2000
    for f in ("l", "m", "u", "v", "w", "x_true", "noise"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert np.count_nonzero(a.x_true) == 5
    assert a.x_true.max() <= 2.0 and a.x_true[a.x_true > 0].min() >= 0.5
    assert np.all(a.u ** 2 + a.v ** 2 <= 500.0 ** 2)
    # the phase-centre pixel exists at (N/2, N/2)
    assert a.l[16 + 32 * 16] == 0.0 and a.m[16 + 32 * 16] == 0.0
    assert abs(a.l.min() + 0.05) < 1e-15 and abs(a.l.max() - (0.05 - 0.1 / 32)) < 1e-15


def test_config2_sizes():
    wl = W.config2()
    assert wl.n_pix == 65_536
    assert wl.n_vis == 97_536 == 8128 * 12
    assert np.count_nonzero(wl.x_true) == 200
    nz = wl.x_true[wl.x_true > 0]
    assert nz.min() >= 0.01 and nz.max() <= 5.0
    assert np.all(wl.l ** 2 + wl.m ** 2 < 1)
    # baselines up to the 3 km array diameter, in wavelengths at 150 MHz
    b = np.sqrt(wl.u ** 2 + wl.v ** 2 + wl.w ** 2)
    assert b.max() <= 3000.0 * 1.01 / (W.SPEED_OF_LIGHT / 150e6) + 50


def test_config3_stokes():
    wl = W.config3()
    assert wl.x_true.shape == (4, 1024)
    np.testing.assert_array_equal(wl.x_true[0], W.config1().x_true)
    src = wl.meta["sources"]
    ratio = wl.x_true[1:, src] / wl.x_true[0, src]
    assert np.all(np.abs(ratio) <= 0.1)


def test_config4_sizes():
    wl = W.config4()
    assert wl.n_pix == 1024 ** 2 + 512 ** 2 + 256 ** 2 + 128 ** 2 == 1_392_640
    assert wl.n_vis == 409_600 == 32_640 * 13 - 14_720
    assert np.all(wl.l ** 2 + wl.m ** 2 < 1)
    assert np.count_nonzero(wl.kind == W.PIX_GAUSS_WIDE) == 512 ** 2 + 256 ** 2 + 128 ** 2
    D = wl.meta["delta"]
    assert set(np.unique(np.round(wl.sigma / D, 9))) == {0.0, 2.0, 4.0, 8.0}
    assert np.count_nonzero(wl.x_true) == 1000
    assert wl.extra_flux.shape[0] == 50 * 25 * 25
    np.testing.assert_allclose(wl.extra_flux.sum(), wl.meta["gauss_flux"].sum(), rtol=1e-12)
    assert np.all(np.abs(np.abs(wl.ant_gain) - 1) < 0.3)


def test_config5_requests():
    t = W.config5_arrivals()
    assert t.shape == (256,) and np.all(np.diff(t) > 0)
    assert 30 < t[-1] < 120
    for r in (0, 1, 17, 255):
        wl = W.config5_request(r)
        assert 4096 <= wl.n_pix <= 262144
        assert 10_000 <= wl.n_vis <= 200_000
        assert np.all(np.abs(wl.l) <= 0.05) and np.all(np.abs(wl.m) <= 0.05)
        wl2 = W.config5_request(r)
        np.testing.assert_array_equal(wl.u, wl2.u)
