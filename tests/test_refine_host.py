"""Host logic of the quad-tree refinement driver (paper_1310_2078_amd.refine)
against the oracle's refinement (oracle.quadtree), written independently:
the same level-0 cells, pixel model and refinement decisions, cell order and
start values, on random images (no GPU needed)."""
import numpy as np
import pytest

import oracle as O
from paper_1310_2078_amd import refine as R


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_split_and_pixel_model_match_oracle(seed):
    rng = np.random.default_rng(seed)
    half, n0 = 0.1, 8
    h_min = 2 * half / n0 / 8
    l, m, h = R.first_cells(n0, half)
    ol, om, oh = O.quadtree.level0_cells(n0, half)
    assert np.array_equal(l, ol) and np.array_equal(m, om) and np.array_equal(h, oh)
    for _ in range(4):
        img = np.where(rng.random(l.size) < 0.4, rng.uniform(0, 1, l.size), 0.0)
        img[rng.integers(l.size)] = 0.01 * img.max()   # exactly at the threshold: kept
        mine = R.split_cells(l, m, h, img, 0.01, h_min)
        ref = O.quadtree.refine(l, m, h, img, 0.01, h_min)
        for a, b in zip(mine, ref):
            assert np.array_equal(a, b)
        s1, k1 = R.pixel_model(mine[2], h_min)
        s2, k2 = O.quadtree.cell_pixels(ref[2], h_min)
        assert np.array_equal(s1, s2) and np.array_equal(k1, k2)
        l, m, h = mine[0], mine[1], mine[2]
