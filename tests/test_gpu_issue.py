"""Issue rates of the operators' instruction classes (sl1m_issue_rates).

The rates price the operator kernels' instruction mix for the issue-slot
roofline that bench.py reports; here they are checked for plausibility on
the GPU they were measured on: every class positive and finite, FP32 FMA at
most 4 wave64 instructions per clock per compute unit (one per SIMD) at the
2.4 GHz peak clock, and no transcendental faster than an FMA.
"""
import math

import pytest

from paper_1310_2078_amd import sl1m

pytestmark = pytest.mark.gpu


def test_issue_rates_plausible():
    r = sl1m.issue_rates("cuda")
    print(f"[case] issue rates (wave64 instr/s/CU): {r}", flush=True)
    for k, v in r.items():
        assert math.isfinite(v) and v > 0.0, k
    assert r["fp32_fma"] <= 4 * 2.4e9 * 1.01
    assert r["sin_cos"] <= r["fp32_fma"] * 1.05 and r["exp"] <= r["fp32_fma"] * 1.05
    print(f"    per clock at 2.4 GHz: fp32 {r['fp32_fma'] / 2.4e9:.3f} "
          f"fp64 {r['fp64_fma'] / 2.4e9:.3f} sin/cos {r['sin_cos'] / 2.4e9:.3f} "
          f"exp {r['exp'] / 2.4e9:.3f}", flush=True)
