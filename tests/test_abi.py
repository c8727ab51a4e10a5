"""The C-ABI library loads and exports every symbol that include/sl1m.h
declares; host-only argument checks behave as documented.  No GPU calls."""
import ctypes
import os
import re

import pytest

from paper_1310_2078_amd import sl1m

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sl1m.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sl1m_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sl1m.LIB_PATH):
        pytest.fail("libsl1m.so is not built: run __graft_entry__.build()")
    return sl1m.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert {"sl1m_forward", "sl1m_adjoint", "sl1m_solve", "sl1m_plan_create"} <= set(names)
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/sl1m.h but not exported"


def test_library_reports_version(L):
    assert "gfx950" in sl1m.version()


def test_host_argument_checks(L):
    nbytes = ctypes.c_size_t(0)
    assert L.sl1m_plan_workspace_bytes(None, ctypes.byref(nbytes)) == sl1m.EINVAL
    pr = sl1m.Problem(n_pix=-1, n_vis=10, precision=sl1m.PREC_FP32)
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert b"negative" in L.sl1m_last_error()
    pr = sl1m.Problem(n_pix=10, n_vis=10, precision=7)
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    fake = ctypes.c_void_p(0x1000)
    pr = sl1m.Problem(n_pix=10, l=fake, m=fake, n_vis=10, u=fake, v=fake, w=fake,
                      precision=sl1m.PREC_FP32, max_rhs=3)
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert b"max_rhs" in L.sl1m_last_error()
    pr = sl1m.Problem(n_pix=10, l=fake, m=fake, n_vis=10, u=fake, v=fake, w=fake,
                      precision=sl1m.PREC_FP32, grid_mode=3)
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert b"grid_mode" in L.sl1m_last_error()
    assert L.sl1m_plan_query(None, None) == sl1m.EINVAL
    pr = sl1m.Problem(n_pix=10, l=fake, m=fake, n_vis=10, u=fake, v=fake, w=fake,
                      precision=sl1m.PREC_FP32, grid_mode=sl1m.GRID_OFF, fwd_vpl=3)
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert b"fwd_vpl" in L.sl1m_last_error()
    assert L.sl1m_tune(None, None, 0, 1, None, None) == sl1m.EINVAL
    pr = sl1m.Problem(n_pix=10, n_vis=10, precision=sl1m.PREC_FP32)   # NULL l, m
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert L.sl1m_forward(None, None, None, None) == sl1m.EINVAL
    assert L.sl1m_solve(None, None, None, None, None, None) == sl1m.EINVAL


def test_workspace_size_grows_with_problem(L):
    """Workspace sizing is host arithmetic on the sizes (delta pixels, no
    kinds or antenna arrays, grid evaluation off, so no device access)."""
    fake = ctypes.c_void_p(0x1000)

    def size(n_pix, n_vis, prec=sl1m.PREC_FP32):
        pr = sl1m.Problem(n_pix=n_pix, l=fake, m=fake, n_vis=n_vis, u=fake, v=fake, w=fake,
                          precision=prec, grid_mode=sl1m.GRID_OFF)
        b = ctypes.c_size_t(0)
        assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(b)) == 0
        return b.value

    a = size(1024, 2000)
    b = size(65536, 97536)
    assert 0 < a < b
    assert size(1024, 2000, sl1m.PREC_FP64) > a
    assert size(0, 0) > 0          # empty problems are legal
    assert b < 2 ** 30             # config-2 workspace stays far below HBM
    fake = ctypes.c_void_p(0x1000)
    pr4 = sl1m.Problem(n_pix=65536, l=fake, m=fake, n_vis=97536, u=fake, v=fake, w=fake,
                       precision=sl1m.PREC_FP32, max_rhs=4, grid_mode=sl1m.GRID_OFF)
    b4 = ctypes.c_size_t(0)
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr4), ctypes.byref(b4)) == 0
    assert b4.value > b


def test_matrix_core_workspace_and_issue_rate_checks(L):
    """Matrix-core plans size extra packed-operand buffers (host arithmetic:
    delta pixels, no kinds or antennas); the issue-rate entry points reject
    NULL arguments before touching the device."""
    fake = ctypes.c_void_p(0x1000)

    def size(prec, max_rhs, n_pix=65536, n_vis=97536):
        pr = sl1m.Problem(n_pix=n_pix, l=fake, m=fake, n_vis=n_vis, u=fake, v=fake, w=fake,
                          precision=prec, grid_mode=sl1m.GRID_OFF, max_rhs=max_rhs)
        b = ctypes.c_size_t(0)
        assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(b)) == 0
        return b.value

    for prec in (sl1m.PREC_MFMA_F16, sl1m.PREC_MFMA_BF16):
        assert size(prec, 4) > 0
        # eight sides pack two groups of four: at least 16 B more per pixel
        # (images) and 32 B more per visibility (residual records)
        assert size(prec, 8) - size(prec, 4) >= 16 * 65536 + 32 * 97536
    # ragged sizes pad to multiples of 32 without failing
    assert size(sl1m.PREC_MFMA_F16, 1, n_pix=1000, n_vis=1999) > 0
    nbytes = ctypes.c_size_t(0)
    assert L.sl1m_issue_scratch_bytes(None) == sl1m.EINVAL
    assert L.sl1m_issue_rates(None, 0, None, None) == sl1m.EINVAL
    pr = sl1m.Problem(n_pix=10, l=fake, m=fake, n_vis=10, u=fake, v=fake, w=fake,
                      precision=sl1m.PREC_FP32_HILO + 1)
    assert L.sl1m_plan_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert b"precision" in L.sl1m_last_error()
    pr = sl1m.Problem(n_pix=10, l=fake, m=fake, n_vis=10, u=fake, v=fake, w=fake,
                      precision=sl1m.PREC_FP32_HILO)
    assert L.sl1m_tune_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert b"hi/lo" in L.sl1m_last_error()
    pr = sl1m.Problem(n_pix=10, l=fake, m=fake, n_vis=10, u=fake, v=fake, w=fake,
                      precision=sl1m.PREC_MFMA_F16)
    assert L.sl1m_tune_workspace_bytes(ctypes.byref(pr), ctypes.byref(nbytes)) == sl1m.EINVAL
    assert b"MFMA" in L.sl1m_last_error()
