"""sl1m_forward_noalloc (the forward operator for callers that cannot
allocate device memory) against sl1m_forward on a plan in caller-allocated
memory, through the C ABI: two calls in a row, the second with a smaller
problem, each bitwise equal to the plan's forward and within the FP32
operator bar (1e-5 norm-relative) of the FP64 oracle; a problem whose plan
workspace exceeds the scratch is refused."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_2078_amd import sl1m
from paper_1310_2078_amd import workloads as W

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20   # SL1M_NOALLOC_SCRATCH_BYTES


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc_forward(plan, x):
    """Calls sl1m_forward_noalloc with the plan's own problem struct (its
    device arrays), so both paths see the same inputs."""
    L = sl1m.lib()
    L.sl1m_forward_noalloc.argtypes = [ctypes.POINTER(sl1m.Problem), ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]
    L.sl1m_forward_noalloc.restype = ctypes.c_int
    xd = torch.as_tensor(np.asarray(x), dtype=torch.float32, device=plan.device)
    out = torch.full((plan.n_vis,), float("nan"), dtype=torch.complex64, device=plan.device)
    st = L.sl1m_forward_noalloc(ctypes.byref(plan._prob), ctypes.c_void_p(xd.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out


@pytest.mark.parametrize("first,second", [
    ((2537, 3001, W.PIX_GAUSS_WIDE, 2e-3, True), (1100, 900, W.PIX_DELTA, 0.0, False)),
    ((4096, 6000, W.PIX_DELTA, 0.0, True), (777, 1234, W.PIX_GAUSS_PARAXIAL, 3e-3, True)),
])
def test_noalloc_forward_matches_plan_forward(first, second):
    for i, (n_pix, n_vis, kind, sigma, gains) in enumerate((first, second)):
        say(f"[case] noalloc call {i} n_pix={n_pix} n_vis={n_vis} kind={kind} gains={gains}")
        wl = W.small_random(30 + i, n_pix, n_vis, kind=kind, sigma=sigma, with_gains=gains,
                            uv_radius=1200.0, w_sigma=300.0)
        plan = sl1m.Plan.from_workload(wl)
        assert plan.workspace_bytes <= SCRATCH_BYTES
        x = np.random.default_rng(40 + i).standard_normal(wl.n_pix)
        ref = plan.forward(x).cpu().numpy()
        st, out = _noalloc_forward(plan, x)
        assert st == sl1m.OK, sl1m.lib().sl1m_last_error().decode()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref)
        Vo = O.forward(O.Problem.from_workload(wl), x)
        err = float(np.linalg.norm(got - Vo) / np.linalg.norm(Vo))
        say(f"    bitwise equal to sl1m_forward; oracle rel err {err:.2e}")
        assert err <= 1e-5
        plan.close()


def test_noalloc_refuses_a_problem_beyond_the_scratch():
    say("[case] noalloc refuses an oversized plan workspace")
    wl = W.config2()
    plan = sl1m.Plan.from_workload(wl)
    assert plan.workspace_bytes > SCRATCH_BYTES
    st, _ = _noalloc_forward(plan, np.zeros(wl.n_pix))
    assert st == sl1m.ENOMEM
    assert "sl1m_forward_noalloc holds at most" in sl1m.lib().sl1m_last_error().decode()
    plan.close()
