"""Python binding of libsl1m.so (the C ABI declared in include/sl1m.h).

Argument marshalling only: every step of the operator and the solver runs in
the library's HIP kernels.  PyTorch provides device memory and streams.  If
the library has not been built the binding raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsl1m.so")

OK, EINVAL, EDOMAIN, ENOMEM, EHIP, EDIVERGED, ECANCELLED = 0, -1, -2, -3, -4, -5, -6
PIX_DELTA, PIX_GAUSS_PARAXIAL, PIX_GAUSS_WIDE = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_MFMA_F16, PREC_MFMA_BF16, PREC_FP32_HILO = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "mfma_f16": PREC_MFMA_F16,
              "mfma_bf16": PREC_MFMA_BF16, "fp32_hilo": PREC_FP32_HILO}

_lib = None


class SL1MError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sl1m status {status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("n_pix", ctypes.c_int64),
        ("l", ctypes.c_void_p),
        ("m", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p),
        ("kind", ctypes.c_void_p),
        ("n_vis", ctypes.c_int64),
        ("u", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("ant_p", ctypes.c_void_p),
        ("ant_q", ctypes.c_void_p),
        ("n_ant", ctypes.c_int32),
        ("ant_gain", ctypes.c_void_p),
        ("ant_fwhm", ctypes.c_void_p),
        ("precision", ctypes.c_int32),
        ("max_rhs", ctypes.c_int32),
        ("tile_blocks", ctypes.c_int32),
        ("grid_mode", ctypes.c_int32),
        ("fwd_vpl", ctypes.c_int32),
        ("adj_ppl", ctypes.c_int32),
    ]


class Timing(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 8), ("total_ms", ctypes.c_double * 8)]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int64),
        ("completed_rounds", ctypes.c_int64),
        ("evals_scheduled", ctypes.c_double),
        ("arena_bytes", ctypes.c_uint64),
        ("arena_used", ctypes.c_uint64),
        ("active", ctypes.c_int32),
        ("pending", ctypes.c_int32),
    ]


class SolveParams(ctypes.Structure):
    _fields_ = [
        ("lam", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("L", ctypes.c_double),
        ("L_safety", ctypes.c_double),
        ("power_iters", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("nnz_eps", ctypes.c_double),
    ]


class FistaState(ctypes.Structure):
    _fields_ = [
        ("img", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("t", ctypes.c_double),
        ("k", ctypes.c_int64),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("L", ctypes.c_double),
        ("F", ctypes.c_double),
        ("l2_term", ctypes.c_double),
        ("l1_term", ctypes.c_double),
        ("nnz", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


def lib() -> ctypes.CDLL:
    """Load libsl1m.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_double)
        L.sl1m_plan_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)]
        L.sl1m_plan_create.argtypes = [ctypes.POINTER(Problem), vp, ctypes.c_size_t, vp,
                                       ctypes.POINTER(vp)]
        L.sl1m_plan_destroy.argtypes = [vp]
        L.sl1m_forward.argtypes = [vp, vp, vp, vp]
        L.sl1m_adjoint.argtypes = [vp, vp, vp, vp]
        L.sl1m_forward_multi.argtypes = [vp, i32, vp, vp, vp]
        L.sl1m_adjoint_multi.argtypes = [vp, i32, vp, vp, vp]
        L.sl1m_estimate_L.argtypes = [vp, i32, u64, vp, ctypes.POINTER(dbl), vp]
        L.sl1m_solve.argtypes = [vp, vp, ctypes.POINTER(SolveParams), vp, ctypes.POINTER(SolveInfo), vp]
        L.sl1m_solve_from.argtypes = [vp, vp, vp, ctypes.POINTER(SolveParams), vp,
                                      ctypes.POINTER(SolveInfo), vp]
        L.sl1m_dirty_image.argtypes = [vp, vp, vp, vp]
        L.sl1m_solve_resume.argtypes = [vp, vp, ctypes.POINTER(FistaState),
                                        ctypes.POINTER(SolveParams), vp,
                                        ctypes.POINTER(SolveInfo), vp]
        L.sl1m_server_create.argtypes = [vp, ctypes.c_size_t, i32, dbl, ctypes.POINTER(vp)]
        L.sl1m_server_submit.argtypes = [vp, ctypes.POINTER(Problem), vp,
                                         ctypes.POINTER(SolveParams), vp,
                                         ctypes.POINTER(ctypes.c_uint64)]
        L.sl1m_server_step.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.sl1m_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(SolveInfo),
                                       ctypes.POINTER(i32), ctypes.POINTER(dbl)]
        L.sl1m_server_cancel.argtypes = [vp, ctypes.c_uint64]
        L.sl1m_server_set_policy.argtypes = [vp, i32]
        L.sl1m_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.sl1m_server_destroy.argtypes = [vp]
        L.sl1m_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.sl1m_tune_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)]
        L.sl1m_tune.argtypes = [ctypes.POINTER(Problem), vp, ctypes.c_size_t, i32, vp,
                                ctypes.POINTER(Tuning)]
        L.sl1m_timing_begin.argtypes = [vp, i32]
        L.sl1m_timing_end.argtypes = [vp, ctypes.POINTER(Timing)]
        L.sl1m_issue_scratch_bytes.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
        L.sl1m_issue_rates.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(dbl), vp]
        L.sl1m_last_error.restype = ctypes.c_char_p
        L.sl1m_version.restype = ctypes.c_char_p
        for name in ("sl1m_plan_workspace_bytes", "sl1m_plan_create", "sl1m_plan_destroy",
                     "sl1m_forward", "sl1m_adjoint", "sl1m_forward_multi",
                     "sl1m_adjoint_multi", "sl1m_estimate_L", "sl1m_solve",
                     "sl1m_solve_from", "sl1m_solve_resume", "sl1m_dirty_image",
                     "sl1m_timing_begin", "sl1m_timing_end", "sl1m_plan_query",
                     "sl1m_tune_workspace_bytes", "sl1m_tune",
                     "sl1m_server_create",
                     "sl1m_server_submit", "sl1m_server_step", "sl1m_server_poll",
                     "sl1m_server_cancel", "sl1m_server_stats", "sl1m_server_destroy",
                     "sl1m_server_set_policy", "sl1m_issue_scratch_bytes", "sl1m_issue_rates"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise SL1MError(status, lib().sl1m_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def issue_rates(device="cuda", stream=None) -> dict:
    """Wave64 instructions per second per compute unit of the instruction
    classes the operators are made of (sl1m_issue_rates)."""
    L = lib()
    nb = ctypes.c_size_t()
    _check(L.sl1m_issue_scratch_bytes(ctypes.byref(nb)))
    buf = torch.empty(max(1, nb.value // 4), dtype=torch.float32, device=torch.device(device))
    r = (ctypes.c_double * 4)()
    _check(L.sl1m_issue_rates(ctypes.c_void_p(buf.data_ptr()), nb, r, _stream(stream)))
    return {"fp32_fma": r[0], "fp64_fma": r[1], "sin_cos": r[2], "exp": r[3]}


def _dev(a, dtype, device):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


GRID_AUTO, GRID_OFF, GRID_REQUIRE = 0, 1, 2
METHODS = {"fista": 0, "mfista": 1}
_GRID = {"auto": GRID_AUTO, "off": GRID_OFF, "require": GRID_REQUIRE}


class Tuning(ctypes.Structure):
    _fields_ = [
        ("tile_blocks", ctypes.c_int32), ("grid_mode", ctypes.c_int32),
        ("fwd_vpl", ctypes.c_int32), ("adj_ppl", ctypes.c_int32),
        ("forward_ms", ctypes.c_double), ("adjoint_ms", ctypes.c_double),
        ("default_forward_ms", ctypes.c_double), ("default_adjoint_ms", ctypes.c_double),
        ("candidates", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}
        d["grid"] = {v: k for k, v in _GRID.items()}[d["grid_mode"]]
        return d


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_pix", ctypes.c_int64), ("n_vis", ctypes.c_int64),
        ("precision", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
        ("grid", ctypes.c_int32), ("grid_abs_l", ctypes.c_int32),
        ("grid_abs_m", ctypes.c_int32), ("n_layers", ctypes.c_int32),
        ("grid_positions", ctypes.c_int64),
        ("fwd_vpl", ctypes.c_int32), ("adj_ppl", ctypes.c_int32),
        ("n_fchunks", ctypes.c_int32), ("n_fchunks_grid", ctypes.c_int32),
        ("n_achunks", ctypes.c_int32), ("grid_pairs", ctypes.c_int32),
        ("grid_multi", ctypes.c_int32), ("grid_mfma", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Plan:
    """A planned SL1M operator on one GPU.

    Inputs are NumPy arrays or torch tensors; they are copied to the device
    and kept alive with the plan.  ``precision`` is "fp32" (FP64 phase,
    FP32 sincos/accumulation), "fp64", "mfma_f16" / "mfma_bf16" (the FP32
    entries and the images or residuals rounded to float16 / bfloat16 and
    contracted on the matrix cores; delta pixels only), or "fp32_hilo" (the
    phase in float32 hi/lo arithmetic instead of FP64; delta pixels only).
    """

    def __init__(self, l, m, u, v, w, sigma=None, kind=None, ant_p=None, ant_q=None,
                 ant_gain=None, ant_fwhm=None, precision: str = "fp32", device="cuda",
                 stream=None, max_rhs: int = 1, tile_blocks: int = 0, grid: str = "auto",
                 fwd_vpl: int = 0, adj_ppl: int = 0):
        self.device = torch.device(device)
        self.precision = PRECISIONS[precision]
        self.rdtype = torch.float64 if self.precision == PREC_FP64 else torch.float32
        self.cdtype = torch.complex128 if self.precision == PREC_FP64 else torch.complex64
        d = self.device
        self._keep = dict(
            l=_dev(l, torch.float64, d), m=_dev(m, torch.float64, d),
            u=_dev(u, torch.float64, d), v=_dev(v, torch.float64, d), w=_dev(w, torch.float64, d),
            sigma=_dev(sigma, torch.float64, d), kind=_dev(kind, torch.uint8, d),
            ant_p=_dev(ant_p, torch.int32, d), ant_q=_dev(ant_q, torch.int32, d),
            ant_fwhm=_dev(ant_fwhm, torch.float64, d))
        if ant_gain is not None:
            g = np.asarray(ant_gain.cpu() if isinstance(ant_gain, torch.Tensor) else ant_gain,
                           np.complex128)
            self._keep["ant_gain"] = torch.as_tensor(np.stack([g.real, g.imag], 1).ravel(),
                                                     dtype=torch.float64, device=d)
            n_ant = g.shape[0]
        else:
            self._keep["ant_gain"] = None
            n_ant = 0
        if ant_p is not None and n_ant == 0:
            n_ant = int(max(int(np.max(np.asarray(ant_p))), int(np.max(np.asarray(ant_q))))) + 1
        if ant_fwhm is not None:
            n_ant = max(n_ant, int(np.asarray(ant_fwhm).shape[0]))
        k = self._keep
        self.n_pix = int(k["l"].shape[0])
        self.n_vis = int(k["u"].shape[0])
        self._prob = Problem(
            n_pix=self.n_pix, l=_ptr(k["l"]), m=_ptr(k["m"]), sigma=_ptr(k["sigma"]),
            kind=_ptr(k["kind"]), n_vis=self.n_vis, u=_ptr(k["u"]), v=_ptr(k["v"]),
            w=_ptr(k["w"]), ant_p=_ptr(k["ant_p"]), ant_q=_ptr(k["ant_q"]), n_ant=n_ant,
            ant_gain=_ptr(k["ant_gain"]), ant_fwhm=_ptr(k["ant_fwhm"]),
            precision=self.precision, max_rhs=int(max_rhs), tile_blocks=int(tile_blocks),
            grid_mode=_GRID[grid], fwd_vpl=int(fwd_vpl), adj_ppl=int(adj_ppl))
        self.max_rhs = int(max_rhs)
        nbytes = ctypes.c_size_t(0)
        _check(lib().sl1m_plan_workspace_bytes(ctypes.byref(self._prob), ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self._ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=d)
        h = ctypes.c_void_p()
        _check(lib().sl1m_plan_create(ctypes.byref(self._prob), _ptr(self._ws),
                                      ctypes.c_size_t(self._ws.numel()), _stream(stream),
                                      ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, wl, precision="fp32", device="cuda", with_kinds=True, max_rhs=1,
                      tile_blocks=0, grid="auto", tuning=None, fwd_vpl=0, adj_ppl=0):
        """Plan of a workload; `tuning` (a dict from Plan.tune) sets the split,
        the evaluation and the lane counts."""
        if tuning is not None:
            tile_blocks = tuning["tile_blocks"]
            grid = tuning["grid"]
            kw_lanes = dict(fwd_vpl=tuning["fwd_vpl"], adj_ppl=tuning["adj_ppl"])
        else:
            kw_lanes = dict(fwd_vpl=fwd_vpl, adj_ppl=adj_ppl)
        kw = {}
        if with_kinds and (np.any(wl.kind != 0) or np.any(wl.sigma != 0)):
            kw = dict(sigma=wl.sigma, kind=wl.kind)
        return cls(wl.l, wl.m, wl.u, wl.v, wl.w, ant_p=wl.ant_p, ant_q=wl.ant_q,
                   ant_gain=wl.ant_gain, ant_fwhm=wl.ant_fwhm, precision=precision,
                   device=device, max_rhs=max_rhs, tile_blocks=tile_blocks, grid=grid,
                   **kw_lanes, **kw)

    def tune(self, reps: int = 3, stream=None) -> dict:
        """Times candidate launch shapes of this plan's problem (sl1m_tune) in a
        scratch workspace and returns the fastest; pass it to
        Plan.from_workload(..., tuning=...)."""
        nbytes = ctypes.c_size_t(0)
        _check(lib().sl1m_tune_workspace_bytes(ctypes.byref(self._prob), ctypes.byref(nbytes)))
        ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        t = Tuning()
        _check(lib().sl1m_tune(ctypes.byref(self._prob), _ptr(ws), ctypes.c_size_t(ws.numel()),
                               int(reps), _stream(stream), ctypes.byref(t)))
        return t.as_dict()

    def info(self) -> dict:
        """The plan's decisions (sl1m_plan_query): grid evaluation, splits."""
        r = PlanInfo()
        _check(lib().sl1m_plan_query(self._h, ctypes.byref(r)))
        return r.as_dict()

    # -- operator -----------------------------------------------------------
    def forward(self, x, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        x = _dev(x, self.rdtype, self.device)
        if out is None:
            out = torch.empty(self.n_vis, dtype=self.cdtype, device=self.device)
        _check(lib().sl1m_forward(self._h, _ptr(x), _ptr(out), _stream(stream)))
        return out

    def adjoint(self, r, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        r = _dev(r, self.cdtype, self.device)
        if out is None:
            out = torch.empty(self.n_pix, dtype=self.rdtype, device=self.device)
        _check(lib().sl1m_adjoint(self._h, _ptr(r), _ptr(out), _stream(stream)))
        return out

    def forward_multi(self, x, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """x: real [R][n_pix] -> complex [R][n_vis]."""
        x = _dev(x, self.rdtype, self.device)
        R = int(x.shape[0])
        if out is None:
            out = torch.empty((R, self.n_vis), dtype=self.cdtype, device=self.device)
        _check(lib().sl1m_forward_multi(self._h, R, _ptr(x), _ptr(out), _stream(stream)))
        return out

    def adjoint_multi(self, r, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """r: complex [R][n_vis] -> real [R][n_pix]."""
        r = _dev(r, self.cdtype, self.device)
        R = int(r.shape[0])
        if out is None:
            out = torch.empty((R, self.n_pix), dtype=self.rdtype, device=self.device)
        _check(lib().sl1m_adjoint_multi(self._h, R, _ptr(r), _ptr(out), _stream(stream)))
        return out

    def estimate_L(self, iters: int = 30, seed: int = 0, x0=None, stream=None) -> float:
        rq = ctypes.c_double(0.0)
        x0t = _dev(x0, self.rdtype, self.device)
        _check(lib().sl1m_estimate_L(self._h, int(iters), ctypes.c_uint64(seed), _ptr(x0t),
                                     ctypes.byref(rq), _stream(stream)))
        return float(rq.value)

    def solve(self, vis, lam: float, max_iter: int, L: float = 0.0, eps: float = 0.0,
              check_every: int = 1, power_iters: int = 30, seed: int = 0,
              L_safety: float = 1.01, out: Optional[torch.Tensor] = None, stream=None,
              x0=None, method: str = "fista", nnz_eps: float = 0.0):
        """FISTA solve (sl1m_solve); with x0 (real [n_pix]) the warm start
        sl1m_solve_from, e.g. from dirty_image() or an upscaled coarser
        solution; method "mfista" runs the monotone variant.  eps / nnz_eps
        stop on a small relative change of the objective / of the non-zero
        count between checks every check_every iterations."""
        vis = _dev(vis, self.cdtype, self.device)
        if out is None:
            out = torch.empty(self.n_pix, dtype=self.rdtype, device=self.device)
        prm = SolveParams(lam=float(lam), eps=float(eps), max_iter=int(max_iter),
                          check_every=int(check_every), L=float(L), L_safety=float(L_safety),
                          power_iters=int(power_iters), method=METHODS[method],
                          seed=ctypes.c_uint64(seed), nnz_eps=float(nnz_eps))
        info = SolveInfo()
        if x0 is None:
            _check(lib().sl1m_solve(self._h, _ptr(vis), ctypes.byref(prm), _ptr(out),
                                    ctypes.byref(info), _stream(stream)))
        else:
            x0 = _dev(x0, self.rdtype, self.device)
            _check(lib().sl1m_solve_from(self._h, _ptr(vis), _ptr(x0), ctypes.byref(prm),
                                         _ptr(out), ctypes.byref(info), _stream(stream)))
        return out, info.as_dict()

    def solve_resume(self, vis, lam: float, max_iter: int, L: float, state=None,
                     out: Optional[torch.Tensor] = None, stream=None):
        """Checkpointed FISTA (sl1m_solve_resume): runs max_iter iterations
        from `state` (None: a fresh start from a zero image) and returns
        (image, info, state); state = {"img", "y" (device tensors, caller
        order), "t", "k"} is the iteration state after the last iteration."""
        vis = _dev(vis, self.cdtype, self.device)
        if out is None:
            out = torch.empty(self.n_pix, dtype=self.rdtype, device=self.device)
        if state is None:
            state = {"img": torch.zeros(self.n_pix, dtype=self.rdtype, device=self.device),
                     "y": torch.zeros(self.n_pix, dtype=self.rdtype, device=self.device),
                     "t": 0.0, "k": 0}
        else:
            state = {"img": state["img"].clone(), "y": state["y"].clone(), "t": state["t"],
                     "k": state["k"]}
        st = FistaState(img=_ptr(state["img"]), y=_ptr(state["y"]), t=float(state["t"]),
                        k=int(state["k"]))
        prm = SolveParams(lam=float(lam), eps=0.0, max_iter=int(max_iter), check_every=1,
                          L=float(L), L_safety=1.01, power_iters=30, method=0,
                          seed=ctypes.c_uint64(0), nnz_eps=0.0)
        info = SolveInfo()
        _check(lib().sl1m_solve_resume(self._h, _ptr(vis), ctypes.byref(st), ctypes.byref(prm),
                                       _ptr(out), ctypes.byref(info), _stream(stream)))
        state["t"], state["k"] = float(st.t), int(st.k)
        return out, info.as_dict(), state

    def dirty_image(self, vis, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """max(0, Re(M^H V) / n_vis) in the caller's pixel order (sl1m_dirty_image)."""
        vis = _dev(vis, self.cdtype, self.device)
        if out is None:
            out = torch.empty(self.n_pix, dtype=self.rdtype, device=self.device)
        _check(lib().sl1m_dirty_image(self._h, _ptr(vis), _ptr(out), _stream(stream)))
        return out

    def timing_begin(self, max_launches: int = 4096):
        _check(lib().sl1m_timing_begin(self._h, int(max_launches)))

    def timing_end(self):
        """Returns {kind: (launches, total_ms)} for the forward and adjoint
        operator kernels, the FISTA update and the grid kernels by launch."""
        t = Timing()
        _check(lib().sl1m_timing_end(self._h, ctypes.byref(t)))
        names = ("forward", "adjoint", "fista", "grid_fwd_delta", "grid_adj_delta",
                 "grid_fwd_gauss", "grid_adj_gauss")
        return {n: (int(t.launches[i]), float(t.total_ms[i])) for i, n in enumerate(names)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sl1m_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return lib().sl1m_version().decode()


class Server:
    """Continuous-batching server (sl1m_server_*): many FP32 solves share one
    GPU.  The arena is a torch uint8 tensor owned by this object; submitted
    requests keep their device inputs and output alive until done."""

    POLICIES = {"fair": 0, "oldest": 1}

    def __init__(self, arena_bytes: int, max_slots: int = 32, round_budget: float = 3e10,
                 device="cuda", policy: str = "oldest"):
        self.device = torch.device(device)
        self._arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(lib().sl1m_server_create(_ptr(self._arena), ctypes.c_size_t(self._arena.numel()),
                                        int(max_slots), float(round_budget), ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self.set_policy(policy)

    def set_policy(self, policy: str):
        """"fair" (equal round shares) or "oldest" (oldest request first)."""
        _check(lib().sl1m_server_set_policy(self._h, self.POLICIES[policy]))

    def submit(self, wl, vis, lam: float, max_iter: int, L: float = 0.0,
               power_iters: int = 30, seed: int = 0, L_safety: float = 1.01,
               grid: str = "auto", tile_blocks: int = 0) -> int:
        """wl: a workload-like object (l, m, u, v, w, sigma, kind, gains);
        vis: complex data [n_vis] (device tensor or array).  grid: "auto"
        lets a request whose pixels form one grid segment use the grid
        evaluation; "off" evaluates every entry directly.  tile_blocks: the
        request's operator split target (0: the server's default)."""
        d = self.device
        keep = dict(
            l=_dev(wl.l, torch.float64, d), m=_dev(wl.m, torch.float64, d),
            u=_dev(wl.u, torch.float64, d), v=_dev(wl.v, torch.float64, d),
            w=_dev(wl.w, torch.float64, d))
        has_kind = wl.kind is not None and (np.any(np.asarray(wl.kind) != 0) or
                                            np.any(np.asarray(wl.sigma) != 0))
        keep["sigma"] = _dev(wl.sigma, torch.float64, d) if has_kind else None
        keep["kind"] = _dev(wl.kind, torch.uint8, d) if has_kind else None
        n_ant = 0
        keep["ant_p"] = _dev(getattr(wl, "ant_p", None), torch.int32, d)
        keep["ant_q"] = _dev(getattr(wl, "ant_q", None), torch.int32, d)
        keep["ant_fwhm"] = _dev(getattr(wl, "ant_fwhm", None), torch.float64, d)
        g = getattr(wl, "ant_gain", None)
        if g is not None:
            g = np.asarray(g, np.complex128)
            keep["ant_gain"] = torch.as_tensor(np.stack([g.real, g.imag], 1).ravel(),
                                               dtype=torch.float64, device=d)
            n_ant = g.shape[0]
        else:
            keep["ant_gain"] = None
        if keep["ant_fwhm"] is not None:
            n_ant = max(n_ant, int(keep["ant_fwhm"].shape[0]))
        if keep["ant_p"] is not None and n_ant == 0:
            n_ant = int(max(int(keep["ant_p"].max()), int(keep["ant_q"].max()))) + 1
        keep["vis"] = _dev(vis, torch.complex64, d)
        n_pix, n_vis = int(keep["l"].shape[0]), int(keep["u"].shape[0])
        keep["out"] = torch.zeros(n_pix, dtype=torch.float32, device=d)
        prob = Problem(n_pix=n_pix, l=_ptr(keep["l"]), m=_ptr(keep["m"]),
                       sigma=_ptr(keep["sigma"]), kind=_ptr(keep["kind"]), n_vis=n_vis,
                       u=_ptr(keep["u"]), v=_ptr(keep["v"]), w=_ptr(keep["w"]),
                       ant_p=_ptr(keep["ant_p"]), ant_q=_ptr(keep["ant_q"]), n_ant=n_ant,
                       ant_gain=_ptr(keep["ant_gain"]), ant_fwhm=_ptr(keep["ant_fwhm"]),
                       precision=PREC_FP32, max_rhs=1, tile_blocks=int(tile_blocks),
                       grid_mode=_GRID[grid])
        prm = SolveParams(lam=float(lam), eps=0.0, max_iter=int(max_iter), check_every=1,
                          L=float(L), L_safety=float(L_safety), power_iters=int(power_iters),
                          method=0, seed=ctypes.c_uint64(seed), nnz_eps=0.0)
        t = ctypes.c_uint64(0)
        torch.cuda.current_stream(d).synchronize()   # inputs written before the server reads them
        _check(lib().sl1m_server_submit(self._h, ctypes.byref(prob), _ptr(keep["vis"]),
                                        ctypes.byref(prm), _ptr(keep["out"]), ctypes.byref(t)))
        self._keep[int(t.value)] = keep
        return int(t.value)

    def step(self):
        a, p = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().sl1m_server_step(self._h, ctypes.byref(a), ctypes.byref(p)))
        return a.value, p.value

    def poll(self, ticket: int):
        info = SolveInfo()
        done = ctypes.c_int32(0)
        times = (ctypes.c_double * 3)()
        _check(lib().sl1m_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(info),
                                      ctypes.byref(done), times))
        return bool(done.value), info.as_dict(), tuple(times)

    def result(self, ticket: int) -> torch.Tensor:
        return self._keep[ticket]["out"]

    def release(self, ticket: int):
        """Drop the references kept for a finished request."""
        self._keep.pop(ticket, None)

    def cancel(self, ticket: int):
        _check(lib().sl1m_server_cancel(self._h, ctypes.c_uint64(ticket)))

    def stats(self):
        s = ServerStats()
        _check(lib().sl1m_server_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def drain(self, tickets, max_steps: int = 10_000_000):
        """Step until every ticket is done."""
        left = set(tickets)
        for _ in range(max_steps):
            self.step()
            left = {t for t in left if not self.poll(t)[0]}
            if not left:
                return
        raise RuntimeError("server did not finish")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sl1m_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
