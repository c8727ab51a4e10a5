"""FP64 CPU oracle for SL1M: measurement operator, adjoint, step size and FISTA.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite,
the package's smoke check and the benchmark's CPU-baseline leg may import
it; the GPU library never calls it and shares no code with it.

Everything is float64 / complex128 NumPy, evaluated entry by entry from the
paper's closed forms (Hardy 2013, "Direct deconvolution of radio synthesis
images using L1 minimisation"):

* delta pixels             -- eq. (deltam), Section "Delta function pixels"
* paraxial Gaussian pixels -- eq. (samlm4), Section "Gaussian pixels in the
                              paraxial approximation", written as printed
                              (three complex exponentials over 1 - i w sigma^2)
* wide-field Gaussian      -- eq. (samlm5), Section "Gaussian pixels in a
                              wide field"
* FISTA with the positive threshold -- Section "Implementation of SL1M",
                              the printed algorithm and eq. (threshp)

Readings taken where the paper is garbled, silent or at odds with itself:

* R1 (eq. samlm4/samlm5 prefactor): the pixel shape eq. (gaus) already has
  unit integral, so the integral over it yields 1/(1 - i w sigma^2); the extra
  1/sigma^2 printed in front is dropped and I_j is the pixel's integrated flux.
* R2 (eq. samlmexp, taylorexp, samlm5): the split of the w phase is
  n - 1 + (l^2 + m^2)/2 (printed with a minus sign).  Only "+" makes the
  split an identity and makes eq. (samlm5) reduce to eq. (deltam) at sigma=0.
* R3 (eq. cme vs the algorithm): the printed iteration with gradient
  M*(M y - V), step 1/L and threshold lambda/L minimises
  F(I) = 1/2 |V - M I|^2 + lambda sum_j I_j over I >= 0; the gradient of this
  real-variable objective is Re(M^H (M y - V)).
* R4 (largest eigenvalue, unspecified): power iteration on x -> Re(M^H M x)
  from a seeded uniform start, L = 1.01 x the last Rayleigh quotient.
* R5 (direction-dependent gain A(l,m;Z,chi), unspecified): baseline gain
  g = E_p(l,m) conj(E_q(l,m)) with E_p = c_p exp(-2 ln2 (l^2+m^2)/F_p^2), so
  the power beam E_p conj(E_p) has full width at half maximum F_p; absent
  antenna data means unit gain.
* R6 (termination): stop when |F_k - F_prev| <= eps * F_prev between two
  consecutive checks (every `check_every` iterations); eps = 0 disables it.
* R16 (warm start, Section "Acceleration strategies"): the paper starts the
  iteration from the dirty image without stating its normalisation.  The
  dirty image here is max(0, Re(M^H V) / N_v) (a unit-gain point source of
  flux S gives S / n^2 at its pixel; the clip keeps the start positive), and
  a warm start from I_0 runs the printed iteration with y_1 = I_0, t_1 = 1.

Indices follow the notation j = pixel, k = visibility; phases are in turns.
"""
from __future__ import annotations

import concurrent.futures as _cf
import math
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PIX_DELTA = 0
PIX_GAUSS_PARAXIAL = 1
PIX_GAUSS_WIDE = 2


def _threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


@dataclass
class Problem:
    """Pixels (l, m, sigma, kind) and visibilities (u, v, w) plus antenna data."""

    l: np.ndarray
    m: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    sigma: Optional[np.ndarray] = None
    kind: Optional[np.ndarray] = None
    ant_p: Optional[np.ndarray] = None
    ant_q: Optional[np.ndarray] = None
    ant_gain: Optional[np.ndarray] = None
    ant_fwhm: Optional[np.ndarray] = None
    threads: int = field(default_factory=_threads)

    def __post_init__(self):
        self.l = np.asarray(self.l, np.float64)
        self.m = np.asarray(self.m, np.float64)
        self.u = np.asarray(self.u, np.float64)
        self.v = np.asarray(self.v, np.float64)
        self.w = np.asarray(self.w, np.float64)
        n = self.l.shape[0]
        self.sigma = np.zeros(n) if self.sigma is None else np.asarray(self.sigma, np.float64)
        if self.kind is None:
            self.kind = np.where(self.sigma > 0, PIX_GAUSS_WIDE, PIX_DELTA).astype(np.uint8)
        self.kind = np.asarray(self.kind, np.uint8)
        if np.any(self.l ** 2 + self.m ** 2 >= 1.0):
            raise ValueError("every pixel needs l^2 + m^2 < 1")

    @property
    def n_pix(self) -> int:
        return int(self.l.shape[0])

    @property
    def n_vis(self) -> int:
        return int(self.u.shape[0])

    @classmethod
    def from_workload(cls, wl, threads: Optional[int] = None) -> "Problem":
        kw = {} if threads is None else {"threads": threads}
        return cls(l=wl.l, m=wl.m, u=wl.u, v=wl.v, w=wl.w, sigma=wl.sigma, kind=wl.kind,
                   ant_p=wl.ant_p, ant_q=wl.ant_q, ant_gain=wl.ant_gain,
                   ant_fwhm=wl.ant_fwhm, **kw)


# --------------------------------------------------------------------------
# matrix entries
# --------------------------------------------------------------------------

def n_of(l, m):
    """n = sqrt(1 - l^2 - m^2): the third direction cosine (eq. fullvis)."""
    return np.sqrt(1.0 - l * l - m * m)


def gain_block(p: Problem, ks, js):
    """Direction-dependent gain g_kj = E_p(l_j, m_j) conj(E_q(l_j, m_j))  (R5)."""
    if p.ant_p is None:
        return None
    ap = np.asarray(p.ant_p)[ks]
    aq = np.asarray(p.ant_q)[ks]
    c = np.ones(int(max(ap.max(), aq.max())) + 1, np.complex128) if p.ant_gain is None \
        else np.asarray(p.ant_gain, np.complex128)
    r2 = (p.l[js] ** 2 + p.m[js] ** 2)[None, :]
    if p.ant_fwhm is None:
        ep = np.broadcast_to(c[ap][:, None], (ap.shape[0], r2.shape[1]))
        eq = np.broadcast_to(c[aq][:, None], (aq.shape[0], r2.shape[1]))
    else:
        F = np.asarray(p.ant_fwhm, np.float64)
        ep = c[ap][:, None] * np.exp(-2.0 * math.log(2.0) * r2 / F[ap][:, None] ** 2)
        eq = c[aq][:, None] * np.exp(-2.0 * math.log(2.0) * r2 / F[aq][:, None] ** 2)
    return ep * np.conj(eq)


def delta_block(p: Problem, ks, js):
    """eq. (deltam): M_kj = A / n_j * exp(-2 pi i (u l + v m + w (n - 1))), A = 1."""
    l, m = p.l[js][None, :], p.m[js][None, :]
    u, v, w = p.u[ks][:, None], p.v[ks][:, None], p.w[ks][:, None]
    n = n_of(l, m)
    return (1.0 / n) * np.exp(-2j * np.pi * (u * l + v * m + w * (n - 1.0)))


def gauss_paraxial_block(p: Problem, ks, js):
    """eq. (samlm4) as printed, with the prefactor 1/sigma^2 dropped (R1).

    M_kj = A / n_j * 1/(1 - i w s2) * exp(-2 pi i (l u + m v)/(1 - i w s2))
           * exp(i pi w (l^2 + m^2)/(1 - i w s2)) * exp(-pi s2 (u^2 + v^2)/(1 - i w s2)),
    with s2 = sigma_j^2 and A = 1.
    """
    l, m = p.l[js][None, :], p.m[js][None, :]
    s2 = (p.sigma[js] ** 2)[None, :]
    u, v, w = p.u[ks][:, None], p.v[ks][:, None], p.w[ks][:, None]
    n = n_of(l, m)
    den = 1.0 - 1j * w * s2
    e1 = np.exp(-2j * np.pi * (l * u + m * v) / den)
    e2 = np.exp(1j * np.pi * w * (l * l + m * m) / den)
    e3 = np.exp(-np.pi * s2 * (u * u + v * v) / den)
    return (1.0 / n) / den * e1 * e2 * e3


def gauss_wide_block(p: Problem, ks, js):
    """eq. (samlm5): eq. (samlm4) times exp(-2 pi i w (n - 1 + (l^2+m^2)/2))  (R2)."""
    l, m = p.l[js][None, :], p.m[js][None, :]
    w = p.w[ks][:, None]
    n = n_of(l, m)
    corr = np.exp(-2j * np.pi * w * (n - 1.0 + (l * l + m * m) / 2.0))
    return gauss_paraxial_block(p, ks, js) * corr


def matrix_block(p: Problem, ks, js):
    """Rows ks (visibilities) x columns js (pixels) of M, complex128."""
    ks = np.asarray(ks)
    js = np.asarray(js)
    kind = p.kind[js]
    out = np.empty((ks.shape[0], js.shape[0]), np.complex128)
    for kd, fn in ((PIX_DELTA, delta_block), (PIX_GAUSS_PARAXIAL, gauss_paraxial_block),
                   (PIX_GAUSS_WIDE, gauss_wide_block)):
        sel = np.nonzero(kind == kd)[0]
        if sel.size:
            out[:, sel] = fn(p, ks, js[sel])
    g = gain_block(p, ks, js)
    if g is not None:
        out *= g
    return out


# --------------------------------------------------------------------------
# operator applications (blocked; never materialises all of M)
# --------------------------------------------------------------------------

_KB = 512
_JB = 2048


def _pool(p: Problem):
    return _cf.ThreadPoolExecutor(max_workers=p.threads)


def forward_rows(p: Problem, x, ks=None):
    """V_k = sum_j M_kj x_j for the visibilities ks (default all).

    x is real [n_pix] or [R, n_pix]; the result is complex [len(ks)] or [R, len(ks)].
    """
    x = np.asarray(x, np.float64)
    multi = x.ndim == 2
    X = x if multi else x[None, :]
    ks = np.arange(p.n_vis) if ks is None else np.asarray(ks)
    out = np.zeros((X.shape[0], ks.shape[0]), np.complex128)
    cols = np.arange(p.n_pix)

    def task(a):
        kb = ks[a:a + _KB]
        acc = np.zeros((X.shape[0], kb.shape[0]), np.complex128)
        for b in range(0, cols.shape[0], _JB):
            jb = cols[b:b + _JB]
            acc += (matrix_block(p, kb, jb) @ X[:, jb].T).T
        out[:, a:a + _KB] = acc

    with _pool(p) as ex:
        list(ex.map(task, range(0, ks.shape[0], _KB)))
    return out if multi else out[0]


def forward(p: Problem, x):
    """V = M x (eq. sme)."""
    return forward_rows(p, x)


def adjoint_cols(p: Problem, r, js=None):
    """g_j = Re sum_k conj(M_kj) r_k for the pixels js (default all)  (R3).

    r is complex [n_vis] or [R, n_vis]; the result is real [len(js)] or [R, len(js)].
    """
    r = np.asarray(r, np.complex128)
    multi = r.ndim == 2
    Rm = r if multi else r[None, :]
    js = np.arange(p.n_pix) if js is None else np.asarray(js)
    out = np.zeros((Rm.shape[0], js.shape[0]), np.float64)

    def task(b):
        jb = js[b:b + _JB]
        acc = np.zeros((Rm.shape[0], jb.shape[0]), np.complex128)
        for a in range(0, p.n_vis, _KB):
            kb = np.arange(a, min(a + _KB, p.n_vis))
            acc += Rm[:, kb] @ np.conj(matrix_block(p, kb, jb))
        out[:, b:b + _JB] = acc.real

    with _pool(p) as ex:
        list(ex.map(task, range(0, js.shape[0], _JB)))
    return out if multi else out[0]


def adjoint(p: Problem, r):
    """Re(M^H r): the back-projection used by the gradient step (R3)."""
    return adjoint_cols(p, r)


def adjoint_complex(p: Problem, r, js=None):
    """Full complex M^H r (used only by identity checks)."""
    r = np.asarray(r, np.complex128)
    js = np.arange(p.n_pix) if js is None else np.asarray(js)
    out = np.zeros(js.shape[0], np.complex128)
    for b in range(0, js.shape[0], _JB):
        jb = js[b:b + _JB]
        for a in range(0, p.n_vis, _KB):
            kb = np.arange(a, min(a + _KB, p.n_vis))
            out[b:b + _JB] += r[kb] @ np.conj(matrix_block(p, kb, jb))
    return out


# --------------------------------------------------------------------------
# operator object used by the solver
# --------------------------------------------------------------------------

class Operator:
    """x -> M x and r -> Re(M^H r) for one problem.

    With ``dense=True`` (default for problems of at most 4e6 entries) the
    matrix is evaluated once from the same closed forms and kept; otherwise
    every application re-evaluates the entries block by block.
    """

    def __init__(self, p: Problem, dense: Optional[bool] = None):
        self.p = p
        if dense is None:
            dense = p.n_pix * p.n_vis <= 4_000_000
        self.M = matrix_block(p, np.arange(p.n_vis), np.arange(p.n_pix)) if dense else None

    @property
    def n_pix(self):
        return self.p.n_pix

    @property
    def n_vis(self):
        return self.p.n_vis

    def forward(self, x):
        if self.M is not None:
            x = np.asarray(x, np.float64)
            return (self.M @ x.T).T
        return forward(self.p, x)

    def adjoint(self, r):
        if self.M is not None:
            r = np.asarray(r, np.complex128)
            return (r @ np.conj(self.M)).real
        return adjoint(self.p, r)


def _as_op(op):
    return op if isinstance(op, Operator) else Operator(op)


# --------------------------------------------------------------------------
# step size
# --------------------------------------------------------------------------

_SM_GAMMA = 0x9E3779B97F4A7C15
_SM_M1 = 0xBF58476D1CE4E5B9
_SM_M2 = 0x94D049BB133111EB


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """U[0,1) from the SplitMix64 generator (Steele, Lea & Flood 2014).

    Counter form: state_i = seed + (i + 1) * gamma; output = mix(state_i);
    uniform = (output >> 11) * 2^-53.
    """
    return (splitmix64_raw(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def splitmix64_raw(seed: int, n: int) -> np.ndarray:
    """The first n 64-bit outputs of SplitMix64 started from state `seed`."""
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * np.uint64(_SM_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_SM_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_SM_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def power_iteration(op, iters: int = 30, seed: int = 0, x0=None, safety: float = 1.01):
    """Largest eigenvalue of Re(M^H M) by power iteration (R4).

    Start x0 (default SplitMix64 uniforms), normalised; each step applies
    x -> Re(M^H (M x)), takes the Rayleigh quotient <x, A x> and renormalises.
    Returns (safety * last Rayleigh quotient, last Rayleigh quotient).
    """
    op = _as_op(op)
    x = splitmix64_uniform(seed, op.n_pix) if x0 is None else np.asarray(x0, np.float64).copy()
    x /= np.linalg.norm(x)
    rq = 0.0
    for _ in range(iters):
        y = op.adjoint(op.forward(x))
        rq = float(np.dot(x, y))
        x = y / np.linalg.norm(y)
    return safety * rq, rq


# --------------------------------------------------------------------------
# FISTA with the positive threshold
# --------------------------------------------------------------------------

def threshold_pos(x, d):
    """eq. (threshp): x_i - d where x_i > d, else 0."""
    return np.where(x > d, x - d, 0.0)


def objective(op, V, I, lam):
    """F(I) = 1/2 |V - M I|^2 + lambda sum_j I_j   (R3); returns (F, l2, l1)."""
    op = _as_op(op)
    res = V - op.forward(I)
    l2 = 0.5 * float(np.vdot(res, res).real)
    l1 = float(np.sum(I))
    return l2 + lam * l1, l2, l1


def momentum_sequence(n: int):
    """t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2; returns t_1..t_{n+1}."""
    t = [1.0]
    for _ in range(n):
        t.append((1.0 + math.sqrt(1.0 + 4.0 * t[-1] ** 2)) / 2.0)
    return np.array(t)


@dataclass
class FistaResult:
    image: np.ndarray
    iters: int
    L: float
    F: float
    l2_term: float
    l1_term: float
    nnz: int
    converged: int         # 0, 1 (objective rule) or 2 (non-zero-count rule)
    history: list
    state: tuple


def fista(op, V, L: float, lam: float, n_iter: int, eps: float = 0.0,
          check_every: int = 1, keep_history: bool = False, state=None,
          nnz_eps: float = 0.0):
    """The printed FISTA iteration (Section "Implementation of SL1M").

    Step 0: y_1 = I_0 = 0, t_1 = 1.  Step k:
      I_k     = T^{lambda/L}( y_k - (1/L) Re M^H (M y_k - V) )
      t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
      y_{k+1} = I_k + ((t_k - 1)/t_{k+1}) (I_k - I_{k-1})
    `state` = (k, t_k, I_{k-1}, y_k) resumes a previous run exactly.
    Stops early when eps > 0 and the relative change of F between two checks
    is at most eps (R6), or when nnz_eps > 0 and the number of non-zero
    pixels changed by less than nnz_eps * max(previous count, 1) between two
    checks (the paper's second stopping rule, same section); `converged` is
    then 1 or 2.
    """
    op = _as_op(op)
    V = np.asarray(V, np.complex128)
    if state is None:
        k0, t, I_prev, y = 0, 1.0, np.zeros(op.n_pix), np.zeros(op.n_pix)
    else:
        k0, t, I_prev, y = state
        I_prev, y = I_prev.copy(), y.copy()
    hist = []
    F_prev = None
    nnz_prev = None
    converged = False
    I = I_prev
    k = k0
    for k in range(k0 + 1, k0 + n_iter + 1):
        grad = op.adjoint(op.forward(y) - V)
        I = threshold_pos(y - grad / L, lam / L)
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        y = I + ((t - 1.0) / t_next) * (I - I_prev)
        I_prev, t = I, t_next
        if keep_history:
            hist.append(I.copy())
        if (eps > 0.0 or nnz_eps > 0.0) and (k - k0) % check_every == 0:
            F_k = objective(op, V, I, lam)[0]
            nnz_k = int(np.count_nonzero(I))
            if eps > 0.0 and F_prev is not None and abs(F_k - F_prev) <= eps * F_prev:
                converged = 1
                break
            if nnz_eps > 0.0 and nnz_prev is not None and \
                    abs(nnz_k - nnz_prev) < nnz_eps * max(nnz_prev, 1):
                converged = 2
                break
            F_prev, nnz_prev = F_k, nnz_k
    F, l2, l1 = objective(op, V, I, lam)
    return FistaResult(image=I, iters=k - k0, L=L, F=F, l2_term=l2, l1_term=l1,
                       nnz=int(np.count_nonzero(I)), converged=converged, history=hist,
                       state=(k, t, I_prev, y))


def dirty_image(op, V):
    """The dirty image, the starting point Section "Acceleration strategies"
    names: max(0, Re(M^H V) / N_v) (reading R16)."""
    op = _as_op(op)
    D = op.adjoint(np.asarray(V, np.complex128)) / op.p.n_vis
    return np.maximum(D, 0.0)


def fista_from(op, V, L: float, lam: float, n_iter: int, I0, eps: float = 0.0,
               check_every: int = 1, keep_history: bool = False):
    """Warm start (Section "Acceleration strategies"): the printed iteration
    from y_1 = I_0 instead of 0, t_1 = 1 (so the first momentum coefficient
    (t_1 - 1)/t_2 is 0 and I_0 enters only through y_1)."""
    I0 = np.asarray(I0, np.float64)
    return fista(op, V, L, lam, n_iter, eps=eps, check_every=check_every,
                 keep_history=keep_history, state=(0, 1.0, I0.copy(), I0.copy()))


def mfista(op, V, L: float, lam: float, n_iter: int, I0=None, keep_history: bool = False):
    """The monotone variant the paper names after the printed algorithm
    (Section "Implementation of SL1M": MFISTA of Beck & Teboulle, at the cost
    of one more evaluation of M per iteration).  From x_0 = y_1 = I_0 (0 when
    not given), t_1 = 1, step k:
      z_k     = T^{lambda/L}( y_k - (1/L) Re M^H (M y_k - V) )
      t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
      x_k     = z_k if F(z_k) <= F(x_{k-1}) else x_{k-1}
      y_{k+1} = x_k + (t_k/t_{k+1}) (z_k - x_k) + ((t_k - 1)/t_{k+1}) (x_k - x_{k-1})
    so F(x_k) never increases."""
    op = _as_op(op)
    V = np.asarray(V, np.complex128)
    x = np.zeros(op.n_pix) if I0 is None else np.asarray(I0, np.float64).copy()
    y = x.copy()
    t = 1.0
    Fx = objective(op, V, x, lam)[0]
    hist = []
    for _ in range(n_iter):
        grad = op.adjoint(op.forward(y) - V)
        z = threshold_pos(y - grad / L, lam / L)
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        Fz = objective(op, V, z, lam)[0]
        x_new = z if Fz <= Fx else x
        y = x_new + (t / t_next) * (z - x_new) + ((t - 1.0) / t_next) * (x_new - x)
        x, t, Fx = x_new, t_next, min(Fz, Fx)
        if keep_history:
            hist.append(x.copy())
    F, l2, l1 = objective(op, V, x, lam)
    return FistaResult(image=x, iters=n_iter, L=L, F=F, l2_term=l2, l1_term=l1,
                       nnz=int(np.count_nonzero(x)), converged=False, history=hist,
                       state=None)


def kkt_residual(op, V, I, lam):
    """Optimality certificate of min 1/2|V - M I|^2 + lam sum I, I >= 0.

    With G = Re M^H (V - M I): G_j = lam where I_j > 0 and G_j <= lam where
    I_j = 0.  Returns the largest violation.
    """
    op = _as_op(op)
    G = op.adjoint(V - op.forward(I))
    on = I > 0
    v_on = np.max(np.abs(G[on] - lam)) if np.any(on) else 0.0
    v_off = np.max(np.maximum(G[~on] - lam, 0.0)) if np.any(~on) else 0.0
    return float(max(v_on, v_off))
