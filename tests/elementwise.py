"""Element-wise error bounds for operator parity (test infrastructure).

Each output of the forward operator is a sum of n_pix products M_kj x_j and
each output of the adjoint a sum of n_vis products conj(M_kj) r_k.  A
computed sum then satisfies

    |err_k| <= (e_entry + lambda sqrt(n) u) * sum_j |M_kj| |x_j|

where e_entry bounds the relative error of one product and the second term is
the probabilistic bound on the accumulated rounding of any summation order
(Higham & Mary, "A new approach to probabilistic rounding error analysis",
SIAM J. Sci. Comput. 2019), exceeded with probability at most
2 n exp(-lambda^2 (1 - u)^2 / 2); lambda = 6 makes that negligible here.

FP32 operator (FP64 phase): the phase is reduced exactly but for three
roundings of 2^-24 turn (1.2e-6 rad), the hardware sine/cosine in turns adds
a few ulp, a grid-evaluated entry is a product of three phasors, and the
amplitude (1/n, gains, beam, Gaussian taper and prefactor) a few roundings:
e_entry = 8e-6.  FP64 plans: e_entry = 1e-13.

The magnitudes sum_j |M_kj| |x_j| come from the oracle's own matrix entries
(blocks of the FP64 definition).
"""
from __future__ import annotations

import concurrent.futures as cf

import numpy as np

import oracle as O

U = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53}
E_ENTRY = {"fp32": 8e-6, "fp64": 1e-13}
LAMBDA = 6.0


def coefficient(n_terms: int, prec: str = "fp32") -> float:
    return E_ENTRY[prec] + LAMBDA * np.sqrt(max(n_terms, 1)) * U[prec]


def abs_forward_rows(p, x, ks=None, workers: int = 8):
    """sum_j |M_kj| |x_j| for the visibilities ks (default all)."""
    ax = np.abs(np.asarray(x, np.float64))
    ks = np.arange(p.n_vis) if ks is None else np.asarray(ks)
    out = np.zeros(ks.shape[0])
    step = int(min(256, max(1, -(-ks.shape[0] // (4 * workers)))))

    def task(a):
        kb = ks[a:a + step]
        acc = np.zeros(kb.shape[0])
        for b in range(0, p.n_pix, 4096):
            jb = np.arange(b, min(b + 4096, p.n_pix))
            acc += np.abs(O.matrix_block(p, kb, jb)) @ ax[jb]
        out[a:a + step] = acc

    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(task, range(0, ks.shape[0], step)))
    return out


def abs_adjoint_cols(p, r, js=None, workers: int = 8):
    """sum_k |M_kj| |r_k| for the pixels js (default all)."""
    ar = np.abs(np.asarray(r, np.complex128))
    js = np.arange(p.n_pix) if js is None else np.asarray(js)
    out = np.zeros(js.shape[0])
    step = int(min(1024, max(1, -(-js.shape[0] // (4 * workers)))))

    def task(b):
        jb = js[b:b + step]
        acc = np.zeros(jb.shape[0])
        for a in range(0, p.n_vis, 1024):
            kb = np.arange(a, min(a + 1024, p.n_vis))
            acc += ar[kb] @ np.abs(O.matrix_block(p, kb, jb))
        out[b:b + step] = acc

    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(task, range(0, js.shape[0], step)))
    return out


def worst_ratio(got, ref, mag, n_terms: int, prec: str = "fp32"):
    """max_k |got_k - ref_k| / (c(n) mag_k): <= 1 when every element is
    within its bound."""
    err = np.abs(np.asarray(got) - np.asarray(ref))
    c = coefficient(n_terms, prec)
    return float(np.max(err / (c * np.maximum(mag, np.finfo(float).tiny)))) if err.size else 0.0
