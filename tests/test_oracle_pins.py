"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values that
can be derived by hand, library routines (FFT, eigvalsh, a bound-constrained
quasi-Newton minimiser, Dawson's integral), numerical quadrature of the
paper's integrals, the paper's own printed numbers (tests/golden), and
theorems about FISTA.  `test_oracle_mutations.py` plants mistakes in the
oracle and shows that these pins catch them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize
import scipy.special

import oracle as O
from paper_1310_2078_amd import workloads as W


def _prob(l, m, u, v, w, **kw):
    return O.Problem(l=np.atleast_1d(np.asarray(l, float)), m=np.atleast_1d(np.asarray(m, float)),
                     u=np.atleast_1d(np.asarray(u, float)), v=np.atleast_1d(np.asarray(v, float)),
                     w=np.atleast_1d(np.asarray(w, float)), threads=2, **kw)


# --------------------------------------------------------------------------
# delta pixels: eq. (deltam)
# --------------------------------------------------------------------------

def test_delta_entries_by_hand():
    """Entries worked out by hand from eq. (deltam).

    Pixel (0.6, 0): n = 0.8, n - 1 = -0.2, 1/n = 1.25.
      (u,v,w) = (5/12, 0, 0)   -> phase 0.25 turn  -> exp(-i pi/2) = -i  -> -1.25i
      (u,v,w) = (0, 0, 1.25)   -> phase -0.25 turn -> exp(+i pi/2) = +i  -> +1.25i
      (u,v,w) = (5/6, 0, 1.25) -> phase 0.5 - 0.25 -> -i                 -> -1.25i
    Pixel (0, 0.6): (u,v,w) = (0, 5/6, 0) -> phase 0.5 -> -1 -> -1.25.
    Pixel (0, 0): every visibility gives exactly 1.
    """
    p = _prob([0.6, 0.0, 0.0], [0.0, 0.6, 0.0],
              [5 / 12, 0.0, 5 / 6, 0.0], [0.0, 0.0, 0.0, 5 / 6], [0.0, 1.25, 1.25, 0.0])
    M = O.matrix_block(p, np.arange(4), np.arange(3))
    np.testing.assert_allclose(M[0, 0], -1.25j, atol=1e-14)
    np.testing.assert_allclose(M[1, 0], 1.25j, atol=1e-14)
    np.testing.assert_allclose(M[2, 0], -1.25j, atol=1e-14)
    np.testing.assert_allclose(M[3, 1], -1.25, atol=1e-14)
    np.testing.assert_allclose(M[:, 2], 1.0, atol=0)


def test_unit_delta_at_phase_centre_gives_constant_visibilities():
    """Check (2): a unit delta at (0, 0) gives V_k = 1 for every k, exactly."""
    wl = W.config1()
    p = O.Problem.from_workload(wl, threads=2)
    x = np.zeros(p.n_pix)
    centre = np.nonzero((wl.l == 0) & (wl.m == 0))[0]
    assert centre.size == 1
    x[centre] = 1.0
    V = O.forward(p, x)
    assert np.all(V == 1.0 + 0.0j)


def test_w0_regular_grid_matches_fft2():
    """Check (3): for w = 0 on an N x N grid and u_p = p/(N D), v_q = q/(N D)
    the operator is a 2-D DFT: V(p, q) = (-1)^(p+q) fft2(X / n)[q, p],
    with X[row, col] = x[col + N row]."""
    N, half = 16, 0.16
    l, m, D = W.grid_pixels(N, half)
    pp, qq = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    u = (pp.ravel() / (N * D))
    v = (qq.ravel() / (N * D))
    p = _prob(l, m, u, v, np.zeros_like(u))
    x = np.random.default_rng(5).standard_normal(N * N)
    V = O.forward(p, x)
    X = (x / np.sqrt(1 - l ** 2 - m ** 2)).reshape(N, N)
    F = np.fft.fft2(X)
    sign = (-1.0) ** (pp + qq)
    expect = (sign * F[qq, pp]).ravel()
    np.testing.assert_allclose(V, expect, rtol=0, atol=1e-11 * np.abs(expect).max())


def test_delta_phase_is_geometric_delay():
    """The w-term is the geometric path difference b.(s - s0) for a direction
    s = (sin t cos f, sin t sin f, cos t) built from spherical angles, and the
    amplitude is 1/cos t (direction cosine n from the angle, not from l, m)."""
    rng = np.random.default_rng(11)
    t = rng.uniform(0.05, 1.2, 7)
    f = rng.uniform(0, 2 * np.pi, 7)
    s = np.stack([np.sin(t) * np.cos(f), np.sin(t) * np.sin(f), np.cos(t)], 1)
    b = rng.normal(0, 300, (9, 3))
    p = _prob(s[:, 0], s[:, 1], b[:, 0], b[:, 1], b[:, 2])
    M = O.matrix_block(p, np.arange(9), np.arange(7))
    delay = b @ (s - np.array([0.0, 0.0, 1.0])).T
    expect = np.exp(-2j * np.pi * delay) / np.cos(t)[None, :]
    np.testing.assert_allclose(M, expect, rtol=1e-10, atol=0)


def test_projection_weight_integrates_to_solid_angle():
    """Sum_j x_j M_0j Delta^2 at (u,v,w) = 0 approximates the solid-angle
    integral of a Gaussian window: int exp(-r^2/s^2) dOmega = 2 pi s D(1/s),
    with D Dawson's integral (dOmega = dl dm / n)."""
    s, N = 0.2, 800
    l, m, D = W.grid_pixels(N, 1.0)
    keep = l ** 2 + m ** 2 < 0.995
    l, m = l[keep], m[keep]
    p = _prob(l, m, [0.0], [0.0], [0.0])
    x = np.exp(-(l ** 2 + m ** 2) / s ** 2)
    V0 = O.forward(p, x)[0].real * D * D
    expect = 2 * np.pi * s * scipy.special.dawsn(1 / s)
    assert abs(V0 - expect) < 1e-9 * expect
    # the flat-sky (no 1/n) value differs at the percent level
    assert abs(np.pi * s * s - expect) > 1e-3 * expect


def test_hermitian_symmetry():
    """Real sky, unit gains: V(-u,-v,-w) = conj(V(u,v,w)) for every pixel kind."""
    for kind, sig in ((O.PIX_DELTA, 0.0), (O.PIX_GAUSS_PARAXIAL, 4e-3), (O.PIX_GAUSS_WIDE, 4e-3)):
        wl = W.small_random(3, 300, 200, kind=kind, sigma=sig)
        p = O.Problem.from_workload(wl, threads=2)
        pn = O.Problem(l=wl.l, m=wl.m, u=-wl.u, v=-wl.v, w=-wl.w, sigma=wl.sigma,
                       kind=wl.kind, threads=2)
        np.testing.assert_allclose(O.forward(pn, wl.x_true), np.conj(O.forward(p, wl.x_true)),
                                   rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,sig,gains,distinct", [
    (O.PIX_DELTA, 0.0, False, False),
    (O.PIX_GAUSS_PARAXIAL, 3e-3, False, False),
    (O.PIX_GAUSS_WIDE, 3e-3, True, False),
    (O.PIX_DELTA, 0.0, True, True),
])
def test_adjoint_identity(kind, sig, gains, distinct):
    """Check (1): Re<M x, r> = <x, Re M^H r> for real x, complex r, with sizes
    that span several oracle blocks and ragged tails; and the complex identity
    <M x, r> = <x, M^H r> for complex x."""
    wl = W.small_random(7, 2500, 700, kind=kind, sigma=sig, with_gains=gains,
                        distinct_fwhm=distinct)
    p = O.Problem.from_workload(wl, threads=4)
    rng = np.random.default_rng(1)
    r = rng.standard_normal(p.n_vis) + 1j * rng.standard_normal(p.n_vis)
    x = rng.standard_normal(p.n_pix)
    lhs = np.vdot(O.forward(p, x), r).real
    rhs = np.dot(x, O.adjoint(p, r))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(r))
    xc = x + 1j * rng.standard_normal(p.n_pix)
    Mx = O.forward(p, xc.real) + 1j * O.forward(p, xc.imag)
    lhs_c = np.vdot(Mx, r)
    rhs_c = np.vdot(xc, O.adjoint_complex(p, r))
    assert abs(lhs_c - rhs_c) <= 1e-12 * np.linalg.norm(xc) * np.linalg.norm(r) * 10


def test_multi_rhs_equals_single_rhs():
    """Config 3 semantics: each right-hand side goes through the same M."""
    wl = W.config3()
    p = O.Problem.from_workload(wl, threads=4)
    V = O.forward(p, wl.x_true)
    for r in range(4):
        np.testing.assert_allclose(V[r], O.forward(p, wl.x_true[r]), rtol=1e-13, atol=1e-13)
    rr = V + 0.1
    G = O.adjoint(p, rr)
    for r in range(4):
        np.testing.assert_allclose(G[r], O.adjoint(p, rr[r]), rtol=1e-13, atol=1e-12)


# --------------------------------------------------------------------------
# Gaussian pixels: eq. (samlm4), eq. (samlm5) against quadrature
# --------------------------------------------------------------------------

def _gauss_quadrature(l0, m0, sig, u, v, w, integrand, h_frac=1 / 24, extent=7.0):
    """Trapezoid quadrature of int f(l,m) K(l,m; u,v,w) dl dm over +-extent*sigma,
    with f = exp(-pi ((l-l0)^2 + (m-m0)^2)/sigma^2) / sigma^2 (eq. gaus)."""
    h = sig * h_frac
    t = np.arange(-extent * sig, extent * sig + h / 2, h)
    L, Mm = np.meshgrid(l0 + t, m0 + t, indexing="xy")
    L, Mm = L.ravel(), Mm.ravel()
    f = np.exp(-np.pi * ((L - l0) ** 2 + (Mm - m0) ** 2) / sig ** 2) / sig ** 2
    out = []
    for uu, vv, ww in zip(u, v, w):
        out.append(np.sum(f * integrand(L, Mm, uu, vv, ww)) * h * h)
    return np.array(out)


def _vis_sample(rng, n, radius, wsig):
    a, b = rng.random(n), rng.random(n)
    return (radius * np.sqrt(a) * np.cos(2 * np.pi * b), radius * np.sqrt(a) * np.sin(2 * np.pi * b),
            wsig * rng.standard_normal(n))


def test_gaussian_paraxial_matches_quadrature_of_eq_samlm3():
    """Check (4a): the closed form eq. (samlm4) equals the quadrature of the
    paraxial integral eq. (samlm3) (gain and 1/n taken at the pixel centre)."""
    rng = np.random.default_rng(2)
    u, v, w = _vis_sample(rng, 6, 400.0, 150.0)
    for (l0, m0, sig) in ((0.03, -0.02, 3e-3), (-0.1, 0.05, 6e-3), (0.0, 0.0, 1e-2)):
        p = _prob([l0], [m0], u, v, w, sigma=[sig], kind=[O.PIX_GAUSS_PARAXIAL])
        M = O.matrix_block(p, np.arange(6), [0])[:, 0]
        n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
        q = _gauss_quadrature(l0, m0, sig, u, v, w,
                              lambda L, Mm, uu, vv, ww: np.exp(1j * np.pi * ww * (L * L + Mm * Mm))
                              * np.exp(-2j * np.pi * (uu * L + vv * Mm)) / n0)
        np.testing.assert_allclose(M, q, rtol=0, atol=1e-10)


def test_gaussian_by_hand():
    """Textbook Gaussian integrals: the unit-integral Gaussian has Fourier
    transform exp(-pi sigma^2 rho^2) (w = 0); at the phase centre with u=v=0
    the defocus integral is 1/(1 - i w sigma^2)."""
    sig = 0.01
    p = _prob([0.0], [0.0], [100.0, 0.0], [0.0, 0.0], [0.0, 700.0], sigma=[sig],
              kind=[O.PIX_GAUSS_PARAXIAL])
    M = O.matrix_block(p, np.arange(2), [0])[:, 0]
    np.testing.assert_allclose(M[0], math.exp(-math.pi), rtol=1e-14)
    np.testing.assert_allclose(M[1], 1 / (1 - 1j * 700 * sig * sig), rtol=1e-14)


def test_gaussian_wide_matches_exact_integral_within_bound():
    """Check (4b): the wide-field form eq. (samlm5) against the quadrature of the
    exact integral eq. (samlm) (full w(n - 1), 1/n varying over the pixel).
    In config 1's regime (|w| <~ 150, r <~ 0.07) the neglected terms are below
    1e-3 of the pixel's flux; at a wide field the wide-field form is far closer
    than the paraxial one."""
    rng = np.random.default_rng(4)
    exact = lambda L, Mm, uu, vv, ww: (np.exp(-2j * np.pi * (uu * L + vv * Mm + ww * (np.sqrt(1 - L * L - Mm * Mm) - 1)))
                                       / np.sqrt(1 - L * L - Mm * Mm))
    u, v, w = _vis_sample(rng, 6, 500.0, 50.0)
    w = np.clip(w, -150, 150)
    l0, m0, sig = 0.04, -0.05, 3.1e-3
    p = _prob([l0], [m0], u, v, w, sigma=[sig], kind=[O.PIX_GAUSS_WIDE])
    Mw = O.matrix_block(p, np.arange(6), [0])[:, 0]
    q = _gauss_quadrature(l0, m0, sig, u, v, w, exact)
    assert np.max(np.abs(Mw - q)) < 1e-3
    # wide field: r ~ 0.35, w ~ 400
    u, v, w = _vis_sample(rng, 6, 400.0, 400.0)
    l0, m0, sig = 0.25, -0.25, 1.5e-3
    pw = _prob([l0], [m0], u, v, w, sigma=[sig], kind=[O.PIX_GAUSS_WIDE])
    pp = _prob([l0], [m0], u, v, w, sigma=[sig], kind=[O.PIX_GAUSS_PARAXIAL])
    q = _gauss_quadrature(l0, m0, sig, u, v, w, exact)
    err_w = np.max(np.abs(O.matrix_block(pw, np.arange(6), [0])[:, 0] - q))
    err_p = np.max(np.abs(O.matrix_block(pp, np.arange(6), [0])[:, 0] - q))
    assert err_w < 0.05
    assert err_p > 20 * err_w


def test_gaussian_limits():
    """sigma -> 0: wide-field Gaussian = delta exactly; paraxial Gaussian =
    paraxial delta exp(-2 pi i (u l + v m - w r^2 / 2)) / n.
    w -> 0: Fourier transform of the Gaussian."""
    wl = W.small_random(9, 50, 40, half_extent=0.3, w_sigma=300.0)
    kw = dict(threads=2)
    base = dict(l=wl.l, m=wl.m, u=wl.u, v=wl.v, w=wl.w)
    Md = O.matrix_block(O.Problem(**base, **kw), np.arange(40), np.arange(50))
    Mw0 = O.matrix_block(O.Problem(**base, sigma=np.zeros(50),
                                   kind=np.full(50, O.PIX_GAUSS_WIDE, np.uint8), **kw),
                         np.arange(40), np.arange(50))
    np.testing.assert_allclose(Mw0, Md, rtol=1e-12, atol=1e-12)
    Mp0 = O.matrix_block(O.Problem(**base, sigma=np.zeros(50),
                                   kind=np.full(50, O.PIX_GAUSS_PARAXIAL, np.uint8), **kw),
                         np.arange(40), np.arange(50))
    u, v, w = wl.u[:, None], wl.v[:, None], wl.w[:, None]
    l, m = wl.l[None, :], wl.m[None, :]
    n = np.sqrt(1 - l * l - m * m)
    np.testing.assert_allclose(Mp0, np.exp(-2j * np.pi * (u * l + v * m - w * (l * l + m * m) / 2)) / n,
                               rtol=1e-12, atol=1e-12)
    sig = np.full(50, 5e-3)
    for kd in (O.PIX_GAUSS_PARAXIAL, O.PIX_GAUSS_WIDE):
        Mg = O.matrix_block(O.Problem(l=wl.l, m=wl.m, u=wl.u, v=wl.v, w=np.zeros(40), sigma=sig,
                                      kind=np.full(50, kd, np.uint8), **kw),
                            np.arange(40), np.arange(50))
        ft = np.exp(-np.pi * sig[None, :] ** 2 * (u * u + v * v)) * np.exp(-2j * np.pi * (u * l + v * m)) / n
        np.testing.assert_allclose(Mg, ft, rtol=1e-12, atol=1e-14)


def test_paraxial_phase_error_matches_paper(golden_dir):
    """The paper quotes ~1e-3 phase error at ~3 degrees for w = 1000; the wide
    minus paraxial phase of the oracle at that point has that size (in turns)."""
    g = json.load(open(os.path.join(golden_dir, "paraxial_phase_error.json")))
    r = math.sin(math.radians(g["angle_deg"]))
    sig = 1e-6
    pw = _prob([r], [0.0], [0.0], [0.0], [g["w"]], sigma=[sig], kind=[O.PIX_GAUSS_WIDE])
    pp = _prob([r], [0.0], [0.0], [0.0], [g["w"]], sigma=[sig], kind=[O.PIX_GAUSS_PARAXIAL])
    ratio = O.matrix_block(pw, [0], [0])[0, 0] / O.matrix_block(pp, [0], [0])[0, 0]
    err_turns = abs(np.angle(ratio)) / (2 * np.pi)
    assert abs(err_turns - g["phase_error"]) <= g["relative_tolerance"] * g["phase_error"]


def test_completed_square_form_equals_printed_form():
    """The numerically stable completed-square form of eq. (samlm4) (used by the
    GPU kernels) is algebraically the printed one: check at random points."""
    wl = W.small_random(13, 64, 64, half_extent=0.3, w_sigma=400.0, uv_radius=1500.0)
    sig = np.random.default_rng(0).uniform(1e-3, 6e-3, 64)
    p = O.Problem(l=wl.l, m=wl.m, u=wl.u, v=wl.v, w=wl.w, sigma=sig,
                  kind=np.full(64, O.PIX_GAUSS_PARAXIAL, np.uint8), threads=2)
    M = O.matrix_block(p, np.arange(64), np.arange(64))
    u, v, w = wl.u[:, None], wl.v[:, None], wl.w[:, None]
    l, m, s2 = wl.l[None, :], wl.m[None, :], sig[None, :] ** 2
    s = w * s2
    D = 1 / (1 + s * s)
    taper = np.exp(-np.pi * s2 * D * ((u - w * l) ** 2 + (v - w * m) ** 2))
    phase = D * (-(u * l + v * m) + 0.5 * w * (l * l + m * m - s2 * s2 * (u * u + v * v)))
    alt = D * (1 + 1j * s) * taper * np.exp(2j * np.pi * phase) / np.sqrt(1 - l * l - m * m)
    np.testing.assert_allclose(M, alt, rtol=1e-9, atol=1e-12)


# --------------------------------------------------------------------------
# gains
# --------------------------------------------------------------------------

def test_gain_power_beam_fwhm_and_reductions():
    """E_p conj(E_p) falls to half at r = F/2 (power-beam FWHM F); unit gain
    constants with no beam reduce to the gain-free operator; equal widths
    factorise into c_p conj(c_q) times a per-pixel beam."""
    F = 0.4
    p = _prob([F / 2, 0.0], [0.0, 0.0], [0.0], [0.0], [0.0], ant_p=np.array([0]),
              ant_q=np.array([0]), ant_gain=np.array([1.0 + 0j]), ant_fwhm=np.array([F]))
    M = O.matrix_block(p, [0], [0, 1])[0]
    n = math.sqrt(1 - (F / 2) ** 2)
    assert abs(M[0] * n / M[1] - 0.5) < 1e-14
    wl = W.small_random(21, 80, 60, with_gains=True)
    base = O.Problem.from_workload(wl, threads=2)
    unit = O.Problem(l=wl.l, m=wl.m, u=wl.u, v=wl.v, w=wl.w, ant_p=wl.ant_p, ant_q=wl.ant_q,
                     ant_gain=np.ones(16, complex), threads=2)
    plain = O.Problem(l=wl.l, m=wl.m, u=wl.u, v=wl.v, w=wl.w, threads=2)
    np.testing.assert_allclose(O.matrix_block(unit, np.arange(60), np.arange(80)),
                               O.matrix_block(plain, np.arange(60), np.arange(80)), rtol=1e-15)
    Mg = O.matrix_block(base, np.arange(60), np.arange(80))
    Mp = O.matrix_block(plain, np.arange(60), np.arange(80))
    cpq = (wl.ant_gain[wl.ant_p] * np.conj(wl.ant_gain[wl.ant_q]))[:, None]
    beam = np.exp(-4 * math.log(2) * (wl.l ** 2 + wl.m ** 2) / 0.4 ** 2)[None, :]
    np.testing.assert_allclose(Mg, cpq * beam * Mp, rtol=1e-13, atol=1e-15)


def test_gain_with_distinct_beam_widths_is_a_product_of_voltage_patterns():
    """Antennas with different primary beams (eq. samdelta's per-visibility
    gain, reading R5): the pair gain is the product of the two antennas'
    voltage patterns, so (a) its power is the geometric mean of the two
    antennas' own power beams, |g_pq|^2 = |g_pp| |g_qq|, each of which is
    pinned by its half-power width above; (b) swapping the antennas
    conjugates it, g_qp = conj(g_pq); (c) its phase is that of c_p conj(c_q)
    (voltage patterns are real).  A pair gain that used one antenna's width
    for both factors breaks (a) and (b)."""
    F = np.array([0.3, 0.55, 0.42])
    c = np.array([1.1 * np.exp(0.3j), 0.9 * np.exp(-0.2j), 1.0 + 0j])
    rng = np.random.default_rng(41)
    l = rng.uniform(-0.3, 0.3, 40)
    m = rng.uniform(-0.3, 0.3, 40)
    # visibilities: every ordered pair (p, q) including p == q; w = 0 and
    # u = v = 0 so the matrix entry is the gain times 1/n
    pairs = [(a, b) for a in range(3) for b in range(3)]
    ap = np.array([a for a, _ in pairs])
    aq = np.array([b for _, b in pairs])
    z = np.zeros(len(pairs))
    p = _prob(l, m, z, z, z, ant_p=ap, ant_q=aq, ant_gain=c, ant_fwhm=F)
    n = np.sqrt(1.0 - l * l - m * m)
    G = O.matrix_block(p, np.arange(len(pairs)), np.arange(40)) * n[None, :]
    row = {pq: G[i] for i, pq in enumerate(pairs)}
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            np.testing.assert_allclose(np.abs(row[(a, b)]) ** 2,
                                       np.abs(row[(a, a)]) * np.abs(row[(b, b)]), rtol=1e-13)
            np.testing.assert_allclose(row[(b, a)], np.conj(row[(a, b)]), rtol=1e-13)
            np.testing.assert_allclose(np.angle(row[(a, b)]),
                                       np.full(40, np.angle(c[a] * np.conj(c[b]))), atol=1e-13)


# --------------------------------------------------------------------------
# step size: largest eigenvalue
# --------------------------------------------------------------------------

def test_power_iteration_vs_eigvalsh():
    """L from power iteration approaches lambda_max(Re M^H M) from below."""
    wl = W.config1()
    p = O.Problem.from_workload(wl, threads=4)
    op = O.Operator(p, dense=True)
    A = (op.M.conj().T @ op.M).real
    lmax = np.linalg.eigvalsh(A)[-1]
    L30, rq30 = O.power_iteration(op, 30, seed=0)
    assert rq30 <= lmax * (1 + 1e-12)
    assert rq30 >= 0.97 * lmax
    assert L30 == pytest.approx(1.01 * rq30)
    prev = 0.0
    for iters in (10, 50, 200, 800):
        _, rq = O.power_iteration(op, iters, seed=0)
        assert prev <= rq <= lmax * (1 + 1e-12)   # non-decreasing for a PSD matrix
        prev = rq
    assert abs(rq - lmax) <= 1e-6 * lmax


def test_splitmix64_reference_outputs():
    """The counter-based start vector uses SplitMix64; its published first
    outputs from state 0 are 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4,
    0x06c45d188009454f."""
    z = O.splitmix64_raw(0, 3)
    assert [int(a) for a in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = O.splitmix64_uniform(123, 10000)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.01


# --------------------------------------------------------------------------
# FISTA
# --------------------------------------------------------------------------

def _small_solve_problem(n_side=8, n_vis=200, seed=31, n_src=3, half=0.05, radius=300.0):
    rng = np.random.default_rng(seed)
    l, m, _ = W.grid_pixels(n_side, half)
    u, v, w = W.disk_uvw(rng, n_vis, radius, 30.0)
    p = O.Problem(l=l, m=m, u=u, v=v, w=w, threads=2)
    x = np.zeros(l.shape[0])
    src = rng.choice(l.shape[0], n_src, replace=False)
    x[src] = rng.uniform(0.5, 2.0, n_src)
    return p, x


def test_threshold_and_momentum_sequence():
    """eq. (threshp) (ties map to 0, no negative branch) and t_2 = (1+sqrt5)/2,
    t_k >= (k + 1)/2."""
    np.testing.assert_array_equal(O.threshold_pos(np.array([-3.0, 0.5, 1.0, 2.5]), 1.0),
                                  [0.0, 0.0, 0.0, 1.5])
    t = O.momentum_sequence(50)
    assert t[0] == 1.0 and t[1] == pytest.approx((1 + math.sqrt(5)) / 2, rel=1e-15)
    assert np.all(t >= (np.arange(1, 52) + 1) / 2 - 1e-12)


def test_fista_first_iterate_closed_form():
    """With y_1 = 0: I_1 = T^{lam/L}(Re M^H V / L)."""
    p, x = _small_solve_problem()
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    L, _ = O.power_iteration(op, 50)
    lam = 0.5
    res = O.fista(op, V, L, lam, 1, keep_history=True)
    np.testing.assert_allclose(res.history[0], O.threshold_pos(op.adjoint(V) / L, lam / L),
                               rtol=1e-14, atol=1e-15)


def test_fista_converges_to_library_minimiser_and_satisfies_kkt():
    """FISTA's limit is the minimiser of 1/2|V - M I|^2 + lam sum I on I >= 0
    found independently by L-BFGS-B; the KKT certificate holds there."""
    p, x = _small_solve_problem(n_vis=60, seed=33)
    op = O.Operator(p, dense=True)
    rng = np.random.default_rng(0)
    V = op.forward(x) + 0.05 * (rng.standard_normal(p.n_vis) + 1j * rng.standard_normal(p.n_vis))
    lam = 0.3
    L, _ = O.power_iteration(op, 100)
    res = O.fista(op, V, L, lam, 4000)

    def fg(I):
        r = op.forward(I) - V
        return 0.5 * np.vdot(r, r).real + lam * I.sum(), op.adjoint(r) + lam

    ref = scipy.optimize.minimize(fg, np.zeros(p.n_pix), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * p.n_pix,
                                  options=dict(ftol=1e-15, gtol=1e-12, maxiter=20000))
    assert res.F <= ref.fun + 1e-9 * abs(ref.fun)
    assert abs(res.F - ref.fun) <= 1e-7 * abs(ref.fun)
    assert O.kkt_residual(op, V, res.image, lam) < 1e-6
    assert res.F == pytest.approx(res.l2_term + lam * res.l1_term)


def test_kkt_residual_on_constructed_points():
    """The optimality certificate on points whose violation is known by hand.
    With M the 2 x 2 identity (entries set directly), V = (3, 0.2) and
    lambda = 0.5, G = Re M^H (V - M I) = V - I: at I = (2.5, 0) G = (0.5, 0.2),
    optimal (residual 0); at I = (2, 0) G = (1, 0.2), the support's
    condition G = lambda is off by 0.5; at I = (2.5, 0) with V_2 = 1.3 the
    off-support condition G <= lambda is off by 0.8; at I = (3.5, 0.1) both
    pixels are on the support and G = (-0.5, 0.1) misses lambda by 1.0 and
    0.4, so the residual is 1.0."""
    p = _prob([0.0, 0.1], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0])
    op = O.Operator(p, dense=True)
    op.M = np.eye(2, dtype=np.complex128)
    lam = 0.5
    cases = [((3.0, 0.2), (2.5, 0.0), 0.0),
             ((3.0, 0.2), (2.0, 0.0), 0.5),
             ((3.0, 1.3), (2.5, 0.0), 0.8),
             ((3.0, 0.2), (3.5, 0.1), 1.0)]
    for V, I, want in cases:
        got = O.kkt_residual(op, np.array(V, complex), np.array(I), lam)
        assert abs(got - want) < 1e-14, (V, I, got, want)


def test_fista_rate_bound():
    """Beck & Teboulle: F(I_k) - F* <= 2 L |I_0 - I*|^2 / (k + 1)^2 for all k."""
    p, x = _small_solve_problem(n_vis=25, seed=35, n_src=4)
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    lam = 0.05
    L, _ = O.power_iteration(op, 200)
    star = O.fista(op, V, L, lam, 30000)
    Fstar = star.F
    res = O.fista(op, V, L, lam, 300, keep_history=True)
    for k, I in enumerate(res.history, start=1):
        gap = O.objective(op, V, I, lam)[0] - Fstar
        assert gap <= 2 * L * np.dot(star.image, star.image) / (k + 1) ** 2 + 1e-12


def test_noiseless_sparse_recovery_closed_form():
    """Check (5): noiseless data from a sparse positive sky; once the support S
    is found, I*_S = x_S - lam (Re M_S^H M_S)^{-1} 1, and the dual condition
    holds off the support."""
    p, x = _small_solve_problem(n_side=12, n_vis=300, seed=37, n_src=5)
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    lam = 0.05
    L, _ = O.power_iteration(op, 100)
    res = O.fista(op, V, L, lam, 3000)
    S = np.nonzero(x)[0]
    assert set(np.nonzero(res.image > 1e-9)[0]) == set(S)
    MS = op.M[:, S]
    A = (MS.conj().T @ MS).real
    closed = x[S] - lam * np.linalg.solve(A, np.ones(S.size))
    assert np.all(closed > 0)
    np.testing.assert_allclose(res.image[S], closed, rtol=0, atol=1e-9)
    G = op.adjoint(V - op.forward(res.image))
    off = np.setdiff1d(np.arange(p.n_pix), S)
    assert np.all(G[off] <= lam + 1e-9)


def test_fista_resume_is_exact():
    """(k, t_k, I_{k-1}, y_k) is the complete state: 50 + 50 iterations = 100."""
    p, x = _small_solve_problem(seed=39)
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    L, _ = O.power_iteration(op, 30)
    a = O.fista(op, V, L, 0.2, 100)
    b1 = O.fista(op, V, L, 0.2, 50)
    b2 = O.fista(op, V, L, 0.2, 50, state=b1.state)
    np.testing.assert_array_equal(a.image, b2.image)


def test_termination_by_relative_change():
    """A larger eps stops no later than a smaller one; eps = 0 runs to the cap."""
    p, x = _small_solve_problem(seed=41)
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    L, _ = O.power_iteration(op, 30)
    loose = O.fista(op, V, L, 0.2, 2000, eps=1e-4)
    tight = O.fista(op, V, L, 0.2, 2000, eps=1e-10)
    off = O.fista(op, V, L, 0.2, 300)
    assert loose.converged and loose.iters <= tight.iters
    assert off.iters == 300 and not off.converged


def test_termination_by_nonzero_count():
    """The second stopping rule of Section "Implementation of SL1M" (the
    count of non-zero pixels has nearly settled), brute-forced from the iterate
    history: the run stops at the first check k (every 5 iterations) whose
    count differs from the previous check's by less than nnz_eps times it,
    and returns that iterate."""
    p, x = _small_solve_problem(seed=45)
    op = O.Operator(p, dense=True)
    V = op.forward(x) + 0.01 * np.random.default_rng(46).standard_normal(p.n_vis)
    L, _ = O.power_iteration(op, 30)
    full = O.fista(op, V, L, 0.05, 400, keep_history=True)
    counts = [int(np.count_nonzero(I)) for I in full.history]
    for nnz_eps in (1e-9, 0.05):
        res = O.fista(op, V, L, 0.05, 400, check_every=5, nnz_eps=nnz_eps)
        checks = list(range(5, 401, 5))
        stop = next((k for a, k in zip(checks, checks[1:])
                     if abs(counts[k - 1] - counts[a - 1]) < nnz_eps * max(counts[a - 1], 1)),
                    None)
        assert stop is not None and res.converged == 2 and res.iters == stop
        np.testing.assert_array_equal(res.image, full.history[stop - 1])
    off = O.fista(op, V, L, 0.05, 60, check_every=5)
    assert off.iters == 60 and not off.converged


def test_fista_second_iterate_is_plain_step():
    """t_1 = 1 makes the first extrapolation vanish: y_2 = I_1, so
    I_2 = T^{lam/L}(I_1 - Re M^H (M I_1 - V) / L)."""
    p, x = _small_solve_problem(seed=43)
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    L, _ = O.power_iteration(op, 50)
    lam = 0.1
    res = O.fista(op, V, L, lam, 2, keep_history=True)
    I1 = res.history[0]
    expect = O.threshold_pos(I1 - op.adjoint(op.forward(I1) - V) / L, lam / L)
    np.testing.assert_allclose(res.history[1], expect, rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# warm starts (Section "Acceleration strategies", reading R16)
# --------------------------------------------------------------------------

def test_dirty_image_of_point_source_closed_form():
    """Unit gains, one point source of flux S at pixel s, no noise: every
    |M_ks|^2 = 1/n_s^2, so Re(M^H V)_s / N_v = S / n_s^2 whatever the uv
    coverage; elsewhere the dirty image is the (clipped) normalised beam."""
    rng = np.random.default_rng(41)
    l = rng.uniform(-0.4, 0.4, 30)
    m = rng.uniform(-0.4, 0.4, 30)
    u, v = rng.uniform(-300, 300, (2, 400))
    w = rng.normal(0, 40, 400)
    p = _prob(l, m, u, v, w)
    op = O.Operator(p, dense=True)
    s, S = 7, 2.5
    x = np.zeros(30)
    x[s] = S
    D = O.dirty_image(op, op.forward(x))
    n_s = math.sqrt(1.0 - l[s] ** 2 - m[s] ** 2)
    assert D[s] == pytest.approx(S / n_s ** 2, rel=1e-12)
    # the beam at other pixels: Re sum_k M_kj conj-weighted / N_v, by brute force
    beam = np.array([np.mean((np.conj(op.M[:, j]) * op.M[:, s]).real) for j in range(30)]) * S
    np.testing.assert_allclose(D, np.maximum(beam, 0.0), rtol=0, atol=1e-12)
    assert np.all(D >= 0)


def test_warm_start_at_the_minimiser_stays_there():
    """The LASSO minimiser (certified by KKT) is a fixed point of the
    proximal-gradient step; a warm start from it stays there (y_1 = I_0, and
    the first momentum coefficient is 0).  A start that ignored I_0 would
    move to the first cold iterate instead."""
    p, x = _small_solve_problem(n_vis=60, seed=33)
    op = O.Operator(p, dense=True)
    rng = np.random.default_rng(0)
    V = op.forward(x) + 0.05 * (rng.standard_normal(p.n_vis) + 1j * rng.standard_normal(p.n_vis))
    lam = 0.3
    L, _ = O.power_iteration(op, 100)
    star = O.fista(op, V, L, lam, 4000).image
    assert O.kkt_residual(op, V, star, lam) < 1e-6
    res = O.fista_from(op, V, L, lam, 5, star, keep_history=True)
    for I in res.history:
        np.testing.assert_allclose(I, star, rtol=0, atol=1e-6)
    cold1 = O.fista(op, V, L, lam, 1).image
    assert np.max(np.abs(cold1 - star)) > 1e-3


def test_warm_start_first_iterate_closed_form():
    """From I_0: I_1 = T^{lam/L}(I_0 - Re M^H (M I_0 - V) / L), and the second
    step's y_2 = I_1 (momentum coefficient (t_1 - 1)/t_2 = 0)."""
    p, x = _small_solve_problem()
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    L, _ = O.power_iteration(op, 50)
    lam = 0.5
    I0 = np.abs(np.random.default_rng(5).standard_normal(p.n_pix))
    res = O.fista_from(op, V, L, lam, 2, I0, keep_history=True)
    I1 = O.threshold_pos(I0 - op.adjoint(op.forward(I0) - V) / L, lam / L)
    np.testing.assert_allclose(res.history[0], I1, rtol=1e-13, atol=1e-14)
    I2 = O.threshold_pos(I1 - op.adjoint(op.forward(I1) - V) / L, lam / L)
    np.testing.assert_allclose(res.history[1], I2, rtol=1e-13, atol=1e-14)


# --------------------------------------------------------------------------
# MFISTA (the monotone variant the paper names)
# --------------------------------------------------------------------------

def test_mfista_is_monotone_and_keeps_the_rate_bound():
    """Beck & Teboulle's MFISTA: F(x_k) never increases, and the same
    F(x_k) - F* <= 2 L |x_0 - x*|^2 / (k + 1)^2 bound as FISTA holds."""
    p, x = _small_solve_problem(n_vis=25, seed=35, n_src=4)
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    lam = 0.05
    L, _ = O.power_iteration(op, 200)
    star = O.fista(op, V, L, lam, 30000)
    res = O.mfista(op, V, L, lam, 300, keep_history=True)
    F = [O.objective(op, V, I, lam)[0] for I in res.history]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(F, F[1:]))
    for k, Fk in enumerate(F, start=1):
        assert Fk - star.F <= 2 * L * np.dot(star.image, star.image) / (k + 1) ** 2 + 1e-12
    # plain FISTA on this problem is not monotone, so the test tells them apart
    fi = O.fista(op, V, L, lam, 300, keep_history=True)
    Ff = [O.objective(op, V, I, lam)[0] for I in fi.history]
    assert any(b > a * (1 + 1e-9) for a, b in zip(Ff, Ff[1:]))


def test_mfista_converges_to_the_minimiser():
    """Same limit as FISTA and L-BFGS-B, certified by KKT."""
    p, x = _small_solve_problem(n_vis=60, seed=33)
    op = O.Operator(p, dense=True)
    rng = np.random.default_rng(0)
    V = op.forward(x) + 0.05 * (rng.standard_normal(p.n_vis) + 1j * rng.standard_normal(p.n_vis))
    lam = 0.3
    L, _ = O.power_iteration(op, 100)
    res = O.mfista(op, V, L, lam, 4000)
    assert O.kkt_residual(op, V, res.image, lam) < 1e-6
    ref = O.fista(op, V, L, lam, 4000)
    assert abs(res.F - ref.F) <= 1e-9 * abs(ref.F)


def test_mfista_first_iterate_closed_form():
    """From x_0 = 0: z_1 = T(Re M^H V / L); x_1 = z_1 when F(z_1) <= F(0) =
    |V|^2 / 2 (always here), and y_2 = x_1 (t_1 = 1)."""
    p, x = _small_solve_problem()
    op = O.Operator(p, dense=True)
    V = op.forward(x)
    L, _ = O.power_iteration(op, 50)
    lam = 0.5
    res = O.mfista(op, V, L, lam, 2, keep_history=True)
    z1 = O.threshold_pos(op.adjoint(V) / L, lam / L)
    np.testing.assert_allclose(res.history[0], z1, rtol=1e-14, atol=1e-15)
    z2 = O.threshold_pos(z1 - op.adjoint(op.forward(z1) - V) / L, lam / L)
    x2 = z2 if O.objective(op, V, z2, lam)[0] <= O.objective(op, V, z1, lam)[0] else z1
    np.testing.assert_allclose(res.history[1], x2, rtol=1e-13, atol=1e-14)
