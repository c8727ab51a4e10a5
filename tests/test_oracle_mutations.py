"""Plant plausible mistakes in the oracle (on the CPU) and show that at least
one pin in test_oracle_pins.py fails for each of them."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.sl1m_oracle as OM
import test_oracle_pins as P


def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def _delta_no_alpha(p, ks, js):
    l, m = p.l[js][None, :], p.m[js][None, :]
    u, v, w = p.u[ks][:, None], p.v[ks][:, None], p.w[ks][:, None]
    n = OM.n_of(l, m)
    return np.exp(-2j * np.pi * (u * l + v * m + w * (n - 1.0)))


def _delta_w_sign(p, ks, js):
    l, m = p.l[js][None, :], p.m[js][None, :]
    u, v, w = p.u[ks][:, None], p.v[ks][:, None], p.w[ks][:, None]
    n = OM.n_of(l, m)
    return (1.0 / n) * np.exp(-2j * np.pi * (u * l + v * m + w * (1.0 - n)))


def _delta_conj(p, ks, js):
    l, m = p.l[js][None, :], p.m[js][None, :]
    u, v, w = p.u[ks][:, None], p.v[ks][:, None], p.w[ks][:, None]
    n = OM.n_of(l, m)
    return (1.0 / n) * np.exp(2j * np.pi * (u * l + v * m + w * (n - 1.0)))


def _delta_lm_swap(p, ks, js):
    l, m = p.m[js][None, :], p.l[js][None, :]
    u, v, w = p.u[ks][:, None], p.v[ks][:, None], p.w[ks][:, None]
    n = OM.n_of(l, m)
    return (1.0 / n) * np.exp(-2j * np.pi * (u * l + v * m + w * (n - 1.0)))


def _gauss_wide_minus(p, ks, js):
    l, m = p.l[js][None, :], p.m[js][None, :]
    w = p.w[ks][:, None]
    n = OM.n_of(l, m)
    corr = np.exp(-2j * np.pi * w * (n - 1.0 - (l * l + m * m) / 2.0))
    return OM.gauss_paraxial_block(p, ks, js) * corr


def _gauss_no_den_in_taper(p, ks, js):
    l, m = p.l[js][None, :], p.m[js][None, :]
    s2 = (p.sigma[js] ** 2)[None, :]
    u, v, w = p.u[ks][:, None], p.v[ks][:, None], p.w[ks][:, None]
    n = OM.n_of(l, m)
    den = 1.0 - 1j * w * s2
    e1 = np.exp(-2j * np.pi * (l * u + m * v) / den)
    e2 = np.exp(1j * np.pi * w * (l * l + m * m) / den)
    e3 = np.exp(-np.pi * s2 * (u * u + v * v))
    return (1.0 / n) / den * e1 * e2 * e3


@pytest.mark.parametrize("mutant,pins", [
    (_delta_no_alpha, ["test_delta_entries_by_hand", "test_projection_weight_integrates_to_solid_angle",
                       "test_delta_phase_is_geometric_delay"]),
    (_delta_w_sign, ["test_delta_entries_by_hand", "test_delta_phase_is_geometric_delay"]),
    (_delta_conj, ["test_delta_entries_by_hand", "test_w0_regular_grid_matches_fft2"]),
    (_delta_lm_swap, ["test_delta_entries_by_hand", "test_delta_phase_is_geometric_delay"]),
])
def test_delta_mutations_are_caught(monkeypatch, mutant, pins):
    monkeypatch.setattr(OM, "delta_block", mutant)
    for name in pins:
        assert _fails(getattr(P, name)), f"{mutant.__name__} not caught by {name}"


def test_gaussian_mutations_are_caught(monkeypatch):
    orig = OM.gauss_paraxial_block

    def printed_prefactor(p, ks, js):
        return orig(p, ks, js) / (p.sigma[js] ** 2)[None, :]

    monkeypatch.setattr(OM, "gauss_paraxial_block", printed_prefactor)
    assert _fails(P.test_gaussian_by_hand)
    assert _fails(P.test_gaussian_paraxial_matches_quadrature_of_eq_samlm3)
    monkeypatch.setattr(OM, "gauss_paraxial_block", orig)

    monkeypatch.setattr(OM, "gauss_wide_block", _gauss_wide_minus)
    assert _fails(P.test_gaussian_limits)
    assert _fails(P.test_gaussian_wide_matches_exact_integral_within_bound)
    monkeypatch.undo()

    monkeypatch.setattr(OM, "gauss_paraxial_block", _gauss_no_den_in_taper)
    assert _fails(P.test_gaussian_paraxial_matches_quadrature_of_eq_samlm3)


def test_gain_mutation_is_caught(monkeypatch):
    orig = OM.gain_block

    def no_conj(p, ks, js):
        """E_p E_q instead of E_p conj(E_q)."""
        g = orig(p, ks, js)
        if g is None:
            return None
        c = np.asarray(p.ant_gain)[np.asarray(p.ant_q)[ks]]
        return g * (c / np.conj(c))[:, None]

    monkeypatch.setattr(OM, "gain_block", no_conj)
    assert _fails(P.test_gain_power_beam_fwhm_and_reductions)


def test_pair_beam_width_mutation_is_caught(monkeypatch):
    """A pair gain that takes antenna p's beam width for both voltage
    patterns (g = c_p conj(c_q) exp(-4 ln2 r^2 / F_p^2))."""
    def one_width(p, ks, js):
        if p.ant_p is None:
            return None
        ap = np.asarray(p.ant_p)[ks]
        aq = np.asarray(p.ant_q)[ks]
        c = np.asarray(p.ant_gain, np.complex128)
        F = np.asarray(p.ant_fwhm, np.float64)
        r2 = (p.l[js] ** 2 + p.m[js] ** 2)[None, :]
        return (c[ap] * np.conj(c[aq]))[:, None] * np.exp(-4 * math.log(2) * r2 / F[ap][:, None] ** 2)

    monkeypatch.setattr(OM, "gain_block", one_width)
    assert _fails(P.test_gain_with_distinct_beam_widths_is_a_product_of_voltage_patterns)


def test_kkt_residual_mutations_are_caught(monkeypatch):
    """A certificate that always reports 0, and one that forgets the
    off-support condition."""
    for mod in (O, OM):
        monkeypatch.setattr(mod, "kkt_residual", lambda op, V, I, lam: 0.0)
    assert _fails(P.test_kkt_residual_on_constructed_points)
    monkeypatch.undo()

    def on_support_only(op, V, I, lam):
        G = op.adjoint(np.asarray(V, np.complex128) - op.forward(I))
        on = I > 0
        return float(np.max(np.abs(G[on] - lam))) if np.any(on) else 0.0

    for mod in (O, OM):
        monkeypatch.setattr(mod, "kkt_residual", on_support_only)
    assert _fails(P.test_kkt_residual_on_constructed_points)


def test_adjoint_mutation_is_caught(monkeypatch):
    def adjoint_cols_noconj(p, r, js=None):
        r = np.asarray(r, np.complex128)
        js = np.arange(p.n_pix) if js is None else np.asarray(js)
        out = np.zeros(js.shape[0])
        for a in range(0, p.n_vis, 512):
            kb = np.arange(a, min(a + 512, p.n_vis))
            out += (r[kb] @ OM.matrix_block(p, kb, js)).real
        return out

    monkeypatch.setattr(O, "adjoint", lambda p, r: adjoint_cols_noconj(p, r))
    assert _fails(P.test_adjoint_identity, O.PIX_DELTA, 0.0, False, False)


def _make_fista(step_sign=1.0, momentum="ok", thr_sign=1.0):
    def fista(op, V, L, lam, n_iter, eps=0.0, check_every=1, keep_history=False, state=None):
        op = OM._as_op(op)
        t, Ip, y = 1.0, np.zeros(op.n_pix), np.zeros(op.n_pix)
        hist = []
        I = Ip
        for _ in range(n_iter):
            g = op.adjoint(op.forward(y) - V)
            z = y - step_sign * g / L
            I = np.where(z > thr_sign * lam / L, z - thr_sign * lam / L, 0.0)
            tn = (1 + math.sqrt(1 + 4 * t * t)) / 2
            if momentum == "ok":
                beta = (t - 1) / tn
            elif momentum == "none":
                beta = 0.0
            else:
                beta = (tn - 1) / tn
            y = I + beta * (I - Ip)
            Ip, t = I, tn
            hist.append(I.copy())
        F, l2, l1 = OM.objective(op, V, I, lam)
        return OM.FistaResult(image=I, iters=n_iter, L=L, F=F, l2_term=l2, l1_term=l1,
                              nnz=int(np.count_nonzero(I)), converged=False, history=hist,
                              state=(n_iter, t, Ip, y))
    return fista


@pytest.mark.parametrize("kw,pins", [
    (dict(momentum="none"), ["test_fista_rate_bound"]),
    (dict(momentum="index"), ["test_fista_second_iterate_is_plain_step"]),
    (dict(thr_sign=-1.0), ["test_fista_first_iterate_closed_form",
                           "test_fista_converges_to_library_minimiser_and_satisfies_kkt"]),
])
def test_fista_mutations_are_caught(monkeypatch, kw, pins):
    bad = _make_fista(**kw)
    monkeypatch.setattr(O, "fista", bad)
    monkeypatch.setattr(OM, "fista", bad)
    for name in pins:
        assert _fails(getattr(P, name)), f"{kw} not caught by {name}"


def test_warm_start_mutations_are_caught(monkeypatch):
    """A dirty image normalised by 2 N_v, or without its clip, and a warm start
    that ignores I_0 (starts from y_1 = 0) are each caught."""
    def dirty_half(op, V):
        op = OM._as_op(op)
        return np.maximum(op.adjoint(np.asarray(V, np.complex128)) / (2 * op.p.n_vis), 0.0)

    monkeypatch.setattr(O, "dirty_image", dirty_half)
    assert _fails(P.test_dirty_image_of_point_source_closed_form)
    monkeypatch.undo()

    def dirty_noclip(op, V):
        op = OM._as_op(op)
        return op.adjoint(np.asarray(V, np.complex128)) / op.p.n_vis

    monkeypatch.setattr(O, "dirty_image", dirty_noclip)
    assert _fails(P.test_dirty_image_of_point_source_closed_form)
    monkeypatch.undo()

    def from_zero(op, V, L, lam, n_iter, I0, **kw):
        return OM.fista(op, V, L, lam, n_iter, **kw)

    monkeypatch.setattr(O, "fista_from", from_zero)
    assert _fails(P.test_warm_start_at_the_minimiser_stays_there)
    assert _fails(P.test_warm_start_first_iterate_closed_form)


def _make_mfista(select=True, flip=False):
    def mfista(op, V, L, lam, n_iter, I0=None, keep_history=False):
        op = OM._as_op(op)
        V = np.asarray(V, np.complex128)
        x = np.zeros(op.n_pix) if I0 is None else np.asarray(I0, float).copy()
        y, t = x.copy(), 1.0
        Fx = OM.objective(op, V, x, lam)[0]
        hist = []
        for _ in range(n_iter):
            z = OM.threshold_pos(y - op.adjoint(op.forward(y) - V) / L, lam / L)
            tn = (1 + math.sqrt(1 + 4 * t * t)) / 2
            Fz = OM.objective(op, V, z, lam)[0]
            take = (Fz >= Fx) if flip else (Fz <= Fx)
            xn = z if (take or not select) else x
            y = xn + (t / tn) * (z - xn) + ((t - 1) / tn) * (xn - x)
            x, t, Fx = xn, tn, (min(Fz, Fx) if select else Fz)
            hist.append(x.copy())
        F, l2, l1 = OM.objective(op, V, x, lam)
        return OM.FistaResult(image=x, iters=n_iter, L=L, F=F, l2_term=l2, l1_term=l1,
                              nnz=int(np.count_nonzero(x)), converged=False, history=hist,
                              state=None)
    return mfista


@pytest.mark.parametrize("kw,pin", [
    (dict(select=False), "test_mfista_is_monotone_and_keeps_the_rate_bound"),
    (dict(flip=True), "test_mfista_is_monotone_and_keeps_the_rate_bound"),
])
def test_mfista_mutations_are_caught(monkeypatch, kw, pin):
    monkeypatch.setattr(O, "mfista", _make_mfista(**kw))
    assert _fails(getattr(P, pin)), f"{kw} not caught by {pin}"
