"""Planted mistakes in the oracle (CPU only) must fail at least one pin.

Each case swaps one oracle function for a plausibly wrong variant, re-runs
the relevant pin test bodies and expects an assertion to fire.
"""
import math

import numpy as np
import pytest

from oracle import lps_oracle as O
import tests.test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _literal_degenerate_slopes(x, y):
    # the printed degenerate fill (m_{i+1} + m_i) / 2 instead of reading R2
    n = len(x)
    m = [(y[i + 1] - y[i]) / (x[i + 1] - x[i]) for i in range(n - 1)]
    w = [abs(m[i + 1] - m[i]) for i in range(n - 2)]
    s = [0.0] * n
    s[0] = (3 * m[0] - m[1]) / 2
    s[n - 1] = (3 * m[n - 2] - m[n - 3]) / 2

    def wt(i, wr, ml, wl, mr):
        if wr + wl == 0.0:
            return (m[i] + m[min(i + 1, n - 2)]) / 2
        return (wr * ml + wl * mr) / (wr + wl)

    s[1] = wt(1, w[1], m[0], w[0], m[1])
    s[n - 2] = wt(n - 2, w[n - 3], m[n - 3], w[n - 4], m[n - 2])
    for i in range(2, n - 2):
        s[i] = wt(i, w[i], m[i - 1], w[i - 2], m[i])
    return m, s


def _literal_boundary_slopes(x, y):
    # the printed right-boundary slope (indices shifted) instead of reading R3:
    # s_{n-2} = (w_{n-4} m_{n-3} + w_{n-3} m_{n-4}) / (w_{n-4} + w_{n-3}), 0-based
    m, s = _ORIG_SLOPES(x, y)
    n = len(x)
    w = [abs(m[i + 1] - m[i]) for i in range(n - 2)]
    den = w[n - 4] + w[n - 3]
    if den != 0.0:
        s[n - 2] = (w[n - 4] * m[n - 3] + w[n - 3] * m[n - 4]) / den
    return m, s


_ORIG_SLOPES = O.akima_slopes


def test_mutation_degenerate_weight(monkeypatch):
    monkeypatch.setattr(O, "akima_slopes", _literal_degenerate_slopes)
    assert _fails(pins.test_degenerate_weight_reading)


def test_mutation_boundary_slope(monkeypatch):
    monkeypatch.setattr(O, "akima_slopes", _literal_boundary_slopes)
    assert _fails(pins.test_akima_equals_scipy, 7)


def test_mutation_tdi_prefactor(monkeypatch):
    orig = O.noise_tdi

    def wrong(f, L, A_oms, A_tm):
        oms, tm = orig(f, L, A_oms, A_tm)
        xi = 2 * math.pi * f * L / O.C_LIGHT
        r = np.sin(xi) ** 4 / np.sin(2 * xi) ** 2       # sin^4 read literally
        return oms * r, tm * r

    monkeypatch.setattr(O, "noise_tdi", wrong)
    assert _fails(pins.test_noise_tdi_matches_brute_force_x2)


def test_mutation_tm_bracket(monkeypatch):
    orig = O.noise_tdi

    def wrong(f, L, A_oms, A_tm):
        oms, tm = orig(f, L, A_oms, A_tm)
        xi = 2 * math.pi * f * L / O.C_LIGHT
        cx = np.cos(xi)
        tm = tm.copy()
        tm[:2] *= (1 + cx) / (1 + cx + cx ** 2)          # dropped cos^2 term
        return oms, tm

    monkeypatch.setattr(O, "noise_tdi", wrong)
    assert _fails(pins.test_noise_tdi_matches_brute_force_x2)


def test_mutation_dropped_segment_weight(monkeypatch):
    orig = O.loglike

    def wrong(ds, D, params, knots, k_max=64):
        if O.state_status(ds, params, knots, k_max):
            return -math.inf
        S, _, _ = O.psd(ds, params, knots)
        return -math.fsum((D / S + np.log(S)).ravel())   # N_k dropped

    monkeypatch.setattr(O, "loglike", wrong)
    assert _fails(pins.test_loglike_matches_gamma_logpdf, "split")


def test_mutation_inverted_ratio(monkeypatch):
    def wrong(ds, D, params, knots, k_max=64):
        S, _, _ = O.psd(ds, params, knots)
        return -math.fsum((ds.nk[None, :] * (S / D + np.log(S))).ravel())   # S/D for D/S

    monkeypatch.setattr(O, "loglike", wrong)
    assert _fails(pins.test_loglike_matches_gamma_logpdf, "split")


def test_mutation_gradient_sign(monkeypatch):
    orig = O.loglike_grad

    def wrong(ds, D, params, knots, k_max=64):
        logL, dp, dy, dx = orig(ds, D, params, knots, k_max)
        return logL, dp, dy, [-v for v in dx]               # wrong sign of dt/dx_i

    monkeypatch.setattr(O, "loglike_grad", wrong)
    assert _fails(pins.test_gradient_matches_finite_differences, "split")


def test_mutation_alpha_pivot(monkeypatch):
    orig = O.sgwb_tdi

    def wrong(f, R, u, alpha, f_knee):
        return orig(f, R, u, alpha, 1.0)                    # pivot frequency ignored

    monkeypatch.setattr(O, "sgwb_tdi", wrong)
    assert _fails(pins.test_sgwb_template_scalings)


@pytest.mark.parametrize("factor", [4.0 * math.pi ** 2, 3.0, 0.5])
def test_mutation_sgwb_constant(monkeypatch, factor):
    orig = O.sgwb_tdi

    def wrong(f, R, u, alpha, f_knee):
        return orig(f, R, u, alpha, f_knee) * factor       # 4 pi^2 or 3 dropped, a one-sided/two-sided slip

    monkeypatch.setattr(O, "sgwb_tdi", wrong)
    assert _fails(pins.test_cosmic_string_background_has_the_papers_snr)


def test_mutation_route_transposed(monkeypatch):
    orig = O.perturbed_terms

    def wrong(ds, params, knots):
        terms = O.template_terms(ds, params)
        P = O.spline_values(ds, knots)
        out = terms.copy()
        for tau in range(4):
            for c in range(3):
                j = ds.route[tau][c]
                if j >= 0:
                    out[tau, c] = terms[tau, c] * 10.0 ** P[(j + 1) % len(P)]   # wrong spline
        return out

    monkeypatch.setattr(O, "perturbed_terms", wrong)
    assert _fails(pins.test_gradient_matches_finite_differences, "split")


# --- full-covariance oracle (reading X1) ---------------------------------
import oracle.covariance as CV  # noqa: E402
import tests.test_oracle_covariance as cpins  # noqa: E402


def _cov_pins_fail():
    bodies = [cpins.test_zero_correlation_is_the_diagonal_likelihood,
              cpins.test_vine_is_positive_definite_with_the_given_partial_correlation,
              cpins.test_wishart_term_is_stationary_at_the_model,
              lambda: [cpins.test_one_correlated_pair_is_a_2x2_block(p) for p in ((0, 1), (0, 2), (1, 2))]]
    return any(_fails(b) for b in bodies)


def test_mutation_cov_pair_order(monkeypatch):
    monkeypatch.setattr(CV, "PAIRS", ((0, 0), (1, 1), (2, 2), (0, 2), (0, 1), (1, 2)))
    assert _cov_pins_fail()


def test_mutation_cov_vine_sign(monkeypatch):
    def vine(q0, q1, q2):
        r01, r02, p12 = np.tanh(q0), np.tanh(q1), np.tanh(q2)
        return r01, r02, -r01 * r02 + p12 * np.sqrt((1 - r01 * r01) * (1 - r02 * r02))
    monkeypatch.setattr(CV, "vine_correlations", vine)
    assert _cov_pins_fail()


def test_mutation_cov_signal_off_diagonal(monkeypatch):
    orig = CV.covariance

    def cov(cds, params, knots):
        C, sn, sh = orig(cds, params, knots)
        C = C.copy()
        C[:, 0, 1] += 0.1 * sh[0]
        C[:, 1, 0] += 0.1 * sh[0]
        return C, sn, sh
    monkeypatch.setattr(CV, "covariance", cov)
    assert _cov_pins_fail()


def test_mutation_cov_data_transposed_half(monkeypatch):
    def dm(P6):
        M = np.zeros((P6.shape[1], 3, 3))
        for i, (a, b) in enumerate(CV.PAIRS):
            M[:, a, b] = P6[i]
        return M            # lower triangle left empty
    monkeypatch.setattr(CV, "data_matrix", dm)
    assert _cov_pins_fail()


def _cov_grad_pins_fail():
    bodies = [lambda: cpins.test_gradient_matches_finite_differences("paper"),
              cpins.test_gradient_vanishes_at_the_model]
    return any(_fails(b) for b in bodies)


def _tangent_with(mistake):
    """A copy of the covariance tangent with one planted mistake."""
    def tangent(sn, dsn, dsh, q, dq):
        r01, r02, r12 = CV.vine_correlations(q[0], q[1], q[2])
        p12 = np.tanh(q[2])
        dr01 = (1.0 - r01 * r01) * dq[0]
        dr02 = (1.0 - r02 * r02) * dq[1]
        dp12 = dq[2] if mistake == "no_tanh_factor" else (1.0 - p12 * p12) * dq[2]
        S = np.sqrt((1.0 - r01 * r01) * (1.0 - r02 * r02))
        dS = -(r01 * dr01 * (1.0 - r02 * r02) + r02 * dr02 * (1.0 - r01 * r01)) / S
        if mistake == "no_dS":
            dS = 0.0 * dS
        dr12 = dr01 * r02 + r01 * dr02 + dp12 * S + p12 * dS
        K = sn.shape[1]
        dC = np.zeros((K, 3, 3))
        for c in range(3):
            dC[:, c, c] = dsn[c] + dsh[c]
        for (a, b), (rv, drv) in {(0, 1): (r01, dr01), (0, 2): (r02, dr02), (1, 2): (r12, dr12)}.items():
            hs = np.sqrt(sn[a] * sn[b])
            bb = a if mistake == "half_index" else b
            dhs = (dsn[a] * sn[bb] + sn[a] * dsn[b]) / (2.0 * hs)
            dC[:, a, b] = dC[:, b, a] = drv * hs + rv * dhs
        return dC
    return tangent


@pytest.mark.parametrize("mistake", ["no_dS", "no_tanh_factor", "half_index"])
def test_mutation_cov_gradient(monkeypatch, mistake):
    monkeypatch.setattr(CV, "_covariance_tangent", _tangent_with(mistake))
    assert _cov_grad_pins_fail()


def test_mutation_cov_gradient_copy_is_faithful(monkeypatch):
    """The mutation copy without a mistake passes the pins (so a failure above
    comes from the planted mistake alone)."""
    monkeypatch.setattr(CV, "_covariance_tangent", _tangent_with(None))
    assert not _cov_grad_pins_fail()


# ---------------------------------------------------------------------------
# Single-link noise shapes: corner frequencies and bracket exponents
# ---------------------------------------------------------------------------

import tests.test_oracle_noise_shapes as shapes   # noqa: E402

_SHAPE_PINS = [shapes.test_oms_is_the_printed_laurent_polynomial, shapes.test_tm_is_the_printed_laurent_polynomial,
               shapes.test_brackets_double_at_their_corners, shapes.test_asymptotic_log_slopes]


def _shape_pins_fail():
    return any(_fails(p) for p in _SHAPE_PINS)


def _tm_variant(f_lo, f_hi, hi_exp):
    def s_tm(f, A_tm):
        return (A_tm ** 2 * (1.0 + (f_lo / f) ** 2) * (1.0 + (f / f_hi) ** hi_exp)
                * (1.0 / (2.0 * math.pi * f * O.C_LIGHT)) ** 2)
    return s_tm


def _oms_variant(f_c, exp):
    def s_oms(f, A_oms):
        return A_oms ** 2 * (1.0 + (f_c / f) ** exp) * (2.0 * math.pi * f / O.C_LIGHT) ** 2
    return s_oms


def test_shape_pins_pass_on_faithful_copies(monkeypatch):
    # the variant builders reproduce the oracle exactly at the printed values
    monkeypatch.setattr(O, "s_tm", _tm_variant(0.4e-3, 8.0e-3, 4))
    monkeypatch.setattr(O, "s_oms", _oms_variant(2.0e-3, 4))
    assert not _shape_pins_fail()


@pytest.mark.parametrize("variant", [(0.4e-3, 8.0e-3, 2),    # high bracket (f / 8 mHz)^2
                                     (0.4e-3, 4.0e-3, 4),    # high corner 4 mHz
                                     (4.0e-3, 8.0e-3, 4)])   # low corner 4 mHz
def test_mutation_tm_shape(monkeypatch, variant):
    monkeypatch.setattr(O, "s_tm", _tm_variant(*variant))
    assert _shape_pins_fail()


@pytest.mark.parametrize("variant", [(3.0e-3, 4),            # OMS corner 3 mHz
                                     (2.0e-3, 2)])           # OMS bracket exponent 2
def test_mutation_oms_shape(monkeypatch, variant):
    monkeypatch.setattr(O, "s_oms", _oms_variant(*variant))
    assert _shape_pins_fail()
