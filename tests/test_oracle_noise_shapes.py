"""Pins of the single-link noise shapes of Sec. "Parametrized noise model".

The oracle's OMS and TM PSDs are checked against the numbers the paper prints
(corner frequencies 2 mHz, 0.4 mHz and 8 mHz; bracket exponents 4, 2 and 4)
without retyping the formulas:

* Asymptotic coefficients are read off the oracle far from every corner
  (where the neglected terms are below 1e-15 relative), and the function is
  then required to be exactly the Laurent polynomial those coefficients
  define at frequencies in between.  The printed shapes are
      OMS:  a_2 f^2 + a_-2 f^-2
      TM:   a_-4 f^-4 + a_-2 f^-2 + a_0 + a_2 f^2,   a_-4 a_2 = a_-2 a_0
  so a wrong bracket exponent leaves the function outside that span, and a
  wrong corner moves a coefficient ratio away from the printed frequency.
* Each bracket equals exactly 2 at its printed corner.
* Log-slopes on both sides of every corner (OMS -2 / +2, TM -4 / -2 / +2).
* The unit conversions (displacement and acceleration to fractional
  frequency) are derived from a sampled sinusoid by numerical
  differentiation, not from the formula.
"""
import math

import numpy as np

from oracle import lps_oracle as O

F_OMS = 2.0e-3      # OMS corner (printed)
F_TM_LO = 0.4e-3    # TM low-frequency corner (printed)
F_TM_HI = 8.0e-3    # TM high-frequency corner (printed)
A_OMS = 7.9e-12     # fiducial amplitudes (printed)
A_TM = 2.4e-15
C = 299792458.0


def _oms(f):
    return O.s_oms(np.asarray(f, dtype=np.float64), A_OMS)


def _tm(f):
    return O.s_tm(np.asarray(f, dtype=np.float64), A_TM)


def _oms_coeffs():
    # a_2 from far above the corner, a_-2 from far below
    a2 = float(_oms(1.0e3) / 1.0e6)
    am2 = float(_oms(1.0e-9) * 1.0e-18)
    return a2, am2


def _tm_coeffs():
    # a_-4 far below both corners, a_2 far above; a_-2 and a_0 from two
    # mid-band frequencies once the outer monomials are removed
    am4 = float(_tm(1.0e-11) * 1.0e-44)
    a2 = float(_tm(1.0e5) / 1.0e10)
    f1, f2 = 1.0e-3, 3.0e-3
    r1 = float(_tm(f1)) - am4 * f1 ** -4 - a2 * f1 ** 2
    r2 = float(_tm(f2)) - am4 * f2 ** -4 - a2 * f2 ** 2
    # r = a_-2 f^-2 + a_0
    am2 = (r1 - r2) / (f1 ** -2 - f2 ** -2)
    a0 = r1 - am2 * f1 ** -2
    return am4, am2, a0, a2


def test_oms_is_the_printed_laurent_polynomial():
    a2, am2 = _oms_coeffs()
    f = np.logspace(-6, 0, 61)
    np.testing.assert_allclose(_oms(f), a2 * f ** 2 + am2 * f ** -2, rtol=1e-13)
    # corner: the two monomials are equal at 2 mHz
    assert abs((am2 / a2) ** 0.25 / F_OMS - 1.0) < 1e-13


def test_tm_is_the_printed_laurent_polynomial():
    am4, am2, a0, a2 = _tm_coeffs()
    f = np.logspace(-6, 0, 61)
    model = am4 * f ** -4 + am2 * f ** -2 + a0 + a2 * f ** 2
    np.testing.assert_allclose(_tm(f), model, rtol=1e-11)
    # product of two brackets: the cross coefficient is fixed by the others
    assert abs(am4 * a2 / (am2 * a0) - 1.0) < 1e-9
    # corners: low bracket 1 + (f1/f)^2, high bracket 1 + (f/f2)^4
    assert abs(math.sqrt(am4 / am2) / F_TM_LO - 1.0) < 1e-11
    assert abs((am2 / a2) ** 0.25 / F_TM_HI - 1.0) < 1e-11


def test_brackets_double_at_their_corners():
    a2, am2 = _oms_coeffs()
    # OMS: the PSD over its high-frequency asymptote is the bracket
    assert abs(float(_oms(F_OMS)) / (a2 * F_OMS ** 2) - 2.0) < 1e-13
    am4, am2t, a0, a2t = _tm_coeffs()
    # TM: S f^2 / a_-2 = [1 + (f1/f)^2] [1 + (f/f2)^4]; divide out the other bracket
    def brackets(f):
        return float(_tm(f)) * f ** 2 / am2t
    hi_at_lo = 1.0 + (a2t / am2t) * F_TM_LO ** 4
    lo_at_hi = 1.0 + (am4 / am2t) / F_TM_HI ** 2
    assert abs(brackets(F_TM_LO) / hi_at_lo - 2.0) < 1e-11
    assert abs(brackets(F_TM_HI) / lo_at_hi - 2.0) < 1e-11


def _log_slope(fn, f, h=1e-4):
    up, dn = float(fn(f * math.exp(h))), float(fn(f * math.exp(-h)))
    return (math.log(up) - math.log(dn)) / (2.0 * h)


def test_asymptotic_log_slopes():
    # OMS: f^-2 below 2 mHz, f^2 above, flat (minimum) at the corner
    assert abs(_log_slope(_oms, 1e-7) + 2.0) < 1e-6
    assert abs(_log_slope(_oms, 10.0) - 2.0) < 1e-6
    assert abs(_log_slope(_oms, F_OMS)) < 1e-6
    # TM: f^-4 below 0.4 mHz, about f^-2 between the corners, f^2 above 8 mHz
    assert abs(_log_slope(_tm, 1e-9) + 4.0) < 1e-6
    assert abs(_log_slope(_tm, math.sqrt(F_TM_LO * F_TM_HI)) + 2.0) < 0.1
    assert abs(_log_slope(_tm, 10.0) - 2.0) < 1e-6
    # at each corner its bracket contributes exactly half of its full slope
    mid_lo = _log_slope(_tm, F_TM_LO) + 2.0    # low bracket: -1, high: +4 (f1/f2)^4 / (...)
    assert abs(mid_lo + 1.0) < 1e-3
    mid_hi = _log_slope(_tm, F_TM_HI) + 2.0    # high bracket: +2, low: -2 (f1/f2)^2 / (...)
    assert abs(mid_hi - 2.0) < 1e-2


def _sampled_power_ratio(order, f0=3e-3, n=200000, cycles=50):
    """Mean square of the order-th time derivative of a unit sinusoid over its
    own mean square: periodic central differences over whole periods (their
    gain sin(w dt)/(w dt) differs from 1 by about 1e-7 at this step)."""
    t = np.arange(n) * (cycles / f0 / n)
    dt = t[1] - t[0]
    x = np.sin(2 * math.pi * f0 * t)
    y = x
    for _ in range(order):
        y = (np.roll(y, -1) - np.roll(y, 1)) / (2.0 * dt)
    return float(np.mean(y ** 2) / np.mean(x ** 2)), f0


def test_unit_conversions_from_sampled_sinusoids():
    # displacement -> fractional frequency: y = (dx/dt) / c
    ratio, f0 = _sampled_power_ratio(1)
    a2, _ = _oms_coeffs()
    assert abs(a2 * f0 ** 2 / A_OMS ** 2 / (ratio / C ** 2) - 1.0) < 1e-5
    # acceleration -> fractional frequency: y = v / c with dv/dt = a, so the
    # acceleration PSD is divided by the power gain of one derivative
    _, am2, _, _ = _tm_coeffs()
    assert abs(am2 * f0 ** -2 / A_TM ** 2 / (1.0 / (ratio * C ** 2)) - 1.0) < 1e-5
