"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the paper's
own definitions evaluated by brute force (TDI delay polynomial), a library
routine that computes the same object (SciPy's Akima interpolator, the Gamma
log-density), closed forms, invariants and exact identities.  A plausible
mistake in the oracle (a dropped term, a wrong sign, index or operand) fails
at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import interpolate, stats

from oracle import lps_oracle as O
from synth import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C = 299792458.0
L = 2.5e9


# ---------------------------------------------------------------------------
# Noise template: brute force from the single-link noise and the X2 definition
# ---------------------------------------------------------------------------

def _tdi_brute_force(f):
    """A/E/T OMS and TM transfer from Eq. (link), the X2 delay polynomial and the
    A/E/T combination of Sec. 'Time-delay Interferometry' (equal arms, 2 pi kept
    in the delay phase).  Returns per-unit-PSD transfers and cross spectra."""
    z = np.exp(-1j * 2 * np.pi * f * L / C)
    pairs = [(1, 2), (2, 1), (1, 3), (3, 1), (2, 3), (3, 2)]
    idx = {}
    for p in pairs:
        idx[("g",) + p] = len(idx)
    for p in pairs:
        idx[("m",) + p] = len(idx)

    def eta(i, j):
        v = np.zeros((len(idx), f.size), complex)
        v[idx[("g", j, i)]] += z      # far test mass, delayed by one arm
        v[idx[("g", i, j)]] += 1.0    # local test mass
        v[idx[("m", i, j)]] += 1.0    # OMS of the link
        return v

    def x2(a, b, c):
        # D_ab D_ba ... with all delays equal to z
        p1 = 1 - z ** 2 - z ** 4 + z ** 6
        return p1 * (eta(a, c) + z * eta(c, a)) - p1 * (eta(a, b) + z * eta(b, a))

    X, Y, Z = x2(1, 2, 3), x2(2, 3, 1), x2(3, 1, 2)
    A = (Z - X) / np.sqrt(2)
    E = (X - 2 * Y + Z) / np.sqrt(6)
    T = (X + Y + Z) / np.sqrt(3)
    out = {}
    for name, v in (("A", A), ("E", E), ("T", T)):
        w = np.abs(v) ** 2
        out[name] = (sum(w[idx[("m",) + p]] for p in pairs), sum(w[idx[("g",) + p]] for p in pairs))
    cross = max(np.abs((A * np.conj(E)).sum(0)).max(), np.abs((A * np.conj(T)).sum(0)).max(),
                np.abs((E * np.conj(T)).sum(0)).max())
    return out, cross


def test_noise_tdi_matches_brute_force_x2():
    f = np.logspace(-4, np.log10(2.9e-2), 41)
    bf, cross = _tdi_brute_force(f)
    A_oms, A_tm = 1.3e-11, 2.7e-15
    oms, tm = O.noise_tdi(f, L, A_oms, A_tm)
    so, st = O.s_oms(f, A_oms), O.s_tm(f, A_tm)
    for c, name in enumerate("AET"):
        np.testing.assert_allclose(oms[c], bf[name][0] * so, rtol=1e-11)
        np.testing.assert_allclose(tm[c], bf[name][1] * st, rtol=1e-11)
    # the A/E/T basis is noise-orthogonal for equal arms
    assert cross < 1e-9 * np.abs(bf["A"][0]).max()


def test_noise_tdi_literal_prefactor_is_rejected():
    """The printed sin^4 prefactor disagrees with the X2 polynomial (reading R1)."""
    f = np.array([1e-3, 1e-2])
    bf, _ = _tdi_brute_force(f)
    xi = 2 * np.pi * f * L / C
    literal = 32 * np.sin(xi) ** 2 * np.sin(xi) ** 4 * (2 + np.cos(xi))
    assert np.all(np.abs(literal / bf["A"][0] - 1) > 0.5)


def test_noise_template_closed_forms():
    f = np.logspace(-4, np.log10(2.9e-2), 200)
    o1, t1 = O.noise_tdi(f, L, 1e-11, 3e-15)
    o2, t2 = O.noise_tdi(f, L, 2e-11, 6e-15)
    # A == E, exact scaling with the squared amplitudes
    assert np.array_equal(o1[0], o1[1]) and np.array_equal(t1[0], t1[1])
    np.testing.assert_allclose(o2, 4 * o1, rtol=1e-14)
    np.testing.assert_allclose(t2, 4 * t1, rtol=1e-14)
    # the transfer vanishes where sin(2 xi) = 0, i.e. f = c / (4 L)
    f0 = np.array([C / (4 * L)])
    o0, t0 = O.noise_tdi(f0, L, 1e-11, 3e-15)
    oref, _ = O.noise_tdi(np.array([1e-3]), L, 1e-11, 3e-15)
    assert np.all(np.abs(o0) < 1e-20 * np.abs(oref).max())
    # single-link shapes: OMS ~ f^2 and TM ~ f^-4 far below their corners
    fl = np.array([1e-6, 2e-6])
    so = O.s_oms(np.array([1.0, 2.0]), 1.0)
    assert abs(so[1] / so[0] - 4.0) < 1e-6
    stl = O.s_tm(fl, 1.0)
    assert abs(stl[1] / stl[0] - 2.0 ** -4) < 1e-3
    # OMS displacement -> fractional frequency: (2 pi f A / c)^2 where the bracket is ~1
    assert abs(O.s_oms(np.array([1.0]), 1e-11)[0] / (2 * np.pi * 1e-11 / C) ** 2 - 1) < 1e-10


def test_sgwb_template_scalings():
    f = np.logspace(-4, np.log10(2.9e-2), 64)
    R = W.response_standin(f)
    s0 = O.sgwb_tdi(f, R, -12.0, 0.0, 1e-3)
    s1 = O.sgwb_tdi(f, R, -11.0, 0.0, 1e-3)
    np.testing.assert_allclose(s1, 10 * s0, rtol=1e-13)
    # S_h / R scales as f^(alpha - 3)
    sa = O.sgwb_tdi(f, R, -12.0, 0.7, 1e-3) / R
    ratio = sa[0, 1:] / sa[0, :-1]
    np.testing.assert_allclose(ratio, (f[1:] / f[:-1]) ** (0.7 - 3.0), rtol=1e-12)
    # at f = f_knee the template does not depend on alpha
    fk = np.array([1e-3])
    Rk = W.response_standin(fk)
    assert np.array_equal(O.sgwb_tdi(fk, Rk, -12.0, 0.9, 1e-3), O.sgwb_tdi(fk, Rk, -12.0, -0.4, 1e-3))
    # H0 = h * 100 km/s/Mpc, printed as ~3.24e-18 h Hz
    assert abs(O.H0_PER_H / 3.24e-18 - 1) < 2e-3


# ---------------------------------------------------------------------------
# Akima spline (App. A)
# ---------------------------------------------------------------------------

def _random_knots(rng, n, lo=-4.0, hi=-1.5):
    x = np.concatenate([[lo], np.sort(rng.uniform(lo, hi, n - 2)), [hi]])
    y = rng.normal(0, 0.1, n)
    return x, y


@pytest.mark.parametrize("n", [4, 5, 6, 7, 11, 22, 42])
def test_akima_equals_scipy(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(20):
        x, y = _random_knots(rng, n)
        xq = np.linspace(x[0], x[-1], 997)
        ref = interpolate.Akima1DInterpolator(x, y)(xq)
        got = O.spline_eval(x, y, xq)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3])
def test_linear_fallback_equals_numpy_interp(n):
    rng = np.random.default_rng(7 + n)
    for _ in range(20):
        x, y = _random_knots(rng, n)
        xq = np.linspace(x[0], x[-1], 501)
        np.testing.assert_allclose(O.spline_eval(x, y, xq), np.interp(xq, x, y), rtol=0, atol=1e-15)


def test_perturbed_noise_spline_fixture():
    g = json.load(open(os.path.join(GOLDEN, "perturbed_noise_spline.json")))
    x, y = np.array(g["log10_f"]), np.array(g["w"])
    xq = np.linspace(x[0], x[-1], 2001)
    ref = interpolate.Akima1DInterpolator(x, y)(xq)
    np.testing.assert_allclose(O.spline_eval(x, y, xq), ref, atol=1e-13)
    np.testing.assert_allclose(O.spline_eval(x, y, x), y, atol=1e-15)


def test_degenerate_weight_reading():
    """All-equal neighbouring slopes: Akima's and SciPy's fill value (reading R2)."""
    x = np.arange(7.0)
    y = np.array([0, 0, 0, 1, 2, 2, 2.0])
    _, s = O.akima_slopes(list(x), list(y))
    np.testing.assert_allclose(s, [0, 0, 0.5, 1, 0.5, 0, 0])
    ref = interpolate.Akima1DInterpolator(x, y).derivative()(x)
    np.testing.assert_allclose(s, ref, atol=1e-14)


def test_spline_invariants():
    rng = np.random.default_rng(5)
    for n in (4, 5, 9, 30):
        x, y = _random_knots(rng, n)
        # interpolation at the knots
        np.testing.assert_allclose(O.spline_eval(x, y, x), y, atol=1e-15)
        # linear data are reproduced exactly
        ylin = 0.3 - 0.7 * x
        xq = np.linspace(x[0], x[-1], 301)
        np.testing.assert_allclose(O.spline_eval(x, ylin, xq), 0.3 - 0.7 * xq, atol=1e-13)
        # equivariance: adding a line to the heights adds the same line
        np.testing.assert_allclose(O.spline_eval(x, y + 0.2 + 0.5 * x, xq),
                                   O.spline_eval(x, y, xq) + 0.2 + 0.5 * xq, atol=1e-13)
        # reflection symmetry x -> -x
        np.testing.assert_allclose(O.spline_eval(-x[::-1], y[::-1], -xq), O.spline_eval(x, y, xq),
                                   atol=1e-13)
        # affine invariance of the abscissa (log10 vs ln and a shift)
        np.testing.assert_allclose(O.spline_eval(x * math.log(10) + 3.0, y, xq * math.log(10) + 3.0),
                                   O.spline_eval(x, y, xq), atol=1e-12)


def test_spline_c1_not_c2():
    rng = np.random.default_rng(11)
    x, y = _random_knots(rng, 9)
    a, b, c, d = O.spline_coeffs(x, y)
    h = np.diff(x)
    # value and first derivative continuous at interior knots, second not
    left_val = a[:-1] + b[:-1] * h[:-1] + c[:-1] * h[:-1] ** 2 + d[:-1] * h[:-1] ** 3
    left_d1 = b[:-1] + 2 * c[:-1] * h[:-1] + 3 * d[:-1] * h[:-1] ** 2
    left_d2 = 2 * c[:-1] + 6 * d[:-1] * h[:-1]
    np.testing.assert_allclose(left_val, a[1:], atol=1e-14)
    np.testing.assert_allclose(left_d1, b[1:], atol=1e-12)
    assert np.max(np.abs(left_d2 - 2 * c[1:])) > 1e-3


def test_spline_locality():
    rng = np.random.default_rng(12)
    n = 12
    x, y = _random_knots(rng, n)
    xq = np.linspace(x[0], x[-1], 2000)
    base = O.spline_eval(x, y, xq)
    idx = O.interval_index(x, xq)
    for j in range(n):
        y2 = y.copy()
        y2[j] += 0.05
        moved = np.abs(O.spline_eval(x, y2, xq) - base) > 0
        # a knot influences intervals i with i-3 <= j <= i+2 ... i.e. j-3 <= i <= j+2
        assert np.all((idx[moved] >= j - 3) & (idx[moved] <= j + 2))


def test_interval_convention():
    x = np.array([-4.0, -3.0, -2.5, -2.0])
    q = np.array([-4.0, -3.0, -2.9999, -2.5, -2.0])
    assert list(O.interval_index(x, q)) == [0, 1, 1, 2, 2]


# ---------------------------------------------------------------------------
# PSD assembly and likelihood
# ---------------------------------------------------------------------------

def _small_dataset(layout="split", n_bins=300, name="grad_25000bins_1024states"):
    ds = W.make_dataset(name, n_bins=n_bins, layout=layout)
    return ds


def _knots(sb, s):
    return [sb.knots(s, j) for j in range(sb.n_spl)]


@pytest.mark.parametrize("layout", ["noise_signal", "split", "split_fg", "paper"])
def test_template_exactness(layout):
    """Disabled or all-zero splines leave the template bit-for-bit unchanged."""
    name = "sweep_250000bins_2048chains" if layout == "split_fg" else "grad_25000bins_1024states"
    ds = _small_dataset(layout, name=name)
    sb = W.make_states(name, ds, n_states=3)
    for s in range(3):
        p = sb.params[:, s]
        kn = _knots(sb, s)
        tmpl = O.template_terms(ds, p)
        expect = (tmpl[0] + tmpl[1]) + (tmpl[2] + tmpl[3])
        zero = [(kx, np.zeros_like(ky)) for (kx, ky) in kn]
        off = [(np.zeros(0), np.zeros(0)) for _ in kn]
        for knots in (zero, off):
            S, _, _ = O.psd(ds, p, knots)
            assert np.array_equal(S, expect)


@pytest.mark.parametrize("layout", ["split", "paper", "noise_signal"])
def test_loglike_matches_gamma_logpdf(layout):
    """D_ck ~ S_ck Gamma(N_k, 1)/N_k: logL differences equal Gamma log-density differences."""
    ds = _small_dataset(layout, n_bins=400)
    S0, _, _ = O.psd(ds, ds.truth.params[:, 0], _knots(ds.truth, 0))
    D = S0 * ds.chi
    sb = W.make_states("grad_25000bins_1024states", ds, n_states=4)
    nk = np.broadcast_to(ds.nk, D.shape)
    ref = []
    got = []
    for s in range(4):
        p, kn = sb.params[:, s], _knots(sb, s)
        S, _, _ = O.psd(ds, p, kn)
        ref.append(math.fsum(stats.gamma.logpdf(D, a=nk, scale=S / nk).ravel()))
        got.append(O.loglike(ds, D, p, kn))
    for s in range(1, 4):
        assert abs((got[s] - got[0]) - (ref[s] - ref[0])) < 1e-7 * max(1.0, abs(ref[s] - ref[0]))


def test_loglike_closed_form_at_noise_free_data():
    ds = _small_dataset("split", n_bins=300)
    p, kn = ds.truth.params[:, 0], _knots(ds.truth, 0)
    S, _, _ = O.psd(ds, p, kn)
    expect = -math.fsum((ds.nk[None, :] * (1.0 + np.log(S))).ravel())
    assert abs(O.loglike(ds, S.copy(), p, kn) - expect) <= 1e-12 * abs(expect)


def test_global_scale_mle():
    """S = kappa S0 is maximised at kappa = sum N D/S0 / sum N (closed form)."""
    ds = _small_dataset("split", n_bins=300)
    p, kn = ds.truth.params[:, 0].copy(), _knots(ds.truth, 0)
    S0, _, _ = O.psd(ds, p, kn)
    D = S0 * ds.chi * 1.37
    nk = np.broadcast_to(ds.nk, D.shape)
    khat = (nk * D / S0).sum() / nk.sum()

    def scaled(k):
        q = p.copy()
        q[0] *= math.sqrt(k)
        q[1] *= math.sqrt(k)
        q[2] += math.log10(k)
        return q

    lhat = O.loglike(ds, D, scaled(khat), kn)
    for k in (khat * 0.999, khat * 1.001, khat * 0.9, khat * 1.1):
        assert O.loglike(ds, D, scaled(k), kn) < lhat
    _, dp, _, _ = O.loglike_grad(ds, D, scaled(khat), kn)
    q = scaled(khat)
    euler = q[0] / 2 * dp[0] + q[1] / 2 * dp[1] + dp[2] / math.log(10)
    assert abs(euler) < 1e-6 * nk.sum()


def test_invalid_states_give_minus_inf():
    ds = _small_dataset("split", n_bins=100)
    sb = W.make_states("grad_25000bins_1024states", ds, n_states=1)
    p, kn = sb.params[:, 0].copy(), _knots(sb, 0)
    D = np.ones((3, 100)) * 1e-40
    bad = list(kn)
    x, y = bad[0]
    bad[0] = (x[::-1].copy(), y)
    assert O.state_status(ds, p, bad) & O.ST_ORDER
    assert O.loglike(ds, D, p, bad) == -math.inf
    bad = list(kn)
    bad[1] = (np.array([-3.0]), np.array([0.0]))
    assert O.state_status(ds, p, bad) & O.ST_COUNT
    bad = list(kn)
    x, y = bad[2]
    bad[2] = (x[1:].copy(), y[1:].copy())
    assert O.state_status(ds, p, bad) & O.ST_COVER
    q = p.copy()
    q[0] = -1.0
    assert O.state_status(ds, q, kn) & O.ST_AMPLITUDE
    q = p.copy()
    q[3] = float("nan")
    assert O.state_status(ds, q, kn) & O.ST_NONFINITE
    assert O.state_status(ds, p, kn) == 0


# ---------------------------------------------------------------------------
# Gradient
# ---------------------------------------------------------------------------

def _grad_case(layout="split", n_bins=240, seed_offset=0):
    name = "sweep_250000bins_2048chains" if layout == "split_fg" else "grad_25000bins_1024states"
    ds = _small_dataset(layout, n_bins=n_bins, name=name)
    S0, _, _ = O.psd(ds, ds.truth.params[:, 0], _knots(ds.truth, 0))
    D = S0 * ds.chi
    sb = W.make_states(name, ds, n_states=2, inbetween=(2, 6), seed_offset=seed_offset)
    return ds, D, sb


@pytest.mark.parametrize("layout", ["split", "paper", "noise_signal", "split_fg"])
def test_gradient_matches_finite_differences(layout):
    ds, D, sb = _grad_case(layout)
    p, kn = sb.params[:, 0].copy(), _knots(sb, 0)
    _, dp, dys, dxs = O.loglike_grad(ds, D, p, kn)
    scales = [p[0], p[1], 1.0, 1.0] + ([1.0] if p.size > 4 else [])
    for i in range(p.size):
        h = 1e-6 * scales[i]
        qp, qm = p.copy(), p.copy()
        qp[i] += h
        qm[i] -= h
        fd = (O.loglike_delta(ds, D, p, kn, qp, kn) - O.loglike_delta(ds, D, p, kn, qm, kn)) / (2 * h)
        assert abs(fd - dp[i]) <= 1e-5 * abs(dp[i]) + 1e-6 * abs(fd) + 1e-3 / scales[i]
    for j, (kx, ky) in enumerate(kn):
        for q in range(len(kx)):
            for which, grad, hh in (("y", dys[j][q], 1e-6), ("x", dxs[j][q], 1e-7)):
                if which == "x" and (q == 0 or q == len(kx) - 1):
                    assert grad == 0.0
                    continue
                kp = [(a.copy(), b.copy()) for (a, b) in kn]
                km = [(a.copy(), b.copy()) for (a, b) in kn]
                arr = 0 if which == "x" else 1
                kp[j][arr][q] += hh
                km[j][arr][q] -= hh
                fd = (O.loglike_delta(ds, D, p, kn, p, kp) - O.loglike_delta(ds, D, p, kn, p, km)) / (2 * hh)
                assert abs(fd - grad) <= 2e-5 * max(abs(grad), abs(fd)) + 2e-3, (which, j, q, fd, grad)


def test_gradient_zero_at_noise_free_truth():
    ds, _, sb = _grad_case("split")
    p, kn = sb.params[:, 0], _knots(sb, 0)
    S, _, _ = O.psd(ds, p, kn)
    logL, dp, dys, dxs = O.loglike_grad(ds, S.copy(), p, kn)
    assert np.all(np.abs(dp * np.array([p[0], p[1], 1, 1])) < 1e-9 * ds.nk.sum())
    for dy, dx in zip(dys, dxs):
        assert np.all(np.abs(dy) < 1e-9 * ds.nk.sum()) and np.all(np.abs(dx) < 1e-8 * ds.nk.sum())
    # and the noise-free truth is a local maximum
    for i, h in ((0, 0.01 * p[0]), (2, 0.01), (3, 0.01)):
        q = p.copy()
        q[i] += h
        assert O.loglike(ds, S, q, kn) < logL


@pytest.mark.parametrize("seed_offset", [0, 1, 2])
def test_gradient_identities(seed_offset):
    """Euler (amplitude scaling), shift and tilt identities from spline equivariance."""
    ds, D, sb = _grad_case("split", seed_offset=seed_offset)
    p, kn = sb.params[:, 1], _knots(sb, 1)
    _, dp, dys, dxs = O.loglike_grad(ds, D, p, kn)
    S, _, _ = O.psd(ds, p, kn)
    rhs = math.fsum((ds.nk[None, :] * (D / S - 1.0)).ravel())
    euler = p[0] / 2 * dp[0] + p[1] / 2 * dp[1] + dp[2] / math.log(10)
    assert abs(euler - rhs) <= 1e-9 * ds.nk.sum() * 3
    ln10 = math.log(10)
    # a common shift of the signal-spline heights acts like u
    assert abs(dys[2].sum() - dp[2]) <= 1e-8 * (abs(dp[2]) + 1)
    # a common shift of the OMS / TM spline heights acts like ln10 A/2 d/dA
    assert abs(dys[0].sum() - ln10 * p[0] / 2 * dp[0]) <= 1e-8 * (abs(dys[0].sum()) + 1)
    assert abs(dys[1].sum() - ln10 * p[1] / 2 * dp[1]) <= 1e-8 * (abs(dys[1].sum()) + 1)
    # a tilt of the signal-spline heights acts like alpha (plus u for the pivot)
    kx = kn[2][0]
    tilt = math.fsum(kx * dys[2])
    expect = dp[3] + math.log10(ds.f_knee) * dp[2]
    assert abs(tilt - expect) <= 1e-8 * (abs(expect) + 1)


def test_cosmic_string_background_has_the_papers_snr():
    """Sec. "Data generation": the cosmic-string background of Eq. (cs) with
    G mu = 1e-13 (flat spectrum), one year of data in the band [1e-4, 2.9e-2] Hz
    at the noise amplitudes of Sec. "Parametrized noise model" (7.9 pm, 2.4 fm),
    has SNR 262 by Eq. (snr).  The response is an
    input here (a stand-in whose normalisation was fitted to that number once and
    is committed in synth/workloads.py); with it fixed, the printed SNR pins the
    absolute scale of S_h = R h^2 Omega 3 (H0/h)^2 / (4 pi^2 f^3) of Eq. (Sh)
    against the noise of Eq. (noise_tdi), which is the only combination of the
    two that the likelihood sees."""
    ds = W.make_dataset("year_912085bins_4096states")
    params = np.array([7.9e-12, 2.4e-15, math.log10(0.55e-11), 0.0])
    assert abs(O.snr(ds, params) - 262.0) < 0.05
