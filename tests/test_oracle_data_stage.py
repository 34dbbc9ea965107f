"""Pins of the data-stage oracle: Parseval's theorem, a pure tone, white-noise
levels with and without a window, the Gamma law of averaged periodograms, the
orthonormal XYZ -> AET map, and exact interpolation of power laws."""
import math

import numpy as np

from oracle import data_stage as DS


def test_parseval_total_power():
    rng = np.random.default_rng(1)
    for n in (1000, 1001):
        x = rng.normal(0, 2.0, (3, n))
        dt = 5.0
        f, P = DS.periodogram(x, dt)
        df = 1.0 / (n * dt)
        np.testing.assert_allclose(P.sum(axis=1) * df, np.mean(x * x, axis=1), rtol=1e-12)
        assert f[1] == df


def test_pure_tone_lands_in_one_bin():
    n, dt, k0, a = 4096, 2.0, 37, 1.7
    t = np.arange(n)
    x = a * np.cos(2 * np.pi * k0 * t / n + 0.3)
    f, P = DS.periodogram(x[None, :], dt)
    assert abs(P[0, k0] - dt * a * a * n / 2) <= 1e-10 * P[0, k0]
    others = np.delete(P[0], k0)
    assert others.max() < 1e-20 * P[0, k0]


def test_white_noise_level_with_and_without_window():
    rng = np.random.default_rng(2)
    n, dt, sig = 1 << 16, 0.5, 3.0
    x = rng.normal(0, sig, (1, n))
    level = 2 * sig * sig * dt
    for w in (None, np.hanning(n)):
        _, P = DS.periodogram(x, dt, window=w)
        m = P[0, 1:-1].mean()
        assert abs(m / level - 1) < 0.02, m / level


def test_averaged_periodogram_follows_the_gamma_law():
    """nu D / S ~ Gamma(nu, 1) for Gaussian white noise: mean S, variance S^2 / nu."""
    rng = np.random.default_rng(3)
    n, dt, sig, nu = 1 << 18, 1.0, 1.0, 16
    x = rng.normal(0, sig, (1, n))
    f, P = DS.periodogram(x, dt)
    n_seg = (f.size - 2) // nu
    fs, D, nus = DS.average_segments(f, P, 1, nu, n_seg)
    S = 2 * sig * sig * dt
    assert np.all(nus == nu)
    assert abs(D.mean() / S - 1) < 0.01
    assert abs(D.var() / (S * S / nu) - 1) < 0.05
    np.testing.assert_allclose(fs, [f[1 + i * nu:1 + (i + 1) * nu].mean() for i in range(n_seg)], rtol=1e-14)


def test_average_of_constant_and_bounds():
    f = np.arange(100) * 0.01
    P = np.full((2, 100), 7.25)
    fs, D, nu = DS.average_segments(f, P, 3, 10, 9)
    assert np.all(D == 7.25) and np.all(nu == 10)
    np.testing.assert_allclose(fs, [np.mean(f[3 + 10 * i:13 + 10 * i]) for i in range(9)], rtol=1e-14)


def test_xyz_to_aet_is_orthonormal():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(3, 50))
    a = DS.xyz_to_aet(x)
    np.testing.assert_allclose((a * a).sum(axis=0), (x * x).sum(axis=0), rtol=1e-13)
    s = rng.normal(size=50)
    a = DS.xyz_to_aet(np.stack([s, s, s]))
    assert np.abs(a[:2]).max() < 1e-14
    np.testing.assert_allclose(a[2], math.sqrt(3) * s, rtol=1e-14)


def test_response_interpolation():
    gf = np.logspace(np.log10(5e-6), -1, 60)
    R = np.stack([3.0 * gf ** 2.5, 0.5 * gf ** -1.0])
    f = np.logspace(-5, -1.2, 333)
    out = DS.interp_response(gf, R, f)
    np.testing.assert_allclose(out[0], 3.0 * f ** 2.5, rtol=1e-12)
    np.testing.assert_allclose(out[1], 0.5 / f, rtol=1e-12)
    np.testing.assert_allclose(DS.interp_response(gf, R, gf), R, rtol=1e-12)
    # a vanishing node: linear in R on the log-f axis
    R0 = R[:1].copy()
    R0[0, 10] = 0.0
    fm = math.exp(0.5 * (math.log(gf[10]) + math.log(gf[11])))
    assert abs(DS.interp_response(gf, R0, [fm])[0, 0] - 0.5 * R0[0, 11]) < 1e-15 + 1e-12 * R0[0, 11]
    assert np.isnan(DS.interp_response(gf, R, [1e-6, 0.2])).all()
