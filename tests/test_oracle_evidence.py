"""Pins of the model-selection oracle (stepping-stone evidence, DIC) against
closed forms: a conjugate Gaussian model whose evidence and tempered
posteriors are known exactly, constant-likelihood identities, and the
effective parameter count of a Gaussian posterior."""
import math

import numpy as np
import pytest

from oracle import evidence as E


def _gaussian_toy(rng, betas, n, d=1.3, sigma=0.4, s0=2.0):
    """Prior N(0, s0^2), likelihood N(d; theta, sigma^2); exact draws from every
    tempered posterior; returns logL[T][n] and the exact log evidence."""
    out = []
    for b in betas:
        lam = 1.0 / s0 ** 2 + b / sigma ** 2
        mu = (b * d / sigma ** 2) / lam
        th = rng.normal(mu, 1.0 / math.sqrt(lam), n)
        out.append(-0.5 * (d - th) ** 2 / sigma ** 2 - 0.5 * math.log(2 * math.pi * sigma ** 2))
    v = s0 ** 2 + sigma ** 2
    log_z = -0.5 * d * d / v - 0.5 * math.log(2 * math.pi * v)
    return np.array(out), log_z


def test_stepping_stone_recovers_the_conjugate_evidence():
    rng = np.random.default_rng(11)
    betas = np.concatenate([[0.0], np.logspace(-4, 0, 24)])
    logL, log_z = _gaussian_toy(rng, betas, 20000)
    est, var, steps = E.stepping_stone(betas, logL)
    assert steps.shape == (betas.size - 1,)
    assert 0 < var < 1e-3
    assert abs(est - log_z) < 5 * math.sqrt(var) + 2e-3, (est, log_z, math.sqrt(var))


def test_stepping_stone_variance_matches_the_spread_of_repeats():
    betas = np.array([0.0, 0.05, 0.3, 1.0])
    est, var = [], []
    for seed in range(40):
        logL, _ = _gaussian_toy(np.random.default_rng(100 + seed), betas, 400)
        e, v, _ = E.stepping_stone(betas, logL)
        est.append(e)
        var.append(v)
    spread = np.var(est)
    assert 0.5 < spread / np.mean(var) < 2.0, (spread, np.mean(var))


def test_each_step_matches_the_ratio_of_tempered_normalisations():
    """E over draws at b of L^(b'-b) = Z_b' / Z_b, Z_b = int L^b prior."""
    d, sigma, s0 = 0.7, 0.5, 1.5

    def log_zb(b):
        if b == 0.0:
            return 0.0
        v = sigma ** 2 / b + s0 ** 2
        return (-0.5 * b * math.log(2 * math.pi * sigma ** 2) + 0.5 * math.log(2 * math.pi * sigma ** 2 / b)
                - 0.5 * d * d / v - 0.5 * math.log(2 * math.pi * v))

    betas = np.array([0.0, 0.2, 0.6, 1.0])
    logL, _ = _gaussian_toy(np.random.default_rng(5), betas, 200000, d=d, sigma=sigma, s0=s0)
    _, var, steps = E.stepping_stone(betas, logL)
    for k in range(1, betas.size):
        exact = log_zb(betas[k]) - log_zb(betas[k - 1])
        assert abs(steps[k - 1] - exact) < 6 * math.sqrt(var) + 1e-4, (k, steps[k - 1], exact)


def test_constant_likelihood_telescopes_exactly():
    betas = np.array([1e-20, 1e-8, 0.3, 1.0])
    c = np.array([-5.0e6, -4.0e6, -1.0e3, 7.0])
    logL = np.repeat(c[:, None], 17, axis=1)
    est, var, steps = E.stepping_stone(betas, logL)
    expect = sum((betas[k] - betas[k - 1]) * c[k - 1] for k in range(1, 4))
    assert abs(est - expect) <= 1e-12 * abs(expect)
    assert abs(var) < 1e-15
    np.testing.assert_allclose(steps, [(betas[k] - betas[k - 1]) * c[k - 1] for k in range(1, 4)], rtol=1e-14)


def test_stepping_stone_handles_huge_log_likelihoods():
    """Tempered weights far outside the double range (logL ~ -1e8, as in the
    paper's year-long data) stay finite: exponentials are relative to the maximum."""
    betas = np.array([0.0, 0.5, 1.0])
    rng = np.random.default_rng(2)
    logL = -2.5e8 + rng.normal(0, 3.0, (3, 1000))
    est, var, _ = E.stepping_stone(betas, logL)
    assert math.isfinite(est) and math.isfinite(var)
    assert abs(est - (-2.5e8)) < 50


def test_dic_of_a_gaussian_posterior_counts_its_parameters():
    """Flat prior, k-dimensional Gaussian likelihood: the posterior is Gaussian,
    D - D(theta_bar) is chi^2 with k degrees of freedom, so p_D = k and
    Var(D) / 2 = k."""
    rng = np.random.default_rng(9)
    k, n = 3, 200000
    d = np.array([0.3, -1.0, 2.0])
    sig = np.array([0.2, 0.5, 1.0])
    th = d + sig * rng.standard_normal((n, k))
    const = -0.5 * np.sum(np.log(2 * np.pi * sig ** 2))
    logL = const - 0.5 * np.sum(((d - th) / sig) ** 2, axis=1)
    th_bar = th.mean(axis=0)
    l_bar = const - 0.5 * np.sum(((d - th_bar) / sig) ** 2)
    mean_d, p_d, dic, var_d = E.dic(logL, l_bar)
    assert abs(p_d - k) < 0.03
    assert abs(var_d / 2 - k) < 0.1
    assert abs(mean_d - (k - 2 * const)) < 0.03
    assert abs(dic - (mean_d + p_d)) < 1e-12


def test_paper_ladder():
    b = E.paper_ladder()
    assert b.shape == (20,)
    assert np.all(np.diff(b) > 0)
    assert b[0] == 1e-20 and b[-1] == 1.0
    # group starts: 1e-20, 1e-12 (rung 5), 1e-5 (rung 15); equal log spacing inside each group
    np.testing.assert_allclose(b[[0, 5, 15]], [1e-20, 1e-12, 1e-5], rtol=1e-12)
    for lo, hi in ((0, 5), (5, 15), (15, 20)):
        steps = np.diff(np.log10(b[lo:hi]))
        np.testing.assert_allclose(steps, steps[0], rtol=1e-9)


def test_library_ladder_equals_the_pinned_oracle_ladder():
    """The library's 20-rung ladder (lps_paper_ladder, a host function) is the
    oracle's pinned ladder of Sec. "MCMC setup"."""
    import os
    lib_path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2507_06300_amd",
                            "liblps.so")
    if not os.path.exists(lib_path):
        pytest.skip("library not built")
    import paper_2507_06300_amd as m
    got = m.paper_ladder()
    want = E.paper_ladder()
    assert got.shape == (20,)
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)
