"""The device sampler at beta > 0 against the oracle's tempered posterior.

Splines disabled (knot count 0, no birth/death) and A_OMS, A_TM held fixed,
so the only free parameters are the background amplitude u and slope alpha
of Eq. (pl).  Each rung of a two-temperature run (beta = 1 and 0.3) must
sample L(u, alpha)^beta pi(u, alpha) (pi uniform over the sampler's Table I
box), where L is the oracle's likelihood evaluated on a fine grid.  Compared:
the means and variances of both marginals and their correlation (tolerances
from the effective sample size, estimated from the chains' integrated
autocorrelation time) and a Kolmogorov-Smirnov test of each marginal on draws
thinned by that time.  Run with Langevin moves alone and with the ensemble
stretch moves added.  A third test runs two rungs at equal beta, whose swaps
must all be accepted.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import lps_oracle as O
from synth import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAME = "avg50_1000bins_64states"
TRUTH_U, TRUTH_ALPHA = -11.3, 0.4


@pytest.fixture(scope="module")
def lps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def problem():
    """Dataset, data and the oracle's log-likelihood on a grid around the mode."""
    ds = W.make_dataset(NAME, n_bins=400, layout="split")
    none = [(np.zeros(0), np.zeros(0))] * ds.n_spl
    a_oms, a_tm = float(ds.truth.params[0, 0]), float(ds.truth.params[1, 0])
    S0, _, _ = O.psd(ds, np.array([a_oms, a_tm, TRUTH_U, TRUTH_ALPHA]), none)
    D = S0 * ds.chi

    def ll(u, a):
        return O.loglike(ds, D, np.array([a_oms, a_tm, u, a]), none)

    # coarse scan for the mode, then a fine grid over +-9 sd of the beta = 0.3 posterior
    us = np.linspace(-12.0, -10.6, 29)
    al = np.linspace(-1.0, 1.8, 29)
    Gc = np.array([[ll(u, a) for a in al] for u in us])
    i, j = np.unravel_index(np.argmax(Gc), Gc.shape)
    u0, a0 = us[i], al[j]
    gu = np.linspace(u0 - 0.4, u0 + 0.4, 161)
    ga = np.linspace(a0 - 1.0, a0 + 1.0, 161)
    G = np.array([[ll(u, a) for a in ga] for u in gu])
    return dict(ds=ds, D=D, none=none, a_oms=a_oms, a_tm=a_tm, gu=gu, ga=ga, G=G)


def _grid_moments(pb, beta):
    P = np.exp(beta * (pb["G"] - pb["G"].max()))
    P /= P.sum()
    gu, ga = pb["gu"], pb["ga"]
    # the posterior must vanish at the grid border (the grid covers it)
    assert P[0, :].sum() + P[-1, :].sum() + P[:, 0].sum() + P[:, -1].sum() < 1e-9
    pu, pa = P.sum(1), P.sum(0)
    mu_u, mu_a = (pu * gu).sum(), (pa * ga).sum()
    var_u, var_a = (pu * (gu - mu_u) ** 2).sum(), (pa * (ga - mu_a) ** 2).sum()
    cov = (P * np.outer(gu - mu_u, ga - mu_a)).sum()
    return dict(P=P, pu=pu, pa=pa, mu=(mu_u, mu_a), var=(var_u, var_a), corr=cov / math.sqrt(var_u * var_a))


def _grid_cdf(grid, p):
    """CDF of a marginal tabulated at grid midpoints (piecewise linear)."""
    c = np.concatenate([[0.0], np.cumsum(p)])
    h = grid[1] - grid[0]
    edges = np.concatenate([[grid[0] - h / 2], grid + h / 2])
    return lambda x: np.interp(x, edges, c)


def _tau(x):
    """Integrated autocorrelation time of walker chains x [n_rec][n_walkers]
    (walker-averaged autocorrelation, Sokal's window with c = 5)."""
    x = x - x.mean(axis=0, keepdims=True)
    n = x.shape[0]
    f = np.fft.rfft(x, n=2 * n, axis=0)
    acf = np.fft.irfft(f * np.conj(f), axis=0)[:n].mean(axis=1)
    acf /= acf[0]
    tau = 1.0
    for m in range(1, n):
        tau = 1.0 + 2.0 * acf[1:m + 1].sum()
        if m >= 5 * tau:
            break
    return max(tau, 1.0)


def _run(lps, pb, betas, n_walkers, step, stretch, seed, n_burn=800, n_rec=500, every=8):
    ds, D = pb["ds"], pb["D"]
    T = len(betas)
    C = T * n_walkers
    rng = np.random.default_rng(seed)
    params = np.empty((4, C))
    params[0], params[1] = pb["a_oms"], pb["a_tm"]
    params[2] = pb["gu"].mean() + 0.02 * rng.standard_normal(C)
    params[3] = pb["ga"].mean() + 0.05 * rng.standard_normal(C)
    sb = W.pack_states(params, [[(np.zeros(0), np.zeros(0))] * ds.n_spl] * C, ds.n_spl)
    ctx = lps.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, max_states=C, f_knee=ds.f_knee,
                      arm_length=ds.arm_length)
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    sm = lps.Sampler(ctx, n_walkers, betas, seed=seed, k_in_max=4, step=step, precision="fp64",
                     fixed_params=(0, 1), rj_moves=False, stretch_moves=stretch)
    sm.set_state(st)
    sm.sweep(n_burn)
    rec = np.empty((n_rec, 2, C))
    for r in range(n_rec):
        sm.sweep(every)
        rec[r] = sm.get_state()["params"].cpu().numpy()[2:4]
    p = sm.get_state()["params"].cpu().numpy()
    assert np.all(p[0] == pb["a_oms"]) and np.all(p[1] == pb["a_tm"])   # held fixed
    return rec, sm.counters()


def _check_rung(rec, t, n_walkers, mom, gu, ga, label):
    x = rec[:, :, t * n_walkers:(t + 1) * n_walkers]          # [n_rec][2][W]
    out = {}
    for q, name, grid, pm in ((0, "u", gu, mom["pu"]), (1, "alpha", ga, mom["pa"])):
        v = x[:, q, :]
        tau = _tau(v)
        n = v.size
        ess = n / tau
        mean, var = v.mean(), v.var()
        mu, sd2 = mom["mu"][q], mom["var"][q]
        z_mean = (mean - mu) / math.sqrt(sd2 / ess)
        z_var = (var / sd2 - 1.0) / math.sqrt(2.0 / ess)
        thin = v[::max(int(math.ceil(tau)), 1), :].ravel()
        ks = stats.kstest(thin, _grid_cdf(grid, pm))
        print(f"{label} {name}: mean {mean:.5f} vs {mu:.5f} (z {z_mean:+.2f}), var ratio {var / sd2:.4f} "
              f"(z {z_var:+.2f}), tau {tau:.1f}, ESS {ess:.0f}, KS p {ks.pvalue:.3g} on {thin.size}", flush=True)
        assert abs(z_mean) < 4.5, (label, name, z_mean)
        assert abs(z_var) < 4.5, (label, name, z_var)
        assert ks.pvalue > 1e-4, (label, name, ks.pvalue)
        out[name] = ess
    # correlation of u and alpha
    cu = x[:, 0, :].ravel() - x[:, 0, :].mean()
    ca = x[:, 1, :].ravel() - x[:, 1, :].mean()
    r = (cu * ca).mean() / math.sqrt((cu ** 2).mean() * (ca ** 2).mean())
    ess = min(out.values())
    print(f"{label} corr {r:.4f} vs {mom['corr']:.4f}", flush=True)
    assert abs(r - mom["corr"]) < 4.5 * (1 - mom["corr"] ** 2) / math.sqrt(ess)


@pytest.mark.parametrize("stretch", [False, True])
def test_tempered_chains_sample_the_oracle_posterior(lps, problem, stretch):
    betas = [1.0, 0.3]
    Wk = 64
    mom1 = _grid_moments(problem, 1.0)
    # Langevin step scale is 1e-3 x step x (1/sqrt(beta)): about one posterior sd of u at beta = 1
    step = math.sqrt(mom1["var"][0]) / 1e-3
    rec, cnt = _run(lps, problem, betas, Wk, step, stretch, seed=21 if stretch else 17)
    print("counters (proposed, accepted) [kind][temp]", cnt.tolist(), flush=True)
    assert cnt[0, 0, 1] > 0.2 * cnt[0, 0, 0]          # Langevin moves are accepted
    if stretch:
        assert cnt[4, :, 1].sum() > 0.1 * cnt[4, :, 0].sum()
    for t, beta in enumerate(betas):
        mom = _grid_moments(problem, beta)
        _check_rung(rec, t, Wk, mom, problem["gu"], problem["ga"], f"beta={beta} stretch={stretch}")


def test_equal_temperature_rungs_always_swap(lps, problem):
    Wk = 16
    mom = _grid_moments(problem, 0.5)
    step = math.sqrt(mom["var"][0]) / 1e-3
    rec, cnt = _run(lps, problem, [0.5, 0.5], Wk, step, False, seed=5, n_burn=40, n_rec=10, every=4)
    proposed, accepted = cnt[3, 0, 0], cnt[3, 0, 1]
    assert proposed > 0 and accepted == proposed, (proposed, accepted)
