"""Pins of the full-covariance oracle (reading X1 of the dense 3x3 model).

* zero correlations reproduce the diagonal likelihood term by term, whatever
  the off-diagonal data rows hold;
* the vine gives a positive-definite correlation matrix whose partial
  correlation (read from its inverse) is tanh Q_2;
* one correlated pair at a time reduces to a 2x2 block, written out by hand,
  plus one scalar channel (this pins the row order of the data and of C);
* the Wishart term is stationary at P = C with value 3 + ln det C per bin
  (determinant from the eigenvalues), and every perturbation lowers it;
* Wishart draws from the generator have mean C and the trace statistic of
  their law, Gamma(3 nu, 1) per bin;
* invalid states: the diagonal model's checks on the extra slots, and a
  singular covariance."""
import math

import numpy as np
import pytest

from oracle import covariance as CV
from oracle import lps_oracle as O
from synth import workloads as W

NAME = "avg50_1000bins_64states"


def _base(n_bins=300):
    return W.make_dataset(NAME, n_bins=n_bins, layout="paper")


def _states(ds, n, seed, corr_inbetween=(0, 4), height_sd=0.5):
    sb = W.make_states(NAME, ds, n_states=n, inbetween=(1, 5), seed_offset=seed)
    x_lo, x_hi = W.band_edges(ds.f)
    return W.append_splines(sb, np.random.default_rng(100 + seed), 3, corr_inbetween, x_lo, x_hi, height_sd)


def _cds(ds, corr=None):
    nb = ds.n_spl
    return CV.CovDataset(base=ds, corr=corr if corr is not None else (nb, nb + 1, nb + 2), n_spl=nb + 3)


def _random_data(ds, rng):
    S, _, _ = O.psd(ds, ds.truth.params[:, 0], [ds.truth.knots(0, j) for j in range(ds.n_spl)])
    P6 = np.zeros((6, ds.f.size))
    P6[:3] = S * rng.gamma(50.0, 1.0 / 50.0, S.shape)
    for i, (a, b) in enumerate(CV.PAIRS[3:]):
        P6[3 + i] = 0.3 * np.sqrt(S[a] * S[b]) * rng.normal(size=ds.f.size)
    return P6


def _knots(sb, s):
    return [sb.knots(s, j) for j in range(sb.n_spl)]


def test_zero_correlation_is_the_diagonal_likelihood():
    ds = _base()
    rng = np.random.default_rng(1)
    P6 = _random_data(ds, rng)
    sb = _states(ds, 4, 1)
    for s in range(sb.n):
        kn = _knots(sb, s)
        want = O.loglike(ds, P6[:3], sb.params[:, s], kn[:4])
        # correlation slots routed nowhere
        got = CV.loglike(_cds(ds, corr=(-1, -1, -1)), P6, sb.params[:, s], kn)
        assert abs(got - want) <= 1e-13 * abs(want)
        # correlation splines present but disabled (no knots)
        kn0 = kn[:4] + [(np.zeros(0), np.zeros(0))] * 3
        got0 = CV.loglike(_cds(ds), P6, sb.params[:, s], kn0)
        assert abs(got0 - want) <= 1e-13 * abs(want)


def test_vine_is_positive_definite_with_the_given_partial_correlation():
    rng = np.random.default_rng(2)
    q = rng.normal(0.0, 1.5, (3, 2000))
    r01, r02, r12 = CV.vine_correlations(q[0], q[1], q[2])
    R = np.zeros((q.shape[1], 3, 3))
    R[:, 0, 0] = R[:, 1, 1] = R[:, 2, 2] = 1.0
    R[:, 0, 1] = R[:, 1, 0] = r01
    R[:, 0, 2] = R[:, 2, 0] = r02
    R[:, 1, 2] = R[:, 2, 1] = r12
    assert np.all(np.linalg.eigvalsh(R)[:, 0] > 0.0)
    Ri = np.linalg.inv(R)
    partial = -Ri[:, 1, 2] / np.sqrt(Ri[:, 1, 1] * Ri[:, 2, 2])
    np.testing.assert_allclose(partial, np.tanh(q[2]), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r01, np.tanh(q[0]), rtol=1e-15)
    np.testing.assert_allclose(r02, np.tanh(q[1]), rtol=1e-15)
    z = np.zeros(5)
    assert np.all(np.array(CV.vine_correlations(z, z, z)) == 0.0)


@pytest.mark.parametrize("pair", [(0, 1), (0, 2), (1, 2)])
def test_one_correlated_pair_is_a_2x2_block(pair):
    ds = _base()
    rng = np.random.default_rng(3)
    P6 = _random_data(ds, rng)
    sb = _states(ds, 3, 3)
    slot = {(0, 1): 0, (0, 2): 1, (1, 2): 2}[pair]
    corr = [-1, -1, -1]
    corr[slot] = 4 + slot
    cds = _cds(ds, corr=tuple(corr))
    a, b = pair
    (c,) = {0, 1, 2} - {a, b}
    row = {(0, 1): 3, (0, 2): 4, (1, 2): 5}[pair]
    x = np.log10(ds.f)
    for s in range(sb.n):
        kn = _knots(sb, s)
        _, sn, sh = O.psd(ds, sb.params[:, s], kn[:4])
        d = sn + sh
        r = np.tanh(O.spline_eval(*kn[4 + slot], x))
        nab = r * np.sqrt(sn[a] * sn[b])
        det = d[a] * d[b] - nab * nab
        tr = (d[b] * P6[a] + d[a] * P6[b] - 2.0 * nab * P6[row]) / det + P6[c] / d[c]
        want = -math.fsum((ds.nk * (tr + np.log(det) + np.log(d[c]))).tolist())
        got = CV.loglike(cds, P6, sb.params[:, s], kn)
        assert abs(got - want) <= 1e-12 * abs(want), (pair, got, want)


def test_wishart_term_is_stationary_at_the_model():
    ds = _base()
    cds = _cds(ds)
    sb = _states(ds, 2, 4)
    kn = _knots(sb, 0)
    p = sb.params[:, 0]
    C, _, _ = CV.covariance(cds, p, kn)
    P6 = CV.unique_entries(C)
    ev = np.linalg.eigvalsh(C)
    want = -math.fsum((ds.nk * (3.0 + np.log(ev).sum(axis=1))).tolist())
    got = CV.loglike(cds, P6, p, kn)
    assert abs(got - want) <= 1e-11 * abs(want)
    # any move away from the model lowers the likelihood
    for j in range(cds.n_spl):
        kx, ky = kn[j]
        for dy in (0.02, -0.02):
            kn2 = list(kn)
            kn2[j] = (kx, ky + dy)
            assert CV.loglike(cds, P6, p, kn2) < got
    for i in range(4):
        p2 = p.copy()
        p2[i] = p2[i] * 1.01 if i < 2 else p2[i] + 0.01
        assert CV.loglike(cds, P6, p2, kn) < got


def test_wishart_draws_have_the_right_mean_and_trace_law():
    ds = _base(400)
    cds = _cds(ds)
    sb = _states(ds, 1, 5)
    kn = _knots(sb, 0)
    C, _, _ = CV.covariance(cds, sb.params[:, 0], kn)
    nu = ds.nk
    rng = np.random.default_rng(6)
    reps = 40
    tr_tot, dev = [], np.zeros((6, ds.f.size))
    for _ in range(reps):
        Pc = W.complex_wishart_mean(rng, C, nu)
        P6 = CV.unique_entries(Pc.real)
        X = np.linalg.solve(C, CV.data_matrix(P6))
        tr_tot.append(np.sum(nu * (X[:, 0, 0] + X[:, 1, 1] + X[:, 2, 2])))
        s = np.sqrt(np.stack([C[:, a, a] * C[:, b, b] for (a, b) in CV.PAIRS]))
        dev += (P6 - CV.unique_entries(C)) / s
        # Hermitian with real diagonal
        assert np.allclose(Pc, np.conj(np.transpose(Pc, (0, 2, 1))), rtol=0, atol=1e-12 * np.abs(Pc).max())
    # nu tr(C^-1 P) ~ Gamma(3 nu, 1) per bin: the sum over bins has mean and variance 3 sum(nu)
    m = 3.0 * nu.sum()
    tr_tot = np.array(tr_tot)
    assert abs(tr_tot.mean() - m) < 5.0 * math.sqrt(m / reps)
    assert abs(tr_tot.var(ddof=1) / m - 1.0) < 0.6
    # E[P] = C entry by entry: each normalised deviation has sd <= 1/sqrt(nu)
    per = dev / reps
    sd = 1.0 / np.sqrt(nu * reps)
    assert np.all(np.abs(per.mean(axis=1)) < 5.0 * sd.mean() / math.sqrt(ds.f.size))


def test_invalid_states_and_a_singular_covariance():
    ds = _base()
    cds = _cds(ds)
    rng = np.random.default_rng(7)
    P6 = _random_data(ds, rng)
    sb = _states(ds, 1, 8)
    p = sb.params[:, 0]
    kn = _knots(sb, 0)
    # a correlation spline with unordered knots / one knot / non-finite height
    kx, ky = kn[5]
    bad = list(kn)
    bad[5] = (kx[::-1].copy(), ky)
    assert CV.state_status(cds, p, bad) & O.ST_ORDER
    bad[5] = (kx[:1], ky[:1])
    assert CV.state_status(cds, p, bad) & O.ST_COUNT
    bad[5] = (kx, np.where(np.arange(ky.size) == 0, np.nan, ky))
    assert CV.state_status(cds, p, bad) & O.ST_NONFINITE
    assert CV.loglike(cds, P6, p, bad) == -math.inf
    # strong but finite correlations are valid
    x_lo, x_hi = W.band_edges(ds.f)
    strong = list(kn)
    strong[4] = (np.array([x_lo, x_hi]), np.array([3.0, 3.0]))
    assert CV.state_status(cds, p, strong) == 0
    # A and E with identical noise, no signal to speak of, and r_AE = tanh(30) = 1
    # in double precision: the covariance is singular
    sing = list(kn)
    sing[1] = kn[0]
    sing[4] = (np.array([x_lo, x_hi]), np.array([30.0, 30.0]))
    p2 = p.copy()
    p2[O.LPS_P_U if hasattr(O, "LPS_P_U") else 2] = -80.0
    assert np.tanh(30.0) == 1.0
    assert CV.state_status(cds, p2, sing) == O.ST_PSD
    assert CV.loglike(cds, P6, p2, sing) == -math.inf


def test_single_draw_wishart_mean():
    """nu = 1 (the unaveraged periodogram): E[z z^H] = C, rank one per bin."""
    ds = _base(50)
    cds = _cds(ds)
    sb = _states(ds, 1, 9)
    C, _, _ = CV.covariance(cds, sb.params[:, 0], _knots(sb, 0))
    rng = np.random.default_rng(10)
    reps = 4000
    acc = np.zeros_like(C)
    for _ in range(reps):
        Pc = W.complex_wishart_mean(rng, C, np.ones(ds.f.size))
        acc += Pc.real
    assert np.all(np.linalg.matrix_rank(Pc) == 1)
    s = np.sqrt(np.einsum("kaa,kbb->kab", C, C))
    assert np.all(np.abs(acc / reps - C) < 6.0 * s / math.sqrt(reps))


# --------------------------------------------------------------------------
# gradient
# --------------------------------------------------------------------------

def _fd(cds, P6, p, kn, move, h):
    """Central difference of logL, summed bin by bin (the large common part of
    the per-bin terms cancels before the sum)."""
    pa, ka = move(+h)
    pb, kb = move(-h)
    ta = CV.loglike_terms(cds, P6, pa, ka)
    tb = CV.loglike_terms(cds, P6, pb, kb)
    return -math.fsum((ta - tb).tolist()) / (2.0 * h)


def _grad_fd_errors(cds, P6, p, kn):
    """Largest |analytic - finite difference| / (family scale) over the template
    parameters, knot heights and interior knot positions."""
    _, dp, dys, dxs = CV.loglike_grad(cds, P6, p, kn)
    worst = {}

    def upd(fam, got, want, scale):
        worst[fam] = max(worst.get(fam, 0.0), abs(got - want) / scale)

    sp = np.abs(dp * np.where(np.arange(p.size) < 2, p, 1.0)).max() + 1.0
    for i in range(p.size):
        h = 1e-6 * abs(p[i]) if i < 2 else 1e-6

        def mv(d, i=i):
            q = p.copy()
            q[i] += d
            return q, kn
        fd = _fd(cds, P6, p, kn, mv, h)
        u = p[i] if i < 2 else 1.0
        upd("params", dp[i] * u, fd * u, sp)
    sy = max(np.abs(g).max() for g in dys if g.size) + 1.0
    sx = max(np.abs(g).max() for g in dxs if g.size) + 1.0
    for j, (kx, ky) in enumerate(kn):
        for i in range(kx.size):
            def my(d, j=j, i=i):
                k2 = list(kn)
                y2 = ky.copy()
                y2[i] += d
                k2[j] = (kx, y2)
                return p, k2
            upd("heights", dys[j][i], _fd(cds, P6, p, kn, my, 1e-6), sy)
            if 0 < i < kx.size - 1:
                def mx(d, j=j, i=i):
                    k2 = list(kn)
                    x2 = kx.copy()
                    x2[i] += d
                    k2[j] = (x2, ky)
                    return p, k2
                # step scaled to the narrower neighbouring interval, where the
                # spline's third derivative grows as width^-2
                hx = 1e-5 * min(kx[i] - kx[i - 1], kx[i + 1] - kx[i])
                upd("positions", dxs[j][i], _fd(cds, P6, p, kn, mx, hx), sx)
            else:
                assert dxs[j][i] == 0.0
    return worst


@pytest.mark.parametrize("layout", ["paper", "split_fg"])
def test_gradient_matches_finite_differences(layout):
    """Every template parameter, knot height and interior knot position of
    all seven splines (four diagonal, three correlation) against central
    differences of the likelihood itself."""
    ds = W.make_dataset(NAME, n_bins=160, layout=layout)
    cds = _cds(ds)
    rng = np.random.default_rng(20)
    P6 = _random_data(ds, rng)
    sb = _states(ds, 2, 21, corr_inbetween=(1, 3))
    for s in range(sb.n):
        worst = _grad_fd_errors(cds, P6, sb.params[:, s], _knots(sb, s))
        assert set(worst) == {"params", "heights", "positions"}
        for fam, e in worst.items():
            assert e < 1e-6, (layout, s, fam, e)


def test_gradient_zero_correlation_is_the_diagonal_gradient():
    """Correlation slots routed nowhere: the diagonal oracle's gradient for the
    diagonal splines, exact zeros for the unrouted ones."""
    ds = _base(250)
    rng = np.random.default_rng(22)
    P6 = _random_data(ds, rng)
    sb = _states(ds, 3, 23)
    cds = _cds(ds, corr=(-1, -1, -1))
    for s in range(sb.n):
        kn = _knots(sb, s)
        l1, dp1, dy1, dx1 = CV.loglike_grad(cds, P6, sb.params[:, s], kn)
        l0, dp0, dy0, dx0 = O.loglike_grad(ds, P6[:3], sb.params[:, s], kn[:4])
        assert abs(l1 - l0) <= 1e-13 * abs(l0)
        u = np.where(np.arange(dp0.size) < 2, sb.params[:dp0.size, s], 1.0)
        np.testing.assert_allclose(dp1 * u, dp0 * u, rtol=1e-9, atol=1e-9 * np.abs(dp0 * u).max())
        for j in range(4):
            np.testing.assert_allclose(dy1[j], dy0[j], rtol=1e-9, atol=1e-9 * (np.abs(dy0[j]).max() + 1.0))
            np.testing.assert_allclose(dx1[j], dx0[j], rtol=1e-9, atol=1e-9 * (np.abs(dx0[j]).max() + 1.0))
        for j in range(4, 7):
            assert np.all(dy1[j] == 0.0) and np.all(dx1[j] == 0.0)


def test_gradient_vanishes_at_the_model():
    """P = C makes the likelihood stationary (the Wishart term's maximum): the
    whole gradient is rounding-sized next to its value at other data."""
    ds = _base(250)
    cds = _cds(ds)
    sb = _states(ds, 1, 24, corr_inbetween=(1, 3))
    p, kn = sb.params[:, 0], _knots(sb, 0)
    C, _, _ = CV.covariance(cds, p, kn)
    _, dp0, dy0, dx0 = CV.loglike_grad(cds, CV.unique_entries(C), p, kn)
    _, dp1, dy1, dx1 = CV.loglike_grad(cds, _random_data(ds, np.random.default_rng(25)), p, kn)
    u = np.where(np.arange(dp0.size) < 2, p[:dp0.size], 1.0)
    assert np.abs(dp0 * u).max() <= 1e-9 * np.abs(dp1 * u).max()
    big_y = max(np.abs(g).max() for g in dy1)
    big_x = max(np.abs(g).max() for g in dx1)
    assert max(np.abs(g).max() for g in dy0) <= 1e-9 * big_y
    assert max(np.abs(g).max() for g in dx0) <= 1e-9 * big_x


def test_gradient_of_an_invalid_state_is_zero():
    ds = _base(100)
    cds = _cds(ds)
    sb = _states(ds, 1, 26)
    p, kn = sb.params[:, 0], _knots(sb, 0)
    bad = list(kn)
    kx, ky = kn[5]
    bad[5] = (kx[::-1].copy(), ky)
    l, dp, dy, dx = CV.loglike_grad(cds, _random_data(ds, np.random.default_rng(27)), p, bad)
    assert l == -math.inf and np.all(dp == 0.0)
    assert all(np.all(g == 0.0) for g in dy + dx)
