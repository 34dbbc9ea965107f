"""Adjoint of the full-covariance likelihood on the GPU against the oracle's
gradient (itself pinned by finite differences of the likelihood).

FP64 end to end: |dg| <= 1e-8 * (||g_family||_inf + 1) per family (template
parameters as dimensionless sensitivities theta dlogL/dtheta for the two
amplitudes, knot heights, knot positions), the bar of the diagonal adjoint;
logL agrees with the likelihood entry point to 1e-12 on well-conditioned
covariances (1e-9 on the one-year draw, which holds near-singular bins)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import covariance as CV  # noqa: E402
from oracle import lps_oracle as O  # noqa: E402
from synth import workloads as W  # noqa: E402

REL = 1e-8


@pytest.fixture(scope="module")
def lps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as m
    m.lib()
    return m


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _knots(sb, s):
    return [sb.knots(s, j) for j in range(sb.n_spl)]


def _data(ds, cds, seed):
    x_lo, x_hi = W.band_edges(ds.f)
    truth = W.append_splines(ds.truth, np.random.default_rng(50 + seed), 3, (1, 4), x_lo, x_hi, 0.5)
    C, _, _ = CV.covariance(cds, truth.params[:, 0], _knots(truth, 0))
    return CV.unique_entries(W.complex_wishart_mean(np.random.default_rng(60 + seed), C, np.rint(ds.nk)).real)


def _setup(name, n_bins, layout, n_states, corr_inbetween=(0, 8), seed=0, corr=None):
    ds = W.make_dataset(name, n_bins=n_bins, layout=layout)
    x_lo, x_hi = W.band_edges(ds.f)
    nb = ds.n_spl
    corr = tuple(corr) if corr is not None else (nb, nb + 1, nb + 2)
    cds = CV.CovDataset(base=ds, corr=corr, n_spl=nb + 3)
    P6 = _data(ds, cds, seed)
    sb = W.make_states(name, ds, n_states=n_states, seed_offset=seed)
    sb = W.append_splines(sb, np.random.default_rng(70 + seed), 3, corr_inbetween, x_lo, x_hi, 0.5)
    return ds, cds, P6, sb


def _ctx(lps, ds, cds, P6, max_states):
    return lps.CovContext(ds.f, ds.nk, P6, ds.R, ds.route, cds.corr, cds.n_spl, Rfg=ds.Rfg,
                          max_states=max_states, f_knee=ds.f_knee, arm_length=ds.arm_length)


def _unpack(sb, s, dkx, dky):
    ys, xs = [], []
    for j in range(sb.n_spl):
        a, b = int(sb.knot_off[s * sb.n_spl + j]), int(sb.knot_off[s * sb.n_spl + j + 1])
        ys.append(dky[a:b])
        xs.append(dkx[a:b])
    return ys, xs


def _compare(sb, s, ref, logL, dp, dkx, dky, label):
    rl, rdp, rdy, rdx = ref
    assert abs(logL[s] - rl) <= 1e-10 * abs(rl), (label, s, logL[s], rl)
    u = np.where(np.arange(rdp.size) < 2, sb.params[:rdp.size, s], 1.0)
    a, b = dp[:, s] * u, rdp * u
    tol = REL * (np.abs(b).max() + 1.0)
    worst = np.abs(a - b).max() / tol
    assert np.all(np.abs(a - b) <= tol), (label, "params", s, a, b)
    gy, gx = _unpack(sb, s, dkx, dky)
    gy, gx, ry, rx = (np.concatenate(v) for v in (gy, gx, rdy, rdx))
    if ry.size:
        for g, r, fam in ((gy, ry, "heights"), (gx, rx, "positions")):
            tol = REL * (np.abs(r).max() + 1.0)
            worst = max(worst, np.abs(g - r).max() / tol)
            assert np.all(np.abs(g - r) <= tol), (label, fam, s, np.abs(g - r).max(), tol)
    return worst


def _check_batch(ctx, cds, P6, sb, idx, label):
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    logL, dp, dkx, dky, status = ctx.loglike_grad_batch(st)
    torch.cuda.synchronize()
    logL, dp, dkx, dky, status = (t.cpu().numpy() for t in (logL, dp, dkx, dky, status))
    worst = 0.0
    for s in idx:
        kn = _knots(sb, s)
        assert status[s] == CV.state_status(cds, sb.params[:, s], kn), (label, s)
        ref = CV.loglike_grad(cds, P6, sb.params[:, s], kn)
        if status[s]:
            assert logL[s] == ref[0] == -math.inf
            assert np.all(dp[:, s] == 0.0)
            gy, gx = _unpack(sb, s, dkx, dky)
            assert all(np.all(g == 0.0) for g in gy + gx)
            continue
        worst = max(worst, _compare(sb, s, ref, logL, dp, dkx, dky, label))
    _say(label, "worst error / tolerance", worst)
    return st, logL, status


@pytest.mark.parametrize("layout", ["paper", "split", "split_fg", "noise_signal"])
def test_gradient_matches_oracle(lps, layout):
    name = "avg50_1000bins_64states"
    _say("cov grad layout", layout)
    ds, cds, P6, sb = _setup(name, 1000, layout, 10, seed=1)
    ctx = _ctx(lps, ds, cds, P6, sb.n)
    st, logL, status = _check_batch(ctx, cds, P6, sb, range(sb.n), layout)
    assert np.all(status == 0)
    ev = ctx.loglike_batch(st)[0].cpu().numpy()
    assert np.all(np.abs(logL - ev) <= 1e-12 * np.abs(ev))


def test_dense_knots_and_ragged_tail(lps):
    """Up to 64 knots per spline: chunks that cross several pieces, and
    K = 2497 leaves a ragged last chunk."""
    name = "daily_2497bins_320states"
    _say("cov grad dense knots")
    ds, cds, P6, sb = _setup(name, None, "paper", 6, corr_inbetween=(20, 62), seed=2)
    ctx = _ctx(lps, ds, cds, P6, sb.n)
    _check_batch(ctx, cds, P6, sb, range(sb.n), "dense")


def test_zero_correlation_equals_the_diagonal_adjoint(lps):
    name = "avg50_1000bins_64states"
    _say("cov grad zero correlation")
    ds, cds, P6, sb = _setup(name, 800, "split", 8, seed=3, corr=(-1, -1, -1))
    ctx = _ctx(lps, ds, cds, P6, sb.n)
    logL, dp, dkx, dky, status = ctx.loglike_grad_batch(ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y))
    dctx = lps.Context(ds.f, ds.nk, P6[:3], ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=sb.n,
                       f_knee=ds.f_knee, arm_length=ds.arm_length)
    base = W.pack_states(sb.params, [_knots(sb, s)[:ds.n_spl] for s in range(sb.n)], ds.n_spl)
    l0, dp0, dkx0, dky0, st0 = dctx.loglike_grad_batch(dctx.states(base.params, base.knot_off, base.knot_x,
                                                                     base.knot_y), "fp64")
    logL, dp, dkx, dky = (t.cpu().numpy() for t in (logL, dp, dkx, dky))
    l0, dp0, dkx0, dky0 = (t.cpu().numpy() for t in (l0, dp0, dkx0, dky0))
    assert np.all(status.cpu().numpy() == 0) and np.all(st0.cpu().numpy() == 0)
    assert np.all(np.abs(logL - l0) <= 1e-12 * np.abs(l0))
    for s in range(sb.n):
        u = np.where(np.arange(dp0.shape[0]) < 2, sb.params[:dp0.shape[0], s], 1.0)
        a, b = dp[:, s] * u, dp0[:, s] * u
        assert np.all(np.abs(a - b) <= 1e-10 * (np.abs(b).max() + 1.0))
        gy, gx = _unpack(sb, s, dkx, dky)
        ry, rx = _unpack(base, s, dkx0, dky0)
        for j in range(ds.n_spl):
            assert np.all(np.abs(gy[j] - ry[j]) <= 1e-10 * (np.abs(ry[j]).max() + 1.0))
            assert np.all(np.abs(gx[j] - rx[j]) <= 1e-10 * (np.abs(rx[j]).max() + 1.0))
        for j in range(ds.n_spl, sb.n_spl):       # correlation slots routed nowhere
            assert np.all(gy[j] == 0.0) and np.all(gx[j] == 0.0)


def test_invalid_states_singular_covariance_and_determinism(lps):
    name = "avg50_1000bins_64states"
    _say("cov grad invalid states")
    ds, cds, P6, sb = _setup(name, 500, "paper", 1, seed=5)
    x_lo, x_hi = W.band_edges(ds.f)
    p = sb.params[:, 0]
    kn = _knots(sb, 0)
    cases = []
    k = list(kn)
    k[5] = (kn[5][0][::-1].copy(), kn[5][1])                      # unordered correlation knots
    cases.append((p, k))
    k = list(kn)
    k[1] = kn[0]                                                   # r_AE = 1 in double: singular
    k[4] = (np.array([x_lo, x_hi]), np.array([30.0, 30.0]))
    p2 = p.copy()
    p2[2] = -80.0
    cases.append((p2, k))
    cases.append((p, kn))                                          # valid
    params = np.stack([c[0] for c in cases], axis=1)
    sbx = W.pack_states(params, [c[1] for c in cases], cds.n_spl)
    ctx = _ctx(lps, ds, cds, P6, 4)
    st, logL, status = _check_batch(ctx, cds, P6, sbx, range(sbx.n), "invalid")
    assert status[0] & O.ST_ORDER and status[1] == O.ST_PSD and status[2] == 0
    a = ctx.loglike_grad_batch(st)
    b = ctx.loglike_grad_batch(st)
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    empty = W.states_subset(sbx, [])
    ctx.loglike_grad_batch(ctx.states(empty.params, empty.knot_off, np.zeros(1), np.zeros(1)))
    with pytest.raises(lps.LpsError):
        big = W.states_subset(sbx, [0] * 5)
        ctx.loglike_grad_batch(ctx.states(big.params, big.knot_off, big.knot_x, big.knot_y))


def test_full_year_grid_sampled(lps):
    """912085 one-year bins and 1024 states with up to 30 interior correlation
    knots; the state with the fewest knots compared with the oracle's gradient
    (about half a minute of oracle time), the rest through logL against the
    likelihood entry point."""
    name = "year_912085bins_4096states"
    _say("cov grad full year")
    ds = W.make_dataset(name, layout="paper")
    x_lo, x_hi = W.band_edges(ds.f)
    nb = ds.n_spl
    cds = CV.CovDataset(base=ds, corr=(nb, nb + 1, nb + 2), n_spl=nb + 3)
    P6 = _data(ds, cds, 8)
    sb = W.states_subset(W.make_states(name, ds), list(range(1024)))
    sb = W.append_splines(sb, np.random.default_rng(82), 3, (0, 30), x_lo, x_hi, 0.5)
    ctx = _ctx(lps, ds, cds, P6, sb.n)
    sizes = np.diff(sb.knot_off).reshape(sb.n, sb.n_spl).sum(axis=1)
    st, logL, status = _check_batch(ctx, cds, P6, sb, [int(np.argmin(sizes))], "year")
    ev, evs = ctx.loglike_batch(st)
    ev, evs = ev.cpu().numpy(), evs.cpu().numpy()
    assert np.array_equal(status, evs)
    ok = status == 0
    # the two kernels form det C by different (equally valid) cofactor
    # expressions; a few drawn states have correlations within 1e-8 of one
    # (det C / prod C_cc ~ 1e-8 at some bins), where rounding of det C is
    # amplified to ~1e-10 of logL in either kernel (both were checked against
    # the oracle there)
    assert np.all(np.abs(logL[ok] - ev[ok]) <= 1e-9 * np.abs(ev[ok]))
    assert np.all(logL[~ok] == -math.inf)


def test_batch_independence_and_graph_replay(lps):
    """A state's results do not depend on the batch it is evaluated in, and the
    call captured into a HIP graph and replayed (eager calls in between) gives
    the eager result every time."""
    name = "avg50_1000bins_64states"
    _say("cov grad batch independence and graph replay")
    ds, cds, P6, sb = _setup(name, 1000, "paper", 24, seed=9)
    ctx = _ctx(lps, ds, cds, P6, sb.n)
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    full = [t.clone() for t in ctx.loglike_grad_batch(st)]
    fl = full[0].cpu().numpy()
    fdp = full[1].cpu().numpy()
    fkx, fky = full[2].cpu().numpy(), full[3].cpu().numpy()
    for idx in ([5], [23, 0, 17], list(range(8, 20))):
        sub = W.states_subset(sb, idx)
        l, dp, dkx, dky, _ = ctx.loglike_grad_batch(ctx.states(sub.params, sub.knot_off, sub.knot_x, sub.knot_y))
        assert np.array_equal(l.cpu().numpy(), fl[idx])
        assert np.array_equal(dp.cpu().numpy(), fdp[:, idx])
        dkx, dky = dkx.cpu().numpy(), dky.cpu().numpy()
        for i, s in enumerate(idx):
            gy, gx = _unpack(sub, i, dkx, dky)
            ry, rx = _unpack(sb, s, fkx, fky)
            assert all(np.array_equal(a, b) for a, b in zip(gy + gx, ry + rx))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.loglike_grad_batch(st, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = ctx.loglike_grad_batch(st)
    for rep in range(3):
        for o in outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for o, f in zip(outs, full):
            assert torch.equal(o, f), rep
        assert torch.equal(ctx.loglike_grad_batch(st)[1], full[1])


def test_disabled_and_linear_splines(lps):
    """Correlation splines with no knots (Q = 0), two or three knots (the
    linear construction) and the Akima construction mixed in one batch."""
    name = "avg50_1000bins_64states"
    _say("cov grad disabled and linear splines")
    ds, cds, P6, sb = _setup(name, 900, "paper", 6, seed=11)
    x_lo, x_hi = W.band_edges(ds.f)
    rng = np.random.default_rng(12)
    knots = []
    for s in range(sb.n):
        kn = _knots(sb, s)
        for j in range(ds.n_spl, sb.n_spl):
            m = (s + j) % 4           # 0, 2, 3 knots or the drawn Akima spline
            if m == 0:
                kn[j] = (np.zeros(0), np.zeros(0))
            elif m in (1, 2):
                n = m + 1
                inner = np.sort(rng.uniform(x_lo, x_hi, n - 2))
                kn[j] = (np.concatenate([[x_lo], inner, [x_hi]]), rng.normal(0.0, 0.5, n))
        knots.append(kn)
    sbx = W.pack_states(sb.params, knots, sb.n_spl)
    ctx = _ctx(lps, ds, cds, P6, sbx.n)
    _, _, status = _check_batch(ctx, cds, P6, sbx, range(sbx.n), "disabled/linear")
    assert np.all(status == 0)
