"""Device sampler sweeps: prior recovery at beta = 0, bitwise resume, graph replay, counters."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from synth import workloads as SW  # noqa: E402
from tests import cases as C  # noqa: E402

NAME = "grad_25000bins_1024states"


@pytest.fixture(scope="module")
def lps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as m
    m.lib()
    return m


def _setup(lps, n_walkers, betas, k_in_max, inbetween, n_bins=600, seed=7, step=0.05):
    ds, D = C.dataset_with_data(NAME, n_bins=n_bins, layout="split")
    n = n_walkers * len(betas)
    sb = SW.make_states(NAME, ds, n_states=n, inbetween=inbetween)
    ctx = C.make_context(lps, ds, D, max_states=n)
    st = C.device_states(ctx, sb)
    sm = lps.Sampler(ctx, n_walkers, betas, seed=seed, k_in_max=k_in_max, step=step, precision="mixed")
    return ctx, sm, st, ds


def _interior(state):
    off, cnt = state["knot_off"].cpu().numpy(), state["knot_cnt"].cpu().numpy()
    kx, ky = state["knot_x"].cpu().numpy(), state["knot_y"].cpu().numpy()
    k_in = cnt - 2
    xs = np.concatenate([kx[o + 1:o + c - 1] for o, c in zip(off, cnt)])
    ys = np.concatenate([ky[o:o + c] for o, c in zip(off, cnt)])
    return k_in, xs, ys


def test_beta_zero_chains_sample_the_prior(lps):
    """With beta = 0 the likelihood drops out: knot counts become uniform on
    {0..k_in_max}, heights N(0, 0.1), in-between positions uniform in the band,
    starting from splines that have no in-between knot at all."""
    k_in_max = 5
    ctx, sm, st, ds = _setup(lps, 64, [0.0, 0.0], k_in_max, (0, 0))
    sm.set_state(st)
    counts, xs_all, ys_all = [], [], []
    sm.sweep(300)                       # burn-in
    for _ in range(60):
        sm.sweep(40)
        k_in, xs, ys = _interior(sm.get_state())
        counts.append(k_in)
        xs_all.append(xs)
        ys_all.append(ys)
    counts = np.concatenate(counts)
    freq = np.bincount(counts, minlength=k_in_max + 1) / counts.size
    print("count frequencies", freq, flush=True)
    assert counts.max() <= k_in_max and counts.min() >= 0
    assert np.all(np.abs(freq - 1.0 / (k_in_max + 1)) < 0.03)
    ys = np.concatenate(ys_all)
    assert abs(ys.mean()) < 0.01 and abs(ys.std() - 0.1) < 0.01
    xs = np.concatenate(xs_all)
    lo, hi = np.log10(ds.f[0]), np.log10(ds.f[-1])
    u = (xs - lo) / (hi - lo)
    assert np.all((u > 0) & (u < 1))
    hist = np.histogram(u, bins=5, range=(0, 1))[0] / u.size
    assert np.all(np.abs(hist - 0.2) < 0.03)
    cnt = sm.counters()
    n_sweeps = 300 + 60 * 40
    assert cnt[0, :, 0].sum() == n_sweeps * sm.C                       # one Langevin proposal per chain
    assert cnt[1, :, 0].sum() + cnt[2, :, 0].sum() == n_sweeps * sm.C  # one birth or death per chain


def test_resume_is_bitwise_identical(lps):
    betas = [1.0, 0.3, 0.05]
    ctx, sm, st, _ = _setup(lps, 16, betas, 8, (0, 8), n_bins=900, seed=11)
    sm.set_state(st)
    sm.sweep(12)
    a = sm.get_state()
    sm2 = lps.Sampler(ctx, 16, betas, seed=11, k_in_max=8, step=0.05, precision="mixed")
    sm2.set_state(st)
    sm2.sweep(5)
    st5, idx, _ = sm2.packed_state()
    assert idx == 5
    sm3 = lps.Sampler(ctx, 16, betas, seed=11, k_in_max=8, step=0.05, precision="mixed")
    sm3.set_state(st5, sweep_index=idx)
    sm3.sweep(7)
    b = sm3.get_state()
    assert a["sweep"] == b["sweep"] == 12
    for key in ("params", "knot_cnt", "logL"):
        assert torch.equal(a[key], b[key]), key
    ka, kb = _interior(a), _interior(b)
    assert np.array_equal(ka[1], kb[1]) and np.array_equal(ka[2], kb[2])


def test_graph_replay_equals_eager(lps):
    betas = [1.0, 0.2]
    ctx, sm, st, _ = _setup(lps, 16, betas, 6, (0, 6), n_bins=700, seed=3)
    sm.set_state(st)
    sm.sweep(4)
    eager = sm.get_state()
    smg = lps.Sampler(ctx, 16, betas, seed=3, k_in_max=6, step=0.05, precision="mixed")
    smg.set_state(st)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        smg.sweep(2)
    torch.cuda.synchronize()
    for _ in range(2):
        g.replay()
        torch.cuda.synchronize()
    got = smg.get_state()
    assert got["sweep"] == 4
    for key in ("params", "knot_cnt", "logL"):
        assert torch.equal(eager[key], got[key]), key


def test_cold_chains_climb_the_likelihood(lps):
    betas = [1.0, 0.5, 0.1]
    ctx, sm, st, _ = _setup(lps, 32, betas, 10, (0, 10), n_bins=1200, seed=5, step=0.05)
    sm.set_state(st)
    l0 = sm.get_state()["logL"].cpu().numpy()[:32]
    sm.sweep(150)
    l1 = sm.get_state()["logL"].cpu().numpy()[:32]
    cnt = sm.counters()
    print("acceptance (proposed, accepted) per kind/temperature", cnt.tolist(), flush=True)
    assert np.all(np.isfinite(l1))
    assert np.median(l1) > np.median(l0)
    assert cnt[0, 0, 1] > 0 and cnt[1:3, :, 1].sum() > 0


def test_stretch_moves_sample_the_template_prior(lps):
    """With beta = 0 and ensemble stretch moves on, the walkers spread from a
    small box over the whole uniform prior of the background amplitude u and
    slope alpha (Table I ranges of the sampler: u in [-20, -10], alpha in [-5, 5])."""
    ds, D = C.dataset_with_data(NAME, n_bins=600, layout="split")
    Wk = 64
    sb = SW.make_states(NAME, ds, n_states=Wk, inbetween=(0, 3))
    ctx = C.make_context(lps, ds, D, max_states=Wk)
    sm = lps.Sampler(ctx, Wk, [0.0], seed=13, k_in_max=5, step=0.05, precision="fp64", rj_moves=False,
                     stretch_moves=True)
    sm.set_state(C.device_states(ctx, sb))
    sm.sweep(300)
    us, als = [], []
    for _ in range(80):
        sm.sweep(5)
        p = sm.get_state()["params"].cpu().numpy()
        us.append(p[2])
        als.append(p[3])
    u, a = np.concatenate(us), np.concatenate(als)
    assert u.min() >= -20 and u.max() <= -10 and a.min() >= -5 and a.max() <= 5
    hu = np.histogram(u, bins=5, range=(-20, -10))[0] / u.size
    ha = np.histogram(a, bins=5, range=(-5, 5))[0] / a.size
    print("u hist", hu, "alpha hist", ha, flush=True)
    assert np.all(np.abs(hu - 0.2) < 0.06) and np.all(np.abs(ha - 0.2) < 0.06)
    cnt = sm.counters()
    assert cnt[4, 0, 0] == 700 * Wk and cnt[4, 0, 1] > 0      # every chain once per sweep
