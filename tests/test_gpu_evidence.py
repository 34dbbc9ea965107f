"""Model-selection reductions on the device against the oracle: stepping-stone
evidence (Eq. (ss)) and DIC over tempered log-likelihood records, on seeded
arrays and on records of a sampler run with the paper's 20-rung ladder."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import evidence as E  # noqa: E402
from synth import workloads as W  # noqa: E402
from tests import cases as C  # noqa: E402


@pytest.fixture(scope="module")
def lps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as m
    m.lib()
    return m


def _by_rung(rec):
    """[n_rec, T, W] -> [T, n_rec * W] in record-major draw order."""
    n_rec, T, Wk = rec.shape
    return np.transpose(rec, (1, 0, 2)).reshape(T, n_rec * Wk)


def _close(a, b, rel=1e-12, abs_=1e-9):
    return abs(a - b) <= rel * abs(b) + abs_


# The variance n sum(w^2) / sum(w)^2 - 1 subtracts nearly equal numbers when the
# tempered weights are nearly uniform, which magnifies the (order-dependent)
# rounding of the two sums: it is compared at 1e-9.
VAR_REL = 1e-9


def test_stepping_stone_and_dic_match_oracle(lps):
    rng = np.random.default_rng(4)
    n_rec, T, Wk = 37, 6, 16
    betas = np.array([1e-20, 1e-12, 1e-7, 1e-3, 0.1, 1.0])
    rec = -2.0e6 + rng.normal(0.0, 50.0, (n_rec, T, Wk)) * np.linspace(30, 1, T)[None, :, None]
    rec[3, 2, 5] = -np.inf          # an invalid chain state among the draws
    dev = torch.as_tensor(rec, device="cuda")
    lz, var, steps, svar = lps.stepping_stone(betas, dev)
    ref_z, ref_var, ref_steps = E.stepping_stone(betas, _by_rung(rec))
    assert _close(lz, ref_z) and _close(var, ref_var, rel=VAR_REL, abs_=1e-14)
    for a, b in zip(steps, ref_steps):
        assert _close(a, b)
    assert abs(np.sum(svar) - var) <= 1e-12 * abs(var) + 1e-15
    lbar = -1.99e6
    got = lps.dic(dev, lbar, rung=T - 1)
    ref = E.dic(_by_rung(rec)[T - 1], lbar)
    for a, b in zip(got, ref):
        assert _close(a, b, abs_=1e-6), (got, ref)
    # repeatable to the bit
    assert lps.stepping_stone(betas, dev)[0] == lz
    with pytest.raises(lps.LpsError):
        lps.stepping_stone(betas[:1], dev[:, :1, :])


def test_evidence_over_sampler_records_with_the_paper_ladder(lps):
    name = "grad_25000bins_1024states"
    ds, D = C.dataset_with_data(name, n_bins=500, layout="split")
    betas = lps.paper_ladder()
    Wk, T = 8, betas.size
    sb = W.make_states(name, ds, n_states=Wk * T, inbetween=(0, 4))
    ctx = C.make_context(lps, ds, D, max_states=Wk * T)
    st = C.device_states(ctx, sb)
    sm = lps.Sampler(ctx, Wk, betas, seed=21, k_in_max=6, step=0.05, precision="mixed")
    sm.set_state(st)
    sm.sweep(20)
    n_rec = 25
    rec = torch.empty((n_rec, T, Wk), dtype=torch.float64, device="cuda")
    for i in range(n_rec):
        sm.sweep(2)
        sm.record_logL(rec[i].view(-1))
    torch.cuda.synchronize()
    host = rec.cpu().numpy()
    assert np.all(np.isfinite(host))
    lz, var, steps, _ = lps.stepping_stone(betas, rec)
    ref_z, ref_var, ref_steps = E.stepping_stone(betas, _by_rung(host))
    assert _close(lz, ref_z) and _close(var, ref_var, rel=VAR_REL, abs_=1e-14)
    np.testing.assert_allclose(steps, ref_steps, rtol=1e-12, atol=1e-9)
    # the hottest rungs barely feel the likelihood: their steps are tiny
    assert np.all(np.abs(steps[:4]) < 1e-3)
    got = lps.dic(rec, float(host[:, -1, :].mean()), rung=T - 1)
    ref = E.dic(_by_rung(host)[T - 1], float(host[:, -1, :].mean()))
    for a, b in zip(got, ref):
        assert _close(a, b, abs_=1e-6)


def test_column_median_matches_numpy(lps):
    """lps_column_median (the step-1 summary of the two-step driver) against
    numpy.median: odd and even counts, ties, a single value."""
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 64, 1001, 4096):
        x = rng.normal(size=(5, n))
        x[1] = np.round(x[1] * 3) / 3           # many ties
        x[2] = 4.25                              # all equal
        got = lps.column_median(torch.as_tensor(x, device="cuda")).cpu().numpy()
        np.testing.assert_array_equal(got, np.median(x, axis=1))
