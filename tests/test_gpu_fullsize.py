"""Full-size parity: the one-year workload (912,085 bins x 4,096 states) in the
launch configuration bench.py times, checked on a sample of states against the
FP64 oracle one by one, plus properties that hold at any size."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from synth import workloads as W  # noqa: E402
from tests import cases as C  # noqa: E402

NAME = "year_912085bins_4096states"


def _largest_spline_excursions(sb, m):
    """The m states whose splines reach the largest |P| (evaluated by the oracle
    at nine points per knot interval): where a scaled PSD can leave the
    single-precision range and the mixed path has to fall back to double range."""
    from oracle import lps_oracle as O
    peak = np.zeros(sb.n)
    for s in range(sb.n):
        for j in range(sb.n_spl):
            x, y = sb.knots(s, j)
            if len(x) < 2:
                continue
            xq = np.concatenate([np.linspace(a, b, 9) for a, b in zip(x[:-1], x[1:])])
            peak[s] = max(peak[s], np.abs(O.spline_eval(x, y, xq)).max())
    return np.argsort(peak)[-m:].tolist()


def test_year_workload_sampled_parity():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as lps
    ds, D = C.dataset_with_data(NAME)
    sb = W.make_states(NAME, ds)
    ctx = C.make_context(lps, ds, D, max_states=sb.n, max_grad_states=0)
    st = C.device_states(ctx, sb)
    for prec in ("mixed", "fp64"):
        ctx.autotune(st, prec, reps=2)
    lm, sm = ctx.loglike_batch(st, "mixed")
    l64, s64 = ctx.loglike_batch(st, "fp64")
    lm, l64 = lm.cpu().numpy(), l64.cpu().numpy()
    sm, s64 = sm.cpu().numpy(), s64.cpu().numpy()
    rng = np.random.default_rng(0)
    extreme = _largest_spline_excursions(sb, 5)
    sample = sorted(set(rng.choice(sb.n, 8, replace=False).tolist()) | {0, sb.n - 1} | set(extreme))
    ref = C.oracle_loglikes(ds, D, sb, sample)
    ref_st = C.oracle_status(ds, sb, sample)
    tol = C.mixed_tolerance(ds, D, sb, sample)
    tol64 = C.fp64_tolerance(ds, D, sb, sample)
    for i, s in enumerate(sample):
        if not np.isfinite(ref[i]):
            assert not np.isfinite(l64[s])
            continue
        assert s64[s] == ref_st[i] and sm[s] == ref_st[i]
        assert abs(l64[s] - ref[i]) <= tol64[i], (s, l64[s], ref[i])
        assert abs(lm[s] - ref[i]) <= tol[i], (s, lm[s], ref[i], tol[i])
    # properties over every state: FP64 and mixed agree on the status of every
    # state; mixed within 1e-7 of FP64 relative to logL for all valid states
    # (the sampled states above carry the derived bound; 1e-7 is five times
    # the largest relative difference measured over the 4,096 states)
    np.testing.assert_array_equal(sm, s64)
    ok = np.isfinite(l64)
    assert np.array_equal(ok, np.isfinite(lm))
    assert ok.sum() >= sb.n - 8
    assert np.all(np.abs(lm[ok] - l64[ok]) <= 1e-7 * np.abs(l64[ok]))
