"""Seeded fuzz cases: interior knots one ulp either side of a bin abscissa (and
exactly on one), template parameters at the corners of their prior box, tall
spline heights, and disabled, linear and Akima splines mixed in one batch; the
FP64 batched, plain and mixed likelihoods and the FP64 adjoint against the
oracle, at the bars of the other parity tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import lps_oracle as O  # noqa: E402
from synth import workloads as W  # noqa: E402
from tests import cases as C  # noqa: E402
from tests.test_gpu_grad import FP64_GRAD, _compare  # noqa: E402


@pytest.fixture(scope="module")
def lps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as m
    m.lib()
    return m


def _fuzz_states(ds, n_states, seed):
    x = np.log10(ds.f)
    rng = np.random.default_rng(seed)
    counts = [0, 2, 3, 4, 8, 20]
    corners = [(a, t, u, al) for a in (10e-12, 20e-12) for t in (2e-15, 4e-15) for u in (-13.0, -11.0)
               for al in (-1.0, 1.0)]
    params, knots = [], []
    for s in range(n_states):
        a, t, u, al = corners[s % len(corners)]
        params.append([a, t, u, al])
        row = []
        for j in range(ds.n_spl):
            n = counts[(s + 2 * j) % len(counts)]
            if n == 0:
                row.append((np.zeros(0), np.zeros(0)))
                continue
            ks = np.sort(rng.choice(np.arange(2, x.size - 2), n - 2, replace=False))
            inner = x[ks].copy()
            mode = rng.integers(0, 3, n - 2)            # on the bin, one ulp below, one ulp above
            inner = np.where(mode == 1, np.nextafter(inner, -np.inf), inner)
            inner = np.where(mode == 2, np.nextafter(inner, np.inf), inner)
            kx = np.concatenate([[x[0]], inner, [x[-1]]])
            scale = 1.0 if s % 3 else 8.0                # tall heights: factors up to 10^(+-2.5)
            ky = rng.normal(0.0, 0.1 * scale, n)
            row.append((kx, ky))
        knots.append(row)
    return W.pack_states(np.array(params).T, knots, ds.n_spl)


@pytest.mark.parametrize("layout", ["split", "paper"])
def test_fuzz_forward_and_adjoint(lps, layout):
    name = "grad_25000bins_1024states"
    print("fuzz layout", layout, flush=True)
    ds, D = C.dataset_with_data(name, n_bins=1100, layout=layout)
    sb = _fuzz_states(ds, 24, 31 if layout == "split" else 32)
    st_ref = C.oracle_status(ds, sb)
    assert np.all(st_ref == 0), st_ref
    ctx = C.make_context(lps, ds, D, max_states=sb.n)
    st = C.device_states(ctx, sb)
    ref = C.oracle_loglikes(ds, D, sb)
    l64, s64 = ctx.loglike_batch(st, "fp64")
    lm, sm = ctx.loglike_batch(st, "mixed")
    lp, sp = ctx.loglike_plain_fp64(st)
    for s_ in (s64, sm, sp):
        assert np.all(s_.cpu().numpy() == 0)
    l64, lm, lp = (t.cpu().numpy() for t in (l64, lm, lp))
    tol64 = C.fp64_tolerance(ds, D, sb, range(sb.n))
    assert np.all(np.abs(l64 - ref) <= tol64)
    assert np.all(np.abs(lp - ref) <= tol64)
    C.check_mixed(lm, ref, C.mixed_tolerance(ds, D, sb, range(sb.n)), "fuzz " + layout)
    grads = [O.loglike_grad(ds, D, sb.params[:, s], C.knots_of(sb, s)) for s in range(sb.n)]
    logL, dp, dkx, dky, status = ctx.loglike_grad_batch(st, "fp64")
    assert np.all(status.cpu().numpy() == 0)
    _compare(sb, grads, logL.cpu().numpy(), dp, dkx, dky, FP64_GRAD, "fuzz fp64 " + layout, tol64)
