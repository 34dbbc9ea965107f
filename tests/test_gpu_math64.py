"""The double-precision elementary functions of the batched FP64 kernels
(exp2 by its series and from the table of 2^(j/64), log2, reciprocal, square
root, reciprocal square root, natural logarithm), each written out from a
hardware estimate, Newton steps or a truncated series, against the host C
library in units in the last place over the whole range the kernels see."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ULP = 4   # documented "within an ulp or two" of the correctly rounded result, plus the host's own error


@pytest.fixture(scope="module")
def lps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as m
    m.lib()
    return m


def _ulps(got, want):
    return np.abs(got - want) / np.spacing(np.abs(want))


@pytest.mark.parametrize("fn", ["exp2", "exp2_table"])
def test_exp2(lps, fn):
    rng = np.random.default_rng(1)
    # uniform spreads, the table's nodes j/64 and the midpoints between them
    # (|r| = 1/128, the series' worst case)
    nodes = np.arange(-640, 641, dtype=np.float64) / 64.0
    x = np.concatenate([rng.uniform(-1000.0, 1000.0, 100000), rng.uniform(-1.0, 1.0, 100000), nodes,
                        nodes + 1.0 / 128.0, np.arange(-60, 61, dtype=np.float64), [0.0, 0.5, -0.5]])
    got = lps.math64_check(fn, x).cpu().numpy()
    want = np.exp2(x)
    assert np.max(_ulps(got, want)) <= ULP, (fn, np.max(_ulps(got, want)))
    assert np.all(got[-124:-3] == want[-124:-3])   # integer powers of two are exact
    edge = lps.math64_check(fn, np.array([1100.0, -1100.0, np.nan])).cpu().numpy()
    assert edge[0] == np.inf and edge[1] == 0.0 and np.isnan(edge[2])


@pytest.mark.parametrize("fn,ref", [("log2", np.log2), ("log", np.log), ("rcp", lambda v: 1.0 / v),
                                    ("sqrt", np.sqrt), ("rsq", lambda v: 1.0 / np.sqrt(v))])
def test_positive_argument_functions(lps, fn, ref):
    rng = np.random.default_rng(2)
    x = np.concatenate([10.0 ** rng.uniform(-300.0, 300.0, 100000), rng.uniform(0.5, 2.0, 100000),
                        [1.0, 2.0, 0.25, 0.70710678118654752, 1.4142135623730951]])
    got = lps.math64_check(fn, x).cpu().numpy()
    want = ref(x)
    if fn in ("log2", "log"):
        # near x = 1 the result is small: bound the error in ulps of the argument's scale
        err = np.abs(got - want) / np.maximum(np.spacing(np.abs(want)), np.spacing(1.0) * np.abs(x - 1.0))
    else:
        err = _ulps(got, want)
    assert np.max(err) <= ULP, (fn, np.max(err))
    if fn == "log2":
        assert lps.math64_check("log2", np.array([1024.0, 0.125])).cpu().numpy().tolist() == [10.0, -3.0]
    if fn == "sqrt":
        assert lps.math64_check("sqrt", np.array([0.0, 4.0, 2.25])).cpu().numpy().tolist() == [0.0, 2.0, 1.5]
