"""The parity checks of tests/cases.py reject a 1-nat error.

For every case that the GPU parity tests check: a planted 1-nat bias on oracle
values fails check_mixed (through its bias check where the per-state bound of a
large N K exceeds a nat), results a quarter of the bound away pass, the
systematic part of the mixed error model stays below 0.15 nats, and the FP64
bound is far below a nat.  CPU only: the oracle alone.
"""
import numpy as np
import pytest

from oracle import lps_oracle as O
from synth import workloads as W
from tests import cases as C
from tests.test_gpu_parity import LAYOUT_CASES


@pytest.mark.parametrize("case", LAYOUT_CASES, ids=[f"{c[1]}-{c[2]}" for c in LAYOUT_CASES])
def test_bounds_reject_a_one_nat_bias(case):
    name, layout, n_bins, n_states, inbetween = case
    ds, D = C.dataset_with_data(name, n_bins=n_bins, layout=layout)
    sb = W.make_states(name, ds, n_states=min(n_states, 12), inbetween=inbetween)
    ref = C.oracle_loglikes(ds, D, sb)
    tol = C.mixed_tolerance(ds, D, sb, range(sb.n))
    tol64 = C.fp64_tolerance(ds, D, sb, range(sb.n))
    assert np.all(tol64 < 1e-3), tol64
    # the model's terms of one sign: 0.2 eps sum N (D/S + 1) per state
    a64, _ = C.term_magnitudes(ds, D, sb, range(sb.n))
    nd = np.array([np.sum(ds.nk[None, :] * (D / O.psd(ds, sb.params[:, s], C.knots_of(sb, s))[0] + 1.0))
                   for s in range(sb.n)])
    assert np.all(0.2 * C.EPS32 * nd < 0.15), nd
    rng = np.random.default_rng(0)
    C.check_mixed(ref + 0.25 * tol * rng.choice([-1.0, 1.0], ref.size), ref, tol, "a quarter of the bound passes")
    with pytest.raises(AssertionError):
        C.check_mixed(ref + 1.0, ref, tol, "planted bias")
    # the same bias on the FP64 bound
    assert np.all(np.abs(1.0) > tol64)
