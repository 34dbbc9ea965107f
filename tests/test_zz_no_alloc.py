"""The allocation-free plain FP64 entry point against the context-based one.

lps_loglike_plain_fp64_noalloc keeps its per-block partial sums in a
device-resident array instead of context workspace.  Two calls in a row, the
second on a smaller dataset (fewer bins, fewer states, another layout), must
each give exactly the logL and status words of lps_loglike_plain_fp64 on the
same inputs, and agree with the oracle; sizes beyond the array are refused on
the host before anything is launched.
"""
import numpy as np
import pytest
import torch

import paper_2507_06300_amd as m
from oracle import lps_oracle as O
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _case(name, n_bins, layout, n_states, seed_offset):
    ds = W.make_dataset(name, n_bins=n_bins, layout=layout)
    truth = [ds.truth.knots(0, j) for j in range(ds.n_spl)]
    S0, _, _ = O.psd(ds, ds.truth.params[:, 0], truth)
    D = S0 * ds.chi
    sb = W.make_states(name, ds, n_states=n_states, inbetween=(0, 8), seed_offset=seed_offset)
    params = sb.params.copy()
    params[1, 1] = -params[1, 1]          # one invalid state (A_TM <= 0)
    sb = W.StateBatch(params=params, knot_off=sb.knot_off, knot_x=sb.knot_x, knot_y=sb.knot_y, n_spl=sb.n_spl)
    return ds, D, sb


def _oracle(ds, D, sb):
    return np.array([O.loglike(ds, D, sb.params[:, s], [sb.knots(s, j) for j in range(sb.n_spl)])
                     for s in range(sb.n)])


def test_noalloc_equals_context_entry_point_on_two_calls():
    cases = [("grad_25000bins_1024states", 3000, "split", 6, 0),
             ("sweep_250000bins_2048chains", 700, "split_fg", 3, 1)]
    runs = []
    for name, K, layout, n, seed in cases:
        ds, D, sb = _case(name, K, layout, n, seed)
        print(f"no-alloc case {name} K={K} layout={layout} states={n}", flush=True)
        ctx = m.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=sb.n, device="cuda:0")
        st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
        got, gst = m.loglike_plain_fp64_noalloc(ctx.f, ctx.nk, ctx.D, ctx.R, ds.route, ds.n_spl, st, Rfg=ctx.Rfg)
        runs.append((ds, D, sb, ctx, st, got, gst))
    # both calls issued back to back; now the context path for each
    for ds, D, sb, ctx, st, got, gst in runs:
        ref, rst = ctx.loglike_plain_fp64(st)
        torch.cuda.synchronize()
        assert torch.equal(got.cpu(), ref.cpu()), (got, ref)
        assert torch.equal(gst.cpu(), rst.cpu())
        orc = _oracle(ds, D, sb)
        g = got.cpu().numpy()
        assert np.array_equal(np.isinf(g), np.isinf(orc))
        fin = np.isfinite(orc)
        assert fin.sum() == sb.n - 1
        assert np.all(np.abs(g[fin] - orc[fin]) <= 1e-12 * np.abs(orc[fin])), (g, orc)
        assert gst.cpu().numpy()[1] & O.ST_AMPLITUDE


def test_noalloc_refuses_sizes_beyond_its_array():
    ds, D, sb = _case("grad_25000bins_1024states", 300, "split", 2, 2)
    f = torch.as_tensor(ds.f, device="cuda:0")
    nk = torch.as_tensor(ds.nk, device="cuda:0")
    Dt = torch.as_tensor(D, device="cuda:0")
    R = torch.as_tensor(ds.R, device="cuda:0")
    ctx = m.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, max_states=sb.n, device="cuda:0")
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    d = m._Desc()
    d.n_bins = (1 << 24) + 1        # one block more than the array holds: refused before any launch
    d.f, d.nk, d.D, d.R, d.Rfg = f.data_ptr(), nk.data_ptr(), Dt.data_ptr(), R.data_ptr(), None
    d.f_knee, d.arm_length, d.n_spl, d.k_max = 1e-3, 2.5e9, ds.n_spl, 64
    flat = [int(v) for row in ds.route for v in row]
    for i in range(12):
        d.route[i] = flat[i]
    out = torch.empty(sb.n, dtype=torch.float64, device="cuda:0")
    c = st._c()
    import ctypes
    code = m.lib().lps_loglike_plain_fp64_noalloc(ctypes.byref(d), ctypes.byref(c), ctypes.c_void_p(out.data_ptr()),
                                                  None, None)
    assert code == 3   # LPS_E_CAPACITY
