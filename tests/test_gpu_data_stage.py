"""Device data stage against the oracle: periodograms (hipFFT) with and without
a window and the XYZ -> AET combination, segment averaging, response
interpolation, and a time series taken through the device data stage into a
context whose log-likelihoods match the oracle's own data stage + likelihood."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import data_stage as DS  # noqa: E402
from oracle import lps_oracle as O  # noqa: E402
from synth import workloads as W  # noqa: E402
from tests import cases as C  # noqa: E402


@pytest.fixture(scope="module")
def lps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("n_t,window,aet", [(1 << 15, False, False), ((1 << 14) + 17, True, False),
                                            (1 << 15, True, True)])
def test_periodogram_and_average_match_oracle(lps, n_t, window, aet):
    rng = np.random.default_rng(n_t)
    dt = 7.5
    x = rng.normal(0.0, 1.0, (3, n_t)) * np.array([[1.0], [3.0], [0.2]])
    w = np.hanning(n_t) if window else None
    xo = DS.xyz_to_aet(x) if aet else x
    f_ref, P_ref = DS.periodogram(xo, dt, window=w)
    f, P = lps.data_periodogram(torch.as_tensor(x, device="cuda"), dt, window=w, xyz_to_aet=aet)
    P = P.cpu().numpy()
    np.testing.assert_allclose(f.cpu().numpy(), f_ref, rtol=1e-15)
    scale = P_ref.max(axis=1, keepdims=True)
    assert np.all(np.abs(P - P_ref) <= 1e-11 * scale + 1e-12 * np.abs(P_ref))
    k0, seg, n_seg = 5, 16, (f_ref.size - 5) // 16
    fs, D, nu = lps.data_average(f, torch.as_tensor(P_ref, device="cuda"), k0, seg, n_seg)
    fs_r, D_r, nu_r = DS.average_segments(f_ref, P_ref, k0, seg, n_seg)
    np.testing.assert_allclose(D.cpu().numpy(), D_r, rtol=1e-13)
    np.testing.assert_allclose(fs.cpu().numpy(), fs_r, rtol=1e-14)
    assert np.all(nu.cpu().numpy() == nu_r)
    with pytest.raises(lps.LpsError):
        lps.data_average(f, torch.as_tensor(P_ref, device="cuda"), k0, seg, n_seg + 2)


def test_response_interpolation_matches_oracle(lps):
    gf = np.logspace(np.log10(5e-6), -1, 400)
    gR = W.response_standin(gf)
    f = np.linspace(1e-4, 2.9e-2, 5001)
    got = lps.data_response(gf, gR, torch.as_tensor(f, device="cuda")).cpu().numpy()
    ref = DS.interp_response(gf, gR, f)
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    out = lps.data_response(gf, gR, torch.as_tensor([1e-6, 0.5], device="cuda")).cpu().numpy()
    assert np.isnan(out).all()


def test_time_series_to_loglike_end_to_end(lps):
    name = "grad_25000bins_1024states"
    n_t, dt, seg = 1 << 17, 15.0, 8
    nf = n_t // 2 + 1
    f_all = np.arange(nf) / (n_t * dt)
    k_lo, k_hi = int(np.ceil(1e-4 * n_t * dt)), int(np.floor(2.9e-2 * n_t * dt))
    band = np.arange(k_lo, k_hi + 1)
    # a truth state on the band, its PSD, and a series with that PSD (flat far outside)
    ref = W.make_dataset(name, n_bins=600, layout="split")
    ds_band = W.Dataset(f=f_all[band], nk=np.ones(band.size), R=W.response_standin(f_all[band]), Rfg=None,
                        chi=np.ones((3, band.size)), truth=ref.truth, layout="split", n_spl=3,
                        route=W.route_table("split"))
    truth = W.make_states(name, ds_band, n_states=1, inbetween=(2, 5))
    S_band = O.psd(ds_band, truth.params[:, 0], C.knots_of(truth, 0))[0]
    psd = np.full((3, nf), 1e-44)
    psd[:, band] = S_band
    x = W.colored_series(np.random.default_rng(77), psd, n_t, dt)
    n_seg = band.size // seg
    gf = np.logspace(np.log10(5e-6), -1, 600)
    gR = W.response_standin(gf)
    # oracle data stage
    f_ref, P_ref = DS.periodogram(x, dt)
    fs_r, D_r, nu_r = DS.average_segments(f_ref, P_ref, k_lo, seg, n_seg)
    R_r = DS.interp_response(gf, gR, fs_r)
    ds_o = W.Dataset(f=fs_r, nk=nu_r, R=R_r, Rfg=None, chi=np.ones((3, n_seg)), truth=truth, layout="split",
                     n_spl=3, route=W.route_table("split"))
    sb = W.make_states(name, ds_o, n_states=6, inbetween=(0, 6))
    want = C.oracle_loglikes(ds_o, D_r, sb)
    # device data stage straight into a context
    xd = torch.as_tensor(x, device="cuda")
    f, P = lps.data_periodogram(xd, dt)
    fs, D, nu = lps.data_average(f, P, k_lo, seg, n_seg)
    R = lps.data_response(gf, gR, fs)
    ctx = lps.Context(fs, nu, D, R, ds_o.route, 3, max_states=sb.n, f_knee=ds_o.f_knee, arm_length=ds_o.arm_length)
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    got64 = ctx.loglike_batch(st, "fp64")[0].cpu().numpy()
    gotm = ctx.loglike_batch(st, "mixed")[0].cpu().numpy()
    # the device's data and the numpy data come from different FFTs (they agree
    # to about 1e-12), so the FP64 bound adds that to the evaluation's own
    tol64 = C.fp64_tolerance(ds_o, D_r, sb, range(sb.n)) + 1e-11 * np.abs(want)
    assert np.all(np.abs(got64 - want) <= tol64), (got64, want)
    assert np.all(np.abs(gotm - want) <= C.mixed_tolerance(ds_o, D_r, sb, range(sb.n)) + 1e-11 * np.abs(want))


def test_planned_periodogram_matches_oracle_and_replays_from_a_graph(lps):
    """The planned periodogram (plan and temporaries made once) gives the oracle's
    periodogram, equals the one-off call bit for bit, and replays from a HIP graph
    with the eager result on every replay (eager work in between)."""
    n_t, dt = (1 << 15) + 6, 5.0
    rng = np.random.default_rng(31)
    x = torch.as_tensor(rng.normal(0.0, 1.0, (3, n_t)), device="cuda")
    w = torch.as_tensor(np.hanning(n_t), device="cuda")
    plan = lps.DataPlan(3, n_t)
    P = plan.periodogram(x, dt, window=w, xyz_to_aet=True)
    _, P1 = lps.data_periodogram(x, dt, window=w, xyz_to_aet=True)
    torch.cuda.synchronize()
    assert torch.equal(P, P1)
    f_ref, P_ref = DS.periodogram(DS.xyz_to_aet(x.cpu().numpy()), dt, window=np.hanning(n_t))
    scale = P_ref.max(axis=1, keepdims=True)
    assert np.all(np.abs(P.cpu().numpy() - P_ref) <= 1e-11 * scale + 1e-12 * np.abs(P_ref))
    # graph capture of the planned call into a fixed output
    out = torch.empty_like(P)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.periodogram(x, dt, window=w, xyz_to_aet=True, out=out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.periodogram(x, dt, window=w, xyz_to_aet=True, out=out)
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, P), rep
        # eager work between replays, on another input
        plan.periodogram(x * 2.0, dt, window=w, xyz_to_aet=True)
        torch.cuda.synchronize()
    plan.close()
