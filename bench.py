#!/usr/bin/env python3
"""Throughput of the batched flexible-PSD / Whittle log-likelihood on one MI355X.

One step = one batched logL evaluation (mixed precision: FP32 per-bin terms,
FP64 per-state reduction) of every state of the workload, inputs resident in
HBM, replayed from a captured HIP graph.  The default workload is the full
one-year unaveraged periodogram (912,085 bins x 3 channels, N_k = 1) with
4,096 states (64 walkers x 16 temperatures x 4 reversible-jump branches).

Printed: one JSON line with the headline value (state.bin evals/s of the
mixed batched path) plus, measured in the same run on the same GPU, the FP64
batched path, the plain FP64 per-state path (on a stated state sample), the
mixed-vs-FP64 error per result, the ALU roofline of the dominant kernel, and
the FP64 CPU oracle timed on a bounded sample of the host's cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "logL state·bin evals/s, batched mixed vs plain FP64 (same GPU); grad evals/s"
UNIT = "state·bin evals/s"

# Algorithmic work per state.bin of the split layout (3 exponent groups, the
# A and E channels merged): three spline exponentials (t, Horner, scale, exp2),
# the power law of the background, PSD assembly, a reciprocal, a multiply, a
# logarithm and two FMAs per distinct channel, and a compensated accumulation:
# about 35 VALU + 8 transcendental instructions, counted as 55 FLOP.
ALGO_FLOP_PER_STATE_BIN = 55
# The paper's own layout (one noise spline per channel, a shared signal
# spline, three distinct channels): four spline exponentials, the power law,
# PSD assembly for three channels and three reciprocals and logarithms,
# about 47 VALU + 11 transcendental instructions, counted as 75 FLOP.
PAPER_FLOP_PER_STATE_BIN = 75
# The adjoint: about twice the forward work per state.bin (per channel the
# score, per spline the four moment FMAs, the template sums): 110 FLOP.
GRAD_FLOP_PER_STATE_BIN = 110

# Issue-slot view of the formulation the kernel implements (the power law is
# folded into the background exponent, one reciprocal and one logarithm serve
# both channels):
#   per group   : cubic in the bin abscissa (3 FMA) and exp2         -> 3 + 1 trans
#   assembly    : 2 channels x 3 groups, one FMA each                -> 6
#   likelihood  : P = S0 S1, num (mul + fma), rcp(P), log2(P S0),
#                 acc += num r, acc += NL lg                          -> 6 + 2 trans
#   accumulate  : one add into the lane's partial                     -> 1
MIXED_FP32_OPS = 3 * 3 + 6 + 6 + 1                  # 22 FP32 VALU instructions
MIXED_TRANS_OPS = 3 + 2                              # exp2 x3, rcp, log2

# MI355X FP32 vector peak: 256 CUs x 128 FP32 FMA lanes/clock x 2 FLOP x
# 2.4 GHz = 157.3 TFLOP/s, i.e. 78.6e12 FMA issue slots/s.  gfx950 issues
# ordinary (non-packed) v_fma_f32 at close to that rate (a dependent-chain
# microbenchmark in the library measures it), so it is the ceiling here.
PEAK_FMA_TFLOPS = 157.3


FORWARD_SOURCES = ["paper_2507_06300_amd/csrc/lps_forward.hip", "paper_2507_06300_amd/csrc/lps_batched.hpp",
                   "paper_2507_06300_amd/csrc/lps_internal.hpp"]
TRAFFIC_PROFILE = "profiles/k_forward_year_912085bins_4096states.md"


def profiled_traffic(workload, shape):
    """HBM bytes per launch of the mixed forward kernel from the committed
    rocprofv3 PMC summary, or None if the kernel sources or the launch shape
    differ from what was profiled (the counters then describe another kernel)."""
    return profiled_forward_field(workload, f"traffic_bytes_per_launch_mixed_{shape[0]}x{shape[1]}")


def profiled_forward_field(workload, key):
    """A machine-readable field of the committed forward-kernel summary, or None
    if the kernel sources no longer hash to the profiled ones."""
    import hashlib
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if workload != "year_912085bins_4096states" or not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in FORWARD_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("    ") and "_" in line.split(":")[0]:
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("forward_source_sha256_16") != h.hexdigest()[:16]:
        return None
    return float(fields[key]) if key in fields else None


def flop_roofline(state_bins, flop_per_state_bin, kernel_ms, peak_tflops, kernel):
    """Algorithmic FLOP of one launch over the kernel's measured duration, against a peak."""
    achieved = state_bins * flop_per_state_bin / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak_tflops, "unit": "TFLOP/s",
            "frac": round(achieved / peak_tflops, 4), "kernel": kernel, "kernel_ms": round(kernel_ms, 4),
            "flop_per_state_bin": flop_per_state_bin, "state_bins_per_launch": state_bins}


def fp64_roofline(workload, state_bins, s_per_call):
    """Issue share of the FP64 batched forward from the committed counter summary
    (VALU lane-instructions per state.bin, every one counted at the FP64 rate),
    or None if the kernel sources changed since they were counted."""
    v = profiled_forward_field(workload, "valu_lane_instr_per_state_bin_fp64")
    if v is None:
        return None
    wi = v * state_bins / 64.0 / s_per_call
    return {"bound": "alu", "achieved": round(wi, 1), "peak": PEAK_FP64_WAVE_INSTR_PER_S,
            "unit": "FP64 VALU wave instructions/s", "frac": round(wi / PEAK_FP64_WAVE_INSTR_PER_S, 4),
            "valu_lane_instr_per_state_bin": v,
            "timed": "whole call (coefficients + forward + finalize); an upper bound on the issue share, since "
                     "32-bit instructions issue faster than FP64 ones"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="year_912085bins_4096states")
    p.add_argument("--plain-states", type=int, default=64,
                   help="states timed on the plain FP64 per-state path (per-state cost is uniform)")
    p.add_argument("--cpu-states", type=int, default=128, help="states in the CPU oracle sample")
    p.add_argument("--cpu-cov-states", type=int, default=32, help="states in the full-covariance CPU sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-grad", action="store_true")
    p.add_argument("--grad-workload", default="grad_25000bins_1024states")
    p.add_argument("--copy-check", action="store_true",
                   help="also run one 1 GiB device-to-device copy (HBM counter calibration)")
    p.add_argument("--eager", action="store_true", help="time eager calls instead of graph replays")
    p.add_argument("--sweeps", type=int, default=1000,
                   help="sampler sweeps timed on the sweep workload (0 skips the sampler leg)")
    p.add_argument("--sweep-workload", default="sweep_250000bins_2048chains")
    p.add_argument("--no-data", action="store_true", help="skip the data-stage leg")
    p.add_argument("--no-cov", action="store_true", help="skip the full-covariance leg")
    p.add_argument("--no-paper", action="store_true", help="skip the paper-layout forward leg")
    p.add_argument("--no-small", action="store_true", help="skip the small-configuration legs")
    p.add_argument("--launch", default="",
                   help="fixed launch shapes, e.g. mixed=8x84,fp64=4x64 (default: the library's default shapes)")
    p.add_argument("--autotune", action="store_true",
                   help="time the headline at the autotuner's pick instead of the library's default shapes")
    return p.parse_args()


EAGER = False
PLAIN_CALLS = 20


def median_call_seconds(torch, fn, calls):
    """Median duration of `calls` eager calls of fn (HIP events around each)."""
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e-3


def timed_graph(torch, fn, steps, warmup):
    """Capture fn() into a graph, replay warmup + steps times; returns seconds for `steps`."""
    if EAGER:
        for _ in range(max(1, warmup)):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3, None
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(max(1, warmup)):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3, g


# Inputs of the CPU legs, set before the worker processes are forked.
_CPU = {}


def cpu_workers():
    """Worker processes for the CPU legs: the cores this process may run on,
    at most 16 (one GPU's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_map(fn, idx):
    """fn over idx in worker processes forked from this one (called before the
    process touches the GPU; the workers run numpy only)."""
    import multiprocessing as mp
    n = cpu_workers()
    if n == 1:
        return [fn(i) for i in idx], 1
    with mp.get_context("fork").Pool(n) as pool:
        return pool.map(fn, idx, chunksize=1), n


def _cpu_diag_one(s):
    from oracle import lps_oracle as O
    ds, D, sb = _CPU["diag"]
    return O.loglike(ds, D, sb.params[:, s], [sb.knots(s, j) for j in range(sb.n_spl)])


def cpu_baseline(name, n_states):
    """Time the FP64 oracle on a bounded sample of the workload (CPU leg), one
    state per task over the host's cores."""
    from oracle import lps_oracle as O
    from synth import workloads as W
    ds = W.make_dataset(name)
    truth = [ds.truth.knots(0, j) for j in range(ds.n_spl)]
    S0, _, _ = O.psd(ds, ds.truth.params[:, 0], truth)
    D = S0 * ds.chi
    sb = W.make_states(name, ds)
    _CPU["diag"] = (ds, D, sb)
    idx = list(range(min(n_states, sb.n)))
    t0 = time.perf_counter()
    _, cores = _cpu_map(_cpu_diag_one, idx)
    dt = time.perf_counter() - t0
    K = ds.f.size
    return {"value": len(idx) * K / dt, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} of {sb.n} states x {K} bins x 3 channels of {name} "
                      f"(numpy FP64, one state per process, {cores} processes), {dt:.1f} s"}


# Full-covariance leg: the one-year grid with the paper's layout (one noise
# spline per channel, one signal spline) plus three correlation splines.
COV_WORKLOAD = "year_912085bins_4096states"
COV_LAYOUT = "paper"
COV_CORR_INBETWEEN = (0, 30)
# Algorithmic work per state.bin of that layout, counting an add or multiply
# as 1, an FMA as 2 and each exp10 / sqrt / tanh / division / log as 1:
#   7 spline cubics (1 sub + 3 FMA)                                    49
#   power-law exponent (sub + FMA)                                      3
#   Sn_c, Sh_c, C_cc for 3 channels                                    30
#   vine (2 squares, products, FMA)                                     7
#   correlation form: 1/(s0 s1 s2), Delta^-1, rho_ab                   14
#   minors, determinant, cofactors                                     17
#   trace numerator (scaled data, 6 products and sums)                 25
#   logdet argument, N_k (tr + ld)                                      5
#   exp10 x5, sqrt x7, tanh x3, division x5, log x1                    21
COV_FLOP_PER_STATE_BIN = 171
PEAK_FP64_TFLOPS = 78.6
# FP64 VALU issue: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 FP64 instruction per
# SIMD every 4 cycles.
PEAK_FP64_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4
# sources of the evaluation kernel (the per-bin table builder's template header
# runs once at create and is not part of the profiled kernel)
COV_SOURCES = ["paper_2507_06300_amd/csrc/lps_cov.hip", "paper_2507_06300_amd/csrc/lps_cov_common.hpp",
               "paper_2507_06300_amd/csrc/lps_math64.hpp"]
COV_PROFILE = "profiles/k_cov_eval_year_912085bins_4096states.md"
COV_GRAD_SOURCES = ["paper_2507_06300_amd/csrc/lps_cov_grad.hip", "paper_2507_06300_amd/csrc/lps_cov_common.hpp",
                    "paper_2507_06300_amd/csrc/lps_spline_back.hpp", "paper_2507_06300_amd/csrc/lps_math64.hpp"]
COV_GRAD_PROFILE = "profiles/k_cov_grad_year_912085bins_4096states.md"


def _profiled_valu(profile, sources, key):
    """VALU lane-instructions per state.bin of a kernel from its committed
    counter summary, or None if the kernel's sources changed since."""
    import hashlib
    path = os.path.join(ROOT, profile)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("    ") and "_" in line.split(":")[0]:
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get(key) != h.hexdigest()[:16]:
        return None
    v = fields.get("valu_lane_instr_per_state_bin")
    return float(v) if v else None


def profiled_cov_valu():
    return _profiled_valu(COV_PROFILE, COV_SOURCES, "cov_source_sha256_16")


def profiled_cov_grad_valu():
    return _profiled_valu(COV_GRAD_PROFILE, COV_GRAD_SOURCES, "cov_grad_source_sha256_16")


def _cov_states(W, ds, name, rng_seed):
    sb = W.make_states(name, ds)
    x_lo, x_hi = W.band_edges(ds.f)
    return W.append_splines(sb, np.random.default_rng(rng_seed), 3, COV_CORR_INBETWEEN, x_lo, x_hi, 0.5)


def cov_bench(torch, lps, W, args, dev):
    """Dense 3x3 covariance likelihood (FP64) of every state of the one-year workload."""
    name = COV_WORKLOAD
    ds = W.make_dataset(name, layout=COV_LAYOUT)
    K = ds.f.size
    nb = ds.n_spl
    corr = (nb, nb + 1, nb + 2)
    x_lo, x_hi = W.band_edges(ds.f)
    truth = W.append_splines(ds.truth, np.random.default_rng(180), 3, (1, 4), x_lo, x_hi, 0.5)
    # data: complex-Wishart draws around the library's own model covariance at the truth state
    ctx0 = lps.CovContext(ds.f, ds.nk, np.ones((6, K)), ds.R, ds.route, corr, nb + 3, max_states=1, device=dev)
    C6, _ = ctx0.build(ctx0.states(truth.params, truth.knot_off, truth.knot_x, truth.knot_y))
    ctx0.close()
    C6 = C6[0].cpu().numpy()
    C = np.empty((K, 3, 3))
    for i, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        C[:, a, b] = C6[i]
        C[:, b, a] = C6[i]
    Pc = W.complex_wishart_mean(np.random.default_rng(181), C, np.rint(ds.nk))
    P6 = np.stack([Pc[:, a, b].real for (a, b) in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])
    del C, Pc
    sb = _cov_states(W, ds, name, 182)
    n = sb.n
    ctx = lps.CovContext(ds.f, ds.nk, P6, ds.R, ds.route, corr, nb + 3, max_states=n, device=dev)
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    steps = max(3, args.steps // 4)
    t, _ = timed_graph(torch, lambda: ctx.loglike_batch(st, out=out, status=status), steps, 1)
    per = t / steps
    valid = int((status == 0).sum().item())
    achieved = n * K * COV_FLOP_PER_STATE_BIN / per / 1e12
    log(f"cov: {per * 1e3:.2f} ms/call, {n * K / per:.3e} state.bin/s, {achieved:.2f} TFLOP/s FP64 "
        f"({achieved / PEAK_FP64_TFLOPS:.1%}); {valid}/{n} states valid")
    # the adjoint (logL and every parameter and knot derivative) of the same batch
    tg, _ = timed_graph(torch, lambda: ctx.loglike_grad_batch(st), steps, 1)
    per_g = tg / steps
    log(f"cov adjoint: {per_g * 1e3:.2f} ms/call, {n * K / per_g:.3e} state.bin/s")
    ctx.close()
    gv = profiled_cov_grad_valu()
    grad_roof = None
    if gv is not None:
        # issue-bound FP64 arithmetic: achieved = wave instructions per second
        wi = gv * n * K / 64.0 / per_g
        grad_roof = {"bound": "alu", "achieved": round(wi, 1), "peak": PEAK_FP64_WAVE_INSTR_PER_S,
                     "unit": "FP64 VALU wave instructions/s", "frac": round(wi / PEAK_FP64_WAVE_INSTR_PER_S, 4),
                     "valu_lane_instr_per_state_bin": gv}
    valu = profiled_cov_valu()
    issue = None if valu is None else valu * n * K / 64.0 / per / PEAK_FP64_WAVE_INSTR_PER_S
    return {"workload": name, "layout": COV_LAYOUT, "n_bins": K, "n_states": n, "splines_per_state": nb + 3,
            "grad": {"ms_per_call": per_g * 1e3, "state_bin_grad_evals_per_s": n * K / per_g,
                     "timed": "whole call (coefficients + adjoint + spline backward), graph replays",
                     "roofline": grad_roof},
            "correlation_in_between_knots": list(COV_CORR_INBETWEEN), "dtype": "f64",
            "value": n * K / per, "unit": UNIT, "ms_per_call": per * 1e3, "valid_states": valid,
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                         "flop_per_state_bin": COV_FLOP_PER_STATE_BIN, "state_bins_per_launch": n * K,
                         "timed": "whole call (coefficients + evaluation + finalize), graph replays",
                         "valu_lane_instr_per_state_bin": valu, "fp64_issue_frac": None if issue is None else round(issue, 4)}}


def cpu_baseline_cov(name, n_states):
    """The full-covariance oracle on a few states of the same workload (CPU leg)."""
    from oracle import covariance as CV
    from synth import workloads as W
    ds = W.make_dataset(name, layout=COV_LAYOUT)
    nb = ds.n_spl
    cds = CV.CovDataset(base=ds, corr=(nb, nb + 1, nb + 2), n_spl=nb + 3)
    x_lo, x_hi = W.band_edges(ds.f)
    truth = W.append_splines(ds.truth, np.random.default_rng(180), 3, (1, 4), x_lo, x_hi, 0.5)
    C, _, _ = CV.covariance(cds, truth.params[:, 0], [truth.knots(0, j) for j in range(truth.n_spl)])
    P6 = CV.unique_entries(W.complex_wishart_mean(np.random.default_rng(181), C, np.rint(ds.nk)).real)
    del C
    sb = _cov_states(W, ds, name, 182)
    _CPU["cov"] = (cds, P6, sb)
    idx = list(range(min(n_states, sb.n)))
    t0 = time.perf_counter()
    _, cores = _cpu_map(_cpu_cov_one, idx)
    dt = time.perf_counter() - t0
    K = ds.f.size
    return {"value": len(idx) * K / dt, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} of {sb.n} states x {K} bins (3x3 per bin) of {name}, {COV_LAYOUT} layout "
                      f"+ 3 correlation splines (numpy FP64, one state per process, {cores} processes), {dt:.1f} s"}


def _cpu_cov_one(s):
    from oracle import covariance as CV
    cds, P6, sb = _CPU["cov"]
    return CV.loglike(cds, P6, sb.params[:, s], [sb.knots(s, j) for j in range(sb.n_spl)])


def main():
    args = parse()
    global EAGER
    EAGER = args.eager
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(states are independent: the path would shard by walker, each GPU holding a replica of the "
              "per-bin tables, with no communication per likelihood call)", file=sys.stderr)
        sys.exit(2)
    # CPU legs first: their worker processes are forked before this process
    # initialises the GPU
    cpu = None
    if not args.no_cpu:
        log(f"cpu oracle sample ({cpu_workers()} processes) ...")
        cpu = cpu_baseline(args.workload, args.cpu_states)
        log(f"  {cpu['value']:.3e} state.bin/s")
        if not args.no_cov:
            cpu["cov"] = cpu_baseline_cov(COV_WORKLOAD, args.cpu_cov_states)
            log(f"  cov: {cpu['cov']['value']:.3e} state.bin/s")

    import torch
    import paper_2507_06300_amd as lps
    from synth import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    name = args.workload
    wl = W.WORKLOADS[name]
    ds = W.make_dataset(name)
    sb = W.make_states(name, ds)
    K, n = ds.f.size, sb.n
    log(f"workload {name}: {K} bins x {n} states ({wl.note})")

    # Data: D = S(truth) * chi, with S(truth) from the library's own psd_build.
    ctx0 = lps.Context(ds.f, ds.nk, np.ones((3, K)), ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg,
                       max_states=1, device=dev)
    S0, _ = ctx0.psd_build(ctx0.states(ds.truth.params, ds.truth.knot_off, ds.truth.knot_x, ds.truth.knot_y))
    D = S0[0] * torch.as_tensor(ds.chi, device=dev)
    ctx0.close()
    ctx = lps.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=n, device=dev,
                      max_grad_states=0)
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)

    if args.copy_check:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # --- launch shape of each precision: the library's default for this batch
    # (deterministic, and the shape the committed counter summaries describe),
    # a fixed one, or the autotuner's pick -------------------------------------
    shapes = {}
    fixed = dict(kv.split("=") for kv in args.launch.split(",") if kv)
    for prec in ("mixed", "fp64"):
        ms, how = None, "default"
        if prec in fixed:
            b, t = (int(v) for v in fixed[prec].split("x"))
            ctx.set_launch(prec, b, t)
            how = "fixed"
        elif args.autotune:
            ms, _ = ctx.autotune(st, prec, reps=3)
            how = "autotuned"
        else:
            ctx.set_launch(prec, 0, 0)
        shp = ctx.get_launch(prec, n)
        shapes[prec] = {"bins_per_lane": shp[0], "states_per_tile": shp[1], "chosen": how, "autotune_ms": ms}
        log(f"launch {prec}: bins/lane {shp[0]}, states/tile {shp[1]} ({how}{'' if ms is None else f', {ms:.3f} ms'})")

    # --- headline: mixed batched, graph-replayed -------------------------------
    log("mixed batched ...")
    t_mixed, _ = timed_graph(torch, lambda: ctx.loglike_batch(st, "mixed", out=out, status=status),
                             args.steps, args.warmup)
    logL_mixed = out.clone()
    n_bad = int((status != 0).sum().item())
    ms_mixed = t_mixed / args.steps * 1e3
    value = n * K / (t_mixed / args.steps)
    log(f"  {ms_mixed:.3f} ms/call, {value:.3e} state.bin/s, invalid states {n_bad}")

    # --- FP64 batched ------------------------------------------------------------
    log("fp64 batched ...")
    steps64 = max(3, args.steps // 4)
    t64, _ = timed_graph(torch, lambda: ctx.loglike_batch(st, "fp64", out=out, status=status), steps64, 1)
    logL64 = out.clone()
    fp64_value = n * K / (t64 / steps64)
    ctx.set_timing(True)
    for _ in range(steps64):
        ctx.loglike_batch(st, "fp64", out=out, status=status)
    kms64, nl64 = ctx.kernel_time()
    ctx.set_timing(False)
    k64_ms = kms64 / nl64
    log(f"  {t64 / steps64 * 1e3:.3f} ms/call, {fp64_value:.3e} state.bin/s (kernel {k64_ms:.3f} ms)")

    # error of the mixed path, per result, against the FP64 batched path
    lm, l64 = logL_mixed.cpu().numpy(), logL64.cpu().numpy()
    both = np.isfinite(lm) & np.isfinite(l64)
    d = lm[both] - l64[both]
    ref = l64[both]
    i0 = int(np.nonzero(both)[0][0])
    dd = (lm[both] - lm[i0]) - (l64[both] - l64[i0])
    mixed_err = {"vs": "fp64 batched (oracle-checked)", "states_compared": int(both.sum()),
                 "invalid_fp64": int((~np.isfinite(l64)).sum()), "invalid_mixed": int((~np.isfinite(lm)).sum()),
                 "max_abs": float(np.abs(d).max()), "median_abs": float(np.median(np.abs(d))),
                 "p99_abs": float(np.quantile(np.abs(d), 0.99)), "max_rel": float(np.max(np.abs(d) / np.abs(ref))),
                 "max_abs_logL_difference": float(np.abs(dd).max())}
    mixed_err["error_model"] = error_model_ratio(torch, lps, W, ctx, ds, sb, D, lm, l64, both)
    log(f"  mixed error / model bound: max {mixed_err['error_model']['max_ratio']:.3f} over "
        f"{mixed_err['error_model']['states']} states (tests allow {mixed_err['error_model']['test_constant']})")

    # --- dominant kernel duration (HIP events around the main kernel) ----------
    ctx.set_timing(True)
    for _ in range(args.steps):
        ctx.loglike_batch(st, "mixed", out=out, status=status)
    kms, nl = ctx.kernel_time()
    ctx.set_timing(False)
    k_avg_ms = kms / nl
    fma_ns, trans_cost, lane_rate = lps.valu_probe(0)
    achieved = n * K * ALGO_FLOP_PER_STATE_BIN / (k_avg_ms * 1e-3) / 1e12
    slots = MIXED_FP32_OPS + MIXED_TRANS_OPS * trans_cost
    slot_rate = n * K * slots / (k_avg_ms * 1e-3)
    traffic = profiled_traffic(name, (shapes["mixed"]["bins_per_lane"], shapes["mixed"]["states_per_tile"]))
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FMA_TFLOPS, 4), "traffic": traffic,
                "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                "kernel": "k_forward<float,split,AE-merged>", "kernel_ms": round(k_avg_ms, 4),
                "flop_per_state_bin": ALGO_FLOP_PER_STATE_BIN, "state_bins_per_launch": n * K,
                "issue_slots_per_state_bin": round(slots, 2), "trans_cost_fma_slots": round(trans_cost, 3),
                "issue_frac": round(slot_rate / (PEAK_FMA_TFLOPS * 0.5e12), 4),
                "issue_frac_of_measured_fma_rate": round(slot_rate / lane_rate, 4),
                "measured_fma_lane_instr_per_s": lane_rate}
    log(f"  main kernel {k_avg_ms:.3f} ms, {achieved:.1f} TFLOP/s ({achieved / PEAK_FMA_TFLOPS:.1%}); "
        f"issue slots {slot_rate:.3e}/s ({roofline['issue_frac']:.1%} of peak, "
        f"{roofline['issue_frac_of_measured_fma_rate']:.1%} of measured FMA rate), trans cost {trans_cost:.2f}")

    result = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": ms_mixed, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
              "config": {"workload": name, "n_bins": K, "n_states": n, "channels": 3,
                         "N_k": wl.nk, "in_between_knots": list(wl.inbetween), "layout": ds.layout,
                         "precision": "mixed"},
              "roofline": roofline,
              "fp64_batched": {"value": fp64_value, "unit": UNIT, "ms_per_call": t64 / steps64 * 1e3,
                               "roofline": flop_roofline(n * K, ALGO_FLOP_PER_STATE_BIN, k64_ms, PEAK_FP64_TFLOPS,
                                                         "k_forward<double>"),
                               "issue_share": fp64_roofline(name, n * K, t64 / steps64)},
              "launch_shapes": shapes,
              "mixed_error": mixed_err}

    # --- plain FP64 per-state path on a state sample ---------------------------
    if not args.no_plain:
        m = min(args.plain_states, n)
        from synth.workloads import states_subset
        sub = states_subset(sb, range(m))
        stp = ctx.states(sub.params, sub.knot_off, sub.knot_x, sub.knot_y)
        lp, _ = ctx.loglike_plain_fp64(stp)
        torch.cuda.synchronize()
        tp = median_call_seconds(torch, lambda: ctx.loglike_plain_fp64(stp), PLAIN_CALLS)
        plain_value = m * K / tp
        err_plain = float((lp - logL64[:m]).abs().max().item())
        result["plain_fp64"] = {"value": plain_value, "unit": UNIT, "sample_states": m,
                                "s_per_call": tp, "timed": f"median of {PLAIN_CALLS} calls (HIP events)",
                                "max_abs_diff_vs_fp64_batched": err_plain}
        result["speedup_mixed_vs_plain"] = value / plain_value
        result["speedup_fp64_batched_vs_plain"] = fp64_value / plain_value
        log(f"plain fp64: {plain_value:.3e} state.bin/s on {m} states; mixed speedup {value / plain_value:.1f}x")

    # --- the paper's own layout on the same grid ----------------------------------
    if not args.no_paper:
        result["paper_layout"] = paper_layout_bench(torch, lps, W, args, dev)

    # --- the small configurations: plain vs batched at their own sizes ------------
    if not args.no_small:
        result["small_configs"] = small_configs_bench(torch, lps, W, args, dev)

    # --- gradient -----------------------------------------------------------------
    if not args.no_grad:
        try:
            result["grad"] = grad_bench(torch, lps, W, args, dev)
        except lps.LpsError as e:
            result["grad"] = {"error": str(e)}

    # --- sampler sweeps -------------------------------------------------------------
    if args.sweeps > 0:
        result["sampler"] = sampler_bench(torch, lps, W, args, dev)

    # --- data stage ------------------------------------------------------------------
    if not args.no_data:
        result["data_stage"] = data_stage_bench(torch, lps, dev)

    # --- full-covariance likelihood ----------------------------------------------------
    if not args.no_cov:
        result["cov"] = cov_bench(torch, lps, W, args, dev)

    # --- CPU oracle baseline (timed before the GPU legs) ------------------------------
    if cpu is not None:
        result["cpu_baseline"] = cpu

    print(json.dumps(result), flush=True)


def _dataset_context(torch, lps, W, name, dev, layout=None, max_grad_states=0):
    """Workload dataset, states and a context whose data are the library's own PSD
    of the truth state times the seeded chi draws."""
    ds = W.make_dataset(name, layout=layout)
    sb = W.make_states(name, ds)
    K = ds.f.size
    ctx0 = lps.Context(ds.f, ds.nk, np.ones((3, K)), ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=1, device=dev,
                       max_grad_states=0)
    S0, _ = ctx0.psd_build(ctx0.states(ds.truth.params, ds.truth.knot_off, ds.truth.knot_x, ds.truth.knot_y))
    D = S0[0] * torch.as_tensor(ds.chi, device=dev)
    ctx0.close()
    ctx = lps.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=sb.n, device=dev,
                      max_grad_states=max_grad_states)
    return ds, sb, ctx, ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)


# The parity tests' bound for the mixed path (tests/cases.py): |dlogL| <=
# MIXED_C * 2^-24 * sum_ck N_k (D/S + 1)(1 + |ln(S / sigma)|), sigma the nominal
# noise (15 pm, 3 fm).  Restated here so that the bench reports the same ratio.
MIXED_TEST_C = 4.0


def error_model_ratio(torch, lps, W, ctx, ds, sb, D, lm, l64, valid, n_worst=8, n_rand=8):
    """|mixed - FP64| over the error model's magnitude, on the states with the
    largest differences plus a seeded sample, with S from the library's FP64
    psd_build (the batched FP64 path is itself checked against the oracle)."""
    d = np.where(valid, np.abs(lm - l64), -1.0)
    worst = [int(i) for i in np.argsort(d)[::-1][:n_worst]]
    rng = np.random.default_rng(7)
    pool = [int(i) for i in np.nonzero(valid)[0] if int(i) not in worst]
    idx = worst + [int(i) for i in rng.choice(pool, min(n_rand, len(pool)), replace=False)]
    sub = W.states_subset(sb, idx)
    S, _ = ctx.psd_build(ctx.states(sub.params, sub.knot_off, sub.knot_x, sub.knot_y))
    nom = np.zeros((sb.params.shape[0], 1))
    nom[0, 0], nom[1, 0], nom[2, 0] = 15e-12, 3e-15, -30.0
    ns = W.pack_states(nom, [[(np.zeros(0), np.zeros(0))] * ds.n_spl], ds.n_spl)
    sig, _ = ctx.psd_build(ctx.states(ns.params, ns.knot_off, ns.knot_x, ns.knot_y))
    N = torch.as_tensor(ds.nk, device=S.device)[None, None, :]
    Dt = torch.as_tensor(D, device=S.device)[None]
    mag = (N * (Dt / S + 1.0) * (1.0 + torch.log(S / sig).abs())).sum(dim=(1, 2)).cpu().numpy()
    ratio = np.abs(lm[idx] - l64[idx]) / (2.0 ** -24 * mag)
    return {"states": len(idx), "max_ratio": float(ratio.max()), "median_ratio": float(np.median(ratio)),
            "test_constant": MIXED_TEST_C,
            "model": "|mixed - fp64| / (2^-24 sum_ck N_k (D/S + 1)(1 + |ln S/sigma|)), 8 largest differences "
                     "+ 8 seeded states"}


def graph_median_seconds(torch, fn, calls):
    """Capture fn() into a HIP graph and return the median of `calls` timed replays."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return median_call_seconds(torch, g.replay, calls)


def paper_layout_bench(torch, lps, W, args, dev):
    """The forward pass in the paper's layout (one noise spline per channel and a
    shared signal spline: four exponent groups, three distinct channels) on the
    one-year grid with the same states' draws."""
    name = args.workload
    ds, sb, ctx, st = _dataset_context(torch, lps, W, name, dev, layout="paper")
    K, n = ds.f.size, sb.n
    out = torch.empty(n, dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    res = {"workload": name, "layout": "paper", "n_bins": K, "n_states": n, "splines_per_state": ds.n_spl}
    logs = {}
    for prec in ("mixed", "fp64"):
        ms_tune, shp = ctx.autotune(st, prec, reps=2)
        steps = args.steps if prec == "mixed" else max(3, args.steps // 4)
        t, _ = timed_graph(torch, lambda: ctx.loglike_batch(st, prec, out=out, status=status), steps, 1)
        logs[prec] = out.cpu().numpy()
        ctx.set_timing(True)
        for _ in range(steps):
            ctx.loglike_batch(st, prec, out=out, status=status)
        kms, nl = ctx.kernel_time()
        ctx.set_timing(False)
        peak = PEAK_FMA_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
        res[prec] = {"value": n * K / (t / steps), "unit": UNIT, "ms_per_call": t / steps * 1e3,
                     "launch": {"bins_per_lane": shp[0], "states_per_tile": shp[1]},
                     "roofline": flop_roofline(n * K, PAPER_FLOP_PER_STATE_BIN, kms / nl, peak,
                                               f"k_forward<{'float' if prec == 'mixed' else 'double'},paper>")}
        log(f"paper layout {prec}: {t / steps * 1e3:.3f} ms/call, kernel {kms / nl:.3f} ms "
            f"({res[prec]['roofline']['frac']:.1%} of {peak})")
    ok = np.isfinite(logs["mixed"]) & np.isfinite(logs["fp64"])
    d = np.abs(logs["mixed"][ok] - logs["fp64"][ok])
    res["mixed_error"] = {"states_compared": int(ok.sum()), "max_abs": float(d.max()),
                          "median_abs": float(np.median(d)), "p99_abs": float(np.quantile(d, 0.99))}
    ctx.close()
    return res


def small_configs_bench(torch, lps, W, args, dev):
    """The two small configurations at their own sizes: the plain FP64 per-state
    path against the batched FP64 and mixed paths (medians of 20 timed calls;
    graph replays for the batched paths)."""
    out = {}
    for name in ("avg50_1000bins_64states", "daily_2497bins_320states"):
        ds, sb, ctx, st = _dataset_context(torch, lps, W, name, dev)
        K, n = ds.f.size, sb.n
        res = {"n_bins": K, "n_states": n, "layout": ds.layout, "N_k": W.WORKLOADS[name].nk,
               "in_between_knots": list(W.WORKLOADS[name].inbetween)}
        tp = median_call_seconds(torch, lambda: ctx.loglike_plain_fp64(st), PLAIN_CALLS)
        res["plain_fp64"] = {"value": n * K / tp, "unit": UNIT, "ms_per_call": tp * 1e3}
        for prec in ("fp64", "mixed"):
            ctx.autotune(st, prec, reps=3)
            o = torch.empty(n, dtype=torch.float64, device=dev)
            t = graph_median_seconds(torch, lambda: ctx.loglike_batch(st, prec, out=o), PLAIN_CALLS)
            res[f"{prec}_batched"] = {"value": n * K / t, "unit": UNIT, "ms_per_call": t * 1e3}
        res["speedup_fp64_batched_vs_plain"] = tp / (n * K / res["fp64_batched"]["value"])
        res["speedup_mixed_vs_plain"] = tp / (n * K / res["mixed_batched"]["value"])
        res["timed"] = f"median of {PLAIN_CALLS} calls each (HIP events)"
        log(f"{name}: plain {tp * 1e3:.3f} ms, fp64 batched {res['fp64_batched']['ms_per_call']:.3f} ms, "
            f"mixed {res['mixed_batched']['ms_per_call']:.3f} ms")
        ctx.close()
        out[name] = res
    return out


def grad_bench(torch, lps, W, args, dev):
    name = args.grad_workload
    ds = W.make_dataset(name)
    sb = W.make_states(name, ds)
    K, n = ds.f.size, sb.n
    ctx0 = lps.Context(ds.f, ds.nk, np.ones((3, K)), ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg,
                       max_states=1, device=dev)
    S0, _ = ctx0.psd_build(ctx0.states(ds.truth.params, ds.truth.knot_off, ds.truth.knot_x, ds.truth.knot_y))
    D = S0[0] * torch.as_tensor(ds.chi, device=dev)
    ctx0.close()
    ctx = lps.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=n, device=dev)
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    res = {"workload": name, "n_bins": K, "n_states": n}
    outs = {}
    for prec in ("mixed", "fp64"):
        steps = max(3, args.steps // 2)
        t, _ = timed_graph(torch, lambda: ctx.loglike_grad_batch(st, prec), steps, 1)
        per = t / steps
        outs[prec] = [v.cpu().numpy() for v in ctx.loglike_grad_batch(st, prec)[:4]]
        # the adjoint kernel alone (HIP events around it on the call's stream)
        ctx.set_timing(True)
        for _ in range(steps):
            ctx.loglike_grad_batch(st, prec)
        kms, nl = ctx.kernel_time()
        ctx.set_timing(False)
        k_ms = kms / nl
        peak = PEAK_FMA_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
        achieved = n * K * GRAD_FLOP_PER_STATE_BIN / (k_ms * 1e-3) / 1e12
        res[prec] = {"grad_evals_per_s": n / per, "state_bin_grad_evals_per_s": n * K / per,
                     "ms_per_call": per * 1e3,
                     "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                                  "frac": round(achieved / peak, 4), "kernel": f"k_grad<{'float' if prec == 'mixed' else 'double'}>",
                                  "kernel_ms": round(k_ms, 4), "flop_per_state_bin": GRAD_FLOP_PER_STATE_BIN,
                                  "state_bins_per_launch": n * K}}
        log(f"grad {prec}: {per * 1e3:.3f} ms/call, {n / per:.3e} grad evals/s; kernel {k_ms:.3f} ms, "
            f"{achieved:.1f} TFLOP/s ({achieved / peak:.1%})")
    # error of the mixed adjoint against the FP64 one, per result
    lm, dpm, dxm, dym = outs["mixed"]
    l6, dp6, dx6, dy6 = outs["fp64"]
    ok = np.isfinite(lm) & np.isfinite(l6)
    d = lm[ok] - l6[ok]
    i0 = int(np.nonzero(ok)[0][0])
    dd = (lm[ok] - lm[i0]) - (l6[ok] - l6[i0])
    scale = np.ones_like(dp6)
    scale[0], scale[1] = sb.params[0], sb.params[1]       # dimensionless: theta dlogL/dtheta for amplitudes
    gp = np.abs((dpm - dp6) * scale)[:, ok].max() / max(np.abs(dp6 * scale)[:, ok].max(), 1e-300)
    gy = np.abs(dym - dy6).max() / max(np.abs(dy6).max(), 1e-300)
    res["mixed_error"] = {"vs": "fp64 adjoint (oracle-checked)", "states_compared": int(ok.sum()),
                          "logL_max_abs": float(np.abs(d).max()), "logL_median_abs": float(np.median(np.abs(d))),
                          "logL_p99_abs": float(np.quantile(np.abs(d), 0.99)),
                          "max_abs_logL_difference": float(np.abs(dd).max()),
                          "grad_params_max_rel_to_largest": float(gp), "grad_heights_max_rel_to_largest": float(gy)}
    log(f"grad mixed error: logL max {res['mixed_error']['logL_max_abs']:.3g}, p99 "
        f"{res['mixed_error']['logL_p99_abs']:.3g}; params {gp:.2e}, heights {gy:.2e}")
    return res


def sampler_bench(torch, lps, W, args, dev):
    """Graph-captured PT-RJMCMC sweeps: 128 walkers x 16 temperatures on the
    250,000-bin workload with the foreground term, up to 40 in-between knots."""
    name = args.sweep_workload
    wl = W.WORKLOADS[name]
    ds = W.make_dataset(name)
    sb = W.make_states(name, ds)
    K, n = ds.f.size, sb.n
    n_temps = 16
    n_walk = n // n_temps
    betas = np.geomspace(1.0, 1e-4, n_temps)
    ctx0 = lps.Context(ds.f, ds.nk, np.ones((3, K)), ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=1,
                       device=dev, max_grad_states=0)
    S0, _ = ctx0.psd_build(ctx0.states(ds.truth.params, ds.truth.knot_off, ds.truth.knot_x, ds.truth.knot_y))
    D = S0[0] * torch.as_tensor(ds.chi, device=dev)
    ctx0.close()
    ctx = lps.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, max_states=n, device=dev)
    st = ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)
    k_in_max = wl.inbetween[1]
    sm = lps.Sampler(ctx, n_walk, betas, seed=2025, k_in_max=k_in_max, step=0.05, precision="mixed")
    sm.set_state(st)
    per_graph = 10
    sm.sweep(1)                                   # load every kernel before capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        sm.sweep(per_graph)
    torch.cuda.synchronize()
    reps = max(1, args.sweeps // per_graph)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    sweeps = reps * per_graph
    cnt = sm.counters()
    acc = {k: float(cnt[i, :, 1].sum()) / max(1.0, float(cnt[i, :, 0].sum())) for i, k in enumerate(sm.KINDS)}
    ev = 2 * sweeps * n * K       # two gradient evaluations of every chain per sweep
    log(f"sampler: {sweeps} sweeps in {sec:.2f} s ({sweeps / sec:.1f} sweeps/s), acceptance {acc}")
    res = {"workload": name, "n_bins": K, "chains": n, "walkers": n_walk, "temperatures": n_temps,
           "sweeps": sweeps, "seconds": sec, "sweeps_per_s": sweeps / sec, "ms_per_sweep": sec / sweeps * 1e3,
           "state_bin_grad_evals_per_s": ev / sec, "acceptance": acc, "graph": f"{per_graph} sweeps per graph"}
    # the chains' logL (from the mixed adjoint that drives the Metropolis tests)
    # against an FP64 evaluation of the same states
    stc, _, lchain = sm.packed_state()
    l64, _ = ctx.loglike_batch(stc, "fp64")
    a, b = lchain.cpu().numpy(), l64.cpu().numpy()
    ok = np.isfinite(a) & np.isfinite(b)
    d = a[ok] - b[ok]
    dd = (a[ok] - a[ok][0]) - (b[ok] - b[ok][0])
    res["mixed_error"] = {"vs": "fp64 batched logL of the same chain states", "chains_compared": int(ok.sum()),
                          "max_abs": float(np.abs(d).max()), "median_abs": float(np.median(np.abs(d))),
                          "p99_abs": float(np.quantile(np.abs(d), 0.99)),
                          "max_abs_logL_difference": float(np.abs(dd).max())}
    log(f"sampler chains: mixed logL vs fp64 max {res['mixed_error']['max_abs']:.3g}, "
        f"p99 {res['mixed_error']['p99_abs']:.3g}")
    # stepping-stone evidence over logL records of the timed chains (one record per sweep)
    n_rec = 64
    rec = torch.empty((n_rec, n_temps, n_walk), dtype=torch.float64, device=dev)
    for i in range(n_rec):
        sm.sweep(1)
        sm.record_logL(rec[i].view(-1))
    torch.cuda.synchronize()
    order = np.argsort(betas)                     # the reduction takes an increasing ladder
    rec_inc = rec[:, torch.as_tensor(order, device=dev), :].contiguous()
    e0.record()
    log_z, var_z, _, _ = lps.stepping_stone(betas[order], rec_inc)
    e1.record()
    torch.cuda.synchronize()
    res["evidence"] = {"records": n_rec, "log_z": log_z, "sd_log_z": float(np.sqrt(var_z)),
                       "ms": e0.elapsed_time(e1)}
    sm.close()
    # the two-step driver (templates only, then splines with the templates fixed)
    from paper_2507_06300_amd.driver import two_step
    tw = 32
    init = np.ascontiguousarray(sb.params[:, :tw * n_temps])
    burn, keep = 10, 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r2 = two_step(ctx, tw, betas, init, k_in_max, burn, keep, burn, keep, seed=7, step=0.05, precision="mixed")
    torch.cuda.synchronize()
    sec2 = time.perf_counter() - t0
    r2.sampler.close()
    res["two_step"] = {"walkers": tw, "temperatures": n_temps, "sweeps": 2 * (burn + keep), "seconds": sec2,
                       "sweeps_per_s": 2 * (burn + keep) / sec2,
                       "note": "eager sweeps with a host read of the cold chains after every kept step-1 sweep"}
    log(f"two-step driver: {2 * (burn + keep)} sweeps of {tw * n_temps} chains in {sec2:.2f} s")
    ctx.close()
    return res


def data_stage_bench(torch, lps, dev):
    """One year of three TDI series (2^21 samples at 15.05 s) through the device
    data stage: XYZ -> AET, Hann window, periodogram, band of single bins, response."""
    n_t, dt = 1 << 21, 15.05
    x = torch.randn((3, n_t), dtype=torch.float64, device=dev)
    w = torch.hann_window(n_t, periodic=False, dtype=torch.float64, device=dev)
    gf = np.logspace(np.log10(5e-6), -1, 1000)
    from synth.workloads import response_standin
    gR = response_standin(gf)
    k_lo, k_hi = int(np.ceil(1e-4 * n_t * dt)), int(np.floor(2.9e-2 * n_t * dt))
    lps.data_periodogram(x, dt, window=w, xyz_to_aet=True)     # kernels warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, P = lps.data_periodogram(x, dt, window=w, xyz_to_aet=True)
    fs, D, nu = lps.data_average(f, P, k_lo, 1, k_hi - k_lo + 1)
    R = lps.data_response(gf, gR, fs)
    torch.cuda.synchronize()
    ms_once = (time.perf_counter() - t0) * 1e3
    # planned: the transform plan and temporaries made once, then per-dataset calls
    t0 = time.perf_counter()
    plan = lps.DataPlan(3, n_t, device=dev)
    torch.cuda.synchronize()
    ms_plan = (time.perf_counter() - t0) * 1e3
    Pp = torch.empty_like(P)
    nb = k_hi - k_lo + 1
    Db = torch.empty((3, nb), dtype=torch.float64, device=dev)
    fsb = torch.empty(nb, dtype=torch.float64, device=dev)
    nub = torch.empty(nb, dtype=torch.float64, device=dev)

    def stage():
        plan.periodogram(x, dt, window=w, xyz_to_aet=True, out=Pp)
        lps.lib().lps_data_average(lps._ptr(Pp), 3, Pp.shape[1], lps._ptr(f), k_lo, 1, nb, lps._ptr(Db),
                                   lps._ptr(fsb), lps._ptr(nub), lps._stream(None))
    ms_call = median_call_seconds(torch, stage, 10) * 1e3
    plan.close()
    log(f"data stage: {n_t} samples x 3 -> {fs.numel()} bins: one-off call {ms_once:.2f} ms; planned "
        f"{ms_call:.3f} ms per dataset (plan {ms_plan:.1f} ms once)")
    return {"samples": n_t, "channels": 3, "bins": int(fs.numel()), "ms": ms_call,
            "ms_per_dataset_planned": ms_call, "ms_plan_once": ms_plan, "ms_one_off_call": ms_once,
            "steps": "xyz->aet, hann window, hipFFT periodogram, band of single bins (planned: median of 10 "
                     "calls, no allocation); response interpolation in the one-off timing"}


if __name__ == "__main__":
    main()
