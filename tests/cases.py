"""Shared test cases: seeded datasets and state batches, data formed by the oracle.

D = S_oracle(truth) * chi, so no input of the oracle (or of the GPU path in
the tests) comes from the HIP library.
"""
import math

import numpy as np

from oracle import lps_oracle as O
from synth import workloads as W


def knots_of(sb, s):
    return [sb.knots(s, j) for j in range(sb.n_spl)]


def dataset_with_data(name, n_bins=None, layout=None):
    ds = W.make_dataset(name, n_bins=n_bins, layout=layout)
    S0, _, _ = O.psd(ds, ds.truth.params[:, 0], knots_of(ds.truth, 0))
    D = S0 * ds.chi
    return ds, D


def oracle_loglikes(ds, D, sb, idx=None):
    idx = range(sb.n) if idx is None else idx
    return np.array([O.loglike(ds, D, sb.params[:, s], knots_of(sb, s)) for s in idx])


def oracle_status(ds, sb, idx=None, k_max=64):
    idx = range(sb.n) if idx is None else idx
    return np.array([O.state_status(ds, sb.params[:, s], knots_of(sb, s), k_max) for s in idx])


def make_context(lps, ds, D, max_states, k_max=64, max_grad_states=None):
    return lps.Context(ds.f, ds.nk, D, ds.R, ds.route, ds.n_spl, Rfg=ds.Rfg, k_max=k_max,
                       max_states=max_states, f_knee=ds.f_knee, arm_length=ds.arm_length,
                       max_grad_states=max_grad_states)


def device_states(ctx, sb):
    return ctx.states(sb.params, sb.knot_off, sb.knot_x, sb.knot_y)


def mixed_tolerance(ds, D, sb, idx):
    """Derived bound for the mixed path.

    Each per-bin term N_k (D/S + ln S~) is formed from single-precision
    operations whose combined relative error is a few tens of units of
    2^-24; with eps = 2^-24 and a budget of 32 eps per term, the bound is
    32 eps * sum_ck N_k (D_ck/S_ck + |ln S_ck / sigma| + 1) where the log of the
    scaled PSD is bounded by 8 over the prior box.
    """
    eps = 2.0 ** -24
    out = []
    for s in idx:
        S, _, _ = O.psd(ds, sb.params[:, s], knots_of(sb, s))
        out.append(32 * eps * math.fsum((ds.nk[None, :] * (D / S + 9.0)).ravel()))
    return np.array(out)
