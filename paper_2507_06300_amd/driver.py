"""Two-step inference (Sec. "Two-step inference").

Step 1 samples the template parameters alone: every spline is disabled, which
is the model with all spline heights zero (P = 0), and the sweeps make no
birth/death moves.  Step 2 fixes the template parameters of every chain at the
medians of the step-1 posterior (the draws of the b = 1 rung) and lets the
splines explore: each spline starts from its two edge knots at zero height and
the sweeps add and remove in-between knots.  All numerical work runs in the
library's kernels; this module only arranges the two runs.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import Context, Sampler, States, column_median


@dataclass
class TwoStepResult:
    medians: np.ndarray                 # [P] template parameters fixed in step 2
    step1_draws: np.ndarray             # [n_draws, P] b = 1 draws of step 1
    step1_logL: np.ndarray              # [n_draws] their log-likelihoods
    sampler: Sampler                    # the step-2 sampler (after its sweeps)
    logL_records: Optional[torch.Tensor] = None   # [n_rec, T, W] step-2 logL records
    notes: List[str] = field(default_factory=list)


def _band(ctx: Context):
    f = ctx.f.detach().cpu().numpy()
    return float(np.log10(f[0])), float(np.log10(f[-1]))


def _cold_rung(betas):
    return int(np.argmax(np.asarray(betas)))


def templates_only_states(ctx: Context, params: np.ndarray) -> States:
    """Chains with the given template parameters [P][C] and every spline disabled."""
    C = params.shape[1]
    off = np.zeros(C * ctx.n_spl + 1, dtype=np.int32)
    unused = np.zeros(1)            # no knot is read: every count is zero
    return ctx.states(params, off, unused, unused)


def edge_states(ctx: Context, params: np.ndarray) -> States:
    """Chains whose splines hold only their two edge knots at zero height."""
    C = params.shape[1]
    x_lo, x_hi = _band(ctx)
    n = C * ctx.n_spl
    off = (2 * np.arange(n + 1)).astype(np.int32)
    kx = np.tile([x_lo, x_hi], n)
    ky = np.zeros(2 * n)
    return ctx.states(params, off, kx, ky)


def two_step(ctx: Context, n_walkers: int, betas, init_params: np.ndarray, k_in_max: int,
             burn1: int, keep1: int, burn2: int, keep2: int, seed: int = 1, step: float = 0.05,
             precision: str = "mixed", record_every: int = 1) -> TwoStepResult:
    """Run both steps; init_params[P][n_walkers * n_temps] start the step-1 chains.
    Step-2 logL records (one per `record_every` sweeps of `keep2`) are returned
    for the evidence and DIC reductions."""
    betas = np.asarray(betas, dtype=np.float64)
    T = betas.size
    C = n_walkers * T
    P = init_params.shape[0]
    cold = _cold_rung(betas)
    # step 1: templates only
    sm1 = Sampler(ctx, n_walkers, betas, seed=seed, k_in_max=0, step=step, precision=precision, rj_moves=False)
    sm1.set_state(templates_only_states(ctx, np.ascontiguousarray(init_params, dtype=np.float64)))
    sm1.sweep(burn1)
    # the b = 1 rung's draws stay on the device ([P][keep1 * W] and [keep1 * W])
    lo, hi = cold * n_walkers, (cold + 1) * n_walkers
    rec_p = torch.empty((P, keep1 * n_walkers), dtype=torch.float64, device=ctx.device)
    rec_l = torch.empty(keep1 * n_walkers, dtype=torch.float64, device=ctx.device)
    for i in range(keep1):
        sm1.sweep(1)
        s = sm1.get_state(sweep_index=False)
        rec_p[:, i * n_walkers:(i + 1) * n_walkers] = s["params"][:, lo:hi]
        rec_l[i * n_walkers:(i + 1) * n_walkers] = s["logL"][lo:hi]
    sm1.close()
    # medians by the library's column-median kernel; one host read at the end
    medians = column_median(rec_p).cpu().numpy() if keep1 > 0 else np.full(P, np.nan)
    draws = rec_p.cpu().numpy().T
    lls = rec_l.cpu().numpy()
    # step 2: template parameters fixed at the medians, splines free
    sm2 = Sampler(ctx, n_walkers, betas, seed=seed + 1, k_in_max=k_in_max, step=step, precision=precision,
                  fixed_params=range(P), rj_moves=True)
    sm2.set_state(edge_states(ctx, np.repeat(medians[:, None], C, axis=1)))
    sm2.sweep(burn2)
    n_rec = keep2 // record_every
    rec = torch.empty((n_rec, T, n_walkers), dtype=torch.float64, device=ctx.device)
    for i in range(n_rec):
        sm2.sweep(record_every)
        sm2.record_logL(rec[i].view(-1))
    return TwoStepResult(medians=medians, step1_draws=draws, step1_logL=lls, sampler=sm2, logL_records=rec)
