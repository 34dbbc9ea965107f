"""Plain FP64 CPU oracle of the model-selection reductions over tempered chains.

TEST INFRASTRUCTURE.  Only the test suite imports this module; the product
path never does, and it shares no code with the HIP library.

What it computes:

* The stepping-stone estimate of the evidence, Eq. (ss) of Sec. "MCMC setup":
  for an increasing inverse-temperature ladder b_0 < b_1 < ... < b_{T-1} and n
  draws theta_i from the chain at each b_{k-1},

      log Z = sum_{k=1}^{T-1} log( (1/n) sum_i L(theta_i at b_{k-1})^(b_k - b_{k-1}) ).

  Reading E1: the paper writes the sum over the K ladder rungs with draws at
  b_{k-1}; its lowest rung is b = 1e-20, which stands in for the prior, so the
  ratios run over consecutive rungs of the given ladder (a caller that runs a
  b = 0 chain gets the exact telescoping product from the prior).
  Reading E2: the +-uncertainty the paper quotes is taken as the delta-method
  variance of each ratio estimate for independent draws,
  Var(log r_k) = (mean(w^2) / mean(w)^2 - 1) / n with w_i = L_i^(b_k - b_{k-1}),
  summed over the steps.

* The deviance information criterion of Sec. "Results": deviance
  D(theta) = -2 log L(theta) (the additive constant dropped), its posterior
  mean over b = 1 draws, p_D = mean(D) - D(theta_bar) with D(theta_bar) the
  deviance at the posterior-mean parameters (computed by the caller), and
  DIC = mean(D) + p_D.  The variance of D is reported as well (half of it is
  the alternative effective-parameter count of Gelman et al.).

Every sum is math.fsum in float64; exponentials are taken relative to the
maximum so that no term overflows.
"""
import math

import numpy as np


def _log_mean_exp(a):
    """log((1/n) sum_i exp(a_i)) with the maximum factored out."""
    a = np.asarray(a, dtype=np.float64)
    m = float(np.max(a))
    if not math.isfinite(m):
        return m
    return m + math.log(math.fsum(np.exp(a - m).tolist())) - math.log(a.size)


def stepping_stone(betas, logL):
    """Eq. (ss).  betas[T] strictly increasing; logL[T][n] = log-likelihoods of
    the n draws of each rung.  Returns (log Z, Var(log Z), per-step log ratios)."""
    betas = np.asarray(betas, dtype=np.float64)
    logL = np.asarray(logL, dtype=np.float64)
    T, n = logL.shape
    assert betas.shape == (T,) and T >= 2 and n >= 1
    assert np.all(np.diff(betas) > 0)
    steps, var = [], []
    for k in range(1, T):
        a = (betas[k] - betas[k - 1]) * logL[k - 1]
        steps.append(_log_mean_exp(a))
        m = float(np.max(a))
        w = np.exp(a - m)
        s1 = math.fsum(w.tolist())
        s2 = math.fsum((w * w).tolist())
        var.append((n * s2 / (s1 * s1) - 1.0) / n)
    return math.fsum(steps), math.fsum(var), np.array(steps)


def dic(logL, logL_at_mean):
    """DIC from the log-likelihoods of b = 1 draws and the log-likelihood at the
    posterior-mean parameters.  Returns (mean D, p_D, DIC, Var D)."""
    logL = np.asarray(logL, dtype=np.float64)
    n = logL.size
    d = -2.0 * logL
    mean_d = math.fsum(d.tolist()) / n
    var_d = math.fsum(((d - mean_d) ** 2).tolist()) / n
    p_d = mean_d - (-2.0 * logL_at_mean)
    return mean_d, p_d, mean_d + p_d, var_d


def paper_ladder():
    """The 20-rung ladder of Sec. "MCMC setup": 5 inverse temperatures
    logarithmically spaced on [1e-20, 1e-12], 10 on [1e-12, 1e-5] and 5 on
    [1e-5, 1].  Reading E3: the printed intervals share their end points; each
    group keeps its lower end and the last group includes b = 1, giving 20
    distinct rungs in increasing order."""
    a = np.logspace(-20, -12, 5, endpoint=False)
    b = np.logspace(-12, -5, 10, endpoint=False)
    c = np.logspace(-5, 0, 5, endpoint=True)
    return np.concatenate([a, b, c])
