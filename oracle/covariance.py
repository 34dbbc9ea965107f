"""Plain FP64 CPU oracle of the full-covariance (dense 3x3) log-likelihood.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg import this module; the product path never does.

The paper keeps the A/E/T noise covariance diagonal and names the dense
treatment as the natural extension (Sec. "Power spectral density breakdown",
the paragraph on independent channel splines, and the outlook of the
conclusions): three more flexible terms for the off-diagonal entries, six
flexible functions in all, combined so that the covariance stays Hermitian
positive definite.  It does not print the construction.  Reading X1 fixes
one:

  frame        A/E/T.  The likelihood below is unchanged under any orthonormal
               change of channel basis applied to both the model and the data,
               so the Michelson X/Y/Z form is the same function written in
               another basis.
  noise        N = Dn^1/2 Rn Dn^1/2.  Dn = diag(S_n,A, S_n,E, S_n,T) is the
               diagonal noise model of the rest of the library (OMS and TM
               templates, each perturbed by its routed spline).  Rn is a
               correlation matrix built from three more splines Q_0, Q_1, Q_2
               (abscissa log10 f, like every spline here) as a partial-
               correlation vine on the ordering A, E, T:
                   r_AE = tanh Q_0,   r_AT = tanh Q_1,   rho_ET|A = tanh Q_2,
                   r_ET = r_AE r_AT + rho_ET|A sqrt((1 - r_AE^2)(1 - r_AT^2)).
               Any real Q_0..Q_2 give a positive-definite Rn, and Q = 0 (a
               disabled spline) gives zero correlation.
  signal       diag(S_h,A, S_h,E, S_h,T): the isotropic background and the
               foreground term of the diagonal model, unchanged.
  data         the real symmetric part of the averaged cross-periodogram,
               six rows per bin in the order AA, EE, TT, AE, AT, ET, with
               E[P] = C (the one-sided normalisation of the diagonal model).
  likelihood   logL = - sum_k N_k ( tr(C_k^-1 P_k) + ln det C_k ), the
               complex-Wishart log-density of the averaged periodogram up to
               theta-independent constants.  With zero correlations it is the
               diagonal expression of the rest of the library term by term.
               (C is real, so the imaginary part of the cross-periodogram
               drops out of the trace.)
  validity     the state checks of the diagonal model, and C_k positive
               definite at every bin (Sylvester's criterion on the correlation
               form of C_k); otherwise logL = -inf and the PSD status bit.
  gradient     loglike_grad(): the matrix-calculus derivative written out in
               forward mode (see its docstring), pinned by finite differences.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import lps_oracle as O

# Order of the six data rows and of the six unique model entries.
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


@dataclass
class CovDataset:
    """A diagonal-model dataset (f, nk, R, Rfg, route, ...) plus the
    correlation routing: corr[i] = spline slot of Q_i or -1 (Q_i = 0)."""
    base: object
    corr: tuple
    n_spl: int

    def __getattr__(self, name):
        return getattr(self.base, name)


def vine_correlations(q0, q1, q2):
    """(r_AE, r_AT, r_ET) from the three correlation splines (reading X1)."""
    r01 = np.tanh(q0)
    r02 = np.tanh(q1)
    p12 = np.tanh(q2)
    r12 = r01 * r02 + p12 * np.sqrt((1.0 - r01 * r01) * (1.0 - r02 * r02))
    return r01, r02, r12


def correlation_splines(cds, knots):
    """Q_0..Q_2 at every bin, [3][K] (zero for a slot of -1 or a disabled spline)."""
    x = np.log10(cds.f)
    out = np.zeros((3, x.size))
    for i, j in enumerate(cds.corr):
        if j >= 0:
            kx, ky = knots[j]
            out[i] = O.spline_eval(kx, ky, x)
    return out


def covariance(cds, params, knots):
    """C_k for every bin, [K][3][3], with the noise and signal parts (Sn, Sh)."""
    pt = O.perturbed_terms(cds, params, knots)
    sn = pt[O.TERM_OMS] + pt[O.TERM_TM]          # [3][K]
    sh = pt[O.TERM_SGWB] + pt[O.TERM_FG]
    q = correlation_splines(cds, knots)
    r01, r02, r12 = vine_correlations(q[0], q[1], q[2])
    K = sn.shape[1]
    Rn = np.zeros((K, 3, 3))
    Rn[:, 0, 0] = Rn[:, 1, 1] = Rn[:, 2, 2] = 1.0
    Rn[:, 0, 1] = Rn[:, 1, 0] = r01
    Rn[:, 0, 2] = Rn[:, 2, 0] = r02
    Rn[:, 1, 2] = Rn[:, 2, 1] = r12
    half = np.sqrt(sn.T)                          # [K][3]
    N = half[:, :, None] * Rn * half[:, None, :]
    C = N.copy()
    for c in range(3):
        C[:, c, c] = sn[c] + sh[c]
    return C, sn, sh


def unique_entries(C):
    """The six unique entries of [K][3][3] matrices as rows [6][K] (PAIRS order)."""
    return np.stack([C[:, a, b] for (a, b) in PAIRS])


def data_matrix(P6):
    """Rows [6][K] (PAIRS order) as symmetric [K][3][3] matrices."""
    K = P6.shape[1]
    M = np.zeros((K, 3, 3))
    for i, (a, b) in enumerate(PAIRS):
        M[:, a, b] = P6[i]
        M[:, b, a] = P6[i]
    return M


def positive_definite(C):
    """Per bin: Sylvester's criterion on the correlation form of C."""
    d = np.stack([C[:, c, c] for c in range(3)], axis=1)
    ok = np.all(np.isfinite(C.reshape(C.shape[0], -1)), axis=1) & np.all(d > 0.0, axis=1)
    s = np.sqrt(np.where(d > 0.0, d, 1.0))
    Ct = C / (s[:, :, None] * s[:, None, :])
    m1 = 1.0 - Ct[:, 0, 1] ** 2
    m2 = np.linalg.det(Ct)
    return ok & (m1 > 0.0) & (m2 > 0.0)


def state_status(cds, params, knots, k_max=64):
    """Status bits: the diagonal model's checks over every spline slot, then ST_PSD."""
    st = O.state_status(cds, params, knots, k_max)
    if st:
        return st
    C, _, _ = covariance(cds, params, knots)
    if not np.all(positive_definite(C)):
        st |= O.ST_PSD
    return st


def loglike_terms(cds, P6, params, knots):
    """Per-bin terms N_k (tr(C_k^-1 P_k) + ln det C_k), [K], of a valid state."""
    C, _, _ = covariance(cds, params, knots)
    P = data_matrix(P6)
    X = np.linalg.solve(C, P)                     # C^-1 P per bin
    tr = X[:, 0, 0] + X[:, 1, 1] + X[:, 2, 2]
    sign, logdet = np.linalg.slogdet(C)
    assert np.all(sign > 0)
    return cds.nk * (tr + logdet)


def loglike(cds, P6, params, knots, k_max=64):
    """- sum_k N_k (tr(C_k^-1 P_k) + ln det C_k); -inf for an invalid state."""
    if state_status(cds, params, knots, k_max):
        return -math.inf
    return -math.fsum(loglike_terms(cds, P6, params, knots).tolist())


def _covariance_tangent(sn, dsn, dsh, q, dq):
    """dC [K][3][3] from tangents of Sn, Sh [3][K] and of Q_0..Q_2 [3][K],
    by forward differentiation of the construction of covariance()."""
    r01, r02, r12 = vine_correlations(q[0], q[1], q[2])
    p12 = np.tanh(q[2])
    dr01 = (1.0 - r01 * r01) * dq[0]
    dr02 = (1.0 - r02 * r02) * dq[1]
    dp12 = (1.0 - p12 * p12) * dq[2]
    S = np.sqrt((1.0 - r01 * r01) * (1.0 - r02 * r02))
    # S = 0 only where a correlation is exactly +-1: S is then 0 for every
    # value of the other one, and its tangent is 0
    num = r01 * dr01 * (1.0 - r02 * r02) + r02 * dr02 * (1.0 - r01 * r01)
    dS = np.where(S > 0.0, -num / np.where(S > 0.0, S, 1.0), 0.0)
    dr12 = dr01 * r02 + r01 * dr02 + dp12 * S + p12 * dS
    r = {(0, 1): (r01, dr01), (0, 2): (r02, dr02), (1, 2): (r12, dr12)}
    K = sn.shape[1]
    dC = np.zeros((K, 3, 3))
    for c in range(3):
        dC[:, c, c] = dsn[c] + dsh[c]
    for (a, b), (rv, drv) in r.items():
        hs = np.sqrt(sn[a] * sn[b])
        dhs = (dsn[a] * sn[b] + sn[a] * dsn[b]) / (2.0 * hs)
        dC[:, a, b] = dC[:, b, a] = drv * hs + rv * dhs
    return dC


def loglike_grad(cds, P6, params, knots, k_max=64):
    """(logL, dlogL/dparams, [dlogL/dy per spline], [dlogL/dx per spline]).

    Along a change dC of the covariance, tr(C^-1 P) + ln det C changes by
    tr(G dC) with G = C^-1 - C^-1 P C^-1 (matrix calculus: d C^-1 =
    -C^-1 dC C^-1, d ln det C = tr(C^-1 dC)), so
        dlogL/dtheta = - sum_k N_k tr(G_k dC_k/dtheta).
    dC/dtheta by forward differentiation of covariance(): the template
    parameters act on Sn and Sh as in the diagonal model, a spline value
    P_j(x_k) through every term routed to it (factor ln 10 10^P_j) or through
    its correlation Q_i; knots through the spline tangents of App. A.
    Edge abscissae get 0.  Invalid states give (-inf, zeros)."""
    npar = len(params)
    zy = [np.zeros(len(kx)) for (kx, _) in knots]
    zx = [np.zeros(len(kx)) for (kx, _) in knots]
    if state_status(cds, params, knots, k_max):
        return -math.inf, np.zeros(npar), zy, zx
    logL = loglike(cds, P6, params, knots, k_max)
    pt = O.perturbed_terms(cds, params, knots)
    sn = pt[O.TERM_OMS] + pt[O.TERM_TM]
    q = correlation_splines(cds, knots)
    C, _, _ = covariance(cds, params, knots)
    Ci = np.linalg.inv(C)
    G = Ci - Ci @ data_matrix(P6) @ Ci
    nu = cds.nk
    K = nu.size
    z3 = np.zeros((3, K))

    def per_bin(dsn, dsh, dq):
        dC = _covariance_tangent(sn, dsn, dsh, q, dq)
        return -nu * np.einsum("kab,kba->k", G, dC)

    lnf = np.log(cds.f / cds.f_knee)[None, :]
    dp = np.zeros(npar)
    dp[0] = math.fsum(per_bin(2.0 * pt[O.TERM_OMS] / params[0], z3, z3).tolist())
    dp[1] = math.fsum(per_bin(2.0 * pt[O.TERM_TM] / params[1], z3, z3).tolist())
    dp[2] = math.fsum(per_bin(z3, O.LN10 * pt[O.TERM_SGWB], z3).tolist())
    dp[3] = math.fsum(per_bin(z3, lnf * pt[O.TERM_SGWB], z3).tolist())
    if npar > 4:
        dp[4] = math.fsum(per_bin(z3, O.LN10 * pt[O.TERM_FG], z3).tolist())
    x = np.log10(cds.f)
    dys, dxs = [], []
    for j, (kx, ky) in enumerate(knots):
        n = len(kx)
        if n == 0:
            dys.append(np.zeros(0))
            dxs.append(np.zeros(0))
            continue
        # dlogL/dP_j(x_k): every diagonal term routed to slot j, and the
        # correlation spline(s) it carries
        dsn, dsh, dq = np.zeros((3, K)), np.zeros((3, K)), np.zeros((3, K))
        for tau in range(4):
            for c in range(3):
                if cds.route[tau][c] == j:
                    tgt = dsn if tau in (O.TERM_OMS, O.TERM_TM) else dsh
                    tgt[c] += O.LN10 * pt[tau, c]
        for i in range(3):
            if cds.corr[i] == j:
                dq[i] = 1.0
        gbar = per_bin(dsn, dsh, dq)
        _, J = O.spline_tangents(kx, ky, x)
        tot = np.array([math.fsum(gbar * J[:, m]) for m in range(J.shape[1])])
        dy = tot[:n].copy()
        dx = np.zeros(n)
        dx[1:n - 1] = tot[n:]
        dys.append(dy)
        dxs.append(dx)
    return logL, dp, dys, dxs
