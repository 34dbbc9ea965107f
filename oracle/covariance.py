"""Plain FP64 CPU oracle of the full-covariance (dense 3x3) log-likelihood.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg import this module; the product path never does.

The paper keeps the A/E/T noise covariance diagonal and names the dense
treatment as the natural extension (Sec. "Power spectral density breakdown",
the paragraph on independent channel splines, and the outlook of the
conclusions): three more flexible terms for the off-diagonal entries, six
flexible functions in all, combined so that the covariance stays Hermitian
positive definite.  It does not print the construction.  Reading X1 (listed
with its reasons in the design notes) fixes one:

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


def loglike(cds, P6, params, knots, k_max=64):
    """- sum_k N_k (tr(C_k^-1 P_k) + ln det C_k); -inf for an invalid state."""
    if state_status(cds, params, knots, k_max):
        return -math.inf
    C, _, _ = covariance(cds, params, knots)
    P = data_matrix(P6)
    X = np.linalg.solve(C, P)                     # C^-1 P per bin
    tr = X[:, 0, 0] + X[:, 1, 1] + X[:, 2, 2]
    sign, logdet = np.linalg.slogdet(C)
    assert np.all(sign > 0)
    return -math.fsum((cds.nk * (tr + logdet)).tolist())
