"""Plain FP64 CPU oracle of the flexible-PSD Whittle log-likelihood.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg import this module; the product path never does.
It shares no code with the HIP library: everything is evaluated from f_k
directly in float64, with numpy vectorised over bins and plain Python loops
over knots.

What it computes (the paper's Secs. "Parametrized noise model",
"Parametrized SGWB model", "Power spectral density breakdown", Eqs. (splines),
the averaged-periodogram likelihood, and App. A for the Akima spline):

  S_c(f_k | theta) = sum over terms tau of  template_tau,c(f_k) * 10**P_{route[tau][c]}(x_k)
  logL(theta)      = - sum_c sum_k N_k (D_ck / S_ck + ln S_ck)

with x_k = log10 f_k.  Readings of passages that are ambiguous or garbled,
each with its reason:

  R1  TDI prefactor of Eq. (noise_tdi): sin^2(xi) * sin^2(2 xi), xi = 2 pi f L / c.
      (Printed as sin^2 * sin^4; the X2 delay polynomial of Sec. "Time-delay
      Interferometry" gives |(1-z^2)(1-z^4)|^2 = 16 sin^2 xi sin^2 2xi.)
  R2  Degenerate Akima weight (w_i + w_{i-2} = 0): s_i = (m_{i-1} + m_i) / 2.
  R3  Right boundary slope: the mirror image of the left one,
      s_{n-2} = (w_{n-3} m_{n-3} + w_{n-4} m_{n-2}) / (w_{n-3} + w_{n-4}) (0-based).
  R4  The degenerate-weight test is an exact comparison with zero.
  R5  The spline abscissa is x = log10 f and the perturbation is 10**P.
  R6  A spline stores its total knot count n (edges included): n = 0 disables
      it (P = 0), n in {2, 3} is the linear interpolant, n >= 4 is Akima,
      n = 1 is invalid.
  R7  Likelihood normalisation: E[D] = S, logL = -sum N (D/S + ln S); the
      1/2 of C_AET and all theta-independent constants are dropped.
  R8  f_knee = 1e-3 Hz; H0/h = 100 km/s/Mpc = 1e5 / 3.0856775814913673e22 Hz.
  R9  A bin with x_k = x_i lies in interval i ([x_i, x_{i+1})); a bin at the
      last edge uses the last interval.  The knots must cover every bin (the
      edge test allows 1e-9 dex so that edges placed at log10 of the first or
      last bin pass whatever rounding log10 had).
  R10 d|z|/dz at z = 0 is taken as 0 in the gradient.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0                       # m/s (not printed in the paper)
H0_PER_H = 1.0e5 / 3.0856775814913673e22    # Hz, reading R8
LN10 = math.log(10.0)

# Per-state status bits (the library's documented status word).
ST_COUNT = 1        # knot count of 1, above the capacity, or inconsistent offsets
ST_ORDER = 2        # knot abscissae not strictly increasing
ST_COVER = 4        # edge knots do not enclose every bin
ST_NONFINITE = 8    # non-finite parameter or knot value
ST_AMPLITUDE = 16   # A_oms <= 0 or A_tm <= 0
ST_PSD = 32         # the total PSD is not finite and positive at some bin
COVER_SLACK = 1e-9  # dex; tolerance of the edge-enclosure test

TERM_OMS, TERM_TM, TERM_SGWB, TERM_FG = 0, 1, 2, 3


# --------------------------------------------------------------------------
# Noise and signal templates (Secs. "Parametrized noise model" and
# "Parametrized SGWB model")
# --------------------------------------------------------------------------

def s_oms(f, A_oms):
    """OMS single-link PSD, Eq. (readout): A^2 [1 + (2 mHz / f)^4] (2 pi f / c)^2."""
    return A_oms ** 2 * (1.0 + (2.0e-3 / f) ** 4) * (2.0 * math.pi * f / C_LIGHT) ** 2


def s_tm(f, A_tm):
    """TM acceleration single-link PSD: A^2 [1 + (0.4 mHz/f)^2][1 + (f/8 mHz)^4] (2 pi f c)^-2."""
    return (A_tm ** 2 * (1.0 + (0.4e-3 / f) ** 2) * (1.0 + (f / 8.0e-3) ** 4)
            * (1.0 / (2.0 * math.pi * f * C_LIGHT)) ** 2)


def noise_tdi(f, arm_length, A_oms, A_tm):
    """A/E/T noise PSDs of Eq. (noise_tdi), split into OMS and TM parts.

    Returns (oms[3][K], tm[3][K]) with channels (A, E, T); A and E are equal
    and the off-diagonal PSDs are zero.  Prefactor per reading R1.
    """
    xi = 2.0 * math.pi * f * arm_length / C_LIGHT
    pref = np.sin(xi) ** 2 * np.sin(2.0 * xi) ** 2
    cx = np.cos(xi)
    # 1 - cos(xi) written as 2 sin^2(xi/2): the same quantity without the
    # cancellation that costs 1 - cos(xi) five digits at 0.1 mHz
    omc = 2.0 * np.sin(0.5 * xi) ** 2
    so = s_oms(f, A_oms)
    st = s_tm(f, A_tm)
    ae_oms = 32.0 * pref * (2.0 + cx) * so
    ae_tm = 32.0 * pref * 4.0 * (1.0 + cx + cx ** 2) * st
    t_oms = 64.0 * pref * omc * so
    t_tm = 64.0 * pref * 2.0 * omc ** 2 * st
    return np.stack([ae_oms, ae_oms, t_oms]), np.stack([ae_tm, ae_tm, t_tm])


def sgwb_tdi(f, R, u, alpha, f_knee):
    """Signal PSD of Eq. (Sh) with the power law of Eq. (pl), A = 10**u, n = alpha.

    S_h,c = R_c(f) * h^2 Omega(f) * 3 (H0/h)^2 / (4 pi^2 f^3).
    """
    h2omega = 10.0 ** u * (f / f_knee) ** alpha
    return R * (h2omega * 3.0 * H0_PER_H ** 2 / (4.0 * math.pi ** 2 * f ** 3))[None, :]


def foreground_tdi(Rfg, u_fg):
    """Foreground term: an input shape table [3][K] times the amplitude 10**u_fg."""
    return Rfg * 10.0 ** u_fg


# --------------------------------------------------------------------------
# Akima spline (App. A) and the linear fallback (Sec. "Power spectral density
# breakdown": fewer than four knots use a linear interpolant)
# --------------------------------------------------------------------------

def akima_slopes(x, y):
    """Knot slopes s_i of App. A for n >= 4 knots (0-based, readings R2-R4)."""
    n = len(x)
    m = [(y[i + 1] - y[i]) / (x[i + 1] - x[i]) for i in range(n - 1)]
    w = [abs(m[i + 1] - m[i]) for i in range(n - 2)]
    s = [0.0] * n
    s[0] = (3.0 * m[0] - m[1]) / 2.0
    s[n - 1] = (3.0 * m[n - 2] - m[n - 3]) / 2.0

    def weighted(wr, ml, wl, mr):
        # Akima's weighted average of the two slopes adjacent to a knot.
        if wr + wl == 0.0:
            return (ml + mr) / 2.0
        return (wr * ml + wl * mr) / (wr + wl)

    s[1] = weighted(w[1], m[0], w[0], m[1])
    s[n - 2] = weighted(w[n - 3], m[n - 3], w[n - 4], m[n - 2])
    for i in range(2, n - 2):
        s[i] = weighted(w[i], m[i - 1], w[i - 2], m[i])
    return m, s


def spline_coeffs(x, y):
    """Per-interval cubic coefficients (a, b, c, d) in t = x - x_i (App. A).

    n >= 4: Akima; n in {2, 3}: linear interpolant (c = d = 0).
    """
    x = [float(v) for v in x]
    y = [float(v) for v in y]
    n = len(x)
    if n >= 4:
        m, s = akima_slopes(x, y)
        a, b, c, d = [], [], [], []
        for i in range(n - 1):
            h = x[i + 1] - x[i]
            a.append(y[i])
            b.append(s[i])
            c.append((3.0 * m[i] - 2.0 * s[i] - s[i + 1]) / h)
            d.append((s[i] + s[i + 1] - 2.0 * m[i]) / h ** 2)
        return np.array(a), np.array(b), np.array(c), np.array(d)
    if n in (2, 3):
        a = np.array(y[:-1])
        b = np.array([(y[i + 1] - y[i]) / (x[i + 1] - x[i]) for i in range(n - 1)])
        return a, b, np.zeros(n - 1), np.zeros(n - 1)
    raise ValueError("spline needs 0 or >= 2 knots")


def interval_index(x_knots, xq):
    """Interval i with x_i <= xq < x_{i+1}; the last edge maps to the last interval (R9)."""
    n = len(x_knots)
    i = np.searchsorted(np.asarray(x_knots[1:n - 1]), xq, side="right")
    return np.clip(i, 0, n - 2)


def spline_eval(x_knots, y_knots, xq):
    """P(xq) for one spline; n = 0 gives exactly 0 (R6)."""
    xq = np.asarray(xq, dtype=np.float64)
    if len(x_knots) == 0:
        return np.zeros_like(xq)
    a, b, c, d = spline_coeffs(x_knots, y_knots)
    i = interval_index(x_knots, xq)
    t = xq - np.asarray(x_knots, dtype=np.float64)[i]
    return a[i] + b[i] * t + c[i] * t ** 2 + d[i] * t ** 3


# --------------------------------------------------------------------------
# State validation
# --------------------------------------------------------------------------

def state_status(ds, params, knots, k_max=64):
    """Status bits for one state (0 = valid); see the ST_* constants."""
    st = 0
    if not all(math.isfinite(float(p)) for p in params):
        st |= ST_NONFINITE
    if not (params[0] > 0.0 and params[1] > 0.0):
        st |= ST_AMPLITUDE
    x_first = math.log10(float(ds.f[0]))
    x_last = math.log10(float(ds.f[-1]))
    for (kx, ky) in knots:
        n = len(kx)
        if n == 0:
            continue
        if n == 1 or n > k_max:
            st |= ST_COUNT
            continue
        if not (np.all(np.isfinite(kx)) and np.all(np.isfinite(ky))):
            st |= ST_NONFINITE
            continue
        if np.any(np.diff(kx) <= 0.0):
            st |= ST_ORDER
        # edges sit at the band extremes; 1e-9 dex absorbs libm rounding of log10
        if kx[0] > x_first + COVER_SLACK or kx[-1] < x_last - COVER_SLACK:
            st |= ST_COVER
    return st


# --------------------------------------------------------------------------
# PSD and likelihood (Eqs. (psd_tot), (splines); the averaged-periodogram
# Wishart likelihood summed over bins)
# --------------------------------------------------------------------------

def template_terms(ds, params):
    """Unperturbed terms [4][3][K] in the order OMS, TM, SGWB, FG (zeros if absent)."""
    f = ds.f
    K = f.size
    oms, tm = noise_tdi(f, ds.arm_length, params[0], params[1])
    sg = sgwb_tdi(f, ds.R, params[2], params[3], ds.f_knee)
    if getattr(ds, "Rfg", None) is not None:
        fg = foreground_tdi(ds.Rfg, params[4])
    else:
        fg = np.zeros((3, K))
    return np.stack([oms, tm, sg, fg])


def spline_values(ds, knots):
    """P_j(x_k) for every spline j, [n_spl][K]."""
    x = np.log10(ds.f)
    return np.stack([spline_eval(kx, ky, x) for (kx, ky) in knots])


def perturbed_terms(ds, params, knots):
    """Each template term times 10**P of the spline routed to it, [4][3][K]."""
    terms = template_terms(ds, params)
    P = spline_values(ds, knots)
    out = terms.copy()
    for tau in range(4):
        for c in range(3):
            j = ds.route[tau][c]
            if j >= 0:
                out[tau, c] = terms[tau, c] * 10.0 ** P[j]
    return out


def psd(ds, params, knots):
    """(S, S_noise, S_signal), each [3][K]: Eq. (psd_tot) with Eqs. (splines)."""
    pt = perturbed_terms(ds, params, knots)
    sn = pt[TERM_OMS] + pt[TERM_TM]
    sh = pt[TERM_SGWB] + pt[TERM_FG]
    return sn + sh, sn, sh


def loglike(ds, D, params, knots, k_max=64):
    """logL = -sum_c sum_k N_k (D_ck/S_ck + ln S_ck) (reading R7); -inf if invalid."""
    if state_status(ds, params, knots, k_max):
        return -math.inf
    S, _, _ = psd(ds, params, knots)
    if not (np.all(np.isfinite(S)) and np.all(S > 0.0)):
        return -math.inf
    terms = ds.nk[None, :] * (D / S + np.log(S))
    return -math.fsum(terms.ravel())


def loglike_delta(ds, D, params_a, knots_a, params_b, knots_b):
    """logL(b) - logL(a) summed term by term, without the large common constant."""
    Sa, _, _ = psd(ds, params_a, knots_a)
    Sb, _, _ = psd(ds, params_b, knots_b)
    terms = ds.nk[None, :] * ((D / Sb - D / Sa) + np.log(Sb / Sa))
    return -math.fsum(terms.ravel())


def snr(ds, params):
    """Eq. (snr) on the dataset's grid: sqrt(T_obs sum_c sum_k (S_h/S_n)^2 df_k)."""
    t = template_terms(ds, params)
    sn = t[TERM_OMS] + t[TERM_TM]
    sh = t[TERM_SGWB]
    df = np.gradient(ds.f)
    return math.sqrt(3.156e7 * math.fsum(((sh / sn) ** 2 * df[None, :]).ravel()))


# --------------------------------------------------------------------------
# Gradient: forward-mode tangents through App. A, then the chain rule
# --------------------------------------------------------------------------

class Dual:
    """A value with tangents with respect to a fixed parameter vector."""

    __slots__ = ("v", "d")

    def __init__(self, v, d):
        self.v = float(v)
        self.d = d

    @staticmethod
    def const(v, npar):
        return Dual(v, np.zeros(npar))

    def __add__(self, o):
        return Dual(self.v + o.v, self.d + o.d)

    def __sub__(self, o):
        return Dual(self.v - o.v, self.d - o.d)

    def __mul__(self, o):
        return Dual(self.v * o.v, self.d * o.v + self.v * o.d)

    def __truediv__(self, o):
        return Dual(self.v / o.v, (self.d * o.v - self.v * o.d) / (o.v * o.v))

    def scale(self, k):
        return Dual(self.v * k, self.d * k)


def _dabs(z):
    sgn = 1.0 if z.v > 0.0 else (-1.0 if z.v < 0.0 else 0.0)   # R10
    return Dual(abs(z.v), z.d * sgn)


def spline_tangents(x_knots, y_knots, xq):
    """P(xq) and dP(xq)/d(theta) for theta = (y_0..y_{n-1}, x_1..x_{n-2}).

    Returns (P [K], J [K][2n-2]) for n >= 2.  The edge abscissae are fixed.
    """
    n = len(x_knots)
    npar = n + (n - 2)
    X = []
    for i in range(n):
        d = np.zeros(npar)
        if 0 < i < n - 1:
            d[n + i - 1] = 1.0
        X.append(Dual(x_knots[i], d))
    Y = []
    for i in range(n):
        d = np.zeros(npar)
        d[i] = 1.0
        Y.append(Dual(y_knots[i], d))
    m = [(Y[i + 1] - Y[i]) / (X[i + 1] - X[i]) for i in range(n - 1)]
    if n >= 4:
        w = [_dabs(m[i + 1] - m[i]) for i in range(n - 2)]

        def weighted(wr, ml, wl, mr):
            if wr.v + wl.v == 0.0:
                return (ml + mr).scale(0.5)
            return (wr * ml + wl * mr) / (wr + wl)

        s = [None] * n
        s[0] = (m[0].scale(3.0) - m[1]).scale(0.5)
        s[n - 1] = (m[n - 2].scale(3.0) - m[n - 3]).scale(0.5)
        s[1] = weighted(w[1], m[0], w[0], m[1])
        s[n - 2] = weighted(w[n - 3], m[n - 3], w[n - 4], m[n - 2])
        for i in range(2, n - 2):
            s[i] = weighted(w[i], m[i - 1], w[i - 2], m[i])
        coef = []
        for i in range(n - 1):
            h = X[i + 1] - X[i]
            c = (m[i].scale(3.0) - s[i].scale(2.0) - s[i + 1]) / h
            dd = (s[i] + s[i + 1] - m[i].scale(2.0)) / (h * h)
            coef.append((Y[i], s[i], c, dd))
    else:
        zero = Dual.const(0.0, npar)
        coef = [(Y[i], m[i], zero, zero) for i in range(n - 1)]
    xq = np.asarray(xq, dtype=np.float64)
    idx = interval_index(x_knots, xq)
    P = np.empty(xq.size)
    J = np.empty((xq.size, npar))
    for i in range(n - 1):
        sel = np.nonzero(idx == i)[0]
        if sel.size == 0:
            continue
        a, b, c, d = coef[i]
        t = xq[sel] - X[i].v
        dt = -X[i].d                      # dt/dtheta (same for every bin)
        P[sel] = a.v + b.v * t + c.v * t ** 2 + d.v * t ** 3
        dPdt = b.v + 2.0 * c.v * t + 3.0 * d.v * t ** 2
        J[sel] = (a.d[None, :] + b.d[None, :] * t[:, None] + c.d[None, :] * (t ** 2)[:, None]
                  + d.d[None, :] * (t ** 3)[:, None] + dPdt[:, None] * dt[None, :])
    return P, J


def loglike_grad(ds, D, params, knots, k_max=64):
    """(logL, dlogL/dparams, [dlogL/dy per spline], [dlogL/dx per spline]).

    dlogL/dS_ck = N_k (D_ck - S_ck) / S_ck^2 (the score of the likelihood);
    template parameters by direct differentiation of the terms, spline
    parameters through the forward tangents of spline_tangents().
    Edge abscissae get 0.  Invalid states give (-inf, zeros).
    """
    npar = len(params)
    zy = [np.zeros(len(kx)) for (kx, _) in knots]
    zx = [np.zeros(len(kx)) for (kx, _) in knots]
    if state_status(ds, params, knots, k_max):
        return -math.inf, np.zeros(npar), zy, zx
    pt = perturbed_terms(ds, params, knots)
    S = pt.sum(axis=0)
    if not (np.all(np.isfinite(S)) and np.all(S > 0.0)):
        return -math.inf, np.zeros(npar), zy, zx
    nk = ds.nk[None, :]
    logL = -math.fsum((nk * (D / S + np.log(S))).ravel())
    g = nk * (D - S) / S ** 2
    lnf = np.log(ds.f / ds.f_knee)[None, :]
    dp = np.zeros(npar)
    dp[0] = math.fsum((g * 2.0 * pt[TERM_OMS] / params[0]).ravel())
    dp[1] = math.fsum((g * 2.0 * pt[TERM_TM] / params[1]).ravel())
    dp[2] = math.fsum((g * LN10 * pt[TERM_SGWB]).ravel())
    dp[3] = math.fsum((g * pt[TERM_SGWB] * lnf).ravel())
    if npar > 4:
        dp[4] = math.fsum((g * LN10 * pt[TERM_FG]).ravel())
    x = np.log10(ds.f)
    dys, dxs = [], []
    for j, (kx, ky) in enumerate(knots):
        n = len(kx)
        if n == 0:
            dys.append(np.zeros(0))
            dxs.append(np.zeros(0))
            continue
        # dlogL/dP_j(x_k) = sum over (term, channel) routed to j of g * ln10 * term
        gbar = np.zeros(ds.f.size)
        for tau in range(4):
            for c in range(3):
                if ds.route[tau][c] == j:
                    gbar = gbar + g[c] * LN10 * pt[tau, c]
        _, J = spline_tangents(kx, ky, x)
        tot = np.array([math.fsum(gbar * J[:, q]) for q in range(J.shape[1])])
        dy = tot[:n].copy()
        dx = np.zeros(n)
        dx[1:n - 1] = tot[n:]
        dys.append(dy)
        dxs.append(dx)
    return logL, dp, dys, dxs
