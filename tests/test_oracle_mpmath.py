"""Brute-force pin of the oracle at 50 significant digits (mpmath).

A second, independent evaluation of the method on a few states and bins,
written from the paper's formulas with arbitrary-precision arithmetic:

* templates: the single-link OMS and TM PSDs of Sec. "Parametrized noise
  model", the A/E/T transfer of Eq. (noise_tdi) (prefactor read as
  sin^2(xi) sin^2(2 xi)), the background of Eqs. (pl) and (Sh), the
  foreground as an input table times 10^u_fg;
* the spline of App. A, here in Hermite form (values and Akima knot slopes
  at both ends of each interval) instead of the oracle's power-basis
  coefficients, with the linear interpolant for two or three knots;
* logL = -sum_c sum_k N_k (D_ck / S_ck + ln S_ck), summed exactly;
* the gradient by central differences at 50 digits (step 1e-20), so
  truncation and rounding are both far below double precision.

The FP64 oracle must agree to 1e-13 relative on logL and the PSD, and to
1e-10 of the largest component per family on the gradient.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import lps_oracle as O
from synth import workloads as W

mp.mp.dps = 50
C = mp.mpf(299792458)
H0 = mp.mpf(10) ** 5 / mp.mpf("3.0856775814913673e22")


def _mp_shapes(f, A_oms, A_tm):
    so = A_oms ** 2 * (1 + (mp.mpf("2e-3") / f) ** 4) * (2 * mp.pi * f / C) ** 2
    st = (A_tm ** 2 * (1 + (mp.mpf("0.4e-3") / f) ** 2) * (1 + (f / mp.mpf("8e-3")) ** 4)
          / (2 * mp.pi * f * C) ** 2)
    return so, st


def _mp_noise(f, L, A_oms, A_tm):
    xi = 2 * mp.pi * f * L / C
    pre = mp.sin(xi) ** 2 * mp.sin(2 * xi) ** 2
    cx = mp.cos(xi)
    so, st = _mp_shapes(f, A_oms, A_tm)
    ae_o = 32 * pre * (2 + cx) * so
    ae_t = 32 * pre * 4 * (1 + cx + cx ** 2) * st
    t_o = 64 * pre * (1 - cx) * so
    t_t = 64 * pre * 2 * (1 - cx) ** 2 * st
    return [ae_o, ae_o, t_o], [ae_t, ae_t, t_t]


def _mp_slopes(x, y):
    n = len(x)
    m = [(y[i + 1] - y[i]) / (x[i + 1] - x[i]) for i in range(n - 1)]
    if n < 4:
        return m, None
    s = [None] * n
    s[0] = (3 * m[0] - m[1]) / 2
    s[n - 1] = (3 * m[n - 2] - m[n - 3]) / 2
    for i in range(1, n - 1):
        # slopes of the two neighbouring intervals on each side of knot i
        ml, mr = m[i - 1], m[i]
        if i == 1:
            wl, wr = abs(m[1] - m[0]), abs(m[2] - m[1])
        elif i == n - 2:
            wl, wr = abs(m[n - 3] - m[n - 4]), abs(m[n - 2] - m[n - 3])
        else:
            wl, wr = abs(m[i - 1] - m[i - 2]), abs(m[i + 1] - m[i])
        s[i] = (ml + mr) / 2 if wl + wr == 0 else (wr * ml + wl * mr) / (wr + wl)
    return m, s


def _mp_spline(x, y, xq):
    n = len(x)
    if n == 0:
        return mp.mpf(0)
    # interval [x_i, x_{i+1}) holding xq, the last edge in the last interval
    i = 0
    while i + 1 < n - 1 and x[i + 1] <= xq:
        i += 1
    m, s = _mp_slopes(x, y)
    h = x[i + 1] - x[i]
    t = (xq - x[i]) / h
    if s is None:
        return y[i] + m[i] * (xq - x[i])
    h00 = 2 * t ** 3 - 3 * t ** 2 + 1
    h10 = t ** 3 - 2 * t ** 2 + t
    h01 = -2 * t ** 3 + 3 * t ** 2
    h11 = t ** 3 - t ** 2
    return h00 * y[i] + h10 * h * s[i] + h01 * y[i + 1] + h11 * h * s[i + 1]


def _mp_psd(ds, params, knots):
    """S[c][k] as mpf, from f_k, the route table and the knots."""
    A_oms, A_tm, u, alpha = (mp.mpf(float(v)) for v in params[:4])
    out = [[None] * ds.f.size for _ in range(3)]
    for k, fk in enumerate(ds.f):
        f = mp.mpf(float(fk))
        xq = mp.log10(f)
        P = [_mp_spline([mp.mpf(float(v)) for v in kx], [mp.mpf(float(v)) for v in ky], xq) for (kx, ky) in knots]
        oms, tm = _mp_noise(f, mp.mpf(float(ds.arm_length)), A_oms, A_tm)
        h2o = mp.mpf(10) ** u * (f / mp.mpf(float(ds.f_knee))) ** alpha
        for c in range(3):
            sg = mp.mpf(float(ds.R[c, k])) * h2o * 3 * H0 ** 2 / (4 * mp.pi ** 2 * f ** 3)
            terms = [oms[c], tm[c], sg, mp.mpf(0)]
            if ds.Rfg is not None:
                terms[3] = mp.mpf(float(ds.Rfg[c, k])) * mp.mpf(10) ** mp.mpf(float(params[4]))
            tot = mp.mpf(0)
            for tau in range(4):
                j = ds.route[tau][c]
                tot += terms[tau] * (mp.mpf(10) ** P[j] if j >= 0 else 1)
            out[c][k] = tot
    return out


def _mp_loglike(ds, D, params, knots):
    S = _mp_psd(ds, params, knots)
    return -mp.fsum(mp.mpf(float(ds.nk[k])) * (mp.mpf(float(D[c, k])) / S[c][k] + mp.log(S[c][k]))
                    for c in range(3) for k in range(ds.f.size))


def _case(layout, n_bins=8, n_states=3, seed=0):
    name = "sweep_250000bins_2048chains" if layout == "split_fg" else "grad_25000bins_1024states"
    ds = W.make_dataset(name, n_bins=n_bins, layout=layout)
    sb = W.make_states(name, ds, n_states=n_states, inbetween=(0, 4), seed_offset=seed)
    truth = [ds.truth.knots(0, j) for j in range(ds.n_spl)]
    S0, _, _ = O.psd(ds, ds.truth.params[:, 0], truth)
    D = S0 * ds.chi
    return ds, sb, D


@pytest.mark.parametrize("layout", ["split", "paper", "noise_signal", "split_fg"])
def test_oracle_loglike_and_psd_at_50_digits(layout):
    ds, sb, D = _case(layout)
    for s in range(sb.n):
        kn = [sb.knots(s, j) for j in range(sb.n_spl)]
        S, _, _ = O.psd(ds, sb.params[:, s], kn)
        Sm = _mp_psd(ds, sb.params[:, s], kn)
        for c in range(3):
            for k in range(ds.f.size):
                assert abs(mp.mpf(float(S[c, k])) / Sm[c][k] - 1) < mp.mpf("1e-13"), (s, c, k)
        ref = _mp_loglike(ds, D, sb.params[:, s], kn)
        got = O.loglike(ds, D, sb.params[:, s], kn)
        assert abs(mp.mpf(got) - ref) <= mp.mpf("1e-13") * abs(ref), (s, got, ref)


def _flat(params, knots):
    """Parameter vector (template params, then per spline heights and interior positions)."""
    v = [float(p) for p in params]
    for (kx, ky) in knots:
        v += [float(t) for t in ky] + [float(t) for t in kx[1:-1]]
    return v


def _unflat(v, npar, counts, edges):
    params = v[:npar]
    knots, p = [], npar
    for n, (xl, xr) in zip(counts, edges):
        y = v[p:p + n]
        p += n
        xi = v[p:p + max(n - 2, 0)]
        p += max(n - 2, 0)
        x = [xl] + list(xi) + [xr] if n else []
        knots.append((x, y))
    return params, knots


def _mp_loglike_v(ds, D, v, npar, counts, edges):
    params, knots = _unflat(v, npar, counts, edges)
    A_oms, A_tm, u, alpha = params[:4]
    terms_all = []
    for k, fk in enumerate(ds.f):
        f = mp.mpf(float(fk))
        xq = mp.log10(f)
        P = [_mp_spline(kx, ky, xq) for (kx, ky) in knots]
        oms, tm = _mp_noise(f, mp.mpf(float(ds.arm_length)), A_oms, A_tm)
        h2o = mp.mpf(10) ** u * (f / mp.mpf(float(ds.f_knee))) ** alpha
        for c in range(3):
            sg = mp.mpf(float(ds.R[c, k])) * h2o * 3 * H0 ** 2 / (4 * mp.pi ** 2 * f ** 3)
            terms = [oms[c], tm[c], sg, mp.mpf(0)]
            tot = mp.mpf(0)
            for tau in range(4):
                j = ds.route[tau][c]
                tot += terms[tau] * (mp.mpf(10) ** P[j] if j >= 0 else 1)
            terms_all.append(mp.mpf(float(ds.nk[k])) * (mp.mpf(float(D[c, k])) / tot + mp.log(tot)))
    return -mp.fsum(terms_all)


@pytest.mark.parametrize("layout", ["split", "paper"])
def test_oracle_gradient_at_50_digits(layout):
    ds, sb, D = _case(layout, n_bins=8, n_states=2, seed=3)
    for s in range(sb.n):
        kn = [sb.knots(s, j) for j in range(sb.n_spl)]
        _, dp, dys, dxs = O.loglike_grad(ds, D, sb.params[:, s], kn)
        counts = [len(kx) for (kx, _) in kn]
        edges = [(mp.mpf(float(kx[0])), mp.mpf(float(kx[-1]))) if len(kx) else (None, None) for (kx, _) in kn]
        v0 = [mp.mpf(t) for t in _flat(sb.params[:4, s], kn)]
        npar = 4
        h = mp.mpf("1e-20")
        grad = []
        for q in range(len(v0)):
            scale = abs(v0[q]) if q < 2 else mp.mpf(1)
            vp = list(v0)
            vm = list(v0)
            vp[q] += h * scale
            vm[q] -= h * scale
            grad.append((_mp_loglike_v(ds, D, vp, npar, counts, edges)
                         - _mp_loglike_v(ds, D, vm, npar, counts, edges)) / (2 * h * scale))
        # oracle vector in the same order
        ref = list(dp[:4])
        for (dy, dx, n) in zip(dys, dxs, counts):
            ref += list(dy) + list(dx[1:n - 1])
        fam = [("params", 0, 4)]
        p = 4
        for n in counts:
            fam.append(("y", p, p + n))
            fam.append(("x", p + n, p + n + max(n - 2, 0)))
            p += n + max(n - 2, 0)
        for nm, a, b in fam:
            if b <= a:
                continue
            if nm == "params":
                # amplitudes are per unit relative step; compare dlogL/dlnA
                for q in range(a, b):
                    w = v0[q] if q < 2 else 1
                    big = max(abs(grad[i] * (v0[i] if i < 2 else 1)) for i in range(a, b))
                    assert abs(mp.mpf(float(ref[q])) - grad[q]) * abs(w) <= mp.mpf("1e-10") * big, (s, q)
            else:
                big = max(abs(grad[i]) for i in range(a, b))
                for q in range(a, b):
                    assert abs(mp.mpf(float(ref[q])) - grad[q]) <= mp.mpf("1e-10") * big + mp.mpf("1e-30"), \
                        (s, nm, q, float(ref[q]), float(grad[q]))
