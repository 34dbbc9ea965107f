"""Plain FP64 CPU oracle of the data stage: periodograms of TDI time series,
their average over consecutive frequency segments, and the response-grid
interpolation.

TEST INFRASTRUCTURE.  Only the test suite imports this module; the product
path never does, and it shares no code with the HIP library.

What it computes:

* One-sided periodogram of a (windowed) time series x_n, n = 0 .. N-1, step dt:
      X_k = sum_n w_n x_n exp(-2 pi i k n / N),   k = 0 .. N/2,
      P_k = c_k dt |X_k|^2 / (N mean(w^2)),   c_k = 1 at k = 0 and k = N/2 (N even), else 2,
  at f_k = k / (N dt), so that E[P_k] is the one-sided PSD.  Reading D1: the
  paper generates its data in the frequency domain and only mentions windowing;
  this is the standard one-sided normalisation with a window-power correction.
* Optional XYZ -> AET combination of the time series (noise-orthogonal
  channels of Sec. "Time-delay Interferometry"):
      A = (Z - X) / sqrt 2,  E = (X - 2Y + Z) / sqrt 6,  T = (X + Y + Z) / sqrt 3.
* Averaged periodogram of Sec. "MCMC setup": segments of n consecutive,
  non-overlapping bins starting at bin k0; D_i = mean of P over the segment,
  nu_i = n, and (reading D2) the segment's frequency is the mean of its bin
  frequencies.
* Response interpolation of Sec. "Parametrized SGWB model": a response tabulated
  on a frequency grid is interpolated to the analysis frequencies.  Reading D3:
  linear in (log f, log R) between grid nodes where both node values are
  positive, linear in (log f, R) otherwise (the response vanishes at transfer
  zeros); frequencies outside the grid give NaN.
"""
import math

import numpy as np


def xyz_to_aet(x):
    x = np.asarray(x, dtype=np.float64)
    X, Y, Z = x
    return np.stack([(Z - X) / math.sqrt(2.0), (X - 2.0 * Y + Z) / math.sqrt(6.0), (X + Y + Z) / math.sqrt(3.0)])


def periodogram(x, dt, window=None):
    """x[n_ch][N] -> (f[N//2+1], P[n_ch][N//2+1])."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    w = np.ones(n) if window is None else np.asarray(window, dtype=np.float64)
    w2 = float(np.mean(w * w))
    X = np.fft.rfft(x * w, axis=-1)
    c = np.full(X.shape[-1], 2.0)
    c[0] = 1.0
    if n % 2 == 0:
        c[-1] = 1.0
    P = c * dt * (X.real ** 2 + X.imag ** 2) / (n * w2)
    f = np.arange(X.shape[-1]) / (n * dt)
    return f, P


def average_segments(f, P, k0, seg_len, n_seg):
    """Segments of seg_len bins from bin k0: (f_seg, D[n_ch][n_seg], nu)."""
    P = np.atleast_2d(np.asarray(P, dtype=np.float64))
    f = np.asarray(f, dtype=np.float64)
    assert k0 >= 0 and seg_len >= 1 and k0 + seg_len * n_seg <= f.size
    fs = np.empty(n_seg)
    D = np.empty((P.shape[0], n_seg))
    for i in range(n_seg):
        a, b = k0 + i * seg_len, k0 + (i + 1) * seg_len
        fs[i] = math.fsum(f[a:b].tolist()) / seg_len
        for c in range(P.shape[0]):
            D[c, i] = math.fsum(P[c, a:b].tolist()) / seg_len
    return fs, D, np.full(n_seg, float(seg_len))


def interp_response(grid_f, grid_R, f):
    """grid_f[n_g] increasing > 0, grid_R[n_ch][n_g] >= 0 -> R[n_ch][len(f)]."""
    gf = np.asarray(grid_f, dtype=np.float64)
    gR = np.atleast_2d(np.asarray(grid_R, dtype=np.float64))
    f = np.asarray(f, dtype=np.float64)
    lg = np.log(gf)
    out = np.full((gR.shape[0], f.size), np.nan)
    for q, fq in enumerate(f):
        if not (gf[0] <= fq <= gf[-1]):
            continue
        j = int(np.searchsorted(gf, fq, side="right")) - 1
        j = min(j, gf.size - 2)
        t = (math.log(fq) - lg[j]) / (lg[j + 1] - lg[j])
        for c in range(gR.shape[0]):
            r0, r1 = gR[c, j], gR[c, j + 1]
            if r0 > 0.0 and r1 > 0.0:
                out[c, q] = math.exp(math.log(r0) + t * (math.log(r1) - math.log(r0)))
            else:
                out[c, q] = r0 + t * (r1 - r0)
    return out
