"""Seeded synthetic workloads with the shapes of the paper's analysis.

Every workload uses the paper's analysis band [1e-4, 2.9e-2] Hz and one year
of data (Sec. "Data generation"), the prior ranges of Table I, and the knot
layout of Sec. "Power spectral density breakdown" (two edge knots at the band
extremes whose heights are free, plus in-between knots with free position and
height).  The paper's own datasets are not available; these inputs stand in
for them.

Nothing here evaluates the noise model, the spline or the likelihood.  The
response table R_c(f) and the foreground shape are *inputs* of the method
(the paper reads R from an external code, Sec. "Parametrized SGWB model"); the
stand-ins below are documented recipes, not part of the method.

Random streams (numpy PCG64):
  data seed   = 1000 + workload index  -> truth state and the chi multipliers
  states seed = 2000 + workload index  -> the batch of walker states
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Band and observation settings (Sec. "Data generation").
F_BAND_LO = 1.0e-4
F_BAND_HI = 2.9e-2
T_OBS = 3.156e7          # one year in seconds
ARM_LENGTH = 2.5e9       # m (Sec. "Time-delay Interferometry")
F_KNEE = 1.0e-3          # Hz; the paper leaves the pivot frequency unstated

# Speed of light, used only by the response stand-in below.
_C_STANDIN = 299792458.0
# Normalisation of the response stand-in.  Written by
# tests/golden/calibrate_response.py (oracle only) so that the cosmic-string
# background of Eq. (cs) at the fiducial noise levels has SNR 262 on the
# one-year grid, the value the paper quotes for its injection.
RESPONSE_ZETA = 0.45243

TERMS = ("oms", "tm", "sgwb", "fg")
CHANNELS = ("A", "E", "T")

# route[term][channel] -> spline index or -1 (term not perturbed).
LAYOUTS = {
    # one noise spline shared by OMS and TM in all channels + one signal spline
    "noise_signal": dict(n_spl=2, route=[[0, 0, 0], [0, 0, 0], [1, 1, 1], [-1, -1, -1]], fg=False),
    # separate OMS, TM and signal splines, all channel independent
    "split": dict(n_spl=3, route=[[0, 0, 0], [1, 1, 1], [2, 2, 2], [-1, -1, -1]], fg=False),
    # as "split" plus a galactic-foreground-shaped term with no spline
    "split_fg": dict(n_spl=3, route=[[0, 0, 0], [1, 1, 1], [2, 2, 2], [-1, -1, -1]], fg=True),
    # the paper's layout: one noise spline per channel, one shared signal spline
    "paper": dict(n_spl=4, route=[[0, 1, 2], [0, 1, 2], [3, 3, 3], [-1, -1, -1]], fg=False),
}


@dataclass(frozen=True)
class Workload:
    name: str
    index: int
    grid: str                 # "log" | "df" | "linspace"
    n_bins: int
    nk: str                   # "const:<N>" | "ramp:<Nmax>"
    n_states: int
    layout: str
    inbetween: tuple          # (lo, hi) inclusive, in-between knots per spline
    df: float = 0.0
    k_first: int = 0
    note: str = ""


WORKLOADS = {
    w.name: w
    for w in [
        Workload("avg50_1000bins_64states", 1, "log", 1000, "const:50", 64,
                 "noise_signal", (4, 4),
                 note="segment-averaged, N_k=50, fixed 4 in-between knots"),
        Workload("daily_2497bins_320states", 2, "df", 2497, "const:365", 320,
                 "split", (2, 20), df=1.0 / 86400.0, k_first=9,
                 note="1/day bins over one year, N_k=365, 32 walkers x 10 temps"),
        Workload("year_912085bins_4096states", 3, "df", 912085, "const:1", 4096,
                 "split", (0, 30), df=1.0 / T_OBS, k_first=3156,
                 note="full one-year Whittle periodogram, 64 walkers x 16 temps x 4 branches"),
        Workload("grad_25000bins_1024states", 4, "log", 25000, "ramp:2000", 1024,
                 "split", (2, 20),
                 note="log bins, N_k rising 1..2000, gradient workload"),
        Workload("sweep_250000bins_2048chains", 5, "linspace", 250000, "const:4", 2048,
                 "split_fg", (0, 40),
                 note="sampler sweep: 128 walkers x 16 temps, 3 splines + foreground"),
    ]
}


@dataclass
class Dataset:
    """Per-bin inputs of one analysis (all float64, channel-major [3][K])."""
    f: np.ndarray
    nk: np.ndarray
    R: np.ndarray
    Rfg: Optional[np.ndarray]
    chi: np.ndarray                 # Gamma(N_k,1)/N_k draws; D = S(truth) * chi
    truth: "StateBatch"
    layout: str
    n_spl: int
    route: list
    f_knee: float = F_KNEE
    arm_length: float = ARM_LENGTH
    k_max: int = 64
    name: str = ""


@dataclass
class StateBatch:
    """Packed ragged states: params[P][n] and CSR knots per (state, spline)."""
    params: np.ndarray              # [P][n] : A_oms, A_tm, u, alpha[, u_fg]
    knot_off: np.ndarray            # int32 [n*n_spl + 1]
    knot_x: np.ndarray              # log10 f of each knot, edges included
    knot_y: np.ndarray              # heights
    n_spl: int

    @property
    def n(self) -> int:
        return int(self.params.shape[1])

    def knots(self, s: int, j: int):
        a = int(self.knot_off[s * self.n_spl + j])
        b = int(self.knot_off[s * self.n_spl + j + 1])
        return self.knot_x[a:b], self.knot_y[a:b]


def route_table(layout: str):
    return [list(r) for r in LAYOUTS[layout]["route"]]


def frequency_grid(w: Workload) -> np.ndarray:
    if w.grid == "log":
        k = np.arange(w.n_bins, dtype=np.float64)
        return F_BAND_LO * (F_BAND_HI / F_BAND_LO) ** (k / (w.n_bins - 1))
    if w.grid == "df":
        k = np.arange(w.k_first, w.k_first + w.n_bins, dtype=np.float64)
        return k * w.df
    if w.grid == "linspace":
        return np.linspace(F_BAND_LO, F_BAND_HI, w.n_bins)
    raise ValueError(w.grid)


def segment_counts(w: Workload) -> np.ndarray:
    kind, val = w.nk.split(":")
    if kind == "const":
        return np.full(w.n_bins, float(val))
    if kind == "ramp":
        k = np.arange(w.n_bins, dtype=np.float64)
        return np.round(float(val) ** (k / (w.n_bins - 1)))
    raise ValueError(w.nk)


def response_standin(f: np.ndarray, arm_length: float = ARM_LENGTH,
                     zeta: float = RESPONSE_ZETA) -> np.ndarray:
    """Stand-in for the sky-averaged A/E/T response R_c(f) (an input table).

    The paper computes R(f) with an external code that is not available; this
    smooth positive shape follows the second-generation TDI factor at low
    frequency and suppresses T as (1 - cos xi)^3.  Only its role as a per-bin
    input matters to the hot path.
    """
    xi = 2.0 * math.pi * f * arm_length / _C_STANDIN
    base = zeta * 32.0 * np.sin(xi) ** 2 * np.sin(2.0 * xi) ** 2 * xi ** 2 / (1.0 + 0.6 * xi ** 2)
    return np.stack([base, base, base * (1.0 - np.cos(xi)) ** 3])


def foreground_shape(f: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Stand-in galactic-foreground template times the response (input table).

    The paper names the galactic foreground but gives no shape; this is a
    log-normal bump of width 0.35 dex centred on 1 mHz.  Its amplitude
    10**u_fg (about 1e-38 / Hz) is a state parameter.
    """
    bump = np.exp(-np.log10(f / 1.0e-3) ** 2 / (2.0 * 0.35 ** 2))
    return R * bump[None, :]


def _draw_states(rng: np.random.Generator, n: int, n_spl: int, inbetween, x_lo: float,
                 x_hi: float, with_fg: bool) -> StateBatch:
    lo, hi = inbetween
    counts = rng.integers(lo, hi + 1, size=(n, n_spl)) + 2
    A_oms = rng.uniform(10.0, 20.0, n) * 1e-12
    A_tm = rng.uniform(2.0, 4.0, n) * 1e-15
    u = rng.uniform(-13.0, -11.0, n)
    alpha = rng.uniform(-1.0, 1.0, n)
    rows = [A_oms, A_tm, u, alpha]
    if with_fg:
        rows.append(rng.uniform(-38.5, -37.5, n))
    params = np.stack(rows)
    flat = counts.reshape(-1)
    off = np.zeros(flat.size + 1, dtype=np.int32)
    off[1:] = np.cumsum(flat)
    total = int(off[-1])
    kx = np.empty(total)
    ky = rng.normal(0.0, 0.1, total)
    for i, c in enumerate(flat):
        a = off[i]
        interior = np.sort(rng.uniform(x_lo, x_hi, int(c) - 2))
        kx[a] = x_lo
        kx[a + 1:a + c - 1] = interior
        kx[a + c - 1] = x_hi
    return StateBatch(params=params, knot_off=off, knot_x=kx, knot_y=ky, n_spl=n_spl)


def band_edges(f: np.ndarray):
    """Edge-knot abscissae: log10 of the first and last analysed bin."""
    return float(np.log10(f[0])), float(np.log10(f[-1]))


def make_dataset(name: str, n_bins: Optional[int] = None, layout: Optional[str] = None) -> Dataset:
    """Grid, segment counts, input tables, truth state and chi for a workload.

    n_bins / layout override the workload's own values for reduced-size
    variants used by the tests (same recipe, fewer bins).
    """
    w = WORKLOADS[name]
    if n_bins is not None and n_bins != w.n_bins:
        w = Workload(**{**w.__dict__, "n_bins": int(n_bins)})
    lay = layout or w.layout
    rng = np.random.Generator(np.random.PCG64(1000 + w.index))
    f = frequency_grid(w)
    nk = segment_counts(w)
    R = response_standin(f)
    Rfg = foreground_shape(f, R) if LAYOUTS[lay]["fg"] else None
    x_lo, x_hi = band_edges(f)
    n_spl = LAYOUTS[lay]["n_spl"]
    truth = _draw_states(rng, 1, n_spl, w.inbetween, x_lo, x_hi, Rfg is not None)
    chi = rng.gamma(shape=np.broadcast_to(nk, (3, nk.size)), scale=1.0) / nk[None, :]
    return Dataset(f=f, nk=nk, R=R, Rfg=Rfg, chi=chi, truth=truth, layout=lay, n_spl=n_spl,
                   route=route_table(lay), name=w.name)


def make_states(name: str, ds: Dataset, n_states: Optional[int] = None,
                inbetween=None, seed_offset: int = 0) -> StateBatch:
    w = WORKLOADS[name]
    rng = np.random.Generator(np.random.PCG64(2000 + w.index + 7919 * seed_offset))
    n = w.n_states if n_states is None else int(n_states)
    x_lo, x_hi = band_edges(ds.f)
    return _draw_states(rng, n, ds.n_spl, inbetween or w.inbetween, x_lo, x_hi, ds.Rfg is not None)


def states_subset(sb: StateBatch, idx) -> StateBatch:
    """Repack a subset of states (keeps CSR layout)."""
    idx = list(idx)
    xs, ys, counts = [], [], []
    for s in idx:
        for j in range(sb.n_spl):
            x, y = sb.knots(s, j)
            xs.append(x)
            ys.append(y)
            counts.append(len(x))
    off = np.zeros(len(counts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    return StateBatch(params=np.ascontiguousarray(sb.params[:, idx]), knot_off=off,
                      knot_x=np.concatenate(xs) if xs else np.zeros(0),
                      knot_y=np.concatenate(ys) if ys else np.zeros(0), n_spl=sb.n_spl)


def pack_states(params: np.ndarray, knots, n_spl: int) -> StateBatch:
    """Build a batch from explicit per-(state, spline) knot lists.

    knots[s][j] = (x array, y array); empty arrays disable the spline.
    """
    xs, ys, counts = [], [], []
    for s in range(params.shape[1]):
        for j in range(n_spl):
            x, y = knots[s][j]
            xs.append(np.asarray(x, dtype=np.float64))
            ys.append(np.asarray(y, dtype=np.float64))
            counts.append(len(xs[-1]))
    off = np.zeros(len(counts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    return StateBatch(params=np.ascontiguousarray(params, dtype=np.float64), knot_off=off,
                      knot_x=np.concatenate(xs) if xs else np.zeros(0),
                      knot_y=np.concatenate(ys) if ys else np.zeros(0), n_spl=n_spl)


def colored_series(rng: np.random.Generator, psd: np.ndarray, n_t: int, dt: float) -> np.ndarray:
    """Gaussian time series [n_ch][n_t] whose one-sided PSD is psd[n_ch][n_t//2+1]
    (given on the grid k / (n_t dt); the k = 0 and, for even n_t, Nyquist entries
    are ignored): Fourier coefficients with E|X_k|^2 = n_t psd_k / (2 dt) and
    uniform phases, transformed back."""
    psd = np.atleast_2d(np.asarray(psd, dtype=np.float64))
    nf = n_t // 2 + 1
    assert psd.shape[1] == nf
    amp = np.sqrt(n_t * psd / (2.0 * dt))
    X = amp * (rng.standard_normal(psd.shape) + 1j * rng.standard_normal(psd.shape)) / np.sqrt(2.0)
    X[:, 0] = 0.0
    if n_t % 2 == 0:
        X[:, -1] = 0.0
    return np.fft.irfft(X, n=n_t, axis=1)


def append_splines(sb: StateBatch, rng: np.random.Generator, n_new: int, inbetween, x_lo: float, x_hi: float,
                   height_sd: float = 0.5) -> StateBatch:
    """The same states with n_new more spline slots per state, drawn like the
    others (edge knots at the band extremes, in-between knots uniform in log10 f,
    heights normal with standard deviation height_sd)."""
    lo, hi = inbetween
    knots = []
    for s in range(sb.n):
        row = [sb.knots(s, j) for j in range(sb.n_spl)]
        for _ in range(n_new):
            c = int(rng.integers(lo, hi + 1)) + 2
            x = np.concatenate([[x_lo], np.sort(rng.uniform(x_lo, x_hi, c - 2)), [x_hi]])
            row.append((x, rng.normal(0.0, height_sd, c)))
        knots.append(row)
    return pack_states(sb.params, knots, sb.n_spl + n_new)


def complex_wishart_mean(rng: np.random.Generator, C: np.ndarray, nu: np.ndarray) -> np.ndarray:
    """W / nu with W ~ complex Wishart(nu, C): the average of nu outer products
    z z^H of independent circular complex Gaussian vectors with E[z z^H] = C.

    C is [K][p][p] real symmetric positive definite, nu [K] positive integers.
    Drawn by the Bartlett decomposition: W = L A A^H L^T with C = L L^T, A lower
    triangular, |A_ii|^2 ~ Gamma(nu - i, 1) and A_ij ~ CN(0, 1) below the
    diagonal.  Bins with nu < p (a singular Wishart) sum nu outer products of
    draws L g, g ~ CN(0, I), instead.  Returns the complex [K][p][p] matrices W / nu."""
    C = np.asarray(C, dtype=np.float64)
    K, p, _ = C.shape
    nu = np.asarray(nu, dtype=np.float64)
    L = np.linalg.cholesky(C)
    few = nu < p
    nu_b = np.where(few, float(p), nu)
    A = np.zeros((K, p, p), dtype=np.complex128)
    for i in range(p):
        A[:, i, i] = np.sqrt(rng.gamma(nu_b - i, 1.0))
        for j in range(i):
            A[:, i, j] = (rng.standard_normal(K) + 1j * rng.standard_normal(K)) / math.sqrt(2.0)
    LA = L @ A
    W = LA @ np.conj(np.transpose(LA, (0, 2, 1)))
    if np.any(few):
        idx = np.nonzero(few)[0]
        Wf = np.zeros((idx.size, p, p), dtype=np.complex128)
        for m in range(1, p):
            sel = nu[idx] >= m
            g = (rng.standard_normal((idx.size, p)) + 1j * rng.standard_normal((idx.size, p))) / math.sqrt(2.0)
            z = np.einsum("kab,kb->ka", L[idx], g)
            Wf += sel[:, None, None] * (z[:, :, None] * np.conj(z[:, None, :]))
        W[idx] = Wf
    return W / nu[:, None, None]
