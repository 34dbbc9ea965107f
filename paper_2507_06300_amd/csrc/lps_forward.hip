// Batched forward pass: logL for every state in one launch.
//
// Work item = (state tile, wave chunk of 64*B consecutive bins).  A wave
// keeps its B bins' table rows in registers for the whole tile and loops over
// the tile's states, so the shared per-bin data are read from memory once per
// tile, not once per state.  For each (state, exponent group) the piece
// holding the chunk is found by a wave-parallel search: lane j compares the
// chunk's first and last abscissae with breakpoint j+1 and two ballots give
// the first and last piece indices.  When they agree (the usual case: a chunk
// spans far less than a knot spacing) the cubic's coefficients are
// wave-uniform scalar loads; otherwise each lane walks the few breakpoints
// inside the chunk.  Each bin then evaluates
//   E_g = exp2(Q_g(x)),  S_c = sum of template rows times E_g  (Eq. (splines)),
//   l   = sum_c N_k (D~_ck / S~_ck + ln S~_ck)
// in scaled units, accumulates l in double per lane, and the wave writes one
// double partial per (state, chunk).  A second kernel adds the partials of a
// state in a fixed order and the scaling constant C0:
//   logL = C0 - sum_chunks partial.
#include <math.h>

#include "lps_internal.hpp"

namespace lps {
namespace {

template <typename R>
struct Math;

template <>
struct Math<float> {
  __device__ static inline float exp2_(float v) { return __builtin_amdgcn_exp2f(v); }
  __device__ static inline float log2_(float v) { return __builtin_amdgcn_logf(v); }
  __device__ static inline float rcp_(float v) { return __builtin_amdgcn_rcpf(v); }
};

template <>
struct Math<double> {
  __device__ static inline double exp2_(double v) { return exp2(v); }
  __device__ static inline double log2_(double v) { return log2(v); }
  __device__ static inline double rcp_(double v) { return 1.0 / v; }
};

template <int MODE>
struct Groups {
  static constexpr int G = MODE == kSplit ? 3 : (MODE == kShared ? 2 : 4);
};

// S~_c for one bin from the group factors E and the template rows.
template <typename R, int MODE, int NCH, bool FG, int B>
__device__ inline R assemble(int c, int b, const R (&Kt)[FG ? 4 : 3][NCH][B], const R (&E)[Groups<MODE>::G][B],
                             R w_oms, R w_tm, R e_fg) {
  R S;
  if constexpr (MODE == kSplit) {
    S = Kt[0][c][b] * E[0][b] + Kt[1][c][b] * E[1][b] + Kt[2][c][b] * E[2][b];
  } else if constexpr (MODE == kShared) {
    S = (w_oms * Kt[0][c][b] + w_tm * Kt[1][c][b]) * E[0][b] + Kt[2][c][b] * E[1][b];
  } else {
    S = (w_oms * Kt[0][c][b] + w_tm * Kt[1][c][b]) * E[c][b] + Kt[2][c][b] * E[3][b];
  }
  if constexpr (FG) S += Kt[3][c][b] * e_fg;
  return S;
}

template <typename R, int MODE, int NCH, bool FG, int B>
__global__ __launch_bounds__(256) void k_forward(int n_states, int n_chunks, int n_tiles, int tile, int K,
                                                 int k_pad, const R* __restrict__ tab,
                                                 const double* __restrict__ x64, const double* __restrict__ bx,
                                                 const R* __restrict__ coef, const int32_t* __restrict__ n_int,
                                                 const StateScalars* __restrict__ scal,
                                                 double* __restrict__ partial) {
  constexpr int G = Groups<MODE>::G;
  constexpr int NT = FG ? 4 : 3;
  constexpr int CH = kWave * B;
  constexpr bool kMixed = sizeof(R) == 4;
  const int lane = threadIdx.x & (kWave - 1);
  const int item = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int chunk = item % n_chunks;
  const int t = item / n_chunks;
  if (t >= n_tiles) return;
  const int s_begin = t * tile;
  const int s_end = min(s_begin + tile, n_states);
  const int kbase = chunk * CH;

  // per-bin rows for this lane's B bins (lane-strided, coalesced)
  R xr[B], NL[B];
  R Kt[NT][NCH][B];
  R ND[NCH][B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int k = kbase + b * kWave + lane;
    xr[b] = tab[k];
#pragma unroll
    for (int term = 0; term < NT; ++term)
#pragma unroll
      for (int c = 0; c < NCH; ++c) Kt[term][c][b] = tab[(size_t)tab_k(term, c, NCH) * k_pad + k];
#pragma unroll
    for (int c = 0; c < NCH; ++c) ND[c][b] = tab[(size_t)tab_nd(c, NT, NCH) * k_pad + k];
    NL[b] = tab[(size_t)tab_nl(NT, NCH) * k_pad + k];
  }
  const int klast = min(kbase + CH, K) - 1;
  const double xf = x64[kbase];
  const double xl = x64[klast];

  for (int s = s_begin; s < s_end; ++s) {
    if (n_int[s * G] == 0) {   // invalid state: reported by the finaliser
      if (lane == 0) partial[(size_t)s * n_chunks + chunk] = 0.0;
      continue;
    }
    R E[G][B];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const size_t base = (size_t)(s * G + g) * kMaxKnots;
      const int ni = n_int[s * G + g];
      const double bl = (lane + 1 < ni) ? bx[base + lane + 1] : INFINITY;
      const int i0 = __popcll(__ballot(bl <= xf));
      const int i1 = __popcll(__ballot(bl <= xl));
      if (i0 == i1) {
        const R* cf = coef + (base + i0) * 4;
        const R a = cf[0], bb = cf[1], c = cf[2], d = cf[3];
        const double b0 = bx[base + i0];
        const R off = kMixed ? (R)(xf - b0) : (R)(-b0);
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const R tt = xr[b] + off;
          E[g][b] = Math<R>::exp2_(a + tt * (bb + tt * (c + tt * d)));
        }
      } else {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const int k = min(kbase + b * kWave + lane, K - 1);
          const double xk = x64[k];
          int idx = i0;
          for (int j = i0 + 1; j <= i1; ++j) idx += (bx[base + j] <= xk) ? 1 : 0;
          const R* cf = coef + (base + idx) * 4;
          const R tt = kMixed ? (R)(xk - bx[base + idx]) : (R)(xr[b] - bx[base + idx]);
          E[g][b] = Math<R>::exp2_(cf[0] + tt * (cf[1] + tt * (cf[2] + tt * cf[3])));
        }
      }
    }
    const StateScalars sc = scal[s];
    const R w_oms = (R)sc.w_oms, w_tm = (R)sc.w_tm, e_fg = (R)sc.e_fg;
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      R v = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const R S = assemble<R, MODE, NCH, FG, B>(c, b, Kt, E, w_oms, w_tm, e_fg);
        const R lw = (NCH == 2 && c == 0) ? (R)2 : (R)1;   // A and E merged: ln S counted twice
        v += ND[c][b] * Math<R>::rcp_(S) + (NL[b] * lw) * Math<R>::log2_(S);
      }
      acc += (double)v;
    }
    acc = wave_sum(acc);
    if (lane == 0) partial[(size_t)s * n_chunks + chunk] = acc;
  }
}

// logL = C0 - sum over chunks (fixed order), -inf for invalid states.
__global__ __launch_bounds__(256) void k_finalize(int n_states, int n_chunks, const double* __restrict__ partial,
                                                  const double* __restrict__ c0,
                                                  const uint32_t* __restrict__ status_ws, double* __restrict__ logL,
                                                  uint32_t* __restrict__ status) {
  const int lane = threadIdx.x & (kWave - 1);
  const int s = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (s >= n_states) return;
  double acc = 0.0;
  for (int c = lane; c < n_chunks; c += kWave) acc += partial[(size_t)s * n_chunks + c];
  acc = wave_sum(acc);
  if (lane == 0) {
    uint32_t st = status_ws[s];
    double v = c0[0] - acc;
    if (st == 0 && !isfinite(v)) st |= LPS_ST_PSD;
    logL[s] = st ? -INFINITY : v;
    if (status) status[s] = st;
  }
}

template <typename R, int B>
hipError_t dispatch(lps_ctx* ctx, int n, int n_chunks, int n_tiles, int tile, const R* tab, const R* coef,
                    hipStream_t s) {
  const Layout& L = ctx->lay;
  const int items = n_chunks * n_tiles;
  dim3 grid((items + kWavesPerBlock - 1) / kWavesPerBlock), block(kWave * kWavesPerBlock);
  const int k_pad = sizeof(R) == 4 ? ctx->k_pad32 : ctx->k_pad64;
#define LPS_FWD(MODE, NCH, FG)                                                                            \
  hipLaunchKernelGGL((k_forward<R, MODE, NCH, FG, B>), grid, block, 0, s, n, n_chunks, n_tiles, tile,   \
                     ctx->n_bins, k_pad, tab, ctx->x, ctx->bx, coef, ctx->n_int, ctx->scal, ctx->partial)
  const bool fg = L.has_fg != 0;
  if (L.mode == kSplit && L.nch == 2 && !fg) LPS_FWD(kSplit, 2, false);
  else if (L.mode == kSplit && L.nch == 2 && fg) LPS_FWD(kSplit, 2, true);
  else if (L.mode == kSplit && L.nch == 3 && !fg) LPS_FWD(kSplit, 3, false);
  else if (L.mode == kSplit && L.nch == 3 && fg) LPS_FWD(kSplit, 3, true);
  else if (L.mode == kShared && L.nch == 2 && !fg) LPS_FWD(kShared, 2, false);
  else if (L.mode == kShared && L.nch == 2 && fg) LPS_FWD(kShared, 2, true);
  else if (L.mode == kShared && L.nch == 3 && !fg) LPS_FWD(kShared, 3, false);
  else if (L.mode == kShared && L.nch == 3 && fg) LPS_FWD(kShared, 3, true);
  else if (L.mode == kPaper && !fg) LPS_FWD(kPaper, 3, false);
  else LPS_FWD(kPaper, 3, true);
#undef LPS_FWD
  return hipGetLastError();
}

}  // namespace

// States per tile: enough work items to fill the chip, at most 64 states.
static int pick_tile(int n_states, int n_chunks) {
  const long target_items = 8192;   // ~32 waves per CU
  long tile = ((long)n_states * n_chunks) / target_items;
  if (tile < 1) tile = 1;
  if (tile > 64) tile = 64;
  if (tile > n_states) tile = n_states;
  return (int)tile;
}

hipError_t launch_forward(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL, uint32_t* status,
                          hipStream_t s) {
  const int n = st->n_states;
  hipError_t e = launch_coeffs(ctx, st, s);
  if (e != hipSuccess) return e;
  const bool mixed = prec == LPS_MIXED;
  const int n_chunks = mixed ? ctx->n_chunks32 : ctx->n_chunks64;
  const int tile = pick_tile(n, n_chunks);
  const int n_tiles = (n + tile - 1) / tile;
  timing_begin(ctx, s);
  if (mixed)
    e = dispatch<float, kB32>(ctx, n, n_chunks, n_tiles, tile, ctx->tab32, ctx->coef32, s);
  else
    e = dispatch<double, kB64>(ctx, n, n_chunks, n_tiles, tile, ctx->tab64, ctx->coef64, s);
  if (e != hipSuccess) return e;
  timing_end(ctx, s);
  hipLaunchKernelGGL(k_finalize, dim3((n + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kWave * kWavesPerBlock), 0,
                     s, n, n_chunks, ctx->partial, ctx->c0, ctx->status_ws, logL, status);
  return hipGetLastError();
}

}  // namespace lps
