// Per-state validation shared by every entry point.
//
// A state is valid when its parameters are finite, A_OMS > 0 and A_TM > 0,
// and every spline slot holds 0 knots (disabled) or 2..k_max knots whose
// abscissae are finite, strictly increasing and enclose the analysed band
// (edge knots at the band extremes, Sec. "Power spectral density breakdown").
// The enclosure test allows 1e-9 dex of slack so that an edge knot placed at
// log10 of the first or last bin frequency passes whatever libm rounded.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lps.h"

namespace lps {

constexpr double kCoverSlack = 1e-9;

// Knot range of spline slot i (= state * n_spl + spline): packed CSR when cnt is
// NULL (count = off[i+1] - off[i]), padded CSR otherwise (count = cnt[i]).
// Returns false, with a = n = 0 so that nothing is read, when the range is not
// inside the knot arrays [0, n_knots).
__host__ __device__ inline bool knot_range(const int32_t* __restrict__ off, const int32_t* __restrict__ cnt, int i,
                                           int64_t n_knots, int& a, int& n) {
  a = off[i];
  n = cnt ? cnt[i] : off[i + 1] - a;
  if (a < 0 || n < 0 || (int64_t)a + n > n_knots) {
    a = 0;
    n = 0;
    return false;
  }
  return true;
}

__host__ __device__ inline uint32_t validate_state(int s, int n_states, int n_spl, int k_max, int n_params,
                                                   const double* __restrict__ params, const int32_t* __restrict__ off,
                                                   const int32_t* __restrict__ kcnt, int64_t n_knots,
                                                   const double* __restrict__ kx, const double* __restrict__ ky,
                                                   double x_first, double x_last) {
  uint32_t st = 0;
  for (int p = 0; p < n_params; ++p)
    if (!__builtin_isfinite(params[p * (size_t)n_states + s])) st |= LPS_ST_NONFINITE;
  const double a_oms = params[LPS_P_AOMS * (size_t)n_states + s];
  const double a_tm = params[LPS_P_ATM * (size_t)n_states + s];
  if (!(a_oms > 0.0 && a_tm > 0.0)) st |= LPS_ST_AMPLITUDE;
  for (int j = 0; j < n_spl; ++j) {
    int a, cnt;
    if (!knot_range(off, kcnt, s * n_spl + j, n_knots, a, cnt)) {
      st |= LPS_ST_COUNT;
      continue;
    }
    if (cnt == 0) continue;
    if (cnt == 1 || cnt > k_max) {
      st |= LPS_ST_COUNT;
      continue;
    }
    bool fin = true;
    for (int i = 0; i < cnt; ++i) fin = fin && __builtin_isfinite(kx[a + i]) && __builtin_isfinite(ky[a + i]);
    if (!fin) {
      st |= LPS_ST_NONFINITE;
      continue;
    }
    for (int i = 0; i + 1 < cnt; ++i)
      if (!(kx[a + i + 1] > kx[a + i])) st |= LPS_ST_ORDER;
    if (kx[a] > x_first + kCoverSlack || kx[a + cnt - 1] < x_last - kCoverSlack) st |= LPS_ST_COVER;
  }
  return st;
}

}  // namespace lps

namespace lps {

__device__ inline uint32_t wave_or(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v |= (uint32_t)__shfl_xor((int)v, o, 64);
  return v;
}

// The same checks as validate_state, made by one wave with a lane per knot
// (k_max <= 64).  Every lane of the wave must call it with the same state;
// every lane receives the state's status bits.
__device__ inline uint32_t validate_state_wave(int lane, int s, int n_states, int n_spl, int k_max, int n_params,
                                               const double* __restrict__ params, const int32_t* __restrict__ off,
                                               const int32_t* __restrict__ kcnt, int64_t n_knots,
                                               const double* __restrict__ kx, const double* __restrict__ ky,
                                               double x_first, double x_last) {
  uint32_t st = 0;
  if (lane < n_params && !isfinite(params[lane * (size_t)n_states + s])) st |= LPS_ST_NONFINITE;
  if (lane == 0) {
    const double a_oms = params[LPS_P_AOMS * (size_t)n_states + s];
    const double a_tm = params[LPS_P_ATM * (size_t)n_states + s];
    if (!(a_oms > 0.0 && a_tm > 0.0)) st |= LPS_ST_AMPLITUDE;
  }
  for (int j = 0; j < n_spl; ++j) {
    int a, cnt;
    if (!knot_range(off, kcnt, s * n_spl + j, n_knots, a, cnt)) {
      if (lane == 0) st |= LPS_ST_COUNT;
      continue;
    }
    if (cnt == 0) continue;
    if (cnt == 1 || cnt > k_max) {
      if (lane == 0) st |= LPS_ST_COUNT;
      continue;
    }
    const bool mine = lane < cnt;
    const double xi = mine ? kx[a + lane] : 0.0;
    const bool bad = mine && !(isfinite(xi) && isfinite(ky[a + lane]));
    if (__ballot(bad) != 0ull) {
      if (lane == 0) st |= LPS_ST_NONFINITE;
      continue;
    }
    if (lane + 1 < cnt && !(kx[a + lane + 1] > xi)) st |= LPS_ST_ORDER;
    if (lane == 0 && (xi > x_first + kCoverSlack || kx[a + cnt - 1] < x_last - kCoverSlack)) st |= LPS_ST_COVER;
  }
  return wave_or(st);
}

}  // namespace lps
