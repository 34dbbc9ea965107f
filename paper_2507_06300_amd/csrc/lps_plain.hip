// Plain FP64 reference path: one launch per state, one thread per bin.
//
// Every thread evaluates its bin from f_k alone: xi = 2 pi f L / c, the
// A/E/T transfer of Eq. (noise_tdi) with sin/cos, the single-link OMS and TM
// PSDs, the power law of Eq. (pl) with pow(), the response input R, each
// routed spline by a binary search over the state's knots and the local
// Akima stencil of App. A, 10^P with exp10(), and
//   l_k = sum_c N_k (D_ck / S_ck + ln S_ck).
// A block reduction writes one partial per block; a second one-block kernel
// sums the partials in order and validates the state.  Nothing is shared
// between states and no per-bin table is used: this is the baseline the
// batched kernels are measured against.
#include <math.h>

#include "lps_internal.hpp"
#include "lps_spline.hpp"
#include "lps_validate.hpp"

namespace lps {
namespace {

struct Route {
  int8_t r[4][3];
};

__device__ inline double spline_value(const double* __restrict__ x, const double* __restrict__ y, int n,
                                      int k_max, double xk) {
  if (n < 2 || n > k_max) return 0.0;
  // interval = number of interior knots <= xk
  int lo = 0, hi = n - 2;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (x[mid] <= xk) lo = mid;
    else hi = mid - 1;
  }
  double a, b, c, d;
  spline_piece(x, y, n, lo, a, b, c, d);
  double t = xk - x[lo];
  return a + b * t + c * t * t + d * t * t * t;
}

__global__ __launch_bounds__(kPlainBlock) void k_plain_bins(
    int K, const double* __restrict__ f, const double* __restrict__ nk, const double* __restrict__ D,
    const double* __restrict__ R, const double* __restrict__ Rfg, double L, double f_knee, int n_spl, int k_max,
    Route route, int n_states, int n_params, int s, const double* __restrict__ params,
    const int32_t* __restrict__ off, const int32_t* __restrict__ kcnt, const double* __restrict__ kx,
    const double* __restrict__ ky, double* __restrict__ part) {
  __shared__ double red[kPlainBlock];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (k < K) {
    const double fk = f[k];
    const double xk = log10(fk);
    const double a_oms = params[LPS_P_AOMS * (size_t)n_states + s];
    const double a_tm = params[LPS_P_ATM * (size_t)n_states + s];
    const double u = params[LPS_P_U * (size_t)n_states + s];
    const double alpha = params[LPS_P_ALPHA * (size_t)n_states + s];
    const double xi = 2.0 * kPi * fk * L / kClight;
    const double sx = sin(xi), cx = cos(xi), s2x = sin(2.0 * xi);
    const double pref = sx * sx * s2x * s2x;
    const double sh = sin(0.5 * xi);
    const double omc = 2.0 * sh * sh;   // 1 - cos xi without cancellation
    const double s_oms = a_oms * a_oms * (1.0 + pow(2.0e-3 / fk, 4.0)) * pow(2.0 * kPi * fk / kClight, 2.0);
    const double s_tm = a_tm * a_tm * (1.0 + pow(0.4e-3 / fk, 2.0)) * (1.0 + pow(fk / 8.0e-3, 4.0)) *
                        pow(2.0 * kPi * fk * kClight, -2.0);
    const double oms[3] = {32.0 * pref * (2.0 + cx) * s_oms, 32.0 * pref * (2.0 + cx) * s_oms,
                           64.0 * pref * omc * s_oms};
    const double tm[3] = {32.0 * pref * 4.0 * (1.0 + cx + cx * cx) * s_tm,
                          32.0 * pref * 4.0 * (1.0 + cx + cx * cx) * s_tm,
                          64.0 * pref * 2.0 * omc * omc * s_tm};
    const double h2omega = exp10(u) * pow(fk / f_knee, alpha);
    const double hfac = h2omega * 3.0 * kH0PerH * kH0PerH / (4.0 * kPi * kPi * fk * fk * fk);
    double P[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < n_spl; ++j) {
      int a, n;
      knot_range(off, kcnt, s * n_spl + j, a, n);
      P[j] = (a >= 0) ? spline_value(kx + a, ky + a, n, k_max, xk) : 0.0;
    }
    const double ufg = n_params > 4 ? params[LPS_P_UFG * (size_t)n_states + s] : 0.0;
    for (int c = 0; c < 3; ++c) {
      double terms[4] = {oms[c], tm[c], R[(size_t)c * K + k] * hfac, Rfg ? Rfg[(size_t)c * K + k] * exp10(ufg) : 0.0};
      double S = 0.0;
      for (int tau = 0; tau < 4; ++tau) {
        const int j = route.r[tau][c];
        S += (j >= 0) ? terms[tau] * exp10(P[j]) : terms[tau];
      }
      l += nk[k] * (D[(size_t)c * K + k] / S + log(S));
    }
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = kPlainBlock / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kPlainBlock) void k_plain_finish(
    int n_blocks, const double* __restrict__ part, int s, int n_states, int n_spl, int k_max, int n_params,
    const double* __restrict__ params, const int32_t* __restrict__ off, const int32_t* __restrict__ kcnt,
    const double* __restrict__ kx, const double* __restrict__ ky, double x_first, double x_last,
    double* __restrict__ logL,
    uint32_t* __restrict__ status) {
  __shared__ double red[kPlainBlock];
  double acc = 0.0;
  for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) acc += part[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kPlainBlock / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    uint32_t st = validate_state(s, n_states, n_spl, k_max, n_params, params, off, kcnt, kx, ky, x_first, x_last);
    const double v = -red[0];
    if (st == 0 && !isfinite(v)) st |= LPS_ST_PSD;
    logL[s] = st ? -INFINITY : v;
    if (status) status[s] = st;
  }
}

}  // namespace

hipError_t launch_plain(lps_ctx* ctx, const lps_states* st, double* logL, uint32_t* status, hipStream_t s) {
  const int n = st->n_states;
  const int K = ctx->n_bins;
  const int nb = ctx->plain_blocks;
  Route route;
  for (int t = 0; t < 4; ++t)
    for (int c = 0; c < 3; ++c) route.r[t][c] = ctx->route[t][c];
  timing_begin(ctx, s);
  for (int i = 0; i < n; ++i) {
    hipLaunchKernelGGL(k_plain_bins, dim3(nb), dim3(kPlainBlock), 0, s, K, ctx->f, ctx->nk, ctx->D, ctx->R,
                       ctx->Rfg, ctx->arm_length, ctx->f_knee, ctx->n_spl, ctx->k_max, route, n, ctx->n_params, i,
                       st->params, st->knot_off, st->knot_cnt, st->knot_x, st->knot_y, ctx->plain_part);
    hipLaunchKernelGGL(k_plain_finish, dim3(1), dim3(kPlainBlock), 0, s, nb, ctx->plain_part, i, n, ctx->n_spl,
                       ctx->k_max, ctx->n_params, st->params, st->knot_off, st->knot_cnt, st->knot_x, st->knot_y,
                       ctx->x_first,
                       ctx->x_last, logL, status);
  }
  timing_end(ctx, s);
  return hipGetLastError();
}

}  // namespace lps
