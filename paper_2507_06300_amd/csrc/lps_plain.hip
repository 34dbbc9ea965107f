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

#include <mutex>

#include "lps_internal.hpp"
#include "lps_spline.hpp"
#include "lps_validate.hpp"
#include "lps_roctx.hpp"

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
    const int32_t* __restrict__ off, const int32_t* __restrict__ kcnt, int64_t n_knots, const double* __restrict__ kx,
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
      knot_range(off, kcnt, s * n_spl + j, n_knots, a, n);
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
    const double* __restrict__ params, const int32_t* __restrict__ off, const int32_t* __restrict__ kcnt, int64_t n_knots,
    const double* __restrict__ kx, const double* __restrict__ ky, const double* __restrict__ f, int K,
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
    // band edges for the coverage test: log10 of the first and last bin
    const double x_first = log10(f[0]), x_last = log10(f[K - 1]);
    uint32_t st = validate_state(s, n_states, n_spl, k_max, n_params, params, off, kcnt, n_knots, kx, ky, x_first, x_last);
    const double v = -red[0];
    if (st == 0 && !isfinite(v)) st |= LPS_ST_PSD;
    logL[s] = st ? -INFINITY : v;
    if (status) status[s] = st;
  }
}

// Every input of the plain path: the dataset arrays and its constants.
struct PlainData {
  int K, n_spl, k_max, n_params;
  const double *f, *nk, *D, *R, *Rfg;
  double L, f_knee;
  Route route;
};

// One bins launch and one finish launch per state, in state order on one
// stream: part[0 .. ceil(K / kPlainBlock)) holds one state's block sums at a
// time, each entry written by the bins launch before the finish launch reads it.
hipError_t launch_plain_core(const PlainData& d, const lps_states* st, double* part, double* logL,
                             uint32_t* status, hipStream_t s) {
  const int n = st->n_states;
  const int nb = (d.K + kPlainBlock - 1) / kPlainBlock;
  for (int i = 0; i < n; ++i) {
    hipLaunchKernelGGL(k_plain_bins, dim3(nb), dim3(kPlainBlock), 0, s, d.K, d.f, d.nk, d.D, d.R, d.Rfg, d.L,
                       d.f_knee, d.n_spl, d.k_max, d.route, n, d.n_params, i, st->params, st->knot_off,
                       st->knot_cnt, st->n_knots, st->knot_x, st->knot_y, part);
    hipLaunchKernelGGL(k_plain_finish, dim3(1), dim3(kPlainBlock), 0, s, nb, part, i, n, d.n_spl, d.k_max,
                       d.n_params, st->params, st->knot_off, st->knot_cnt, st->n_knots, st->knot_x, st->knot_y, d.f, d.K, logL,
                       status);
  }
  return hipGetLastError();
}

// Scratch of the allocation-free entry point: the per-block sums of one state
// (one double per kPlainBlock bins), 512 KiB, so at most 2^24 bins.  Each GPU
// holds its own copy for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr int kNoallocBlocks = 1 << 16;
static __device__ __align__(256) double scratch[kNoallocBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

hipError_t launch_plain(lps_ctx* ctx, const lps_states* st, double* logL, uint32_t* status, hipStream_t s) {
  PlainData d;
  d.K = ctx->n_bins;
  d.n_spl = ctx->n_spl;
  d.k_max = ctx->k_max;
  d.n_params = ctx->n_params;
  d.f = ctx->f;
  d.nk = ctx->nk;
  d.D = ctx->D;
  d.R = ctx->R;
  d.Rfg = ctx->Rfg;
  d.L = ctx->arm_length;
  d.f_knee = ctx->f_knee;
  for (int t = 0; t < 4; ++t)
    for (int c = 0; c < 3; ++c) d.route.r[t][c] = ctx->route[t][c];
  timing_begin(ctx, s);
  const hipError_t e = launch_plain_core(d, st, ctx->plain_part, logL, status, s);
  timing_end(ctx, s);
  return e;
}

}  // namespace lps

extern "C" lps_status lps_loglike_plain_fp64_noalloc(const lps_dataset_desc* d, const lps_states* st,
                                                     double* logL, uint32_t* status, void* stream) {
  LPS_API_RANGE();
  if (!d || !st) return LPS_E_NULL;
  if (!d->f || !d->nk || !d->D || !d->R) return LPS_E_NULL;
  if (d->n_bins < 1 || d->n_spl < 0 || d->n_spl > 4) return LPS_E_SHAPE;
  if ((d->n_bins + lps::kPlainBlock - 1) / lps::kPlainBlock > lps::kNoallocBlocks) return LPS_E_CAPACITY;
  if (d->k_max < 2 || d->k_max > lps::kMaxKnots) return LPS_E_CAPACITY;
  if (!(d->f_knee > 0.0) || !(d->arm_length > 0.0)) return LPS_E_SHAPE;
  for (int t = 0; t < 4; ++t)
    for (int c = 0; c < 3; ++c) {
      const int j = d->route[t][c];
      if (j < -1 || j >= d->n_spl || (t == LPS_TERM_FG && j != -1)) return LPS_E_ROUTING;
    }
  if (st->n_states < 0 || st->n_knots < 0) return LPS_E_SHAPE;
  if (st->n_states == 0) return LPS_OK;
  if (!st->params || !st->knot_off || !logL) return LPS_E_NULL;
  if (d->n_spl > 0 && (!st->knot_x || !st->knot_y)) return LPS_E_NULL;
  double* part = nullptr;
  hipError_t e = lps::scratch_address(&part);
  if (e != hipSuccess) return lps::device_status(e);
  lps::PlainData pd;
  pd.K = d->n_bins;
  pd.n_spl = d->n_spl;
  pd.k_max = d->k_max;
  pd.n_params = d->Rfg ? 5 : 4;
  pd.f = d->f;
  pd.nk = d->nk;
  pd.D = d->D;
  pd.R = d->R;
  pd.Rfg = d->Rfg;
  pd.L = d->arm_length;
  pd.f_knee = d->f_knee;
  for (int t = 0; t < 4; ++t)
    for (int c = 0; c < 3; ++c) pd.route.r[t][c] = d->route[t][c];
  return lps::device_status(lps::launch_plain_core(pd, st, part, logL, status, (hipStream_t)stream));
}
