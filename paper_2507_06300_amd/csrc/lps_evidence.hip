// Model-selection reductions over stored tempered log-likelihoods.
//
// Samples are the sampler's logL records, laid out logL[n_rec][T][W] (record,
// temperature rung, walker; chain c = t * W + w as in a sweep), so rung t has
// n = n_rec * W draws.
//
// Stepping-stone evidence, Eq. (ss): for the increasing ladder b_0 < ... < b_{T-1},
//   log r_k = log( (1/n) sum_i exp((b_k - b_{k-1}) L_i) ),  draws i at rung k-1,
//   log Z   = sum_{k=1}^{T-1} log r_k,
// with the exponentials taken relative to the step's maximum, and the
// delta-method variance Var(log r_k) = (n sum w^2 / (sum w)^2 - 1) / n summed
// over the steps (w_i = exp((b_k - b_{k-1}) L_i - max)).
//
// DIC (Sec. "Results"): D = -2 L over the draws of one rung (b = 1),
//   mean D, p_D = mean D - D(theta_bar), DIC = mean D + p_D, Var D,
// where D(theta_bar) = -2 logL at the posterior-mean parameters is an input.
//
// One block per reduction, fixed thread strides and a fixed LDS tree: every
// result is deterministic.
#include <math.h>

#include "lps_internal.hpp"
#include "lps_roctx.hpp"

namespace lps {
namespace {

constexpr int kRedThreads = 256;

// fixed-order block sum (all threads receive the total)
__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// block k-1 computes step k: out[2 + (k-1)] = log r_k, var[k-1]
__global__ __launch_bounds__(kRedThreads) void k_ss_steps(const double* __restrict__ betas, int T, int n_rec, int W,
                                                          const double* __restrict__ logL,
                                                          double* __restrict__ log_r, double* __restrict__ var) {
  __shared__ double sh[kRedThreads];
  const int k = blockIdx.x + 1;
  const double db = betas[k] - betas[k - 1];
  const long n = (long)n_rec * W;
  auto a_at = [&](long i) {
    const long rec = i / W, w = i - rec * W;
    return db * logL[(rec * T + (k - 1)) * W + w];
  };
  double m = -INFINITY;
  for (long i = threadIdx.x; i < n; i += kRedThreads) m = fmax(m, a_at(i));
  m = block_max(m, sh);
  double s1 = 0.0, s2 = 0.0;
  if (isfinite(m)) {
    for (long i = threadIdx.x; i < n; i += kRedThreads) {
      const double w = exp(a_at(i) - m);
      s1 += w;
      s2 += w * w;
    }
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    const double dn = (double)n;
    log_r[k - 1] = isfinite(m) ? m + log(s1) - log(dn) : m;
    var[k - 1] = isfinite(m) ? (dn * s2 / (s1 * s1) - 1.0) / dn : NAN;
  }
}

// out[0] = log Z, out[1] = Var(log Z): ordered sums over the steps
__global__ void k_ss_total(int n_steps, const double* __restrict__ log_r, const double* __restrict__ var,
                           double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double z = 0.0, v = 0.0;
  for (int k = 0; k < n_steps; ++k) {
    z += log_r[k];
    v += var[k];
  }
  out[0] = z;
  out[1] = v;
}

__global__ __launch_bounds__(kRedThreads) void k_dic(int T, int n_rec, int W, int rung,
                                                     const double* __restrict__ logL,
                                                     const double* __restrict__ logL_at_mean,
                                                     double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  const long n = (long)n_rec * W;
  auto d_at = [&](long i) {
    const long rec = i / W, w = i - rec * W;
    return -2.0 * logL[(rec * T + rung) * W + w];
  };
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += kRedThreads) s += d_at(i);
  const double mean = block_sum(s, sh) / (double)n;
  double q = 0.0;
  for (long i = threadIdx.x; i < n; i += kRedThreads) {
    const double e = d_at(i) - mean;
    q += e * e;
  }
  const double var = block_sum(q, sh) / (double)n;
  if (threadIdx.x == 0) {
    const double p_d = mean + 2.0 * logL_at_mean[0];
    out[0] = mean;
    out[1] = p_d;
    out[2] = mean + p_d;
    out[3] = var;
  }
}

// Median of each of m columns x[col * ld + i], i < n (numpy's definition: the
// middle value, or the mean of the two middle values for even n).  One block
// per column; a value is the k-th smallest when fewer than k + 1 values are
// below it and more than k are at or below it, and among equal values the one
// with the lowest index reports it, so no two threads write one output.
__global__ __launch_bounds__(kRedThreads) void k_column_median(int n, int ld, const double* __restrict__ x,
                                                               double* __restrict__ out) {
  __shared__ double pick[2];
  const double* col = x + (size_t)blockIdx.x * ld;
  const int k_lo = (n - 1) / 2, k_hi = n / 2;
  for (int i = threadIdx.x; i < n; i += kRedThreads) {
    const double v = col[i];
    int lt = 0, le = 0, eq_before = 0;
    for (int j = 0; j < n; ++j) {
      const double u = col[j];
      lt += u < v;
      le += u <= v;
      eq_before += (u == v) && (j < i);
    }
    if (eq_before == 0) {
      if (lt <= k_lo && k_lo < le) pick[0] = v;
      if (lt <= k_hi && k_hi < le) pick[1] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = 0.5 * (pick[0] + pick[1]);
}

}  // namespace
}  // namespace lps

extern "C" {

// The 20 rungs of the ladder of Sec. "MCMC setup", increasing: 5 log-spaced
// from 1e-20 (up to, not including, 1e-12), 10 from 1e-12 (up to 1e-5), 5 from
// 1e-5 to 1 inclusive.
lps_status lps_paper_ladder(double* betas) {
  LPS_API_RANGE();
  if (!betas) return LPS_E_NULL;
  struct Group {
    double lo, hi;
    int num;
    bool endpoint;
  };
  const Group groups[3] = {{-20.0, -12.0, 5, false}, {-12.0, -5.0, 10, false}, {-5.0, 0.0, 5, true}};
  int k = 0;
  for (const Group& g : groups) {
    const int div = g.endpoint ? g.num - 1 : g.num;
    const double step = (g.hi - g.lo) / div;
    for (int i = 0; i < g.num; ++i) {
      const double e = (g.endpoint && i == g.num - 1) ? g.hi : g.lo + i * step;
      betas[k++] = pow(10.0, e);
    }
  }
  return LPS_OK;
}

lps_status lps_column_median(const double* x, int32_t n, int32_t m, int32_t ld, double* out, void* stream) {
  LPS_API_RANGE();
  if (!x || !out) return LPS_E_NULL;
  if (n < 1 || m < 1 || ld < n || n > (1 << 16)) return LPS_E_SHAPE;
  hipLaunchKernelGGL(lps::k_column_median, dim3(m), dim3(lps::kRedThreads), 0, (hipStream_t)stream, n, ld, x, out);
  return lps::device_status(hipGetLastError());
}

lps_status lps_stepping_stone(const double* betas, int32_t n_temps, const double* logL, int32_t n_rec,
                              int32_t n_walkers, double* out, void* stream) {
  LPS_API_RANGE();
  if (!betas || !logL || !out) return LPS_E_NULL;
  if (n_temps < 2 || n_rec < 1 || n_walkers < 1) return LPS_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  const int steps = n_temps - 1;
  double* log_r = out + 2;
  double* var = out + 2 + steps;
  hipLaunchKernelGGL(lps::k_ss_steps, dim3(steps), dim3(lps::kRedThreads), 0, s, betas, n_temps, n_rec, n_walkers,
                     logL, log_r, var);
  hipLaunchKernelGGL(lps::k_ss_total, dim3(1), dim3(64), 0, s, steps, log_r, var, out);
  return lps::device_status(hipGetLastError());
}

lps_status lps_dic(const double* logL, int32_t n_rec, int32_t n_temps, int32_t n_walkers, int32_t rung,
                   const double* logL_at_mean, double* out, void* stream) {
  LPS_API_RANGE();
  if (!logL || !logL_at_mean || !out) return LPS_E_NULL;
  if (n_temps < 1 || n_rec < 1 || n_walkers < 1 || rung < 0 || rung >= n_temps) return LPS_E_SHAPE;
  hipLaunchKernelGGL(lps::k_dic, dim3(1), dim3(lps::kRedThreads), 0, (hipStream_t)stream, n_temps, n_rec, n_walkers,
                     rung, logL, logL_at_mean, out);
  return lps::device_status(hipGetLastError());
}

}  // extern "C"
