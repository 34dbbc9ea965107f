// Data stage on the device: from TDI time series to the averaged periodogram
// and the per-bin response that lps_create takes.
//
//   periodogram:  X_k = sum_n w_n x_n exp(-2 pi i k n / N) (hipFFT, double),
//                 P_k = c_k dt |X_k|^2 / (N mean(w^2)),  c_k = 1 at k = 0 and
//                 k = N/2 (N even), else 2 (one-sided: E[P_k] is the PSD);
//                 optionally after the XYZ -> AET combination of the series
//                 A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3.
//   averaging:    segments of n consecutive non-overlapping bins (Sec. "MCMC
//                 setup"): D_i = mean of P over the segment, nu_i = n, f_i = mean
//                 of the segment's bin frequencies.
//   response:     a response tabulated on a frequency grid, interpolated to the
//                 analysis frequencies (Sec. "Parametrized SGWB model"): linear
//                 in (log f, log R) where both grid values are positive, linear
//                 in (log f, R) otherwise; NaN outside the grid.
#include <hipfft/hipfft.h>
#include <math.h>

#include "lps_internal.hpp"
#include "lps_roctx.hpp"

namespace lps {
namespace {

constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt3 = 0.57735026918962576451;
constexpr double kInvSqrt6 = 0.40824829046386301637;

__global__ void k_prep_series(int n_ch, int n, const double* __restrict__ x, const double* __restrict__ w, int aet,
                              double* __restrict__ xw) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double wi = w ? w[i] : 1.0;
  if (aet) {
    const double X = x[i], Y = x[(size_t)n + i], Z = x[2 * (size_t)n + i];
    xw[i] = wi * ((Z - X) * kInvSqrt2);
    xw[(size_t)n + i] = wi * ((X - 2.0 * Y + Z) * kInvSqrt6);
    xw[2 * (size_t)n + i] = wi * ((X + Y + Z) * kInvSqrt3);
  } else {
    for (int c = 0; c < n_ch; ++c) xw[(size_t)c * n + i] = wi * x[(size_t)c * n + i];
  }
}

// mean(w^2) in two fixed-order stages (1 when there is no window): kWinParts
// blocks each add a grid-strided share of w^2, then one block adds the partials.
constexpr int kWinParts = 256;

__global__ __launch_bounds__(256) void k_window_part(int n, const double* __restrict__ w,
                                                     double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  if (w)
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)kWinParts * 256) acc += w[i] * w[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_window_power(int n, const double* __restrict__ w,
                                                      const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kWinParts];
  sh[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int s = kWinParts / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = w ? sh[0] / (double)n : 1.0;
}

__global__ void k_power(int n_ch, int n, int nf, double dt, const hipfftDoubleComplex* __restrict__ X,
                        const double* __restrict__ w2, double* __restrict__ P) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_ch * nf) return;
  const int k = (int)(i % nf);
  const double c = (k == 0 || (n % 2 == 0 && k == n / 2)) ? 1.0 : 2.0;
  const hipfftDoubleComplex z = X[i];
  P[i] = c * dt * (z.x * z.x + z.y * z.y) / ((double)n * w2[0]);
}

__global__ void k_average(int n_ch, int n_f, int k0, int seg_len, int n_seg, const double* __restrict__ P,
                          const double* __restrict__ f, double* __restrict__ D, double* __restrict__ f_seg,
                          double* __restrict__ nu) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)(n_ch + 1) * n_seg) return;
  const int c = (int)(i / n_seg), s = (int)(i % n_seg);
  const long a = (long)k0 + (long)s * seg_len;
  const double* src = c < n_ch ? P + (size_t)c * n_f : f;
  double acc = 0.0;
  for (int j = 0; j < seg_len; ++j) acc += src[a + j];
  acc /= (double)seg_len;
  if (c < n_ch) {
    D[(size_t)c * n_seg + s] = acc;
  } else {
    if (f_seg) f_seg[s] = acc;
    if (nu) nu[s] = (double)seg_len;
  }
}

__global__ void k_response(int n_ch, int n_g, const double* __restrict__ gf, const double* __restrict__ gR, int n,
                           const double* __restrict__ f, double* __restrict__ R) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_ch * n) return;
  const int c = (int)(i / n), q = (int)(i % n);
  const double fq = f[q];
  double out = NAN;
  if (fq >= gf[0] && fq <= gf[n_g - 1]) {
    int lo = 0, hi = n_g - 1;   // last node <= fq, kept below n_g - 1
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (gf[mid] <= fq) lo = mid;
      else hi = mid;
    }
    const double l0 = log(gf[lo]), l1 = log(gf[lo + 1]);
    const double t = (log(fq) - l0) / (l1 - l0);
    const double r0 = gR[(size_t)c * n_g + lo], r1 = gR[(size_t)c * n_g + lo + 1];
    if (r0 > 0.0 && r1 > 0.0) {
      const double a = log(r0);
      out = exp(a + t * (log(r1) - a));
    } else {
      out = r0 + t * (r1 - r0);
    }
  }
  R[i] = out;
}

inline dim3 blocks_for(long n, int tpb) { return dim3((unsigned)((n + tpb - 1) / tpb)); }

}  // namespace
}  // namespace lps

// A planned periodogram: the transform plan, its work area and the
// temporaries, all made once so that every periodogram call is asynchronous
// and allocates nothing.
struct lps_data_ctx {
  int device;
  int n_ch, n_t, nf;
  hipfftHandle plan;
  bool have_plan;
  void* work;                  // transform work area (owned)
  double* xw;                  // [n_ch][n_t] windowed (and combined) series
  hipfftDoubleComplex* X;      // [n_ch][nf] transforms
  double* w2;                  // [1 + kWinParts]: mean(w^2), then the partial sums
};

namespace {

void free_data_ctx(lps_data_ctx* c) {
  if (c->have_plan) (void)hipfftDestroy(c->plan);
  void* ptrs[] = {c->work, c->xw, c->X, c->w2};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

lps_status periodogram_on(lps_data_ctx* c, const double* x, double dt, const double* window, int32_t xyz_to_aet,
                          double* P, hipStream_t s) {
  const int n_ch = c->n_ch, n_t = c->n_t, nf = c->nf;
  if (hipfftSetStream(c->plan, s) != HIPFFT_SUCCESS) return LPS_E_DEVICE;
  hipLaunchKernelGGL(lps::k_prep_series, lps::blocks_for(n_t, 256), dim3(256), 0, s, n_ch, n_t, x, window,
                     xyz_to_aet, c->xw);
  hipLaunchKernelGGL(lps::k_window_part, dim3(lps::kWinParts), dim3(256), 0, s, n_t, window, c->w2 + 1);
  hipLaunchKernelGGL(lps::k_window_power, dim3(1), dim3(lps::kWinParts), 0, s, n_t, window, c->w2 + 1, c->w2);
  if (hipfftExecD2Z(c->plan, (hipfftDoubleReal*)c->xw, c->X) != HIPFFT_SUCCESS) return LPS_E_DEVICE;
  hipLaunchKernelGGL(lps::k_power, lps::blocks_for((long)n_ch * nf, 256), dim3(256), 0, s, n_ch, n_t, nf, dt, c->X,
                     c->w2, P);
  return lps::device_status(hipGetLastError());
}

}  // namespace

extern "C" {

lps_status lps_data_create(int32_t n_ch, int32_t n_t, int device, lps_data_ctx** out) {
  LPS_API_RANGE();
  if (!out) return LPS_E_NULL;
  *out = nullptr;
  if (n_ch < 1 || n_t < 2) return LPS_E_SHAPE;
  if (hipSetDevice(device) != hipSuccess) return LPS_E_DEVICE;
  lps_data_ctx* c = new lps_data_ctx;
  c->device = device;
  c->n_ch = n_ch;
  c->n_t = n_t;
  c->nf = n_t / 2 + 1;
  c->plan = 0;
  c->have_plan = false;
  c->work = nullptr;
  c->xw = nullptr;
  c->X = nullptr;
  c->w2 = nullptr;
  const int nf = c->nf;
  bool ok = hipMalloc((void**)&c->xw, (size_t)n_ch * n_t * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->X, (size_t)n_ch * nf * sizeof(hipfftDoubleComplex)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->w2, (1 + lps::kWinParts) * sizeof(double)) == hipSuccess;
  if (!ok) {
    free_data_ctx(c);
    return LPS_E_NOMEM;
  }
  // batched real-to-complex plan with a caller-owned work area
  int n[1] = {n_t};
  int inembed[1] = {n_t}, onembed[1] = {nf};
  size_t work = 0;
  if (hipfftCreate(&c->plan) != HIPFFT_SUCCESS) {
    free_data_ctx(c);
    return LPS_E_DEVICE;
  }
  c->have_plan = true;
  if (hipfftSetAutoAllocation(c->plan, 0) != HIPFFT_SUCCESS ||
      hipfftMakePlanMany(c->plan, 1, n, inembed, 1, n_t, onembed, 1, nf, HIPFFT_D2Z, n_ch, &work) !=
          HIPFFT_SUCCESS) {
    free_data_ctx(c);
    return LPS_E_DEVICE;
  }
  if (work > 0) {
    if (hipMalloc(&c->work, work) != hipSuccess) {
      free_data_ctx(c);
      return LPS_E_NOMEM;
    }
    if (hipfftSetWorkArea(c->plan, c->work) != HIPFFT_SUCCESS) {
      free_data_ctx(c);
      return LPS_E_DEVICE;
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    free_data_ctx(c);
    return LPS_E_DEVICE;
  }
  *out = c;
  return LPS_OK;
}

lps_status lps_data_destroy(lps_data_ctx* ctx) {
  LPS_API_RANGE();
  if (!ctx) return LPS_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_data_ctx(ctx);
  return LPS_OK;
}

lps_status lps_data_periodogram_planned(lps_data_ctx* ctx, const double* x, double dt, const double* window,
                                        int32_t xyz_to_aet, double* P, void* stream) {
  LPS_API_RANGE();
  if (!ctx || !x || !P) return LPS_E_NULL;
  if (!(dt > 0.0) || (xyz_to_aet && ctx->n_ch != 3)) return LPS_E_SHAPE;
  return periodogram_on(ctx, x, dt, window, xyz_to_aet, P, (hipStream_t)stream);
}

lps_status lps_data_periodogram(const double* x, int32_t n_ch, int32_t n_t, double dt, const double* window,
                                int32_t xyz_to_aet, double* P, void* stream) {
  LPS_API_RANGE();
  if (!x || !P) return LPS_E_NULL;
  if (n_ch < 1 || n_t < 2 || !(dt > 0.0) || (xyz_to_aet && n_ch != 3)) return LPS_E_SHAPE;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return LPS_E_DEVICE;
  lps_data_ctx* c = nullptr;
  lps_status st = lps_data_create(n_ch, n_t, device, &c);
  if (st != LPS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = periodogram_on(c, x, dt, window, xyz_to_aet, P, s);
  // the temporaries are released after the stream has consumed them
  const hipError_t sync = hipStreamSynchronize(s);
  if (st == LPS_OK && sync != hipSuccess) st = lps::device_status(sync);
  free_data_ctx(c);
  return st;
}

lps_status lps_data_average(const double* P, int32_t n_ch, int32_t n_f, const double* f, int32_t k0, int32_t seg_len,
                            int32_t n_seg, double* D, double* f_seg, double* nu, void* stream) {
  LPS_API_RANGE();
  if (!P || !f || !D) return LPS_E_NULL;
  if (n_ch < 1 || n_f < 1 || k0 < 0 || seg_len < 1 || n_seg < 1 || (long)k0 + (long)seg_len * n_seg > n_f)
    return LPS_E_SHAPE;
  hipLaunchKernelGGL(lps::k_average, lps::blocks_for((long)(n_ch + 1) * n_seg, 256), dim3(256), 0,
                     (hipStream_t)stream, n_ch, n_f, k0, seg_len, n_seg, P, f, D, f_seg, nu);
  return lps::device_status(hipGetLastError());
}

lps_status lps_data_response(const double* grid_f, const double* grid_R, int32_t n_ch, int32_t n_g, const double* f,
                             int32_t n, double* R, void* stream) {
  LPS_API_RANGE();
  if (!grid_f || !grid_R || !f || !R) return LPS_E_NULL;
  if (n_ch < 1 || n_g < 2 || n < 1) return LPS_E_SHAPE;
  hipLaunchKernelGGL(lps::k_response, lps::blocks_for((long)n_ch * n, 256), dim3(256), 0, (hipStream_t)stream, n_ch,
                     n_g, grid_f, grid_R, n, f, R);
  return lps::device_status(hipGetLastError());
}

}  // extern "C"
