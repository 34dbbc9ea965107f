// VALU issue-rate calibration used to express the batched kernels' work in
// FP32-FMA-equivalent issue slots.
//
// Two dependent-chain microkernels run on every CU: one issues FP32 FMAs,
// the other issues the single-precision transcendental sequence the mixed
// kernel uses (exp2, log2, rcp).  Eight independent chains per lane keep the
// pipelines full.  The ratio of their per-instruction times is the issue
// cost of a transcendental in FMA slots; the FMA time itself gives the
// achieved lane-instruction rate of the device.
#include "lps_internal.hpp"
#include "lps_math64.hpp"
#include "lps_roctx.hpp"

namespace lps {
namespace {

constexpr int kChains = 16;

__global__ __launch_bounds__(256) void k_fma_chain(int iters, float seed, float* __restrict__ out) {
  float v[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) v[c] = seed + 1e-3f * (threadIdx.x + c);
  const float m = 0.999999f, a = 1e-7f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = __builtin_fmaf(v[c], m, a);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// exp2 / log2 / rcp in a ring so that values stay in range: each step does one
// of each on every chain (3 transcendental instructions per chain per step).
__global__ __launch_bounds__(256) void k_trans_chain(int iters, float seed, float* __restrict__ out) {
  float v[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) v[c] = seed + 1e-3f * (threadIdx.x + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      float e = __builtin_amdgcn_exp2f(v[c]);
      float l = __builtin_amdgcn_logf(e);
      v[c] = __builtin_amdgcn_rcpf(__builtin_amdgcn_rcpf(l));
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_math64(int n, int fn, const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double tab[kExp2Tab];   // for exp2_t, filled before any thread leaves
  fill_exp2_table(tab, (int)threadIdx.x);
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  double r;
  switch (fn) {
    case 0: r = exp2_d(v); break;
    case 1: r = log2_d(v); break;
    case 2: r = rcp_d(v); break;
    case 3: r = sqrt_d(v); break;
    case 4: r = log_d(v); break;
    case 5: r = exp2_t(v, tab); break;
    default: r = rsq_d(v); break;
  }
  out[i] = r;
}

}  // namespace
}  // namespace lps

extern "C" lps_status lps_math64_check(const double* x, int32_t n, int32_t fn, double* out, void* stream) {
  LPS_API_RANGE();
  if (n == 0) return LPS_OK;
  if (!x || !out) return LPS_E_NULL;
  if (n < 0 || fn < 0 || fn > 6) return LPS_E_SHAPE;
  hipLaunchKernelGGL(lps::k_math64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, fn, x,
                     out);
  return lps::device_status(hipGetLastError());
}

extern "C" lps_status lps_valu_probe(int device, double* fma_ns_per_wave_instr, double* trans_over_fma,
                                     double* lane_instr_per_s) {
  LPS_API_RANGE();
  if (!fma_ns_per_wave_instr || !trans_over_fma || !lane_instr_per_s) return LPS_E_NULL;
  if (hipSetDevice(device) != hipSuccess) return LPS_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return LPS_E_DEVICE;
  const int blocks = prop.multiProcessorCount * 16;   // 16 blocks of 4 waves per CU
  const int threads = 256;
  float* out = nullptr;
  if (hipMalloc((void**)&out, (size_t)blocks * threads * sizeof(float)) != hipSuccess) return LPS_E_NOMEM;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int iters = 4096;
  float t_fma = 0.f, t_tr = 0.f;
  for (int rep = 0; rep < 3; ++rep) {
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(lps::k_fma_chain, dim3(blocks), dim3(threads), 0, nullptr, iters, 0.5f, out);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&t_fma, e0, e1);
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(lps::k_trans_chain, dim3(blocks), dim3(threads), 0, nullptr, iters, 0.5f, out);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&t_tr, e0, e1);
  }
  const double waves = (double)blocks * threads / 64.0;
  const double fma_instr = waves * iters * lps::kChains;          // wave-level instructions
  const double tr_instr = waves * iters * lps::kChains * 4.0;      // exp2, log2, rcp, rcp
  const double ns_fma = t_fma * 1e6 / fma_instr * prop.multiProcessorCount * 4;   // per SIMD
  const double ns_tr = t_tr * 1e6 / tr_instr * prop.multiProcessorCount * 4;
  *fma_ns_per_wave_instr = ns_fma;
  *trans_over_fma = ns_tr / ns_fma;
  *lane_instr_per_s = fma_instr * 64.0 / (t_fma * 1e-3);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return hipGetLastError() == hipSuccess ? LPS_OK : LPS_E_DEVICE;
}
