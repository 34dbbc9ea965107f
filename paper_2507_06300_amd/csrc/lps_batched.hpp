// Device helpers shared by the batched forward and adjoint kernels.
#pragma once

#include <math.h>

#include "lps_internal.hpp"
#include "lps_math64.hpp"

namespace lps {

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
  __device__ static inline double exp2_(double v) { return exp2_d(v); }
  __device__ static inline double log2_(double v) { return log2_d(v); }
  __device__ static inline double rcp_(double v) { return rcp_d(v); }
};

template <int MODE>
struct Groups {
  static constexpr int G = MODE == kSplit ? 3 : (MODE == kShared ? 2 : 4);
};

template <typename R>
__device__ inline R readlane_r(R v, int lane);
template <>
__device__ inline float readlane_r<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <>
__device__ inline double readlane_r<double>(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Orders LDS writes and reads of one wavefront (lanes exchange data through LDS).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of interior breakpoints bx[1 .. ni-1] that are <= v (binary search).
__device__ inline int count_le(const double* __restrict__ bxs, int ni, double v) {
  int lo = 0, hi = ni - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (bxs[1 + mid] <= v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}


}  // namespace lps
