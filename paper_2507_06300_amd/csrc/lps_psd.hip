// PSD build: S, S_n and S_h in physical units for a bin range of every state.
//
// S_c = S_n,c + S_h,c (Eq. (psd_tot)); each term is its unit template times
// the state's amplitude and 10^P of its routed spline (Eqs. (splines)), i.e.
// ref_tau * T_tau,c(f) * exp2(Q_g(x)) with the exponent pieces of the
// coefficient kernel.  One thread per (state, bin); the piece is found by a
// binary search over the state's breakpoints.  This entry point writes
// 3 * 8 bytes per output row and bin and is bound by HBM writes.
#include <math.h>

#include "lps_internal.hpp"

namespace lps {
namespace {

__device__ inline double eval_group(const double* __restrict__ bx, const double* __restrict__ coef, int ni,
                                    double xk) {
  int lo = 0, hi = ni - 1;   // last piece with bx <= xk (piece 0 when xk < bx[1])
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (bx[mid] <= xk) lo = mid;
    else hi = mid - 1;
  }
  double t = xk - bx[lo];
  const double* c = coef + (size_t)lo * 4;
  return exp2(c[0] + t * (c[1] + t * (c[2] + t * c[3])));
}

__global__ void k_psd(int n_states, int K, int k0, int k1, Layout lay, const double* __restrict__ x,
                      const double* __restrict__ tmpl, const double* __restrict__ bx,
                      const double* __restrict__ coef, const int32_t* __restrict__ n_int,
                      const StateScalars* __restrict__ scal, double* __restrict__ S, double* __restrict__ Sn,
                      double* __restrict__ Sh) {
  const int nb = k1 - k0;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n_states * nb) return;
  const int s = (int)(gid / nb);
  const int kk = (int)(gid % nb);
  const int k = k0 + kk;
  const int G = lay.n_grp;
  const size_t o = (size_t)s * 3 * nb + kk;
  if (n_int[s * G] == 0) {
    for (int c = 0; c < 3; ++c) {
      S[o + (size_t)c * nb] = NAN;
      if (Sn) Sn[o + (size_t)c * nb] = NAN;
      if (Sh) Sh[o + (size_t)c * nb] = NAN;
    }
    return;
  }
  const double xk = x[k];
  double E[kMaxGroups];
  for (int g = 0; g < G; ++g) {
    const size_t base = (size_t)(s * G + g) * kMaxKnots;
    E[g] = eval_group(bx + base, coef + base * 4, n_int[s * G + g], xk);
  }
  const StateScalars sc = scal[s];
  const double ref_oms = kRefAoms * kRefAoms, ref_tm = kRefAtm * kRefAtm;
  const double ref_h = exp2(kRefU * kLog2_10), ref_fg = exp2(kRefUfg * kLog2_10);
  for (int c = 0; c < 3; ++c) {
    const double t_oms = ref_oms * tmpl[(0 * 3 + c) * (size_t)K + k];
    const double t_tm = ref_tm * tmpl[(1 * 3 + c) * (size_t)K + k];
    const double t_h = ref_h * tmpl[(2 * 3 + c) * (size_t)K + k];
    double sn, sh;
    if (lay.mode == kSplit) {
      sn = t_oms * E[0] + t_tm * E[1];
      sh = t_h * E[2];
    } else if (lay.mode == kShared) {
      sn = (sc.w_oms * t_oms + sc.w_tm * t_tm) * E[0];
      sh = t_h * E[1];
    } else {
      sn = (sc.w_oms * t_oms + sc.w_tm * t_tm) * E[c];
      sh = t_h * E[3];
    }
    if (lay.has_fg) sh += ref_fg * tmpl[(3 * 3 + c) * (size_t)K + k] * sc.e_fg;
    S[o + (size_t)c * nb] = sn + sh;
    if (Sn) Sn[o + (size_t)c * nb] = sn;
    if (Sh) Sh[o + (size_t)c * nb] = sh;
  }
}

__global__ void k_copy_status(int n, const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) dst[s] = src[s];
}

}  // namespace

hipError_t launch_psd(lps_ctx* ctx, const lps_states* st, int32_t k0, int32_t k1, double* S, double* Sn, double* Sh,
                      uint32_t* status, hipStream_t s) {
  const int n = st->n_states;
  hipError_t e = launch_coeffs(ctx, st, s);
  if (e != hipSuccess) return e;
  const size_t total = (size_t)n * (size_t)(k1 - k0);
  if (total > 0) {
    const int tpb = 256;
    hipLaunchKernelGGL(k_psd, dim3((unsigned)((total + tpb - 1) / tpb)), dim3(tpb), 0, s, n, ctx->n_bins, k0, k1,
                       ctx->lay, ctx->x, ctx->tmpl, ctx->bx, ctx->coef64, ctx->n_int, ctx->scal, S, Sn, Sh);
  }
  if (status)
    hipLaunchKernelGGL(k_copy_status, dim3((n + 255) / 256), dim3(256), 0, s, n, ctx->status_ws, status);
  return hipGetLastError();
}

}  // namespace lps
