// Per-state validation and exponent pieces (one wave per state, one lane per piece).
//
// For every exponent group of a state this kernel turns the state's knots
// and template parameters into the pieces of
//   Q_g(x) = cst_g + lin_g (x - log10 f_knee) + log2(10) P_j(x)
// (see lps_internal.hpp), where P_j is the Akima / linear spline of App. A
// with the knot convention of Sec. "Power spectral density breakdown" (two
// edge knots at the band extremes plus in-between knots), cst_g is log2 of
// the state's amplitude relative to the reference amplitude, and lin_g is
// alpha log2(10) for the background power law of Eq. (pl).
#include <math.h>

#include "lps_internal.hpp"
#include "lps_spline.hpp"
#include "lps_validate.hpp"

namespace lps {
namespace {

// One wave per state: the lanes validate the knots together and then each
// lane builds one piece of every exponent group.
__global__ __launch_bounds__(256) void k_coeffs(int n_states, int n_spl, int k_max, Layout lay, int n_params,
                                                const double* __restrict__ params, const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ kcnt, int64_t n_knots, const double* __restrict__ kx,
                                                const double* __restrict__ ky, double x_first, double x_last,
                                                double x_knee, double* __restrict__ bx, double* __restrict__ coef64,
                                                float* __restrict__ coef32, int32_t* __restrict__ n_int,
                                                StateScalars* __restrict__ scal, uint32_t* __restrict__ status_ws,
                                                uint32_t* __restrict__ wide_count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *wide_count = 0u;   // per-call queue of the mixed path
  const int lane = threadIdx.x & (kWave - 1);
  const int s = uniform(blockIdx.x * (blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (s >= n_states) return;
  const int G = lay.n_grp;
  const uint32_t st =
      validate_state_wave(lane, s, n_states, n_spl, k_max, n_params, params, off, kcnt, n_knots, kx, ky, x_first, x_last);
  if (lane == 0) status_ws[s] = st;
  if (st) {
    if (lane < G) n_int[s * G + lane] = 0;
    return;
  }
  const double a_oms = params[LPS_P_AOMS * (size_t)n_states + s];
  const double a_tm = params[LPS_P_ATM * (size_t)n_states + s];
  const double u = params[LPS_P_U * (size_t)n_states + s];
  const double alpha = params[LPS_P_ALPHA * (size_t)n_states + s];
  const double u_fg = n_params > 4 ? params[LPS_P_UFG * (size_t)n_states + s] : kRefUfg;
  if (lane == 0) {
    StateScalars sc;
    sc.w_oms = (a_oms / kRefAoms) * (a_oms / kRefAoms);
    sc.w_tm = (a_tm / kRefAtm) * (a_tm / kRefAtm);
    sc.e_fg = exp2((u_fg - kRefUfg) * kLog2_10);
    sc.pad = 0.0;
    scal[s] = sc;
  }
  for (int g = 0; g < G; ++g) {
    double cst = 0.0, lin = 0.0;
    switch (lay.grp_kind[g]) {
      case kGOms: cst = 2.0 * log2(a_oms / kRefAoms); break;
      case kGTm: cst = 2.0 * log2(a_tm / kRefAtm); break;
      case kGSgwb: cst = (u - kRefU) * kLog2_10; lin = alpha * kLog2_10; break;
      default: break;   // noise groups: amplitudes enter as per-bin weights
    }
    const int j = lay.grp_spline[g];
    const size_t base = (size_t)(s * G + g) * kMaxKnots;
    int cnt = 0, a0 = 0;
    if (j >= 0) knot_range(off, kcnt, s * n_spl + j, n_knots, a0, cnt);
    const int n_pieces = cnt == 0 ? 1 : cnt - 1;
    if (lane == 0) n_int[s * G + g] = n_pieces;
    if (lane >= n_pieces) continue;
    double A, B, C, Dd, x0;
    if (cnt == 0) {
      x0 = x_first;
      A = cst + lin * (x_first - x_knee);
      B = lin;
      C = 0.0;
      Dd = 0.0;
    } else {
      const double* x = kx + a0;
      const double* y = ky + a0;
      double a, b, c, d;
      spline_piece(x, y, cnt, lane, a, b, c, d);
      x0 = x[lane];
      A = kLog2_10 * a + cst + lin * (x0 - x_knee);
      B = kLog2_10 * b + lin;
      C = kLog2_10 * c;
      Dd = kLog2_10 * d;
    }
    const size_t i = base + lane;
    bx[i] = x0;
    coef64[i * 4 + 0] = A;
    coef64[i * 4 + 1] = B;
    coef64[i * 4 + 2] = C;
    coef64[i * 4 + 3] = Dd;
    coef32[i * 4 + 0] = (float)A;
    coef32[i * 4 + 1] = (float)B;
    coef32[i * 4 + 2] = (float)C;
    coef32[i * 4 + 3] = (float)Dd;
  }
}

}  // namespace

hipError_t launch_coeffs(lps_ctx* ctx, const lps_states* st, hipStream_t s) {
  const int n = st->n_states;
  const int waves = 4;
  hipLaunchKernelGGL(k_coeffs, dim3((n + waves - 1) / waves), dim3(waves * kWave), 0, s, n, ctx->n_spl, ctx->k_max, ctx->lay,
                     ctx->n_params, st->params, st->knot_off, st->knot_cnt, st->n_knots, st->knot_x, st->knot_y, ctx->x_first,
                     ctx->x_last,
                     log10(ctx->f_knee), ctx->bx, ctx->coef64, ctx->coef32, ctx->n_int, ctx->scal, ctx->status_ws,
                     ctx->wide_count);
  return hipGetLastError();
}

}  // namespace lps
