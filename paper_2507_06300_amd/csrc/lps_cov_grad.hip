// Adjoint of the full-covariance likelihood (model and numerics as in
// lps_cov_common.hpp): logL and its derivatives with respect to the
// template parameters and every knot, one wave per state.
#include <hip/hip_runtime.h>
#include <math.h>

#include "lps.h"
#include "lps_internal.hpp"
#include "lps_math64.hpp"
#include "lps_spline_back.hpp"
#include "lps_validate.hpp"
#include "lps_cov_common.hpp"
#include "lps_roctx.hpp"

namespace lps {
namespace {

using namespace covk;

// ---------------------------------------------------------------------------
// Adjoint of the full-covariance likelihood (FP64), one wave per state.
//
// Per bin, with G = C^-1 - C^-1 P C^-1 (the derivative of tr(C^-1 P) + ln det C
// with respect to the symmetric C), dlogL/dC_aa = -N G_aa and, for the pair
// a < b, dlogL/dC_ab = -2 N G_ab.  Through C_cc = Sn_c + Sh_c and
// C_ab = r_ab sqrt(Sn_a Sn_b):
//   dSh_c = dC_cc,   dSn_c = dC_cc + sum_{b != c} dC_cb C_cb / (2 Sn_c),
//   dr_ab = dC_ab sqrt(Sn_a Sn_b),
// then the vine (r_ET = r_AE r_AT + p S, S = sqrt((1 - r_AE^2)(1 - r_AT^2))),
// dq = dr (1 - r^2) for r = tanh q, and d(10^P)/dP = ln 10 10^P for the level
// slots.  The slot derivatives dlogL/dP_j(x) are summed per spline piece as
// moments M_m = sum dP t^m (t from the piece start), and the Akima backward
// turns them into knot derivatives.
//
// The wave walks the band in passes of 64 bins, one bin per lane, in three
// phases: the spline values (one spline at a time), the bin's model and its
// adjoint, then the moments.  The adjoint adds each of its derivative terms
// (OMS, TM and background per channel, three correlations) into the slot it is
// routed to with an LDS atomic add (no read-modify-write in the wave), and
// the moment phase reads one sum per spline.  A lane keeps the moments of the
// piece under the cursor in registers; a pass that crosses a knot adds the
// bins beyond it piece by piece (wave sums), and a finished piece's moments go
// to the state's moment table in global memory, where lane q alone reads and
// writes the entries of piece q (so no fence is needed between the lanes).
// The cursor state is uniform and held across lanes of two registers, picked
// by lane index: lane 3j + f of cv holds field f of spline j (the piece under
// the cursor, the last piece this pass reaches, the number of pieces) and
// lane 6j + f of rec field f of that piece (start, four coefficients, start
// of the next piece), so no cursor read waits on memory.
// ---------------------------------------------------------------------------

// Per wave; lane-private columns.  The Akima backward at the end reuses them.
struct CovGradLds {
  double val[kSlots][kWave];   // slot values of the lane's bin
  double gp[kSlots][kWave];    // dlogL / d(slot argument) of the lane's bin
};
static_assert(sizeof(BackLds) <= sizeof(CovGradLds), "backward LDS aliases val and gp");

__device__ inline void mo_add(double* __restrict__ m, const double (&v)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) m[i] += v[i];
}

__device__ inline void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// NS >= n_spl: the splines whose piece moments a lane keeps in registers.
// Two waves per SIMD; the polynomial coefficients of exp2 and log sit in scalar
// registers, since the moment accumulators leave few vector registers.
template <int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_cov_grad(
    CovArgs A, double* __restrict__ mo_ws, const int32_t* __restrict__ off, const int32_t* __restrict__ kcnt,
    int64_t n_knots, const double* __restrict__ kx, const double* __restrict__ ky, int n_params,
    const double* __restrict__ c0, double* __restrict__ logL, double* __restrict__ dparams, double* __restrict__ dkx,
    double* __restrict__ dky, uint32_t* __restrict__ status_out) {
  __shared__ CovGradLds lds[4];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = (int)(threadIdx.x / kWave);
  const int s = uniform(blockIdx.x * 4 + w);
  if (s >= A.n_states) return;
  CovGradLds& L = lds[w];
  const int n_spl = A.n_spl;
  uint32_t st = A.status[s];
  auto zero_outputs = [&]() {
    if (lane < n_params) dparams[lane * (size_t)A.n_states + s] = 0.0;
    for (int j = 0; j < n_spl; ++j) {
      int a, cn;
      knot_range(off, kcnt, s * n_spl + j, n_knots, a, cn);
      for (int i = lane; i < cn; i += kWave) {
        dkx[a + i] = 0.0;
        dky[a + i] = 0.0;
      }
    }
  };
  if (st != 0u) {
    if (lane == 0) {
      logL[s] = -INFINITY;
      if (status_out) status_out[s] = st;
    }
    zero_outputs();
    return;
  }
  double* mo = mo_ws + (size_t)s * kCovMaxSpl * kMaxKnots * 4;   // lane q owns mo[j][q][*]
  for (int j = 0; j < n_spl; ++j)
#pragma unroll
    for (int m = 0; m < 4; ++m) mo[((size_t)j * kMaxKnots + lane) * 4 + m] = 0.0;
  // lanes 6j .. 6j + 5 of rec take piece q of spline j
  double rec = 0.0;
  auto load_rec = [&](int j, int q, int np) {
    const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
    const int f = lane - 6 * j;
    if (f == 0) rec = A.bx[row + q];
    else if (f >= 1 && f <= 4) rec = A.coef[(row + q) * 4 + (f - 1)];
    else if (f == 5) rec = q + 1 < np ? A.bx[row + q + 1] : INFINITY;
  };
  // cursors at the first bin
  const double x_first = A.tab[tab_index(kRx, 0)];
  int cv = 0;
#pragma unroll 1
  for (int j = 0; j < n_spl; ++j) {
    const int np = uniform(A.npc[(size_t)s * kCovMaxSpl + j]);
    int cur = -1;
    if (np > 0) {
      const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
      const double bl = lane < np ? A.bx[row + lane] : INFINITY;
      cur = uniform(max(__popcll(__ballot(bl <= x_first)) - 1, 0));
      load_rec(j, cur, np);
    }
    cv = lane == 3 * j || lane == 3 * j + 1 ? cur : (lane == 3 * j + 2 ? np : cv);
  }
  L.val[kSlotOne][lane] = 1.0;
  L.val[kSlotZero][lane] = 0.0;
#pragma unroll
  for (int j = 0; j < kSlots; ++j) L.gp[j][lane] = 0.0;
  const StateScal sc = state_scalars(A.params, A.n_states, s, A.has_fg);
  double acc[NS][4];
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[j][m] = 0.0;
  double lsum = 0.0, g_wo = 0.0, g_wt = 0.0, g_lin = 0.0, g_linx = 0.0, g_fg = 0.0;
  bool bad = false;
  const int n_pass = A.n_chunks * (kCovChunk / kWave);
  const double* const xrow = A.tab + kRx * kWave + lane;
  double x_next = xrow[0];   // the abscissae one pass ahead
  for (int ps = 0; ps < n_pass; ++ps) {
    const int kb = ps * kWave;
    const double x = x_next;
    if (ps + 1 < n_pass) x_next = xrow[(size_t)(ps + 1) * kCovBlock];
    const double xl = readlane_r(x, kWave - 1);
    // pieces that start inside this pass
#pragma unroll 1
    for (int j = 0; j < n_spl; ++j) {
      const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
      if (cur < 0 || !(xl >= readlane_r(rec, 6 * j + 5))) continue;
      const int np = __builtin_amdgcn_readlane(cv, 3 * j + 2);
      const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
      int h = cur + 1;
      while (h + 1 < np && A.bx[row + h + 1] <= xl) ++h;
      cv = lane == 3 * j + 1 ? h : cv;
    }
    const TabRow rw{A.tab + (size_t)ps * kCovBlock + lane};
    // spline values
    const double lin = sc.u + sc.alpha * (x - A.x_knee);
#pragma unroll 1
    for (int j = 0; j < n_spl; ++j) {
      const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
      double pv = 0.0;
      if (cur >= 0) {
        double x0 = readlane_r(rec, 6 * j), a0 = readlane_r(rec, 6 * j + 1), a1 = readlane_r(rec, 6 * j + 2);
        double a2 = readlane_r(rec, 6 * j + 3), a3 = readlane_r(rec, 6 * j + 4);
        const int hi = __builtin_amdgcn_readlane(cv, 3 * j + 1);
        if (hi != cur) {
          const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
          const int np = __builtin_amdgcn_readlane(cv, 3 * j + 2);
          for (int q = cur + 1; q <= hi; ++q) {
            const PieceRec nq = load_piece(A, row, q, np);
            if (x >= nq.x0) {
              x0 = nq.x0;
              a0 = nq.a0;
              a1 = nq.a1;
              a2 = nq.a2;
              a3 = nq.a3;
            }
          }
        }
        const double tt = x - x0;
        pv = a0 + tt * (a1 + tt * (a2 + tt * a3));
      }
      L.val[j][lane] = slot_value<true>(pv, j, A.rt, lin);
    }
    // the bin's model and adjoint
    {
      const LdsVal val{&L.val[0][lane]};
      const double hf = background_factor<true>(A.rt, sc, x, A.x_knee);
      CovPoint p;
      cov_point_h(val, A.rt, sc, hf, rw, p);
      // sqrt(Sn_a Sn_b) = sqrt(Sn_a) sqrt(Sn_b) and the 1 / Sn_c below from
      // three reciprocal square roots (0 where Sn_c = 0, as sqrt gives)
      double ir[3], qs[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ir[c] = p.sn[c] > 0.0 ? rsq_d(p.sn[c]) : 0.0;
        qs[c] = p.sn[c] * ir[c];
      }
      const CovAdj cj = cov_adj_s(p, qs[0] * qs[1], qs[0] * qs[2], qs[1] * qs[2]);
      const double id = rcp_d(cj.det);
      lsum += cov_term_tr<true>(cj, p, rw, cov_trace_num(cj, rw) * id, bad);
      const double nu = rw(kRnu);
      const double ci00 = cj.a00 * id, ci11 = cj.a11 * id, ci22 = cj.a22 * id;
      const double ci01 = cj.a01 * id, ci02 = cj.a02 * id, ci12 = cj.a12 * id;
      const double P00 = rw(kRP + 0), P11 = rw(kRP + 1), P22 = rw(kRP + 2);
      const double P01 = rw(kRP + 3), P02 = rw(kRP + 4), P12 = rw(kRP + 5);
      // X = C^-1 P (row a, column c), then G = C^-1 - X C^-1 (symmetric)
      const double X00 = ci00 * P00 + ci01 * P01 + ci02 * P02;
      const double X01 = ci00 * P01 + ci01 * P11 + ci02 * P12;
      const double X02 = ci00 * P02 + ci01 * P12 + ci02 * P22;
      const double X10 = ci01 * P00 + ci11 * P01 + ci12 * P02;
      const double X11 = ci01 * P01 + ci11 * P11 + ci12 * P12;
      const double X12 = ci01 * P02 + ci11 * P12 + ci12 * P22;
      const double X20 = ci02 * P00 + ci12 * P01 + ci22 * P02;
      const double X21 = ci02 * P01 + ci12 * P11 + ci22 * P12;
      const double X22 = ci02 * P02 + ci12 * P12 + ci22 * P22;
      const double G00 = ci00 - (X00 * ci00 + X01 * ci01 + X02 * ci02);
      const double G11 = ci11 - (X10 * ci01 + X11 * ci11 + X12 * ci12);
      const double G22 = ci22 - (X20 * ci02 + X21 * ci12 + X22 * ci22);
      const double G01 = ci01 - (X00 * ci01 + X01 * ci11 + X02 * ci12);
      const double G02 = ci02 - (X00 * ci02 + X01 * ci12 + X02 * ci22);
      const double G12 = ci12 - (X10 * ci02 + X11 * ci12 + X12 * ci22);
      // dlogL / dC (pairs counted once)
      const double gC00 = -nu * G00, gC11 = -nu * G11, gC22 = -nu * G22;
      const double gC01 = -2.0 * nu * G01, gC02 = -2.0 * nu * G02, gC12 = -2.0 * nu * G12;
      const double c01 = p.r01 * cj.s01, c02 = p.r02 * cj.s02, c12 = p.r12 * cj.s12;
      const double gsh[3] = {gC00, gC11, gC22};
      const double gsn[3] = {gC00 + (gC01 * c01 + gC02 * c02) * (0.5 * ir[0] * ir[0]),
                             gC11 + (gC01 * c01 + gC12 * c12) * (0.5 * ir[1] * ir[1]),
                             gC22 + (gC02 * c02 + gC12 * c12) * (0.5 * ir[2] * ir[2])};
      double gr01 = gC01 * cj.s01, gr02 = gC02 * cj.s02;
      const double gr12 = gC12 * cj.s12;
      const double pp = val(A.rt.gc[2]);
      const double S = p.vs;
      // S = 0 only where a correlation is exactly +-1; S is then 0 whatever the
      // other correlation, so its derivative terms drop out
      const double iS = S > 0.0 ? rcp_d(S) : 0.0;
      gr01 += gr12 * (p.r02 - pp * p.r01 * (1.0 - p.r02 * p.r02) * iS);
      gr02 += gr12 * (p.r01 - pp * p.r02 * (1.0 - p.r01 * p.r01) * iS);
      lds_add(&L.gp[A.rt.gc[0]][lane], gr01 * (1.0 - p.r01 * p.r01));
      lds_add(&L.gp[A.rt.gc[1]][lane], gr02 * (1.0 - p.r02 * p.r02));
      lds_add(&L.gp[A.rt.gc[2]][lane], gr12 * S * (1.0 - pp * pp));
      // level slots: the OMS, TM and background terms of each channel
      double gl = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double oms = rw(c < 2 ? kRomsAE : kRomsT), tm = rw(c < 2 ? kRtmAE : kRtmT);
        const double fo = oms * val(A.rt.g[0][c]), ft = tm * val(A.rt.g[1][c]);
        const double th = rw(kRsg + c) * hf * val(A.rt.g[2][c]);
        g_wo += gsn[c] * fo;
        g_wt += gsn[c] * ft;
        g_fg += gsh[c] * rw(kRfg + c);
        gl += gsh[c] * th;
        lds_add(&L.gp[A.rt.g[0][c]][lane], kLn10 * gsn[c] * (sc.w_oms * fo));
        lds_add(&L.gp[A.rt.g[1][c]][lane], kLn10 * gsn[c] * (sc.w_tm * ft));
        lds_add(&L.gp[A.rt.g[2][c]][lane], kLn10 * gsh[c] * th);
      }
      g_lin += kLn10 * gl;
      g_linx += kLn10 * gl * (x - A.x_knee);
    }
    // moments: the cursor piece in registers, later pieces of a crossing pass by wave sums
    double gj[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      gj[j] = L.gp[j][lane];
      L.gp[j][lane] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      if (j >= n_spl) break;
      const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
      if (cur < 0) continue;
      const double g = gj[j];
      const int hi = __builtin_amdgcn_readlane(cv, 3 * j + 1);
      double tt = x - readlane_r(rec, 6 * j);
      int pc = cur;
      if (hi != cur) {
        const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
        for (int q = cur + 1; q <= hi; ++q) {
          const double xq = A.bx[row + q];
          if (x >= xq) {
            tt = x - xq;
            pc = q;
          }
        }
      }
      const double u1 = g * tt, u2 = u1 * tt;
      const double v4[4] = {g, u1, u2, u2 * tt};
      if (hi == cur) {
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[j][m] += v4[m];
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[j][m] += pc == cur ? v4[m] : 0.0;
        for (int q = cur + 1; q <= hi; ++q) {
          double sq[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) sq[m] = wave_sum(pc == q ? v4[m] : 0.0);
          if (lane == q) mo_add(mo + ((size_t)j * kMaxKnots + q) * 4, sq);
        }
      }
    }
    // finished pieces: flush the cursor piece and move the cursor
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      if (j >= n_spl) break;
      const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
      const int hi = __builtin_amdgcn_readlane(cv, 3 * j + 1);
      if (cur < 0 || hi == cur) continue;
      double sq[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        sq[m] = wave_sum(acc[j][m]);
        acc[j][m] = 0.0;
      }
      if (lane == cur) mo_add(mo + ((size_t)j * kMaxKnots + cur) * 4, sq);
      load_rec(j, hi, __builtin_amdgcn_readlane(cv, 3 * j + 2));
      cv = lane == 3 * j ? hi : cv;
    }
  }
  // the last pieces
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    if (j >= n_spl) break;
    const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
    if (cur < 0) continue;
    double sq[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) sq[m] = wave_sum(acc[j][m]);
    if (lane == cur) mo_add(mo + ((size_t)j * kMaxKnots + cur) * 4, sq);
  }
  // state results
  const double Ls = wave_sum(lsum);
  if (__ballot(bad) != 0ull || !isfinite(Ls)) st |= LPS_ST_PSD;
  if (lane == 0) {
    logL[s] = st ? -INFINITY : -(Ls + c0[0]);
    if (status_out) status_out[s] = st;
  }
  if (st) {
    zero_outputs();
    return;
  }
  const double Gwo = wave_sum(g_wo), Gwt = wave_sum(g_wt), Glin = wave_sum(g_lin), Glinx = wave_sum(g_linx);
  const double Gfg = wave_sum(g_fg);
  if (lane == 0) {
    const double a_oms = A.params[LPS_P_AOMS * (size_t)A.n_states + s];
    const double a_tm = A.params[LPS_P_ATM * (size_t)A.n_states + s];
    dparams[LPS_P_AOMS * (size_t)A.n_states + s] = 2.0 * a_oms * Gwo;
    dparams[LPS_P_ATM * (size_t)A.n_states + s] = 2.0 * a_tm * Gwt;
    dparams[LPS_P_U * (size_t)A.n_states + s] = Glin;
    dparams[LPS_P_ALPHA * (size_t)A.n_states + s] = Glinx;
    if (n_params > 4) dparams[LPS_P_UFG * (size_t)A.n_states + s] = kLn10 * sc.efg * Gfg;
  }
  wave_lds_sync();
  BackLds& B = *reinterpret_cast<BackLds*>(&L.val[0][0]);
  for (int j = 0; j < n_spl; ++j) {
    int a, n;
    knot_range(off, kcnt, s * n_spl + j, n_knots, a, n);
    if (n == 0) continue;
    double M[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane + 1 < n)
#pragma unroll
      for (int m = 0; m < 4; ++m) M[m] = mo[((size_t)j * kMaxKnots + lane) * 4 + m];
    spline_backward_wave(lane, kx + a, ky + a, n, M, dky + a, dkx + a, B);
  }
}

}  // namespace
}  // namespace lps

using namespace lps::covk;

extern "C" {

lps_status lps_cov_loglike_grad_batch(lps_cov_ctx* c, const lps_states* st, double* logL, double* dparams,
                                      double* dknot_x, double* dknot_y, uint32_t* status, void* stream) {
  LPS_API_RANGE();
  using namespace lps;
  lps_status cs = check_cov_states(c, st);
  if (cs != LPS_OK) return cs;
  const int n = st->n_states;
  if (n == 0) return LPS_OK;
  if (!logL || !dparams) return LPS_E_NULL;
  if (c->n_spl > 0 && (!dknot_x || !dknot_y)) return LPS_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_cov_coeffs(c, st, s);
  if (e != hipSuccess) return device_status(e);
  const CovArgs A = cov_args(c, st);
  auto kern = c->n_spl <= 4 ? k_cov_grad<4> : (c->n_spl <= 7 ? k_cov_grad<7> : k_cov_grad<kCovMaxSpl>);
  hipLaunchKernelGGL(kern, dim3((n + 3) / 4), dim3(256), 0, s, A, c->gmo, st->knot_off, st->knot_cnt, st->n_knots, st->knot_x,
                     st->knot_y, c->n_params, c->c0, logL, dparams, dknot_x, dknot_y, status);
  return device_status(hipGetLastError());
}

}  // extern "C"
