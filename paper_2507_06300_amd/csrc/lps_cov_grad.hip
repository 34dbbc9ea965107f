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
// turns them into knot derivatives.  A lane keeps the moments of the piece
// under the cursor in registers; a chunk that crosses a knot adds the bins
// beyond it piece by piece (wave sums) and the finished piece's moments go to
// the state's moment table in global memory, where lane q alone reads and
// writes the entries of piece q (so no fence is needed between the lanes).
// ---------------------------------------------------------------------------
// Per wave; the kCovB bins of a lane go through each phase together (their
// arithmetic is independent, which gives the scheduler two chains to
// interleave).  Slots kSlotOne and kSlotZero of gp collect the derivatives
// of terms that no spline perturbs; they are never read.  val, gp, t and pc
// are lane-private columns; rec is written by lane 0 and read by every lane.
struct CovGradLds {
  double val[kCovB][kSlots][kWave];      // slot values of the lane's bins
  double gp[kCovB][kSlots][kWave];       // dlogL / d(slot argument)
  double t[kCovB][kCovMaxSpl][kWave];    // x - start of the bin's piece
  int pc[kCovB][kCovMaxSpl][kWave];      // the bin's piece
  PieceRec rec[kCovMaxSpl];              // the piece under each spline's cursor
};
static_assert(sizeof(BackLds) <= sizeof(double) * kCovB * kSlots * kWave, "backward LDS aliases val");

struct RegRow {
  double v[kCovRows];
  __device__ double operator()(int r) const { return v[r]; }
};

__device__ inline void mo_add(double* __restrict__ m, const double (&v)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) m[i] += v[i];
}

__global__ __launch_bounds__(256) void k_cov_grad(CovArgs A, double* __restrict__ mo_ws,
                                                  const int32_t* __restrict__ off, const int32_t* __restrict__ kcnt, int64_t n_knots,
                                                  const double* __restrict__ kx, const double* __restrict__ ky,
                                                  int n_params, const double* __restrict__ c0,
                                                  double* __restrict__ logL, double* __restrict__ dparams,
                                                  double* __restrict__ dkx, double* __restrict__ dky,
                                                  uint32_t* __restrict__ status_out) {
  __shared__ CovGradLds lds[4];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = (int)(threadIdx.x / kWave);
  const int s = uniform(blockIdx.x * 4 + w);
  if (s >= A.n_states) return;
  CovGradLds& L = lds[w];
  const size_t kp = (size_t)A.k_pad;
  const int n_spl = A.n_spl;
  uint32_t st = A.status[s];
  auto zero_outputs = [&]() {
    if (lane < n_params) dparams[lane * (size_t)A.n_states + s] = 0.0;
    for (int j = 0; j < n_spl; ++j) {
      int a, cn;
      knot_range(off, kcnt, s * n_spl + j, n_knots, a, cn);
      if (a < 0) continue;
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
  // cursors at the first bin.  The cursor state is uniform and lives in
  // scalar registers (the spline loops are unrolled): cur = piece under the
  // cursor (-1: disabled spline), hi = last piece that this chunk reaches,
  // npc = pieces, xn = start of the piece after the cursor.
  const double x_first = A.tab[kRx * kp];
  int cur[kCovMaxSpl], hi[kCovMaxSpl], npc[kCovMaxSpl];
  double xn[kCovMaxSpl];
#pragma unroll
  for (int j = 0; j < kCovMaxSpl; ++j) {
    cur[j] = -1;
    hi[j] = -1;
    npc[j] = 0;
    xn[j] = INFINITY;
    if (j >= n_spl) continue;
    const int np = uniform(A.npc[(size_t)s * kCovMaxSpl + j]);
    npc[j] = np;
    if (np > 0) {
      const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
      const double bl = lane < np ? A.bx[row + lane] : INFINITY;
      cur[j] = uniform(max(__popcll(__ballot(bl <= x_first)) - 1, 0));
      hi[j] = cur[j];
      const PieceRec pr = load_piece(A, row, cur[j], np);
      xn[j] = pr.xn;
      if (lane == 0) L.rec[j] = pr;
    }
  }
#pragma unroll
  for (int bb = 0; bb < kCovB; ++bb) {
    L.val[bb][kSlotOne][lane] = 1.0;
    L.val[bb][kSlotZero][lane] = 0.0;
  }
  wave_lds_sync();
  const StateScal sc = state_scalars(A.params, A.n_states, s, A.has_fg);
  double acc[kCovMaxSpl][4];
#pragma unroll
  for (int j = 0; j < kCovMaxSpl; ++j)
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[j][m] = 0.0;
  double lsum = 0.0, g_wo = 0.0, g_wt = 0.0, g_lin = 0.0, g_linx = 0.0, g_fg = 0.0;
  bool bad = false;
  for (int ch = 0; ch < A.n_chunks; ++ch) {
    const int kb = ch * kCovChunk;
    const double* tb = A.tab + kb + lane;
    const double xl = A.tab[kRx * kp + kb + kCovChunk - 1];
    // pieces that start inside this chunk
#pragma unroll
    for (int j = 0; j < kCovMaxSpl; ++j) {
      if (j >= n_spl) break;
      if (cur[j] < 0 || !(xl >= xn[j])) continue;
      const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
      int h = cur[j] + 1;
      while (h + 1 < npc[j] && A.bx[row + h + 1] <= xl) ++h;
      hi[j] = h;
    }
    // the bins' table entries, loaded ahead of the LDS exchanges below (whose
    // fences would otherwise hold every load back until the spline work is done)
    RegRow row[kCovB];
    double x[kCovB], lin[kCovB];
#pragma unroll
    for (int bb = 0; bb < kCovB; ++bb) {
#pragma unroll
      for (int r = 0; r < kCovRows; ++r) row[bb].v[r] = tb[bb * kWave + r * kp];
      x[bb] = row[bb](kRx);
      lin[bb] = sc.u + sc.alpha * (x[bb] - A.x_knee);
    }
    // forward: slot values, the bin's piece and abscissa offset per spline
#pragma unroll
    for (int j = 0; j < kCovMaxSpl; ++j) {
      if (j >= n_spl) break;
      const int cur_j = cur[j];
      double pv[kCovB], tt[kCovB];
      int pc[kCovB];
      if (cur_j >= 0) {
        PieceRec pr[kCovB];
#pragma unroll
        for (int bb = 0; bb < kCovB; ++bb) {
          pr[bb] = L.rec[j];
          pc[bb] = cur_j;
        }
        if (hi[j] != cur_j) {
          const size_t rw = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
          for (int q = cur_j + 1; q <= hi[j]; ++q) {
            const PieceRec nq = load_piece(A, rw, q, npc[j]);
#pragma unroll
            for (int bb = 0; bb < kCovB; ++bb)
              if (x[bb] >= nq.x0) {
                pr[bb] = nq;
                pc[bb] = q;
              }
          }
        }
#pragma unroll
        for (int bb = 0; bb < kCovB; ++bb) {
          tt[bb] = x[bb] - pr[bb].x0;
          pv[bb] = pr[bb].a0 + tt[bb] * (pr[bb].a1 + tt[bb] * (pr[bb].a2 + tt[bb] * pr[bb].a3));
        }
      } else {
#pragma unroll
        for (int bb = 0; bb < kCovB; ++bb) {
          pv[bb] = 0.0;
          tt[bb] = 0.0;
          pc[bb] = cur_j;
        }
      }
#pragma unroll
      for (int bb = 0; bb < kCovB; ++bb) {
        L.val[bb][j][lane] = slot_value(pv[bb], j, A.rt, lin[bb]);
        L.t[bb][j][lane] = tt[bb];
        L.pc[bb][j][lane] = pc[bb];
        L.gp[bb][j][lane] = 0.0;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int bb = 0; bb < kCovB; ++bb) {
      const LdsVal val{&L.val[bb][0][lane]};
      const RegRow& rw = row[bb];
      CovPoint p;
      cov_point(val, A.rt, sc, A.x_knee, rw, p);
      const CovAdj cj = cov_adj(p);
      lsum += cov_term_adj(cj, p, rw, bad);
      // adjoint of the bin
      const double nu = rw(kRnu);
      const double n0 = p.sn[0], n1 = p.sn[1], n2 = p.sn[2];
      const double c01 = p.r01 * cj.s01, c02 = p.r02 * cj.s02, c12 = p.r12 * cj.s12;
      const double id = rcp_d(cj.det);
      const double ci[3][3] = {{cj.a00 * id, cj.a01 * id, cj.a02 * id},
                               {cj.a01 * id, cj.a11 * id, cj.a12 * id},
                               {cj.a02 * id, cj.a12 * id, cj.a22 * id}};
      const double P[3][3] = {{rw(kRP + 0), rw(kRP + 3), rw(kRP + 4)},
                              {rw(kRP + 3), rw(kRP + 1), rw(kRP + 5)},
                              {rw(kRP + 4), rw(kRP + 5), rw(kRP + 2)}};
      double X[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) X[a][c] = ci[a][0] * P[0][c] + ci[a][1] * P[1][c] + ci[a][2] * P[2][c];
      auto Gm = [&](int a, int c) { return ci[a][c] - (X[a][0] * ci[0][c] + X[a][1] * ci[1][c] + X[a][2] * ci[2][c]); };
      // dlogL / dC (pairs counted once)
      const double gC00 = -nu * Gm(0, 0), gC11 = -nu * Gm(1, 1), gC22 = -nu * Gm(2, 2);
      const double gC01 = -2.0 * nu * Gm(0, 1), gC02 = -2.0 * nu * Gm(0, 2), gC12 = -2.0 * nu * Gm(1, 2);
      const double gsh[3] = {gC00, gC11, gC22};
      const double gsn[3] = {gC00 + (gC01 * c01 + gC02 * c02) * (0.5 * rcp_d(n0)),
                             gC11 + (gC01 * c01 + gC12 * c12) * (0.5 * rcp_d(n1)),
                             gC22 + (gC02 * c02 + gC12 * c12) * (0.5 * rcp_d(n2))};
      double gr01 = gC01 * cj.s01, gr02 = gC02 * cj.s02;
      const double gr12 = gC12 * cj.s12;
      const double pp = val(A.rt.gc[2]);
      const double S = sqrt_d((1.0 - p.r01 * p.r01) * (1.0 - p.r02 * p.r02));
      const double gpp = gr12 * S;
      // S = 0 only where a correlation is exactly +-1; S is then 0 whatever the
      // other correlation, so its derivative terms drop out
      const double iS = S > 0.0 ? rcp_d(S) : 0.0;
      gr01 += gr12 * (p.r02 - pp * p.r01 * (1.0 - p.r02 * p.r02) * iS);
      gr02 += gr12 * (p.r01 - pp * p.r02 * (1.0 - p.r01 * p.r01) * iS);
      const double gq[3] = {gr01 * (1.0 - p.r01 * p.r01), gr02 * (1.0 - p.r02 * p.r02), gpp * (1.0 - pp * pp)};
      // slot derivatives (a slot may serve several terms: accumulate in LDS)
      const double oms[3] = {rw(kRomsAE), rw(kRomsAE), rw(kRomsT)};
      const double tm[3] = {rw(kRtmAE), rw(kRtmAE), rw(kRtmT)};
      const double hf = background_factor(A.rt, sc, x[bb], A.x_knee);
      double gl = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double fo = val(A.rt.g[0][c]), ft = val(A.rt.g[1][c]), fh = val(A.rt.g[2][c]);
        const double to = sc.w_oms * oms[c] * fo, tt2 = sc.w_tm * tm[c] * ft, th = rw(kRsg + c) * hf * fh;
        g_wo += gsn[c] * oms[c] * fo;
        g_wt += gsn[c] * tm[c] * ft;
        g_fg += gsh[c] * rw(kRfg + c) * sc.efg;
        gl += gsh[c] * th;
        L.gp[bb][A.rt.g[0][c]][lane] += kLn10 * gsn[c] * to;
        L.gp[bb][A.rt.g[1][c]][lane] += kLn10 * gsn[c] * tt2;
        L.gp[bb][A.rt.g[2][c]][lane] += kLn10 * gsh[c] * th;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) L.gp[bb][A.rt.gc[i]][lane] += gq[i];
      g_lin += kLn10 * gl;
      g_linx += kLn10 * gl * (x[bb] - A.x_knee);
    }
    wave_lds_sync();
    // moments: the cursor piece in registers, later pieces of a crossing chunk by wave sums
#pragma unroll
    for (int j = 0; j < kCovMaxSpl; ++j) {
      if (j >= n_spl) break;
      if (cur[j] < 0) continue;
      double v4[kCovB][4];
      int pc[kCovB];
#pragma unroll
      for (int bb = 0; bb < kCovB; ++bb) {
        const double g = L.gp[bb][j][lane], tt = L.t[bb][j][lane];
        pc[bb] = L.pc[bb][j][lane];
        const double u1 = g * tt, u2 = u1 * tt;
        v4[bb][0] = g;
        v4[bb][1] = u1;
        v4[bb][2] = u2;
        v4[bb][3] = u2 * tt;
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[j][m] += pc[bb] == cur[j] ? v4[bb][m] : 0.0;
      }
      for (int q = cur[j] + 1; q <= hi[j]; ++q) {
        double sq[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          double v = 0.0;
#pragma unroll
          for (int bb = 0; bb < kCovB; ++bb) v += pc[bb] == q ? v4[bb][m] : 0.0;
          sq[m] = wave_sum(v);
        }
        if (lane == q) mo_add(mo + ((size_t)j * kMaxKnots + q) * 4, sq);
      }
    }
    wave_lds_sync();
    // finished pieces: flush the cursor piece and move the cursor
#pragma unroll
    for (int j = 0; j < kCovMaxSpl; ++j) {
      if (j >= n_spl) break;
      if (cur[j] < 0 || hi[j] == cur[j]) continue;
      double sq[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        sq[m] = wave_sum(acc[j][m]);
        acc[j][m] = 0.0;
      }
      const PieceRec pr = load_piece(A, ((size_t)s * kCovMaxSpl + j) * kMaxKnots, hi[j], npc[j]);
      if (lane == cur[j]) mo_add(mo + ((size_t)j * kMaxKnots + cur[j]) * 4, sq);
      if (lane == 0) L.rec[j] = pr;
      cur[j] = hi[j];
      xn[j] = pr.xn;
    }
    wave_lds_sync();
  }
  // the last pieces
#pragma unroll
  for (int j = 0; j < kCovMaxSpl; ++j) {
    if (j >= n_spl) break;
    if (cur[j] < 0) continue;
    double sq[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) sq[m] = wave_sum(acc[j][m]);
    if (lane == cur[j]) mo_add(mo + ((size_t)j * kMaxKnots + cur[j]) * 4, sq);
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
    if (n_params > 4) dparams[LPS_P_UFG * (size_t)A.n_states + s] = kLn10 * Gfg;
  }
  wave_lds_sync();
  BackLds& B = *reinterpret_cast<BackLds*>(&L.val[0][0][0]);
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
  hipLaunchKernelGGL(k_cov_grad, dim3((n + 3) / 4), dim3(256), 0, s, A, c->gmo, st->knot_off, st->knot_cnt, st->n_knots, st->knot_x,
                     st->knot_y, c->n_params, c->c0, logL, dparams, dknot_x, dknot_y, status);
  return device_status(hipGetLastError());
}

}  // extern "C"
