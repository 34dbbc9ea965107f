// Full-covariance likelihood: a dense, real symmetric 3x3 covariance per bin.
//
// The paper keeps the A/E/T noise covariance diagonal and names the dense
// treatment, with three more flexible terms for the off-diagonal entries, as
// the natural extension (Sec. "Power spectral density breakdown" and the
// outlook of the conclusions); it does not print a construction.  The
// library implements the one documented in lps.h:
//
//   Sn_c, Sh_c   the diagonal model of the rest of the library (templates,
//                amplitudes, routed splines), per channel c = A, E, T;
//   r_AE = tanh Q0, r_AT = tanh Q1, r_ET = r_AE r_AT + tanh Q2 sqrt((1 - r_AE^2)(1 - r_AT^2))
//                (a partial-correlation vine: positive definite for any Q);
//   C_cc = Sn_c + Sh_c,  C_ab = r_ab sqrt(Sn_a Sn_b);
//   logL = - sum_k N_k ( tr(C_k^-1 P_k) + ln det C_k ).
//
// Numerics (FP64 throughout).  The per-bin table is divided by a reference
// level sigma_k (the A-channel noise at the library's reference amplitudes), so
// every entry is O(1) whatever the units; ln det C gains 3 ln sigma_k, whose
// N-weighted sum is a constant added once per state.  In those units the
// kernel forms det C and the cofactors directly from Sn, C_cc and the
// correlations,
//   det C  = C_AA C_EE C_TT + 2 r_AE r_AT r_ET Sn_A Sn_E Sn_T
//            - C_AA r_ET^2 Sn_E Sn_T - C_EE r_AT^2 Sn_A Sn_T - C_TT r_AE^2 Sn_A Sn_E,
//   adj_AE = sqrt(Sn_A Sn_E) (r_AT r_ET Sn_T - r_AE C_TT)   (and cyclically),
// so that only the three off-diagonal cofactors need a square root;
// tr(C^-1 P) = sum_ab adj_ab P_ab / det C.  Positive definiteness is
// Sylvester's criterion (C_AA > 0, C_AA C_EE - r_AE^2 Sn_A Sn_E > 0,
// det C > 0).  Powers of ten and tanh use exp2 by range reduction to
// [-1/2, 1/2] and a degree-11 near-minimax polynomial for e^t (within 0.15
// ulp before rounding), scaled by ldexp.
//
// Definitions shared by the likelihood (lps_cov.hip) and its adjoint
// (lps_cov_grad.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lps.h"
#include "lps_internal.hpp"
#include "lps_math64.hpp"

namespace lps {
namespace covk {

constexpr int kCovMaxSpl = LPS_COV_MAX_SPLINES;
constexpr int kCovB = 2;                    // bins per lane in one chunk
constexpr int kCovChunk = kWave * kCovB;    // 128 bins
constexpr int kCovMaxTile = 8;              // states per wave
constexpr int kCovGroups = 64;              // chunk groups per dataset (fixed by K alone)

// Rows of the per-bin table; every PSD-valued row is divided by sigma_k.  The
// table is stored in blocks of 64 consecutive bins, each holding its rows one
// after the other ([k_pad / 64][kCovRows][64], tab_index), so that a lane's
// entries of one bin lie at fixed offsets from a single address.
enum : int {
  kRx = 0,       // log10 f
  kRnu = 1,      // N_k (0 for padding)
  kRomsAE = 2,   // OMS transfer x single-link PSD per unit A_OMS^2, channels A and E
  kRomsT = 3,    //   channel T
  kRtmAE = 4,    // TM, per unit A_TM^2
  kRtmT = 5,
  kRsg = 6,      // R_c 3 (H0/h)^2 / (4 pi^2 f^3), c = A, E, T
  kRP = 9,       // data rows AA, EE, TT, AE, AT, ET
  kRfg = 15,     // foreground shape, c = A, E, T (0 without a foreground)
  kCovRows = 18
};


// Per-slot values of one bin: 10^P_j for a slot feeding a diagonal term,
// tanh P_j for a correlation slot; two fixed entries stand for "no spline".
constexpr int kSlotOne = kCovMaxSpl;        // 1 (an unperturbed diagonal term)
constexpr int kSlotZero = kCovMaxSpl + 1;   // 0 (zero correlation)
constexpr int kSlots = kCovMaxSpl + 2;

struct CovRoute {
  uint8_t g[3][3];      // [OMS, TM, SGWB][channel] slot of the factor 10^P (kSlotOne: none)
  uint8_t gc[3];        // slots of tanh Q0, tanh Q1, tanh Q2 (kSlotZero: none)
  uint32_t diag_mask;   // bit j: slot j feeds a diagonal term (value 10^P_j)
  uint32_t corr_mask;   // bit j: slot j is a correlation term (value tanh P_j)
  int32_t sg_slot;      // slot carrying the background in all channels and nothing else, or -1
};

}  // namespace covk
}  // namespace lps

struct lps_cov_ctx {
  int device;
  int32_t n_bins, k_pad, n_chunks, chunks_per_group, n_groups;
  int32_t n_spl, n_params, k_max, max_states, has_fg;
  lps::covk::CovRoute rt;
  double x_knee, x_first, x_last;
  double* tab;          // [k_pad / 64][kCovRows][64] (tab_index)
  double* bx;           // [max_states][kCovMaxSpl][kMaxKnots] piece start abscissae
  double* coef;         // [max_states][kCovMaxSpl][kMaxKnots][4]
  int32_t* npc;         // [max_states][kCovMaxSpl] pieces (0: disabled or invalid state)
  uint32_t* status;     // [max_states]
  double* partial;      // [max_states][n_groups]
  double* sigma;        // [K] reference level sigma_k of the scaled table
  double* c0;           // [1] 3 sum_k N_k ln sigma_k
  double* gmo;          // [max_states][kCovMaxSpl][kMaxKnots][4] piece moments of the adjoint
};

namespace lps {
namespace covk {

struct StateScal {
  double w_oms, w_tm, u, alpha, efg;
};

__device__ inline StateScal state_scalars(const double* __restrict__ params, int n_states, int s, int has_fg) {
  StateScal r;
  const double a_oms = params[LPS_P_AOMS * (size_t)n_states + s];
  const double a_tm = params[LPS_P_ATM * (size_t)n_states + s];
  r.w_oms = a_oms * a_oms;
  r.w_tm = a_tm * a_tm;
  r.u = params[LPS_P_U * (size_t)n_states + s];
  r.alpha = params[LPS_P_ALPHA * (size_t)n_states + s];
  r.efg = has_fg ? exp10(params[LPS_P_UFG * (size_t)n_states + s]) : 0.0;
  return r;
}

// kSgpr: polynomial coefficients in scalar registers (see fma3).
template <bool kSgpr = false>
__device__ inline double exp10_d(double y) { return exp2_d<kSgpr>(y * kLog2_10); }

// tanh q = sign(q) (1 - e) / (1 + e), e = exp(-2|q|) in (0, 1]
template <bool kSgpr = false>
__device__ inline double tanh_d(double q) {
  const double e = exp2_d<kSgpr>(-2.0 * kLog2e * fabs(q));
  const double den = 1.0 + e, num = 1.0 - e;
  const double r = rcp_d(den);
  const double t = num * r;
  return copysign(fma(fma(-den, t, num), r, t), q);
}

struct CovPoint {
  double d[3];    // C_cc (scaled)
  double sn[3];   // Sn_c (scaled)
  double r01, r02, r12;
  double vs;      // the vine's sqrt((1 - r_AE^2)(1 - r_AT^2))
};

// The value of slot j at one bin: 10^P, tanh P, or P itself for an unused slot.
// lin = u + alpha (x - log10 f_knee) is added to the exponent of the slot that
// carries the background in every channel (rt.sg_slot), which then holds the
// whole background factor 10^(u + alpha (x - x_knee) + P).
template <bool kSgpr = false>
__device__ inline double slot_value(double pv, int j, const CovRoute& rt, double lin) {
  if (j == rt.sg_slot) return exp10_d<kSgpr>(pv + lin);
  if ((rt.diag_mask >> j) & 1u) return exp10_d<kSgpr>(pv);
  if ((rt.corr_mask >> j) & 1u) return tanh_d<kSgpr>(pv);
  return pv;
}

// The power-law factor 10^(u + alpha (x - x_knee)) of the background, or 1
// where the slot rt.sg_slot already carries it.
template <bool kSgpr = false>
__device__ inline double background_factor(const CovRoute& rt, const StateScal& sc, double x, double x_knee) {
  return rt.sg_slot >= 0 ? 1.0 : exp10_d<kSgpr>(sc.u + sc.alpha * (x - x_knee));
}

// The model at one bin from the slot values V (read through `val(slot)`), the
// background factor hf and the bin's table entries (read through `row(r)`).
template <typename Val, typename Row>
__device__ inline void cov_point_h(const Val& val, const CovRoute& rt, const StateScal& sc, double hf, const Row& row,
                                   CovPoint& o) {
  const double oms[3] = {row(kRomsAE), row(kRomsAE), row(kRomsT)};
  const double tm[3] = {row(kRtmAE), row(kRtmAE), row(kRtmT)};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double sn = sc.w_oms * oms[c] * val(rt.g[0][c]) + sc.w_tm * tm[c] * val(rt.g[1][c]);
    const double sh = row(kRsg + c) * hf * val(rt.g[2][c]) + row(kRfg + c) * sc.efg;
    o.d[c] = sn + sh;
    o.sn[c] = sn;
  }
  o.r01 = val(rt.gc[0]);
  o.r02 = val(rt.gc[1]);
  o.vs = sqrt_d((1.0 - o.r01 * o.r01) * (1.0 - o.r02 * o.r02));
  o.r12 = o.r01 * o.r02 + val(rt.gc[2]) * o.vs;
}

template <typename Val, typename Row>
__device__ inline void cov_point(const Val& val, const CovRoute& rt, const StateScal& sc, double x_knee, const Row& row,
                                 CovPoint& o) {
  cov_point_h(val, rt, sc, background_factor(rt, sc, row(kRx), x_knee), row, o);
}

// Cofactors adj_ab and det C at one bin in scaled units (see the file
// comment), with s_ab = sqrt(Sn_a Sn_b) for the pairs AE, AT, ET.
struct CovAdj {
  double a00, a11, a22, a01, a02, a12, det, s01, s02, s12;
};

// The same from given s_ab.
__device__ inline CovAdj cov_adj_s(const CovPoint& p, double s01, double s02, double s12) {
  const double d0 = p.d[0], d1 = p.d[1], d2 = p.d[2];
  const double n0 = p.sn[0], n1 = p.sn[1], n2 = p.sn[2];
  const double q01 = p.r01 * p.r01 * (n0 * n1);
  const double q02 = p.r02 * p.r02 * (n0 * n2);
  const double q12 = p.r12 * p.r12 * (n1 * n2);
  CovAdj c;
  c.a00 = d1 * d2 - q12;
  c.a11 = d0 * d2 - q02;
  c.a22 = d0 * d1 - q01;
  c.det = d0 * c.a00 - d1 * q02 - d2 * q01 + 2.0 * (p.r01 * p.r02 * p.r12) * (n0 * n1 * n2);
  c.s01 = s01;
  c.s02 = s02;
  c.s12 = s12;
  c.a01 = c.s01 * (p.r02 * p.r12 * n2 - p.r01 * d2);
  c.a02 = c.s02 * (p.r01 * p.r12 * n1 - p.r02 * d1);
  c.a12 = c.s12 * (p.r01 * p.r02 * n0 - p.r12 * d0);
  return c;
}

__device__ inline CovAdj cov_adj(const CovPoint& p) {
  return cov_adj_s(p, sqrt_d(p.sn[0] * p.sn[1]), sqrt_d(p.sn[0] * p.sn[2]), sqrt_d(p.sn[1] * p.sn[2]));
}

// det C tr(C^-1 P) = sum_ab adj_ab P_ab from the cofactors.
template <typename Row>
__device__ inline double cov_trace_num(const CovAdj& c, const Row& row) {
  return c.a00 * row(kRP + 0) + c.a11 * row(kRP + 1) + c.a22 * row(kRP + 2) +
         2.0 * (c.a01 * row(kRP + 3) + c.a02 * row(kRP + 4) + c.a12 * row(kRP + 5));
}

// N_k (tr + ln det C) at one bin in scaled units, given tr = tr(C^-1 P);
// `bad` is set where C is not positive definite or the term is not finite.
template <bool kSgpr = false, typename Row>
__device__ inline double cov_term_tr(const CovAdj& c, const CovPoint& p, const Row& row, double tr, bool& bad) {
  const double ld = log_d<kSgpr>(c.det);
  const bool ok = p.d[0] > 0.0 && c.a22 > 0.0 && c.det > 0.0 && isfinite(tr) && isfinite(ld);
  bad = bad || !ok;
  return row(kRnu) * (tr + ld);
}

template <bool kSgpr = false, typename Row>
__device__ inline double cov_term_adj(const CovAdj& c, const CovPoint& p, const Row& row, bool& bad) {
  return cov_term_tr<kSgpr>(c, p, row, cov_trace_num(c, row) / c.det, bad);
}

template <typename Row>
__device__ inline double cov_term(const CovPoint& p, const Row& row, bool& bad) {
  return cov_term_adj(cov_adj(p), p, row, bad);
}

struct CovArgs {
  const double* tab;
  int k_pad, n_chunks, chunks_per_group, n_groups;
  int n_states, tile, n_tiles, n_spl, has_fg;
  CovRoute rt;
  double x_knee;
  const double* params;
  uint32_t* status;
  const double* bx;
  const double* coef;
  const int32_t* npc;
  double* partial;
};

struct LdsVal {
  const double* p;   // &lval[wave][0][lane]
  __device__ double operator()(int j) const { return p[j * kWave]; }
};

constexpr int kCovBlock = kCovRows * kWave;   // doubles per 64-bin block of the table

// Position of row r, bin k in the blocked table.
__host__ __device__ inline size_t tab_index(int r, size_t k) {
  return (k / kWave) * kCovBlock + (size_t)r * kWave + (k % kWave);
}

// The entries of one bin: p = &tab[tab_index(0, k)], rows kWave apart.
struct TabRow {
  const double* __restrict__ p;
  __device__ double operator()(int r) const { return p[r * kWave]; }
};

// The piece of spline (s, j) that holds a bin and the start of the next one.
struct PieceRec {
  double x0, a0, a1, a2, a3, xn;
};

__device__ inline PieceRec load_piece(const CovArgs& A, size_t row, int q, int np) {
  PieceRec p;
  p.x0 = A.bx[row + q];
  const double* c = A.coef + (row + q) * 4;
  p.a0 = c[0];
  p.a1 = c[1];
  p.a2 = c[2];
  p.a3 = c[3];
  p.xn = q + 1 < np ? A.bx[row + q + 1] : INFINITY;
  return p;
}

// Host helpers (lps_cov.hip).
lps_status check_cov_states(const lps_cov_ctx* ctx, const lps_states* st);
// Validates every state and stores its spline pieces (k_cov_coeffs) on `s`.
hipError_t launch_cov_coeffs(lps_cov_ctx* c, const lps_states* st, hipStream_t s);
CovArgs cov_args(const lps_cov_ctx* c, const lps_states* st);

}  // namespace covk
}  // namespace lps
