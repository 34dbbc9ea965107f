// Full-covariance likelihood: a dense, real symmetric 3x3 covariance per bin.
//
// The paper keeps the A/E/T noise covariance diagonal and names the dense
// treatment, with three more flexible terms for the off-diagonal entries, as
// the natural extension (Sec. "Power spectral density breakdown" and the
// outlook of the conclusions); it does not print a construction.  This file
// implements the one documented in lps.h:
//
//   Sn_c, Sh_c   the diagonal model of the rest of the library (templates,
//                amplitudes, routed splines), per channel c = A, E, T;
//   r_AE = tanh Q0, r_AT = tanh Q1, r_ET = r_AE r_AT + tanh Q2 sqrt((1 - r_AE^2)(1 - r_AT^2))
//                (a partial-correlation vine: positive definite for any Q);
//   C_cc = Sn_c + Sh_c,  C_ab = r_ab sqrt(Sn_a Sn_b);
//   logL = - sum_k N_k ( tr(C_k^-1 P_k) + ln det C_k ).
//
// Per bin the kernel works in the correlation form C = Delta Ct Delta with
// Delta = diag(sqrt C_cc): Ct has a unit diagonal and off-diagonal entries
// rho_ab = r_ab sqrt(Sn_a / C_aa) sqrt(Sn_b / C_bb), so its cofactors and
// determinant are O(1) whatever the channel levels; then
//   tr(C^-1 P) = sum_ab adj(Ct)_ab P_ab / (Delta_a Delta_b det Ct),
//   ln det C   = ln(C_AA C_EE C_TT det Ct),
// and positive definiteness is Sylvester's criterion on Ct
// (C_cc > 0, 1 - rho_AE^2 > 0, det Ct > 0).
//
// Work decomposition (FP64 throughout): the coefficient kernel validates
// every state and stores the cubic pieces of its splines (one wave per
// state, one lane per piece).  The evaluation kernel gives each wave one tile
// of states and one group of consecutive 128-bin chunks; it walks the chunks
// and, inside each chunk, the states of its tile, so that the waves of a
// workgroup read the same table rows (held in L1) for many states.  A
// spline's pieces covering a chunk are found with two ballots over the
// piece abscissae (lane = piece), usually one piece for the whole chunk, in
// which case its coefficients are uniform loads.  Each wave keeps the sum of
// state i of its tile in lane i; partial sums per (state, chunk group) are
// added in a fixed order by the finalize kernel, so results do not depend on
// the batch size.
#include <math.h>
#include <string.h>

#include <vector>

#include "lps_internal.hpp"
#include "lps_spline.hpp"
#include "lps_validate.hpp"

namespace lps {
namespace {

constexpr int kCovMaxSpl = LPS_COV_MAX_SPLINES;
constexpr int kCovB = 2;                    // bins per lane in one chunk
constexpr int kCovChunk = kWave * kCovB;    // 128 bins
constexpr int kCovMaxTile = 16;             // states per wave
constexpr int kCovGroups = 64;              // chunk groups per dataset (fixed by K alone)

// Rows of the per-bin table [kCovRows][k_pad].
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

struct CovRoute {
  int8_t r[3][3];   // [OMS, TM, SGWB][channel] spline slot or -1
  int8_t corr[3];   // slots of Q0, Q1, Q2 or -1
};

}  // namespace
}  // namespace lps

struct lps_cov_ctx {
  int device;
  int32_t n_bins, k_pad, n_chunks, chunks_per_group, n_groups;
  int32_t n_spl, n_params, k_max, max_states, has_fg;
  lps::CovRoute rt;
  uint32_t diag_mask;   // bit j: spline slot j feeds a diagonal term
  double x_knee, x_first, x_last;
  double* tab;          // [kCovRows][k_pad]
  double* bx;           // [max_states][kCovMaxSpl][kMaxKnots] piece start abscissae
  double* coef;         // [max_states][kCovMaxSpl][kMaxKnots][4]
  int32_t* npc;         // [max_states][kCovMaxSpl] pieces (0: disabled or invalid state)
  uint32_t* status;     // [max_states]
  double* partial;      // [max_states][n_groups]
};

namespace lps {
namespace {

__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ void k_cov_table(int K, int k_pad, const double* __restrict__ f, const double* __restrict__ nk,
                            const double* __restrict__ P, const double* __restrict__ R,
                            const double* __restrict__ Rfg, double L, double* __restrict__ tab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k_pad) return;
  // padding repeats the last bin with N = 0 and no data: it adds exactly 0
  const int kk = k < K ? k : K - 1;
  const double fk = f[kk];
  double oms_ae, oms_t, tm_ae, tm_t, h;
  unit_templates(fk, L, oms_ae, oms_t, tm_ae, tm_t, h);
  double row[kCovRows];
  row[kRx] = log10(fk);
  row[kRnu] = k < K ? nk[kk] : 0.0;
  row[kRomsAE] = oms_ae;
  row[kRomsT] = oms_t;
  row[kRtmAE] = tm_ae;
  row[kRtmT] = tm_t;
  for (int c = 0; c < 3; ++c) {
    row[kRsg + c] = R[c * (size_t)K + kk] * h;
    row[kRfg + c] = Rfg ? Rfg[c * (size_t)K + kk] : 0.0;
  }
  for (int i = 0; i < 6; ++i) row[kRP + i] = k < K ? P[i * (size_t)K + kk] : 0.0;
  for (int r = 0; r < kCovRows; ++r) tab[r * (size_t)k_pad + k] = row[r];
}

// One wave per state: validation (every spline slot), then one lane per piece.
__global__ __launch_bounds__(256) void k_cov_coeffs(int n_states, int n_spl, int k_max, int n_params,
                                                    const double* __restrict__ params, const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ kcnt, const double* __restrict__ kx,
                                                    const double* __restrict__ ky, double x_first, double x_last,
                                                    double* __restrict__ bx, double* __restrict__ coef,
                                                    int32_t* __restrict__ npc, uint32_t* __restrict__ status) {
  const int lane = threadIdx.x & (kWave - 1);
  const int s = uniform(blockIdx.x * (blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (s >= n_states) return;
  const uint32_t st =
      validate_state_wave(lane, s, n_states, n_spl, k_max, n_params, params, off, kcnt, kx, ky, x_first, x_last);
  if (lane == 0) status[s] = st;
  for (int j = 0; j < kCovMaxSpl; ++j) {
    int a = 0, n = 0;
    if (j < n_spl && st == 0) knot_range(off, kcnt, s * n_spl + j, a, n);
    const int np = n >= 2 ? n - 1 : 0;
    const size_t row = (size_t)s * kCovMaxSpl + j;
    if (lane == 0) npc[row] = np;
    if (lane < np) {
      double A, B, C, D;
      spline_piece(kx + a, ky + a, n, lane, A, B, C, D);
      bx[row * kMaxKnots + lane] = kx[a + lane];
      double* q = coef + (row * kMaxKnots + lane) * 4;
      q[0] = A;
      q[1] = B;
      q[2] = C;
      q[3] = D;
    }
  }
}

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

struct CovPoint {
  double d[3];   // C_cc
  double h[3];   // sqrt(Sn_c)
  double r01, r02, r12;
};

// The model at one bin from the spline values Pv and the bin's table entries
// (read through `row(r)`).
template <typename Row>
__device__ inline void cov_point(const double (&Pv)[kCovMaxSpl], int n_spl, const CovRoute& rt, uint32_t diag_mask,
                                 const StateScal& sc, double x_knee, const Row& row, CovPoint& o) {
  double fo[3] = {1.0, 1.0, 1.0}, ft[3] = {1.0, 1.0, 1.0}, fh[3] = {1.0, 1.0, 1.0};
  double q[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kCovMaxSpl; ++j) {
    if (j >= n_spl) break;
    if ((diag_mask >> j) & 1u) {
      const double e = exp10(Pv[j]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (rt.r[0][c] == j) fo[c] = e;
        if (rt.r[1][c] == j) ft[c] = e;
        if (rt.r[2][c] == j) fh[c] = e;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (rt.corr[i] == j) q[i] = Pv[j];
  }
  const double hf = exp10(sc.u + sc.alpha * (row(kRx) - x_knee));
  const double oms[3] = {row(kRomsAE), row(kRomsAE), row(kRomsT)};
  const double tm[3] = {row(kRtmAE), row(kRtmAE), row(kRtmT)};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double sn = sc.w_oms * oms[c] * fo[c] + sc.w_tm * tm[c] * ft[c];
    const double sh = row(kRsg + c) * hf * fh[c] + row(kRfg + c) * sc.efg;
    o.d[c] = sn + sh;
    o.h[c] = sqrt(sn);
  }
  o.r01 = tanh(q[0]);
  o.r02 = tanh(q[1]);
  o.r12 = o.r01 * o.r02 + tanh(q[2]) * sqrt((1.0 - o.r01 * o.r01) * (1.0 - o.r02 * o.r02));
}

// N_k (tr(C^-1 P) + ln det C) at one bin; `bad` is set where C is not
// positive definite or the term is not finite.
template <typename Row>
__device__ inline double cov_term(const CovPoint& p, const Row& row, bool& bad) {
  const double s0 = sqrt(p.d[0]), s1 = sqrt(p.d[1]), s2 = sqrt(p.d[2]);
  const double inv = 1.0 / (s0 * s1 * s2);
  const double i0 = inv * s1 * s2, i1 = inv * s0 * s2, i2 = inv * s0 * s1;
  // sqrt(Sn_c / C_cc) by a correctly rounded division: exactly 1 when the
  // channel has no signal, so that a unit correlation gives an exactly
  // singular Ct
  const double g0 = p.h[0] / s0, g1 = p.h[1] / s1, g2 = p.h[2] / s2;
  const double a = p.r01 * g0 * g1, b = p.r02 * g0 * g2, c = p.r12 * g1 * g2;
  const double m22 = 1.0 - a * a;
  const double det = m22 - b * b - c * c + 2.0 * a * b * c;
  const double m00 = 1.0 - c * c, m11 = 1.0 - b * b;
  const double m01 = b * c - a, m02 = a * c - b, m12 = a * b - c;
  const double num = m00 * row(kRP + 0) * (i0 * i0) + m11 * row(kRP + 1) * (i1 * i1) +
                     m22 * row(kRP + 2) * (i2 * i2) +
                     2.0 * (m01 * row(kRP + 3) * (i0 * i1) + m02 * row(kRP + 4) * (i0 * i2) +
                            m12 * row(kRP + 5) * (i1 * i2));
  const double tr = num / det;
  const double ld = log(p.d[0] * p.d[1] * p.d[2] * det);
  const bool ok = p.d[0] > 0.0 && p.d[1] > 0.0 && p.d[2] > 0.0 && m22 > 0.0 && det > 0.0 && isfinite(tr) &&
                  isfinite(ld);
  bad = bad || !ok;
  return row(kRnu) * (tr + ld);
}

struct CovArgs {
  const double* tab;
  int k_pad, n_chunks, chunks_per_group, n_groups;
  int n_states, tile, n_tiles, n_spl, has_fg;
  CovRoute rt;
  uint32_t diag_mask;
  double x_knee;
  const double* params;
  uint32_t* status;
  const double* bx;
  const double* coef;
  const int32_t* npc;
  double* partial;
};

struct TabRow {
  const double* __restrict__ p;
  size_t stride;
  __device__ double operator()(int r) const { return p[r * stride]; }
};

__global__ __launch_bounds__(256) void k_cov_eval(CovArgs A) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = uniform(xcd_block(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (wid >= A.n_tiles * A.n_groups) return;
  const int g = wid / A.n_tiles, t = wid - g * A.n_tiles;
  const int s0 = t * A.tile;
  const int ns = min(A.tile, A.n_states - s0);
  const int c_begin = g * A.chunks_per_group;
  const int c_end = min(A.n_chunks, c_begin + A.chunks_per_group);
  double acc = 0.0;   // lane i: the sum of state s0 + i over this group
  for (int ch = c_begin; ch < c_end; ++ch) {
    const int kb = ch * kCovChunk;
    const double xf = A.tab[kRx * (size_t)A.k_pad + kb];
    const double xl = A.tab[kRx * (size_t)A.k_pad + kb + kCovChunk - 1];
    for (int i = 0; i < ns; ++i) {
      const int s = s0 + i;
      if (A.status[s] != 0u) continue;
      const StateScal sc = state_scalars(A.params, A.n_states, s, A.has_fg);
      // pieces of every spline over this chunk
      int lo[kCovMaxSpl], hi[kCovMaxSpl], np[kCovMaxSpl];
      double bl[kCovMaxSpl];
#pragma unroll
      for (int j = 0; j < kCovMaxSpl; ++j) {
        np[j] = j < A.n_spl ? A.npc[(size_t)s * kCovMaxSpl + j] : 0;
        lo[j] = hi[j] = 0;
        bl[j] = 0.0;
        if (np[j] > 0) {
          const double* br = A.bx + ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
          bl[j] = lane < np[j] ? br[lane] : INFINITY;
          lo[j] = max(__popcll(__ballot(bl[j] <= xf)) - 1, 0);
          hi[j] = max(__popcll(__ballot(bl[j] <= xl)) - 1, 0);
        }
      }
      double v = 0.0;
      bool bad = false;
#pragma unroll
      for (int b = 0; b < kCovB; ++b) {
        const int k = kb + b * kWave + lane;
        const TabRow row{A.tab + k, (size_t)A.k_pad};
        const double x = row(kRx);
        double Pv[kCovMaxSpl];
#pragma unroll
        for (int j = 0; j < kCovMaxSpl; ++j) {
          Pv[j] = 0.0;
          if (np[j] == 0) continue;
          const double* cr = A.coef + ((size_t)s * kCovMaxSpl + j) * kMaxKnots * 4;
          double x0, c0, c1, c2, c3;
          if (lo[j] == hi[j]) {
            x0 = readlane_d(bl[j], lo[j]);
            c0 = cr[lo[j] * 4 + 0];
            c1 = cr[lo[j] * 4 + 1];
            c2 = cr[lo[j] * 4 + 2];
            c3 = cr[lo[j] * 4 + 3];
          } else {
            int pc = lo[j];
            for (int p = lo[j] + 1; p <= hi[j]; ++p)
              if (x >= readlane_d(bl[j], p)) pc = p;
            x0 = __shfl(bl[j], pc, kWave);
            c0 = cr[pc * 4 + 0];
            c1 = cr[pc * 4 + 1];
            c2 = cr[pc * 4 + 2];
            c3 = cr[pc * 4 + 3];
          }
          const double tt = x - x0;
          Pv[j] = c0 + tt * (c1 + tt * (c2 + tt * c3));
        }
        CovPoint p;
        cov_point(Pv, A.n_spl, A.rt, A.diag_mask, sc, A.x_knee, row, p);
        v += cov_term(p, row, bad);
      }
      if (__ballot(bad) != 0ull && lane == 0) atomicOr(&A.status[s], (unsigned)LPS_ST_PSD);
      v = wave_sum(v);
      acc = lane == i ? acc + v : acc;
    }
  }
  if (lane < ns) A.partial[(size_t)(s0 + lane) * A.n_groups + g] = acc;
}

__global__ void k_cov_finalize(int n_states, int n_groups, const double* __restrict__ partial,
                               const uint32_t* __restrict__ status, double* __restrict__ logL,
                               uint32_t* __restrict__ status_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_states) return;
  const uint32_t st = status[s];
  double sum = 0.0;
  for (int g = 0; g < n_groups; ++g) sum += partial[(size_t)s * n_groups + g];
  logL[s] = st ? -INFINITY : -sum;
  if (status_out) status_out[s] = st;
}

// The six unique entries of C for bins [k0, k1) of every state (binary search
// for the piece of each bin).
__global__ void k_cov_build(int n_states, int k0, int n_out, int k_pad, const double* __restrict__ tab, int n_spl,
                            CovRoute rt, uint32_t diag_mask, double x_knee, int has_fg,
                            const double* __restrict__ params, const uint32_t* __restrict__ status,
                            const double* __restrict__ bx, const double* __restrict__ coef,
                            const int32_t* __restrict__ npc, double* __restrict__ C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_states * n_out) return;
  const int s = (int)(i / n_out), q = (int)(i % n_out), k = k0 + q;
  double* out = C + (size_t)s * 6 * n_out + q;
  if (status[s] != 0u) {
    for (int e = 0; e < 6; ++e) out[(size_t)e * n_out] = NAN;
    return;
  }
  const TabRow row{tab + k, (size_t)k_pad};
  const double x = row(kRx);
  double Pv[kCovMaxSpl];
  for (int j = 0; j < kCovMaxSpl; ++j) {
    Pv[j] = 0.0;
    const int n = j < n_spl ? npc[(size_t)s * kCovMaxSpl + j] : 0;
    if (n == 0) continue;
    const double* br = bx + ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
    int lo = 0, hi = n - 1;   // last piece whose start is <= x, clamped to [0, n-1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (br[mid] <= x) lo = mid;
      else hi = mid - 1;
    }
    const double* cr = coef + (((size_t)s * kCovMaxSpl + j) * kMaxKnots + lo) * 4;
    const double tt = x - br[lo];
    Pv[j] = cr[0] + tt * (cr[1] + tt * (cr[2] + tt * cr[3]));
  }
  const StateScal sc = state_scalars(params, n_states, s, has_fg);
  CovPoint p;
  cov_point(Pv, n_spl, rt, diag_mask, sc, x_knee, row, p);
  const double r[3] = {p.r01, p.r02, p.r12};
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int c = 0; c < 3; ++c) out[(size_t)c * n_out] = p.d[c];
  for (int e = 0; e < 3; ++e) out[(size_t)(3 + e) * n_out] = p.h[pa[e]] * r[e] * p.h[pb[e]];
}

lps_status check_cov_states(const lps_cov_ctx* ctx, const lps_states* st) {
  if (!ctx || !st) return LPS_E_NULL;
  if (st->n_states < 0) return LPS_E_SHAPE;
  if (st->n_states > ctx->max_states) return LPS_E_CAPACITY;
  if (st->n_states == 0) return LPS_OK;
  if (!st->params || !st->knot_off) return LPS_E_NULL;
  if (ctx->n_spl > 0 && (!st->knot_x || !st->knot_y)) return LPS_E_NULL;
  return LPS_OK;
}

hipError_t launch_cov_coeffs(lps_cov_ctx* c, const lps_states* st, hipStream_t s) {
  const int n = st->n_states;
  hipLaunchKernelGGL(k_cov_coeffs, dim3((n + 3) / 4), dim3(256), 0, s, n, c->n_spl, c->k_max, c->n_params,
                     st->params, st->knot_off, st->knot_cnt, st->knot_x, st->knot_y, c->x_first, c->x_last, c->bx,
                     c->coef, c->npc, c->status);
  return hipGetLastError();
}

// States per wave: enough waves to fill the chip for small batches, up to
// kCovMaxTile states sharing each table chunk for large ones.  The per-state
// summation order does not depend on it.
int cov_tile(const lps_cov_ctx* c, int n_states) {
  const long per = (long)n_states * c->n_groups / 8192;
  return (int)(per < 1 ? 1 : per > kCovMaxTile ? kCovMaxTile : per);
}

}  // namespace
}  // namespace lps

extern "C" {

lps_status lps_cov_create(const lps_cov_desc* d, int device, lps_cov_ctx** out) {
  using namespace lps;
  if (!d || !out) return LPS_E_NULL;
  *out = nullptr;
  if (!d->f || !d->nk || !d->P || !d->R) return LPS_E_NULL;
  if (d->n_bins < 1 || d->n_spl < 0 || d->n_spl > kCovMaxSpl) return LPS_E_SHAPE;
  if (d->k_max < 2 || d->k_max > kMaxKnots || d->max_states < 1) return LPS_E_CAPACITY;
  if (!(d->f_knee > 0.0) || !(d->arm_length > 0.0)) return LPS_E_SHAPE;
  for (int t = 0; t < 4; ++t)
    for (int c = 0; c < 3; ++c)
      if (d->route[t][c] < -1 || d->route[t][c] >= d->n_spl || (t == LPS_TERM_FG && d->route[t][c] != -1))
        return LPS_E_ROUTING;
  for (int i = 0; i < 3; ++i)
    if (d->corr[i] < -1 || d->corr[i] >= d->n_spl) return LPS_E_ROUTING;
  if (hipSetDevice(device) != hipSuccess) return LPS_E_DEVICE;
  const int K = d->n_bins;
  std::vector<double> fh(K);
  if (hipMemcpy(fh.data(), d->f, (size_t)K * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return LPS_E_DEVICE;
  for (int k = 0; k < K; ++k)
    if (!(fh[k] > 0.0) || (k > 0 && !(fh[k] > fh[k - 1]))) return LPS_E_SHAPE;

  lps_cov_ctx* c = new lps_cov_ctx;
  memset(c, 0, sizeof(*c));
  c->device = device;
  c->n_bins = K;
  c->n_chunks = (K + kCovChunk - 1) / kCovChunk;
  c->k_pad = c->n_chunks * kCovChunk;
  c->chunks_per_group = (c->n_chunks + kCovGroups - 1) / kCovGroups;
  c->n_groups = (c->n_chunks + c->chunks_per_group - 1) / c->chunks_per_group;
  c->n_spl = d->n_spl;
  c->has_fg = d->Rfg != nullptr;
  c->n_params = c->has_fg ? 5 : 4;
  c->k_max = d->k_max;
  c->max_states = d->max_states;
  for (int t = 0; t < 3; ++t)
    for (int ch = 0; ch < 3; ++ch) {
      c->rt.r[t][ch] = d->route[t][ch];
      if (d->route[t][ch] >= 0) c->diag_mask |= 1u << d->route[t][ch];
    }
  for (int i = 0; i < 3; ++i) c->rt.corr[i] = d->corr[i];
  c->x_knee = log10(d->f_knee);
  c->x_first = log10(fh[0]);
  c->x_last = log10(fh[K - 1]);

  const size_t S = (size_t)d->max_states;
  bool ok = hipMalloc((void**)&c->tab, (size_t)kCovRows * c->k_pad * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->bx, S * kCovMaxSpl * kMaxKnots * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->coef, S * kCovMaxSpl * kMaxKnots * 4 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->npc, S * kCovMaxSpl * sizeof(int32_t)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->status, S * sizeof(uint32_t)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->partial, S * c->n_groups * sizeof(double)) == hipSuccess;
  if (!ok) {
    lps_cov_destroy(c);
    return LPS_E_NOMEM;
  }
  hipLaunchKernelGGL(k_cov_table, dim3((c->k_pad + 255) / 256), dim3(256), 0, 0, K, c->k_pad, d->f, d->nk, d->P,
                     d->R, d->Rfg, d->arm_length, c->tab);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    lps_cov_destroy(c);
    return device_status(e);
  }
  *out = c;
  return LPS_OK;
}

lps_status lps_cov_destroy(lps_cov_ctx* c) {
  if (!c) return LPS_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  void* ptrs[] = {c->tab, c->bx, c->coef, c->npc, c->status, c->partial};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
  return LPS_OK;
}

lps_status lps_cov_loglike_batch(lps_cov_ctx* c, const lps_states* st, double* logL, uint32_t* status,
                                 void* stream) {
  using namespace lps;
  lps_status cs = check_cov_states(c, st);
  if (cs != LPS_OK) return cs;
  const int n = st->n_states;
  if (n == 0) return LPS_OK;
  if (!logL) return LPS_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_cov_coeffs(c, st, s);
  if (e != hipSuccess) return device_status(e);
  CovArgs A;
  A.tab = c->tab;
  A.k_pad = c->k_pad;
  A.n_chunks = c->n_chunks;
  A.chunks_per_group = c->chunks_per_group;
  A.n_groups = c->n_groups;
  A.n_states = n;
  A.tile = cov_tile(c, n);
  A.n_tiles = (n + A.tile - 1) / A.tile;
  A.n_spl = c->n_spl;
  A.has_fg = c->has_fg;
  A.rt = c->rt;
  A.diag_mask = c->diag_mask;
  A.x_knee = c->x_knee;
  A.params = st->params;
  A.status = c->status;
  A.bx = c->bx;
  A.coef = c->coef;
  A.npc = c->npc;
  A.partial = c->partial;
  const long waves = (long)A.n_tiles * A.n_groups;
  hipLaunchKernelGGL(k_cov_eval, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return device_status(e);
  hipLaunchKernelGGL(k_cov_finalize, dim3((n + 255) / 256), dim3(256), 0, s, n, c->n_groups, c->partial, c->status,
                     logL, status);
  return device_status(hipGetLastError());
}

lps_status lps_cov_build(lps_cov_ctx* c, const lps_states* st, int32_t k0, int32_t k1, double* C, uint32_t* status,
                         void* stream) {
  using namespace lps;
  lps_status cs = check_cov_states(c, st);
  if (cs != LPS_OK) return cs;
  if (k0 < 0 || k1 > c->n_bins || k0 >= k1) return LPS_E_SHAPE;
  const int n = st->n_states;
  if (n == 0) return LPS_OK;
  if (!C) return LPS_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_cov_coeffs(c, st, s);
  if (e != hipSuccess) return device_status(e);
  const int n_out = k1 - k0;
  const long total = (long)n * n_out;
  hipLaunchKernelGGL(k_cov_build, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, k0, n_out, c->k_pad,
                     c->tab, c->n_spl, c->rt, c->diag_mask, c->x_knee, c->has_fg, st->params, c->status, c->bx,
                     c->coef, c->npc, C);
  e = hipGetLastError();
  if (e == hipSuccess && status)
    e = hipMemcpyAsync(status, c->status, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
  return device_status(e);
}

}  // extern "C"
