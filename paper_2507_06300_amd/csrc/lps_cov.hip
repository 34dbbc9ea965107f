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
// Work decomposition: the coefficient kernel validates every state and
// stores the cubic pieces of its splines (one wave per state, one lane per
// piece).  In the evaluation kernel a workgroup of four waves takes one group
// of consecutive 128-bin chunks and four tiles of up to eight states; every
// wave runs through the states of its tile on each chunk, reading the chunk's
// table rows from memory (the four waves share them in L1).  Each (state,
// spline) has a cursor: the piece holding the chunk's first bin, found by a
// ballot over the piece abscissae (lane = piece) at the start of the group
// and advanced chunk by chunk; a chunk that reaches further pieces loads
// their records and selects per bin.  A state's cursors are read into one
// register and picked by lane index.  Spline values go through LDS so that
// the spline loop need not be unrolled.  Each wave keeps the sum of state i
// of its tile in lane i; partial sums per (state, chunk group) are added in a
// fixed order by the finalize kernel, so results do not depend on the batch
// size.  The adjoint (lps_cov_grad.hip) shares the model code through
// lps_cov_common.hpp.
#include <math.h>
#include <string.h>

#include <vector>

#include "lps_internal.hpp"
#include "lps_math64.hpp"
#include "lps_templates.hpp"
#include "lps_spline.hpp"
#include "lps_validate.hpp"
#include "lps_cov_common.hpp"
#include "lps_roctx.hpp"


namespace lps {
namespace {

using namespace covk;

// Orders the LDS accesses of one wavefront's lanes (lane 0 writes, all read).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ void k_cov_table(int K, int k_pad, const double* __restrict__ f, const double* __restrict__ nk,
                            const double* __restrict__ P, const double* __restrict__ R,
                            const double* __restrict__ Rfg, double L, double* __restrict__ tab,
                            double* __restrict__ sig) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k_pad) return;
  // padding repeats the last bin with N = 0 and no data: it adds exactly 0
  const int kk = k < K ? k : K - 1;
  const double fk = f[kk];
  double oms_ae, oms_t, tm_ae, tm_t, h;
  unit_templates(fk, L, oms_ae, oms_t, tm_ae, tm_t, h);
  const double sigma = kRefAoms * kRefAoms * oms_ae + kRefAtm * kRefAtm * tm_ae;
  const double is = 1.0 / sigma;
  double row[kCovRows];
  row[kRx] = log10(fk);
  row[kRnu] = k < K ? nk[kk] : 0.0;
  row[kRomsAE] = oms_ae * is;
  row[kRomsT] = oms_t * is;
  row[kRtmAE] = tm_ae * is;
  row[kRtmT] = tm_t * is;
  for (int c = 0; c < 3; ++c) {
    row[kRsg + c] = R[c * (size_t)K + kk] * h * is;
    row[kRfg + c] = Rfg ? Rfg[c * (size_t)K + kk] * is : 0.0;
  }
  for (int i = 0; i < 6; ++i) row[kRP + i] = k < K ? P[i * (size_t)K + kk] * is : 0.0;
  for (int r = 0; r < kCovRows; ++r) tab[tab_index(r, k)] = row[r];
  if (k < K) sig[k] = sigma;
}

// C0 = 3 sum_k N_k ln sigma_k in one block, fixed order.
__global__ __launch_bounds__(256) void k_cov_c0(int K, const double* __restrict__ nk,
                                                const double* __restrict__ sig, double* __restrict__ c0) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < K; k += 256) acc += nk[k] * log(sig[k]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) c0[0] = 3.0 * sh[0];
}

// One wave per state: validation (every spline slot), then one lane per piece.
__global__ __launch_bounds__(256) void k_cov_coeffs(int n_states, int n_spl, int k_max, int n_params,
                                                    const double* __restrict__ params, const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ kcnt, int64_t n_knots, const double* __restrict__ kx,
                                                    const double* __restrict__ ky, double x_first, double x_last,
                                                    double* __restrict__ bx, double* __restrict__ coef,
                                                    int32_t* __restrict__ npc, uint32_t* __restrict__ status) {
  const int lane = threadIdx.x & (kWave - 1);
  const int s = uniform(blockIdx.x * (blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (s >= n_states) return;
  const uint32_t st =
      validate_state_wave(lane, s, n_states, n_spl, k_max, n_params, params, off, kcnt, n_knots, kx, ky, x_first, x_last);
  if (lane == 0) status[s] = st;
  for (int j = 0; j < kCovMaxSpl; ++j) {
    int a = 0, n = 0;
    if (j < n_spl && st == 0) knot_range(off, kcnt, s * n_spl + j, n_knots, a, n);
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


// Four waves per SIMD: the register budget of 128 costs a few spills to
// scratch but hides more latency than three waves without them.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_cov_eval(CovArgs A) {
  // per wave: slot values of the current bin, and for every (state, spline) of
  // its tile the piece under the cursor (cursor, last piece this chunk, pieces)
  __shared__ double lval[4][kSlots][kWave];
  __shared__ PieceRec lrec[4][kCovMaxTile][kCovMaxSpl];
  __shared__ int lcur[4][kCovMaxTile][kCovMaxSpl][3];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = (int)(threadIdx.x / kWave);
  const int quads = (A.n_tiles + 3) / 4;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  if (blk >= quads * A.n_groups) return;
  const int g = blk / quads;
  const int t = (blk - g * quads) * 4 + w;
  const int s0 = t * A.tile;
  const int ns = t < A.n_tiles ? min(A.tile, A.n_states - s0) : 0;
  const int c_begin = g * A.chunks_per_group;
  const int c_end = min(A.n_chunks, c_begin + A.chunks_per_group);
  lval[w][kSlotOne][lane] = 1.0;
  lval[w][kSlotZero][lane] = 0.0;
  const LdsVal val{&lval[w][0][lane]};

  // cursors at the first bin of the group (lane = piece)
  const double xg = A.tab[tab_index(kRx, (size_t)c_begin * kCovChunk)];
  for (int i = 0; i < ns; ++i) {
    const int s = s0 + i;
    if (A.status[s] != 0u) continue;
#pragma unroll 1
    for (int j = 0; j < A.n_spl; ++j) {
      const int np = A.npc[(size_t)s * kCovMaxSpl + j];
      int cur = -1;
      if (np > 0) {
        const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
        const double bl = lane < np ? A.bx[row + lane] : INFINITY;
        cur = uniform(max(__popcll(__ballot(bl <= xg)) - 1, 0));
        const PieceRec pr = load_piece(A, row, cur, np);
        if (lane == 0) lrec[w][i][j] = pr;
      }
      if (lane == 0) {
        lcur[w][i][j][0] = cur;
        lcur[w][i][j][1] = cur;
        lcur[w][i][j][2] = np;
      }
    }
  }

  wave_sync();
  double acc = 0.0;   // lane i: the sum of state s0 + i over this group
  int* const lcur_w = &lcur[w][0][0][0];
  for (int ch = c_begin; ch < c_end; ++ch) {
    const int kb = ch * kCovChunk;
    const double* tb = A.tab + tab_index(0, kb) + lane;   // row r, bin b of the chunk: tb[b * kCovBlock + r * kWave]
    const double xl = A.tab[tab_index(kRx, kb + kCovChunk - 1)];
    for (int i = 0; i < ns; ++i) {
      const int s = s0 + i;
      if (A.status[s] != 0u) continue;
      const StateScal sc = state_scalars(A.params, A.n_states, s, A.has_fg);
      // the state's cursors in one register: lane 3j + q holds field q of
      // spline j (cursor piece, last piece this chunk, pieces), lane j the
      // start of the piece after spline j's cursor; read by lane index, so
      // no uniform branch below waits on LDS
      int* const lc = lcur_w + i * kCovMaxSpl * 3;
      int cv = lane < 3 * kCovMaxSpl ? lc[lane] : 0;
      const double xnv = lane < kCovMaxSpl ? lrec[w][i][lane].xn : 0.0;
      // pieces that start inside this chunk
#pragma unroll 1
      for (int j = 0; j < A.n_spl; ++j) {
        const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
        if (cur < 0 || !(xl >= readlane_d(xnv, j))) continue;
        const int np = __builtin_amdgcn_readlane(cv, 3 * j + 2);
        const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
        int hi = cur + 1;
        while (hi + 1 < np && A.bx[row + hi + 1] <= xl) ++hi;
        cv = lane == 3 * j + 1 ? hi : cv;
      }
      double v = 0.0;
      bool bad = false;
#pragma unroll 1
      for (int b = 0; b < kCovB; ++b) {
        const double x = tb[(size_t)b * kCovBlock + kRx * kWave];
        const double lin = sc.u + sc.alpha * (x - A.x_knee);
#pragma unroll 1
        for (int j = 0; j < A.n_spl; ++j) {
          const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
          double pv = 0.0;
          if (cur >= 0) {
            PieceRec pr = lrec[w][i][j];
            const int hi = __builtin_amdgcn_readlane(cv, 3 * j + 1);
            if (hi != cur) {
              const size_t row = ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
              const int np = __builtin_amdgcn_readlane(cv, 3 * j + 2);
              for (int q = cur + 1; q <= hi; ++q) {
                const PieceRec nq = load_piece(A, row, q, np);
                if (x >= nq.x0) pr = nq;
              }
            }
            const double tt = x - pr.x0;
            pv = pr.a0 + tt * (pr.a1 + tt * (pr.a2 + tt * pr.a3));
          }
          lval[w][j][lane] = slot_value(pv, j, A.rt, lin);
        }
        const TabRow row{tb + (size_t)b * kCovBlock};
        CovPoint p;
        cov_point(val, A.rt, sc, A.x_knee, row, p);
        v += cov_term(p, row, bad);
      }
      // move the cursors to the piece of the chunk's last bin
#pragma unroll 1
      for (int j = 0; j < A.n_spl; ++j) {
        const int cur = __builtin_amdgcn_readlane(cv, 3 * j);
        const int hi = __builtin_amdgcn_readlane(cv, 3 * j + 1);
        if (hi == cur) continue;
        const int np = __builtin_amdgcn_readlane(cv, 3 * j + 2);
        const PieceRec pr = load_piece(A, ((size_t)s * kCovMaxSpl + j) * kMaxKnots, hi, np);
        if (lane == 0) lrec[w][i][j] = pr;
        cv = lane == 3 * j ? hi : cv;
      }
      if (lane < 3 * kCovMaxSpl) lc[lane] = cv;
      wave_sync();
      if (__ballot(bad) != 0ull && lane == 0) atomicOr(&A.status[s], (unsigned)LPS_ST_PSD);
      v = wave_sum(v);
      acc = lane == i ? acc + v : acc;
    }
  }
  if (lane < ns) A.partial[(size_t)(s0 + lane) * A.n_groups + g] = acc;
}

__global__ void k_cov_finalize(int n_states, int n_groups, const double* __restrict__ partial,
                               const double* __restrict__ c0, const uint32_t* __restrict__ status,
                               double* __restrict__ logL, uint32_t* __restrict__ status_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_states) return;
  const uint32_t st = status[s];
  double sum = 0.0;
  for (int g = 0; g < n_groups; ++g) sum += partial[(size_t)s * n_groups + g];
  logL[s] = st ? -INFINITY : -(sum + c0[0]);
  if (status_out) status_out[s] = st;
}

// The six unique entries of C for bins [k0, k1) of every state (binary search
// for the piece of each bin).
__global__ void k_cov_build(int n_states, int k0, int n_out, int k_pad, const double* __restrict__ tab, int n_spl,
                            CovRoute rt, double x_knee, int has_fg,
                            const double* __restrict__ params, const uint32_t* __restrict__ status,
                            const double* __restrict__ bx, const double* __restrict__ coef,
                            const int32_t* __restrict__ npc, const double* __restrict__ sigma,
                            double* __restrict__ C) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_states * n_out) return;
  const int s = (int)(i / n_out), q = (int)(i % n_out), k = k0 + q;
  double* out = C + (size_t)s * 6 * n_out + q;
  if (status[s] != 0u) {
    for (int e = 0; e < 6; ++e) out[(size_t)e * n_out] = NAN;
    return;
  }
  const TabRow row{tab + tab_index(0, k)};
  const double x = row(kRx);
  const StateScal sc = state_scalars(params, n_states, s, has_fg);
  const double lin = sc.u + sc.alpha * (x - x_knee);
  double V[kSlots];
  V[kSlotOne] = 1.0;
  V[kSlotZero] = 0.0;
  for (int j = 0; j < kCovMaxSpl; ++j) {
    V[j] = 0.0;
    const int n = j < n_spl ? npc[(size_t)s * kCovMaxSpl + j] : 0;
    if (n == 0) {
      V[j] = slot_value(0.0, j, rt, lin);
      continue;
    }
    const double* br = bx + ((size_t)s * kCovMaxSpl + j) * kMaxKnots;
    int lo = 0, hi = n - 1;   // last piece whose start is <= x, clamped to [0, n-1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (br[mid] <= x) lo = mid;
      else hi = mid - 1;
    }
    const double* cr = coef + (((size_t)s * kCovMaxSpl + j) * kMaxKnots + lo) * 4;
    const double tt = x - br[lo];
    V[j] = slot_value(cr[0] + tt * (cr[1] + tt * (cr[2] + tt * cr[3])), j, rt, lin);
  }
  CovPoint p;
  cov_point([&](int j) { return V[j]; }, rt, sc, x_knee, row, p);
  const double r[3] = {p.r01, p.r02, p.r12};
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  const double sg = sigma[k];
  for (int c = 0; c < 3; ++c) out[(size_t)c * n_out] = p.d[c] * sg;
  for (int e = 0; e < 3; ++e)
    out[(size_t)(3 + e) * n_out] = sqrt_d(p.sn[pa[e]]) * r[e] * sqrt_d(p.sn[pb[e]]) * sg;
}


}  // namespace

namespace covk {

lps_status check_cov_states(const lps_cov_ctx* ctx, const lps_states* st) {
  if (!ctx || !st) return LPS_E_NULL;
  if (st->n_states < 0 || st->n_knots < 0) return LPS_E_SHAPE;
  if (st->n_states > ctx->max_states) return LPS_E_CAPACITY;
  if (st->n_states == 0) return LPS_OK;
  if (!st->params || !st->knot_off) return LPS_E_NULL;
  if (ctx->n_spl > 0 && (!st->knot_x || !st->knot_y)) return LPS_E_NULL;
  return LPS_OK;
}

hipError_t launch_cov_coeffs(lps_cov_ctx* c, const lps_states* st, hipStream_t s) {
  const int n = st->n_states;
  hipLaunchKernelGGL(k_cov_coeffs, dim3((n + 3) / 4), dim3(256), 0, s, n, c->n_spl, c->k_max, c->n_params,
                     st->params, st->knot_off, st->knot_cnt, st->n_knots, st->knot_x, st->knot_y, c->x_first, c->x_last, c->bx,
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

CovArgs cov_args(const lps_cov_ctx* c, const lps_states* st) {
  const int n = st->n_states;
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
  A.x_knee = c->x_knee;
  A.params = st->params;
  A.status = c->status;
  A.bx = c->bx;
  A.coef = c->coef;
  A.npc = c->npc;
  A.partial = c->partial;
  return A;
}

}  // namespace covk
}  // namespace lps

using namespace lps::covk;

extern "C" {

lps_status lps_cov_create(const lps_cov_desc* d, int device, lps_cov_ctx** out) {
  LPS_API_RANGE();
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
      const int j = d->route[t][ch];
      c->rt.g[t][ch] = (uint8_t)(j >= 0 ? j : kSlotOne);
      if (j >= 0) c->rt.diag_mask |= 1u << j;
    }
  for (int i = 0; i < 3; ++i) {
    const int j = d->corr[i];
    c->rt.gc[i] = (uint8_t)(j >= 0 ? j : kSlotZero);
    if (j >= 0) c->rt.corr_mask |= 1u << j;
  }
  if (c->rt.diag_mask & c->rt.corr_mask) {
    delete c;
    return LPS_E_ROUTING;
  }
  c->rt.sg_slot = -1;
  {
    const int j = d->route[LPS_TERM_SGWB][0];
    bool only = j >= 0 && d->route[LPS_TERM_SGWB][1] == j && d->route[LPS_TERM_SGWB][2] == j;
    for (int t = 0; t < 2 && only; ++t)
      for (int ch = 0; ch < 3; ++ch) only = only && d->route[t][ch] != j;
    if (only) c->rt.sg_slot = j;
  }
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
  ok = ok && hipMalloc((void**)&c->sigma, (size_t)K * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->c0, sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->gmo, S * kCovMaxSpl * kMaxKnots * 4 * sizeof(double)) == hipSuccess;
  if (!ok) {
    lps_cov_destroy(c);
    return LPS_E_NOMEM;
  }
  hipLaunchKernelGGL(k_cov_table, dim3((c->k_pad + 255) / 256), dim3(256), 0, 0, K, c->k_pad, d->f, d->nk, d->P,
                     d->R, d->Rfg, d->arm_length, c->tab, c->sigma);
  hipLaunchKernelGGL(k_cov_c0, dim3(1), dim3(256), 0, 0, K, d->nk, c->sigma, c->c0);
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
  LPS_API_RANGE();
  if (!c) return LPS_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  void* ptrs[] = {c->tab, c->bx, c->coef, c->npc, c->status, c->partial, c->sigma, c->c0, c->gmo};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
  return LPS_OK;
}

lps_status lps_cov_loglike_batch(lps_cov_ctx* c, const lps_states* st, double* logL, uint32_t* status,
                                 void* stream) {
  LPS_API_RANGE();
  using namespace lps;
  lps_status cs = check_cov_states(c, st);
  if (cs != LPS_OK) return cs;
  const int n = st->n_states;
  if (n == 0) return LPS_OK;
  if (!logL) return LPS_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_cov_coeffs(c, st, s);
  if (e != hipSuccess) return device_status(e);
  const CovArgs A = cov_args(c, st);
  const long blocks = (long)((A.n_tiles + 3) / 4) * A.n_groups;
  hipLaunchKernelGGL(k_cov_eval, dim3((unsigned)blocks), dim3(256), 0, s, A);
  e = hipGetLastError();
  if (e != hipSuccess) return device_status(e);
  hipLaunchKernelGGL(k_cov_finalize, dim3((n + 255) / 256), dim3(256), 0, s, n, c->n_groups, c->partial, c->c0,
                     c->status, logL, status);
  return device_status(hipGetLastError());
}

lps_status lps_cov_build(lps_cov_ctx* c, const lps_states* st, int32_t k0, int32_t k1, double* C, uint32_t* status,
                         void* stream) {
  LPS_API_RANGE();
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
                     c->tab, c->n_spl, c->rt, c->x_knee, c->has_fg, st->params, c->status, c->bx,
                     c->coef, c->npc, c->sigma, C);
  e = hipGetLastError();
  if (e == hipSuccess && status)
    e = hipMemcpyAsync(status, c->status, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
  return device_status(e);
}

}  // extern "C"
