// Adjoint of the batched forward pass: logL and dlogL/d(theta) for every state.
//
// The score of the segment-averaged Whittle likelihood is
//   dlogL/dS_ck = N_k (D_ck - S_ck) / S_ck^2
// (from logL = -sum N_k (D/S + ln S)).  A PSD term tau enters S as
// T_tau,c * 10^{P_j(x)} * amp_tau, so, with h_ck = dlogL/dS_ck,
//   dlogL/d ln amp_tau   = sum_k sum_c h_ck T~_tau,ck
//   dlogL/dP_j(x_k)      = ln 10 * sum over terms routed to spline j of h_ck T~_tau,ck
// and the spline's knots enter through the per-piece moments
//   M^p_i = sum_{k in piece i} dlogL/dP(x_k) (x_k - x_i)^p ,   p = 0..3,
// followed by an O(n) backward through the Akima construction of App. A
// (cubic coefficients -> knot slopes -> slope weights -> segment slopes ->
// knots).  The power law of Eq. (pl) is part of the background group's
// exponent, so dlogL/du and dlogL/dalpha follow from that group's moments.
//
// Two launches after the coefficient kernel:
//   k_grad        per (chunk, state tile): logL partial, template sums and
//                 first-piece moments per group in one 16/32-value record,
//                 last-piece moments and interior pieces for chunks that
//                 straddle a knot;
//   k_grad_finish one workgroup per state: stitches the chunk records into
//                 per-piece moments (one group per wave, fixed order,
//                 deterministic), then logL, template gradients and the
//                 Akima backward (one spline per wave, lane per knot).
#include <math.h>

#include <type_traits>

#include "lps_batched.hpp"
#include "lps_spline.hpp"
#include "lps_spline_back.hpp"
#include "lps_validate.hpp"

namespace lps {
namespace {

constexpr int kBGrad32 = 4;                       // bins per lane, mixed adjoint
constexpr int kBGrad64 = 2;                       // bins per lane, FP64 adjoint
constexpr int kChunkGrad32 = kWave * kBGrad32;    // 256
constexpr int kChunkGrad64 = kWave * kBGrad64;    // 128

template <int G>
struct RecSize {
  static constexpr int NVR = 4 + 4 * G;
  static constexpr int M = NVR <= 16 ? 4 : 5;
  static constexpr int NV = 1 << M;
};

// 64-lane reduce-scatter of NV = 2^M values through the wave's LDS block
// buf[NV][64]: lane l writes its values to column l, then the P = 64 / NV lanes
// of value v = l >> (6 - M) each add NV consecutive entries of row v in order
// and finish with an xor butterfly over those P lanes.  On return every lane
// holds the full sum of value index (lane >> (6 - M)); the order of every sum is
// fixed, so the result is deterministic.
template <int M, typename T>
__device__ inline T reduce_scatter(const T (&v)[1 << M], T* __restrict__ buf, int lane) {
  constexpr int NV = 1 << M;
  constexpr int P = kWave >> M;
#pragma unroll
  for (int i = 0; i < NV; ++i) buf[i * kWave + lane] = v[i];
  wave_lds_sync();
  const T* row = buf + (lane >> (6 - M)) * kWave + (lane & (P - 1)) * NV;
  T r = 0;
#pragma unroll
  for (int i = 0; i < NV; ++i) r += row[i];
#pragma unroll
  for (int off = 1; off < P; off <<= 1) r += __shfl_xor(r, off, kWave);
  wave_lds_sync();
  return r;
}

// Sum over the wave in double without LDS traffic.  v_permlane32_swap and
// v_permlane16_swap exchange the upper half of their first operand with the
// lower half of their second (across the wave's two halves, or between the
// two rows of each 32-lane half), so swapping a value with itself gives every
// lane its partner's copy; DPP then reads another lane of the same row (row
// mirror x -> x ^ 15, half mirror x -> x ^ 7, quad x -> x ^ 2, x ^ 1).  Lanes
// are paired as l ^ 32, l ^ 16, l ^ 15, l ^ 7, l ^ 2, l ^ 1 (six independent
// pairings: every lane ends with the total, in the same fixed order).
// Against the xor butterfly of __shfl_xor (twelve LDS permutes per sum) this
// is 4 % faster on the gradient workload, where it runs once per state and
// chunk.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int kDppRowMirror = 0x140;    // x -> x ^ 15 within a row of 16
constexpr int kDppHalfMirror = 0x141;   // x -> x ^ 7 within 8
constexpr int kDppQuadXor2 = 0x4E;      // quad permutation (2, 3, 0, 1)
constexpr int kDppQuadXor1 = 0xB1;      // quad permutation (1, 0, 3, 2)

template <bool kRows>
__device__ inline double swap_add(double x) {
  const uint64_t u = __double_as_longlong(x);
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  uint32_t l0, l1, h0, h1;
  if constexpr (kRows) {
    const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    l0 = rl[0], l1 = rl[1], h0 = rh[0], h1 = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    l0 = rl[0], l1 = rl[1], h0 = rh[0], h1 = rh[1];
  }
  // the lower lane's value first on both lanes of the pair
  return __longlong_as_double((long long)(((uint64_t)h0 << 32) | l0)) +
         __longlong_as_double((long long)(((uint64_t)h1 << 32) | l1));
}

__device__ inline double wave_sum_regs(double v) {
  v = swap_add<false>(v);
  v = swap_add<true>(v);
  v += dpp_d<kDppRowMirror>(v);
  v += dpp_d<kDppHalfMirror>(v);
  v += dpp_d<kDppQuadXor2>(v);
  v += dpp_d<kDppQuadXor1>(v);
  return v;
}

// Reduce-scatter of NV = 2^M doubles over the wave in registers (FP64
// adjoint): lanes l and l ^ m (m = 32, 16, 15, 7, then 3 for M = 5) exchange
// halves of their remaining values, the lane with bit b of l clear keeping the
// lower half; a quad (M = 4) or pair (M = 5) butterfly completes the sums.
// Lane l ends with the full sum of value l >> (6 - M), as the LDS version.
// Without the LDS transpose (32 KB per workgroup in FP64) the kernel runs
// three waves per SIMD instead of two: 0.318 -> 0.262 ms on 25,000 bins x
// 1,024 states, 4.36 -> 3.94 ms on 250,000 bins x 2,048 chains.  (The
// single-precision kernel keeps the LDS version: in registers it measured
// 2 % slower with the foreground term, where it is VALU-bound.)
template <bool kRows>
__device__ inline double swap_pair_add(double x, double y) {
  const uint64_t ux = __double_as_longlong(x), uy = __double_as_longlong(y);
  uint32_t l0, l1, h0, h1;
  if constexpr (kRows) {
    const auto rl = __builtin_amdgcn_permlane16_swap((uint32_t)ux, (uint32_t)uy, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap((uint32_t)(ux >> 32), (uint32_t)(uy >> 32), false, false);
    l0 = rl[0], l1 = rl[1], h0 = rh[0], h1 = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane32_swap((uint32_t)ux, (uint32_t)uy, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap((uint32_t)(ux >> 32), (uint32_t)(uy >> 32), false, false);
    l0 = rl[0], l1 = rl[1], h0 = rh[0], h1 = rh[1];
  }
  return __longlong_as_double((long long)(((uint64_t)h0 << 32) | l0)) +
         __longlong_as_double((long long)(((uint64_t)h1 << 32) | l1));
}
constexpr int kDppQuadRev = 0x1B;       // quad permutation (3, 2, 1, 0)

template <int M>
__device__ inline double reduce_scatter_regs(const double (&v)[1 << M], int lane) {
  static_assert(M == 4 || M == 5, "16 or 32 values");
  constexpr int NV = 1 << M;
  double a[NV / 2];
#pragma unroll
  for (int i = 0; i < NV / 2; ++i) a[i] = swap_pair_add<false>(v[i], v[i + NV / 2]);
  double b[NV / 4];
#pragma unroll
  for (int i = 0; i < NV / 4; ++i) b[i] = swap_pair_add<true>(a[i], a[i + NV / 4]);
  const bool lo3 = (lane & 8) == 0, lo2 = (lane & 4) == 0;
  double c[NV / 8];
#pragma unroll
  for (int i = 0; i < NV / 8; ++i)
    c[i] = (lo3 ? b[i] : b[i + NV / 8]) + dpp_d<kDppRowMirror>(lo3 ? b[i + NV / 8] : b[i]);
  double d[NV / 16];
#pragma unroll
  for (int i = 0; i < NV / 16; ++i)
    d[i] = (lo2 ? c[i] : c[i + NV / 16]) + dpp_d<kDppHalfMirror>(lo2 ? c[i + NV / 16] : c[i]);
  double r;
  if constexpr (M == 4) {
    r = d[0] + dpp_d<kDppQuadXor1>(d[0]);
    r = r + dpp_d<kDppQuadXor2>(r);
  } else {
    const bool lo1 = (lane & 2) == 0;
    r = (lo1 ? d[0] : d[1]) + dpp_d<kDppQuadRev>(lo1 ? d[1] : d[0]);
    r = r + dpp_d<kDppQuadXor1>(r);
  }
  return r;
}

// Elementary functions of the per-bin score.  WIDE = false: the working
// precision of the adjoint (hardware single-precision functions, the logarithm
// taken on the mantissa with the exponent added exactly; or the library's FP64
// functions).  WIDE = true: the double-range redo of a single-precision lane
// (exact exponent, single-precision accuracy).
template <typename T, bool WIDE>
struct ScoreMath;
template <>
struct ScoreMath<float, false> {
  __device__ static inline float exp2(float q) { return __builtin_amdgcn_exp2f(q); }
  __device__ static inline float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
  // the exponent exactly, the hardware logarithm on the mantissa in [1/2, 1)
  // (its error is then a fixed absolute amount, not a fraction of log2 v)
  __device__ static inline float log2(float v) {
    int e;
    const float m = frexpf(v, &e);
    return __builtin_amdgcn_logf(m) + (float)e;
  }
};
template <>
struct ScoreMath<double, false> {
  __device__ static inline double exp2(double q) { return exp2_d(q); }
  __device__ static inline double rcp(double v) { return rcp_d(v); }
  __device__ static inline double log2(double v) { return log2_d(v); }
};
template <>
struct ScoreMath<double, true> {
  // 2^q over the double range: the integer part exactly, the fraction in single precision
  __device__ static inline double exp2(float q) {
    const double qd = (double)q;
    const double n = fmin(fmax(floor(qd), -2100.0), 2100.0);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(qd - n)), (int)n);
  }
  __device__ static inline double rcp(double v) { return 1.0 / v; }
  __device__ static inline double log2(double v) {
    int e = 0;
    const double m = frexp(v, &e);
    return (double)e + (double)__builtin_amdgcn_logf((float)m);
  }
};

// Channel PSDs, logL term, score and group sensitivities of bin b from the
// group exponents qx[g] = Q_g(x_b) (factors 2^Q).  Returns the bin's logL term
// (in units of the table rows), adds the template sums of the shared and paper
// layouts to v1 (OMS), v2 (TM) and the foreground sum to v3, and writes the
// sensitivity dlogL/dQ_g / ln 2 of every group to gq.  T is the arithmetic
// type: the working precision, or double for a lane whose single-precision
// values left the range.
template <typename T, bool WIDE, int MODE, int NCH, bool FG, int G, int NT, int B, typename R>
__device__ inline T bin_score(int b, const R (&qx)[G], const R (&Kt)[NT][NCH][B], const R (&ND)[NCH][B], R nl,
                              R w_oms, R w_tm, R e_fg, T& v1, T& v2, T& v3, T (&gq)[G]) {
  using SM = ScoreMath<T, WIDE>;
  T e[G];
#pragma unroll
  for (int g = 0; g < G; ++g) e[g] = SM::exp2(qx[g]);
  T S[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) S[c] = FG ? (T)Kt[3][c][b] * (T)e_fg : (T)0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if constexpr (MODE == kSplit) {
      // the OMS row is 1 in this layout (the tables are scaled by it)
#pragma unroll
      for (int c = 0; c < NCH; ++c) S[c] = g == 0 ? (FG ? S[c] + e[g] : e[g]) : S[c] + (T)Kt[g][c][b] * e[g];
    } else if constexpr (MODE == kShared) {
#pragma unroll
      for (int c = 0; c < NCH; ++c)
        S[c] += (g == 0 ? ((T)w_oms * (T)Kt[0][c][b] + (T)w_tm * (T)Kt[1][c][b]) : (T)Kt[2][c][b]) * e[g];
    } else {
      if (g < 3) {
        S[g] += ((T)w_oms * (T)Kt[0][g][b] + (T)w_tm * (T)Kt[1][g][b]) * e[g];
      } else {
#pragma unroll
        for (int c = 0; c < NCH; ++c) S[c] += (T)Kt[2][c][b] * e[g];
      }
    }
  }
  const T Nn = (T)nl * (T)(1.0 / kLn2);
  T h[NCH];
  T l = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const T lw = (NCH == 2 && c == 0) ? (T)2 : (T)1;
    const T r = SM::rcp(S[c]);
    const T q1 = (T)ND[c][b] * r;
    l += q1;
    h[c] = (q1 - lw * Nn) * r;       // dlogL/dS~ (scaled units), A and E summed when merged
  }
  // sum_c w_c ln S_c = ln2 log2 prod_c S_c^w_c (w = 2 for the merged A/E row): one logarithm
  const T Lp = NCH == 2 ? S[0] * S[0] * S[1] : S[0] * S[1] * S[NCH - 1];
  l += (T)nl * SM::log2(Lp);
  if constexpr (FG) {
    T fg_sum = 0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) fg_sum += h[c] * (T)Kt[3][c][b];
    v3 += fg_sum * (T)e_fg;
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if constexpr (MODE == kSplit) {
      T a = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) a += g == 0 ? h[c] : h[c] * (T)Kt[g][c][b];
      gq[g] = a * e[g];
    } else {
      const bool noise = MODE == kShared ? g == 0 : g < 3;
      if (noise) {
        T ao = 0, at = 0;
        if constexpr (MODE == kShared) {
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            ao += h[c] * (T)Kt[0][c][b];
            at += h[c] * (T)Kt[1][c][b];
          }
        } else {
          ao = h[g] * (T)Kt[0][g][b];
          at = h[g] * (T)Kt[1][g][b];
        }
        const T ro_ = (T)w_oms * ao * e[g], rt_ = (T)w_tm * at * e[g];
        v1 += ro_;
        v2 += rt_;
        gq[g] = ro_ + rt_;
      } else {
        T a = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) a += h[c] * (T)Kt[2][c][b];
        gq[g] = a * e[g];
      }
    }
  }
  return l;
}

// Inputs and outputs of the double-range redo of one lane (passed by value to
// an out-of-line function, so that the rare redo adds nothing to the register
// budget of the common path).
template <int G, int NT, int NCH, int B>
struct WideLane {
  float qe[G][B];
  float Kt[NT][NCH][B];
  float ND[NCH][B];
  float NL[B];
  float w_oms, w_tm, e_fg;
};
template <int G, int B>
struct WideOut {
  double l, v1, v2, v3;
  float gq[G][B];
};

template <int MODE, int NCH, bool FG, int G, int NT, int B>
__device__ __noinline__ WideOut<G, B> redo_lane_wide(WideLane<G, NT, NCH, B> in) {
  WideOut<G, B> o;
  o.l = o.v1 = o.v2 = o.v3 = 0.0;
  // one bin at a time (the inputs live in the by-value copy): few registers
#pragma unroll 1
  for (int b = 0; b < B; ++b) {
    float qx[G];
    double gq[G];
#pragma unroll
    for (int g = 0; g < G; ++g) qx[g] = in.qe[g][b];
    o.l += bin_score<double, true, MODE, NCH, FG, G, NT, B>(b, qx, in.Kt, in.ND, in.NL[b], in.w_oms, in.w_tm, in.e_fg,
                                                      o.v1, o.v2, o.v3, gq);
#pragma unroll
    for (int g = 0; g < G; ++g) o.gq[g][b] = (float)gq[g];
  }
  return o;
}

// Waves per SIMD the register allocation must allow: four for the
// single-precision kernels with merged A/E rows (128 registers and about
// 100 bytes more spilled than at three waves, outside the bin loop; 4 % faster
// on the sampler workload), the compiler's choice otherwise.
template <typename R, int NCH>
struct GradWaves {
  static constexpr int v = (sizeof(R) == 4 && NCH == 2) ? 4 : 1;
};

template <typename R, int MODE, int NCH, bool FG, int B>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GradWaves<R, NCH>::v))) void k_grad(int n_states, int n_chunks, int n_tiles, int tile, int K, int k_pad,
                                              int ref_chunk, const R* __restrict__ tab,
                                              const double* __restrict__ x64, const double* __restrict__ bx,
                                              const R* __restrict__ coef, const double* __restrict__ coef64,
                                              const int32_t* __restrict__ n_int,
                                              const StateScalars* __restrict__ scal, R* __restrict__ rec,
                                              int2* __restrict__ gidx, double* __restrict__ glast,
                                              double* __restrict__ moments, double* __restrict__ lrec) {
  constexpr int G = Groups<MODE>::G;
  constexpr int NT = FG ? 4 : 3;
  constexpr int CH = kWave * B;
  constexpr int SUB = kWave / G;
  constexpr int M = RecSize<G>::M;
  constexpr int NV = RecSize<G>::NV;
  constexpr bool kMixed = sizeof(R) == 4;
  constexpr bool kScalars = FG || MODE != kSplit;
  using R4 = typename std::conditional<kMixed, float4, double4>::type;
  // Per wave: the located piece of every (state, group) pair of the sub-tile
  // and, for a chunk that crosses the next breakpoint, that next piece and the
  // abscissa where it takes over (all in table units); per-state scalars.
  // lc0/lc1 hold each piece's exponent cubic about an origin chosen as in the
  // forward kernel (single precision: the block midpoint for a piece that
  // covers the whole chunk, else the chunk start or the piece's own start;
  // offsets lq0/lq1 = xo - origin), loff0/loff1 the offsets xo - x_piece of
  // the piece-relative abscissa t that the moments use.
  __shared__ R4 lc0[kWavesPerBlock][kWave];
  __shared__ R4 lc1[kWavesPerBlock][kWave];
  __shared__ R lq0[kWavesPerBlock][kWave];
  __shared__ R lq1[kWavesPerBlock][kWave];
  __shared__ R loff0[kWavesPerBlock][kWave];
  __shared__ R loff1[kWavesPerBlock][kWave];
  __shared__ R llim[kWavesPerBlock][kWave];
  __shared__ R lscal[kWavesPerBlock][SUB][4];
  __shared__ R lred[kWavesPerBlock][kMixed ? NV * kWave : 1];   // reduce-scatter transpose (single precision)
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = uniform(threadIdx.x >> 6);
  // same work order as the forward kernel: tile groups per chunk over
  // XCD-contiguous block ranges
  const int item = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wv;
  const int tg = item / (n_chunks * kTileGroupGrad);
  const int rem = item - tg * (n_chunks * kTileGroupGrad);
  const int tl = min(kTileGroupGrad, n_tiles - tg * kTileGroupGrad);
  if (tl <= 0) return;
  const int chunk = rem / tl;
  const int t = tg * kTileGroupGrad + (rem - chunk * tl);
  if (chunk >= n_chunks) return;
  const int s_begin = t * tile;
  const int s_end = min(s_begin + tile, n_states);
  const int kbase = chunk * CH;

  R xr[B], NL[B];
  R Kt[NT][NCH][B];
  R ND[NCH][B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int k = kbase + b * kWave + lane;
    xr[b] = tab[k];
#pragma unroll
    for (int term = 0; term < NT; ++term)
#pragma unroll
      for (int c = 0; c < NCH; ++c) Kt[term][c][b] = tab[(size_t)tab_k(term, c, NCH) * k_pad + k];
#pragma unroll
    for (int c = 0; c < NCH; ++c) ND[c][b] = tab[(size_t)tab_nd(c, NT, NCH) * k_pad + k];
    NL[b] = tab[(size_t)tab_nl(NT, NCH) * k_pad + k];
  }
  const int klast = min(kbase + CH, K) - 1;
  const double xf = x64[kbase];
  const double xl = x64[klast];
  // abscissa origin of the single-precision table rows (midpoint of their 512-bin block)
  const double xo = kMixed ? block_origin(x64, (kbase / ref_chunk) * ref_chunk, K) : 0.0;
  // powers of the bins' abscissae about the chunk's first abscissa xf, shared
  // by every state: the first-piece moments are summed about xf (one add and
  // three FMAs per group and bin) and moved to the piece start b <= xf by the
  // finisher; x - xf >= 0 and xf - b >= 0 keep every term of that move of one
  // sign
  R P1[B], P2[B], P3[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    P1[b] = kMixed ? xr[b] - (R)(xf - xo) : (R)(xr[b] - xf);
    P2[b] = P1[b] * P1[b];
    P3[b] = P2[b] * P1[b];
  }

  for (int sub = s_begin; sub < s_end; sub += SUB) {
    const int nsub = min(SUB, s_end - sub);
    // the lane index, opaque to the compiler here: the LDS addresses below are
    // formed again per sub-tile instead of being held (and spilled) across the
    // whole work item
    int ln = lane;
    asm volatile("" : "+v"(ln));
    // ---- locate: lane p owns the piece of (state sub + p / G, group p % G) ----
    const int ps = lane / G, pg = lane - (lane / G) * G;
    const bool pv = ps < nsub;
    const size_t pbase = (size_t)((sub + ps) * G + pg) * kMaxKnots;
    const int pni = pv ? n_int[(sub + ps) * G + pg] : 0;
    int pi0 = 0, pi1 = 0;
    if (pni > 0) {
      pi0 = count_le(bx + pbase, pni, xf);
      const double b_next = pi0 + 1 < pni ? bx[pbase + pi0 + 1] : (double)INFINITY;
      pi1 = b_next <= xl ? count_le(bx + pbase, pni, xl) : pi0;
      const double b0 = bx[pbase + pi0];
      // exponent cubic of piece i (start bi) about origin org, and its offset
      auto stage = [&](int i, double bi, double org, R4& r4, R& off) {
        if constexpr (kMixed) {
          const double* cf = coef64 + (pbase + i) * 4;
          const double t0 = org - bi;
          const double a = cf[0], b = cf[1], c = cf[2], d = cf[3];
          r4.x = (R)(a + t0 * (b + t0 * (c + t0 * d)));
          r4.y = (R)(b + t0 * (2.0 * c + 3.0 * d * t0));
          r4.z = (R)(c + 3.0 * d * t0);
          r4.w = (R)d;
          off = (R)(xo - org);
        } else {
          const R* cf = coef + (pbase + i) * 4;
          r4.x = cf[0];
          r4.y = cf[1];
          r4.z = cf[2];
          r4.w = cf[3];
          off = (R)(-bi);
        }
      };
      R4 r4;
      R qo;
      stage(pi0, b0, pi1 > pi0 ? xf : xo, r4, qo);
      lc0[wv][ln] = r4;
      lq0[wv][ln] = qo;
      loff0[wv][ln] = kMixed ? (R)(xo - b0) : (R)(-b0);
      if (pi1 > pi0) {
        stage(pi0 + 1, b_next, b_next, r4, qo);
        lc1[wv][ln] = r4;
        lq1[wv][ln] = qo;
        loff1[wv][ln] = kMixed ? (R)(xo - b_next) : (R)(-b_next);
        llim[wv][ln] = kMixed ? (R)(b_next - xo) : (R)b_next;
      }
    }
    if constexpr (kScalars) {
      if (pv && pg == 0) {
        const StateScalars sc = scal[sub + ps];
        lscal[wv][ps][0] = (R)sc.w_oms;
        lscal[wv][ps][1] = (R)sc.w_tm;
        lscal[wv][ps][2] = (R)sc.e_fg;
      }
    }
    const unsigned long long straddle = __ballot(pv && pni > 0 && pi1 > pi0);
    const unsigned long long multi = __ballot(pv && pni > 0 && pi1 > pi0 + 1);
    const unsigned long long invalid = __ballot(pv && pg == 0 && pni == 0);
    unsigned long long cross_state = straddle;
#pragma unroll
    for (int g = 1; g < G; ++g) cross_state |= straddle >> g;
    wave_lds_sync();

    for (int q = 0; q < nsub; ++q) {
      const int s = sub + q;
      const size_t ro = (size_t)s * n_chunks + chunk;
      if ((invalid >> (q * G)) & 1ull) {   // invalid state: the finisher reports it
        if (lane < NV) rec[ro * NV + lane] = (R)0;
        if (lane < G) gidx[ro * G + lane] = make_int2(0, 0);
        continue;
      }
      R w_oms = 0, w_tm = 0, e_fg = 0;
      if constexpr (kScalars) {
        w_oms = lscal[wv][q][0];
        w_tm = lscal[wv][q][1];
        e_fg = lscal[wv][q][2];
      }
      const bool crossing = (cross_state >> (q * G)) & 1ull;

      // group exponents Q (factors 2^Q) and piece abscissae T (t = x - x_piece) per bin
      R Qe[G][B], T[G][B];
      if (!crossing) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const R4 c0 = lc0[wv][q * G + g];
          const R o0 = loff0[wv][q * G + g];
#pragma unroll
          for (int b = 0; b < B; ++b) {
            // single precision: the cubic about the block midpoint (offset 0)
            const R tq = kMixed ? xr[b] : xr[b] + o0;
            Qe[g][b] = c0.x + tq * (c0.y + tq * (c0.z + tq * c0.w));
          }
        }
      } else {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int pl = q * G + g;
          if (!((multi >> pl) & 1ull)) {   // at most one breakpoint: both staged pieces from LDS
            const R4 c0 = lc0[wv][pl];
            const R o0 = loff0[wv][pl], d0 = lq0[wv][pl];
            const bool str = (straddle >> pl) & 1ull;
            const R4 c1 = str ? lc1[wv][pl] : c0;
            const R o1 = str ? loff1[wv][pl] : o0;
            const R d1 = str ? lq1[wv][pl] : d0;
            const R lim = str ? llim[wv][pl] : (R)INFINITY;
#pragma unroll
            for (int b = 0; b < B; ++b) {
              const bool second = xr[b] >= lim;
              const R4 cc = second ? c1 : c0;
              T[g][b] = xr[b] + (second ? o1 : o0);
              const R tq = xr[b] + (second ? d1 : d0);
              Qe[g][b] = cc.x + tq * (cc.y + tq * (cc.z + tq * cc.w));
            }
          } else {         // several breakpoints: each piece from memory, select per bin
            const int i0 = __builtin_amdgcn_readlane(pi0, pl);
            const int i1 = __builtin_amdgcn_readlane(pi1, pl);
            const size_t base = (size_t)(s * G + g) * kMaxKnots;
            R Q[B] = {};
            for (int j = i0; j <= i1; ++j) {
              const R* cf = coef + (base + j) * 4;
              const double bj = bx[base + j];
              // the first piece as staged (about the chunk start in single
              // precision); the later ones start inside the chunk
              const bool first = kMixed && j == i0;
              const R4 c0 = lc0[wv][pl];
              const R a = first ? c0.x : cf[0], bb = first ? c0.y : cf[1];
              const R cc = first ? c0.z : cf[2], dd = first ? c0.w : cf[3];
              const R off = kMixed ? (R)(xo - bj) : (R)(-bj);
              const R qoff = first ? lq0[wv][pl] : off;
              const R lim = kMixed ? (R)(bj - xo) : (R)bj;
#pragma unroll
              for (int b = 0; b < B; ++b) {
                const R tt = xr[b] + off;
                const R tq = xr[b] + qoff;
                const R qv = a + tq * (bb + tq * (cc + tq * dd));
                const bool sel = (j == i0) || (xr[b] >= lim);
                Q[b] = sel ? qv : Q[b];
                T[g][b] = sel ? tt : T[g][b];
              }
            }
#pragma unroll
            for (int b = 0; b < B; ++b) Qe[g][b] = Q[b];
          }
        }
      }

      // channel PSDs, score, per-group sensitivities; lane sums in R
      R vf[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) vf[i] = 0;
      R gq_keep[G][B];
      R l0 = 0;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        R qx[G], gq[G];
#pragma unroll
        for (int g = 0; g < G; ++g) qx[g] = Qe[g][b];
        l0 += bin_score<R, false, MODE, NCH, FG, G, NT, B>(b, qx, Kt, ND, NL[b], w_oms, w_tm, e_fg, vf[1], vf[2], vf[3], gq);
#pragma unroll
        for (int g = 0; g < G; ++g) gq_keep[g][b] = gq[g];
      }
      // the lane's logL terms in double (the per-state sum runs over every chunk)
      double ld = (double)l0;
      if constexpr (kMixed) {
        if (!isfinite(l0)) {
          // A channel PSD left the single-precision range (an extreme state):
          // redo the lane's bins with the group factors in double range (exact
          // exponent, single-precision mantissa), so that such a state gets the
          // status and values of the FP64 path.
          WideLane<G, NT, NCH, B> in;
#pragma unroll
          for (int b = 0; b < B; ++b) {
#pragma unroll
            for (int g = 0; g < G; ++g) in.qe[g][b] = Qe[g][b];
#pragma unroll
            for (int term = 0; term < NT; ++term)
#pragma unroll
              for (int c = 0; c < NCH; ++c) in.Kt[term][c][b] = Kt[term][c][b];
#pragma unroll
            for (int c = 0; c < NCH; ++c) in.ND[c][b] = ND[c][b];
            in.NL[b] = NL[b];
          }
          in.w_oms = w_oms;
          in.w_tm = w_tm;
          in.e_fg = e_fg;
          const WideOut<G, B> o = redo_lane_wide<MODE, NCH, FG, G, NT, B>(in);
          ld = o.l;
          vf[1] = (R)o.v1;
          vf[2] = (R)o.v2;
          vf[3] = (R)o.v3;
#pragma unroll
          for (int b = 0; b < B; ++b)
#pragma unroll
            for (int g = 0; g < G; ++g) gq_keep[g][b] = o.gq[g][b];
        }
      }
      // moments of the first piece about the chunk origin: bins before the next breakpoint
      auto accum_moments = [&](auto first_piece_only) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int pl = q * G + g;
          R lim1 = (R)INFINITY;
          if constexpr (decltype(first_piece_only)::value)
            lim1 = ((straddle >> pl) & 1ull) ? llim[wv][pl] : (R)INFINITY;
#pragma unroll
          for (int b = 0; b < B; ++b) {
            R gq = gq_keep[g][b];
            if constexpr (decltype(first_piece_only)::value) gq = xr[b] < lim1 ? gq : (R)0;
            vf[4 + 4 * g + 0] += gq;
            vf[4 + 4 * g + 1] = fma(gq, P1[b], vf[4 + 4 * g + 1]);
            vf[4 + 4 * g + 2] = fma(gq, P2[b], vf[4 + 4 * g + 2]);
            vf[4 + 4 * g + 3] = fma(gq, P3[b], vf[4 + 4 * g + 3]);
          }
        }
      };
      // a chunk inside one piece of every group needs no per-bin piece test
      if (crossing) accum_moments(std::true_type{});
      else accum_moments(std::false_type{});
      // the logL partial is added over the wave in double; the other lane sums
      // (B bins each) in the working precision, stored in it (the finisher adds
      // the records in double)
      if constexpr (kMixed) {
        const double lw = wave_sum_regs(ld);
        if (lane == 0) lrec[ro] = lw;
      } else {
        vf[0] = l0;
      }
      R red;
      if constexpr (kMixed) red = reduce_scatter<M>(vf, lred[wv], lane);
      else red = reduce_scatter_regs<M>(vf, lane);
      if ((lane & ((1 << (6 - M)) - 1)) == 0) rec[ro * NV + (lane >> (6 - M))] = red;
      {
        int a0 = 0, a1 = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int u0 = __builtin_amdgcn_readlane(pi0, q * G + g);
          const int u1 = __builtin_amdgcn_readlane(pi1, q * G + g);
          if (lane == g) {
            a0 = u0;
            a1 = u1;
          }
        }
        if (lane < G) gidx[ro * G + lane] = make_int2(a0, a1);
      }
      if (!crossing) continue;
      // later pieces of the groups that cross a breakpoint in this chunk:
      // interior pieces are complete here and go straight to the moment table;
      // the last piece is stitched with the next chunk by the finisher
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int pl = q * G + g;
        if (!((straddle >> pl) & 1ull)) continue;
        const int i0 = __builtin_amdgcn_readlane(pi0, pl);
        const int i1 = __builtin_amdgcn_readlane(pi1, pl);
        const size_t base = (size_t)(s * G + g) * kMaxKnots;
        for (int j = i0 + 1; j <= i1; ++j) {
          const R lo = j == i0 + 1 ? llim[wv][pl] : (kMixed ? (R)(bx[base + j] - xo) : (R)bx[base + j]);
          R hi = (R)INFINITY;
          if (j < i1) hi = kMixed ? (R)(bx[base + j + 1] - xo) : (R)bx[base + j + 1];
          R mm[4] = {0, 0, 0, 0};
#pragma unroll
          for (int b = 0; b < B; ++b) {
            const bool in = (xr[b] >= lo) && (xr[b] < hi);
            const R gq = in ? gq_keep[g][b] : (R)0;
            const R tt = T[g][b];
            const R u1 = gq * tt, u2 = u1 * tt;
            mm[0] += gq;
            mm[1] += u1;
            mm[2] += u2;
            mm[3] += u2 * tt;
          }
          double md[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) md[p] = wave_sum((double)mm[p]);
          if (lane == 0) {
            double* dst = (j == i1) ? glast + (ro * G + g) * 4 : moments + ((size_t)(s * G + g) * kMaxKnots + j) * 4;
#pragma unroll
            for (int p = 0; p < 4; ++p) dst[p] = md[p];
          }
        }
      }
    }
    wave_lds_sync();
  }
}

// Origin xc of the first-piece moments of chunk c (chunks of `bins` bins):
// the chunk's first abscissa.
struct ChunkOrigin {
  const double* x;
  int bins;
  __device__ double at(int c) const { return x[(size_t)c * bins]; }
};

// Per-wave LDS of the finishing kernel.

// LDS of the finishing kernel: one workgroup per state.
struct FinishLds {
  double mo[kMaxGroups][kMaxKnots][4];   // per-piece moments M^p_i of every group
  double part[kWavesPerBlock][4];        // per-wave partial record sums
  BackLds back[kWavesPerBlock];
};

// One step of a segmented inclusive scan over the wave by DPP (no LDS): lane
// l adds the four values of the lane the pattern CTRL names (row shift right
// by 1, 2, 4, 8, or lane 15 / 31 broadcast to the following rows under
// ROWMASK) when that lane carries the same key; a lane without a source gets
// the key INT_MIN and adds nothing.  Keys must not decrease along the lanes,
// so an equal key at the source means the same key on every lane between.
// (Against the __shfl_up butterfly, nine LDS permutes per step, the finishing
// kernel ran 126 -> 116 us on 2,048 chains of 977 chunks.)
template <int CTRL, int ROWMASK>
__device__ inline void seg_scan_step(int key, double (&v)[4]) {
  const int ku = __builtin_amdgcn_update_dpp((int)0x80000000, key, CTRL, ROWMASK, 0xF, false);
  double vu[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const uint64_t u = __double_as_longlong(v[p]);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWMASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWMASK, 0xF, false);
    vu[p] = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  }
  if (ku == key) {
#pragma unroll
    for (int p = 0; p < 4; ++p) v[p] += vu[p];
  }
}

__device__ inline uint64_t wave_or64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, kWave);
    v |= ((uint64_t)hi << 32) | lo;
  }
  return v;
}

// Per-piece moments of group g of state s from the chunk records.  Piece i
// collects the last-piece moments of the chunk that straddles into it (if
// any) followed by the first-piece moments of every chunk that starts in it,
// in chunk order; pieces lying strictly inside a straddling chunk were
// written to `moments` by k_grad.  A record's first-piece moments R_k are
// taken about its chunk's first abscissa xc and moved here to the piece
// start b (d = xc - b >= 0): M_m = sum_k C(m, k) d^(m - k) R_k.  Lanes walk 64 chunks at a time; a
// segmented scan keyed by the starting piece sums the chunks of one piece,
// so the order of every sum is fixed.
template <typename RT>
__device__ void stitch_group(int lane, int s, int g, int G, int NV, int n_chunks, int ni, const ChunkOrigin& org,
                             const double* __restrict__ bx, const RT* __restrict__ rec,
                             const int2* __restrict__ gidx, const double* __restrict__ glast,
                             const double* __restrict__ moments, double (*mo)[4]) {
  for (int p = 0; p < 4; ++p) mo[lane][p] = 0.0;
  uint64_t inner = 0;
  wave_lds_sync();
  for (int cb = 0; cb < n_chunks; cb += kWave) {
    const int c = cb + lane;
    const bool have = c < n_chunks;
    const size_t ro = (size_t)s * n_chunks + (have ? c : 0);
    const int2 ab = have ? gidx[ro * G + g] : make_int2(-1, -1);
    double v[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) v[p] = have ? (double)rec[ro * NV + 4 + 4 * g + p] : 0.0;
    if (have) {
      const double d = org.at(c) - bx[(size_t)(s * G + g) * kMaxKnots + ab.x];
      const double m0 = v[0], m1 = v[1], m2 = v[2];
      v[1] = m1 + d * m0;
      v[2] = m2 + d * (2.0 * m1 + d * m0);
      v[3] = v[3] + d * (3.0 * m2 + d * (3.0 * m1 + d * m0));
    }
    if (ab.y > ab.x) {
      const double* last = glast + (ro * G + g) * 4;
#pragma unroll
      for (int p = 0; p < 4; ++p) mo[ab.y][p] += last[p];
      if (ab.y - ab.x >= 2) inner |= ((1ull << ab.y) - 1ull) & ~((1ull << (ab.x + 1)) - 1ull);
    }
    const int key = ab.x;
    // within rows of 16 lanes, then across rows
    seg_scan_step<0x111, 0xF>(key, v);   // row_shr:1
    seg_scan_step<0x112, 0xF>(key, v);   // row_shr:2
    seg_scan_step<0x114, 0xF>(key, v);   // row_shr:4
    seg_scan_step<0x118, 0xF>(key, v);   // row_shr:8
    seg_scan_step<0x142, 0xA>(key, v);   // row_bcast:15 into rows 1 and 3
    seg_scan_step<0x143, 0xC>(key, v);   // row_bcast:31 into rows 2 and 3
    const int kn = __shfl_down(key, 1, kWave);
    const bool seg_end = have && (lane == kWave - 1 || kn != key);
    wave_lds_sync();
    if (seg_end) {
#pragma unroll
      for (int p = 0; p < 4; ++p) mo[key][p] += v[p];
    }
    wave_lds_sync();
  }
  inner = wave_or64(inner);
  if (lane < ni && ((inner >> lane) & 1ull)) {
    const double* src = moments + ((size_t)(s * G + g) * kMaxKnots + lane) * 4;
#pragma unroll
    for (int p = 0; p < 4; ++p) mo[lane][p] = src[p];
  }
  wave_lds_sync();
}

// One workgroup per state: the four waves add the chunk records' logL and
// template sums (a quarter of the chunks each, combined in wave order), stitch
// the groups' records (type RT: the working precision of the adjoint kernel)
// into per-piece moments one group per wave, then form the template-parameter
// gradients and run the spline backward one spline per wave.
template <typename RT>
__global__ __launch_bounds__(256) void k_grad_finish(
    int n_states, int n_spl, int n_params, int NV, int n_chunks, ChunkOrigin org, Layout lay, double x_knee,
    const double* __restrict__ params, const int32_t* __restrict__ off, const int32_t* __restrict__ kcnt, int64_t n_knots,
    const double* __restrict__ kx, const double* __restrict__ ky, const int32_t* __restrict__ n_int,
    const double* __restrict__ bx, const RT* __restrict__ rec, const int2* __restrict__ gidx,
    const double* __restrict__ glast, const double* __restrict__ moments, const double* __restrict__ lrec,
    const double* __restrict__ c0, const uint32_t* __restrict__ status_ws, double* __restrict__ logL,
    double* __restrict__ dparams, double* __restrict__ dkx, double* __restrict__ dky, uint32_t* __restrict__ status) {
  __shared__ FinishLds L;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = uniform(threadIdx.x >> 6);
  const int s = blockIdx.x;
  if (s >= n_states) return;   // the whole workgroup
  const int G = lay.n_grp;
  uint32_t st = status_ws[s];
  double sums[4] = {0.0, 0.0, 0.0, 0.0};
  if (st == 0) {   // uniform over the workgroup
    double ps[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = wv * kWave + lane; c < n_chunks; c += kWavesPerBlock * kWave) {
      const RT* r = rec + ((size_t)s * n_chunks + c) * NV;
      // logL partials: a double array beside single-precision records, else slot 0
      ps[0] += lrec ? lrec[(size_t)s * n_chunks + c] : (double)r[0];
#pragma unroll
      for (int i = 1; i < 4; ++i) ps[i] += (double)r[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) ps[i] = wave_sum(ps[i]);
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i) L.part[wv][i] = ps[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
      for (int w = 0; w < kWavesPerBlock; ++w) sums[i] += L.part[w][i];
  }
  const double Lv = c0[0] - sums[0];
  if (st == 0 && !isfinite(Lv)) st |= LPS_ST_PSD;
  if (wv == 0 && lane == 0) {
    if (status) status[s] = st;
    logL[s] = st ? -INFINITY : Lv;
  }
  if (st) {
    if (wv == 0 && lane < n_params) dparams[lane * (size_t)n_states + s] = 0.0;
    for (int j = wv; j < n_spl; j += kWavesPerBlock) {
      int a, cn;
      knot_range(off, kcnt, s * n_spl + j, n_knots, a, cn);
      if (a < 0) continue;
      for (int i = lane; i < cn; i += kWave) {
        dkx[a + i] = 0.0;
        dky[a + i] = 0.0;
      }
    }
    return;
  }
  for (int g = wv; g < G; g += kWavesPerBlock)
    stitch_group(lane, s, g, G, NV, n_chunks, n_int[s * G + g], org, bx, rec, gidx, glast, moments, L.mo[g]);
  __syncthreads();
  if (wv == 0) {
    const double a_oms = params[LPS_P_AOMS * (size_t)n_states + s];
    const double a_tm = params[LPS_P_ATM * (size_t)n_states + s];
    double r_oms = sums[1], r_tm = sums[2];
    double du = 0.0, dalpha = 0.0;
    for (int g = 0; g < G; ++g) {
      const int ni = n_int[s * G + g];
      double m0 = 0.0, m1x = 0.0;
      if (lane < ni) {
        const double b = bx[(size_t)(s * G + g) * kMaxKnots + lane];
        m0 = L.mo[g][lane][0];
        m1x = L.mo[g][lane][1] + (b - x_knee) * m0;
      }
      m0 = wave_sum(m0);
      m1x = wave_sum(m1x);
      switch (lay.grp_kind[g]) {
        case kGOms: r_oms = m0; break;
        case kGTm: r_tm = m0; break;
        case kGSgwb:
          du = kLn10 * m0;
          dalpha = kLn10 * m1x;
          break;
        default: break;
      }
    }
    if (lane == 0) {
      dparams[LPS_P_AOMS * (size_t)n_states + s] = 2.0 * r_oms / a_oms;
      dparams[LPS_P_ATM * (size_t)n_states + s] = 2.0 * r_tm / a_tm;
      dparams[LPS_P_U * (size_t)n_states + s] = du;
      dparams[LPS_P_ALPHA * (size_t)n_states + s] = dalpha;
      if (n_params > 4) dparams[LPS_P_UFG * (size_t)n_states + s] = kLn10 * sums[3];
    }
  }
  // spline knots: the moments of every group fed by the spline, summed in group order
  for (int j = wv; j < n_spl; j += kWavesPerBlock) {
    int a, n;
    knot_range(off, kcnt, s * n_spl + j, n_knots, a, n);
    if (n == 0) continue;
    double M[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane + 1 < n) {
      for (int g = 0; g < G; ++g) {
        if (lay.grp_spline[g] != j) continue;
#pragma unroll
        for (int p = 0; p < 4; ++p) M[p] += kLn10 * L.mo[g][lane][p];
      }
    }
    spline_backward_wave(lane, kx + a, ky + a, n, M, dky + a, dkx + a, L.back[wv]);
  }
}

template <typename R, int B>
hipError_t dispatch_grad(lps_ctx* ctx, int n, int n_chunks, int n_tiles, int tile, const R* tab, const R* coef,
                         int NV, R* rec, int2* gidx, double* glast, double* lrec, hipStream_t s) {
  const Layout& L = ctx->lay;
  const int items = n_chunks * n_tiles;
  dim3 grid((items + kWavesPerBlock - 1) / kWavesPerBlock), block(kWave * kWavesPerBlock);
  const int k_pad = sizeof(R) == 4 ? ctx->k_pad32 : ctx->k_pad64;
#define LPS_GRAD(MODE, NCH, FG)                                                                            \
  hipLaunchKernelGGL((k_grad<R, MODE, NCH, FG, B>), grid, block, 0, s, n, n_chunks, n_tiles, tile,       \
                     ctx->n_bins, k_pad, kChunk32, tab, ctx->x, ctx->bx, coef, ctx->coef64, ctx->n_int,       \
                     ctx->scal, rec,                                                                          \
                     gidx, glast, ctx->moments, lrec)
  const bool fg = L.has_fg != 0;
  if (L.mode == kSplit && L.nch == 2 && !fg) LPS_GRAD(kSplit, 2, false);
  else if (L.mode == kSplit && L.nch == 2 && fg) LPS_GRAD(kSplit, 2, true);
  else if (L.mode == kSplit && L.nch == 3 && !fg) LPS_GRAD(kSplit, 3, false);
  else if (L.mode == kSplit && L.nch == 3 && fg) LPS_GRAD(kSplit, 3, true);
  else if (L.mode == kShared && L.nch == 2 && !fg) LPS_GRAD(kShared, 2, false);
  else if (L.mode == kShared && L.nch == 2 && fg) LPS_GRAD(kShared, 2, true);
  else if (L.mode == kShared && L.nch == 3 && !fg) LPS_GRAD(kShared, 3, false);
  else if (L.mode == kShared && L.nch == 3 && fg) LPS_GRAD(kShared, 3, true);
  else if (L.mode == kPaper && !fg) LPS_GRAD(kPaper, 3, false);
  else LPS_GRAD(kPaper, 3, true);
#undef LPS_GRAD
  return hipGetLastError();
}

int grad_nv(const Layout& L) {
  const int nvr = 4 + 4 * L.n_grp;
  return nvr <= 16 ? 16 : 32;
}

}  // namespace

size_t grad_workspace_bytes(const lps_ctx* ctx) {
  const size_t S = (size_t)ctx->max_grad_states;
  if (S == 0) return 256;
  const size_t nch = (size_t)((ctx->n_bins + kChunkGrad64 - 1) / kChunkGrad64);
  const size_t G = (size_t)ctx->lay.n_grp;
  const size_t nv = (size_t)grad_nv(ctx->lay);
  return S * nch * (nv * 8 + G * 8 + G * 4 * 8) + 256;
}

hipError_t launch_grad(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL, double* dparams,
                       double* dkx, double* dky, uint32_t* status, hipStream_t s) {
  const int n = st->n_states;
  hipError_t e = launch_coeffs(ctx, st, s);
  if (e != hipSuccess) return e;
  const bool mixed = prec == LPS_MIXED;
  const int chunk = mixed ? kChunkGrad32 : kChunkGrad64;
  const int n_chunks = (ctx->n_bins + chunk - 1) / chunk;
  const int G = ctx->lay.n_grp;
  const int NV = grad_nv(ctx->lay);
  // records in the working precision, then piece indices and last-piece
  // moments (the layout is sized for double records, so it always fits)
  const size_t rec_bytes = (size_t)n * n_chunks * NV * (mixed ? sizeof(float) : sizeof(double));
  char* base = (char*)ctx->gpartial;
  int2* gidx = (int2*)(base + ((rec_bytes + 15) & ~(size_t)15));
  double* glast = (double*)(gidx + (size_t)n * n_chunks * G);
  // mixed path: per-(state, chunk) logL partials in double after the last-piece
  // moments (single-precision records leave room for them in a layout sized
  // for double records of half the chunk length)
  double* lrec = mixed ? glast + (size_t)n * n_chunks * G * 4 : nullptr;
  // enough work items to fill the chip, at most 64 states (measured: 63, a
  // whole number of the 21-state sub-tiles of the split layout, was 9% slower
  // on 2,048 chains, whose 33 tiles of 63 leave a short last tile)
  const long target = 8192;
  long tile = ((long)n * n_chunks) / target;
  if (tile < 1) tile = 1;
  if (tile > 64) tile = 64;
  if (tile > n) tile = n;
  const int n_tiles = (n + (int)tile - 1) / (int)tile;
  timing_begin(ctx, s);
  const dim3 fgrid(n), fblock(kWave * kWavesPerBlock);   // one workgroup per state
  if (mixed) {
    float* rec = (float*)base;
    e = dispatch_grad<float, kBGrad32>(ctx, n, n_chunks, n_tiles, (int)tile, ctx->tab32, ctx->coef32, NV, rec, gidx,
                                       glast, lrec, s);
    if (e != hipSuccess) return e;
    timing_end(ctx, s);
    hipLaunchKernelGGL(k_grad_finish<float>, fgrid, fblock, 0, s, n, ctx->n_spl, ctx->n_params, NV, n_chunks,
                       ChunkOrigin{ctx->x, chunk}, ctx->lay, log10(ctx->f_knee), st->params, st->knot_off, st->knot_cnt, st->n_knots, st->knot_x, st->knot_y,
                       ctx->n_int, ctx->bx, rec, gidx, glast, ctx->moments, lrec, ctx->c0, ctx->status_ws, logL,
                       dparams, dkx, dky, status);
  } else {
    double* rec = (double*)base;
    e = dispatch_grad<double, kBGrad64>(ctx, n, n_chunks, n_tiles, (int)tile, ctx->tab64, ctx->coef64, NV, rec,
                                        gidx, glast, nullptr, s);
    if (e != hipSuccess) return e;
    timing_end(ctx, s);
    hipLaunchKernelGGL(k_grad_finish<double>, fgrid, fblock, 0, s, n, ctx->n_spl, ctx->n_params, NV, n_chunks,
                       ChunkOrigin{ctx->x, chunk}, ctx->lay, log10(ctx->f_knee), st->params, st->knot_off, st->knot_cnt, st->n_knots, st->knot_x, st->knot_y,
                       ctx->n_int, ctx->bx, rec, gidx, glast, ctx->moments, nullptr, ctx->c0, ctx->status_ws, logL,
                       dparams, dkx, dky, status);
  }
  return hipGetLastError();
}

}  // namespace lps
