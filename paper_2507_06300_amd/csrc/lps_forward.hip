// Batched forward pass: logL for every state in one launch.
//
// Work item = (state tile, wave chunk of 64*B consecutive bins).  A wave
// keeps its B bins' table rows in registers for the whole tile and loops over
// the tile's states, so the shared per-bin data are read from memory once per
// tile, not once per state.  States are taken in sub-tiles of 64/G: lane p
// locates the piece of (state p / G, group p % G) that holds the chunk's first
// bin (binary search over the breakpoints), checks whether the next
// breakpoint falls inside the chunk, and stages the piece's cubic (and, for a
// crossing chunk, the next piece's) in LDS; ballots mark crossing and invalid
// pairs.  For the single-precision path each cubic is re-expanded in FP64
// about an origin inside the stretch it covers (the table block's midpoint for
// a piece that covers the whole chunk), so each bin's Horner runs on the stored
// abscissa plus a small offset with well-conditioned coefficients.
// Each bin then evaluates
//   E_g = exp2(Q_g(x)),  S_c = sum of template rows times E_g  (Eq. (splines)),
//   l   = sum_c N_k (D~_ck / S~_ck + ln S~_ck)
// in scaled units with one reciprocal and one logarithm for all channels.  A
// state whose chunk lies inside one piece of every group (the usual case)
// runs a straight-line body; a crossing state selects the piece per bin.
// Lane sums are stored transposed in LDS and one lane per state adds the 64
// of them in a fixed order, in double, giving one partial per (state, chunk),
// stored chunk-major so that a tile's partials of one chunk are contiguous.
// Two small kernels then add the partials of a state in a fixed order (runs
// of consecutive chunks, then the runs in order) and the scaling constant C0:
//   logL = C0 - sum_chunks partial.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "lps_batched.hpp"

namespace lps {
namespace {

// 2^q and log2(v) over the double-precision range with single-precision
// accuracy: the integer part of the exponent is applied exactly (ldexp /
// frexp) and only the fraction goes through the hardware transcendental.
__device__ inline double exp2_wide(double q) {
  const double n = fmin(fmax(floor(q), -2100.0), 2100.0);
  return ldexp((double)__builtin_amdgcn_exp2f((float)(q - n)), (int)n);
}
__device__ inline double log2_wide(double v) {
  int e = 0;
  const double m = frexp(v, &e);
  return (double)e + (double)__builtin_amdgcn_logf((float)m);
}

// One lane's bins k = kbase + b*64 + lane (b < nb) of state s, evaluated from
// the FP64 tables and pieces in double range at single-precision accuracy;
// the piece of each group is located once and then advanced along the lane's
// increasing abscissae.
template <int MODE, int NCH, bool FG>
__device__ double lane_terms_wide(int s, int kbase, int nb, int lane, int K, int k_pad,
                                  const double* __restrict__ tab64, const double* __restrict__ bx,
                                  const double* __restrict__ coef64, const int32_t* __restrict__ n_int,
                                  const StateScalars* __restrict__ scal) {
  constexpr int G = Groups<MODE>::G;
  constexpr int NT = FG ? 4 : 3;
  const StateScalars sc = scal[s];
  auto row = [&](int r, int k) { return tab64[(size_t)r * k_pad + k]; };
  int piece[G];
#pragma unroll
  for (int g = 0; g < G; ++g) piece[g] = -1;
  double acc = 0.0;
#pragma unroll 1
  for (int b = 0; b < nb; ++b) {
    const int k = kbase + b * kWave + lane;
    if (k >= K) break;
    const double x = row(0, k);
    double S[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) S[c] = FG ? row(tab_k(3, c, NCH), k) * sc.e_fg : 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const size_t base = (size_t)(s * G + g) * kMaxKnots;
      const int ni = n_int[s * G + g];
      int i = piece[g];
      if (i < 0) {
        i = count_le(bx + base, ni, x);
      } else {
        while (i + 1 < ni && bx[base + i + 1] <= x) ++i;
      }
      piece[g] = i;
      const double* cf = coef64 + (base + i) * 4;
      const double t = x - bx[base + i];
      const double E = exp2_wide(cf[0] + t * (cf[1] + t * (cf[2] + t * cf[3])));
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        if constexpr (MODE == kSplit) {
          S[c] += row(tab_k(g, c, NCH), k) * E;
        } else if constexpr (MODE == kShared) {
          S[c] += (g == 0 ? sc.w_oms * row(tab_k(0, c, NCH), k) + sc.w_tm * row(tab_k(1, c, NCH), k)
                          : row(tab_k(2, c, NCH), k)) * E;
        } else {
          if (g < 3) {
            if (c == g) S[c] += (sc.w_oms * row(tab_k(0, c, NCH), k) + sc.w_tm * row(tab_k(1, c, NCH), k)) * E;
          } else {
            S[c] += row(tab_k(2, c, NCH), k) * E;
          }
        }
      }
    }
    const double nl = row(tab_nl(NT, NCH), k);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const double lw = (NCH == 2 && c == 0) ? 2.0 : 1.0;
      acc += row(tab_nd(c, NT, NCH), k) / S[c] + lw * nl * log2_wide(S[c]);
    }
  }
  return acc;
}

// The double-range pass of the mixed path: one wave per queued (state, chunk),
// a fixed grid of eight workgroups per CU striding over the queue (empty in
// the usual case).  The chunk's
// partial is replaced by the fixed-order wave sum of its bins' terms.
template <int MODE, int NCH, bool FG>
__global__ __launch_bounds__(256) void k_wide(int n_chunks, int chunk_bins, int K, int k_pad,
                                              const double* __restrict__ tab64, const double* __restrict__ bx,
                                              const double* __restrict__ coef64, const int32_t* __restrict__ n_int,
                                              const StateScalars* __restrict__ scal,
                                              const uint32_t* __restrict__ wide_count,
                                              const int2* __restrict__ wide_list, int wide_cap, int n_states,
                                              double* __restrict__ partial) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
  const int nw = gridDim.x * kWavesPerBlock;
  const int n = min((int)*wide_count, wide_cap);
  for (int i = w; i < n; i += nw) {
    const int2 it = wide_list[i];
    const int s = uniform(it.x), chunk = uniform(it.y);
    const double d = wave_sum(lane_terms_wide<MODE, NCH, FG>(s, chunk * chunk_bins, chunk_bins / kWave, lane, K,
                                                             k_pad, tab64, bx, coef64, n_int, scal));
    if (lane == 0) partial[(size_t)chunk * n_states + s] = d;
  }
}

// Waves per SIMD the register allocation must allow: four for the
// single-precision split layout with merged A/E rows, no foreground and eight
// bins per lane (the one-year workload's kernel: 128 registers and no
// spills, 5-7 % faster than three waves at 141
// registers); the other instantiations would spill inside their bin loops at
// four (the paper layout ran 6x slower) and keep the compiler's choice.  (The
// FP64 kernel of the same layout at four bins per lane, capped at three waves,
// ran about 1 % faster but spilled 68 bytes per lane, written once per wave:
// 0.66 GB more HBM writes per launch.)
template <typename R, int MODE, int NCH, bool FG, int B>
struct FwdWaves {
  static constexpr int v = (sizeof(R) == 4 && MODE == kSplit && NCH == 2 && !FG && B == 8) ? 4 : 1;
};

template <typename R, int MODE, int NCH, bool FG, int B, int M, bool UNI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FwdWaves<R, MODE, NCH, FG, B>::v))) void k_forward(int n_states, int n_chunks, int n_tiles, int tile, int K,
                                                 int k_pad, int ref_chunk, R nl_uni, const R* __restrict__ tab,
                                                 const double* __restrict__ x64, const double* __restrict__ bx,
                                                 const R* __restrict__ coef, const double* __restrict__ coef64,
                                                 uint32_t* __restrict__ wide_count, int2* __restrict__ wide_list,
                                                 int wide_cap,
                                                 const int32_t* __restrict__ n_int,
                                                 const StateScalars* __restrict__ scal,
                                                 double* __restrict__ partial) {
  constexpr int G = Groups<MODE>::G;
  constexpr int NT = FG ? 4 : 3;
  constexpr int CH = kWave * B;
  constexpr bool kMixed = sizeof(R) == 4;
  // states whose pieces one wave locates at once (fewer for FP64 to bound LDS)
  constexpr int SUB = (kWave / G) < (kMixed ? 32 : 16) ? (kWave / G) : (kMixed ? 32 : 16);
  // Single precision: each staged piece's cubic is re-expanded in FP64 around
  // an origin inside the stretch of the chunk that the piece covers (the table
  // block's midpoint when the piece covers the whole chunk, else the chunk
  // start or the piece's own start), so that the per-bin Horner runs on
  // x - origin = (table abscissa) + (small offset) with well-conditioned
  // coefficients: a short, steep piece expanded about a distant point would
  // lose its value to cancellation.
  constexpr bool kLocalPoly = kMixed;
  constexpr bool kScalars = FG || MODE != kSplit;
  // Per wave: the located piece of every (state, group) pair of the sub-tile
  // (a, b, c, d, offset), the per-state scalars, and the per-state lane
  // partials stored transposed (red[source lane][state]).
  using Acc = typename std::conditional<kMixed, float, double>::type;
  using R4 = typename std::conditional<kMixed, float4, double4>::type;
  __shared__ R4 lcoef[kWavesPerBlock][kWave];
  __shared__ R loff[kWavesPerBlock][kWave];
  __shared__ R4 lcoef2[kWavesPerBlock][kWave];   // next piece of a chunk that crosses one breakpoint
  __shared__ R loff2[kWavesPerBlock][kWave];
  __shared__ R lscal[kWavesPerBlock][SUB][4];
  __shared__ Acc red[kWavesPerBlock][kWave * SUB];
  // FP64: the table of 2^(j/64) for exp2_t
  __shared__ double lexp2[kMixed ? 1 : kExp2Tab];
  if constexpr (!kMixed) {
    fill_exp2_table(lexp2, (int)threadIdx.x);
    __syncthreads();
  }
  // 2^q: the hardware instruction in single precision, the table in FP64
  auto ex2 = [&](R q) -> R {
    if constexpr (kMixed) return Math<R>::exp2_(q);
    else return exp2_t(q, lexp2);
  };
  const int lane = threadIdx.x & (kWave - 1);
  // wave-uniform work-item index: keeps all per-state addressing scalar
  const int wv = uniform(threadIdx.x >> 6);
  // Work order: the tiles are taken kTileGroup at a time; within a group the
  // items run chunk by chunk with the group's tiles innermost, and each XCD
  // walks one contiguous range of that order.  A chunk's table rows then
  // reach an XCD's L2 once per tile group instead of once per tile, while the
  // group's state records (pieces, breakpoints) stay resident in that L2.
  // A wave takes items first, first + stride, ... (one item when the grid has
  // a wave per item; a persistent grid of a few workgroups per CU strides).
  const int n_items = n_chunks * n_tiles;
  const int stride = gridDim.x * kWavesPerBlock;
  for (int item = xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wv; item < n_items; item += stride) {
  const int tg = item / (n_chunks * kTileGroup);
  const int rem = item - tg * (n_chunks * kTileGroup);
  const int tl = min(kTileGroup, n_tiles - tg * kTileGroup);   // tiles in this group
  if (tl <= 0) continue;
  const int chunk = rem / tl;
  const int t = tg * kTileGroup + (rem - chunk * tl);
  if (chunk >= n_chunks) continue;
  const int s_begin = t * tile;
  const int s_end = min(s_begin + tile, n_states);
  const int kbase = chunk * CH;

  // per-bin rows for this lane's B bins (lane-strided, coalesced); with a
  // uniform N_k the log weight is the scalar nl_uni and needs no row
  R xr[B], NL[UNI ? 1 : B];
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
    if constexpr (!UNI) NL[b] = tab[(size_t)tab_nl(NT, NCH) * k_pad + k];
  }
  // bins of this chunk past the last one (the padded tail of the final chunk)
  const bool tail = kbase + CH > K;
  const int klast = min(kbase + CH, K) - 1;
  const double xf = x64[kbase];
  const double xl = x64[klast];
  // abscissa origin of the single-precision table rows (midpoint of their block)
  const double xo = kMixed ? block_origin(x64, (kbase / ref_chunk) * ref_chunk, K) : 0.0;
  // the chunk's half-span about xo (a cubic term d dx^3 over the chunk has
  // |dx| <= h3r), uniform: a scalar register pair for the whole work item
  const double h3r = readlane_r(fmax(xl - xo, xo - xf), 0);

  for (int sub = s_begin; sub < s_end; sub += SUB) {
    const int nsub = min(SUB, s_end - sub);
    // the lane index, opaque to the compiler here: the LDS addresses below are
    // formed again per sub-tile instead of being held (and spilled) across the
    // whole work item
    int ln = lane;
    asm volatile("" : "+v"(ln));
    // ---- locate: lane p owns the piece of (state sub + p / G, group p % G) ----
    const int ps = lane / G, pg = lane - (lane / G) * G;
    const bool pv = ps < nsub && ps < SUB;
    const size_t pbase = (size_t)((sub + ps) * G + pg) * kMaxKnots;
    const int pni = pv ? n_int[(sub + ps) * G + pg] : 0;
    int pi0 = 0, pi1 = 0;
    bool pquad = true;
    if (pni > 0) {
      pi0 = count_le(bx + pbase, pni, xf);
      // the chunk usually ends in the piece it starts in: one more breakpoint
      // decides, and only a crossing chunk searches for its last piece
      const double b_next = pi0 + 1 < pni ? bx[pbase + pi0 + 1] : (double)INFINITY;
      pi1 = b_next <= xl ? count_le(bx + pbase, pni, xl) : pi0;
      // record of piece i (breakpoint bi): cubic coefficients and abscissa
      // offset (single precision: about origin org, offset xo - org)
      auto piece_rec = [&](int i, double bi, double org, R4& r4, R& off) {
        if constexpr (kLocalPoly) {
          // Q(x) = a + b t + c t^2 + d t^3, t = x - bi = t0 + dx  ->  polynomial in dx = x - org
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
          off = kMixed ? (R)(xo - bi) : (R)(-bi);
        }
      };
      R4 r4;
      R off;
      // a piece that covers the whole chunk is expanded about the block
      // midpoint xo (offset 0); in a crossing chunk the first piece about the
      // chunk start and the next one about its own start
      piece_rec(pi0, bx[pbase + pi0], pi1 > pi0 ? xf : xo, r4, off);
      if constexpr (kLocalPoly) {
        // the cubic term d dx^3 over the chunk
        pquad = fabs(coef64[(pbase + pi0) * 4 + 3]) * h3r * h3r * h3r <= kQuadTol;
      }
      lcoef[wv][ln] = r4;
      loff[wv][ln] = off;
      if (pi1 > pi0) {
        // the chunk crosses breakpoint pi0 + 1: stage the next piece as well;
        // its offset is minus the abscissa (in the table's units) where it
        // takes over, (R)(xo - b1) in single precision and -b1 in FP64
        const double b1 = b_next;
        piece_rec(pi0 + 1, b1, b1, r4, off);
        lcoef2[wv][ln] = r4;
        loff2[wv][ln] = off;
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
    // pair lanes whose chunk straddles a breakpoint, and states that are invalid
    const unsigned long long straddle = __ballot(pv && pni > 0 && pi0 != pi1);
    const unsigned long long multi = __ballot(pv && pni > 0 && pi1 > pi0 + 1);
    // bit q*G set when any group of state q crosses a breakpoint in this chunk,
    // or needs the cubic term
    unsigned long long cross_state = straddle;
    const unsigned long long cubic = __ballot(pv && pni > 0 && !pquad);
    unsigned long long cubic_state = cubic;
#pragma unroll
    for (int g = 1; g < G; ++g) {
      cross_state |= straddle >> g;
      cubic_state |= cubic >> g;
    }
    const unsigned long long invalid = __ballot(pv && pg == 0 && pni == 0);
    wave_lds_sync();

    for (int q = 0; q < nsub; ++q) {
      const int s = sub + q;
      if ((invalid >> (q * G)) & 1ull) {   // invalid state: the finaliser reports it
        red[wv][lane * SUB + q] = (Acc)0;
        continue;
      }
      R w_oms = 0, w_tm = 0, e_fg = 0;
      if constexpr (kScalars) {
        w_oms = lscal[wv][q][0];
        w_tm = lscal[wv][q][1];
        e_fg = lscal[wv][q][2];
      }
      R S[NCH][B];
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int b = 0; b < B; ++b) S[c][b] = FG ? Kt[3][c][b] * e_fg : (R)0;
      // E = 2^Q of the piece staged for pair pl, for the lane's bins
      auto uniform_E = [&](int pl, R(&E)[B]) {
        const R4 c0 = lcoef[wv][pl];
        if constexpr (kLocalPoly) {
#pragma unroll
          for (int b = 0; b < B; ++b) E[b] = ex2(c0.x + xr[b] * (c0.y + xr[b] * (c0.z + xr[b] * c0.w)));
        } else {
          const R off = loff[wv][pl];
#pragma unroll
          for (int b = 0; b < B; ++b) {
            const R tt = xr[b] + off;
            E[b] = ex2(c0.x + tt * (c0.y + tt * (c0.z + tt * c0.w)));
          }
        }
      };
      // fold group g's factor into the channel PSDs
      auto fold = [&](int g, const R(&E)[B]) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          if constexpr (MODE == kSplit) {
            // the OMS row is 1 in this layout (the tables are scaled by it)
#pragma unroll
            for (int c = 0; c < NCH; ++c)
              S[c][b] = g == 0 ? (FG ? S[c][b] + E[b] : E[b]) : S[c][b] + Kt[g][c][b] * E[b];
          } else if constexpr (MODE == kShared) {
            // OMS and TM share the noise exponent; their amplitudes weight the rows
#pragma unroll
            for (int c = 0; c < NCH; ++c)
              S[c][b] += (g == 0 ? (w_oms * Kt[0][c][b] + w_tm * Kt[1][c][b]) : Kt[2][c][b]) * E[b];
          } else {
            if (g < 3) {
              S[g][b] += (w_oms * Kt[0][g][b] + w_tm * Kt[1][g][b]) * E[b];
            } else {
#pragma unroll
              for (int c = 0; c < NCH; ++c) S[c][b] += Kt[2][c][b] * E[b];
            }
          }
        }
      };
      if (!((cross_state >> (q * G)) & 1ull)) {
        // the usual case: the chunk lies inside one piece of every group, so
        // the state's body is straight-line code; where every group's cubic
        // term is below kQuadTol over the chunk (high frequencies, where a
        // chunk spans little of log10 f) the exponents are quadratics
        if (kLocalPoly && !((cubic_state >> (q * G)) & 1ull)) {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const R4 c0 = lcoef[wv][q * G + g];
            R E[B];
#pragma unroll
            for (int b = 0; b < B; ++b) E[b] = ex2(c0.x + xr[b] * (c0.y + xr[b] * c0.z));
            fold(g, E);
          }
        } else {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            R E[B];
            uniform_E(q * G + g, E);
            fold(g, E);
          }
        }
      } else {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int pl = q * G + g;
          const bool str = (straddle >> pl) & 1ull;
          const bool mul = (multi >> pl) & 1ull;
          R Q[B] = {};
          if (mul) {   // several breakpoints inside the chunk: each piece from memory, select per bin
            const int i0 = __builtin_amdgcn_readlane(pi0, pl);
            const int i1 = __builtin_amdgcn_readlane(pi1, pl);
            const size_t base = (size_t)(s * G + g) * kMaxKnots;
            for (int j = i0; j <= i1; ++j) {
              const R* cf = coef + (base + j) * 4;
              const double bj = bx[base + j];
              // the first piece as staged (expanded about the chunk start); the
              // later ones start inside the chunk and are used about their start
              const bool first = kLocalPoly && j == i0;
              const R4 c0 = lcoef[wv][pl];
              const R a = first ? c0.x : cf[0], bb = first ? c0.y : cf[1];
              const R cc = first ? c0.z : cf[2], dd = first ? c0.w : cf[3];
              const R off = first ? loff[wv][pl] : (kMixed ? (R)(xo - bj) : (R)(-bj));
              const R lim = kMixed ? (R)(bj - xo) : (R)bj;   // bin is in piece j when xr >= lim
#pragma unroll
              for (int b = 0; b < B; ++b) {
                const R tt = xr[b] + off;
                const R qv = a + tt * (bb + tt * (cc + tt * dd));
                Q[b] = (j == i0 || xr[b] >= lim) ? qv : Q[b];
              }
            }
          } else {     // at most one breakpoint: both staged pieces from LDS, select per bin
            const R4 c0 = lcoef[wv][pl];
            const R4 c1 = lcoef2[wv][pl];
            const R o0 = loff[wv][pl], o2 = loff2[wv][pl];
            const R lim = str ? -o2 : (R)INFINITY;
            const R o1 = str ? o2 : o0;
#pragma unroll
            for (int b = 0; b < B; ++b) {
              const bool second = xr[b] >= lim;
              const R4 cc = second ? c1 : c0;
              const R t = xr[b] + (second ? o1 : o0);
              Q[b] = cc.x + t * (cc.y + t * (cc.z + t * cc.w));
            }
          }
          R E[B];
#pragma unroll
          for (int b = 0; b < B; ++b) E[b] = ex2(Q[b]);
          fold(g, E);
        }
      }
      // Per bin, all channels at once:
      //   sum_c ND_c / S_c = num / P,  P = prod_c S_c,
      //   sum_c w_c ln S_c = ln2 log2 L,  L = prod_c S_c^w_c  (w = 2 for the merged A/E row).
      // Groups of M consecutive bins of the lane then share one reciprocal,
      //   num_a / P_a + num_b / P_b = (num_a P_b + num_b P_a) / (P_a P_b),
      // and, when every bin carries the same N_k, one logarithm,
      //   N ln2 (log2 L_a + log2 L_b) = N ln2 log2 (L_a L_b).
      // A lane whose group products are not normal numbers (an extreme state
      // left the single-precision range) takes the per-channel path below.
      // L = P S0 (merged A/E) or P (three channels): a group's product of L is
      // the product of P times, for the merged rows, the product of S0.
      R v = 0;
      R Pm[B], Nm[B], Lm[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if constexpr (NCH == 2) {
          Pm[b] = S[0][b] * S[1][b];
          Nm[b] = ND[1][b] * S[0][b] + ND[0][b] * S[1][b];
          Lm[b] = UNI ? S[0][b] : Pm[b] * S[0][b];
        } else {
          const R P01 = S[0][b] * S[1][b];
          Pm[b] = P01 * S[2][b];
          Nm[b] = S[2][b] * (ND[1][b] * S[0][b] + ND[0][b] * S[1][b]) + ND[2][b] * P01;
          Lm[b] = UNI ? (R)1 : Pm[b];
        }
      }
      if constexpr (UNI) {
        // padded bins of the final chunk: N = 0 there, so their log term is
        // dropped (L = 1: P and S0 set to 1; their num is 0)
        if (tail) {
#pragma unroll
          for (int b = 0; b < B; ++b) {
            const bool in = kbase + b * kWave + lane < K;
            Lm[b] = in ? Lm[b] : (R)1;
            Pm[b] = in ? Pm[b] : (R)1;
          }
        }
      }
#pragma unroll
      for (int w = 1; w < M; w *= 2)
#pragma unroll
        for (int b = 0; b < B; b += 2 * w) {
          Nm[b] = Nm[b] * Pm[b + w] + Nm[b + w] * Pm[b];
          Pm[b] = Pm[b] * Pm[b + w];
          if constexpr (UNI && NCH == 2) Lm[b] = Lm[b] * Lm[b + w];
        }
      if constexpr (UNI) {
#pragma unroll
        for (int b = 0; b < B; b += M) Lm[b] = NCH == 2 ? Pm[b] * Lm[b] : Pm[b];
      }
      bool ok = true;
      // With a uniform N_k the lane's B bins need one logarithm: the group
      // products are split into mantissa and exponent, the mantissas (in
      // [1/2, 1)) multiplied and the exponents added exactly, so the hardware
      // logarithm only sees an argument in [2^-(B/M), 1) and its error does not
      // grow with the size of log2 L.
      R mprod = 1;
      int esum = 0;
#pragma unroll
      for (int b = 0; b < B; b += M) {
        v += Nm[b] * Math<R>::rcp_(Pm[b]);
        ok = ok && __builtin_isnormal(Pm[b]);
        if constexpr (UNI) {
          int e;
          mprod *= frexp(Lm[b], &e);
          esum += e;
          ok = ok && __builtin_isnormal(Lm[b]);
        }
      }
      if constexpr (UNI) {
        v += nl_uni * (Math<R>::log2_(mprod) + (R)esum);
      } else {
        // one logarithm per bin; in single precision again on the mantissa
        // alone: the hardware logarithm's bias is a fraction of the result's
        // last place, which for log2 L of tens would add up coherently over
        // the bins of a state
#pragma unroll
        for (int b = 0; b < B; ++b) {
          if constexpr (kMixed) {
            int e;
            const R m = frexp(Lm[b], &e);
            v += NL[b] * (Math<R>::log2_(m) + (R)e);
            ok = ok && __builtin_isnormal(Lm[b]);
          } else {
            v += NL[b] * Math<R>::log2_(Lm[b]);
          }
        }
      }
      Acc acc = (Acc)v;
      if (!ok || !isfinite(acc)) {
        // A channel product left the floating-point range (an extreme state):
        // redo the lane's bins with one reciprocal and logarithm per channel, so
        // that only a non-finite or vanishing channel PSD marks the state.
        R w = 0;
#pragma unroll
        for (int b = 0; b < B; ++b) {
          R nl;
          if constexpr (UNI) nl = kbase + b * kWave + lane < K ? nl_uni : (R)0;
          else nl = NL[b];
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const R lw = (NCH == 2 && c == 0) ? (R)2 : (R)1;
            int e;
            const R m = frexp(S[c][b], &e);
            w += ND[c][b] * Math<R>::rcp_(S[c][b]) + (lw * nl) * (Math<R>::log2_(m) + (R)e);
          }
        }
        acc = (Acc)w;
      }
      red[wv][lane * SUB + q] = acc;
    }
    // The 64 lane partials of each state are added in double by LP lanes, each
    // taking a fixed run of them, and the LP sums are then added in lane order
    // (lane LP q ends with the total of state sub + q): a fixed order throughout.
    wave_lds_sync();
    {
      constexpr int LP = kWave / SUB;
      constexpr int RUN = (kWave + LP - 1) / LP;
      const int q = lane / LP, r = lane - q * LP;
      const bool mine = q < nsub;
      double sum = 0.0;
      if (mine) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
        for (int i = 0; i < RUN; i += 2) {
          const int i0 = r * RUN + i;
          if (i0 < kWave && i < RUN) s0 += (double)red[wv][i0 * SUB + q];
          if (i0 + 1 < kWave && i + 1 < RUN) s1 += (double)red[wv][(i0 + 1) * SUB + q];
        }
        sum = s0 + s1;
      }
      double tot = sum;
#pragma unroll
      for (int d = 1; d < LP; ++d) tot += __shfl_down(sum, d, kWave);
      if (mine && r == 0) {
        partial[(size_t)chunk * n_states + (sub + q)] = tot;
        if (kMixed && !isfinite(tot)) {
          // a channel PSD left the single-precision range (a wildly swinging
          // spline): queue the (state, chunk) for the double-range pass
          const unsigned slot = atomicAdd(wide_count, 1u);
          if (slot < (unsigned)wide_cap) wide_list[slot] = make_int2(sub + q, chunk);
        }
      }
    }
    wave_lds_sync();
  }
  }   // items
}

// Sum of the partials of chunks [run * run_len, (run + 1) * run_len) of every
// state, one lane per state (the chunk-major partials make each load of a
// wave one contiguous row); eight interleaved sums, so that eight loads are in
// flight, added in a fixed order.
__global__ __launch_bounds__(kWave) void k_finalize_runs(int n_states, int n_chunks, int run_len,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ run_sum) {
  const int s = blockIdx.x * kWave + threadIdx.x;
  const int run = blockIdx.y;
  if (s >= n_states) return;
  const int c0 = run * run_len, c1 = min(n_chunks, c0 + run_len);
  const double* p = partial + s;
  const size_t n = (size_t)n_states;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int c = c0;
  for (; c + 7 < c1; c += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[(c + u) * n];
  for (; c < c1; ++c) a[0] += p[c * n];
  run_sum[(size_t)run * n + s] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// logL = C0 - the runs' sums added in run order (all loads issued first); the
// state's status word.
__global__ __launch_bounds__(256) void k_finalize(int n_states, int n_runs, const double* __restrict__ run_sum,
                                                  const double* __restrict__ c0,
                                                  const uint32_t* __restrict__ status_ws, double* __restrict__ logL,
                                                  uint32_t* __restrict__ status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_states) return;
  double v[kFinalizeRuns];
#pragma unroll
  for (int r = 0; r < kFinalizeRuns; ++r) v[r] = r < n_runs ? run_sum[(size_t)r * n_states + s] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < kFinalizeRuns; ++r) acc += v[r];
  uint32_t st = status_ws[s];
  const double val = c0[0] - acc;
  if (st == 0 && !isfinite(val)) st |= LPS_ST_PSD;
  logL[s] = st ? -INFINITY : val;
  if (status) status[s] = st;
}

template <typename R, int B, bool UNI>
hipError_t dispatch(lps_ctx* ctx, int n, int n_chunks, int n_tiles, int tile, const R* tab, const R* coef,
                    hipStream_t s) {
  const Layout& L = ctx->lay;
  const int items = n_chunks * n_tiles;
  int blocks = (items + kWavesPerBlock - 1) / kWavesPerBlock;
  if (kForwardPersistent && ctx->n_cu > 0 && blocks > ctx->n_cu * kPersistBlocksPerCu)
    blocks = ctx->n_cu * kPersistBlocksPerCu;
  dim3 grid(blocks), block(kWave * kWavesPerBlock);
  const int k_pad = sizeof(R) == 4 ? ctx->k_pad32 : ctx->k_pad64;
  constexpr int M = kMergeBins < B ? kMergeBins : B;
  const R nl_uni = (R)(ctx->nk_uniform * kLn2);
#define LPS_FWD(MODE, NCH, FG)                                                                              \
  hipLaunchKernelGGL((k_forward<R, MODE, NCH, FG, B, M, UNI>), grid, block, 0, s, n, n_chunks, n_tiles, tile, \
                     ctx->n_bins, k_pad, kChunk32, nl_uni, tab, ctx->x, ctx->bx, coef, ctx->coef64,           \
                     ctx->wide_count, ctx->wide_list, ctx->wide_cap, ctx->n_int,                               \
                     ctx->scal,                                                                               \
                     ctx->partial)
  const bool fg = L.has_fg != 0;
  if (L.mode == kSplit && L.nch == 2 && !fg) LPS_FWD(kSplit, 2, false);
  else if (L.mode == kSplit && L.nch == 2 && fg) LPS_FWD(kSplit, 2, true);
  else if (L.mode == kSplit && L.nch == 3 && !fg) LPS_FWD(kSplit, 3, false);
  else if (L.mode == kSplit && L.nch == 3 && fg) LPS_FWD(kSplit, 3, true);
  else if (L.mode == kShared && L.nch == 2 && !fg) LPS_FWD(kShared, 2, false);
  else if (L.mode == kShared && L.nch == 2 && fg) LPS_FWD(kShared, 2, true);
  else if (L.mode == kShared && L.nch == 3 && !fg) LPS_FWD(kShared, 3, false);
  else if (L.mode == kShared && L.nch == 3 && fg) LPS_FWD(kShared, 3, true);
  else if (L.mode == kPaper && !fg) LPS_FWD(kPaper, 3, false);
  else LPS_FWD(kPaper, 3, true);
#undef LPS_FWD
  return hipGetLastError();
}

hipError_t dispatch_wide(lps_ctx* ctx, int n_states, int n_chunks, int chunk_bins, hipStream_t s) {
  const Layout& L = ctx->lay;
  // eight workgroups per CU: a queued chunk is a chain of dependent loads (the
  // piece search, then the pieces and table rows), so the pass needs many
  // waves in flight once the queue is long (measured on the one-year grid in
  // the paper's layout, 0.23 -> 0.09 ms beside the main kernel against one
  // workgroup per CU); with an empty queue every wave exits after one load
  const dim3 grid(ctx->n_cu > 0 ? ctx->n_cu * 8 : 2048), block(kWave * kWavesPerBlock);
#define LPS_WIDE(MODE, NCH, FG)                                                                               \
  hipLaunchKernelGGL((k_wide<MODE, NCH, FG>), grid, block, 0, s, n_chunks, chunk_bins, ctx->n_bins, ctx->k_pad64, \
                     ctx->tab64, ctx->bx, ctx->coef64, ctx->n_int, ctx->scal, ctx->wide_count, ctx->wide_list,  \
                     ctx->wide_cap, n_states, ctx->partial)
  const bool fg = L.has_fg != 0;
  if (L.mode == kSplit && L.nch == 2 && !fg) LPS_WIDE(kSplit, 2, false);
  else if (L.mode == kSplit && L.nch == 2 && fg) LPS_WIDE(kSplit, 2, true);
  else if (L.mode == kSplit && L.nch == 3 && !fg) LPS_WIDE(kSplit, 3, false);
  else if (L.mode == kSplit && L.nch == 3 && fg) LPS_WIDE(kSplit, 3, true);
  else if (L.mode == kShared && L.nch == 2 && !fg) LPS_WIDE(kShared, 2, false);
  else if (L.mode == kShared && L.nch == 2 && fg) LPS_WIDE(kShared, 2, true);
  else if (L.mode == kShared && L.nch == 3 && !fg) LPS_WIDE(kShared, 3, false);
  else if (L.mode == kShared && L.nch == 3 && fg) LPS_WIDE(kShared, 3, true);
  else if (L.mode == kPaper && !fg) LPS_WIDE(kPaper, 3, false);
  else LPS_WIDE(kPaper, 3, true);
#undef LPS_WIDE
  return hipGetLastError();
}

}  // namespace

// States whose pieces one wave locates at once (the kernel's sub-tile): 64/G
// pairs per wave, at most 32 (mixed) or 16 (FP64) states.
int sub_states(const lps_ctx* ctx, lps_precision prec) {
  const int per_wave = kWave / ctx->lay.n_grp;
  const int cap = prec == LPS_MIXED ? 32 : 16;
  return per_wave < cap ? per_wave : cap;
}

// States per tile: a whole number of sub-tiles (a tile that is not locates
// pieces for a partial one), six in single precision and four in FP64 (the
// fastest on the one-year workload), fewer when that leaves too few work items
// to fill the chip (~32 waves per CU).
int auto_tile(int n_states, int n_chunks, int sub, int subtiles) {
  const long target_items = 8192;
  long tile = (long)subtiles * sub;
  const long fill = ((long)n_states * n_chunks) / target_items;
  if (fill < tile) tile = fill >= sub ? (fill / sub) * sub : (fill < 1 ? 1 : fill);
  if (tile > n_states) tile = n_states;
  return (int)tile;
}

// Launch shape of the batched forward kernel for one precision.
LaunchShape forward_shape(const lps_ctx* ctx, lps_precision prec, int n_states) {
  LaunchShape sh = ctx->fwd_shape[prec == LPS_MIXED ? 1 : 0];
  if (sh.bins_per_lane == 0) sh.bins_per_lane = prec == LPS_MIXED ? kB32 : kB64;
  const int chunk = kWave * sh.bins_per_lane;
  const int n_chunks = (ctx->n_bins + chunk - 1) / chunk;
  if (sh.tile == 0) sh.tile = auto_tile(n_states, n_chunks, sub_states(ctx, prec), prec == LPS_MIXED ? 6 : 4);
  if (sh.tile > n_states) sh.tile = n_states;
  return sh;
}

hipError_t launch_forward(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL, uint32_t* status,
                          hipStream_t s) {
  const int n = st->n_states;
  hipError_t e = launch_coeffs(ctx, st, s);
  if (e != hipSuccess) return e;
  const bool mixed = prec == LPS_MIXED;
  const LaunchShape sh = forward_shape(ctx, prec, n);
  const int chunk = kWave * sh.bins_per_lane;
  const int n_chunks = (ctx->n_bins + chunk - 1) / chunk;
  const int n_tiles = (n + sh.tile - 1) / sh.tile;
  timing_begin(ctx, s);
  const bool uni = ctx->nk_uniform > 0.0;
  if (mixed) {
    if (sh.bins_per_lane == 4)
      e = uni ? dispatch<float, 4, true>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab32, ctx->coef32, s)
              : dispatch<float, 4, false>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab32, ctx->coef32, s);
    else
      e = uni ? dispatch<float, 8, true>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab32, ctx->coef32, s)
              : dispatch<float, 8, false>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab32, ctx->coef32, s);
  } else {
    if (sh.bins_per_lane == 2)
      e = uni ? dispatch<double, 2, true>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab64, ctx->coef64, s)
              : dispatch<double, 2, false>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab64, ctx->coef64, s);
    else
      e = uni ? dispatch<double, 4, true>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab64, ctx->coef64, s)
              : dispatch<double, 4, false>(ctx, n, n_chunks, n_tiles, sh.tile, ctx->tab64, ctx->coef64, s);
  }
  if (e != hipSuccess) return e;
  timing_end(ctx, s);
  if (mixed) {
    e = dispatch_wide(ctx, n, n_chunks, chunk, s);
    if (e != hipSuccess) return e;
  }
  // runs of consecutive chunks: their number depends on n_chunks alone, so a
  // state's sum order does not depend on the batch it is evaluated in
  const int n_runs = std::min(kFinalizeRuns, n_chunks);
  const int run_len = (n_chunks + n_runs - 1) / n_runs;
  hipLaunchKernelGGL(k_finalize_runs, dim3((n + kWave - 1) / kWave, n_runs), dim3(kWave), 0, s, n, n_chunks, run_len,
                     ctx->partial, ctx->run_sum);
  hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, s, n, n_runs, ctx->run_sum, ctx->c0,
                     ctx->status_ws, logL, status);
  return hipGetLastError();
}

bool valid_bins_per_lane(lps_precision prec, int b) {
  return prec == LPS_MIXED ? (b == 4 || b == 8) : (b == 2 || b == 4);
}

}  // namespace lps
