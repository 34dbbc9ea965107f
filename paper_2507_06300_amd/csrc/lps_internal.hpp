// Internal definitions of the HIP library (not part of the C ABI).
//
// Representation used by the batched kernels.  Every (state, exponent group)
// is stored as a piecewise cubic in base-2 exponent units,
//
//     Q_g(x) = a_i + b_i t + c_i t^2 + d_i t^3,   t = x - bx_i,  x in [bx_i, bx_{i+1}),
//
// so that each perturbed PSD term is  Ktilde_g,c(f_k) * exp2(Q_g(x_k)).  Q_g
// folds in log2(10) * P_j (the Akima or linear spline of App. A), the state's
// amplitude relative to a reference amplitude, and, for the background, the
// power law alpha log2(10) (x - log10 f_knee) of Eq. (pl).  A disabled spline
// is one piece with c = d = 0.
//
// Per-bin tables are scaled by a reference PSD sigma_c(f_k) (the noise
// template at reference amplitudes) so that every single-precision quantity
// is O(1); the constant C0 = -sum N_k ln sigma_ck is kept in double.  In the
// split layout sigma_c is the OMS term alone (at the reference amplitude), so
// that the OMS row is exactly 1 and the kernels add the OMS group's factor
// without a product; its ratio to the whole noise stays below about 110 over
// the analysis band (the TM term dominates A and E only below a few mHz).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lps.h"

namespace lps {

constexpr int kMaxGroups = 4;
constexpr int kMaxKnots = 64;
constexpr int kWave = 64;

// Reference amplitudes defining the scaled units of the per-bin tables.
constexpr double kRefAoms = 15.0e-12;
constexpr double kRefAtm = 3.0e-15;
constexpr double kRefU = -12.0;
constexpr double kRefUfg = -38.0;

constexpr double kLog2_10 = 3.321928094887362347870319429489390175864831393;
constexpr double kLn2 = 0.693147180559945309417232121458176568075500134360;
constexpr double kLn10 = 2.302585092994045684017991454684364207601101488629;
constexpr double kPi = 3.141592653589793238462643383279502884197169399375;
constexpr double kClight = 299792458.0;
constexpr double kH0PerH = 1.0e5 / 3.0856775814913673e22;   // 100 km/s/Mpc in Hz

enum Mode : int { kSplit = 0, kShared = 1, kPaper = 2 };

// Kinds of exponent groups.
enum GroupKind : int { kGOms = 0, kGTm = 1, kGSgwb = 2, kGFg = 3, kGNoise = 4 };

// Routing classified at create time.
struct Layout {
  int mode;
  int nch;                       // 2: A and E merged (identical); 3: separate
  int has_fg;
  int n_grp;                     // exponent groups per state
  int grp_kind[kMaxGroups];
  int grp_spline[kMaxGroups];    // spline slot feeding the group, -1 = none
  int grp_channel[kMaxGroups];   // paper mode noise groups: channel, else -1
  int n_terms;                   // terms with a table: OMS, TM, SGWB (+FG)
  int n_tab;                     // per-bin table rows
};

// True when the scaled OMS row is exactly 1 (split layout: the tables are
// scaled by the OMS reference term, see the top of this file).
__host__ __device__ inline bool unit_oms_row(const Layout& L) { return L.mode == kSplit; }

// Per-bin table rows (same order in the FP64 and FP32 tables):
//   row 0                     : x (FP64 table) or x - x_chunk (FP32 table)
//   rows 1 .. n_terms*nch     : Ktilde[term][channel]
//   next nch rows             : N_k * Dtilde_c   (A/E merged: N (Dt_A + Dt_E))
//   last row                  : N_k * ln 2
__host__ __device__ inline int tab_k(int term, int c, int nch) { return 1 + term * nch + c; }
__host__ __device__ inline int tab_nd(int c, int n_terms, int nch) { return 1 + n_terms * nch + c; }
__host__ __device__ inline int tab_nl(int n_terms, int nch) { return 1 + n_terms * nch + nch; }

// Launch shape of a batched kernel: bins per lane (chunk = 64 x that) and
// states per tile; 0 selects the built-in default.
struct LaunchShape {
  int bins_per_lane;
  int tile;
};

// Per-state scalars written by the coefficient kernel.
struct StateScalars {
  double w_oms;     // (A_oms / ref)^2   (shared / paper modes)
  double w_tm;      // (A_tm / ref)^2
  double e_fg;      // 10^(u_fg - ref)   (constant foreground factor)
  double pad;
};

}  // namespace lps

// The opaque context.
struct lps_ctx {
  int device;
  int n_cu;        // compute units of the device (persistent grids)
  int32_t n_bins;
  int32_t k_pad64;        // bins padded to the FP64 chunk
  int32_t k_pad32;        // bins padded to the mixed chunk
  int32_t n_chunks64;
  int32_t n_chunks32;
  int32_t n_spl;
  int32_t n_params;
  int8_t route[4][3];
  int32_t k_max;
  int32_t max_states;
  int32_t max_grad_states;
  double f_knee;
  double arm_length;
  double x_first, x_last;   // log10 of the first and last bin (coverage test)
  double nk_uniform;        // the common N_k when every bin has the same one, else 0
  lps::Layout lay;

  // dataset copies (FP64)
  double* f;       // [K]
  double* nk;      // [K]
  double* D;       // [3][K]
  double* R;       // [3][K]
  double* Rfg;     // [3][K] or nullptr
  double* x;       // [K] log10 f
  double* sigma;   // [3][K] reference PSD used for scaling
  double* tmpl;    // [4][3][K] unscaled unit templates (OMS, TM per unit A^2; SGWB per unit h2Omega at alpha = 0; FG per unit amp)
  double* tab64;   // [n_tab][k_pad64]
  float* tab32;    // [n_tab][k_pad32]
  double* c0;      // [1] C0 = -sum N ln sigma

  // workspace (sized for max_states)
  double* bx;          // [max_states][n_grp][kMaxKnots]  piece start abscissae
  double* coef64;      // [max_states][n_grp][kMaxKnots][4]
  float* coef32;       // [max_states][n_grp][kMaxKnots][4]
  int32_t* n_int;      // [max_states][n_grp] pieces (0 = state invalid)
  lps::StateScalars* scal;   // [max_states]
  uint32_t* status_ws; // [max_states]
  double* partial;     // [max(n_chunks64, n_chunks32)][n_states] (chunk-major)
  double* run_sum;     // [kFinalizeRuns][n_states] partial sums over runs of chunks
  double* gpartial;    // gradient workspace (see lps_grad.hip)
  size_t gpartial_bytes;
  double* moments;     // [max_grad_states][n_grp][kMaxKnots][4] per-piece adjoint moments
  double* plain_part;  // [max_states][plain blocks]
  int32_t plain_blocks;
  uint32_t* sticky;    // [1] device error flags
  // (state, chunk) pairs of a mixed call whose single-precision partial is not
  // finite, re-evaluated in double range before the final sums
  int2* wide_list;     // [wide_cap]
  uint32_t* wide_count;  // [1], cleared by the coefficient kernel of every call
  int32_t wide_cap;

  // launch shapes of the forward kernel: [0] FP64, [1] mixed
  lps::LaunchShape fwd_shape[2];

  // timing
  int timing;
  hipEvent_t ev0, ev1;
  double time_ms;
  int32_t time_launches;
};

namespace lps {

// Launchers implemented in the .hip files.
hipError_t build_tables(lps_ctx* ctx, hipStream_t s);
// Maps a HIP result to a status; a failure is remembered (per host thread)
// for lps_last_device_error.
lps_status device_status(hipError_t e);

hipError_t launch_coeffs(lps_ctx* ctx, const lps_states* st, hipStream_t s);
hipError_t launch_forward(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL,
                          uint32_t* status, hipStream_t s);
hipError_t launch_psd(lps_ctx* ctx, const lps_states* st, int32_t k0, int32_t k1, double* S,
                      double* Sn, double* Sh, uint32_t* status, hipStream_t s);
hipError_t launch_plain(lps_ctx* ctx, const lps_states* st, double* logL, uint32_t* status,
                        hipStream_t s);
hipError_t launch_grad(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL,
                       double* dparams, double* dkx, double* dky, uint32_t* status, hipStream_t s);
size_t grad_workspace_bytes(const lps_ctx* ctx);
LaunchShape forward_shape(const lps_ctx* ctx, lps_precision prec, int n_states);
int sub_states(const lps_ctx* ctx, lps_precision prec);
bool valid_bins_per_lane(lps_precision prec, int b);

// Chunk geometry of the batched kernels.
constexpr int kWavesPerBlock = 4;
constexpr int kB64 = 4;                        // bins per lane, FP64 kernel
constexpr int kB32 = 8;                        // bins per lane, mixed kernel
// Bins of a lane that share one reciprocal (and, with a uniform N_k, one
// logarithm) in the batched forward kernel.
constexpr int kMergeBins = 4;
constexpr int kChunk64 = kWave * kB64;         // 256 bins per wave
constexpr int kChunk32 = kWave * kB32;         // 512 bins per wave

// Origin of the single-precision abscissa row of the table block that starts
// at bin kb (kChunk32 consecutive bins): the midpoint of the block's first and
// last bin abscissae, so that |x - origin| is at most half the block's span.
__host__ __device__ inline double block_origin(const double* x, int kb, int K) {
  const int k0 = kb < K ? kb : K - 1;
  const int k1 = kb + kChunk32 - 1 < K ? kb + kChunk32 - 1 : K - 1;
  return 0.5 * (x[k0] + x[k1]);
}

constexpr int kPlainBlock = 256;

// The batched forward adds a state's chunk partials in this many runs of
// consecutive chunks (fewer where there are fewer chunks), then adds the runs.
constexpr int kFinalizeRuns = 64;

// A piece whose cubic term changes its exponent by at most this much (log2
// units, 4e-8 relative in 2^Q: under one unit in the last place of a single-
// precision result) anywhere in a chunk is evaluated as a quadratic there.
constexpr double kQuadTol = 1.0 / (1 << 24);

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline float wave_sumf(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The chip's eight XCDs (each with its own L2) receive workgroups round-robin
// by workgroup index.  xcd_block renumbers the grid so that each XCD works
// through one contiguous range of logical blocks; a bijection on [0, n).
constexpr int kXcds = 8;
constexpr int kTileGroup = 8;       // forward: state tiles that share a chunk's table rows in L2
constexpr int kTileGroupGrad = 4;   // adjoint (its records per state tile fill L2 sooner)
// Forward kernel grid: with kForwardPersistent, kPersistBlocksPerCu workgroups
// per CU whose waves stride over the work items; else one item per wave.  On
// the one-year workload the persistent grid measured 2.9-3.3 ms against
// 2.62 ms for one item per wave (2, 3, 4 and 6 workgroups per CU; the
// hardware dispatcher balances the uneven items better than a fixed stride).
constexpr bool kForwardPersistent = false;
constexpr int kPersistBlocksPerCu = 3;
__device__ inline int xcd_block(int b, int n) {
  const int q = n / kXcds, r = n % kXcds;
  const int x = b % kXcds, local = b / kXcds;
  return x * q + (x < r ? x : r) + local;
}

// Optional event timing of a main kernel (synchronises; never used under capture).
inline void timing_begin(lps_ctx* ctx, hipStream_t s) {
  if (ctx->timing) (void)hipEventRecord(ctx->ev0, s);
}
inline void timing_end(lps_ctx* ctx, hipStream_t s) {
  if (!ctx->timing) return;
  (void)hipEventRecord(ctx->ev1, s);
  (void)hipEventSynchronize(ctx->ev1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
  ctx->time_ms += ms;
  ctx->time_launches += 1;
}

}  // namespace lps
