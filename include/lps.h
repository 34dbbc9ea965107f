/*
 * lps.h -- C ABI of the batched flexible-PSD / Whittle log-likelihood library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for a batch of MCMC states theta (every walker,
 * temperature and reversible-jump branch at once), the model of the paper
 * "A flexible, GPU-accelerated approach for the joint characterization of
 * LISA instrumental noise and Stochastic Gravitational Wave Backgrounds":
 *
 *   S_c(f_k) = sum_tau  T_tau,c(f_k) * amp_tau(theta) * 10^{P_{r(tau,c)}(log10 f_k)}
 *   logL     = - sum_{c in A,E,T} sum_k  N_k ( D_ck / S_ck + ln S_ck )
 *
 *  - T_OMS,c and T_TM,c: the A/E/T noise transfer of Eq. (noise_tdi) applied
 *    to the OMS and test-mass PSDs of Sec. "Parametrized noise model"
 *    (amp = A_OMS^2 and A_TM^2).  The TDI prefactor is sin^2(xi) sin^2(2 xi),
 *    xi = 2 pi f L / c (the second-generation delay polynomial).
 *  - T_SGWB,c = R_c(f) 3 (H0/h)^2 / (4 pi^2 f^3) with amp = 10^u (f/f_knee)^alpha:
 *    the power law of Eq. (pl) through Eq. (Sh).
 *  - T_FG,c = an optional input shape table with amp = 10^u_fg.
 *  - P_j: Akima spline (App. A) in log10 f, linear for 2 or 3 knots, zero
 *    when disabled (Eqs. (splines); Sec. "Power spectral density breakdown").
 *  - logL: the per-bin complex-Wishart term of Sec. "MCMC setup" summed over
 *    bins (segment averaging over N_k frequencies; N_k = 1 is Whittle), with
 *    E[D] = S and theta-independent constants dropped.
 *
 * Conventions
 *  - Every pointer is a DEVICE pointer unless marked [host].  Arrays of
 *    per-channel data are channel-major: X[c * n_bins + k], c = 0 (A), 1 (E), 2 (T).
 *  - Every call is asynchronous on the given stream (hipStream_t passed as
 *    void*; NULL = the default stream) and never allocates, frees or
 *    synchronises, so calls may be captured into a HIP graph.  Only
 *    lps_create, lps_destroy and lps_get_error synchronise.
 *  - Ownership: the caller owns every buffer passed in; the library never
 *    keeps a caller pointer after a call returns.  lps_create copies the
 *    dataset into memory owned by the context and sizes all workspace for
 *    max_states, so later calls need no allocation.
 *  - Errors: structural problems (NULL pointers, sizes, capacity, routing,
 *    precision) return a status before anything is launched.  Problems of
 *    individual states (see LPS_ST_*) never abort a call: the state's status
 *    word gets the bit, its logL is -inf and its gradient is zero.
 *  - A context is not thread-safe; separate contexts are independent.
 */
#ifndef LPS_H
#define LPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lps_ctx lps_ctx;

typedef enum {
  LPS_OK = 0,
  LPS_E_NULL = 1,       /* a required pointer is NULL */
  LPS_E_SHAPE = 2,      /* a size or range argument is out of bounds */
  LPS_E_CAPACITY = 3,   /* n_states > max_states (max_grad_states for the gradient), or k_max outside [2, 64] */
  LPS_E_ROUTING = 4,    /* the routing table is not one the kernels implement */
  LPS_E_PRECISION = 5,  /* unknown precision enum */
  LPS_E_DEVICE = 6,     /* a HIP runtime call failed */
  LPS_E_NOMEM = 7,      /* device allocation failed in lps_create */
  LPS_E_STATE = 8,      /* the call needs a state the batch does not provide */
  LPS_E_DATA = 9        /* dataset values out of their domain: N_k < 1 or not finite, D < 0 or
                           not finite, a response or foreground entry not finite */
} lps_status;

typedef enum { LPS_FP64 = 0, LPS_MIXED = 1 } lps_precision;

/* Per-state status bits (0 = valid). */
#define LPS_ST_COUNT 1u       /* a spline has 1 knot, more than k_max knots, or offsets outside the knot arrays */
#define LPS_ST_ORDER 2u       /* knot abscissae not strictly increasing */
#define LPS_ST_COVER 4u       /* the edge knots do not enclose every bin */
#define LPS_ST_NONFINITE 8u   /* a parameter or knot value is not finite */
#define LPS_ST_AMPLITUDE 16u  /* A_OMS <= 0 or A_TM <= 0 */
#define LPS_ST_PSD 32u        /* the total PSD is not finite and positive at some bin */

/* Terms of the routing table. */
#define LPS_TERM_OMS 0
#define LPS_TERM_TM 1
#define LPS_TERM_SGWB 2
#define LPS_TERM_FG 3

/* Parameter rows of lps_states.params. */
#define LPS_P_AOMS 0   /* OMS amplitude A_OMS [m Hz^-1/2] */
#define LPS_P_ATM 1    /* TM amplitude A_TM [m s^-2 Hz^-1/2] */
#define LPS_P_U 2      /* u = log10 of h^2 Omega at f_knee (Eq. (pl) amplitude A) */
#define LPS_P_ALPHA 3  /* spectral slope n of Eq. (pl) */
#define LPS_P_UFG 4    /* log10 of the foreground amplitude (only with a FG table) */

/* The analysed dataset (copied by lps_create). */
typedef struct {
  int32_t n_bins;        /* K >= 1 */
  const double* f;       /* [K] bin frequencies in Hz, strictly increasing, > 0 */
  const double* nk;      /* [K] N_k >= 1, frequencies averaged into bin k */
  const double* D;       /* [3][K] averaged periodogram, E[D] = S (one-sided PSD units) */
  const double* R;       /* [3][K] sky-averaged SGWB response R_c(f_k) (input table) */
  const double* Rfg;     /* [3][K] foreground shape table, or NULL for no FG term */
  double f_knee;         /* pivot of the power law in Hz (1e-3) */
  double arm_length;     /* L in m (2.5e9) */
  int32_t n_spl;         /* number of spline slots per state, 0..4 */
  int8_t route[4][3];    /* route[term][channel] = spline slot or -1 (unperturbed);
                            route[LPS_TERM_FG][*] must be -1 */
  int32_t k_max;         /* max knots per spline including edges, 2..64 */
  int32_t max_states;    /* workspace capacity in states (>= 1) */
  int32_t max_grad_states; /* states a gradient call may take (0..max_states; 0 = no
                              gradient workspace).  The adjoint keeps per-chunk moment
                              records: about 250 bytes per state per 128 bins. */
} lps_dataset_desc;

/* A batch of states: parameters plus ragged CSR knots (device arrays). */
typedef struct {
  int32_t n_states;          /* 0..max_states */
  const double* params;      /* [P][n_states]; P = 4, or 5 with a FG table */
  const int32_t* knot_off;   /* [n_states * n_spl + 1]; spline j of state s owns
                                knots knot_off[s*n_spl+j] .. knot_off[s*n_spl+j+1]-1.
                                Count 0 disables the spline (P = 0); 2 or 3 is linear;
                                4..k_max is Akima; 1 is invalid. */
  const double* knot_x;      /* log10 f of each knot, edges included, strictly increasing */
  const double* knot_y;      /* knot heights (P is in dex: the factor is 10^P) */
  const int32_t* knot_cnt;   /* NULL: packed CSR as above.  Otherwise padded CSR: spline i
                                (= s*n_spl+j) owns knot_cnt[i] knots starting at knot_off[i],
                                so slots may have spare capacity (used by the sampler to
                                edit knots in place); knot_off then needs n_states*n_spl entries. */
  int64_t n_knots;           /* entries of knot_x and knot_y (>= 0).  A spline whose range
                                [start, start + count) does not lie inside [0, n_knots) marks
                                its state LPS_ST_COUNT and none of its knots is read. */
} lps_states;

/*
 * Create a context on HIP device `device` for one dataset.  Copies the data,
 * builds the per-bin tables (template transfer factors, log10 f, scaled
 * FP32 copies for the mixed path) on the device, and allocates workspace for
 * desc->max_states states.  Supported routings (any spline slot may be -1):
 *   split:  OMS, TM, SGWB each on their own channel-independent spline;
 *   shared: OMS and TM on one channel-independent spline, SGWB on another;
 *   paper:  OMS and TM on one spline per channel, SGWB on a shared spline
 *           (the layout of Sec. "Power spectral density breakdown").
 * Returns LPS_E_ROUTING for any other table.  Synchronises the device.
 */
lps_status lps_create(const lps_dataset_desc* desc /*[host]*/, int device, lps_ctx** out /*[host]*/);

/* Free a context and all of its device memory (NULL is a no-op).  It
 * synchronises the device and frees memory, so it must not be called while
 * any stream of the process is being captured into a graph. */
lps_status lps_destroy(lps_ctx* ctx);

/*
 * Total PSD (Eq. (psd_tot) with Eqs. (splines)) for bins [k0, k1) of every
 * state, FP64: S[s][c][k - k0].  Optional Sn (noise: OMS + TM terms) and Sh
 * (signal: SGWB + FG terms) with the same layout; pass NULL to skip.
 * Invalid states get NaN rows and their status bits.
 */
lps_status lps_psd_build(lps_ctx* ctx, const lps_states* st /*[host]*/, int32_t k0, int32_t k1,
                         double* S, double* Sn, double* Sh, uint32_t* status, void* stream);

/*
 * logL[s] for every state in one batched launch: the per-bin complex Wishart
 * log-density of Sec. "MCMC setup" (minus the trace of C^-1 Y, minus nu log
 * det C, the two unnumbered equations there) with the diagonal A/E/T
 * covariance C_k = diag(S_A, S_E, S_T)(f_k) of Eq. (psd_tot) with Eqs.
 * (splines), Y_k = N_k D_k and nu_k = N_k, summed over bins (the combined
 * likelihood that follows them; N_k = 1 gives the Whittle likelihood):
 *   logL = - sum_k sum_c N_k (D_ck / S_ck + ln S_ck).
 * Inputs: st [host struct naming device arrays, see lps_states]; outputs
 * logL[n_states] and status[n_states] [device, caller-owned].  Invalid
 * states get logL = -inf and their LPS_ST_* bits; a malformed batch returns
 * LPS_E_SHAPE / LPS_E_CAPACITY before anything is launched.  LPS_FP64 evaluates every
 * per-bin term in double precision; LPS_MIXED evaluates them in single
 * precision in per-bin scaled units (hardware exp2/log2/rcp) and keeps the
 * per-state bin reduction and the scaling constant in double precision.
 * status (nullable) receives the LPS_ST_* bits.
 */
lps_status lps_loglike_batch(lps_ctx* ctx, const lps_states* st /*[host]*/, lps_precision prec,
                             double* logL, uint32_t* status, void* stream);

/*
 * logL of lps_loglike_batch and its gradient with respect to every state
 * input (hand-written adjoint of the same sum: the template derivatives of
 * Eqs. (noise_tdi), (pl), (Sh), the spline derivatives of App. A with
 * respect to knot abscissae and heights, chained through Eq. (splines)):
 *   dparams[p][s]   = dlogL/d params[p][s]   (same layout as params)
 *   dknot_x[i], dknot_y[i] = dlogL/d knot_x[i], knot_y[i] (same CSR layout as
 *   the knots; edge abscissae get 0 because they are fixed).
 * Derivatives of |.| at 0 are taken as 0.  Invalid states get zeros.
 */
lps_status lps_loglike_grad_batch(lps_ctx* ctx, const lps_states* st /*[host]*/, lps_precision prec,
                                  double* logL, double* dparams, double* dknot_x, double* dknot_y,
                                  uint32_t* status, void* stream);

/*
 * The likelihood of lps_loglike_batch (Sec. "MCMC setup", PSD of Eq.
 * (psd_tot) with Eqs. (splines)) on the reference path: plain FP64, one
 * launch per state, one thread per bin,
 * every factor evaluated from f_k (sin, cos, pow, exp10, log), a binary
 * search and a local Akima stencil per bin, and a two-pass reduction.
 */
lps_status lps_loglike_plain_fp64(lps_ctx* ctx, const lps_states* st /*[host]*/, double* logL,
                                  uint32_t* status, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the plain
 * FP64 path of lps_loglike_plain_fp64 without a context.  desc [host] names
 * the dataset's device arrays directly (f, nk, D, R, Rfg as in lps_create;
 * max_states and max_grad_states are ignored; any routing whose slots are in
 * [-1, n_spl) with route[LPS_TERM_FG][*] = -1 is accepted), and nothing is
 * copied, built or allocated: the per-block partial sums live in a 512 KiB
 * device-resident array that each GPU holds for the life of the process.
 * Limits: n_bins <= 2^24 (LPS_E_CAPACITY beyond), k_max in [2, 64].
 * f must be strictly increasing and positive (not checked: no host copy is
 * made).  States, outputs, status bits and errors as lps_loglike_plain_fp64;
 * results are identical to it for the same inputs.  All calls on one GPU
 * share the array (the last call's contents stay in it; every entry a call
 * reads it writes first): calls that overlap in time on one GPU, on any
 * streams or host threads, race and must be serialised by the caller.
 */
lps_status lps_loglike_plain_fp64_noalloc(const lps_dataset_desc* desc /*[host]*/, const lps_states* st /*[host]*/,
                                          double* logL, uint32_t* status, void* stream);

/*
 * Launch shape of the batched forward kernel for one precision: bins per lane
 * (the wave's chunk is 64 times that; mixed: 4 or 8, FP64: 2 or 4) and states
 * per work item (1..4096).  0 selects the built-in default (mixed 8, FP64 4;
 * six (mixed) or four (FP64) of the kernel's sub-tiles of min(64 / groups,
 * 32 mixed or 16 FP64) states, fewer if that launches under about 8192 wave
 * work items).
 */
lps_status lps_set_launch(lps_ctx* ctx, lps_precision prec, int32_t bins_per_lane, int32_t states_per_tile);

/* The launch shape a call with n_states states would use [host outputs]. */
lps_status lps_get_launch(lps_ctx* ctx, lps_precision prec, int32_t n_states, int32_t* bins_per_lane /*[host]*/,
                          int32_t* states_per_tile /*[host]*/);

/*
 * Autotuner: times every candidate launch shape of the forward kernel on the
 * given batch (reps timed calls each, HIP events on `stream`), keeps the
 * fastest for this precision and reports its milliseconds per call in
 * *best_ms [host].  A setup call: it allocates a scratch output and
 * synchronises; do not call it while capturing a graph.
 */
lps_status lps_autotune(lps_ctx* ctx, const lps_states* st /*[host]*/, lps_precision prec, int32_t reps,
                        double* best_ms /*[host]*/, void* stream);

/*
 * Per-kernel timing: when enabled, the forward and gradient entry points
 * record HIP events around their main kernel on the call's stream.
 * lps_kernel_time_ms synchronises and returns the summed milliseconds and
 * launch count of the main kernel since the last reset.  Not graph-safe:
 * keep it disabled while capturing.
 */
lps_status lps_set_timing(lps_ctx* ctx, int enable);
lps_status lps_kernel_time_ms(lps_ctx* ctx, double* total_ms /*[host]*/, int32_t* launches /*[host]*/);

/* ------------------------------------------------------------------------
 * Parallel-tempered reversible-jump sampler sweep on the device.
 *
 * Chains c = t * n_walkers + w.  Each sweep: a preconditioned Langevin
 * (MALA) move of all continuous parameters driven by the adjoint gradient,
 * a birth/death move of one in-between knot of one spline per chain (births
 * from the priors of Table I; Sec. "Power spectral density breakdown"),
 * FP64 tempered Metropolis-Hastings decisions, and swaps between adjacent
 * temperatures.  A sweep is a fixed launch sequence on one stream that never
 * allocates or synchronises, so sweeps may be captured into a HIP graph.
 * Random numbers: Philox4x32-10 keyed by the seed, indexed by (chain, sweep,
 * purpose); the sweep counter lives in device memory.
 * ------------------------------------------------------------------------ */
typedef struct lps_sampler lps_sampler;

typedef struct {
  int32_t n_walkers;
  int32_t n_temps;
  const double* betas;        /* [host] n_temps inverse temperatures in [0, 1] */
  const double* temp_scales;  /* [host] per-temperature step multipliers, or NULL for min(1/sqrt(beta), 1e3) */
  uint64_t seed;
  int32_t k_in_max;           /* maximum in-between knots per spline; k_in_max + 2 <= k_max */
  double step;                /* Langevin step multiplier (> 0) */
  lps_precision precision;    /* precision of the likelihood and gradient evaluations */
  uint32_t fixed_params;      /* bit p set: template parameter p (LPS_P_*) is held fixed (not moved) */
  int32_t rj_moves;           /* 0: sweeps make no birth/death moves (fixed knot counts) */
  int32_t stretch_moves;      /* non-zero: ensemble stretch moves of the free template parameters
                                 within each temperature, the walker halves in turn (a = 2) */
} lps_sampler_desc;

/* Allocate chain storage for n_walkers * n_temps chains (<= max_grad_states of ctx). */
lps_status lps_sampler_create(lps_ctx* ctx, const lps_sampler_desc* desc /*[host]*/, lps_sampler** out /*[host]*/);
/* Free a sampler (NULL is a no-op); the context must still exist.  Like
 * lps_destroy it synchronises and frees device memory: not during a capture. */
lps_status lps_sampler_destroy(lps_sampler* sm);

/* Load the chains from a packed-CSR batch (n_states = chains, every spline with
 * 2..k_in_max+2 knots), set the sweep counter, evaluate logL and gradients.
 * Synchronises.  Returns LPS_E_CAPACITY if a spline does not fit its slot. */
lps_status lps_sampler_set_state(lps_sampler* sm, const lps_states* init /*[host]*/, uint64_t sweep_index,
                                 void* stream);

/* Run n_sweeps sweeps (asynchronous, graph-capturable). */
lps_status lps_sampler_sweep(lps_sampler* sm, int32_t n_sweeps, void* stream);

/* Copy the current chains out (device outputs, any may be NULL): params [P][C],
 * padded-CSR knot_off/knot_cnt [C*n_spl] and knot_x/knot_y [C*n_spl*(k_in_max+2)],
 * logL [C]; sweep_index [host] (synchronises when requested). */
lps_status lps_sampler_get_state(lps_sampler* sm, double* params, int32_t* knot_off, int32_t* knot_cnt,
                                 double* knot_x, double* knot_y, double* logL, uint64_t* sweep_index /*[host]*/,
                                 void* stream);

/* Move statistics [host] uint32[5][n_temps][2] = (proposed, accepted) for the
 * kinds Langevin, birth, death, swap (counted at the lower temperature) and
 * stretch.  Synchronises. */
lps_status lps_sampler_counters(lps_sampler* sm, uint32_t* counters /*[host]*/, void* stream);

/* The sampler's generator: out[4i..4i+3] = Philox4x32-10(counter = (first + i) as
 * (low word, high word, 0, 0), key = (seed low, seed high)).  Device output. */
lps_status lps_philox4x32_10(uint64_t seed, uint64_t first_counter, int32_t n, uint32_t* out, void* stream);

/*
 * Model-selection reductions over stored tempered log-likelihoods.  Samples are
 * logL[n_rec][n_temps][n_walkers] (device, FP64): records of the sampler's
 * chain log-likelihoods (lps_sampler_get_state with only logL set copies one
 * record), chain c = t * n_walkers + w; rung t has n = n_rec * n_walkers draws.
 * Asynchronous on `stream`, no allocation, deterministic (fixed-order sums).
 *
 * Stepping-stone evidence, Eq. (ss) (Sec. "MCMC setup"): betas[n_temps]
 * (device) strictly increasing, the last normally 1; the ratios run over
 * consecutive rungs (a lowest rung near 0 stands in for the prior).  out
 * (device) receives 2 + 2 (n_temps - 1) doubles: log Z, Var(log Z) (delta
 * method, independent draws), then log r_k and Var(log r_k) for k = 1 .. n_temps - 1.
 * LPS_E_NULL / LPS_E_SHAPE for missing pointers or n_temps < 2, n_rec < 1, n_walkers < 1.
 */
lps_status lps_stepping_stone(const double* betas, int32_t n_temps, const double* logL, int32_t n_rec,
                              int32_t n_walkers, double* out, void* stream);

/* Deviance information criterion (Sec. "Results"): D = -2 logL over the draws of
 * rung `rung` (normally the b = 1 rung) and *logL_at_mean (device) = logL at the
 * posterior-mean parameters.  out (device) receives mean D, p_D = mean D - D(theta_bar),
 * DIC = mean D + p_D, Var D.  LPS_E_SHAPE for a rung outside [0, n_temps). */
lps_status lps_dic(const double* logL, int32_t n_rec, int32_t n_temps, int32_t n_walkers, int32_t rung,
                   const double* logL_at_mean, double* out, void* stream);

/* The 20-rung inverse-temperature ladder of Sec. "MCMC setup" [host output,
 * 20 values, increasing]: 5 log-spaced from 1e-20 up to (not including) 1e-12,
 * 10 from 1e-12 up to 1e-5, 5 from 1e-5 to 1 inclusive. */
lps_status lps_paper_ladder(double* betas /*[host]*/);

/* Median of each of m columns x[col * ld + i], i < n (device input and output
 * out[m]; the mean of the two middle values when n is even), as used for the
 * step-1 summary of Sec. "Two-step inference".  Asynchronous on `stream`, no
 * allocation; O(n^2) per column, n <= 65536 (LPS_E_SHAPE beyond). */
lps_status lps_column_median(const double* x, int32_t n, int32_t m, int32_t ld, double* out, void* stream);

/*
 * Data stage: from TDI time series to the inputs of lps_create.
 *
 * One-sided periodogram of n_ch time series x[n_ch][n_t] (device, step dt s),
 * optionally windowed by window[n_t] (device, NULL = none) and, when
 * xyz_to_aet is non-zero (n_ch = 3), combined first into the noise-orthogonal
 * channels A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3.
 * P[n_ch][n_t/2 + 1] (device) receives c_k dt |X_k|^2 / (n_t mean(w^2)) at
 * f_k = k / (n_t dt), c_k = 1 at k = 0 and k = n_t/2 (n_t even), else 2, with X
 * the discrete Fourier transform (hipFFT, double).  A one-off call: it plans,
 * allocates temporaries, synchronises `stream` and frees them (not for graph
 * capture; repeated calls use lps_data_create / lps_data_periodogram_planned).
 */
lps_status lps_data_periodogram(const double* x, int32_t n_ch, int32_t n_t, double dt, const double* window,
                                int32_t xyz_to_aet, double* P, void* stream);

/* A planned periodogram for n_ch series of n_t samples on `device`: the hipFFT
 * plan, its work area and the temporaries are allocated once here (synchronises;
 * not during a capture), so that lps_data_periodogram_planned allocates nothing. */
typedef struct lps_data_ctx lps_data_ctx;
lps_status lps_data_create(int32_t n_ch, int32_t n_t, int device, lps_data_ctx** out /*[host]*/);
/* Free a planned periodogram (NULL is a no-op); synchronises, not during a capture. */
lps_status lps_data_destroy(lps_data_ctx* ctx);
/* lps_data_periodogram on a planned context (the same arguments and output):
 * asynchronous on `stream`, no allocation and no synchronisation, so it may be
 * captured into a HIP graph.  One call at a time per context (the temporaries
 * are shared). */
lps_status lps_data_periodogram_planned(lps_data_ctx* ctx, const double* x, double dt, const double* window,
                                        int32_t xyz_to_aet, double* P, void* stream);

/* Averaged periodogram (Sec. "MCMC setup"): n_seg segments of seg_len consecutive
 * non-overlapping bins starting at bin k0 of P[n_ch][n_f] with frequencies f[n_f]
 * (device).  D[n_ch][n_seg] = segment means, f_seg[n_seg] = mean bin frequency,
 * nu[n_seg] = seg_len (the segment counts N_k of lps_create); f_seg and nu may be
 * NULL.  LPS_E_SHAPE if the segments run past n_f. */
lps_status lps_data_average(const double* P, int32_t n_ch, int32_t n_f, const double* f, int32_t k0, int32_t seg_len,
                            int32_t n_seg, double* D, double* f_seg, double* nu, void* stream);

/* Response interpolation (Sec. "Parametrized SGWB model"): grid_R[n_ch][n_g]
 * tabulated at increasing grid_f[n_g] > 0 Hz, evaluated at f[n] into R[n_ch][n]
 * (all device): linear in (log f, log R) between nodes whose values are both
 * positive, linear in (log f, R) otherwise; NaN outside [grid_f[0], grid_f[n_g-1]]. */
lps_status lps_data_response(const double* grid_f, const double* grid_R, int32_t n_ch, int32_t n_g, const double* f,
                             int32_t n, double* R, void* stream);

/* ------------------------------------------------------------------------
 * Full-covariance likelihood (dense 3x3 A/E/T covariance per bin).
 *
 * The paper keeps the noise covariance diagonal and names the dense treatment
 * as its extension: three more flexible terms for the off-diagonal entries,
 * six flexible functions for the noise in all, combined so that the matrix
 * stays positive definite (Sec. "Power spectral density breakdown", the
 * paragraph on independent channel splines; outlook of the conclusions).  It
 * prints no construction; this library uses the following one.
 *
 *   Sn_c, Sh_c  noise (OMS + TM) and signal (SGWB + FG) parts of the diagonal
 *               model above, per channel, with the same templates, parameters
 *               and routed splines;
 *   Q_0..Q_2    three further spline slots (abscissa log10 f, P = 0 when
 *               disabled or routed nowhere);
 *   r_AE = tanh Q_0,  r_AT = tanh Q_1,
 *   r_ET = r_AE r_AT + tanh(Q_2) sqrt((1 - r_AE^2)(1 - r_AT^2))
 *               (tanh Q_2 is the partial correlation of E and T given A; the
 *               correlation matrix is positive definite for any real Q);
 *   C_cc = Sn_c + Sh_c,   C_ab = r_ab sqrt(Sn_a Sn_b)   (a != b);
 *   logL = - sum_k N_k ( tr(C_k^-1 P_k) + ln det C_k ),
 * the complex-Wishart log-density of an averaged cross-periodogram with
 * E[P] = C, up to theta-independent constants.  Zero correlations give the
 * diagonal likelihood of lps_loglike_batch exactly.  Any orthonormal change
 * of channel basis applied to both C and P (e.g. A/E/T -> X/Y/Z) leaves
 * logL unchanged, so this is also the dense Michelson-basis likelihood.
 * A state is invalid (logL = -inf) under the LPS_ST_* rules of the diagonal
 * model applied to every slot, or with LPS_ST_PSD when C_k is not positive
 * definite (or not finite) at some bin.  Everything is FP64.
 * ------------------------------------------------------------------------ */
#define LPS_COV_MAX_SPLINES 8

typedef struct lps_cov_ctx lps_cov_ctx;

typedef struct {
  int32_t n_bins;        /* K >= 1 */
  const double* f;       /* [K] bin frequencies in Hz, strictly increasing, > 0 */
  const double* nk;      /* [K] N_k >= 1 */
  const double* P;       /* [6][K] real part of the averaged cross-periodogram, rows
                            AA, EE, TT, AE, AT, ET; one-sided units, E[P] = C */
  const double* R;       /* [3][K] SGWB response per channel (as in lps_dataset_desc) */
  const double* Rfg;     /* [3][K] foreground shape, or NULL */
  double f_knee;         /* pivot of the power law in Hz */
  double arm_length;     /* L in m */
  int32_t n_spl;         /* spline slots per state, 0..LPS_COV_MAX_SPLINES */
  int8_t route[4][3];    /* diagonal routing as in lps_dataset_desc, any slot or -1 per
                            (term, channel); route[LPS_TERM_FG][*] must be -1 */
  int8_t corr[3];        /* slots of Q_0 (A-E), Q_1 (A-T), Q_2 (E-T given A), or -1 */
  int32_t k_max;         /* max knots per spline including edges, 2..64 */
  int32_t max_states;    /* workspace capacity in states (>= 1); about 37 KB per state */
} lps_cov_desc;

/* Create a full-covariance context on `device`: copies the data into a per-bin
 * table and allocates workspace for max_states.  LPS_E_ROUTING for a slot out
 * of range or a perturbed foreground.  Synchronises the device. */
lps_status lps_cov_create(const lps_cov_desc* desc /*[host]*/, int device, lps_cov_ctx** out /*[host]*/);

/* Free a context (NULL is a no-op).  Synchronises the device and frees memory:
 * not while any stream of the process is being captured into a graph. */
lps_status lps_cov_destroy(lps_cov_ctx* ctx);

/* logL[s] for every state of the batch (states as in lps_loglike_batch, with
 * the context's n_spl slots per state).  status (nullable) receives the
 * LPS_ST_* bits.  Asynchronous on `stream`, no allocation; one batch at a
 * time per context (the workspace is shared). */
lps_status lps_cov_loglike_batch(lps_cov_ctx* ctx, const lps_states* st /*[host]*/, double* logL,
                                 uint32_t* status, void* stream);

/* logL and its gradient for every state of the batch (hand-written adjoint,
 * FP64): dparams[p][s] = dlogL/dparams[p][s] (same layout as params) and
 * dknot_x, dknot_y = dlogL/d knot_x, knot_y (the states' CSR layout; edge
 * abscissae get 0), with the conventions of lps_loglike_grad_batch.  Invalid
 * states, including those whose covariance is not positive definite, get
 * logL = -inf and zero derivatives.  One wave per state walks every bin;
 * asynchronous on `stream`, no allocation; one batch at a time per context. */
lps_status lps_cov_loglike_grad_batch(lps_cov_ctx* ctx, const lps_states* st /*[host]*/, double* logL,
                                      double* dparams, double* dknot_x, double* dknot_y, uint32_t* status,
                                      void* stream);

/* The model covariance for bins [k0, k1) of every state: C[s][e][k - k0] with
 * e = AA, EE, TT, AE, AT, ET.  Structurally invalid states get NaN rows and
 * their status bits (the positive-definiteness bit is left to
 * lps_cov_loglike_batch).  Asynchronous on `stream`, no allocation. */
lps_status lps_cov_build(lps_cov_ctx* ctx, const lps_states* st /*[host]*/, int32_t k0, int32_t k1, double* C,
                         uint32_t* status, void* stream);

/* Synchronise the stream and report the sticky device error flags (0 = none). */
lps_status lps_get_error(lps_ctx* ctx, void* stream, uint32_t* sticky_flags /*[host]*/);

/* Static text for a status code. */
const char* lps_strerror(lps_status s);

/* The HIP error behind the most recent LPS_E_DEVICE returned on the calling
 * host thread (0 = none yet); *name, if name is not NULL, receives its static
 * HIP error name. */
int32_t lps_last_device_error(const char** name /*[host]*/);

/* Number of bins per wave chunk used by the batched kernels (for sizing checks). */
int32_t lps_chunk_bins(lps_precision prec);

/*
 * Device calibration for roofline reporting (not part of the hot path):
 * times a dependent FP32 FMA chain and an exp2/log2/rcp chain on every CU.
 * Outputs [host]: nanoseconds per wave64 FMA instruction per SIMD, the issue
 * cost of one single-precision transcendental in FMA slots, and the achieved
 * FP32 lane-instruction rate of the whole device.  Allocates and synchronises.
 */
lps_status lps_valu_probe(int device, double* fma_ns_per_wave_instr, double* trans_over_fma,
                          double* lane_instr_per_s);

/*
 * Diagnostic (not part of the hot path): applies one of the double-precision
 * elementary functions of the batched FP64 kernels to x[0..n): fn = 0 exp2
 * (series), 1 log2, 2 reciprocal, 3 square root, 4 natural logarithm, 5 exp2
 * from the 64-entry table of 2^(j/64) (the FP64 forward kernel's), 6
 * reciprocal square root; out[i] receives the result.  Device pointers,
 * asynchronous on `stream`, no allocation; LPS_E_SHAPE for fn outside 0..6.
 */
lps_status lps_math64_check(const double* x, int32_t n, int32_t fn, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LPS_H */
