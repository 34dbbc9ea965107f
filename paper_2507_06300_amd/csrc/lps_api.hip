// C ABI entry points: context life cycle, structural validation, dispatch.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lps_internal.hpp"
#include "lps_roctx.hpp"

using lps::Layout;

namespace lps {

namespace {
thread_local hipError_t g_last_device_error = hipSuccess;
}

lps_status device_status(hipError_t e) {
  if (e == hipSuccess) return LPS_OK;
  g_last_device_error = e;
  return LPS_E_DEVICE;
}

}  // namespace lps

namespace {

// Classify the routing table into one of the implemented layouts.
lps_status classify(const lps_dataset_desc* d, bool ae_tables_equal, Layout* out) {
  Layout L;
  memset(&L, 0, sizeof(L));
  for (int g = 0; g < lps::kMaxGroups; ++g) {
    L.grp_spline[g] = -1;
    L.grp_channel[g] = -1;
  }
  const int ns = d->n_spl;
  for (int t = 0; t < 4; ++t)
    for (int c = 0; c < 3; ++c)
      if (d->route[t][c] < -1 || d->route[t][c] >= ns) return LPS_E_ROUTING;
  for (int c = 0; c < 3; ++c)
    if (d->route[LPS_TERM_FG][c] != -1) return LPS_E_ROUTING;
  auto indep = [&](int t) { return d->route[t][0] == d->route[t][1] && d->route[t][1] == d->route[t][2]; };
  L.has_fg = d->Rfg != nullptr;
  L.n_terms = L.has_fg ? 4 : 3;
  const int ro = d->route[LPS_TERM_OMS][0], rt = d->route[LPS_TERM_TM][0], rh = d->route[LPS_TERM_SGWB][0];
  if (indep(LPS_TERM_OMS) && indep(LPS_TERM_TM) && indep(LPS_TERM_SGWB)) {
    if (ro >= 0 && ro == rt) {
      L.mode = lps::kShared;
      L.n_grp = 2;
      L.grp_kind[0] = lps::kGNoise;
      L.grp_spline[0] = ro;
      L.grp_kind[1] = lps::kGSgwb;
      L.grp_spline[1] = rh;
    } else {
      L.mode = lps::kSplit;
      L.n_grp = 3;
      L.grp_kind[0] = lps::kGOms;
      L.grp_spline[0] = ro;
      L.grp_kind[1] = lps::kGTm;
      L.grp_spline[1] = rt;
      L.grp_kind[2] = lps::kGSgwb;
      L.grp_spline[2] = rh;
    }
    L.nch = ae_tables_equal ? 2 : 3;
  } else {
    // one noise spline per channel shared by OMS and TM, channel-independent signal
    for (int c = 0; c < 3; ++c)
      if (d->route[LPS_TERM_OMS][c] != d->route[LPS_TERM_TM][c]) return LPS_E_ROUTING;
    if (!indep(LPS_TERM_SGWB)) return LPS_E_ROUTING;
    L.mode = lps::kPaper;
    L.n_grp = 4;
    for (int c = 0; c < 3; ++c) {
      L.grp_kind[c] = lps::kGNoise;
      L.grp_spline[c] = d->route[LPS_TERM_OMS][c];
      L.grp_channel[c] = c;
    }
    L.grp_kind[3] = lps::kGSgwb;
    L.grp_spline[3] = rh;
    L.nch = 3;
  }
  L.n_tab = 1 + L.n_terms * L.nch + L.nch + 1;
  *out = L;
  return LPS_OK;
}

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, n * sizeof(T) > 0 ? n * sizeof(T) : 16);
}

void free_ctx(lps_ctx* c) {
  if (!c) return;
  void* ptrs[] = {c->f,      c->nk,        c->D,       c->R,        c->Rfg,      c->x,       c->sigma,
                  c->tmpl,   c->tab64,     c->tab32,   c->c0,       c->bx,       c->coef64,  c->coef32,
                  c->n_int,  c->scal,      c->status_ws, c->partial, c->run_sum, c->gpartial, c->moments, c->plain_part,
                  c->sticky, c->wide_list, c->wide_count};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

lps_status check_states(const lps_ctx* ctx, const lps_states* st) {
  if (!ctx || !st) return LPS_E_NULL;
  if (st->n_states < 0 || st->n_knots < 0) return LPS_E_SHAPE;
  if (st->n_states > ctx->max_states) return LPS_E_CAPACITY;
  if (st->n_states == 0) return LPS_OK;
  if (!st->params || !st->knot_off) return LPS_E_NULL;
  if (ctx->n_spl > 0 && (!st->knot_x || !st->knot_y)) return LPS_E_NULL;
  return LPS_OK;
}

}  // namespace

extern "C" {

const char* lps_strerror(lps_status s) {
  switch (s) {
    case LPS_OK: return "ok";
    case LPS_E_NULL: return "a required pointer is NULL";
    case LPS_E_SHAPE: return "a size or range argument is out of bounds";
    case LPS_E_CAPACITY: return "capacity exceeded (n_states > max_states or k_max outside [2, 64])";
    case LPS_E_ROUTING: return "routing table not supported";
    case LPS_E_PRECISION: return "unknown precision";
    case LPS_E_DEVICE: return "HIP runtime error";
    case LPS_E_NOMEM: return "device allocation failed";
    case LPS_E_STATE: return "state batch does not provide what the call needs";
    case LPS_E_DATA: return "dataset values out of domain (N_k >= 1, D >= 0, finite D, R and Rfg)";
  }
  return "unknown status";
}

int32_t lps_last_device_error(const char** name) {
  const hipError_t e = lps::g_last_device_error;
  if (name) *name = hipGetErrorName(e);
  return (int32_t)e;
}

int32_t lps_chunk_bins(lps_precision prec) { return prec == LPS_MIXED ? lps::kChunk32 : lps::kChunk64; }

lps_status lps_create(const lps_dataset_desc* d, int device, lps_ctx** out) {
  LPS_API_RANGE();
  if (!d || !out) return LPS_E_NULL;
  *out = nullptr;
  if (!d->f || !d->nk || !d->D || !d->R) return LPS_E_NULL;
  if (d->n_bins < 1 || d->n_spl < 0 || d->n_spl > 4) return LPS_E_SHAPE;
  if (d->k_max < 2 || d->k_max > lps::kMaxKnots || d->max_states < 1) return LPS_E_CAPACITY;
  if (d->max_grad_states < 0 || d->max_grad_states > d->max_states) return LPS_E_CAPACITY;
  if (!(d->f_knee > 0.0) || !(d->arm_length > 0.0)) return LPS_E_SHAPE;
  if (hipSetDevice(device) != hipSuccess) return LPS_E_DEVICE;
  const int K = d->n_bins;
  // A and E can be merged when their response (and foreground) rows agree bitwise.
  bool ae_equal = true;
  double nk_uniform = 0.0;
  {
    // per-channel tables: finite values (D also >= 0); A and E merge when their
    // response (and foreground) rows agree bitwise
    std::vector<double> h(3 * (size_t)K);
    const double* tabs[3] = {d->R, d->Rfg, d->D};
    for (int i = 0; i < 3; ++i) {
      if (!tabs[i]) continue;
      if (hipMemcpy(h.data(), tabs[i], 3 * (size_t)K * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return LPS_E_DEVICE;
      for (size_t q = 0; q < 3 * (size_t)K; ++q)
        if (!std::isfinite(h[q]) || (i == 2 && h[q] < 0.0)) return LPS_E_DATA;
      if (i < 2) ae_equal = ae_equal && memcmp(h.data(), h.data() + K, (size_t)K * sizeof(double)) == 0;
    }
    std::vector<double> fh(K);
    if (hipMemcpy(fh.data(), d->f, (size_t)K * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return LPS_E_DEVICE;
    for (int k = 0; k < K; ++k)
      if (!(fh[k] > 0.0) || (k > 0 && !(fh[k] > fh[k - 1]))) return LPS_E_SHAPE;
    if (hipMemcpy(fh.data(), d->nk, (size_t)K * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return LPS_E_DEVICE;
    nk_uniform = fh[0];
    for (int k = 0; k < K; ++k) {
      if (!(fh[k] >= 1.0) || !std::isfinite(fh[k])) return LPS_E_DATA;   // N_k >= 1
      if (fh[k] != fh[0]) nk_uniform = 0.0;
    }
  }
  Layout L;
  lps_status rs = classify(d, ae_equal, &L);
  if (rs != LPS_OK) return rs;

  lps_ctx* c = new lps_ctx;
  memset(c, 0, sizeof(*c));
  c->device = device;
  {
    hipDeviceProp_t prop;
    c->n_cu = hipGetDeviceProperties(&prop, device) == hipSuccess ? prop.multiProcessorCount : 0;
  }
  c->n_bins = K;
  c->k_pad64 = ((K + lps::kChunk64 - 1) / lps::kChunk64) * lps::kChunk64;
  c->k_pad32 = ((K + lps::kChunk32 - 1) / lps::kChunk32) * lps::kChunk32;
  c->n_chunks64 = c->k_pad64 / lps::kChunk64;
  c->n_chunks32 = c->k_pad32 / lps::kChunk32;
  c->n_spl = d->n_spl;
  c->n_params = L.has_fg ? 5 : 4;
  memcpy(c->route, d->route, sizeof(c->route));
  c->k_max = d->k_max;
  c->max_states = d->max_states;
  c->max_grad_states = d->max_grad_states;
  c->f_knee = d->f_knee;
  c->arm_length = d->arm_length;
  c->lay = L;
  c->plain_blocks = (K + lps::kPlainBlock - 1) / lps::kPlainBlock;
  c->nk_uniform = nk_uniform;

  const size_t S = (size_t)d->max_states;
  const size_t G = (size_t)L.n_grp;
  // partial sums per (state, chunk) for the smallest chunk any launch shape uses (128 bins)
  const size_t nchunk = (size_t)((K + 127) / 128);
  bool ok = true;
  ok = ok && dalloc(&c->f, K) == hipSuccess && dalloc(&c->nk, K) == hipSuccess;
  ok = ok && dalloc(&c->D, 3 * (size_t)K) == hipSuccess && dalloc(&c->R, 3 * (size_t)K) == hipSuccess;
  if (L.has_fg) ok = ok && dalloc(&c->Rfg, 3 * (size_t)K) == hipSuccess;
  ok = ok && dalloc(&c->x, K) == hipSuccess && dalloc(&c->sigma, 3 * (size_t)K) == hipSuccess;
  ok = ok && dalloc(&c->tmpl, 12 * (size_t)K) == hipSuccess;
  ok = ok && dalloc(&c->tab64, (size_t)L.n_tab * c->k_pad64) == hipSuccess;
  ok = ok && dalloc(&c->tab32, (size_t)L.n_tab * c->k_pad32) == hipSuccess;
  ok = ok && dalloc(&c->c0, 1) == hipSuccess;
  ok = ok && dalloc(&c->bx, S * G * lps::kMaxKnots) == hipSuccess;
  ok = ok && dalloc(&c->coef64, S * G * lps::kMaxKnots * 4) == hipSuccess;
  ok = ok && dalloc(&c->coef32, S * G * lps::kMaxKnots * 4) == hipSuccess;
  ok = ok && dalloc(&c->n_int, S * G) == hipSuccess;
  ok = ok && dalloc(&c->scal, S) == hipSuccess;
  ok = ok && dalloc(&c->status_ws, S) == hipSuccess;
  ok = ok && dalloc(&c->partial, S * nchunk) == hipSuccess;
  ok = ok && dalloc(&c->run_sum, S * lps::kFinalizeRuns) == hipSuccess;
  ok = ok && dalloc(&c->plain_part, (size_t)c->plain_blocks) == hipSuccess;
  ok = ok && dalloc(&c->sticky, 1) == hipSuccess;
  // queue of single-precision chunk partials to re-evaluate in double range
  // (pairs beyond the capacity keep a non-finite partial: the state is reported invalid)
  c->wide_cap = (int32_t)std::min<size_t>(S * nchunk, (size_t)1 << 20);
  ok = ok && dalloc(&c->wide_list, (size_t)c->wide_cap) == hipSuccess;
  ok = ok && dalloc(&c->wide_count, 1) == hipSuccess;
  if (ok) {
    c->gpartial_bytes = lps::grad_workspace_bytes(c);
    ok = hipMalloc((void**)&c->gpartial, c->gpartial_bytes) == hipSuccess;
  }
  ok = ok && dalloc(&c->moments, (size_t)(d->max_grad_states > 0 ? d->max_grad_states : 1) * G * lps::kMaxKnots * 4) ==
                 hipSuccess;
  if (!ok) {
    free_ctx(c);
    return LPS_E_NOMEM;
  }
  bool cp = true;
  cp = cp && hipMemcpy(c->f, d->f, K * sizeof(double), hipMemcpyDeviceToDevice) == hipSuccess;
  cp = cp && hipMemcpy(c->nk, d->nk, K * sizeof(double), hipMemcpyDeviceToDevice) == hipSuccess;
  cp = cp && hipMemcpy(c->D, d->D, 3 * (size_t)K * sizeof(double), hipMemcpyDeviceToDevice) == hipSuccess;
  cp = cp && hipMemcpy(c->R, d->R, 3 * (size_t)K * sizeof(double), hipMemcpyDeviceToDevice) == hipSuccess;
  if (L.has_fg)
    cp = cp && hipMemcpy(c->Rfg, d->Rfg, 3 * (size_t)K * sizeof(double), hipMemcpyDeviceToDevice) == hipSuccess;
  cp = cp && hipMemset(c->sticky, 0, sizeof(uint32_t)) == hipSuccess;
  cp = cp && hipMemset(c->wide_count, 0, sizeof(uint32_t)) == hipSuccess;
  cp = cp && hipEventCreate(&c->ev0) == hipSuccess && hipEventCreate(&c->ev1) == hipSuccess;
  cp = cp && lps::build_tables(c, nullptr) == hipSuccess;
  cp = cp && hipDeviceSynchronize() == hipSuccess;
  if (!cp) {
    free_ctx(c);
    return LPS_E_DEVICE;
  }
  double xf = 0, xl = 0;
  if (hipMemcpy(&xf, c->x, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&xl, c->x + (K - 1), sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    free_ctx(c);
    return LPS_E_DEVICE;
  }
  c->x_first = xf;
  c->x_last = xl;
  *out = c;
  return LPS_OK;
}

lps_status lps_destroy(lps_ctx* ctx) {
  LPS_API_RANGE();
  if (!ctx) return LPS_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_ctx(ctx);
  return LPS_OK;
}

lps_status lps_psd_build(lps_ctx* ctx, const lps_states* st, int32_t k0, int32_t k1, double* S, double* Sn,
                         double* Sh, uint32_t* status, void* stream) {
  LPS_API_RANGE();
  lps_status r = check_states(ctx, st);
  if (r != LPS_OK) return r;
  if (k0 < 0 || k1 > ctx->n_bins || k0 > k1) return LPS_E_SHAPE;
  if (st->n_states == 0) return LPS_OK;
  if (!S && k1 > k0) return LPS_E_NULL;
  return lps::device_status(lps::launch_psd(ctx, st, k0, k1, S, Sn, Sh, status, (hipStream_t)stream));
}

lps_status lps_loglike_batch(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL,
                             uint32_t* status, void* stream) {
  LPS_API_RANGE();
  lps_status r = check_states(ctx, st);
  if (r != LPS_OK) return r;
  if (prec != LPS_FP64 && prec != LPS_MIXED) return LPS_E_PRECISION;
  if (st->n_states == 0) return LPS_OK;
  if (!logL) return LPS_E_NULL;
  return lps::device_status(lps::launch_forward(ctx, st, prec, logL, status, (hipStream_t)stream));
}

lps_status lps_loglike_grad_batch(lps_ctx* ctx, const lps_states* st, lps_precision prec, double* logL,
                                  double* dparams, double* dknot_x, double* dknot_y, uint32_t* status,
                                  void* stream) {
  LPS_API_RANGE();
  lps_status r = check_states(ctx, st);
  if (r != LPS_OK) return r;
  if (prec != LPS_FP64 && prec != LPS_MIXED) return LPS_E_PRECISION;
  if (st->n_states > ctx->max_grad_states) return LPS_E_CAPACITY;
  if (st->n_states == 0) return LPS_OK;
  if (!logL || !dparams) return LPS_E_NULL;
  if (ctx->n_spl > 0 && (!dknot_x || !dknot_y)) return LPS_E_NULL;
  return lps::device_status(
      lps::launch_grad(ctx, st, prec, logL, dparams, dknot_x, dknot_y, status, (hipStream_t)stream));
}

lps_status lps_loglike_plain_fp64(lps_ctx* ctx, const lps_states* st, double* logL, uint32_t* status,
                                  void* stream) {
  LPS_API_RANGE();
  lps_status r = check_states(ctx, st);
  if (r != LPS_OK) return r;
  if (st->n_states == 0) return LPS_OK;
  if (!logL) return LPS_E_NULL;
  return lps::device_status(lps::launch_plain(ctx, st, logL, status, (hipStream_t)stream));
}

lps_status lps_set_launch(lps_ctx* ctx, lps_precision prec, int32_t bins_per_lane, int32_t states_per_tile) {
  LPS_API_RANGE();
  if (!ctx) return LPS_E_NULL;
  if (prec != LPS_FP64 && prec != LPS_MIXED) return LPS_E_PRECISION;
  if (bins_per_lane != 0 && !lps::valid_bins_per_lane(prec, bins_per_lane)) return LPS_E_SHAPE;
  if (states_per_tile < 0 || states_per_tile > 4096) return LPS_E_SHAPE;
  ctx->fwd_shape[prec == LPS_MIXED ? 1 : 0] = {bins_per_lane, states_per_tile};
  return LPS_OK;
}

lps_status lps_get_launch(lps_ctx* ctx, lps_precision prec, int32_t n_states, int32_t* bins_per_lane,
                          int32_t* states_per_tile) {
  LPS_API_RANGE();
  if (!ctx || !bins_per_lane || !states_per_tile) return LPS_E_NULL;
  if (prec != LPS_FP64 && prec != LPS_MIXED) return LPS_E_PRECISION;
  if (n_states < 1) return LPS_E_SHAPE;
  const lps::LaunchShape sh = lps::forward_shape(ctx, prec, n_states);
  *bins_per_lane = sh.bins_per_lane;
  *states_per_tile = sh.tile;
  return LPS_OK;
}

lps_status lps_autotune(lps_ctx* ctx, const lps_states* st, lps_precision prec, int32_t reps, double* best_ms,
                        void* stream) {
  LPS_API_RANGE();
  lps_status r = check_states(ctx, st);
  if (r != LPS_OK) return r;
  if (prec != LPS_FP64 && prec != LPS_MIXED) return LPS_E_PRECISION;
  if (st->n_states == 0 || reps < 1) return LPS_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  const int n = st->n_states;
  double* logL = nullptr;
  if (hipMalloc((void**)&logL, (size_t)n * sizeof(double)) != hipSuccess) return LPS_E_NOMEM;
  const int bpl[2][2] = {{4, 2}, {8, 4}};   // default first
  // candidate tiles: the default, then whole numbers of the kernel's sub-tile
  const int sub = lps::sub_states(ctx, prec);
  const int tiles[] = {0, sub, 2 * sub, 3 * sub, 4 * sub, 6 * sub, 8 * sub, 12 * sub};
  constexpr int n_tiles_c = sizeof(tiles) / sizeof(tiles[0]);
  const int pi = prec == LPS_MIXED ? 1 : 0;
  const lps::LaunchShape saved = ctx->fwd_shape[pi];
  const int saved_timing = ctx->timing;
  ctx->timing = 0;
  hipEvent_t e0 = ctx->ev0, e1 = ctx->ev1;
  double t_default = 1e300, best = 1e300;
  lps::LaunchShape best_sh = saved;
  bool ok = true;
  for (int bi = 0; bi < 2 && ok; ++bi) {
    for (int ti = 0; ti < n_tiles_c && ok; ++ti) {
      if (tiles[ti] > n) continue;
      ctx->fwd_shape[pi] = {bpl[pi][bi], tiles[ti]};
      ok = lps::launch_forward(ctx, st, prec, logL, nullptr, s) == hipSuccess;   // warm-up
      ok = ok && hipEventRecord(e0, s) == hipSuccess;
      for (int k = 0; k < reps && ok; ++k) ok = lps::launch_forward(ctx, st, prec, logL, nullptr, s) == hipSuccess;
      ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.f;
      ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      // the first candidate is the default shape; the fastest of the others
      // replaces it only if it beats it by 2% (timing noise is about 1%)
      const double t_call = ms / reps;
      if (!ok) break;
      if (bi == 0 && ti == 0) {
        t_default = t_call;
      } else if (t_call < best) {
        best = t_call;
        best_sh = ctx->fwd_shape[pi];
      }
    }
  }
  if (!(best < 0.98 * t_default)) {
    best = t_default;
    best_sh = {bpl[pi][0], 0};
  }
  (void)hipFree(logL);
  ctx->timing = saved_timing;
  ctx->fwd_shape[pi] = ok ? best_sh : saved;
  if (best_ms) *best_ms = ok ? best : -1.0;
  return ok ? LPS_OK : LPS_E_DEVICE;
}

lps_status lps_set_timing(lps_ctx* ctx, int enable) {
  LPS_API_RANGE();
  if (!ctx) return LPS_E_NULL;
  ctx->timing = enable ? 1 : 0;
  ctx->time_ms = 0.0;
  ctx->time_launches = 0;
  return LPS_OK;
}

lps_status lps_kernel_time_ms(lps_ctx* ctx, double* total_ms, int32_t* launches) {
  LPS_API_RANGE();
  if (!ctx || !total_ms || !launches) return LPS_E_NULL;
  *total_ms = ctx->time_ms;
  *launches = ctx->time_launches;
  return LPS_OK;
}

lps_status lps_get_error(lps_ctx* ctx, void* stream, uint32_t* sticky_flags) {
  LPS_API_RANGE();
  if (!ctx || !sticky_flags) return LPS_E_NULL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return LPS_E_DEVICE;
  uint32_t v = 0;
  if (hipMemcpy(&v, ctx->sticky, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return LPS_E_DEVICE;
  *sticky_flags = v;
  return hipGetLastError() == hipSuccess ? LPS_OK : LPS_E_DEVICE;
}

}  // extern "C"
