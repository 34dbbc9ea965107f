// Per-bin tables, built once per dataset on the device.
//
// For every bin the noise transfer of Eq. (noise_tdi) (prefactor
// sin^2 xi sin^2 2xi, xi = 2 pi f L / c) times the single-link OMS and TM
// PSDs of Sec. "Parametrized noise model" per unit squared amplitude, the
// background factor R_c(f) 3 (H0/h)^2 / (4 pi^2 f^3) of Eq. (Sh) per unit
// h^2 Omega, the foreground shape, and the scaled rows used by the batched
// kernels (see lps_internal.hpp for the row order).
#include <math.h>

#include "lps_internal.hpp"
#include "lps_templates.hpp"

namespace lps {
namespace {

__global__ void k_templates(int K, const double* __restrict__ f, double L, const double* __restrict__ R,
                            const double* __restrict__ Rfg, int unit_oms, double* __restrict__ x,
                            double* __restrict__ tmpl, double* __restrict__ sigma) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double fk = f[k];
  x[k] = log10(fk);
  double oms_ae, oms_t, tm_ae, tm_t, h;
  unit_templates(fk, L, oms_ae, oms_t, tm_ae, tm_t, h);
  double oms[3] = {oms_ae, oms_ae, oms_t};
  double tm[3] = {tm_ae, tm_ae, tm_t};
  for (int c = 0; c < 3; ++c) {
    tmpl[(0 * 3 + c) * (size_t)K + k] = oms[c];
    tmpl[(1 * 3 + c) * (size_t)K + k] = tm[c];
    tmpl[(2 * 3 + c) * (size_t)K + k] = R[c * (size_t)K + k] * h;
    tmpl[(3 * 3 + c) * (size_t)K + k] = Rfg ? Rfg[c * (size_t)K + k] : 0.0;
    // the OMS row of the scaled table is then ref * oms / (ref * oms) = 1 exactly
    sigma[c * (size_t)K + k] = unit_oms ? kRefAoms * kRefAoms * oms[c]
                                        : kRefAoms * kRefAoms * oms[c] + kRefAtm * kRefAtm * tm[c];
  }
}

// Scaled rows.  Padded bins (k >= K) contribute exactly zero: N = 0 and the
// templates are 1 so that S stays finite.
__global__ void k_scaled(int K, int k_pad, int chunk, Layout lay, const double* __restrict__ x,
                         const double* __restrict__ nk, const double* __restrict__ D,
                         const double* __restrict__ tmpl, const double* __restrict__ sigma,
                         double* __restrict__ tab64, float* __restrict__ tab32, int write32) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= k_pad) return;
  const int nch = lay.nch;
  const double ref[4] = {kRefAoms * kRefAoms, kRefAtm * kRefAtm, pow(10.0, kRefU), pow(10.0, kRefUfg)};
  double row[1 + 4 * 3 + 3 + 1];
  int n_tab = lay.n_tab;
  if (k < K) {
    double xk = x[k];
    int kc = (k / chunk) * chunk;           // first bin of this bin's wave chunk
    row[0] = write32 ? (xk - block_origin(x, kc, K)) : xk;
    for (int term = 0; term < lay.n_terms; ++term)
      for (int c = 0; c < nch; ++c) {
        const int pc = (nch == 2 && c == 1) ? 2 : c;   // merged rows are (A = E, T)
        row[tab_k(term, c, nch)] = ref[term] * tmpl[(term * 3 + pc) * (size_t)K + k] / sigma[pc * (size_t)K + k];
      }
    double n = nk[k];
    if (nch == 2) {
      row[tab_nd(0, lay.n_terms, nch)] =
          n * (D[0 * (size_t)K + k] / sigma[0 * (size_t)K + k] + D[1 * (size_t)K + k] / sigma[1 * (size_t)K + k]);
      row[tab_nd(1, lay.n_terms, nch)] = n * D[2 * (size_t)K + k] / sigma[2 * (size_t)K + k];
    } else {
      for (int c = 0; c < 3; ++c)
        row[tab_nd(c, lay.n_terms, nch)] = n * D[c * (size_t)K + k] / sigma[c * (size_t)K + k];
    }
    row[tab_nl(lay.n_terms, nch)] = n * kLn2;
  } else {
    // abscissa of the last bin keeps every spline piece finite on padding
    int kc = (k / chunk) * chunk;
    row[0] = write32 ? (x[K - 1] - block_origin(x, kc, K)) : x[K - 1];
    for (int r = 1; r < n_tab; ++r) row[r] = 1.0;
    for (int c = 0; c < nch; ++c) row[tab_nd(c, lay.n_terms, nch)] = 0.0;
    row[tab_nl(lay.n_terms, nch)] = 0.0;
  }
  for (int r = 0; r < n_tab; ++r) {
    if (write32)
      tab32[r * (size_t)k_pad + k] = (float)row[r];
    else
      tab64[r * (size_t)k_pad + k] = row[r];
  }
}

// C0 = -sum_c sum_k N_k ln sigma_ck, fixed-order single-block reduction.
__global__ void k_c0(int K, const double* __restrict__ nk, const double* __restrict__ sigma,
                     double* __restrict__ c0) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double l = log(sigma[k]) + log(sigma[(size_t)K + k]) + log(sigma[2 * (size_t)K + k]);
    acc += nk[k] * l;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) c0[0] = -red[0];
}

}  // namespace

hipError_t build_tables(lps_ctx* ctx, hipStream_t s) {
  const int K = ctx->n_bins;
  const int tpb = 256;
  hipLaunchKernelGGL(k_templates, dim3((K + tpb - 1) / tpb), dim3(tpb), 0, s, K, ctx->f, ctx->arm_length,
                     ctx->R, ctx->Rfg, unit_oms_row(ctx->lay) ? 1 : 0, ctx->x, ctx->tmpl, ctx->sigma);
  hipLaunchKernelGGL(k_scaled, dim3((ctx->k_pad64 + tpb - 1) / tpb), dim3(tpb), 0, s, K, ctx->k_pad64, kChunk64,
                     ctx->lay, ctx->x, ctx->nk, ctx->D, ctx->tmpl, ctx->sigma, ctx->tab64, (float*)nullptr, 0);
  hipLaunchKernelGGL(k_scaled, dim3((ctx->k_pad32 + tpb - 1) / tpb), dim3(tpb), 0, s, K, ctx->k_pad32, kChunk32,
                     ctx->lay, ctx->x, ctx->nk, ctx->D, ctx->tmpl, ctx->sigma, (double*)nullptr, ctx->tab32, 1);
  hipLaunchKernelGGL(k_c0, dim3(1), dim3(256), 0, s, K, ctx->nk, ctx->sigma, ctx->c0);
  return hipGetLastError();
}

}  // namespace lps
