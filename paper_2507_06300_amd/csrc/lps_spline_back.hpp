// Reverse-mode derivative of the Akima / linear spline construction (App. A)
// with respect to the knots, one wave per spline and one lane per knot; shared
// by the adjoints of the diagonal and the full-covariance likelihoods.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "lps_batched.hpp"
#include "lps_internal.hpp"
#include "lps_spline.hpp"

namespace lps {

// Per-wave LDS of the spline backward.
struct BackLds {
  double m[kMaxKnots], h[kMaxKnots], s[kMaxKnots], w[kMaxKnots];
  double sbn[kMaxKnots], sb[kMaxKnots], pl[kMaxKnots], pr[kMaxKnots], cr[kMaxKnots], cl[kMaxKnots];
  double wbs[kMaxKnots], q[kMaxKnots], hb[kMaxKnots];
};

// Backward through the spline construction of App. A for one spline of n
// knots, one lane per knot (and per piece: piece i spans knots i, i+1).
// M0..M3 are the moments of dlogL/dP over the lane's piece (already times
// ln 10).  Forward quantities: h_i, m_i (segments), w_i = |m_{i+1} - m_i|,
// knot slopes s_i; pieces a = y_i, b = s_i, c, d.  Every scatter of the
// sequential adjoint becomes a gather of fixed neighbours through LDS.
__device__ inline void spline_backward_wave(int lane, const double* __restrict__ x, const double* __restrict__ y, int n,
                                     const double (&M)[4], double* __restrict__ dy, double* __restrict__ dx,
                                     BackLds& L) {
  const int i = lane;
  const bool knot = i < n, seg = i + 1 < n;
  const double xi = knot ? x[i] : 0.0;
  const double yi = knot ? y[i] : 0.0;
  double hi = 1.0, mi = 0.0;
  if (seg) {
    hi = x[i + 1] - xi;
    mi = (y[i + 1] - yi) / hi;
  }
  L.m[i] = mi;
  L.h[i] = hi;
  wave_lds_sync();
  const bool akima = n >= 4;
  double si = mi;
  if (akima) {
    if (i + 2 < n) L.w[i] = fabs(L.m[i + 1] - mi);
    wave_lds_sync();
    if (i == 0) si = 0.5 * (3.0 * L.m[0] - L.m[1]);
    else if (i == n - 1) si = 0.5 * (3.0 * L.m[n - 2] - L.m[n - 3]);
    else if (i < n - 1) {
      const int ir = i < n - 2 ? i : n - 3;
      const int il = i - 2 > 0 ? i - 2 : 0;
      si = akima_avg(L.w[ir], L.m[i - 1], L.w[il], mi);
    }
    L.s[i] = si;
    wave_lds_sync();
  }
  // pieces -> (y, s, m, h, x)
  double yb = 0.0, xb = 0.0, sbo = 0.0, sbn = 0.0, mb = 0.0, hb = 0.0;
  if (seg) {
    if (akima) {
      const double s1 = L.s[i + 1];
      const double h2 = hi * hi;
      const double c = (3.0 * mi - 2.0 * si - s1) / hi;
      const double d = (si + s1 - 2.0 * mi) / h2;
      yb = M[0];
      xb = -(si * M[0] + 2.0 * c * M[1] + 3.0 * d * M[2]);   // t = x - x_i
      sbo = M[1] - 2.0 * M[2] / hi + M[3] / h2;
      sbn = -M[2] / hi + M[3] / h2;
      mb = 3.0 * M[2] / hi - 2.0 * M[3] / h2;
      hb = -M[2] * c / hi - 2.0 * M[3] * d / hi;
    } else {
      yb = M[0];
      mb = M[1];
      xb = -mi * M[0];
    }
  }
  if (akima) {
    L.sbn[i] = sbn;
    wave_lds_sync();
    const double sbi = knot ? sbo + (i >= 1 ? L.sbn[i - 1] : 0.0) : 0.0;
    // knot slopes -> (m, w)
    double pl = 0.0, pr = 0.0, cr = 0.0, cl = 0.0;
    if (i >= 1 && i <= n - 2) {
      const int ir = i < n - 2 ? i : n - 3;
      const int il = i - 2 > 0 ? i - 2 : 0;
      const double wr = L.w[ir], wl = L.w[il], den = wr + wl;
      if (den == 0.0) {
        pl = 0.5 * sbi;
        pr = 0.5 * sbi;
      } else {
        pl = sbi * wr / den;
        pr = sbi * wl / den;
        cr = sbi * (L.m[i - 1] - si) / den;
        cl = sbi * (mi - si) / den;
      }
    }
    L.sb[i] = sbi;
    L.pl[i] = pl;
    L.pr[i] = pr;
    L.cr[i] = cr;
    L.cl[i] = cl;
    wave_lds_sync();
    // segment k = i gathers the knot-slope terms aimed at m_k
    if (seg) {
      if (i >= 1 && i <= n - 2) mb += L.pr[i];
      if (i + 1 <= n - 2) mb += L.pl[i + 1];
      if (i == 0) mb += 1.5 * L.sb[0];
      if (i == 1) mb -= 0.5 * L.sb[0];
      if (i == n - 2) mb += 1.5 * L.sb[n - 1];
      if (i == n - 3) mb -= 0.5 * L.sb[n - 1];
    }
    // slope weight k = i gathers the terms aimed at w_k (clamped stencils at both ends)
    double ws = 0.0;
    if (i <= n - 3) {
      double wb = 0.0;
      if (i >= 1) wb += L.cr[i];
      if (i == n - 3) wb += L.cr[n - 2];
      if (i + 2 <= n - 2) wb += L.cl[i + 2];
      if (i == 0) wb += L.cl[1];
      const double dlt = L.m[i + 1] - mi;
      const double sg = dlt > 0.0 ? 1.0 : (dlt < 0.0 ? -1.0 : 0.0);
      ws = wb * sg;
    }
    L.wbs[i] = ws;
    wave_lds_sync();
    if (seg) mb += (i >= 1 ? L.wbs[i - 1] : 0.0) - ws;
  }
  // segment slopes m_i = (y_{i+1} - y_i) / h_i and widths h_i = x_{i+1} - x_i
  double q = 0.0;
  if (seg) {
    q = mb / hi;
    hb -= mb * mi / hi;
  } else {
    hb = 0.0;
  }
  L.q[i] = q;
  L.hb[i] = hb;
  wave_lds_sync();
  if (knot) {
    yb += (i >= 1 ? L.q[i - 1] : 0.0) - q;
    xb += (i >= 1 ? L.hb[i - 1] : 0.0) - hb;
    dy[i] = yb;
    dx[i] = (i == 0 || i == n - 1) ? 0.0 : xb;
  }
  wave_lds_sync();
}

}  // namespace lps
