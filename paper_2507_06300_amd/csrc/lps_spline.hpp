// Device-side Akima spline pieces (App. A), evaluated from a local stencil.
//
// With 0-based knots x_0 < ... < x_{n-1}, segment slopes
//   m_i = (y_{i+1} - y_i) / (x_{i+1} - x_i),   w_i = |m_{i+1} - m_i|,
// the knot slope is Akima's weighted average of the two segment slopes that
// meet at the knot,
//   s_i = (w_i m_{i-1} + w_{i-2} m_i) / (w_i + w_{i-2}),
// with the average (m_{i-1} + m_i)/2 when both weights vanish.  At the two
// knots next to an edge the missing weight is replaced by the nearest
// existing one (s_1 uses w_0 for w_{-1}; s_{n-2} uses w_{n-3} for w_{n-2}),
// and the edge slopes are s_0 = (3 m_0 - m_1)/2, s_{n-1} = (3 m_{n-2} - m_{n-3})/2,
// following the SciPy boundary rule the paper adopts.  Each interval's cubic
// in t = x - x_i has a = y_i, b = s_i, c = (3 m_i - 2 s_i - s_{i+1}) / h_i,
// d = (s_i + s_{i+1} - 2 m_i) / h_i^2.  Fewer than four knots use the linear
// interpolant (b = m_i, c = d = 0).
#pragma once

#include <hip/hip_runtime.h>

namespace lps {

__device__ inline double seg_slope(const double* __restrict__ x, const double* __restrict__ y, int i) {
  return (y[i + 1] - y[i]) / (x[i + 1] - x[i]);
}

__device__ inline double akima_avg(double wr, double ml, double wl, double mr) {
  double den = wr + wl;
  if (den == 0.0) return 0.5 * (ml + mr);
  return (wr * ml + wl * mr) / den;
}

// Knot slope s_i for n >= 4 knots, reading only the knots it depends on.
__device__ inline double akima_knot_slope(const double* __restrict__ x, const double* __restrict__ y, int n,
                                          int i) {
  if (i == 0) return 0.5 * (3.0 * seg_slope(x, y, 0) - seg_slope(x, y, 1));
  if (i == n - 1) return 0.5 * (3.0 * seg_slope(x, y, n - 2) - seg_slope(x, y, n - 3));
  // w_r = |m_{i+1} - m_i| (clamped to w_{n-3} at i = n-2), w_l = |m_{i-1} - m_{i-2}| (w_0 at i = 1)
  int ir = i < n - 2 ? i : n - 3;
  int il = i - 2 > 0 ? i - 2 : 0;
  double m_l = seg_slope(x, y, i - 1);
  double m_r = seg_slope(x, y, i);
  double wr = fabs(seg_slope(x, y, ir + 1) - seg_slope(x, y, ir));
  double wl = fabs(seg_slope(x, y, il + 1) - seg_slope(x, y, il));
  return akima_avg(wr, m_l, wl, m_r);
}

// Cubic coefficients of interval i (0 <= i <= n-2) for n >= 2 knots.
__device__ inline void spline_piece(const double* __restrict__ x, const double* __restrict__ y, int n, int i,
                                    double& a, double& b, double& c, double& d) {
  a = y[i];
  if (n < 4) {
    b = seg_slope(x, y, i);
    c = 0.0;
    d = 0.0;
    return;
  }
  double h = x[i + 1] - x[i];
  double m = (y[i + 1] - y[i]) / h;
  double s0 = akima_knot_slope(x, y, n, i);
  double s1 = akima_knot_slope(x, y, n, i + 1);
  b = s0;
  c = (3.0 * m - 2.0 * s0 - s1) / h;
  d = (s0 + s1 - 2.0 * m) / (h * h);
}

}  // namespace lps
