// Per-bin noise and background templates shared by the table builders.
#pragma once

#include <math.h>

#include "lps_internal.hpp"

namespace lps {

// Per-bin templates at unit amplitudes: the A/E and T noise transfer of
// Eq. (noise_tdi) (prefactor sin^2 xi sin^2 2xi, xi = 2 pi f L / c) times the
// single-link OMS PSD per unit A_OMS^2 and TM PSD per unit A_TM^2 of Sec.
// "Parametrized noise model", and the background factor 3 (H0/h)^2 / (4 pi^2 f^3)
// of Eq. (Sh) per unit h^2 Omega (to be multiplied by the response R_c).
__device__ inline void unit_templates(double fk, double L, double& oms_ae, double& oms_t, double& tm_ae,
                                      double& tm_t, double& h) {
  const double xi = 2.0 * kPi * fk * L / kClight;
  const double sx = sin(xi), cx = cos(xi), s2x = sin(2.0 * xi);
  const double pref = sx * sx * s2x * s2x;
  const double r2 = 2.0e-3 / fk;
  const double s_oms = (1.0 + r2 * r2 * r2 * r2) * (2.0 * kPi * fk / kClight) * (2.0 * kPi * fk / kClight);
  const double r4 = 0.4e-3 / fk, r8 = fk / 8.0e-3;
  const double q = 1.0 / (2.0 * kPi * fk * kClight);
  const double s_tm = (1.0 + r4 * r4) * (1.0 + r8 * r8 * r8 * r8) * q * q;
  oms_ae = 32.0 * pref * (2.0 + cx) * s_oms;
  tm_ae = 32.0 * pref * 4.0 * (1.0 + cx + cx * cx) * s_tm;
  // 1 - cos xi as 2 sin^2(xi/2), free of cancellation at low frequency
  const double sh = sin(0.5 * xi);
  const double omc = 2.0 * sh * sh;
  oms_t = 64.0 * pref * omc * s_oms;
  tm_t = 64.0 * pref * 2.0 * omc * omc * s_tm;
  h = 3.0 * kH0PerH * kH0PerH / (4.0 * kPi * kPi * fk * fk * fk);
}

}  // namespace lps
