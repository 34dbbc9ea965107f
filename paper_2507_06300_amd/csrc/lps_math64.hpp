// Double-precision elementary functions of the batched kernels, written out
// from their textbook constructions: a hardware estimate (v_rcp_f64,
// v_rsq_f64) refined by Newton steps, range reduction plus a polynomial
// (near-minimax, Taylor or atanh series).  Each stays within a few ulp of the
// host C library over the arguments the kernels produce (positive normal
// numbers for the reciprocal, square root and logarithms; lps_math64_check
// exposes them for that test), at a fraction of the cost of the library
// versions, which carry double-double steps.
#pragma once

#include <math.h>

#include "lps_internal.hpp"

namespace lps {

constexpr double kLog2e = 1.442695040888963407359924681001892137426645954153;

// v_fma_f64 with every operand in a register: the addend c (a polynomial
// coefficient at the call sites) in a vector register, or in a scalar register
// pair with kSgpr (for kernels whose vector registers are the scarcer kind).
// (Written out because the compiler otherwise turns a Horner step with a
// constant addend into a move plus a two-address fmac.)
template <bool kSgpr = false>
__device__ inline double fma3(double a, double b, double c) {
  double r;
  if constexpr (kSgpr)
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  else
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// 2^y: y = n + f with n = rint(y), |f| <= 1/2; e^t, t = f ln 2, by the degree-11
// polynomial that interpolates e^t at the 12 Chebyshev nodes of [-ln 2 / 2,
// ln 2 / 2] (coefficients from gen_exp2_poly.py, beside the build script:
// within 0.15 ulp of e^t before the Horner roundings; two FMAs fewer than the
// Taylor series to degree 13), scaled by 2^n.  Propagates NaN; saturates to
// 0 / inf.
template <bool kSgpr = false>
__device__ inline double exp2_d(double y) {
  const double n = rint(y);
  const double t = (y - n) * kLn2;
  double p = 0x1.af631d0059becp-26;
  p = fma3<kSgpr>(p, t, 0x1.28b4057f44145p-22);
  p = fma3<kSgpr>(p, t, 0x1.71ddf5749d126p-19);
  p = fma3<kSgpr>(p, t, 0x1.a01991ac8730ap-16);
  p = fma3<kSgpr>(p, t, 0x1.a01a01b14378fp-13);
  p = fma3<kSgpr>(p, t, 0x1.6c16c187fbe02p-10);
  p = fma3<kSgpr>(p, t, 0x1.111111110f225p-7);
  p = fma3<kSgpr>(p, t, 0x1.555555554f0cfp-5);
  p = fma3<kSgpr>(p, t, 0x1.555555555555ap-3);
  p = fma3<kSgpr>(p, t, 0x1.0000000000011p-1);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  const int e = (int)fmax(fmin(n, 2100.0), -2100.0);
  return ldexp(p, e);
}


// Table for exp2_t: kExp2Tab entries 2^(j / kExp2Tab), j = 0 .. kExp2Tab - 1,
// filled by a kernel from exp2_d (within an ulp).
constexpr int kExp2Shift = 6;
constexpr int kExp2Tab = 1 << kExp2Shift;

__device__ inline void fill_exp2_table(double* tab, int i) {
  if (i < kExp2Tab) tab[i] = exp2_d((double)i * (1.0 / kExp2Tab));
}

// 2^y from a table in LDS: y = n + j / 64 + r with k = rint(64 y) = 64 n + j
// and |r| <= 1/128 (r = y - k/64 is exact), 2^r = e^(r ln 2) by the Taylor
// series to degree 5 (truncation below 2^-54 relative), times tab[j] and 2^n:
// within about two ulp, a dependent chain of ten steps instead of exp2_d's
// eighteen.  Propagates NaN; saturates to 0 / inf.
__device__ inline double exp2_t(double y, const double* tab) {
  const double k = rint(y * (double)kExp2Tab);
  const double r = fma(k, -1.0 / kExp2Tab, y);
  const double t = r * kLn2;
  double p = fma(t, 1.0 / 120.0, 1.0 / 24.0);
  p = fma(p, t, 1.0 / 6.0);
  p = fma(p, t, 0.5);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  const int ki = (int)fmax(fmin(k, 2100.0 * kExp2Tab), -2100.0 * kExp2Tab);
  return ldexp(tab[ki & (kExp2Tab - 1)] * p, ki >> kExp2Shift);
}

// 1/a for a normal positive a: hardware estimate, two Newton steps and a
// residual correction (within an ulp or two).
__device__ inline double rcp_d(double a) {
  double q = __builtin_amdgcn_rcp(a);
  q = fma(fma(-a, q, 1.0), q, q);
  q = fma(fma(-a, q, 1.0), q, q);
  return q;
}


// sqrt x for x >= 0 (0 for x = 0): hardware reciprocal square root estimate,
// one coupled Newton step for sqrt and 1/(2 sqrt), and a residual correction.
__device__ inline double sqrt_d(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : (x == 0.0 ? 0.0 : NAN);
}

// 1/sqrt x for a positive normal x: hardware estimate and two Newton steps
// y <- y + y (1 - x y^2) / 2 (within an ulp or two).
__device__ inline double rsq_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// ln x for a positive normal x: x = m 2^e with m in [1/sqrt2, sqrt2),
// ln m = 2 atanh s, s = (m - 1)/(m + 1), |s| < 0.172, by its odd series to
// s^21 (truncation below 2^-56 relative); e ln 2 with a two-part ln 2 whose
// leading part has trailing zero bits (exact products for |e| < 2^11).
// Non-positive or non-finite x gives NaN (the caller flags the bin).
template <bool kSgpr = false>
__device__ inline double log_d(double x) {
  int e = __builtin_amdgcn_frexp_exp(x);
  double m = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double num = m - 1.0, den = m + 1.0;
  const double r = rcp_d(den);
  double sv = num * r;
  sv = fma(fma(-den, sv, num), r, sv);
  const double z = sv * sv;
  double p = 2.0 / 21.0;
  p = fma3<kSgpr>(p, z, 2.0 / 19.0);
  p = fma3<kSgpr>(p, z, 2.0 / 17.0);
  p = fma3<kSgpr>(p, z, 2.0 / 15.0);
  p = fma3<kSgpr>(p, z, 2.0 / 13.0);
  p = fma3<kSgpr>(p, z, 2.0 / 11.0);
  p = fma3<kSgpr>(p, z, 2.0 / 9.0);
  p = fma3<kSgpr>(p, z, 2.0 / 7.0);
  p = fma3<kSgpr>(p, z, 2.0 / 5.0);
  p = fma3<kSgpr>(p, z, 2.0 / 3.0);
  const double lm = fma(sv * z, p, 2.0 * sv);
  const double fe = (double)e;
  const double res = fma(fe, 6.93147180369123816490e-01, fma(fe, 1.90821492927058770002e-10, lm));
  return x > 0.0 && x < INFINITY ? res : NAN;
}

// log2 x = ln x / ln 2 with the exponent kept exact.
__device__ inline double log2_d(double x) {
  int e = __builtin_amdgcn_frexp_exp(x);
  double m = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double num = m - 1.0, den = m + 1.0;
  const double r = rcp_d(den);
  double sv = num * r;
  sv = fma(fma(-den, sv, num), r, sv);
  const double z = sv * sv;
  double p = 2.0 / 21.0;
  p = fma3(p, z, 2.0 / 19.0);
  p = fma3(p, z, 2.0 / 17.0);
  p = fma3(p, z, 2.0 / 15.0);
  p = fma3(p, z, 2.0 / 13.0);
  p = fma3(p, z, 2.0 / 11.0);
  p = fma3(p, z, 2.0 / 9.0);
  p = fma3(p, z, 2.0 / 7.0);
  p = fma3(p, z, 2.0 / 5.0);
  p = fma3(p, z, 2.0 / 3.0);
  const double lm = fma(sv * z, p, 2.0 * sv);   // ln m
  const double res = fma(lm, kLog2e, (double)e);
  return x > 0.0 && x < INFINITY ? res : (x == 0.0 ? -INFINITY : (x == INFINITY ? INFINITY : NAN));
}

}  // namespace lps
