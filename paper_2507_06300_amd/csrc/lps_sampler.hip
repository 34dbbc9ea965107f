// Parallel-tempered reversible-jump sampler sweep, entirely on the device.
//
// Chains c = t * W + w (temperature t, walker w) keep their states in a padded
// CSR layout with a fixed capacity per spline slot, so knots are inserted and
// removed in place and every sweep is a fixed sequence of launches on one
// stream (capturable in a HIP graph; the sweep counter lives in device memory).
//
// One sweep:
//  1. within-model move: preconditioned Langevin (MALA) proposal for all
//     continuous parameters (template parameters, knot heights, interior knot
//     positions) driven by the adjoint gradient of logL; the tempered target is
//     beta_t logL + log prior, with the priors of Table I;
//  2. logL and gradient of the proposals (lps_loglike_grad_batch kernels);
//  3. Metropolis-Hastings accept/reject in FP64 with the Langevin proposal
//     densities in both directions;
//  4. between-models move per chain on one randomly chosen spline: birth of an
//     in-between knot drawn from the prior (position uniform over the band,
//     height N(0, 0.1)) or death of a uniformly chosen in-between knot, each
//     with probability 1/2 (Sec. "Power spectral density breakdown");
//  5. logL and gradient of the proposals;
//  6. accept with probability min(1, (L'/L)^beta_t): with births from the
//     prior, a uniform prior on the number of in-between knots and equal
//     birth/death probabilities, the prior and proposal densities cancel;
//  7. optionally, ensemble stretch moves of the template parameters within each
//     temperature, the two walker halves in turn (with their adjoint evaluations);
//  8. swaps between adjacent temperatures of each walker (even pairs on even
//     sweeps, odd pairs on odd sweeps): accept min(1, exp((b_t - b_{t+1})(L_{t+1} - L_t)));
//  9. advance the sweep counter.
// Random numbers come from the counter-based Philox4x32-10 generator of
// Salmon, Moraes, Dror and Shaw (SC 2011), keyed by the seed and indexed by
// (chain, sweep, purpose, draw), so results do not depend on launch shapes
// and a run resumed from saved states continues the same streams.
#include <math.h>
#include <string.h>

#include <vector>

#include "lps_internal.hpp"
#include "lps_validate.hpp"
#include "lps_roctx.hpp"

namespace lps {

struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

}  // namespace lps

// ---------------------------------------------------------------------------
struct lps_sampler {
  lps_ctx* ctx;
  int W, T, C, P, NS, KC;          // walkers, temperatures, chains, params, splines, slot capacity
  uint64_t seed;
  double eps;
  lps_precision prec;
  double x_lo, x_hi;               // band edges (log10 f of the first and last bin)
  // current and proposed chain states (padded CSR)
  double *cp, *pp;                 // params [P][C]
  int32_t* off;                    // [C*NS] slot starts (shared)
  int32_t *ccnt, *pcnt;            // counts [C*NS]
  double *cx, *cy, *px, *py;       // knots [C*NS*KC]
  double *cl, *pl;                 // logL [C]
  uint32_t *cst, *pst;             // status [C]
  double *cgp, *pgp;               // dlogL/dparams [P][C]
  double *cgx, *cgy, *pgx, *pgy;   // dlogL/dknots [C*NS*KC]
  int32_t* flag;                   // [C] proposal admissible
  double* beta;                    // [T]
  double* scale;                   // [T] step multiplier per temperature
  unsigned long long* sweep;       // [1] sweep counter
  uint32_t* counters;              // [kKinds][T][2]: proposed, accepted
  uint32_t fixed;                  // bit p: template parameter p is not moved
  int rj;                          // birth/death moves on (1) or off (0)
  int stretch;                     // ensemble stretch moves on (1) or off (0)
  double* zs;                      // [C] stretch factor of the pending stretch proposal
};

namespace lps {
namespace {

enum Purpose : uint32_t { kPMala = 1, kPMalaAcc = 2, kPRj = 3, kPRjAcc = 4, kPSwap = 5, kPStretch = 6,
                          kPStretchAcc = 7 };
constexpr int kKinds = 5;            // Langevin, birth, death, swap, stretch
constexpr double kStretchA = 2.0;    // stretch factors z in [1/a, a], density proportional to 1/sqrt(z)

struct Rng {
  uint32_t k0, k1, chain, slo, shi, purpose;
  __device__ U4 block(uint32_t i) const {
    U4 c = {chain, slo, shi, (purpose << 24) ^ i};
    return philox4x32_10(c, k0, k1);
  }
  // 53-bit uniform in (0, 1) from two 32-bit words
  __device__ static double u01(uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * (1.0 / 9007199254740992.0);
  }
  // pair of standard normals (Box-Muller) from draw block i
  __device__ void normal2(uint32_t i, double& z0, double& z1) const {
    const U4 r = block(i);
    const double u1 = u01(r.x, r.y), u2 = u01(r.z, r.w);
    const double rad = sqrt(-2.0 * log(u1));
    z0 = rad * cos(2.0 * kPi * u2);
    z1 = rad * sin(2.0 * kPi * u2);
  }
  __device__ double uniform(uint32_t i) const {
    const U4 r = block(i);
    return u01(r.x, r.y);
  }
};

__device__ inline Rng make_rng(uint64_t seed, const unsigned long long* sweep, int chain, uint32_t purpose) {
  const unsigned long long sw = *sweep;
  Rng g;
  g.k0 = (uint32_t)seed;
  g.k1 = (uint32_t)(seed >> 32);
  g.chain = (uint32_t)chain;
  g.slo = (uint32_t)sw;
  g.shi = (uint32_t)(sw >> 32);
  g.purpose = purpose;
  return g;
}

// Table I priors (plus the foreground amplitude stand-in) and the height prior width.
constexpr double kSigmaW = 0.1;
__device__ inline bool param_in_prior(int p, double v) {
  switch (p) {
    case LPS_P_AOMS: return v >= 1e-2 * 1e-12 && v <= 1e2 * 1e-12;
    case LPS_P_ATM: return v >= 1e-2 * 1e-15 && v <= 1e2 * 1e-15;
    case LPS_P_U: return v >= -20.0 && v <= -10.0;
    case LPS_P_ALPHA: return v >= -5.0 && v <= 5.0;
    default: return v >= -40.0 && v <= -36.0;
  }
}
// Langevin step scales (square root of the diagonal preconditioner)
__device__ inline double param_scale(int p) {
  switch (p) {
    case LPS_P_AOMS: return 1e-14;
    case LPS_P_ATM: return 3e-18;
    default: return 1e-3;
  }
}
constexpr double kScaleY = 1e-3, kScaleX = 1e-3;

// Every sweep kernel runs one wave per chain (or chain pair) with one lane per
// knot slot (capacity <= 64), so knot loops become lane-parallel and the
// accesses of a chain's padded slots are contiguous.
__device__ inline int wave_chain(int n) {
  const int c = uniform((int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave));
  return c < n ? c : -1;
}

// standard normal number d of a chain's stream (pairs from Box-Muller blocks)
__device__ inline double normal_at(const Rng& g, uint32_t d) {
  double z0, z1;
  g.normal2(d >> 1, z0, z1);
  return (d & 1u) ? z1 : z0;
}

// log prior (up to a constant) of a chain state; -inf outside the support.
// Identical on every lane of the wave.
__device__ double log_prior(int lane, const double* p, int P, int C, int c, const int32_t* off, const int32_t* cnt,
                            const double* kx, const double* ky, int NS, double x_lo, double x_hi) {
  bool out = lane < P && !param_in_prior(lane, p[lane * (size_t)C + c]);
  double lp = 0.0;
  for (int j = 0; j < NS; ++j) {
    const int a = off[c * NS + j], n = cnt[c * NS + j];
    const int i = lane;
    if (i < n) {
      const double y = ky[a + i];
      lp -= 0.5 * (y / kSigmaW) * (y / kSigmaW);
      if (i > 0 && i < n - 1) {
        const double x = kx[a + i];
        if (!(x > x_lo && x < x_hi) || !(x > kx[a + i - 1])) out = true;
      }
    }
  }
  if (__ballot(out)) return -INFINITY;
  return wave_sum(lp);
}

struct ChainView {
  double* p;
  int32_t* cnt;
  double *x, *y, *l;
  uint32_t* st;
  double *gp, *gx, *gy;
};

__device__ inline void copy_chain(int lane, const ChainView& s, const ChainView& d, int c, int C, int P, int NS,
                                  const int32_t* off, bool with_grad) {
  if (lane < P) {
    d.p[lane * (size_t)C + c] = s.p[lane * (size_t)C + c];
    if (with_grad) d.gp[lane * (size_t)C + c] = s.gp[lane * (size_t)C + c];
  }
  for (int j = 0; j < NS; ++j) {
    const int a = off[c * NS + j];
    const int n = s.cnt[c * NS + j];
    if (lane == 0) d.cnt[c * NS + j] = n;
    if (lane < n) {
      d.x[a + lane] = s.x[a + lane];
      d.y[a + lane] = s.y[a + lane];
      if (with_grad) {
        d.gx[a + lane] = s.gx[a + lane];
        d.gy[a + lane] = s.gy[a + lane];
      }
    }
  }
  if (with_grad && lane == 0) {
    d.l[c] = s.l[c];
    d.st[c] = s.st[c];
  }
}

// ---- 1. Langevin proposal ----------------------------------------------------
// Normal number order per chain: the P template parameters, then per spline
// and knot the height and (interior knots only) the position.
__global__ __launch_bounds__(256) void k_mala_propose(lps_sampler sm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = wave_chain(sm.C);
  if (c < 0) return;
  const int t = c / sm.W;
  const double beta = sm.beta[t];
  const double h = sm.eps * sm.scale[t];
  const Rng g = make_rng(sm.seed, sm.sweep, c, kPMala);
  const int C = sm.C;
  if (lane < sm.P) {
    const int q = lane;
    if ((sm.fixed >> q) & 1u) {
      sm.pp[q * (size_t)C + c] = sm.cp[q * (size_t)C + c];
    } else {
      const double s = h * param_scale(q);
      const double grad = beta * sm.cgp[q * (size_t)C + c];
      sm.pp[q * (size_t)C + c] = sm.cp[q * (size_t)C + c] + 0.5 * s * s * grad + s * normal_at(g, (uint32_t)q);
    }
  }
  uint32_t base = (uint32_t)sm.P;
  for (int j = 0; j < sm.NS; ++j) {
    const int a = sm.off[c * sm.NS + j], n = sm.ccnt[c * sm.NS + j];
    if (lane == 0) sm.pcnt[c * sm.NS + j] = n;
    const int i = lane;
    if (i < n) {
      const uint32_t dy = base + (i == 0 ? 0u : 2u * i - 1u);
      const double y = sm.cy[a + i];
      const double sy = h * kScaleY;
      const double gy = beta * sm.cgy[a + i] - y / (kSigmaW * kSigmaW);
      sm.py[a + i] = y + 0.5 * sy * sy * gy + sy * normal_at(g, dy);
      const double x = sm.cx[a + i];
      if (i == 0 || i == n - 1) {
        sm.px[a + i] = x;   // edge abscissae are fixed
      } else {
        const double sx = h * kScaleX;
        sm.px[a + i] = x + 0.5 * sx * sx * beta * sm.cgx[a + i] + sx * normal_at(g, dy + 1u);
      }
    }
    base += (uint32_t)(n >= 2 ? 2 * n - 2 : n);
  }
}

// log q(to | from) of the Langevin proposal (up to a constant), with the
// gradient of the tempered log target at `from`.  Identical on every lane.
__device__ double log_q(int lane, const ChainView& from, const ChainView& to, int c, int C, int P, int NS,
                        const int32_t* off, double beta, double h, uint32_t fixed) {
  double acc = 0.0;
  if (lane < P && !((fixed >> lane) & 1u)) {
    const int q = lane;
    const double s = h * param_scale(q);
    const double m = from.p[q * (size_t)C + c] + 0.5 * s * s * beta * from.gp[q * (size_t)C + c];
    const double d = (to.p[q * (size_t)C + c] - m) / s;
    acc -= 0.5 * d * d;
  }
  for (int j = 0; j < NS; ++j) {
    const int a = off[c * NS + j], n = from.cnt[c * NS + j];
    const int i = lane;
    if (i < n) {
      const double sy = h * kScaleY;
      const double gy = beta * from.gy[a + i] - from.y[a + i] / (kSigmaW * kSigmaW);
      const double dy = (to.y[a + i] - from.y[a + i] - 0.5 * sy * sy * gy) / sy;
      acc -= 0.5 * dy * dy;
      if (i > 0 && i < n - 1) {
        const double sx = h * kScaleX;
        const double dx = (to.x[a + i] - from.x[a + i] - 0.5 * sx * sx * beta * from.gx[a + i]) / sx;
        acc -= 0.5 * dx * dx;
      }
    }
  }
  return wave_sum(acc);
}

// ---- 3. Langevin accept --------------------------------------------------------
__global__ __launch_bounds__(256) void k_mala_accept(lps_sampler sm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = wave_chain(sm.C);
  if (c < 0) return;
  const int t = c / sm.W;
  const double beta = sm.beta[t];
  const double h = sm.eps * sm.scale[t];
  const ChainView cur = {sm.cp, sm.ccnt, sm.cx, sm.cy, sm.cl, sm.cst, sm.cgp, sm.cgx, sm.cgy};
  const ChainView pro = {sm.pp, sm.pcnt, sm.px, sm.py, sm.pl, sm.pst, sm.pgp, sm.pgx, sm.pgy};
  bool accept = false;
  if (sm.pst[c] == 0 && isfinite(sm.pl[c])) {
    const double lp1 = log_prior(lane, sm.pp, sm.P, sm.C, c, sm.off, sm.pcnt, sm.px, sm.py, sm.NS, sm.x_lo, sm.x_hi);
    if (isfinite(lp1)) {
      const double lp0 =
          log_prior(lane, sm.cp, sm.P, sm.C, c, sm.off, sm.ccnt, sm.cx, sm.cy, sm.NS, sm.x_lo, sm.x_hi);
      const double dl = (sm.pl[c] - sm.cl[c]) * beta;
      const double la = dl + (lp1 - lp0) + log_q(lane, pro, cur, c, sm.C, sm.P, sm.NS, sm.off, beta, h, sm.fixed) -
                        log_q(lane, cur, pro, c, sm.C, sm.P, sm.NS, sm.off, beta, h, sm.fixed);
      const double u = make_rng(sm.seed, sm.sweep, c, kPMalaAcc).uniform(0);
      accept = log(u) < la;
    }
  }
  if (lane == 0) {
    atomicAdd(&sm.counters[(0 * sm.T + t) * 2 + 0], 1u);
    if (accept) atomicAdd(&sm.counters[(0 * sm.T + t) * 2 + 1], 1u);
  }
  if (accept) copy_chain(lane, pro, cur, c, sm.C, sm.P, sm.NS, sm.off, true);
}

// ---- 4. birth / death proposal -------------------------------------------------
__global__ __launch_bounds__(256) void k_rj_propose(lps_sampler sm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = wave_chain(sm.C);
  if (c < 0) return;
  const ChainView cur = {sm.cp, sm.ccnt, sm.cx, sm.cy, sm.cl, sm.cst, sm.cgp, sm.cgx, sm.cgy};
  const ChainView pro = {sm.pp, sm.pcnt, sm.px, sm.py, sm.pl, sm.pst, sm.pgp, sm.pgx, sm.pgy};
  copy_chain(lane, cur, pro, c, sm.C, sm.P, sm.NS, sm.off, false);
  const Rng g = make_rng(sm.seed, sm.sweep, c, kPRj);
  const U4 r0 = g.block(0);
  const int j = (int)(r0.x % (uint32_t)sm.NS);
  const bool birth = (r0.y & 1u) != 0;
  const int a = sm.off[c * sm.NS + j];
  const int n = sm.ccnt[c * sm.NS + j];
  const int k_in = n - 2;
  const int i = lane;
  int ok = 0;
  if (n == 0) {
    // a disabled spline stays disabled: no proposal (counted as rejected)
  } else if (birth && n < sm.KC) {
    const double xs = sm.x_lo + (sm.x_hi - sm.x_lo) * Rng::u01(r0.z, r0.w);
    double z0, z1;
    g.normal2(1, z0, z1);
    const double ys = kSigmaW * z0;
    // insert after the interior knots at or below xs (edges stay put)
    const int p = 1 + __popcll(__ballot(i >= 1 && i <= n - 2 && sm.cx[a + i] <= xs));
    if (i <= n) {
      const double nx = i < p ? sm.cx[a + i] : (i == p ? xs : sm.cx[a + i - 1]);
      const double ny = i < p ? sm.cy[a + i] : (i == p ? ys : sm.cy[a + i - 1]);
      sm.px[a + i] = nx;
      sm.py[a + i] = ny;
    }
    if (lane == 0) sm.pcnt[c * sm.NS + j] = n + 1;
    ok = (xs > sm.x_lo && xs < sm.x_hi) ? 1 : 0;
  } else if (!birth && k_in > 0) {
    const U4 r1 = g.block(2);
    const int d = 1 + (int)(r1.x % (uint32_t)k_in);   // interior knot to remove
    if (i >= d && i < n - 1) {
      sm.px[a + i] = sm.cx[a + i + 1];
      sm.py[a + i] = sm.cy[a + i + 1];
    }
    if (lane == 0) sm.pcnt[c * sm.NS + j] = n - 1;
    ok = 1;
  }
  if (lane == 0) sm.flag[c] = ok ? (birth ? 1 : 2) : 0;
}

// ---- 6. birth / death accept ---------------------------------------------------
__global__ __launch_bounds__(256) void k_rj_accept(lps_sampler sm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = wave_chain(sm.C);
  if (c < 0) return;
  const int t = c / sm.W;
  const int kind = sm.flag[c];           // 1 birth, 2 death, 0 impossible (rejected)
  const int slot = kind == 2 ? 2 : 1;
  bool accept = false;
  if (kind != 0 && sm.pst[c] == 0 && isfinite(sm.pl[c])) {
    const double la = sm.beta[t] * (sm.pl[c] - sm.cl[c]);
    const double u = make_rng(sm.seed, sm.sweep, c, kPRjAcc).uniform(0);
    accept = log(u) < la;
  }
  if (lane == 0) {
    atomicAdd(&sm.counters[(slot * sm.T + t) * 2 + 0], 1u);
    if (accept) atomicAdd(&sm.counters[(slot * sm.T + t) * 2 + 1], 1u);
  }
  if (accept) {
    const ChainView cur = {sm.cp, sm.ccnt, sm.cx, sm.cy, sm.cl, sm.cst, sm.cgp, sm.cgx, sm.cgy};
    const ChainView pro = {sm.pp, sm.pcnt, sm.px, sm.py, sm.pl, sm.pst, sm.pgp, sm.pgx, sm.pgy};
    copy_chain(lane, pro, cur, c, sm.C, sm.P, sm.NS, sm.off, true);
  }
}

__device__ inline void swap_d(double& a, double& b) {
  const double t = a;
  a = b;
  b = t;
}

// ---- 7. temperature swaps --------------------------------------------------------
__global__ __launch_bounds__(256) void k_swap(lps_sampler sm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int parity = (int)(*sm.sweep & 1ull);
  const int npair = sm.T / 2 + 1;
  const int id = wave_chain(sm.W * npair);
  if (id < 0) return;
  const int w = id % sm.W, pair = id / sm.W;
  const int t = 2 * pair + parity;
  if (t + 1 >= sm.T) return;
  const int c1 = t * sm.W + w, c2 = (t + 1) * sm.W + w;
  const double la = (sm.beta[t] - sm.beta[t + 1]) * (sm.cl[c2] - sm.cl[c1]);
  const double u = make_rng(sm.seed, sm.sweep, c1, kPSwap).uniform(0);
  const bool accept = log(u) < la;
  if (lane == 0) {
    atomicAdd(&sm.counters[(3 * sm.T + t) * 2 + 0], 1u);
    if (accept) atomicAdd(&sm.counters[(3 * sm.T + t) * 2 + 1], 1u);
  }
  if (!accept) return;
  const int C = sm.C;
  if (lane < sm.P) {
    const int q = lane;
    swap_d(sm.cp[q * (size_t)C + c1], sm.cp[q * (size_t)C + c2]);
    swap_d(sm.cgp[q * (size_t)C + c1], sm.cgp[q * (size_t)C + c2]);
  }
  for (int j = 0; j < sm.NS; ++j) {
    const int a1 = sm.off[c1 * sm.NS + j], a2 = sm.off[c2 * sm.NS + j];
    const int n1 = sm.ccnt[c1 * sm.NS + j], n2 = sm.ccnt[c2 * sm.NS + j];
    const int n = n1 > n2 ? n1 : n2;
    const int i = lane;
    if (i < n) {
      swap_d(sm.cx[a1 + i], sm.cx[a2 + i]);
      swap_d(sm.cy[a1 + i], sm.cy[a2 + i]);
      swap_d(sm.cgx[a1 + i], sm.cgx[a2 + i]);
      swap_d(sm.cgy[a1 + i], sm.cgy[a2 + i]);
    }
    if (lane == 0) {
      sm.ccnt[c1 * sm.NS + j] = n2;
      sm.ccnt[c2 * sm.NS + j] = n1;
    }
  }
  if (lane == 0) {
    swap_d(sm.cl[c1], sm.cl[c2]);
    const uint32_t s1 = sm.cst[c1];
    sm.cst[c1] = sm.cst[c2];
    sm.cst[c2] = s1;
  }
}

// ---- 8. ensemble stretch move on the template parameters --------------------------
// Affine-invariant stretch move (Goodman and Weare 2010) within each
// temperature: the walkers are split into halves w < h and w >= h (h = W / 2);
// a chain of the moving half draws a partner j uniformly from the other half
// at its temperature and z from g(z) ~ 1/sqrt(z) on [1/a, a], and proposes
// theta' = theta_j + z (theta - theta_j) for its free template parameters
// (knots unchanged).  Accept: (d - 1) log z + beta (L' - L) + log prior ratio,
// d = number of free parameters.  Chains of the resting half propose their
// current state (and are not updated).
__device__ inline bool in_half(int w, int W, int half) { return (w < W / 2) == (half == 0); }

__global__ __launch_bounds__(256) void k_stretch_propose(lps_sampler sm, int half) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = wave_chain(sm.C);
  if (c < 0) return;
  const ChainView cur = {sm.cp, sm.ccnt, sm.cx, sm.cy, sm.cl, sm.cst, sm.cgp, sm.cgx, sm.cgy};
  const ChainView pro = {sm.pp, sm.pcnt, sm.px, sm.py, sm.pl, sm.pst, sm.pgp, sm.pgx, sm.pgy};
  copy_chain(lane, cur, pro, c, sm.C, sm.P, sm.NS, sm.off, false);
  const int t = c / sm.W, w = c - t * sm.W;
  if (!in_half(w, sm.W, half)) return;
  const int h = sm.W / 2;
  const int lo = half == 0 ? h : 0, n_other = half == 0 ? sm.W - h : h;
  const Rng g = make_rng(sm.seed, sm.sweep, c, kPStretch + 8u * (uint32_t)half);
  const U4 r = g.block(0);
  const int j = t * sm.W + lo + (int)(r.x % (uint32_t)n_other);
  const double u = Rng::u01(r.y, r.z);
  const double sq = (kStretchA - 1.0) * u + 1.0;
  const double z = sq * sq / kStretchA;
  if (lane == 0) sm.zs[c] = z;
  if (lane < sm.P && !((sm.fixed >> lane) & 1u)) {
    const size_t q = (size_t)lane * sm.C;
    sm.pp[q + c] = sm.cp[q + j] + z * (sm.cp[q + c] - sm.cp[q + j]);
  }
}

__global__ __launch_bounds__(256) void k_stretch_accept(lps_sampler sm, int half) {
  const int lane = threadIdx.x & (kWave - 1);
  const int c = wave_chain(sm.C);
  if (c < 0) return;
  const int t = c / sm.W, w = c - t * sm.W;
  if (!in_half(w, sm.W, half)) return;
  int d = 0;
  for (int q = 0; q < sm.P; ++q) d += ((sm.fixed >> q) & 1u) ? 0 : 1;
  bool accept = false;
  if (sm.pst[c] == 0 && isfinite(sm.pl[c])) {
    const double lp1 = log_prior(lane, sm.pp, sm.P, sm.C, c, sm.off, sm.pcnt, sm.px, sm.py, sm.NS, sm.x_lo, sm.x_hi);
    if (isfinite(lp1)) {
      const double lp0 =
          log_prior(lane, sm.cp, sm.P, sm.C, c, sm.off, sm.ccnt, sm.cx, sm.cy, sm.NS, sm.x_lo, sm.x_hi);
      const double la = (d - 1) * log(sm.zs[c]) + sm.beta[t] * (sm.pl[c] - sm.cl[c]) + (lp1 - lp0);
      const double u = make_rng(sm.seed, sm.sweep, c, kPStretchAcc + 8u * (uint32_t)half).uniform(0);
      accept = log(u) < la;
    }
  }
  if (lane == 0) {
    atomicAdd(&sm.counters[(4 * sm.T + t) * 2 + 0], 1u);
    if (accept) atomicAdd(&sm.counters[(4 * sm.T + t) * 2 + 1], 1u);
  }
  if (accept) {
    const ChainView cur = {sm.cp, sm.ccnt, sm.cx, sm.cy, sm.cl, sm.cst, sm.cgp, sm.cgx, sm.cgy};
    const ChainView pro = {sm.pp, sm.pcnt, sm.px, sm.py, sm.pl, sm.pst, sm.pgp, sm.pgx, sm.pgy};
    copy_chain(lane, pro, cur, c, sm.C, sm.P, sm.NS, sm.off, true);
  }
}

__global__ void k_advance(unsigned long long* sweep) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *sweep += 1ull;
}

// Initial state: packed CSR input -> padded slots.
__global__ void k_load(lps_sampler sm, const double* __restrict__ params, const int32_t* __restrict__ off,
                       int64_t n_knots, const double* __restrict__ kx, const double* __restrict__ ky,
                       int32_t* __restrict__ bad) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= sm.C) return;
  for (int q = 0; q < sm.P; ++q) sm.cp[q * (size_t)sm.C + c] = params[q * (size_t)sm.C + c];
  for (int j = 0; j < sm.NS; ++j) {
    const int a = off[c * sm.NS + j];
    const int n = off[c * sm.NS + j + 1] - a;
    const int d = sm.off[c * sm.NS + j];
    if (n == 1 || n < 0 || n > sm.KC || a < 0 || (int64_t)a + n > n_knots) {   // 0 = disabled spline
      atomicOr(bad, 1);
      sm.ccnt[c * sm.NS + j] = 0;
      continue;
    }
    sm.ccnt[c * sm.NS + j] = n;
    for (int i = 0; i < n; ++i) {
      sm.cx[d + i] = kx[a + i];
      sm.cy[d + i] = ky[a + i];
    }
  }
}

__global__ void k_slot_offsets(int n_slots, int KC, int32_t* __restrict__ off) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_slots) off[i] = i * KC;
}

__global__ void k_zero_u32(int n, uint32_t* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_philox_fill(uint64_t seed, uint64_t first, int n, uint32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t ctr = first + (uint64_t)i;
  U4 c = {(uint32_t)ctr, (uint32_t)(ctr >> 32), 0u, 0u};
  const U4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  out[4 * i + 0] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

inline dim3 grid_for(int n, int tpb) { return dim3((n + tpb - 1) / tpb); }

lps_states proposal_states(const lps_sampler* sm) {
  lps_states s;
  s.n_states = sm->C;
  s.params = sm->pp;
  s.knot_off = sm->off;
  s.knot_x = sm->px;
  s.knot_y = sm->py;
  s.knot_cnt = sm->pcnt;
  s.n_knots = (int64_t)sm->C * sm->NS * sm->KC;
  return s;
}

lps_states current_states(const lps_sampler* sm) {
  lps_states s;
  s.n_states = sm->C;
  s.params = sm->cp;
  s.knot_off = sm->off;
  s.knot_x = sm->cx;
  s.knot_y = sm->cy;
  s.knot_cnt = sm->ccnt;
  s.n_knots = (int64_t)sm->C * sm->NS * sm->KC;
  return s;
}

}  // namespace
}  // namespace lps

extern "C" {

lps_status lps_sampler_create(lps_ctx* ctx, const lps_sampler_desc* d, lps_sampler** out) {
  LPS_API_RANGE();
  if (!ctx || !d || !out || !d->betas) return LPS_E_NULL;
  *out = nullptr;
  if (d->n_walkers < 1 || d->n_temps < 1 || d->k_in_max < 0 || d->k_in_max + 2 > ctx->k_max) return LPS_E_SHAPE;
  const int C = d->n_walkers * d->n_temps;
  if (C > ctx->max_grad_states) return LPS_E_CAPACITY;
  if (ctx->n_spl < 1) return LPS_E_SHAPE;
  if (!(d->step > 0.0)) return LPS_E_SHAPE;
  for (int t = 0; t < d->n_temps; ++t)
    if (!(d->betas[t] >= 0.0 && d->betas[t] <= 1.0)) return LPS_E_SHAPE;
  if (hipSetDevice(ctx->device) != hipSuccess) return LPS_E_DEVICE;
  lps_sampler* sm = new lps_sampler;
  memset(sm, 0, sizeof(*sm));
  sm->ctx = ctx;
  sm->W = d->n_walkers;
  sm->T = d->n_temps;
  sm->C = C;
  sm->P = ctx->n_params;
  sm->NS = ctx->n_spl;
  sm->KC = d->k_in_max + 2;
  sm->seed = d->seed;
  sm->eps = d->step;
  sm->prec = d->precision;
  sm->fixed = d->fixed_params;
  sm->rj = d->rj_moves != 0;
  sm->stretch = d->stretch_moves != 0;
  sm->x_lo = ctx->x_first;
  sm->x_hi = ctx->x_last;
  const size_t P = sm->P, NS = sm->NS, KC = sm->KC;
  const size_t nk = (size_t)C * NS * KC;
  bool ok = true;
  auto al = [&](void** p, size_t bytes) { ok = ok && hipMalloc(p, bytes > 0 ? bytes : 16) == hipSuccess; };
  al((void**)&sm->cp, P * C * 8);
  al((void**)&sm->pp, P * C * 8);
  al((void**)&sm->off, (size_t)C * NS * 4);
  al((void**)&sm->ccnt, (size_t)C * NS * 4);
  al((void**)&sm->pcnt, (size_t)C * NS * 4);
  for (double** p : {&sm->cx, &sm->cy, &sm->px, &sm->py, &sm->cgx, &sm->cgy, &sm->pgx, &sm->pgy}) al((void**)p, nk * 8);
  al((void**)&sm->cl, (size_t)C * 8);
  al((void**)&sm->pl, (size_t)C * 8);
  al((void**)&sm->cst, (size_t)C * 4);
  al((void**)&sm->pst, (size_t)C * 4);
  al((void**)&sm->cgp, P * C * 8);
  al((void**)&sm->pgp, P * C * 8);
  al((void**)&sm->flag, (size_t)C * 4);
  al((void**)&sm->beta, (size_t)sm->T * 8);
  al((void**)&sm->scale, (size_t)sm->T * 8);
  al((void**)&sm->sweep, 8);
  al((void**)&sm->counters, (size_t)lps::kKinds * sm->T * 2 * 4);
  al((void**)&sm->zs, (size_t)C * 8);
  if (!ok) {
    lps_sampler_destroy(sm);
    return LPS_E_NOMEM;
  }
  std::vector<double> sc(sm->T);
  for (int t = 0; t < sm->T; ++t) {
    const double b = d->betas[t];
    sc[t] = d->temp_scales ? d->temp_scales[t] : (b > 1e-6 ? fmin(1.0 / sqrt(b), 1e3) : 1e3);
  }
  const unsigned long long zero = 0ull;
  ok = ok && hipMemcpy(sm->beta, d->betas, (size_t)sm->T * 8, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(sm->scale, sc.data(), (size_t)sm->T * 8, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(sm->sweep, &zero, 8, hipMemcpyHostToDevice) == hipSuccess;
  hipLaunchKernelGGL(lps::k_slot_offsets, lps::grid_for(C * sm->NS, 256), dim3(256), 0, nullptr, C * sm->NS, sm->KC,
                     sm->off);
  hipLaunchKernelGGL(lps::k_zero_u32, lps::grid_for(lps::kKinds * sm->T * 2, 64), dim3(64), 0, nullptr,
                     lps::kKinds * sm->T * 2, sm->counters);
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    lps_sampler_destroy(sm);
    return LPS_E_DEVICE;
  }
  *out = sm;
  return LPS_OK;
}

lps_status lps_sampler_destroy(lps_sampler* sm) {
  LPS_API_RANGE();
  if (!sm) return LPS_OK;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {sm->cp,  sm->pp,  sm->off, sm->ccnt, sm->pcnt, sm->cx,  sm->cy,   sm->px,    sm->py,
                  sm->cl,  sm->pl,  sm->cst, sm->pst,  sm->cgp,  sm->pgp, sm->cgx,  sm->cgy,   sm->pgx,
                  sm->pgy, sm->flag, sm->beta, sm->scale, sm->sweep, sm->counters, sm->zs};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete sm;
  return LPS_OK;
}

lps_status lps_sampler_set_state(lps_sampler* sm, const lps_states* init, uint64_t sweep_index, void* stream) {
  LPS_API_RANGE();
  if (!sm || !init || !init->params || !init->knot_off || !init->knot_x || !init->knot_y) return LPS_E_NULL;
  if (init->n_states != sm->C || init->knot_cnt || init->n_knots < 0) return LPS_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  int32_t* bad = (int32_t*)sm->flag;   // reused as a flag word before any sweep
  if (hipMemsetAsync(bad, 0, 4, s) != hipSuccess) return LPS_E_DEVICE;
  hipLaunchKernelGGL(lps::k_load, lps::grid_for(sm->C, 64), dim3(64), 0, s, *sm, init->params, init->knot_off,
                     init->n_knots, init->knot_x, init->knot_y, bad);
  int32_t hb = 0;
  if (hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return LPS_E_DEVICE;
  if (hb) return LPS_E_CAPACITY;
  const unsigned long long sw = sweep_index;
  if (hipMemcpy(sm->sweep, &sw, 8, hipMemcpyHostToDevice) != hipSuccess) return LPS_E_DEVICE;
  lps_states cur = lps::current_states(sm);
  if (lps::launch_grad(sm->ctx, &cur, sm->prec, sm->cl, sm->cgp, sm->cgx, sm->cgy, sm->cst, s) != hipSuccess)
    return LPS_E_DEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? LPS_OK : LPS_E_DEVICE;
}

lps_status lps_sampler_sweep(lps_sampler* sm, int32_t n_sweeps, void* stream) {
  LPS_API_RANGE();
  if (!sm) return LPS_E_NULL;
  if (n_sweeps < 0) return LPS_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  const dim3 g = lps::grid_for(sm->C, lps::kWavesPerBlock), b(lps::kWave * lps::kWavesPerBlock);
  lps_states pro = lps::proposal_states(sm);
  for (int i = 0; i < n_sweeps; ++i) {
    hipLaunchKernelGGL(lps::k_mala_propose, g, b, 0, s, *sm);
    if (lps_status r = lps::device_status(
            lps::launch_grad(sm->ctx, &pro, sm->prec, sm->pl, sm->pgp, sm->pgx, sm->pgy, sm->pst, s)))
      return r;
    hipLaunchKernelGGL(lps::k_mala_accept, g, b, 0, s, *sm);
    if (sm->rj) {
      hipLaunchKernelGGL(lps::k_rj_propose, g, b, 0, s, *sm);
      if (lps_status r = lps::device_status(
              lps::launch_grad(sm->ctx, &pro, sm->prec, sm->pl, sm->pgp, sm->pgx, sm->pgy, sm->pst, s)))
        return r;
      hipLaunchKernelGGL(lps::k_rj_accept, g, b, 0, s, *sm);
    }
    if (sm->stretch && sm->W >= 2) {
      for (int half = 0; half < 2; ++half) {
        hipLaunchKernelGGL(lps::k_stretch_propose, g, b, 0, s, *sm, half);
        if (lps_status r = lps::device_status(
                lps::launch_grad(sm->ctx, &pro, sm->prec, sm->pl, sm->pgp, sm->pgx, sm->pgy, sm->pst, s)))
          return r;
        hipLaunchKernelGGL(lps::k_stretch_accept, g, b, 0, s, *sm, half);
      }
    }
    hipLaunchKernelGGL(lps::k_swap, lps::grid_for(sm->W * (sm->T / 2 + 1), lps::kWavesPerBlock), b, 0, s, *sm);
    hipLaunchKernelGGL(lps::k_advance, dim3(1), dim3(64), 0, s, sm->sweep);
  }
  return lps::device_status(hipGetLastError());
}

lps_status lps_sampler_get_state(lps_sampler* sm, double* params, int32_t* knot_off, int32_t* knot_cnt,
                                 double* knot_x, double* knot_y, double* logL, uint64_t* sweep_index, void* stream) {
  LPS_API_RANGE();
  if (!sm) return LPS_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  const size_t C = sm->C, P = sm->P, NS = sm->NS, KC = sm->KC;
  bool ok = true;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (dst) ok = ok && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess;
  };
  cp(params, sm->cp, P * C * 8);
  cp(knot_off, sm->off, C * NS * 4);
  cp(knot_cnt, sm->ccnt, C * NS * 4);
  cp(knot_x, sm->cx, C * NS * KC * 8);
  cp(knot_y, sm->cy, C * NS * KC * 8);
  cp(logL, sm->cl, C * 8);
  if (sweep_index) {
    unsigned long long sw = 0;
    ok = ok && hipMemcpyAsync(&sw, sm->sweep, 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
    *sweep_index = sw;
  }
  return ok ? LPS_OK : LPS_E_DEVICE;
}

lps_status lps_sampler_counters(lps_sampler* sm, uint32_t* counters, void* stream) {
  LPS_API_RANGE();
  if (!sm || !counters) return LPS_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(counters, sm->counters, (size_t)lps::kKinds * sm->T * 2 * 4, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LPS_E_DEVICE;
  return LPS_OK;
}

lps_status lps_philox4x32_10(uint64_t seed, uint64_t first_counter, int32_t n, uint32_t* out, void* stream) {
  LPS_API_RANGE();
  if (!out && n > 0) return LPS_E_NULL;
  if (n < 0) return LPS_E_SHAPE;
  if (n == 0) return LPS_OK;
  hipLaunchKernelGGL(lps::k_philox_fill, lps::grid_for(n, 256), dim3(256), 0, (hipStream_t)stream, seed,
                     first_counter, n, out);
  return lps::device_status(hipGetLastError());
}

}  // extern "C"
