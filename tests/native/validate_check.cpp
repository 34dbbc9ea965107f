// Host-side check of the per-state validation rules (built with address and
// undefined-behaviour sanitizers by tests/test_validate_host.py).
//
// Every state below is malformed in one way: offsets before the knot arrays,
// past their end, negative or inverted counts, a single knot, too many knots,
// non-finite values, unsorted or non-covering knots, bad amplitudes.  The
// knot arrays are allocated at exactly n_knots entries, so any read outside
// them is reported by the sanitizer; the program prints the status word of
// each state, one per line, for the test to compare with the expected bits.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lps_validate.hpp"

int main() {
  const int n_spl = 2, k_max = 8, n_params = 4;
  const double x_first = -4.0, x_last = -1.5;
  struct Case {
    std::vector<int> off;   // packed CSR offsets of this state's splines (n_spl + 1 entries, relative)
    std::vector<double> kx, ky;
    double a_oms, a_tm;
    int64_t n_knots_delta;  // n_knots = kx.size() + delta (negative: arrays shorter than the offsets claim)
  };
  std::vector<Case> cases = {
      {{0, 4, 6}, {-4.0, -3.0, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, 0},   // valid
      {{0, 4, 6}, {-4.0, -3.0, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, -1},  // past the end
      {{0, 4, 6}, {-4.0, -3.0, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, -6},  // no knots at all
      {{-2, 4, 6}, {-4.0, -3.0, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, 0},  // before the start
      {{0, 4, 3}, {-4.0, -3.0, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, 0},   // negative count
      {{0, 1, 3}, {-4.0, -4.0, -1.5}, {0, 0, 0}, 1e-11, 3e-15, 0},                               // one knot
      {{0, 9, 11}, {-4, -3.9, -3.8, -3.7, -3.6, -3.5, -3.4, -3.3, -1.5, -4, -1.5},
       {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, 0},                                     // above k_max
      {{0, 4, 6}, {-4.0, NAN, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, 0},    // non-finite
      {{0, 4, 6}, {-4.0, -2.0, -3.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, 0},   // unsorted
      {{0, 4, 6}, {-3.9, -3.0, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, 1e-11, 3e-15, 0},   // not covering
      {{0, 4, 6}, {-4.0, -3.0, -2.0, -1.5, -4.0, -1.5}, {0, 0, 0, 0, 0, 0}, -1e-11, 3e-15, 0},  // amplitude
      {{0, 0, 2}, {-4.0, -1.5}, {0, INFINITY}, 1e-11, 3e-15, 0},                                 // disabled + non-finite y
  };
  for (const Case& c : cases) {
    const int64_t n_knots = (int64_t)c.kx.size() + c.n_knots_delta;
    // exactly n_knots entries (at least one allocation byte so the pointer is valid)
    double* kx = (double*)std::malloc(sizeof(double) * (size_t)(n_knots > 0 ? n_knots : 0) + 1);
    double* ky = (double*)std::malloc(sizeof(double) * (size_t)(n_knots > 0 ? n_knots : 0) + 1);
    for (int64_t i = 0; i < n_knots && i < (int64_t)c.kx.size(); ++i) {
      kx[i] = c.kx[i];
      ky[i] = c.ky[i];
    }
    double params[n_params] = {c.a_oms, c.a_tm, -12.0, 0.0};
    const uint32_t st = lps::validate_state(0, 1, n_spl, k_max, n_params, params, c.off.data(), nullptr, n_knots, kx,
                                            ky, x_first, x_last);
    std::printf("%u\n", st);
    std::free(kx);
    std::free(ky);
  }
  return 0;
}
