// Exact minimiser of a 1-D convex piecewise quadratic over [lo, hi].
//
// The derivative is D(x) = A x + B + sum_r w_r * m_r(x + e_r) with m_r = min(0, .)
// for a row whose slack enters with a minus sign and max(0, .) for a plus sign:
// continuous, piecewise linear and increasing (A > 0).  The bracket [a, b] with
// D(a) < 0 <= D(b) is shrunk at every kink inside it -- no sorting, no dynamically
// indexed arrays, so everything stays in registers -- and the root is the zero of
// the one linear piece left, whose active rows are read at the bracket midpoint.
// Plain IEEE arithmetic (contraction off) in any translation unit.
#pragma once
#include "ucac_dev.hpp"

namespace ucac {

template <int NR>
struct Pwl {
  double A, B;
  double w[NR], e[NR];
  bool neg[NR];

  __device__ inline double D(double x) const {
#pragma clang fp contract(off)
    double d = A * x + B;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double m = x + e[r];
      d += w[r] * (neg[r] ? fmin(m, 0.0) : fmax(m, 0.0));
    }
    return d;
  }

  __device__ inline double argmin(double lo, double hi) const {
#pragma clang fp contract(off)
    if (D(lo) >= 0.0) return lo;
    if (D(hi) <= 0.0) return hi;
    double a = lo, b = hi;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double k = -e[r];
      if (k > a && k < b) {
        if (D(k) < 0.0) a = k; else b = k;
      }
    }
    const double m = 0.5 * (a + b);
    double slope = A, cst = B;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const bool act = neg[r] ? (m + e[r] < 0.0) : (m + e[r] > 0.0);
      if (act) { slope += w[r]; cst += w[r] * e[r]; }
    }
    return clampd(-cst / slope, a, b);
  }
};

}  // namespace ucac
