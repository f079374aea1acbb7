// Symmetric tridiagonal eigen-solver pieces (host and device).
//
// T has diagonal d[0..n) and off-diagonal e[0..n-1) (real).  Eigenvalues are
// found by bisection on Sturm counts; eigenvectors by the twisted
// factorisation T - lambda I = L+ D+ L+^T = U- D- U-^T, which gives an
// eigenvector of an accurate eigenvalue in O(n) without pivoting.  Written
// without HIP types so that the same code is compiled for the device and for
// a host-side unit test.
#pragma once

#include <cmath>

#ifndef PISCO_HD
#if defined(__HIPCC__) || defined(__HIP__)
#define PISCO_HD __host__ __device__
#else
#define PISCO_HD
#endif
#endif

namespace pisco {
namespace tri {

// Division used by the recurrences below: IEEE a / b by default; a caller
// may pass a policy with its own (a reciprocal refined by Newton's method).
struct ExactDiv {
  PISCO_HD static double div(double a, double b) { return a / b; }
};

// Number of eigenvalues of T smaller than x (Sturm count of the LDL^T
// pivots).  e2[i] = e[i]^2; pivmin guards zero pivots.
template <class Div = ExactDiv>
PISCO_HD inline int negcount(const double* d, const double* e2, int n, double x,
                             double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - Div::div(e2[i - 1], q);
    if (std::fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Gershgorin interval containing the spectrum.
PISCO_HD inline void gershgorin(const double* d, const double* e, int n, double* lo,
                                double* hi) {
  double a = d[0], b = d[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    a = std::fmin(a, d[i] - r);
    b = std::fmax(b, d[i] + r);
  }
  const double w = std::fmax(std::fabs(a), std::fabs(b));
  *lo = a - 4e-16 * w - 1e-300;
  *hi = b + 4e-16 * w + 1e-300;
}

// j-th smallest eigenvalue (0-based) by bisection in [lo, hi] to a width of
// about 4 eps max(|lo|,|hi|) + abstol.
template <class Div = ExactDiv>
PISCO_HD inline double bisect(const double* d, const double* e2, int n, int j, double lo,
                              double hi, double pivmin, double abstol) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double w = hi - lo;
    if (w <= 4.4e-16 * std::fmax(std::fabs(lo), std::fabs(hi)) + abstol || mid == lo ||
        mid == hi)
      break;
    if (negcount<Div>(d, e2, n, mid, pivmin) > j)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Eigenvector z (length n, unit 2-norm) of T for the eigenvalue lambda by the
// twisted factorisation.  Lp, Um are n-length scratch arrays.
template <class Div = ExactDiv>
PISCO_HD inline void twisted_vector(const double* d, const double* e, int n, double lambda,
                                    double pivmin, double* Lp, double* Um, double* z) {
  if (n == 1) {
    z[0] = 1.0;
    return;
  }
  // top-down: D+(i), L+(i) = e_i / D+(i)
  double dp = d[0] - lambda;
  if (std::fabs(dp) < pivmin) dp = -pivmin;
  // store D+ in z temporarily, L+ in Lp
  z[0] = dp;
  for (int i = 0; i + 1 < n; ++i) {
    Lp[i] = Div::div(e[i], dp);
    dp = d[i + 1] - lambda - Lp[i] * e[i];
    if (std::fabs(dp) < pivmin) dp = -pivmin;
    z[i + 1] = dp;
  }
  // bottom-up: D-(i), U-(i) = e_{i-1} / D-(i); twist gamma_i = D+ + D- - (d_i - lambda)
  double dm = d[n - 1] - lambda;
  if (std::fabs(dm) < pivmin) dm = -pivmin;
  int r = n - 1;
  double best = std::fabs(z[n - 1]);  // gamma_{n-1} = D+(n-1)
  for (int i = n - 1; i > 0; --i) {
    Um[i] = Div::div(e[i - 1], dm);
    const double dnext = d[i - 1] - lambda - Um[i] * e[i - 1];
    dm = std::fabs(dnext) < pivmin ? -pivmin : dnext;
    const double gamma = z[i - 1] + dm - (d[i - 1] - lambda);
    if (std::fabs(gamma) < best) {
      best = std::fabs(gamma);
      r = i - 1;
    }
  }
  // z_r = 1, recurrences outward
  for (int i = 0; i < n; ++i) z[i] = 0.0;
  z[r] = 1.0;
  for (int i = r - 1; i >= 0; --i) z[i] = -Lp[i] * z[i + 1];
  for (int i = r + 1; i < n; ++i) z[i] = -Um[i] * z[i - 1];
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += z[i] * z[i];
  s = 1.0 / std::sqrt(s);
  for (int i = 0; i < n; ++i) z[i] *= s;
}

// Gaussian elimination with partial pivoting of T - sigma I.  U has the
// diagonal u0 and the super-diagonals u1, u2; lm holds the multipliers and
// sw[k] = 1 where rows k and k+1 were exchanged.  Pivots smaller than `tiny`
// in magnitude are replaced by +-tiny (T - sigma I is singular to working
// precision at an eigenvalue, which is what inverse iteration wants).
PISCO_HD inline void lu_factor(const double* d, const double* e, int n, double sigma,
                               double tiny, double* u0, double* u1, double* u2, double* lm,
                               int* sw) {
  double a = d[0] - sigma;           // diagonal of the current pivot row
  double c = n > 1 ? e[0] : 0.0;     // its super-diagonal
  for (int k = 0; k + 1 < n; ++k) {
    const double sub = e[k];
    const double dn = d[k + 1] - sigma;
    const double en = k + 2 < n ? e[k + 1] : 0.0;
    if (std::fabs(a) >= std::fabs(sub)) {
      if (std::fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
      const double l = sub / a;
      u0[k] = a;
      u1[k] = c;
      u2[k] = 0.0;
      lm[k] = l;
      sw[k] = 0;
      a = dn - l * c;
      c = en;
    } else {
      const double l = a / sub;
      u0[k] = sub;
      u1[k] = dn;
      u2[k] = en;
      lm[k] = l;
      sw[k] = 1;
      a = c - l * dn;
      c = -l * en;
    }
  }
  if (std::fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
  u0[n - 1] = a;
}

// y <- (T - sigma I)^{-1} y up to a positive scale factor (the vector is
// rescaled when it grows past 1e150; inverse iteration normalises anyway).
PISCO_HD inline void lu_solve(int n, const double* u0, const double* u1, const double* u2,
                              const double* lm, const int* sw, double* y) {
  for (int k = 0; k + 1 < n; ++k) {
    if (sw[k]) {
      const double tmp = y[k];
      y[k] = y[k + 1];
      y[k + 1] = tmp;
    }
    y[k + 1] -= lm[k] * y[k];
  }
  for (int k = n - 1; k >= 0; --k) {
    double v = y[k];
    if (k + 1 < n) v -= u1[k] * y[k + 1];
    if (k + 2 < n) v -= u2[k] * y[k + 2];
    v /= u0[k];
    y[k] = v;
    if (std::fabs(v) > 1e150) {
      for (int i = 0; i < n; ++i) y[i] *= 1e-150;
    }
  }
}

// Deterministic start vector entry in (-1, 1) for inverse iteration: a
// 64-bit mix (the splitmix64 finaliser) of the vector and row indices.
PISCO_HD inline double start_value(int vec, int row) {
  unsigned long long x = (static_cast<unsigned long long>(vec) << 32) ^
                         static_cast<unsigned long long>(row) ^ 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return static_cast<double>(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace tri
}  // namespace pisco
