// Host check of the Rayleigh-Ritz eigensolver's arithmetic: the
// tridiagonal routines of tridiag.hpp (shared with the device kernels) and
// the same reduction / cluster / back-transformation steps as heev.hip,
// written sequentially.  Prints one line per case; exits 1 if any residual
// or orthogonality bound is missed.
//   tridiag_check <b> <mode>   mode 0 graded spectrum, 1 exact cluster,
//                              2 zero matrix, 3 near cluster (gap 1e-9)
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <cmath>
#include <cfloat>
#include <random>
#include <algorithm>
#include "tridiag.hpp"
using cd = std::complex<double>;
using namespace pisco::tri;

static void hetrd(std::vector<cd>& A, int b, std::vector<cd>& refl, std::vector<cd>& tau,
                  std::vector<double>& d, std::vector<double>& e) {
  std::vector<cd> vs(b), x(b), w(b);
  for (int k = 0; k + 1 < b; ++k) {
    int m = b - k - 1;
    cd* col = &A[size_t(k) * b + k + 1];
    double s = 0; for (int i = 1; i < m; ++i) s += std::norm(col[i]);
    cd al = col[0]; cd tk = 0, scale = 0; double beta = al.real();
    if (s > 0 || al.imag() != 0) {
      double nrm = std::sqrt(std::norm(al) + s);
      beta = al.real() >= 0 ? -nrm : nrm;
      tk = cd((beta - al.real()) / beta, -al.imag() / beta);
      scale = 1.0 / (al - beta);
    }
    for (int i = 0; i < m; ++i) { vs[i] = i == 0 ? cd(1) : col[i] * scale; refl[size_t(k)*b + k+1+i] = vs[i]; }
    tau[k] = tk; e[k] = beta; d[k] = A[size_t(k)*b+k].real();
    cd* a22 = &A[size_t(k+1)*b + k+1];
    cd dot = 0;
    for (int i = 0; i < m; ++i) { cd acc = 0; for (int j = 0; j < m; ++j) acc += a22[size_t(j)*b+i]*vs[j]; x[i] = tk*acc; dot += std::conj(x[i])*vs[i]; }
    cd ap = -0.5 * tk * dot;
    for (int i = 0; i < m; ++i) w[i] = x[i] + ap * vs[i];
    for (int j = 0; j < m; ++j) for (int i = 0; i < m; ++i) a22[size_t(j)*b+i] -= vs[i]*std::conj(w[j]) + w[i]*std::conj(vs[j]);
  }
  d[b-1] = A[size_t(b-1)*b + b-1].real();
}

// Division by a reciprocal with the worst relative error of the hardware
// estimate (4.6e-8, measured over 2^20 values) refined by one Newton step,
// as the per-voxel Lanczos solver divides on the device.
struct NewtonDiv {
  static double div(double a, double b) {
    const double r0 = (1.0 / b) * (1.0 + 4.6e-8);
    const double e = std::fma(-b, r0, 1.0);
    return a * std::fma(r0, e, r0);
  }
};

int main(int argc, char** argv) {
  int b = argc > 1 ? atoi(argv[1]) : 96;
  int mode = argc > 2 ? atoi(argv[2]) : 0;
  std::mt19937_64 g(7);
  std::normal_distribution<double> N(0, 1);
  // A = V diag(l) V^H with graded spectrum / clusters
  std::vector<cd> V(size_t(b)*b);
  for (auto& v : V) v = cd(N(g), N(g));
  // Gram-Schmidt
  for (int j = 0; j < b; ++j) {
    for (int p = 0; p < 2; ++p) for (int q = 0; q < j; ++q) { cd s = 0; for (int i = 0; i < b; ++i) s += std::conj(V[q*b+i])*V[j*b+i]; for (int i = 0; i < b; ++i) V[j*b+i] -= s*V[q*b+i]; }
    double nn = 0; for (int i = 0; i < b; ++i) nn += std::norm(V[j*b+i]); nn = std::sqrt(nn); for (int i = 0; i < b; ++i) V[j*b+i] /= nn;
  }
  std::vector<double> l(b);
  for (int k = 0; k < b; ++k) {
    if (mode == 0) l[k] = 1e6 * std::pow(10.0, -5.0 * k / b);
    else if (mode == 1) l[k] = k < b/2 ? 1e6 * std::pow(10.0, -3.0*k/b) : 1.0;  // exact cluster
    else if (mode == 2) l[k] = 0.0;
    else l[k] = k < b/2 ? 1e6 * std::pow(10.0, -3.0*k/b) : 1.0 + 1e-9 * k;
  }
  std::vector<cd> A(size_t(b)*b, 0);
  for (int i = 0; i < b; ++i) for (int j = 0; j < b; ++j) { cd s = 0; for (int k = 0; k < b; ++k) s += V[k*b+i]*l[k]*std::conj(V[k*b+j]); A[size_t(j)*b+i] = s; }
  std::vector<cd> A0 = A;
  std::vector<cd> refl(size_t(b)*b), tau(b);
  std::vector<double> d(b), e(b, 0.0);
  hetrd(A, b, refl, tau, d, e);
  // eigenvalues by bisection (plain)
  std::vector<double> e2(b, 0.0); double emax2 = 0; for (int i = 0; i + 1 < b; ++i) { e2[i] = e[i]*e[i]; emax2 = std::max(emax2, e2[i]); }
  double pivmin = DBL_MIN * std::max(1.0, emax2);
  double lo, hi; gershgorin(d.data(), e.data(), b, &lo, &hi);
  std::vector<double> lam(b);
  for (int j = 0; j < b; ++j) lam[j] = bisect(d.data(), e2.data(), b, j, lo, hi, pivmin, 0.0);
  double nrm = std::max(std::fabs(lam[0]), std::fabs(lam[b-1]));
  // the same eigenvalues and single-eigenvalue vectors with the refined
  // reciprocal in place of the division
  {
    std::vector<double> Lq(b), Uq(b), zq(b);
    for (int j = 0; j < b; ++j) {
      const double l2 = bisect<NewtonDiv>(d.data(), e2.data(), b, j, lo, hi, pivmin, 0.0);
      if (!(std::fabs(l2 - lam[j]) <= 1e-13 * std::max(nrm, 1e-300) + 1e-300)) {
        printf("refined-reciprocal bisection differs at j=%d: %.3e\n", j, l2 - lam[j]);
        return 1;
      }
      const bool single = (j == 0 || lam[j] - lam[j - 1] > 1e-6 * nrm) &&
                          (j + 1 == b || lam[j + 1] - lam[j] > 1e-6 * nrm);
      if (!single || nrm == 0.0) continue;
      twisted_vector<NewtonDiv>(d.data(), e.data(), b, lam[j], pivmin, Lq.data(), Uq.data(),
                                zq.data());
      double r = 0;
      for (int i = 0; i < b; ++i) {
        double v = (d[i] - lam[j]) * zq[i];
        if (i > 0) v += e[i - 1] * zq[i - 1];
        if (i + 1 < b) v += e[i] * zq[i + 1];
        r = std::max(r, std::fabs(v));
      }
      if (!(r <= 1e3 * b * 2.2e-16 * nrm + pivmin)) {
        printf("refined-reciprocal twisted vector residual %.3e at j=%d\n", r, j);
        return 1;
      }
    }
  }
  std::vector<double> Z(size_t(b)*b), Lp(b), Um(b), z(b);
  double ctol = 1e-12 * nrm;
  int nclus = 0;
  std::vector<double> u0(b), u1(b), u2(b), lm(b); std::vector<int> sw(b);
  const double tiny = std::max(2.2e-16 * nrm, pivmin);
  for (int j = 0; j < b; ++j) {
    int cs = j; while (cs > 0 && lam[cs]-lam[cs-1] <= ctol) --cs;
    int ce = j; while (ce+1 < b && lam[ce+1]-lam[ce] <= ctol) ++ce;
    if (cs != j) continue;
    bool inv = ce > cs;
    if (!inv) {
      twisted_vector(d.data(), e.data(), b, lam[j], pivmin, Lp.data(), Um.data(), z.data());
      double r = 0;
      for (int i = 0; i < b; ++i) { double v = (d[i]-lam[j])*z[i]; if (i>0) v += e[i-1]*z[i-1]; if (i+1<b) v += e[i]*z[i+1]; r = std::max(r, std::fabs(v)); }
      if (!(r <= 1e3 * b * 2.2e-16 * nrm + pivmin)) inv = true;
      else for (int i = 0; i < b; ++i) Z[size_t(j)*b+i] = z[i];
    }
    if (inv) {
      ++nclus;
      for (int q = cs; q <= ce; ++q) {
        for (int i = 0; i < b; ++i) z[i] = start_value(q, i);
        lu_factor(d.data(), e.data(), b, lam[q], tiny, u0.data(), u1.data(), u2.data(), lm.data(), sw.data());
        for (int it = 0; it < 3; ++it) {
          lu_solve(b, u0.data(), u1.data(), u2.data(), lm.data(), sw.data(), z.data());
          for (int pass = 0; pass < 2; ++pass)
            for (int p = cs; p < q; ++p) { double s = 0; for (int i = 0; i < b; ++i) s += Z[size_t(p)*b+i]*z[i]; for (int i = 0; i < b; ++i) z[i] -= s*Z[size_t(p)*b+i]; }
          double mx = 0; for (int i = 0; i < b; ++i) mx = std::max(mx, std::fabs(z[i]));
          for (int i = 0; i < b; ++i) z[i] /= mx;
          double nn = 0; for (int i = 0; i < b; ++i) nn += z[i]*z[i]; nn = 1/std::sqrt(nn);
          for (int i = 0; i < b; ++i) z[i] *= nn;
        }
        for (int i = 0; i < b; ++i) Z[size_t(q)*b+i] = z[i];
      }
    }
  }
  // back-transform
  std::vector<cd> U(size_t(b)*b);
  for (int j = 0; j < b; ++j) {
    std::vector<cd> u(b); for (int i = 0; i < b; ++i) u[i] = Z[size_t(j)*b+i];
    for (int k = b-2; k >= 0; --k) { cd s = 0; for (int r = k+1; r < b; ++r) s += std::conj(refl[size_t(k)*b+r])*u[r]; for (int r = k+1; r < b; ++r) u[r] -= tau[k]*s*refl[size_t(k)*b+r]; }
    for (int i = 0; i < b; ++i) U[size_t(j)*b+i] = u[i];
  }
  double res = 0, orth = 0, everr = 0;
  std::vector<double> ls = l; std::sort(ls.begin(), ls.end());
  for (int j = 0; j < b; ++j) {
    everr = std::max(everr, std::fabs(lam[j]-ls[j]) / std::max(nrm, 1e-300));
    for (int i = 0; i < b; ++i) { cd s = 0; for (int k = 0; k < b; ++k) s += A0[size_t(k)*b+i]*U[size_t(j)*b+k]; res = std::max(res, std::abs(s - lam[j]*U[size_t(j)*b+i]) / std::max(nrm,1e-300)); }
    for (int q = 0; q < b; ++q) { cd s = 0; for (int i = 0; i < b; ++i) s += std::conj(U[size_t(q)*b+i])*U[size_t(j)*b+i]; orth = std::max(orth, std::abs(s - (q==j ? 1.0 : 0.0))); }
  }
  printf("b=%d mode=%d clusters=%d everr=%.2e res=%.2e orth=%.2e\n", b, mode, nclus, everr, res, orth);
  const bool ok = (mode == 2 ? true : (everr <= 1e-13 && res <= 1e-12)) && orth <= 1e-12;
  return ok ? 0 : 1;
}
