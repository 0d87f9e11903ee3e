// Host linear algebra for the entanglement-entropy callback: eigenvalues of a
// small Hermitian matrix (the reduced density matrix, at most 1024 x 1024).
//
// Householder reduction to a real symmetric tridiagonal matrix (Golub & Van
// Loan, Matrix Computations, Sec. 8.3.1, in its complex Hermitian form), then
// each eigenvalue by bisection on the Sturm sequence count of the
// tridiagonal matrix (Golub & Van Loan, Sec. 8.4.1).  Eigenvalues only; the
// error is a few units of roundoff times the matrix norm.
#include "linalg.h"

#include <algorithm>
#include <cmath>

namespace qs {

namespace {

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x: the
// negative pivots of the LDL^T factorisation of T - x I.
int sturm_below(const std::vector<double>& d, const std::vector<double>& e2, double x) {
  const int n = (int)d.size();
  int count = 0;
  double q = d[0] - x;
  for (int i = 0;; ++i) {
    if (q < 0) ++count;
    if (i + 1 == n) break;
    if (q == 0.0) q = 1e-300;
    q = d[i + 1] - x - e2[i] / q;
  }
  return count;
}

}  // namespace

std::vector<double> hermitian_eigenvalues(int n, std::vector<std::complex<double>> A) {
  using cd = std::complex<double>;
  std::vector<double> d(n, 0.0), e(n > 1 ? n - 1 : 0, 0.0);
  auto at = [&](int i, int j) -> cd& { return A[size_t(i) * n + j]; };
  std::vector<cd> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    // reflect x = A[k+1.., k] onto alpha e_1 with |alpha| = |x|, arg(alpha) = arg(-x_0)
    double xn2 = 0.0;
    for (int i = k + 1; i < n; ++i) xn2 += std::norm(at(i, k));
    const double xn = std::sqrt(xn2);
    d[k] = at(k, k).real();
    if (xn == 0.0) {
      e[k] = 0.0;
      continue;
    }
    const cd x0 = at(k + 1, k);
    const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
    const cd alpha = -ph * xn;
    double vn2 = 0.0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = at(i, k);
      if (i == k + 1) v[i] -= alpha;
      vn2 += std::norm(v[i]);
    }
    const double tau = 2.0 / vn2;
    // trailing block B <- H B H with H = I - tau v v^H:  p = tau B v,
    // K = (tau / 2) v^H p (real), w = p - K v, B -= v w^H + w v^H
    cd K(0.0, 0.0);
    for (int i = k + 1; i < n; ++i) {
      cd s(0.0, 0.0);
      for (int j = k + 1; j < n; ++j) s += at(i, j) * v[j];
      p[i] = tau * s;
      K += std::conj(v[i]) * p[i];
    }
    K *= 0.5 * tau;
    for (int i = k + 1; i < n; ++i) w[i] = p[i] - K.real() * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) at(i, j) -= v[i] * std::conj(w[j]) + w[i] * std::conj(v[j]);
    e[k] = xn;  // |alpha|: a diagonal unitary similarity makes the off-diagonal real
  }
  if (n >= 2) {
    d[n - 2] = at(n - 2, n - 2).real();
    e[n - 2] = std::abs(at(n - 1, n - 2));
  }
  if (n >= 1) d[n - 1] = at(n - 1, n - 1).real();

  // bisection on the Sturm count within the Gershgorin interval
  std::vector<double> e2(e.size());
  for (size_t i = 0; i < e.size(); ++i) e2[i] = e[i] * e[i];
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? e[i - 1] : 0.0) + (i + 1 < n ? e[i] : 0.0);
    lo = i ? std::min(lo, d[i] - r) : d[i] - r;
    hi = i ? std::max(hi, d[i] + r) : d[i] + r;
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  lo -= 1e-12 * scale + 1e-300;
  hi += 1e-12 * scale + 1e-300;
  std::vector<double> ev(n);
  for (int k = 0; k < n; ++k) {
    // the (k+1)-th smallest eigenvalue: the smallest x with sturm_below(x) > k
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 2e-16 * std::max(std::fabs(a), std::fabs(b)) + 1e-300; ++it) {
      const double m = 0.5 * (a + b);
      if (m <= a || m >= b) break;
      if (sturm_below(d, e2, m) > k) b = m;
      else a = m;
    }
    ev[k] = 0.5 * (a + b);
  }
  return ev;
}

double entropy_of_eigenvalues(const std::vector<double>& ev) {
  double s = 0.0;
  for (double l : ev)
    if (l > 1e-15) s -= l * std::log(l);
  return s;
}

}  // namespace qs

extern "C" {
// Host helpers of the entropy callback, exported for the host-side tests only
// (no device involvement): eigenvalues of an n x n Hermitian complex128 matrix
// (row-major, interleaved) into ev (ascending).
int qs_test_hermitian_eigenvalues(int n, const double* a, double* ev) {
  if (n < 1 || !a || !ev) return -1;
  std::vector<std::complex<double>> A(size_t(n) * n);
  for (size_t i = 0; i < A.size(); ++i) A[i] = {a[2 * i], a[2 * i + 1]};
  const std::vector<double> r = qs::hermitian_eigenvalues(n, std::move(A));
  for (int i = 0; i < n; ++i) ev[i] = r[i];
  return 0;
}
}
