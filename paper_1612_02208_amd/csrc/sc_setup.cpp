// Host helper of the Schur-complement smoother set-up: the largest real part
// of the eigenvalues of a small upper Hessenberg matrix (the Ritz values of
// the Arnoldi estimate of the Chebyshev interval).
//
// Shifted QR iteration on the active unreduced block: with the shift mu (the
// eigenvalue of the trailing 2 x 2 block nearer its last diagonal entry, or
// that entry when the pair is complex), H - mu I = Q R by Givens rotations
// and H <- R Q + mu I.  Negligible subdiagonal entries split the matrix; a
// trailing 1 x 1 block gives a real eigenvalue and a trailing 2 x 2 block its
// two eigenvalues from the quadratic formula (real parts of a complex pair).
#include <cmath>
#include <vector>

#include "sc_smoother.hpp"

namespace ibmg {

namespace {

void eig2(double a, double b, double c, double d, double* r1, double* r2) {
  const double tr = 0.5 * (a + d);
  const double disc = 0.25 * (a - d) * (a - d) + b * c;
  if (disc >= 0.0) {
    const double s = std::sqrt(disc);
    *r1 = tr + s;
    *r2 = tr - s;
  } else {
    *r1 = *r2 = tr;
  }
}

}  // namespace

double hessenberg_max_real_eig(std::vector<double> H, int n) {
  auto A = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
  std::vector<double> ev;
  int hi = n - 1;
  int iters = 0;
  const double eps = 1e-15;
  while (hi >= 0) {
    if (hi == 0) {
      ev.push_back(A(0, 0));
      break;
    }
    int lo = hi;
    while (lo > 0 && std::fabs(A(lo, lo - 1)) > eps * (std::fabs(A(lo - 1, lo - 1)) + std::fabs(A(lo, lo)))) --lo;
    if (lo == hi) {
      ev.push_back(A(hi, hi));
      --hi;
      iters = 0;
      continue;
    }
    if (lo == hi - 1) {
      double r1, r2;
      eig2(A(hi - 1, hi - 1), A(hi - 1, hi), A(hi, hi - 1), A(hi, hi), &r1, &r2);
      ev.push_back(r1);
      ev.push_back(r2);
      hi -= 2;
      iters = 0;
      continue;
    }
    if (++iters > 2000) {  // no convergence: report the diagonal of the block
      for (int i = lo; i <= hi; ++i) ev.push_back(A(i, i));
      hi = lo - 1;
      iters = 0;
      continue;
    }
    double r1, r2;
    eig2(A(hi - 1, hi - 1), A(hi - 1, hi), A(hi, hi - 1), A(hi, hi), &r1, &r2);
    double mu = std::fabs(r1 - A(hi, hi)) < std::fabs(r2 - A(hi, hi)) ? r1 : r2;
    if (iters % 11 == 10) mu += 0.75 * std::fabs(A(hi, hi - 1));  // occasional perturbed shift
    for (int i = lo; i <= hi; ++i) A(i, i) -= mu;
    std::vector<double> cs(hi - lo), sn(hi - lo);
    for (int k = lo; k < hi; ++k) {
      const double a = A(k, k), b = A(k + 1, k);
      const double r = std::hypot(a, b);
      const double c = r != 0.0 ? a / r : 1.0, s = r != 0.0 ? b / r : 0.0;
      cs[k - lo] = c;
      sn[k - lo] = s;
      for (int j = k; j < n; ++j) {
        const double x = A(k, j), y = A(k + 1, j);
        A(k, j) = c * x + s * y;
        A(k + 1, j) = -s * x + c * y;
      }
    }
    for (int k = lo; k < hi; ++k) {
      const double c = cs[k - lo], s = sn[k - lo];
      const int top = std::min(k + 2, hi);
      for (int i = 0; i <= top; ++i) {
        const double x = A(i, k), y = A(i, k + 1);
        A(i, k) = c * x + s * y;
        A(i, k + 1) = -s * x + c * y;
      }
    }
    for (int i = lo; i <= hi; ++i) A(i, i) += mu;
  }
  double best = -HUGE_VAL;
  for (double v : ev) best = std::max(best, v);
  return best;
}

}  // namespace ibmg
