// Schur-complement smoother of one level (Sec. 3.3.2, Eq.
// approx-fact-Stokes-IB), host side:
//   y_u = A~^{-1} r_u
//   y_p = M~^{-1} (r_p + D y_u)
//   z_u = y_u - A~^{-1} G y_p,   z_p = y_p
// A~^{-1}: cheb_its first-kind Chebyshev iterations (Saad, Iterative Methods
// for Sparse Linear Systems, Alg. 12.1) from zero, preconditioned by one
// symmetric multicolour Gauss-Seidel sweep on A_IB.  M~^{-1}: the same
// iteration on the positive semidefinite -D A~^{-1} G with right-hand side
// -(r_p + D y_u), preconditioned by symmetric Gauss-Seidel on
// -M^ = -D diag(A_IB)^{-1} G; the pressure output has zero mean.  Chebyshev
// intervals are [0.1 lam, 1.1 lam], lam the largest Ritz value of ten
// Arnoldi steps (classical Gram-Schmidt twice) on the preconditioned operator
// from the start vector frac(k g) - 1/2, g = (sqrt 5 - 1)/2, with its
// null-space components removed.  Colours: greedy over rows in index order
// on the structural pattern (five-point stencil plus the IB rows), smallest
// colour unused by already coloured neighbours.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace ibmg {

// Gauss-Seidel colours with at least this many rows get a full-grid launch;
// runs of smaller colours are swept inside one work-group.
constexpr int kGsBigColour = 256;

template <typename T>
void launch_gs_sweep(T* x, const T* b, const int* cptr_dev, const std::vector<int>& cptr, const int* rows,
                     int ncol, bool mhat, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, const T* diag,
                     const T* dinv, T ih2, int nbig, const std::vector<char>& long_rows, hipStream_t s);

// a colour whose longest IB row exceeds this many entries is swept with
// lane groups per row
constexpr int kGsLongRow = 8;
template <typename T>
void launch_aib_apply(const T* x, T* y, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, hipStream_t s);
template <typename T>
void launch_grad(const T* p, T* f, int N, T gi, hipStream_t s);
template <typename T>
void launch_div_comb(const T* u, const T* y, T* out, int N, T gi, T a, T b, hipStream_t s);
template <typename T>
void launch_axpby(size_t n, T a, const T* x, T b, const T* y, T* out, hipStream_t s);
template <typename T>
void launch_weyl(T* x, size_t n, hipStream_t s);
template <typename T>
void launch_cheb_init(size_t n, T theta_inv, const T* sv, T* d, T* x, const T* r, T* rc, hipStream_t s);
template <typename T>
void launch_cheb_step(size_t n, T c1, T c2, const T* sv, T* d, T* x, hipStream_t s);
template <typename T>
void launch_aib_sub(const T* x, T* y, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, hipStream_t s);
template <typename T>
void launch_sc_diag(int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, T ih2, T* diag, T* dinv, T* mdiag,
                    hipStream_t s);
template <typename T>
void launch_sub_mean(T* x, size_t n, const double* partial, int nblk, hipStream_t s);

// Largest real part of the eigenvalues of the k x k upper Hessenberg matrix
// H (row-major), by the Francis double-shift QR iteration.
double hessenberg_max_real_eig(std::vector<double> H, int k);

// Greedy colouring, rows in index order; nbrs(r, out) lists the structural
// neighbours of row r.
template <typename F>
std::vector<int> greedy_colours(int n, F nbrs) {
  std::vector<int> col(n, -1), mark;
  std::vector<int> nb;
  for (int r = 0; r < n; ++r) {
    nb.clear();
    nbrs(r, nb);
    for (int q : nb)
      if (q != r && col[q] >= 0) {
        if ((int)mark.size() <= col[q]) mark.resize(col[q] + 1, -1);
        mark[col[q]] = r;
      }
    int c = 0;
    while (c < (int)mark.size() && mark[c] == r) ++c;
    col[r] = c;
  }
  return col;
}

struct ColourLists {
  std::vector<int> ptr, rows;  // rows grouped by colour, ascending within a colour
  std::vector<char> long_rows;  // per colour: holds an IB row longer than kGsLongRow
  DBuf<int> d_ptr, d_rows;
  int ncol = 0;
  void build(const std::vector<int>& col, hipStream_t s) {
    ncol = col.empty() ? 0 : *std::max_element(col.begin(), col.end()) + 1;
    ptr.assign(ncol + 1, 0);
    for (int c : col) ptr[c + 1]++;
    for (int c = 0; c < ncol; ++c) ptr[c + 1] += ptr[c];
    rows.assign(col.size(), 0);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int r = 0; r < (int)col.size(); ++r) rows[fill[col[r]]++] = r;
    d_ptr.upload(ptr, s);
    d_rows.upload(rows, s);
  }
};

template <typename T>
struct ScLevel {
  int N = 0, its = 2;
  bool rho_zero = false;
  StokesCoef<T> c{};
  CsrT<T> tu{}, tv{};
  T ih2 = 0;
  ColourLists colu, colp;
  DBuf<T> diag, dinv, mdiag;  // A_IB diagonal (and inverse) on faces, -M^ diagonal on cells
  // Chebyshev coefficients: x = d0 + d1 + ..., d0 = B^{-1} r / theta,
  // d_{k+1} = c1[k] d_k + c2[k] B^{-1} r_{k+1}
  double lamA = 0, lamM = 0;
  std::vector<T> a_c1, a_c2, m_c1, m_c2;
  T a_theta_inv = 0, m_theta_inv = 0;
  // work vectors (velocity: 2 N^2, cells: N^2)
  DBuf<T> yu, ga, gx, ad, ar, at, as, s, md, mr, mt, ms, ones;
  DBuf<double> part;

  static void cheb_coefs(double lam, int its, T* theta_inv, std::vector<T>& c1, std::vector<T>& c2) {
    const double lmin = 0.1 * lam, lmax = 1.1 * lam;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma;
    *theta_inv = (T)(1.0 / theta);
    c1.clear();
    c2.clear();
    for (int k = 0; k + 1 < its; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1.push_back((T)(rn * rho));
      c2.push_back((T)(2.0 * rn / delta));
      rho = rn;
    }
  }

  void sgs_a(const T* b, T* x, hipStream_t st) {
    const size_t n2 = 2 * (size_t)N * N;
    launch_axpby<T>(n2, T(0), b, T(0), nullptr, x, st);
    launch_gs_sweep<T>(x, b, colu.d_ptr.p, colu.ptr, colu.d_rows.p, colu.ncol, false, N, c, tu, tv, diag.p,
                       dinv.p, ih2, kGsBigColour, colu.long_rows, st);
  }
  void sgs_m(const T* b, T* x, hipStream_t st) {
    const size_t n1 = (size_t)N * N;
    launch_axpby<T>(n1, T(0), b, T(0), nullptr, x, st);
    launch_gs_sweep<T>(x, b, colp.d_ptr.p, colp.ptr, colp.d_rows.p, colp.ncol, true, N, c, tu, tv, mdiag.p,
                       dinv.p, ih2, kGsBigColour, colp.long_rows, st);
  }

  // x = A~^{-1} r (velocity vectors); residual r_k = r - A x kept in ar
  void a_tilde(const T* r, T* x, hipStream_t st) {
    const size_t n2 = 2 * (size_t)N * N;
    sgs_a(r, as.p, st);
    launch_cheb_init<T>(n2, a_theta_inv, as.p, ad.p, x, r, its > 1 ? ar.p : nullptr, st);
    for (int k = 0; k + 1 < its; ++k) {
      launch_aib_sub<T>(ad.p, ar.p, N, c, tu, tv, st);
      sgs_a(ar.p, as.p, st);
      launch_cheb_step<T>(n2, a_c1[k], a_c2[k], as.p, ad.p, x, st);
    }
  }

  // out = -D A~^{-1} G q (cells)
  void schur_op(const T* q, T* out, hipStream_t st) {
    launch_grad<T>(q, ga.p, N, c.gi, st);
    a_tilde(ga.p, gx.p, st);
    launch_div_comb<T>(gx.p, nullptr, out, N, c.gi, T(-1), T(0), st);
  }

  // y = M~^{-1} s: Chebyshev on -D A~^{-1} G with right-hand side -s;
  // residual kept in mr (mr - (-D A~^{-1} G d) = mr + D A~^{-1} G d)
  void m_tilde(const T* s_in, T* y, hipStream_t st) {
    const size_t n1 = (size_t)N * N;
    launch_axpby<T>(n1, T(-1), s_in, T(0), nullptr, mr.p, st);
    sgs_m(mr.p, ms.p, st);
    launch_cheb_init<T>(n1, m_theta_inv, ms.p, md.p, y, nullptr, nullptr, st);
    for (int k = 0; k + 1 < its; ++k) {
      launch_grad<T>(md.p, ga.p, N, c.gi, st);
      a_tilde(ga.p, gx.p, st);
      launch_div_comb<T>(gx.p, mr.p, mr.p, N, c.gi, T(1), T(1), st);
      sgs_m(mr.p, ms.p, st);
      launch_cheb_step<T>(n1, m_c1[k], m_c2[k], ms.p, md.p, y, st);
    }
    const int nblk = dots_blocks(n1, 256);
    launch_dots<T>(ones.p, 1, n1, y, n1, part.p, nblk, st);
    launch_sub_mean<T>(y, n1, part.p, nblk, st);
  }

  // z = L~^{-1} r on a level vector [u | v | p]
  void apply(const T* r, T* z, hipStream_t st) {
    const size_t n1 = (size_t)N * N, n2 = 2 * n1;
    a_tilde(r, yu.p, st);
    launch_div_comb<T>(yu.p, r + n2, s.p, N, c.gi, T(1), T(1), st);
    m_tilde(s.p, z + n2, st);
    launch_grad<T>(z + n2, ga.p, N, c.gi, st);
    a_tilde(ga.p, gx.p, st);
    launch_axpby<T>(n2, T(1), yu.p, T(-1), gx.p, z, st);
  }
};

}  // namespace ibmg
