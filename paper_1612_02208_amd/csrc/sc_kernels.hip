// Schur-complement smoother kernels (Sec. 3.3.2, Eq. approx-fact-Stokes-IB):
// multicolour Gauss-Seidel on A_IB (stencil + Galerkin IB rows) and on the
// approximate Schur complement -M^ = -D diag(A_IB)^{-1} G, the
// velocity-only A_IB product, G and D, and the vector combinations of the
// Chebyshev iterations.
//
// Gauss-Seidel rows of one colour are mutually uncoupled, so a colour is one
// parallel update.  The two large colours (the red/black classes of the
// stencil away from the structure) run as full-grid launches; the many small
// colours of the IB band run in sequence inside one work-group, separated by
// work-group barriers (all waves of a work-group share one CU, so global
// writes are visible to the whole group after the barrier).
#include "sc_smoother.hpp"

namespace ibmg {

static inline int cdiv(size_t a, int b) { return (int)((a + b - 1) / b); }

// (A_IB x)_r for a velocity row r = comp * N^2 + j * N + i (x = [u | v]);
// the IB rows' columns index [u | v], so coupled components need nothing
// extra.
template <typename T>
__device__ __forceinline__ T aib_row(const T* __restrict__ x, int r, int N, const StokesCoef<T>& c,
                                     const CsrT<T>& tu, const CsrT<T>& tv) {
  const int NN = N * N;
  const int comp = r >= NN ? 1 : 0;
  const int q = r - comp * NN;
  const int i = q % N, j = q / N;
  const T* f = x + (size_t)comp * NN;
  const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
  const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
  const T xc = f[q];
  T a = c.alpha * xc - c.beta * (f[j * N + im] + f[j * N + ip] + f[jm * N + i] + f[jp * N + i] - T(4) * xc);
  const CsrT<T>& t = comp ? tv : tu;
  for (int k = t.ptr[q]; k < t.ptr[q + 1]; ++k) a += t.val[k] * x[t.col[k]];
  return a;
}

// (-M^ p)_ij = (1/h^2) sum over the 4 faces of (p_ij - p_nb) / diag(A_IB)_face
template <typename T>
__device__ __forceinline__ T mhat_row(const T* __restrict__ p, int q, int N, T ih2,
                                      const T* __restrict__ dinv) {
  const int NN = N * N;
  const int i = q % N, j = q / N;
  const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
  const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
  const T pc = p[q];
  const T a = dinv[q] * (pc - p[j * N + im]) + dinv[j * N + ip] * (pc - p[j * N + ip]) +
              dinv[NN + q] * (pc - p[jm * N + i]) + dinv[NN + jp * N + i] * (pc - p[jp * N + i]);
  return ih2 * a;
}

// x_r += (b_r - (A x)_r) / diag_r for the rows of one colour
template <typename T, bool MHAT>
__global__ void k_gs_colour(T* x, const T* __restrict__ b, const int* __restrict__ rows, int count, int N,
                            StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, const T* __restrict__ diag,
                            const T* __restrict__ dinv, T ih2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int r = rows[t];
  const T ax = MHAT ? mhat_row<T>(x, r, N, ih2, dinv) : aib_row<T>(x, r, N, c, tu, tv);
  x[r] += (b[r] - ax) / diag[r];
}

// colours [c_first, c_last] in order (step +1 or -1) inside one work-group
// (pressure rows: one thread per row)
template <typename T>
__global__ void __launch_bounds__(1024) k_gs_band_p(T* x, const T* __restrict__ b, const int* __restrict__ cptr,
                                                    const int* __restrict__ rows, int c_first, int c_last, int step,
                                                    int N, const T* __restrict__ diag, const T* __restrict__ dinv,
                                                    T ih2) {
  for (int col = c_first;; col += step) {
    for (int t = cptr[col] + threadIdx.x; t < cptr[col + 1]; t += blockDim.x) {
      const int r = rows[t];
      x[r] += (b[r] - mhat_row<T>(x, r, N, ih2, dinv)) / diag[r];
    }
    __syncthreads();
    if (col == c_last) break;
  }
}

// Velocity rows whose IB part is long (near the structure): groups of G
// lanes share a row, each lane summing every G-th IB entry, the group's
// partial sums combined by shuffles in a fixed order.  Every lane of the
// wave calls this (live = false for lanes without a row).
constexpr int kGsGroup = 16;

template <typename T>
__device__ __forceinline__ void gs_row_group(T* x, const T* __restrict__ b, int r, bool live, int sub, int N,
                                             const StokesCoef<T>& c, const CsrT<T>& tu, const CsrT<T>& tv,
                                             const T* __restrict__ diag) {
  constexpr int G = kGsGroup;
  const int NN = N * N;
  const int comp = r >= NN ? 1 : 0;
  const int q = r - comp * NN;
  const T* f = x + (size_t)comp * NN;
  const CsrT<T>& tm = comp ? tv : tu;
  T a = 0;
  if (live)
    for (int k = tm.ptr[q] + sub; k < tm.ptr[q + 1]; k += G) a += tm.val[k] * x[tm.col[k]];
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, G);
  if (live && sub == 0) {
    const int i = q % N, j = q / N;
    const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
    const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
    const T xc = f[q];
    const T ax = c.alpha * xc - c.beta * (f[j * N + im] + f[j * N + ip] + f[jm * N + i] + f[jp * N + i] -
                                          T(4) * xc) + a;
    x[r] += (b[r] - ax) / diag[r];
  }
}

// one colour over the grid, a lane group per row
template <typename T>
__global__ void k_gs_colour_g(T* x, const T* __restrict__ b, const int* __restrict__ rows, int count, int N,
                              StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, const T* __restrict__ diag) {
  const int g = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kGsGroup);
  const bool live = g < count;
  gs_row_group<T>(x, b, live ? rows[g] : 0, live, threadIdx.x % kGsGroup, N, c, tu, tv, diag);
}

// colours [c_first, c_last] in order inside one work-group, lane groups per row
template <typename T>
__global__ void __launch_bounds__(1024) k_gs_band(T* x, const T* __restrict__ b, const int* __restrict__ cptr,
                                                  const int* __restrict__ rows, int c_first, int c_last,
                                                  int step, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv,
                                                  const T* __restrict__ diag) {
  constexpr int G = kGsGroup;
  const int grp = threadIdx.x / G, sub = threadIdx.x % G;
  for (int col = c_first;; col += step) {
    const int r0 = cptr[col], r1 = cptr[col + 1];
    // uniform trip count across the work-group (shuffles inside)
    for (int base = r0; base < r1; base += blockDim.x / G) {
      const int t = base + grp;
      const bool live = t < r1;
      gs_row_group<T>(x, b, live ? rows[t] : 0, live, sub, N, c, tu, tv, diag);
    }
    __syncthreads();
    if (col == c_last) break;
  }
}

template <typename T>
void launch_gs_sweep(T* x, const T* b, const int* cptr_dev, const std::vector<int>& cptr, const int* rows,
                     int ncol, bool mhat, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, const T* diag,
                     const T* dinv, T ih2, int nbig, const std::vector<char>& long_rows, hipStream_t s) {
  // forward over colours then backward; colours >= nbig rows are full-grid
  // launches, with lane groups per row when they hold long IB rows
  auto big = [&](int col) {
    const int cnt = cptr[col + 1] - cptr[col];
    if (!cnt) return;
    if (!mhat && col < (int)long_rows.size() && long_rows[col]) {
      IBMG_KLAUNCH((k_gs_colour_g<T>), dim3(cdiv((size_t)cnt * kGsGroup, 256)), dim3(256), 0, s, x, b,
                         rows + cptr[col], cnt, N, c, tu, tv, diag);
    } else if (mhat)
      IBMG_KLAUNCH((k_gs_colour<T, true>), dim3(cdiv(cnt, 256)), dim3(256), 0, s, x, b, rows + cptr[col],
                         cnt, N, c, tu, tv, diag, dinv, ih2);
    else
      IBMG_KLAUNCH((k_gs_colour<T, false>), dim3(cdiv(cnt, 256)), dim3(256), 0, s, x, b, rows + cptr[col],
                         cnt, N, c, tu, tv, diag, dinv, ih2);
    IBMG_LAUNCH_CHECK();
  };
  auto band = [&](int first, int last, int step) {
    if (mhat)
      IBMG_KLAUNCH((k_gs_band_p<T>), dim3(1), dim3(1024), 0, s, x, b, cptr_dev, rows, first, last, step, N,
                         diag, dinv, ih2);
    else
      IBMG_KLAUNCH((k_gs_band<T>), dim3(1), dim3(1024), 0, s, x, b, cptr_dev, rows, first, last, step, N, c,
                         tu, tv, diag);
    IBMG_LAUNCH_CHECK();
  };
  // a colour with at least nbig rows gets its own full-grid launch; runs of
  // smaller colours go through one work-group in sequence
  auto is_big = [&](int col) { return cptr[col + 1] - cptr[col] >= nbig; };
  for (int col = 0; col < ncol;) {
    if (is_big(col)) {
      big(col);
      ++col;
      continue;
    }
    int last = col;
    while (last + 1 < ncol && !is_big(last + 1)) ++last;
    band(col, last, 1);
    col = last + 1;
  }
  for (int col = ncol - 1; col >= 0;) {
    if (is_big(col)) {
      big(col);
      --col;
      continue;
    }
    int first = col;
    while (first - 1 >= 0 && !is_big(first - 1)) --first;
    band(col, first, -1);
    col = first - 1;
  }
}

// y = A_IB x (velocity only), IB term from the explicit Galerkin rows
template <typename T>
__global__ void k_aib_apply(const T* __restrict__ x, T* __restrict__ y, int N, StokesCoef<T> c, CsrT<T> tu,
                            CsrT<T> tv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * N * N) return;
  y[r] = aib_row<T>(x, r, N, c, tu, tv);
}

// faces = G p  ((p_ij - p_{i-1,j}) / h, (p_ij - p_{i,j-1}) / h)
template <typename T>
__global__ void k_grad(const T* __restrict__ p, T* __restrict__ f, int N, T gi) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * N) return;
  const int i = q % N, j = q / N;
  const int im = i == 0 ? N - 1 : i - 1, jm = j == 0 ? N - 1 : j - 1;
  f[q] = gi * (p[q] - p[j * N + im]);
  f[N * N + q] = gi * (p[q] - p[jm * N + i]);
}

// cells = a (D u) + b y   (D u = (u_{i+1} - u_i + v_{j+1} - v_j) / h); out may be y
template <typename T>
__global__ void k_div_comb(const T* __restrict__ u, const T* y, T* out, int N, T gi, T a, T b) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * N) return;
  const int i = q % N, j = q / N;
  const int ip = i == N - 1 ? 0 : i + 1, jp = j == N - 1 ? 0 : j + 1;
  const int NN = N * N;
  const T d = gi * (u[j * N + ip] - u[q] + u[NN + jp * N + i] - u[NN + q]);
  out[q] = a * d + (y ? b * y[q] : T(0));
}

// out = a x + b y  (y may be null)
template <typename T>
__global__ void k_axpby(size_t n, T a, const T* x, T b, const T* y, T* out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = a * x[i] + (y ? b * y[i] : T(0));
}

// Chebyshev start: d = theta_inv s, x = d, and (rc != null) rc = r
template <typename T>
__global__ void k_cheb_init(size_t n, T theta_inv, const T* __restrict__ sv, T* __restrict__ d, T* __restrict__ x,
                            const T* __restrict__ r, T* __restrict__ rc) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const T di = theta_inv * sv[i];
    d[i] = di;
    x[i] = di;
    if (rc) rc[i] = r[i];
  }
}

// Chebyshev step: d = c1 d + c2 s, x += d
template <typename T>
__global__ void k_cheb_step(size_t n, T c1, T c2, const T* __restrict__ sv, T* __restrict__ d, T* __restrict__ x) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const T di = c1 * d[i] + c2 * sv[i];
    d[i] = di;
    x[i] = x[i] + di;
  }
}

// y -= A_IB x (velocity only)
template <typename T>
__global__ void k_aib_sub(const T* __restrict__ x, T* __restrict__ y, int N, StokesCoef<T> c, CsrT<T> tu,
                          CsrT<T> tv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * N * N) return;
  y[r] = y[r] - aib_row<T>(x, r, N, c, tu, tv);
}

// x = frac(k g) - 1/2, g = (sqrt 5 - 1) / 2 (deterministic Arnoldi start vector)
template <typename T>
__global__ void k_weyl(T* x, size_t n) {
  const double g = 0.5 * (sqrt(5.0) - 1.0);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = (double)i * g;
    x[i] = (T)(v - floor(v) - 0.5);
  }
}

template <typename T>
void launch_aib_apply(const T* x, T* y, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, hipStream_t s) {
  IBMG_KLAUNCH((k_aib_apply<T>), dim3(cdiv(2 * (size_t)N * N, 256)), dim3(256), 0, s, x, y, N, c, tu, tv);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_grad(const T* p, T* f, int N, T gi, hipStream_t s) {
  IBMG_KLAUNCH((k_grad<T>), dim3(cdiv((size_t)N * N, 256)), dim3(256), 0, s, p, f, N, gi);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_div_comb(const T* u, const T* y, T* out, int N, T gi, T a, T b, hipStream_t s) {
  IBMG_KLAUNCH((k_div_comb<T>), dim3(cdiv((size_t)N * N, 256)), dim3(256), 0, s, u, y, out, N, gi, a, b);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_axpby(size_t n, T a, const T* x, T b, const T* y, T* out, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_axpby<T>), dim3(g), dim3(256), 0, s, n, a, x, b, y, out);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_cheb_init(size_t n, T theta_inv, const T* sv, T* d, T* x, const T* r, T* rc, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_cheb_init<T>), dim3(g), dim3(256), 0, s, n, theta_inv, sv, d, x, r, rc);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_cheb_step(size_t n, T c1, T c2, const T* sv, T* d, T* x, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_cheb_step<T>), dim3(g), dim3(256), 0, s, n, c1, c2, sv, d, x);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_aib_sub(const T* x, T* y, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, hipStream_t s) {
  IBMG_KLAUNCH((k_aib_sub<T>), dim3(cdiv(2 * (size_t)N * N, 256)), dim3(256), 0, s, x, y, N, c, tu, tv);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_weyl(T* x, size_t n, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_weyl<T>), dim3(g), dim3(256), 0, s, x, n);
  IBMG_LAUNCH_CHECK();
}

#define IBMG_INST_SC(T)                                                                                      \
  template void launch_gs_sweep<T>(T*, const T*, const int*, const std::vector<int>&, const int*, int, bool,  \
                                   int, StokesCoef<T>, CsrT<T>, CsrT<T>, const T*, const T*, T, int,          \
                                   const std::vector<char>&, hipStream_t);                                   \
  template void launch_aib_apply<T>(const T*, T*, int, StokesCoef<T>, CsrT<T>, CsrT<T>, hipStream_t);        \
  template void launch_grad<T>(const T*, T*, int, T, hipStream_t);                                           \
  template void launch_div_comb<T>(const T*, const T*, T*, int, T, T, T, hipStream_t);                       \
  template void launch_axpby<T>(size_t, T, const T*, T, const T*, T*, hipStream_t);                          \
  template void launch_weyl<T>(T*, size_t, hipStream_t);                                                     \
  template void launch_cheb_init<T>(size_t, T, const T*, T*, T*, const T*, T*, hipStream_t);                  \
  template void launch_cheb_step<T>(size_t, T, T, const T*, T*, T*, hipStream_t);                             \
  template void launch_aib_sub<T>(const T*, T*, int, StokesCoef<T>, CsrT<T>, CsrT<T>, hipStream_t);

IBMG_INST_SC(double)
IBMG_INST_SC(float)


// A_IB diagonal on faces (alpha + 4 beta + IB diagonal), its inverse, and the
// diagonal of -M^ on cells: (1/h^2) sum of the four face inverses.
template <typename T>
__global__ void k_sc_face_diag(int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, T* diag, T* dinv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int NN = N * N;
  if (r >= 2 * NN) return;
  const int comp = r >= NN ? 1 : 0, q = r - comp * NN;
  const CsrT<T>& t = comp ? tv : tu;
  T d = c.alpha + T(4) * c.beta;
  for (int k = t.ptr[q]; k < t.ptr[q + 1]; ++k)
    if (t.col[k] == r) d += t.val[k];
  diag[r] = d;
  dinv[r] = T(1) / d;
}

template <typename T>
__global__ void k_sc_cell_diag(int N, const T* __restrict__ dinv, T ih2, T* mdiag) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int NN = N * N;
  if (q >= NN) return;
  const int i = q % N, j = q / N;
  const int ip = i == N - 1 ? 0 : i + 1, jp = j == N - 1 ? 0 : j + 1;
  mdiag[q] = ih2 * (dinv[q] + dinv[j * N + ip] + dinv[NN + q] + dinv[NN + jp * N + i]);
}

template <typename T>
void launch_sc_diag(int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, T ih2, T* diag, T* dinv, T* mdiag,
                    hipStream_t s) {
  IBMG_KLAUNCH((k_sc_face_diag<T>), dim3(cdiv(2 * (size_t)N * N, 256)), dim3(256), 0, s, N, c, tu, tv,
                     diag, dinv);
  IBMG_LAUNCH_CHECK();
  IBMG_KLAUNCH((k_sc_cell_diag<T>), dim3(cdiv((size_t)N * N, 256)), dim3(256), 0, s, N, dinv, ih2, mdiag);
  IBMG_LAUNCH_CHECK();
}

// x -= (sum of the partial sums of x) / n
template <typename T>
__global__ void __launch_bounds__(256) k_sub_mean(T* x, size_t n, const double* __restrict__ partial, int nblk) {
  __shared__ double red[4];
  __shared__ double tot;
  double a[1] = {0.0};
  for (int b = threadIdx.x; b < nblk; b += 256) a[0] += partial[b];
  block_sums256<1>(a, 1, red, &tot, threadIdx.x);
  const double mean = tot / (double)n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = (T)((double)x[i] - mean);
}

template <typename T>
void launch_sub_mean(T* x, size_t n, const double* partial, int nblk, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 1024) g = 1024;
  IBMG_KLAUNCH((k_sub_mean<T>), dim3(g), dim3(256), 0, s, x, n, partial, nblk);
  IBMG_LAUNCH_CHECK();
}

template void launch_sc_diag<double>(int, StokesCoef<double>, CsrT<double>, CsrT<double>, double, double*,
                                     double*, double*, hipStream_t);
template void launch_sc_diag<float>(int, StokesCoef<float>, CsrT<float>, CsrT<float>, float, float*, float*,
                                    float*, hipStream_t);
template void launch_sub_mean<double>(double*, size_t, const double*, int, hipStream_t);
template void launch_sub_mean<float>(float*, size_t, const double*, int, hipStream_t);

}  // namespace ibmg
