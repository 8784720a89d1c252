// Dense pieces of the V-cycle: Schwarz box matrices L_k = R_k L R_k^T
// (Alg. 2) assembled from the level stencils and the Galerkin IB rows, their
// batched inversion, the restricted additive Schwarz application, and the
// coarsest-level direct solve (Alg. 1, coarse-grid equation).
//
// Box local ordering (m = b + 2o cells per side): x-faces jj*(m+1) + ii for
// ii in [0, m], jj in [0, m); y-faces m(m+1) + jj*m + ii for ii in [0, m),
// jj in [0, m]; cells 2m(m+1) + jj*m + ii.  Owned unknowns (b x b cells with
// their left x-face and bottom y-face) are ordered x-faces, y-faces, cells,
// each (oj, oi) row-major.
#include "internal.hpp"

namespace ibmg {

static inline int cdiv(size_t a, int b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ int pmod(int a, int N) {
  a %= N;
  return a < 0 ? a + N : a;
}

struct CsrView {
  const int* ptr;
  const int* col;
  const double* val;
};

__global__ void __launch_bounds__(256) k_patch_assemble(const int* __restrict__ patch_ids, BoxGeom g,
                                                        StokesCoef<double> c, CsrView tu, CsrView tv,
                                                        double* __restrict__ mats) {
  const int pid = patch_ids[blockIdx.x];
  const int N = g.N, m = g.m, n = g.nloc;
  const int x0 = (pid % g.npd) * g.b - g.o;
  const int y0 = (pid / g.npd) * g.b - g.o;
  double* A = mats + (size_t)blockIdx.x * n * n;
  for (size_t k = threadIdx.x; k < (size_t)n * n; k += blockDim.x) A[k] = 0.0;
  __syncthreads();
  const int nu = m * (m + 1);
  const int p0 = 2 * nu;
  const double dg = c.alpha + 4.0 * c.beta;
  for (int row = threadIdx.x; row < n; row += blockDim.x) {
    double* Ar = A + (size_t)row * n;
    if (row < nu) {  // x-face (ii, jj)
      const int ii = row % (m + 1), jj = row / (m + 1);
      Ar[row] += dg;
      if (ii >= 1) Ar[row - 1] -= c.beta;
      if (ii <= m - 1) Ar[row + 1] -= c.beta;
      if (jj >= 1) Ar[row - (m + 1)] -= c.beta;
      if (jj <= m - 2) Ar[row + (m + 1)] -= c.beta;
      if (ii <= m - 1) Ar[p0 + jj * m + ii] += c.gi;
      if (ii >= 1) Ar[p0 + jj * m + ii - 1] -= c.gi;
      const int r = pmod(y0 + jj, N) * N + pmod(x0 + ii, N);
      for (int k = tu.ptr[r]; k < tu.ptr[r + 1]; ++k) {
        const int col = tu.col[k];
        const int li = pmod(col % N - x0, N), lj = pmod(col / N - y0, N);
        if (li <= m && lj <= m - 1) Ar[lj * (m + 1) + li] += tu.val[k];
      }
    } else if (row < p0) {  // y-face (ii, jj)
      const int q = row - nu;
      const int ii = q % m, jj = q / m;
      Ar[row] += dg;
      if (ii >= 1) Ar[row - 1] -= c.beta;
      if (ii <= m - 2) Ar[row + 1] -= c.beta;
      if (jj >= 1) Ar[row - m] -= c.beta;
      if (jj <= m - 1) Ar[row + m] -= c.beta;
      if (jj <= m - 1) Ar[p0 + jj * m + ii] += c.gi;
      if (jj >= 1) Ar[p0 + (jj - 1) * m + ii] -= c.gi;
      const int r = pmod(y0 + jj, N) * N + pmod(x0 + ii, N);
      for (int k = tv.ptr[r]; k < tv.ptr[r + 1]; ++k) {
        const int col = tv.col[k];
        const int li = pmod(col % N - x0, N), lj = pmod(col / N - y0, N);
        if (li <= m - 1 && lj <= m) Ar[nu + lj * m + li] += tv.val[k];
      }
    } else {  // cell (ii, jj): -(D u)
      const int q = row - p0;
      const int ii = q % m, jj = q / m;
      Ar[jj * (m + 1) + ii + 1] -= c.gi;
      Ar[jj * (m + 1) + ii] += c.gi;
      Ar[nu + (jj + 1) * m + ii] -= c.gi;
      Ar[nu + jj * m + ii] += c.gi;
    }
  }
}

void launch_patch_assemble(const int* patch_ids, int count, BoxGeom g, StokesCoef<double> c,
                           const int* tptr_u, const int* tcol_u, const double* tval_u,
                           const int* tptr_v, const int* tcol_v, const double* tval_v, double* mats,
                           hipStream_t s) {
  if (!count) return;
  CsrView tu{tptr_u, tcol_u, tval_u}, tv{tptr_v, tcol_v, tval_v};
  hipLaunchKernelGGL(k_patch_assemble, dim3(count), dim3(256), 0, s, patch_ids, g, c, tu, tv, mats);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched in-place Gauss-Jordan inversion without pivoting, blocked by NB
// columns.  The box matrices are ordered velocities first: the velocity block
// R_k A_IB R_k^T is symmetric positive definite (a principal submatrix of
// rho/dt - mu Lap + IB with the periodic constants cut off), and the pressure
// pivots come from the negative definite Schur complement -G^T A^{-1} G, so
// no pivot vanishes.  One work-group per matrix.
// Step K: D = A_KK -> D^{-1};  A_Kj <- D^{-1} A_Kj;  A_ij <- A_ij - A_iK A_Kj;
//         A_iK <- -A_iK D^{-1};  A_KK <- D^{-1}.
// ---------------------------------------------------------------------------
constexpr int GJ_NB = 16;

__global__ void __launch_bounds__(512) k_gj_invert(double* __restrict__ mats, int n,
                                                   double* __restrict__ colk_all) {
  __shared__ double Dm[GJ_NB][GJ_NB + 1];
  double* A = mats + (size_t)blockIdx.x * n * n;
  double* colK = colk_all + (size_t)blockIdx.x * n * GJ_NB;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int kb = 0; kb < n; kb += GJ_NB) {
    const int w = n - kb < GJ_NB ? n - kb : GJ_NB;
    // diagonal block into LDS and unblocked in-place inversion
    for (int t = tid; t < w * w; t += nt) Dm[t / w][t % w] = A[(size_t)(kb + t / w) * n + kb + t % w];
    __syncthreads();
    for (int k = 0; k < w; ++k) {
      const double piv = Dm[k][k];
      const double ip = 1.0 / piv;
      // other rows / columns use the old row k and column k
      double rk = 0.0, ck = 0.0;
      const int t = tid;
      const bool act = t < w * w;
      const int ti = act ? t / w : 0, tj = act ? t % w : 0;
      if (act) {
        rk = Dm[k][tj];
        ck = Dm[ti][k];
      }
      __syncthreads();
      if (act) {
        double val = Dm[ti][tj];
        if (ti == k && tj == k) val = ip;
        else if (ti == k) val = rk * ip;
        else if (tj == k) val = -ck * ip;
        else val = val - ck * rk * ip;
        Dm[ti][tj] = val;
      }
      __syncthreads();
    }
    // save the old block column A_iK
    for (size_t t = tid; t < (size_t)n * w; t += nt) {
      const int i = (int)(t / w), k = (int)(t % w);
      colK[(size_t)i * GJ_NB + k] = A[(size_t)i * n + kb + k];
    }
    __syncthreads();
    // row panel A_Kj <- D^{-1} A_Kj (j outside K), A_KK <- D^{-1}
    for (int j = tid; j < n; j += nt) {
      if (j >= kb && j < kb + w) {
        for (int k = 0; k < w; ++k) A[(size_t)(kb + k) * n + j] = Dm[k][j - kb];
      } else {
        double col[GJ_NB];
        for (int k = 0; k < w; ++k) col[k] = A[(size_t)(kb + k) * n + j];
        for (int k = 0; k < w; ++k) {
          double a = 0.0;
          for (int q = 0; q < w; ++q) a += Dm[k][q] * col[q];
          A[(size_t)(kb + k) * n + j] = a;
        }
      }
    }
    __syncthreads();
    // trailing update of every row outside K
    for (size_t t = tid; t < (size_t)n * n; t += nt) {
      const int i = (int)(t / n), j = (int)(t % n);
      if (i >= kb && i < kb + w) continue;
      const double* ck = colK + (size_t)i * GJ_NB;
      double a;
      if (j >= kb && j < kb + w) {
        a = 0.0;
        for (int k = 0; k < w; ++k) a -= ck[k] * Dm[k][j - kb];
      } else {
        a = A[t];
        for (int k = 0; k < w; ++k) a -= ck[k] * A[(size_t)(kb + k) * n + j];
      }
      A[t] = a;
    }
    __syncthreads();
  }
}

void launch_gj_invert(double* mats, int n, int count, double* colk, hipStream_t s) {
  if (!count) return;
  hipLaunchKernelGGL(k_gj_invert, dim3(count), dim3(512), 0, s, mats, n, colk);
  IBMG_LAUNCH_CHECK();
}

__device__ __forceinline__ int own_local(int r, const BoxGeom& g) {
  const int bb = g.b * g.b;
  const int comp = r / bb, q = r % bb;
  const int oi = q % g.b + g.o, oj = q / g.b + g.o;
  const int m = g.m;
  if (comp == 0) return oj * (m + 1) + oi;
  if (comp == 1) return m * (m + 1) + oj * m + oi;
  return 2 * m * (m + 1) + oj * m + oi;
}

// out[(blk * nloc + j) * nown + r] = A^{-1}[own(r)][j]  (owned rows, column-major)
template <typename T>
__global__ void k_extract_owned(const double* __restrict__ mats, int count, BoxGeom g,
                                T* __restrict__ out) {
  const size_t per = (size_t)g.nloc * g.nown;
  const size_t tot = per * count;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const size_t blk = t / per;
    const size_t rem = t % per;
    const int j = (int)(rem / g.nown), r = (int)(rem % g.nown);
    const double* A = mats + blk * g.nloc * g.nloc;
    out[t] = (T)A[(size_t)own_local(r, g) * g.nloc + j];
  }
}

template <typename T>
void launch_extract_owned(const double* mats, int count, BoxGeom g, T* out, hipStream_t s) {
  if (!count) return;
  size_t tot = (size_t)g.nloc * g.nown * count;
  int grid = cdiv(tot, 256);
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL((k_extract_owned<T>), dim3(grid), dim3(256), 0, s, mats, count, g, out);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Restricted additive Schwarz (Alg. 2 from a zero guess):
//   z[G~_k] = (L_k^{-1} R_k r)[G~_k]  for every box k.
// One work-group per box gathers R_k r into LDS and multiplies by the stored
// owned rows of L_k^{-1}; the owned sets partition the unknowns, so every z
// entry is written by exactly one work-group.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_ras_apply(const T* __restrict__ r, T* __restrict__ z,
                                                   BoxGeom g, const T* __restrict__ inv,
                                                   const int* __restrict__ blk_of_patch) {
  extern __shared__ char smem_raw[];
  T* x = reinterpret_cast<T*>(smem_raw);
  const int pid = blockIdx.x;
  const int N = g.N, m = g.m;
  const int pi = pid % g.npd, pj = pid / g.npd;
  const int x0 = pi * g.b - g.o, y0 = pj * g.b - g.o;
  const size_t nn = (size_t)N * N;
  const int nu = m * (m + 1);
  for (int k = threadIdx.x; k < g.nloc; k += blockDim.x) {
    size_t gi;
    if (k < nu) {
      const int ii = k % (m + 1), jj = k / (m + 1);
      gi = (size_t)pmod(y0 + jj, N) * N + pmod(x0 + ii, N);
    } else if (k < 2 * nu) {
      const int q = k - nu, ii = q % m, jj = q / m;
      gi = nn + (size_t)pmod(y0 + jj, N) * N + pmod(x0 + ii, N);
    } else {
      const int q = k - 2 * nu, ii = q % m, jj = q / m;
      gi = 2 * nn + (size_t)pmod(y0 + jj, N) * N + pmod(x0 + ii, N);
    }
    x[k] = r[gi];
  }
  __syncthreads();
  const T* Mt = inv + (size_t)blk_of_patch[pid] * g.nloc * g.nown;
  const int bb = g.b * g.b;
  for (int row = threadIdx.x; row < g.nown; row += blockDim.x) {
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int j = 0;
    for (; j + 3 < g.nloc; j += 4) {
      a0 += Mt[(size_t)j * g.nown + row] * x[j];
      a1 += Mt[(size_t)(j + 1) * g.nown + row] * x[j + 1];
      a2 += Mt[(size_t)(j + 2) * g.nown + row] * x[j + 2];
      a3 += Mt[(size_t)(j + 3) * g.nown + row] * x[j + 3];
    }
    for (; j < g.nloc; ++j) a0 += Mt[(size_t)j * g.nown + row] * x[j];
    const int comp = row / bb, q = row % bb;
    const int gi = pi * g.b + q % g.b, gj = pj * g.b + q / g.b;
    z[comp * nn + (size_t)gj * N + gi] = (a0 + a1) + (a2 + a3);
  }
}

template <typename T>
void launch_ras_apply(const T* r, T* z, BoxGeom g, const T* inv, const int* blk_of_patch,
                      hipStream_t s) {
  const int nbox = g.npd * g.npd;
  int threads = ((g.nown + 63) / 64) * 64;
  if (threads > 256) threads = 256;
  hipLaunchKernelGGL((k_ras_apply<T>), dim3(nbox), dim3(threads), g.nloc * sizeof(T), s, r, z, g, inv,
                     blk_of_patch);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Coarsest level: bordered matrix [[L0, C], [C^T, 0]] (C = null vectors: the
// constant pressure, plus constant u and v when rho = 0), augmented by the
// identity and reduced by Gauss-Jordan with partial pivoting in one
// work-group.  aug is (nn) x (2 nn) row-major, nn = 3 N^2 + nb.
// ---------------------------------------------------------------------------
__global__ void k_coarse_assemble(int N, StokesCoef<double> c, CsrView tu, CsrView tv, int nb,
                                  double* __restrict__ aug) {
  const int n = 3 * N * N, nn = n + nb, ld = 2 * nn;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nn) return;
  double* Ar = aug + (size_t)row * ld;
  Ar[nn + row] = 1.0;
  const int NN = N * N;
  // block -> border column: rho = 0: u->0, v->1, p->2; else p->0
  auto border = [&](int blk) -> int {
    if (nb == 3) return n + blk;
    return blk == 2 ? n : -1;
  };
  if (row >= n) {
    const int cidx = row - n;
    const int blk = nb == 3 ? cidx : 2;
    for (int k = 0; k < NN; ++k) Ar[blk * NN + k] = 1.0;
    return;
  }
  const int blk = row / NN, q = row % NN;
  const int i = q % N, j = q / N;
  const int im = pmod(i - 1, N), ip = pmod(i + 1, N), jm = pmod(j - 1, N), jp = pmod(j + 1, N);
  const double dg = c.alpha + 4.0 * c.beta;
  if (blk == 0) {
    Ar[q] += dg;
    Ar[j * N + im] -= c.beta;
    Ar[j * N + ip] -= c.beta;
    Ar[jm * N + i] -= c.beta;
    Ar[jp * N + i] -= c.beta;
    Ar[2 * NN + j * N + i] += c.gi;
    Ar[2 * NN + j * N + im] -= c.gi;
    for (int k = tu.ptr[q]; k < tu.ptr[q + 1]; ++k) Ar[tu.col[k]] += tu.val[k];
  } else if (blk == 1) {
    Ar[NN + q] += dg;
    Ar[NN + j * N + im] -= c.beta;
    Ar[NN + j * N + ip] -= c.beta;
    Ar[NN + jm * N + i] -= c.beta;
    Ar[NN + jp * N + i] -= c.beta;
    Ar[2 * NN + j * N + i] += c.gi;
    Ar[2 * NN + jm * N + i] -= c.gi;
    for (int k = tv.ptr[q]; k < tv.ptr[q + 1]; ++k) Ar[NN + tv.col[k]] += tv.val[k];
  } else {
    Ar[j * N + ip] -= c.gi;
    Ar[j * N + i] += c.gi;
    Ar[NN + jp * N + i] -= c.gi;
    Ar[NN + j * N + i] += c.gi;
  }
  const int bc = border(blk);
  if (bc >= 0) Ar[bc] += 1.0;
}

void launch_coarse_assemble(int N, StokesCoef<double> c, const int* tptr_u, const int* tcol_u,
                            const double* tval_u, const int* tptr_v, const int* tcol_v,
                            const double* tval_v, int nb, double* aug, hipStream_t s) {
  CsrView tu{tptr_u, tcol_u, tval_u}, tv{tptr_v, tcol_v, tval_v};
  const int nn = 3 * N * N + nb;
  hipLaunchKernelGGL(k_coarse_assemble, dim3(cdiv(nn, 64)), dim3(64), 0, s, N, c, tu, tv, nb, aug);
  IBMG_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(1024) k_coarse_invert(double* __restrict__ aug, int nn) {
  __shared__ double vmax[1024];
  __shared__ int imax[1024];
  __shared__ double fac[1024];
  const int ld = 2 * nn;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < nn; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < nn; i += nt) {
      const double a = fabs(aug[(size_t)i * ld + k]);
      if (a > best) { best = a; bi = i; }
    }
    vmax[tid] = best;
    imax[tid] = bi;
    __syncthreads();
    for (int sft = nt / 2; sft > 0; sft >>= 1) {
      if (tid < sft) {
        const double o = vmax[tid + sft];
        const int oi = imax[tid + sft];
        if (o > vmax[tid] || (o == vmax[tid] && oi < imax[tid])) { vmax[tid] = o; imax[tid] = oi; }
      }
      __syncthreads();
    }
    const int p = imax[0];
    if (p != k) {
      for (int j = tid; j < ld; j += nt) {
        const double t = aug[(size_t)k * ld + j];
        aug[(size_t)k * ld + j] = aug[(size_t)p * ld + j];
        aug[(size_t)p * ld + j] = t;
      }
    }
    __syncthreads();
    const double ip = 1.0 / aug[(size_t)k * ld + k];
    __syncthreads();
    for (int j = tid; j < ld; j += nt) aug[(size_t)k * ld + j] *= ip;
    for (int i = tid; i < nn; i += nt) fac[i] = aug[(size_t)i * ld + k];
    __syncthreads();
    for (size_t t = tid; t < (size_t)nn * ld; t += nt) {
      const int i = (int)(t / ld);
      if (i == k) continue;
      const int j = (int)(t % ld);
      aug[t] -= fac[i] * aug[(size_t)k * ld + j];
    }
    __syncthreads();
  }
}

void launch_coarse_invert(double* aug, int nn, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_invert, dim3(1), dim3(1024), 0, s, aug, nn);
  IBMG_LAUNCH_CHECK();
}

__global__ void k_coarse_extract(const double* __restrict__ aug, int nn, int n0, double* __restrict__ inv) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 * n0) return;
  const int i = t / n0, j = t % n0;
  inv[t] = aug[(size_t)i * 2 * nn + nn + j];
}

void launch_coarse_extract(const double* aug, int nn, int n0, double* inv, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_extract, dim3(cdiv((size_t)n0 * n0, 256)), dim3(256), 0, s, aug, nn, n0, inv);
  IBMG_LAUNCH_CHECK();
}

// z = inv r on the coarsest level, FP64 arithmetic whatever T is.
template <typename T>
__global__ void k_coarse_apply(const double* __restrict__ inv, int n0, const T* __restrict__ r,
                               T* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0) return;
  const double* row = inv + (size_t)i * n0;
  double a = 0.0;
  for (int j = 0; j < n0; ++j) a += row[j] * (double)r[j];
  z[i] = (T)a;
}

template <typename T>
void launch_coarse_apply(const double* inv, int n0, const T* r, T* z, hipStream_t s) {
  hipLaunchKernelGGL((k_coarse_apply<T>), dim3(cdiv(n0, 64)), dim3(64), 0, s, inv, n0, r, z);
  IBMG_LAUNCH_CHECK();
}

template void launch_extract_owned<double>(const double*, int, BoxGeom, double*, hipStream_t);
template void launch_extract_owned<float>(const double*, int, BoxGeom, float*, hipStream_t);
template void launch_ras_apply<double>(const double*, double*, BoxGeom, const double*, const int*,
                                       hipStream_t);
template void launch_ras_apply<float>(const float*, float*, BoxGeom, const float*, const int*,
                                      hipStream_t);
template void launch_coarse_apply<double>(const double*, int, const double*, double*, hipStream_t);
template void launch_coarse_apply<float>(const double*, int, const float*, float*, hipStream_t);

}  // namespace ibmg
