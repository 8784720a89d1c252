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

// Add an IB entry of a box row: col indexes the level's [u | v] vector; the
// entry lands on the box's x-face or y-face unknown when that face lies in
// the enlarged box.
__device__ __forceinline__ void add_ib_entry(double* Ar, int col, double v, int N, int x0, int y0, int m) {
  const int NN = N * N;
  const int comp = col >= NN ? 1 : 0;
  const int f = col - comp * NN;
  const int li = pmod(f % N - x0, N), lj = pmod(f / N - y0, N);
  if (comp == 0) {
    if (li <= m && lj <= m - 1) Ar[lj * (m + 1) + li] += v;
  } else {
    if (li <= m - 1 && lj <= m) Ar[m * (m + 1) + lj * m + li] += v;
  }
}

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
      for (int k = tu.ptr[r]; k < tu.ptr[r + 1]; ++k) add_ib_entry(Ar, tu.col[k], tu.val[k], N, x0, y0, m);
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
      for (int k = tv.ptr[r]; k < tv.ptr[r + 1]; ++k) add_ib_entry(Ar, tv.col[k], tv.val[k], N, x0, y0, m);
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
  IBMG_KLAUNCH(k_patch_assemble, dim3(count), dim3(256), 0, s, patch_ids, g, c, tu, tv, mats);
  IBMG_LAUNCH_CHECK();
}

// Operand layout of the 16x16x4 MFMA: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; its result register v holds D[row][l % 16] with
// row = 4 (l / 16) + v for FP32 and row = l / 16 + 4 v for FP64 (checked on
// gfx950 with a one-wave probe).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
};

// ---------------------------------------------------------------------------
// Batched in-place inversion of the symmetric box matrices by block sweeps
// (the symmetric form of Gauss-Jordan elimination, no pivoting), 128 columns
// per step.  The box matrices are ordered velocities first: the velocity
// block R_k A_IB R_k^T is symmetric positive definite (a principal submatrix
// of rho/dt - mu Lap + IB with the periodic constants cut off), and the
// pressure pivots come from the negative definite Schur complement
// -G^T A^{-1} G, so no pivot vanishes.  L_IB is symmetric (G = -D^T,
// S = J^*), so every swept matrix is too, and only the 64 x 64 tiles on or
// below the diagonal (tiles I >= J, diagonal tiles in full) are kept.
// Sweeping block K (columns kb .. kb+127, tiles K0 = kb/64 and K1 = K0 + 1)
// of a symmetric S with D = S_KK:
//   S_IJ <- S_IJ - S_IK D^{-1} S_KJ   (I, J outside K),
//   S_IK <- S_IK D^{-1},  S_KK <- -D^{-1};
// after every block S = -A^{-1}.  Step K, five launches over every matrix:
//   diag       (a work-group per matrix): D^{-1} in LDS (128 x 128, the
//              160 KB of gfx950), to dinv;
//   panel read (64-row tiles): C = S_:K from the kept tiles (a tile above
//              K0 or K1 from that tile row's tile, transposed) and C^T;
//   scale      (64-row tiles x two column halves): E = C D^{-1};
//   update     (kept 64 x 64 tiles outside K): S_IJ <- S_IJ - E_I C_J^T;
//   panel write: S_IK <- E_I below K, S_KI <- E_I^T above it, S_KK <- -D^{-1}.
// The last block may be narrower (w < 128 columns): D is padded with the
// identity, and the panel columns beyond w are zero, so they change nothing.
// The scale and update products are 64 x 64 tiles with a 128-long reduction
// on the FP64 matrix cores (16x16x4 MFMA, four waves of 2 x 2 tiles): twice
// the flops per pass over the kept tiles of 64-column steps.
constexpr int GJ_NB = kGjNb;   // 128
static_assert(GJ_NB == 128, "the sweep kernels are written for 128-column blocks of two 64-wide tiles");

// D^{-1} of the 128 x 128 pivot block by in-place Gauss-Jordan, one
// work-group of 1024 threads per matrix.  Thread t holds column t mod 128 of
// rows t / 128 + 8 q (q < 16) in registers; per pivot k only row k and
// column k pass through LDS (two buffers by pivot parity, so one barrier per
// pivot): the threads holding them publish them, and every thread updates
// its sixteen entries from its column's row-k value and its rows' column-k
// values (the latter the same for a whole wave, read as broadcasts).
__global__ void __launch_bounds__(1024) k_gj_diag(const double* __restrict__ mats, int n, int kb,
                                                  double* __restrict__ dinv_all) {
  __shared__ double rowk[2][GJ_NB];
  __shared__ double colk[2][GJ_NB];
  const double* A = mats + (size_t)blockIdx.x * n * n;
  double* Di = dinv_all + (size_t)blockIdx.x * GJ_NB * GJ_NB;
  const int tid = threadIdx.x;
  const int b = tid & 127, a0 = tid >> 7;   // column, first row (rows a0 + 8 q)
  const int w = n - kb < GJ_NB ? n - kb : GJ_NB;
  // the padding of a narrow last block is the identity, so the pivots stay
  // nonzero; the padded rows and columns never reach the matrix.  Above the
  // diagonal tiles only tile (K1, K0) is kept: D[a][b] with a in the first
  // half and b in the second is read as D[b][a].
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int a = a0 + 8 * q;
    double x = a == b ? 1.0 : 0.0;
    if (a < w && b < w) {
      const bool upper = (a >> 6) < (b >> 6);
      x = upper ? A[(size_t)(kb + b) * n + kb + a] : A[(size_t)(kb + a) * n + kb + b];
    }
    v[q] = x;
  }
  for (int k = 0; k < GJ_NB; ++k) {
    const int buf = k & 1;
    // publish row k (the thread holding row k of column b) and column k
    if ((k & 7) == a0) rowk[buf][b] = v[k >> 3];
    if (b == k) {
#pragma unroll
      for (int q = 0; q < 16; ++q) colk[buf][a0 + 8 * q] = v[q];
    }
    __syncthreads();
    // every LDS read is issued before any arithmetic, so a pivot costs one
    // round trip to LDS, not sixteen
    const double pk = rowk[buf][k];
    const double rk = rowk[buf][b];
    double ck[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) ck[q] = colk[buf][a0 + 8 * q];
    const double ip = 1.0 / pk;
    const double rip = rk * ip;
    // the pivot block's FP64 vector work bounds this kernel (one CU per
    // matrix): the common entries take one FMA, and only row k (held at
    // q = k / 8 by the threads with a0 = k mod 8) and column k (the threads
    // of column k) are set apart
    if (b != k) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = v[q] - ck[q] * rip;
      if ((k & 7) == a0) v[k >> 3] = rip;
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = -ck[q] * ip;
      if ((k & 7) == a0) v[k >> 3] = ip;
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) Di[(size_t)(a0 + 8 * q) * GJ_NB + b] = v[q];
}

struct GjTileSmem {
  double Xs[32][65];   // [reduction index of the chunk][row]
  double Ys[32][65];   // [reduction index of the chunk][column]
};

// acc = X Y for the wave's 32 x 32 quarter of a 64 x 64 tile: X is a
// row-major block with GJ_NB columns (rows beyond xrows read as zero), Y the
// rows 0 .. GJ_NB-1 of a row-major array with row stride ldy, columns
// J0 .. J0+63 (zero for rows >= yrows or columns >= ycols); the reduction runs
// in chunks of 32 through LDS, the next chunk's values loading into
// registers during the current chunk's MFMA steps.
__device__ __forceinline__ void gj_tile_product(GjTileSmem& sm, Mfma<double>::acc_t acc[2][2],
                                                const double* __restrict__ X, int xrows,
                                                const double* __restrict__ Y, size_t ldy, int yrows, int ycols,
                                                int J0) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 1, wc = wave >> 1, kq = lane >> 4, ln = lane & 15;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<double>::acc_t{0, 0, 0, 0};
  double xr[8], yr[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = tid + 256 * q;
      const int row = t >> 5, k = t & 31;
      xr[q] = row < xrows ? X[(size_t)row * GJ_NB + k0 + k] : 0.0;
      const int ky = t >> 6, c = t & 63;
      const int r = k0 + ky, j = J0 + c;
      yr[q] = (r < yrows && j < ycols) ? Y[(size_t)r * ldy + j] : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < GJ_NB; k0 += 32) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = tid + 256 * q;
      sm.Xs[t & 31][t >> 5] = xr[q];
      sm.Ys[t >> 6][t & 63] = yr[q];
    }
    __syncthreads();
    if (k0 + 32 < GJ_NB) load(k0 + 32);
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      const int kk = 4 * st + kq;
      const double a0 = sm.Xs[kk][32 * wr + ln], a1 = sm.Xs[kk][32 * wr + 16 + ln];
      const double b0 = sm.Ys[kk][32 * wc + ln], b1 = sm.Ys[kk][32 * wc + 16 + ln];
      acc[0][0] = Mfma<double>::mma(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<double>::mma(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<double>::mma(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<double>::mma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
}

// C = S[:, K] and C^T (n x 128 and 128 x n, zero beyond w) for one 64-row
// tile I, one 64-column half h at a time (tile Kh = K0 + h): I >= Kh holds
// S_I,Kh; above Kh, S_I,Kh = S_Kh,I^T is read from tile row Kh.  work holds
// C, C^T and E per matrix.
__global__ void __launch_bounds__(256) k_sw_panel_read(const double* __restrict__ mats, int n, int kb,
                                                       double* __restrict__ work) {
  __shared__ double Ts[64][65];   // [row of the tile][column of the half]
  const int I0 = blockIdx.x * 64, I = blockIdx.x;
  const double* A = mats + (size_t)blockIdx.y * n * n;
  double* C = work + (size_t)blockIdx.y * 3 * n * GJ_NB;
  double* Ct = C + (size_t)n * GJ_NB;
  const int w = n - kb < GJ_NB ? n - kb : GJ_NB;
  const int tid = threadIdx.x;
  for (int h = 0; h < 2; ++h) {
    const int kbh = kb + 64 * h, Kh = kbh / 64;
    const int wh = w - 64 * h;   // live columns of this half (<= 0: none)
    if (I >= Kh) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int t = tid + 256 * q, a = t >> 6, k = t & 63, i = I0 + a;
        Ts[a][k] = (i < n && k < wh) ? A[(size_t)i * n + kbh + k] : 0.0;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int t = tid + 256 * q, k = t >> 6, c = t & 63, i = I0 + c;
        Ts[c][k] = (k < wh && i < n) ? A[(size_t)(kbh + k) * n + i] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = tid + 256 * q, a = t >> 6, k = t & 63, i = I0 + a;
      if (i < n) C[(size_t)i * GJ_NB + 64 * h + k] = Ts[a][k];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = tid + 256 * q, k = t >> 6, a = t & 63, i = I0 + a;
      if (i < n) Ct[(size_t)(64 * h + k) * n + i] = Ts[a][k];
    }
    __syncthreads();
  }
}

// E_I (columns 64 h .. 64 h + 63) = C_I D^{-1} for one 64-row tile I outside K
__global__ void __launch_bounds__(256) k_sw_scale(const double* __restrict__ dinv_all, int n, int kb,
                                                  double* __restrict__ work) {
  const int I0 = blockIdx.x * 64, I = blockIdx.x, K0 = kb / 64, h = blockIdx.z;
  if (I == K0 || I == K0 + 1) return;   // E_K is not used
  __shared__ GjTileSmem sm;
  const double* C = work + (size_t)blockIdx.y * 3 * n * GJ_NB;
  double* E = work + (size_t)blockIdx.y * 3 * n * GJ_NB + (size_t)2 * n * GJ_NB;
  const double* Di = dinv_all + (size_t)blockIdx.y * GJ_NB * GJ_NB;
  const int rows = n - I0 < 64 ? n - I0 : 64;
  Mfma<double>::acc_t acc[2][2];
  gj_tile_product(sm, acc, C + (size_t)I0 * GJ_NB, rows, Di, GJ_NB, GJ_NB, GJ_NB, 64 * h);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 1, wc = wave >> 1, kq = lane >> 4, ln = lane & 15;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 32 * wr + 16 * a + Mfma<double>::row(kq, v);
        if (row < rows) E[(size_t)(I0 + row) * GJ_NB + 64 * h + 32 * wc + 16 * b + ln] = acc[a][b][v];
      }
}

// S_IJ <- S_IJ - E_I C_J^T over the kept tiles I >= J outside K (tiles K0
// and K0 + 1); work-group p takes the p-th tile of the lower triangle in
// row order.  Eight waves per tile, each a 32 x 16 block (two 16 x 16 MFMA
// tiles), so four waves share each SIMD and hide one another's waits; the
// reduction runs in chunks of 32 through LDS, the next chunk's values
// loading into registers during the current chunk's MFMA steps.
__global__ void __launch_bounds__(512) k_sw_update(double* __restrict__ mats, int n, int kb,
                                                   const double* __restrict__ work) {
  const int p = blockIdx.x;
  int I = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  while (I * (I + 1) / 2 > p) --I;
  while ((I + 1) * (I + 2) / 2 <= p) ++I;
  const int J = p - I * (I + 1) / 2, K0 = kb / 64;
  if (I == K0 || I == K0 + 1 || J == K0 || J == K0 + 1) return;
  __shared__ GjTileSmem sm;
  const int I0 = I * 64, J0 = J * 64;
  double* A = mats + (size_t)blockIdx.y * n * n;
  const double* Ct = work + (size_t)blockIdx.y * 3 * n * GJ_NB + (size_t)n * GJ_NB;
  const double* E = Ct + (size_t)n * GJ_NB + (size_t)I0 * GJ_NB;
  const int xrows = n - I0 < 64 ? n - I0 : 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 1, wc = wave >> 1, kq = lane >> 4, ln = lane & 15;   // rows 32 wr, columns 16 wc
  // the tile's old values load first, so their trip from memory overlaps the
  // product (no work-group of this launch writes another's tile, E or C^T)
  double old[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = I0 + 32 * wr + 16 * a + Mfma<double>::row(kq, v);
      const int j = J0 + 16 * wc + ln;
      old[a][v] = (i < n && j < n) ? A[(size_t)i * n + j] : 0.0;
    }
  Mfma<double>::acc_t acc[2];
  acc[0] = acc[1] = Mfma<double>::acc_t{0, 0, 0, 0};
  double xr[4], yr[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = tid + 512 * q;
      const int row = t >> 5, k = t & 31;
      xr[q] = row < xrows ? E[(size_t)row * GJ_NB + k0 + k] : 0.0;
      const int ky = t >> 6, c = t & 63, j = J0 + c;
      yr[q] = j < n ? Ct[(size_t)(k0 + ky) * n + j] : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < GJ_NB; k0 += 32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = tid + 512 * q;
      sm.Xs[t & 31][t >> 5] = xr[q];
      sm.Ys[t >> 6][t & 63] = yr[q];
    }
    __syncthreads();
    if (k0 + 32 < GJ_NB) load(k0 + 32);
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      const int kk = 4 * st + kq;
      const double a0 = sm.Xs[kk][32 * wr + ln], a1 = sm.Xs[kk][32 * wr + 16 + ln];
      const double b0 = sm.Ys[kk][16 * wc + ln];
      acc[0] = Mfma<double>::mma(a0, b0, acc[0]);
      acc[1] = Mfma<double>::mma(a1, b0, acc[1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = I0 + 32 * wr + 16 * a + Mfma<double>::row(kq, v);
      const int j = J0 + 16 * wc + ln;
      if (i < n && j < n) A[(size_t)i * n + j] = old[a][v] - acc[a][v];
    }
}

// Row and column K of the swept matrix, one 64-row tile I per work-group:
// the kept tiles of S_KK (K0,K0), (K1,K0), (K1,K1) <- -D^{-1}; below K,
// S_I,Kh <- E_I's half h; above K, S_Kh,I <- that half transposed.
__global__ void __launch_bounds__(256) k_sw_panel_write(double* __restrict__ mats, int n, int kb,
                                                        const double* __restrict__ work,
                                                        const double* __restrict__ dinv_all) {
  __shared__ double Ts[64][65];
  const int I0 = blockIdx.x * 64, K0 = kb / 64, I = blockIdx.x;
  double* A = mats + (size_t)blockIdx.y * n * n;
  const double* E = work + (size_t)blockIdx.y * 3 * n * GJ_NB + (size_t)2 * n * GJ_NB;
  const double* Di = dinv_all + (size_t)blockIdx.y * GJ_NB * GJ_NB;
  const int w = n - kb < GJ_NB ? n - kb : GJ_NB;
  const int tid = threadIdx.x;
  if (I == K0 || I == K0 + 1) {
    // row tile I of D's kept lower part: columns 0 .. 64 (I - K0) + 63
    const int r0 = 64 * (I - K0);
    for (int h = 0; h <= I - K0; ++h) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int t = tid + 256 * q, a = t >> 6, b = t & 63;
        const int ra = r0 + a, cb = 64 * h + b;
        if (ra < w && cb < w) A[(size_t)(kb + ra) * n + kb + cb] = -Di[(size_t)ra * GJ_NB + cb];
      }
    }
    return;
  }
  if (I > K0 + 1) {    // S_IK <- E_I
#pragma unroll 4
    for (int q = 0; q < 32; ++q) {
      const int t = tid + 256 * q, a = t >> 7, k = t & 127, i = I0 + a;
      if (i < n && k < w) A[(size_t)i * n + kb + k] = E[(size_t)i * GJ_NB + k];
    }
    return;
  }
  // above K the kept tiles are S_Kh,I <- (E_I's half h)^T
  for (int h = 0; h < 2; ++h) {
    const int wh = w - 64 * h;
    if (wh <= 0) break;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = tid + 256 * q, a = t >> 6, k = t & 63, i = I0 + a;
      Ts[a][k] = i < n ? E[(size_t)i * GJ_NB + 64 * h + k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = tid + 256 * q, k = t >> 6, c = t & 63, i = I0 + c;
      if (k < wh && i < n) A[(size_t)(kb + 64 * h + k) * n + i] = Ts[c][k];
    }
    __syncthreads();
  }
}

void launch_gj_invert(double* mats, int n, int count, double* work, double* dinv, hipStream_t s) {
  if (!count) return;
  const int tiles = (n + 63) / 64;
  const int pairs = tiles * (tiles + 1) / 2;
  for (int kb = 0; kb < n; kb += GJ_NB) {
    IBMG_KLAUNCH(k_gj_diag, dim3(count), dim3(1024), 0, s, mats, n, kb, dinv);
    IBMG_LAUNCH_CHECK();
    IBMG_KLAUNCH(k_sw_panel_read, dim3(tiles, count), dim3(256), 0, s, mats, n, kb, work);
    IBMG_LAUNCH_CHECK();
    IBMG_KLAUNCH(k_sw_scale, dim3(tiles, count, 2), dim3(256), 0, s, dinv, n, kb, work);
    IBMG_LAUNCH_CHECK();
    IBMG_KLAUNCH(k_sw_update, dim3(pairs, count), dim3(512), 0, s, mats, n, kb, work);
    IBMG_LAUNCH_CHECK();
    IBMG_KLAUNCH(k_sw_panel_write, dim3(tiles, count), dim3(256), 0, s, mats, n, kb, work, dinv);
    IBMG_LAUNCH_CHECK();
  }
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

// global index of local unknown k of box pid (periodic wrap)
__device__ __forceinline__ size_t box_glob(const BoxGeom& g, int pid, int k) {
  const int N = g.N, m = g.m, nu = m * (m + 1);
  const int x0 = (pid % g.npd) * g.b - g.o, y0 = (pid / g.npd) * g.b - g.o;
  const size_t nn = (size_t)N * N;
  int ii, jj;
  size_t off;
  if (k < nu) {
    ii = k % (m + 1);
    jj = k / (m + 1);
    off = 0;
  } else if (k < 2 * nu) {
    const int q = k - nu;
    ii = q % m;
    jj = q / m;
    off = nn;
  } else {
    const int q = k - 2 * nu;
    ii = q % m;
    jj = q / m;
    off = 2 * nn;
  }
  return off + (size_t)pmod(y0 + jj, N) * N + pmod(x0 + ii, N);
}

// global index of owned row r of box pid
__device__ __forceinline__ size_t own_glob(const BoxGeom& g, int pid, int r) {
  const int bb = g.b * g.b;
  const int comp = r / bb, q = r % bb;
  const int gi = (pid % g.npd) * g.b + q % g.b, gj = (pid / g.npd) * g.b + q / g.b;
  return (size_t)comp * g.N * g.N + (size_t)gj * g.N + gi;
}

// Owned rows of A^{-1}, stored per box as row chunks of 64: element (row, j)
// at (row / 64) * nloc * 64 + j * 64 + row % 64 (rows beyond nown are 0), so
// a chunk's 64 rows of one column are contiguous and a chunk is one
// contiguous stream of nloc * 64 values.
template <typename T>
__global__ void k_extract_owned(const double* __restrict__ mats, int count, BoxGeom g,
                                T* __restrict__ out, bool full) {
  const size_t per = (size_t)g.nch * g.nloc * 64;
  const size_t tot = per * count;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const size_t blk = t / per;
    size_t rem = t % per;
    const int c = (int)(rem / ((size_t)g.nloc * 64));
    rem %= (size_t)g.nloc * 64;
    const int j = (int)(rem / 64), rr = (int)(rem % 64);
    const int row = c * 64 + rr;
    const double* A = mats + blk * g.nloc * g.nloc;
    // the swept matrix holds -A^{-1} in the tiles on or below the diagonal
    T v = 0;
    if (row < g.nown) {
      const int lr = full ? row : own_local(row, g);
      v = (T)(-((lr >> 6) >= (j >> 6) ? A[(size_t)lr * g.nloc + j] : A[(size_t)j * g.nloc + lr]));
    }
    out[t] = v;
  }
}

template <typename T>
void launch_extract_owned(const double* mats, int count, BoxGeom g, T* out, hipStream_t s, bool full) {
  if (!count) return;
  size_t tot = (size_t)g.nch * g.nloc * 64 * count;
  int grid = cdiv(tot, 256);
  if (grid > 16384) grid = 16384;
  IBMG_KLAUNCH((k_extract_owned<T>), dim3(grid), dim3(256), 0, s, mats, count, g, out, full);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Symmetric storage of the IB boxes' owned rows.  The owned-by-owned block
// of L_k^{-1} is a principal submatrix of a symmetric inverse (L_IB is
// symmetric), so only its tiles on and below the diagonal are kept: chunk c
// (owned rows 64c .. 64c+63) holds ncol_c = 64 (c + 1) + (nloc - nown)
// columns of 64 rows, in the permuted local order perm (the owned unknowns
// first, in owned order, then the non-owned ones in increasing local index):
// column q < 64 (c + 1) is owned column q, column q >= 64 (c + 1) is
// non-owned column nown + q - 64 (c + 1) of that order.  The owned columns
// of later tiles are the transposes of those tiles' entries: the chunks
// holding them add them as column sums (the apply kernel below).  At
// 16 x 16/4 boxes this streams 8.75 MB per box instead of 10.9 MB.
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t sym_chunk_off(const BoxGeom& g, int c) {
  const size_t ne = (size_t)(g.nloc - g.nown);
  return 64 * (64 * (size_t)c * (size_t)(c + 1) / 2 + (size_t)c * ne);
}
__host__ __device__ inline size_t sym_stride(const BoxGeom& g) { return sym_chunk_off(g, g.nch); }
size_t sym_box_stride(const BoxGeom& g) { return sym_stride(g); }
// partials per box, the chunks' columns cut into ks slices: chunk c's 64
// row sums of each slice, then its 64 c column sums
__host__ __device__ inline int sym_part_off(int c, int ks) { return 64 * ks * c + 32 * c * (c - 1); }
int sym_part_len(const BoxGeom& g, int n_ib) { return sym_part_off(g.nch, ras_ib_ksplit(g, n_ib)); }

template <typename T>
__global__ void k_extract_sym(const double* __restrict__ mats, int count, BoxGeom g, const int* __restrict__ perm,
                              T* __restrict__ out) {
  const size_t per = sym_stride(g);
  const size_t tot = per * count;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const size_t blk = t / per;
    size_t rem = t % per;
    int c = 0;
    while (c + 1 < g.nch && sym_chunk_off(g, c + 1) <= rem) ++c;
    rem -= sym_chunk_off(g, c);
    const int q = (int)(rem / 64), rr = (int)(rem % 64);
    const int row = c * 64 + rr;   // owned row (nown is a multiple of 64 here)
    const int nq = 64 * (c + 1);
    const int j = perm[q < nq ? q : g.nown + (q - nq)];
    const int lr = own_local(row, g);
    const double* A = mats + blk * g.nloc * g.nloc;
    // the swept matrix holds -A^{-1} in the tiles on or below the diagonal
    out[t] = (T)(-((lr >> 6) >= (j >> 6) ? A[(size_t)lr * g.nloc + j] : A[(size_t)j * g.nloc + lr]));
  }
}

template <typename T>
void launch_extract_sym(const double* mats, int count, BoxGeom g, const int* perm, T* out, hipStream_t s) {
  if (!count) return;
  if (g.nown % 64) throw Error(IBMG_ERR_ARG, "symmetric storage needs whole 64-row chunks");
  const size_t tot = sym_stride(g) * count;
  int grid = cdiv(tot, 256);
  if (grid > 16384) grid = 16384;
  IBMG_KLAUNCH((k_extract_sym<T>), dim3(grid), dim3(256), 0, s, mats, count, g, perm, out);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Restricted additive Schwarz (Alg. 2 from a zero guess):
//   z[G~_k] = (L_k^{-1} R_k r)[G~_k]  for every box k.
// The owned sets partition the unknowns, so every z entry is written by
// exactly one work-group and no atomics are needed.
//
// Boxes with their own inverse (IB boxes): work-group = (box, 64-row chunk).
// R_k r is gathered into LDS; each wave streams a quarter of the chunk's
// columns with 16-byte loads (a wave reads 1 KB of contiguous inverse per
// load: VEC rows per lane, VEC columns side by side), lane groups are summed
// by shuffles and the four quarters in a fixed order.
// ---------------------------------------------------------------------------
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};

// One (box, 64-row chunk) item over columns [cb, ce) of the chunk: Mc is the
// chunk of the box's owned-row inverse, r and z the box's system vectors; x
// holds nloc values (LDS, indexed by column), part 256.  With pout the 64
// row sums of this column slice go to pout instead of z.  PRE issues the
// first loads of the inverse before the gather (it holds their registers
// across it, which the batched kernel cannot spare).
template <typename T, bool PRE>
__device__ __forceinline__ void ras_ib_chunk(const T* __restrict__ r, T* __restrict__ z, const BoxGeom& g,
                                             const T* __restrict__ Mc, int pid, int chunk, T* x, T* part,
                                             bool acc_mode, int cb, int ce, T* __restrict__ pout) {
  using V = typename Vec16<T>::type;
  constexpr int VEC = Vec16<T>::n;
  constexpr int LPC = 64 / VEC;  // lanes per column
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int cph = lane / LPC;           // column phase 0..VEC-1
  const int rl = (lane % LPC) * VEC;    // first of this lane's VEC rows
  const int per = ((ce - cb + 4 * VEC - 1) / (4 * VEC)) * VEC;
  const int j0 = cb + q * per, j1 = j0 + per < ce ? j0 + per : ce;
  Mc += rl;
  int j = j0 + cph;
  // eight 16-byte loads in flight per lane, summed in a fixed tree; the
  // inverse streams through once per sweep, so its loads are non-temporal
  // and leave the caches to the level's vectors.  With PRE the first eight
  // are issued before the residual gather, so that they overlap it.
  constexpr int UNR = 8;
  auto load8 = [&](V* m, int jj) {
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      m[u] = __builtin_nontemporal_load(reinterpret_cast<const V*>(Mc + (size_t)(jj + u * VEC) * 64));
  };
  T acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  auto fma8 = [&](const V* m, int jj) {
    T xv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) xv[u] = x[jj + u * VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      T t[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) t[u] = reinterpret_cast<const T*>(&m[u])[v] * xv[u];
      acc[v] += ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    }
  };
  const bool first = PRE && j + (UNR - 1) * VEC < j1;
  V m0[UNR];
  if (first) load8(m0, j);
  for (int k = cb + threadIdx.x; k < ce; k += blockDim.x) x[k] = r[box_glob(g, pid, k)];
  __syncthreads();
  if (first) {
    fma8(m0, j);
    j += UNR * VEC;
  }
  for (; j + (UNR - 1) * VEC < j1; j += UNR * VEC) {
    V m[UNR];
    load8(m, j);
    fma8(m, j);
  }
  for (; j < j1; j += VEC) {
    const V m0 = __builtin_nontemporal_load(reinterpret_cast<const V*>(Mc + (size_t)j * 64));
    const T* a0 = reinterpret_cast<const T*>(&m0);
    const T x0 = x[j];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += a0[v] * x0;
  }
  // sum the VEC column phases (lanes l, l + LPC, ...)
#pragma unroll
  for (int off = 32; off >= LPC; off >>= 1)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += __shfl_down(acc[v], off, 64);
  if (lane < LPC)
#pragma unroll
    for (int v = 0; v < VEC; ++v) part[q * 64 + rl + v] = acc[v];
  __syncthreads();
  if (q == 0) {
    const int row = chunk * 64 + lane;
    const T v = (part[lane] + part[64 + lane]) + (part[128 + lane] + part[192 + lane]);
    if (pout) {
      pout[lane] = v;
    } else if (row < g.nown) {
      const size_t o = own_glob(g, pid, row);
      z[o] = acc_mode ? z[o] + v : v;
    }
  }
}

// grid (boxes, row chunks, column slices); with more than one slice the
// slices' row sums go to spart[((slice * n_ib + box) * nch + chunk) * 64 + row]
template <typename T>
__global__ void __launch_bounds__(256) k_ras_ib(const T* __restrict__ r, T* __restrict__ z, BoxGeom g,
                                                const T* __restrict__ inv, const int* __restrict__ boxes, bool acc,
                                                T* __restrict__ spart) {
  extern __shared__ char smem_raw[];
  T* x = reinterpret_cast<T*>(smem_raw);
  T* part = x + ((g.nloc + 3) & ~3);
  const int slot = blockIdx.x, ks = gridDim.z;
  const int cs = ((g.nloc + ks - 1) / ks + 63) / 64 * 64;
  const int cb = blockIdx.z * cs, ce = cb + cs < g.nloc ? cb + cs : g.nloc;
  T* pout = ks > 1 ? spart + (((size_t)blockIdx.z * gridDim.x + slot) * g.nch + blockIdx.y) * 64 : nullptr;
  ras_ib_chunk<T, true>(r, z, g, inv + ((size_t)slot * g.nch + blockIdx.y) * g.nloc * 64, boxes[slot],
                        blockIdx.y, x, part, acc, cb < ce ? cb : ce, ce, pout);
}

// IB boxes from the symmetric storage: work-group = (box, 64-row chunk c,
// column slice).  R_k r is gathered into LDS in the permuted local order.
// The chunk's stored columns are cut into gridDim.z slices of whole
// 64-column tiles; a slice's columns stream in batches of UNR x VEC
// (16-byte loads, eight in flight per lane), batches dealt to the four
// waves in turn.  Every column adds
// its entries times x_q to the rows (lane sums, as in k_ras_ib); a column
// of an earlier owned tile (q < 64 c) also forms its transposed product,
// the sum over the chunk's rows of M[row][q] x_row, reduced over the lanes
// of its column phase, which belongs to owned row q of an earlier chunk.
// The box's partials: the chunk's row sums per slice at sym_part_off(c,
// ks), its column sums after them (each column in one slice).
// Sum over the 16 lanes of a DPP row (every lane of the row ends with the
// same bits): swap neighbours and pairs within quads, then mirror within
// halves and within the row, adding after each step.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <typename T>
__device__ __forceinline__ T row16_sum(T p) {
  p += dpp_move<0xB1>(p);    // quad_perm [1,0,3,2]
  p += dpp_move<0x4E>(p);    // quad_perm [2,3,0,1]
  p += dpp_move<0x141>(p);   // row_half_mirror
  p += dpp_move<0x140>(p);   // row_mirror
  return p;
}

template <typename T>
__global__ void __launch_bounds__(256) k_ras_ib_sym(const T* __restrict__ r, BoxGeom g, const T* __restrict__ inv,
                                                    const int* __restrict__ boxes, const int* __restrict__ perm,
                                                    T* __restrict__ part) {
  using V = typename Vec16<T>::type;
  constexpr int VEC = Vec16<T>::n;
  constexpr int LPC = 64 / VEC;   // lanes per column
  constexpr int UNR = 8, B = UNR * VEC;
  extern __shared__ char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  T* red = xs + ((g.nloc + 3) & ~3);   // 4 waves x 64 row sums
  T* tcol = red + 256;                 // the chunk's 64 c column sums
  const int slot = blockIdx.x, c = blockIdx.y, sl = blockIdx.z, ks = gridDim.z, pid = boxes[slot];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cph = lane / LPC, rl = (lane % LPC) * VEC;
  const int nq = 64 * (c + 1), ntr = 64 * c, ncol = nq + (g.nloc - g.nown);
  const int cs = ((ncol + ks - 1) / ks + 63) / 64 * 64;
  const int cb = sl * cs < ncol ? sl * cs : ncol, ce = cb + cs < ncol ? cb + cs : ncol;
  const T* Mc = inv + (size_t)slot * sym_stride(g) + sym_chunk_off(g, c) + rl;
  // the wave's first batch of the inverse is issued before the residual
  // gather, so its trip from memory overlaps the gather
  const int jb0 = cb + wave * B;
  const bool pre = jb0 + B <= ce;
  V m0[UNR];
  if (pre)
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      m0[u] = __builtin_nontemporal_load(reinterpret_cast<const V*>(Mc + (size_t)(jb0 + cph + u * VEC) * 64));
  for (int k = tid; k < g.nloc; k += 256) xs[k] = r[box_glob(g, pid, perm[k])];
  __syncthreads();
  T xr[VEC];   // this lane's rows' residual values (owned rows 64 c + rl + v)
#pragma unroll
  for (int v = 0; v < VEC; ++v) xr[v] = xs[64 * c + rl + v];
  T acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  auto xcol = [&](int q) { return xs[q < nq ? q : g.nown + (q - nq)]; };
  // one column's contribution; tr: the column also needs its transposed sum
  auto column = [&](const V& m, int q, bool tr) {
    const T* a = reinterpret_cast<const T*>(&m);
    const T x = xcol(q);
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += a[v] * x;
    if (tr) {
      T p = 0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) p += a[v] * xr[v];
      // the column phase's LPC lanes: rows of 16 by DPP, then across rows
      p = row16_sum(p);
      if constexpr (LPC == 32) p += __shfl_xor(p, 16, 64);
      if (lane % LPC == 0) tcol[q] = p;
    }
  };
  int jstart = jb0;
  if (pre) {
    const bool tr = jb0 + B <= ntr;
#pragma unroll
    for (int u = 0; u < UNR; ++u) column(m0[u], jb0 + cph + u * VEC, tr);
    jstart += 4 * B;
  }
  for (int jb = jstart; jb < ce; jb += 4 * B) {
    if (jb + B <= ce) {
      V m[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u)
        m[u] = __builtin_nontemporal_load(reinterpret_cast<const V*>(Mc + (size_t)(jb + cph + u * VEC) * 64));
      const bool tr = jb + B <= ntr;   // batches never straddle ntr (slices start at multiples of 64)
#pragma unroll
      for (int u = 0; u < UNR; ++u) column(m[u], jb + cph + u * VEC, tr);
    } else {
      for (int u = 0; u < UNR; ++u) {
        const int q = jb + cph + u * VEC;
        if (q >= ce) break;
        const V m0 = __builtin_nontemporal_load(reinterpret_cast<const V*>(Mc + (size_t)q * 64));
        column(m0, q, false);   // a partial batch only ends the last slice, in the non-owned columns
      }
    }
  }
  // sum the VEC column phases, then the four waves
#pragma unroll
  for (int off = 32; off >= LPC; off >>= 1)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += __shfl_down(acc[v], off, 64);
  if (lane < LPC)
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[wave * 64 + rl + v] = acc[v];
  __syncthreads();
  T* pb = part + (size_t)slot * sym_part_off(g.nch, ks) + sym_part_off(c, ks);
  if (tid < 64) pb[64 * sl + tid] = (red[tid] + red[64 + tid]) + (red[128 + tid] + red[192 + tid]);
  for (int q = cb + tid; q < (ce < ntr ? ce : ntr); q += 256) pb[64 * ks + q] = tcol[q];
}

// z[owned rows] (=, or += with acc) the sum of a split launch's slices, in
// slice order, for the IB boxes (pa: ksa slices of na boxes) and the interior
// boxes (pb: ksb slices of nb boxes) of one sweep in one launch; slice sl of
// box b holds row `row` at p[(sl * n + b) * nch * 64 + row].  A list that was
// not split has n = 0.
// The symmetric IB list (ps: partials of ns boxes, kss column slices) comes
// first: owned row r = 64 c + i is chunk c's row sums i of its slices, in
// slice order, plus the column sums at r of every later chunk, added in
// chunk order.
template <typename T>
__global__ void k_ras_sum(const T* __restrict__ pa, const int* __restrict__ ba, int na, int ksa,
                          const T* __restrict__ pb, const int* __restrict__ bb, int nb, int ksb,
                          const T* __restrict__ ps, int ns, int kss, T* __restrict__ z, BoxGeom g, bool acc) {
  const int nown_pad = g.nch * 64;
  const size_t t0 = (size_t)ns * g.nown;
  const size_t ta = (size_t)na * g.nown, tot = t0 + ta + (size_t)nb * g.nown;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    if (t < t0) {
      const int b = (int)(t / g.nown), row = (int)(t % g.nown);
      const int cr = row >> 6;
      const T* pp = ps + (size_t)b * sym_part_off(g.nch, kss);
      const T* pr = pp + sym_part_off(cr, kss) + (row & 63);
      // the row's kss slice sums, then the later chunks' column sums: read
      // eight at a time, added one by one in that order
      const int m = kss + (g.nch - cr - 1);
      auto val = [&](int i) { return i < kss ? pr[64 * i] : pp[sym_part_off(cr + 1 + i - kss, kss) + 64 * kss + row]; };
      T a = pr[0];
      for (int i0 = 1; i0 < m; i0 += 8) {
        T v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = i0 + j < m ? val(i0 + j) : T(0);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (i0 + j < m) a += v[j];
      }
      const size_t o = own_glob(g, ba[b], row);
      z[o] = acc ? z[o] + a : a;
      continue;
    }
    const bool first = t - t0 < ta;
    const size_t u = first ? t - t0 : t - t0 - ta;
    const int b = (int)(u / g.nown), row = (int)(u % g.nown);
    const T* p = first ? pa : pb;
    const int n = first ? na : nb, ks = first ? ksa : ksb;
    T a = 0;
    for (int s0 = 0; s0 < ks; s0 += 8) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = s0 + j < ks ? p[((size_t)(s0 + j) * n + b) * nown_pad + row] : T(0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (s0 + j < ks) a += v[j];
    }
    const size_t o = own_glob(g, (first ? ba : bb)[b], row);
    z[o] = acc ? z[o] + a : a;
  }
}

// Column slices of the IB-box kernel: enough work-groups to cover the
// device (>= 1024) while every slice keeps at least 128 columns.
int ras_ib_ksplit(const BoxGeom& g, int n_ib) {
  if (n_ib <= 0) return 1;
  int ks = 1;
  while (ks < 16 && n_ib * g.nch * ks < 1024 && g.nloc / (2 * ks) >= 128) ks *= 2;
  return ks;
}

// ---------------------------------------------------------------------------
// Interior boxes share one inverse (translation invariance of the periodic
// stencil away from the structure), so they form one dense contraction
//   Z[64-row chunk, 32 boxes] = M[chunk, :] X[:, boxes]
// on the matrix cores: wave w owns rows 16w..16w+15 of the chunk and two
// 16 x 16 output tiles (boxes 0-15, 16-31), accumulated with 16x16x4 MFMA
// steps.  A fragments stream straight from the chunk layout (16 contiguous
// rows per reduction index), B fragments come from the boxes' residuals,
// gathered 64 reduction indices at a time into LDS.

// Reference tile width of the single-system interior product: the number of
// reduction slices is derived from it, so the sums (and the results) do not
// depend on the tile width a level runs with (16 or 32, picked by timing).
constexpr int kIntTile = 32;

// Gathers of a box's local residual.  The level's local-unknown table holds
// nloc codes (comp << 24 | jj << 12 | ii) followed by nloc linear offsets
// comp N^2 + jj N + ii.  A box whose enlarged region (corner x0, y0, faces up
// to x0 + m, y0 + m) lies clear of the periodic edges reads unknown k at
// base + y0 N + x0 + offset[k] (box_lin returns that start, or -1 where the
// region wraps and each coordinate is reduced instead).
__device__ __forceinline__ long long box_lin(const BoxGeom& g, size_t base, int x0, int y0) {
  const bool clear = x0 >= 0 && y0 >= 0 && x0 + g.m < g.N && y0 + g.m < g.N;
  return clear ? (long long)base + (long long)y0 * g.N + x0 : -1;
}

template <typename T>
__device__ __forceinline__ T box_value(const T* __restrict__ r, const BoxGeom& g, const int* __restrict__ loc_tab,
                                       int k, size_t base, long long lin, int x0, int y0) {
  if (lin >= 0) return r[lin + loc_tab[g.nloc + k]];
  const int N = g.N;
  const int code = loc_tab[k];
  int ii = (code & 0xfff) + x0, jj = ((code >> 12) & 0xfff) + y0;
  ii = ii < 0 ? ii + N : (ii >= N ? ii - N : ii);
  jj = jj < 0 ? jj + N : (jj >= N ? jj - N : jj);
  return r[base + (size_t)(code >> 24) * N * N + (size_t)jj * N + ii];
}

// Shared memory of one interior tile: the gathered residual columns and the
// tile's box table.
constexpr int kIntLinTab = 2048;   // linear offsets of one item's reduction range kept in LDS

template <typename T, int TB>
struct IntTileSmem {
  T Xs[64][TB + 1];
  size_t base[TB];   // system offset of each box's vectors
  long long lin[TB];  // see box_lin
  int bid[TB], bx0[TB], by0[TB];
  int ltab[kIntLinTab];
};

// One interior tile (boxes ents[tile * TB ..], 64-row chunk, reduction slice
// kslice of ksplit): box entry e = s * nbox + box id, system s at r + s
// sys_n; boxes of inactive systems are left out.
template <typename T, int TB, bool REGPLAN = true>
__device__ __forceinline__ void ras_int_tile(const T* __restrict__ r, T* __restrict__ z, const BoxGeom& g,
                                             size_t sys_n, int nbox, const T* __restrict__ M,
                                             const int* __restrict__ ents, int nlist, int tile, int chunk,
                                             int kslice, int ksplit, const int* __restrict__ loc_tab,
                                             const int* __restrict__ active, T* __restrict__ part,
                                             IntTileSmem<T, TB>& sm, bool acc_mode) {
  constexpr int KC = 64, GPT = KC * TB / 256, AS = KC / 4;
  using acc_t = typename Mfma<T>::acc_t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int bt = tile * TB;
  if (tid < TB) {
    const int b = bt + tid;
    int pid = -1, sy = 0;
    if (b < nlist) {
      const int e = ents[b];
      sy = e / nbox;
      pid = e - sy * nbox;
      if (active && !active[sy]) pid = -1;
    }
    sm.bid[tid] = pid;
    sm.base[tid] = (size_t)sy * sys_n;
    sm.bx0[tid] = pid >= 0 ? (pid % g.npd) * g.b - g.o : 0;
    sm.by0[tid] = pid >= 0 ? (pid / g.npd) * g.b - g.o : 0;
    sm.lin[tid] = box_lin(g, sm.base[tid], sm.bx0[tid], sm.by0[tid]);
  }
  // this item's slice of the reduction index: chunks [c0, c1) of KC columns
  const int nchunk = (g.nloc + KC - 1) / KC;
  const int per = (nchunk + ksplit - 1) / ksplit;
  const int c0 = kslice * per;
  const int c1 = c0 + per < nchunk ? c0 + per : nchunk;
  // the slice's linear offsets in LDS (when they fit), so a gather waits on
  // one trip to memory, not two
  const int kb0 = c0 * KC, kspan = (c1 - c0) * KC;
  const bool ltab_lds = kspan <= kIntLinTab;
  if (ltab_lds)
    for (int k = tid; k < kspan; k += 256) sm.ltab[k] = kb0 + k < g.nloc ? loc_tab[g.nloc + kb0 + k] : 0;
  __syncthreads();
  const T* Mrow = M + (size_t)chunk * g.nloc * 64 + 16 * wave + (lane & 15);
  const int kq = lane >> 4, bl = lane & 15;
  constexpr int NT = TB / 16;  // 16 x 16 output tiles per wave
  acc_t acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = acc_t{0, 0, 0, 0};
  T ga[AS];
  // the gather runs along the reduction index (a wave reads 64 consecutive
  // local unknowns of one box, mostly contiguous rows of the grid) and is
  // transposed into Xs[k][box].  A thread's reduction index within a chunk
  // (tid mod KC) and its boxes (one per u) are fixed, so the boxes' linear
  // starts stay in registers and a chunk costs one offset read per thread;
  // boxes that wrap the periodic edges (or an offset table not in LDS) take
  // the general path.
  // (REGPLAN = false, the batched launch: the boxes' starts are re-read from
  // LDS per value, which keeps that kernel's register count down)
  long long glin[GPT];
  bool gslow = false;
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const int b = (tid + u * 256) / KC;
    glin[u] = sm.bid[b] >= 0 ? sm.lin[b] : -2;
    gslow |= sm.bid[b] >= 0 && (!ltab_lds || sm.lin[b] < 0);
  }
  auto gather = [&](int c, T* gxo) {
    if constexpr (!REGPLAN) {
      const int j0 = c * KC;
#pragma unroll
      for (int u = 0; u < GPT; ++u) {
        const int t = tid + u * 256;
        const int k = t % KC, b = t / KC;
        const int jk = j0 + k;
        T val = 0;
        if (jk < g.nloc && sm.bid[b] >= 0) {
          if (ltab_lds && sm.lin[b] >= 0) val = r[sm.lin[b] + sm.ltab[jk - kb0]];
          else val = box_value<T>(r, g, loc_tab, jk, sm.base[b], sm.lin[b], sm.bx0[b], sm.by0[b]);
        }
        gxo[u] = val;
      }
      return;
    }
    const int jk = c * KC + tid % KC;
    const bool in = jk < g.nloc;
    const int off = in && ltab_lds ? sm.ltab[jk - kb0] : 0;
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      T val = 0;
      if (in && glin[u] >= 0 && ltab_lds) {
        val = r[glin[u] + off];
      } else if (in && gslow && glin[u] != -2) {
        const int b = (tid + u * 256) / KC;
        val = box_value<T>(r, g, loc_tab, jk, sm.base[b], sm.lin[b], sm.bx0[b], sm.by0[b]);
      }
      gxo[u] = val;
    }
  };
  auto load_a = [&](int c, T* gao) {
    const int j0 = c * KC;
    if (j0 + KC <= g.nloc) {   // a full chunk: no bounds to test
      const T* Mj = Mrow + (size_t)(j0 + kq) * 64;
#pragma unroll
      for (int s = 0; s < AS; ++s) gao[s] = Mj[(size_t)s * 256];
    } else {
#pragma unroll
      for (int s = 0; s < AS; ++s) {
        const int jk = j0 + 4 * s + kq;
        gao[s] = jk < g.nloc ? Mrow[(size_t)jk * 64] : (T)0;
      }
    }
  };
  // the next chunk's gather and inverse rows load during the MFMAs
  T gx[GPT];
  if (c0 < c1) {
    gather(c0, gx);
    load_a(c0, ga);
  }
  for (int c = c0; c < c1; ++c) {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int t = tid + u * 256;
      sm.Xs[t % KC][t / KC] = gx[u];
    }
    __syncthreads();
    T a[AS];
#pragma unroll
    for (int s = 0; s < AS; ++s) a[s] = ga[s];
    if (c + 1 < c1) {
      gather(c + 1, gx);
      load_a(c + 1, ga);
    }
#pragma unroll
    for (int s = 0; s < AS; ++s) {
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[q] = Mfma<T>::mma(a[s], sm.Xs[4 * s + kq][16 * q + bl], acc[q]);
    }
    __syncthreads();
  }
  const int nown_pad = g.nch * 64;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = chunk * 64 + 16 * wave + Mfma<T>::row(kq, v);
    if (row >= g.nown) continue;
    if (ksplit == 1) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int bb = 16 * q + bl;
        if (sm.bid[bb] >= 0) {
          const size_t o = sm.base[bb] + own_glob(g, sm.bid[bb], row);
          z[o] = acc_mode ? z[o] + acc[q][v] : acc[q][v];
        }
      }
    } else {
      T* pp = part + (size_t)kslice * nlist * nown_pad;
#pragma unroll
      for (int q = 0; q < NT; ++q)
        if (bt + 16 * q + bl < nlist) pp[(size_t)(bt + 16 * q + bl) * nown_pad + row] = acc[q][v];
    }
  }
}

// Register-blocked form of the interior product: a work-group owns a
// 64-row chunk and 64 boxes, its four waves 2 x 2 blocks of 32 rows x 32
// boxes (four 16 x 16 MFMA tiles each).  Each 32-wide reduction step stages
// the chunk's A block (32 x 64, contiguous rows) and the boxes' gathered
// residuals (32 x 64) in LDS, the next step's values loading into registers
// during the MFMAs.  The reduction runs over the same 64-column chunks and
// slices, in the same order, as the narrow tiles, so the sums agree.
template <typename T>
struct GemmSmem {
  T As[32][64];        // [reduction index][row of the chunk]
  T Bs[32][65];        // [reduction index][box]
  size_t base[64];
  long long lin[64];
  int bid[64], bx0[64], by0[64];
};

template <typename T>
__device__ __forceinline__ void ras_int_gemm(const T* __restrict__ r, T* __restrict__ z, const BoxGeom& g,
                                             size_t sys_n, int nbox, const T* __restrict__ M,
                                             const int* __restrict__ ents, int nlist, int tile, int chunk,
                                             int kslice, int ksplit, const int* __restrict__ loc_tab,
                                             const int* __restrict__ active, T* __restrict__ part,
                                             GemmSmem<T>& sm, bool acc_mode) {
  constexpr int TBX = 64, KC = 32, GP = KC * TBX / 256;
  using acc_t = typename Mfma<T>::acc_t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 1, wb = wave >> 1;
  const int bt = tile * TBX;
  if (tid < TBX) {
    const int b = bt + tid;
    int pid = -1, sy = 0;
    if (b < nlist) {
      const int e = ents[b];
      sy = e / nbox;
      pid = e - sy * nbox;
      if (active && !active[sy]) pid = -1;
    }
    sm.bid[tid] = pid;
    sm.base[tid] = (size_t)sy * sys_n;
    sm.bx0[tid] = pid >= 0 ? (pid % g.npd) * g.b - g.o : 0;
    sm.by0[tid] = pid >= 0 ? (pid / g.npd) * g.b - g.o : 0;
    sm.lin[tid] = box_lin(g, sm.base[tid], sm.bx0[tid], sm.by0[tid]);
  }
  __syncthreads();
  const int nchunk = (g.nloc + 63) / 64;
  const int per = (nchunk + ksplit - 1) / ksplit;
  const int c0 = kslice * per, c1 = c0 + per < nchunk ? c0 + per : nchunk;
  const int kb = c0 * 64, ke = c1 * 64;     // reduction indices beyond nloc read as zero
  const T* Mc = M + (size_t)chunk * g.nloc * 64;
  const int kq = lane >> 4, ln = lane & 15;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  T ga[GP], gb[GP];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < GP; ++u) {
      const int t = tid + u * 256;
      const int ka = t / 64, row = t % 64;   // A: 64 consecutive rows per index
      const int ja = k0 + ka;
      ga[u] = ja < g.nloc ? Mc[(size_t)ja * 64 + row] : (T)0;
      const int kx = t % KC, b = t / KC;     // X: consecutive indices of one box
      const int jx = k0 + kx;
      T val = 0;
      if (jx < g.nloc && sm.bid[b] >= 0)
        val = box_value<T>(r, g, loc_tab, jx, sm.base[b], sm.lin[b], sm.bx0[b], sm.by0[b]);
      gb[u] = val;
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int u = 0; u < GP; ++u) {
      const int t = tid + u * 256;
      sm.As[t / 64][t % 64] = ga[u];
      sm.Bs[t % KC][t / KC] = gb[u];
    }
    __syncthreads();
    if (k0 + KC < ke) load(k0 + KC);   // in flight during the MFMAs below
#pragma unroll
    for (int st = 0; st < KC / 4; ++st) {
      const int kk = 4 * st + kq;
      const T a0 = sm.As[kk][32 * wr + ln], a1 = sm.As[kk][32 * wr + 16 + ln];
      const T b0 = sm.Bs[kk][32 * wb + ln], b1 = sm.Bs[kk][32 * wb + 16 + ln];
      acc[0][0] = Mfma<T>::mma(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mma(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mma(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  const int nown_pad = g.nch * 64;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = chunk * 64 + 32 * wr + 16 * a + Mfma<T>::row(kq, v);
        const int bb = 32 * wb + 16 * b + ln;
        if (row >= g.nown) continue;
        if (ksplit == 1) {
          if (sm.bid[bb] >= 0) {
            const size_t o = sm.base[bb] + own_glob(g, sm.bid[bb], row);
            z[o] = acc_mode ? z[o] + acc[a][b][v] : acc[a][b][v];
          }
        } else if (bt + bb < nlist) {
          part[((size_t)kslice * nlist + bt + bb) * nown_pad + row] = acc[a][b][v];
        }
      }
}

template <typename T>
__global__ void __launch_bounds__(256) k_ras_interior_g(const T* __restrict__ r, T* __restrict__ z, BoxGeom g,
                                                        const T* __restrict__ M, const int* __restrict__ boxes,
                                                        int nlist, const int* __restrict__ loc_tab,
                                                        T* __restrict__ part, int ksplit, bool acc) {
  __shared__ GemmSmem<T> sm;
  ras_int_gemm<T>(r, z, g, 0, g.npd * g.npd, M, boxes, nlist, blockIdx.x, blockIdx.y, blockIdx.z, ksplit, loc_tab,
                  nullptr, part, sm, acc);
}

template <typename T, int TB>
__global__ void __launch_bounds__(256) k_ras_interior(const T* __restrict__ r, T* __restrict__ z,
                                                      BoxGeom g, const T* __restrict__ M,
                                                      const int* __restrict__ boxes, int nlist,
                                                      const int* __restrict__ loc_tab,
                                                      T* __restrict__ part, int ksplit, bool acc) {
  __shared__ IntTileSmem<T, TB> sm;
  ras_int_tile<T, TB>(r, z, g, 0, g.npd * g.npd, M, boxes, nlist, blockIdx.x, blockIdx.y, blockIdx.z, ksplit,
                      loc_tab, nullptr, part, sm, acc);
}

// Pipelined form of the interior product: a work-group owns a 64-row chunk,
// 64 boxes and one reduction slice; wave w the chunk's rows 16w..16w+15
// against all 64 boxes (four 16 x 16 output tiles), its inverse fragments
// loading straight into registers.  The boxes' gathered residuals pass
// through two LDS buffers, 32 reduction indices at a time: the next step's
// inverse fragments and gathers load while the MFMAs read the current
// buffer, and one barrier per step hands the buffers over.  The grid is one
// dimensional and remapped so that the work-groups one XCD receives (the
// hardware deals them to the eight XCDs in turn) form a contiguous run of
// tasks, chunk-major: each XCD's L2 then serves few chunks of the shared
// inverse.  Slices and the order of every output's MFMA steps are those of
// the tile kernels above, so the sums agree bit for bit.
constexpr int kPipeKC = 32;

template <typename T>
struct PipeSmem {
  T Xs[2][kPipeKC][65];   // [buffer][reduction index][box]
  size_t base[64];
  long long lin[64];
  int bid[64], bx0[64], by0[64];
  int ltab[kIntLinTab];
};

// Task of work-group wg of nwg: XCD x = wg mod 8 receives wg = x, x + 8, ...;
// those map to the run [x q + min(x, rem), ...) of length q + (x < rem),
// q = nwg / 8, rem = nwg mod 8, a bijection onto [0, nwg).
__device__ __forceinline__ int xcd_task(int wg, int nwg) {
  const int q = nwg >> 3, rem = nwg & 7, x = wg & 7, u = wg >> 3;
  return x * q + (x < rem ? x : rem) + u;
}

template <typename T>
__global__ void __launch_bounds__(256) k_ras_interior_p(const T* __restrict__ r, T* __restrict__ z, BoxGeom g,
                                                        const T* __restrict__ M, const int* __restrict__ boxes,
                                                        int nlist, const int* __restrict__ loc_tab,
                                                        T* __restrict__ part, int ksplit, bool acc_mode) {
  constexpr int TB = 64, KC = kPipeKC, GPT = KC * TB / 256, AS = KC / 4, NT = TB / 16;
  __shared__ PipeSmem<T> sm;
  using acc_t = typename Mfma<T>::acc_t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ntb = (nlist + TB - 1) / TB;
  const int task = xcd_task(blockIdx.x, gridDim.x);
  const int tile = task % ntb, cs = task / ntb;
  const int kslice = cs % ksplit, chunk = cs / ksplit;
  const int bt = tile * TB;
  if (tid < TB) {
    const int b = bt + tid;
    const int pid = b < nlist ? boxes[b] : -1;
    sm.bid[tid] = pid;
    sm.base[tid] = 0;
    sm.bx0[tid] = pid >= 0 ? (pid % g.npd) * g.b - g.o : 0;
    sm.by0[tid] = pid >= 0 ? (pid / g.npd) * g.b - g.o : 0;
    sm.lin[tid] = box_lin(g, 0, sm.bx0[tid], sm.by0[tid]);
  }
  // the slice: 64-column chunks [c0, c1) of the reduction index, as above
  const int nchunk = (g.nloc + 63) / 64;
  const int per = (nchunk + ksplit - 1) / ksplit;
  const int c0 = kslice * per;
  const int c1 = c0 + per < nchunk ? c0 + per : nchunk;
  const int kb = c0 * 64, kspan = c1 > c0 ? (c1 - c0) * 64 : 0;
  const bool ltab_lds = kspan <= kIntLinTab;
  if (ltab_lds)
    for (int k = tid; k < kspan; k += 256) sm.ltab[k] = kb + k < g.nloc ? loc_tab[g.nloc + kb + k] : 0;
  __syncthreads();
  const T* Mrow = M + (size_t)chunk * g.nloc * 64 + 16 * wave + (lane & 15);
  const int kq = lane >> 4, bl = lane & 15;
  acc_t acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = acc_t{0, 0, 0, 0};
  // as in the tile kernels: fixed reduction index and boxes per thread, the
  // boxes' linear starts in registers, one offset read per step
  long long glin[GPT];
  bool gslow = false;
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const int b = (tid + u * 256) / KC;
    glin[u] = sm.bid[b] >= 0 ? sm.lin[b] : -2;
    gslow |= sm.bid[b] >= 0 && (!ltab_lds || sm.lin[b] < 0);
  }
  auto gather = [&](int j0, T* gxo) {
    const int jk = j0 + tid % KC;
    const bool in = jk < g.nloc;
    const int off = in && ltab_lds ? sm.ltab[jk - kb] : 0;
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      T val = 0;
      if (in && glin[u] >= 0 && ltab_lds) {
        val = r[glin[u] + off];
      } else if (in && gslow && glin[u] != -2) {
        const int b = (tid + u * 256) / KC;
        val = box_value<T>(r, g, loc_tab, jk, 0, sm.lin[b], sm.bx0[b], sm.by0[b]);
      }
      gxo[u] = val;
    }
  };
  auto load_a = [&](int j0, T* gao) {
    if (j0 + KC <= g.nloc) {
      const T* Mj = Mrow + (size_t)(j0 + kq) * 64;
#pragma unroll
      for (int s = 0; s < AS; ++s) gao[s] = Mj[(size_t)s * 256];
    } else {
#pragma unroll
      for (int s = 0; s < AS; ++s) {
        const int jk = j0 + 4 * s + kq;
        gao[s] = jk < g.nloc ? Mrow[(size_t)jk * 64] : (T)0;
      }
    }
  };
  auto stage = [&](int buf, const T* gxi) {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int t = tid + u * 256;
      sm.Xs[buf][t % KC][t / KC] = gxi[u];
    }
  };
  const int nsteps = kspan / KC;
  T ga[AS], gx[GPT];
  if (nsteps > 0) {
    load_a(kb, ga);
    gather(kb, gx);
    stage(0, gx);
  }
  __syncthreads();
  for (int st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    T a[AS];
#pragma unroll
    for (int s = 0; s < AS; ++s) a[s] = ga[s];
    const bool more = st + 1 < nsteps;
    if (more) {
      load_a(kb + (st + 1) * KC, ga);
      gather(kb + (st + 1) * KC, gx);
    }
#pragma unroll
    for (int s = 0; s < AS; ++s) {
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[q] = Mfma<T>::mma(a[s], sm.Xs[buf][4 * s + kq][16 * q + bl], acc[q]);
    }
    if (more) stage(buf ^ 1, gx);
    __syncthreads();
  }
  const int nown_pad = g.nch * 64;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = chunk * 64 + 16 * wave + Mfma<T>::row(kq, v);
    if (row >= g.nown) continue;
    if (ksplit == 1) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int bb = 16 * q + bl;
        if (sm.bid[bb] >= 0) {
          const size_t o = own_glob(g, sm.bid[bb], row);
          z[o] = acc_mode ? z[o] + acc[q][v] : acc[q][v];
        }
      }
    } else {
      T* pp = part + (size_t)kslice * nlist * nown_pad;
#pragma unroll
      for (int q = 0; q < NT; ++q)
        if (bt + 16 * q + bl < nlist) pp[(size_t)(bt + 16 * q + bl) * nown_pad + row] = acc[q][v];
    }
  }
}

// Reduction slices for the interior product: enough blocks to cover the
// device (>= 768) while every slice keeps at least two column chunks.
int ras_interior_ksplit(const BoxGeom& g, int n_int) {
  if (n_int <= 0) return 1;
  const int tiles = (n_int + kIntTile - 1) / kIntTile;
  const int nchunk = (g.nloc + 63) / 64;
  int ks = 1;
  while (ks < 8 && tiles * g.nch * ks < 768 && nchunk / (2 * ks) >= 2) ks *= 2;
  return ks;
}

// ---------------------------------------------------------------------------
// Interior product on gathered operands: the boxes' local residuals are
// gathered once into X[k][box] (nloc x nbp, boxes padded to 128), then
// Z = M X runs as 64-row x 128-box tiles on the matrix cores: four waves of
// 2 x 4 16x16x4 tiles, the reduction staged through LDS 32 indices at a time.
// The reduction slices and the order of each output's MFMA steps are those
// of the tile kernels above, so the results are the same.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_int_gather(const T* __restrict__ r, T* __restrict__ X, BoxGeom g,
                                                    const int* __restrict__ boxes, int nlist, int nbp,
                                                    const int* __restrict__ loc_tab) {
  const size_t tot = (size_t)g.nloc * nbp;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t / nbp), b = (int)(t % nbp);
    T v = 0;
    if (b < nlist) {
      const int pid = boxes[b];
      const int x0 = (pid % g.npd) * g.b - g.o, y0 = (pid / g.npd) * g.b - g.o;
      v = box_value<T>(r, g, loc_tab, k, 0, box_lin(g, 0, x0, y0), x0, y0);
    }
    X[t] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_int_gemm(const T* __restrict__ M, const T* __restrict__ X, T* __restrict__ z,
                                                  BoxGeom g, const int* __restrict__ boxes, int nlist, int nbp,
                                                  T* __restrict__ part, int ksplit, bool acc_mode) {
  constexpr int KC = 32;
  __shared__ T As[KC][64];
  __shared__ T Bs[KC][128];
  using acc_t = typename Mfma<T>::acc_t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 1, wb = wave >> 1, kq = lane >> 4, ln = lane & 15;
  const int chunk = blockIdx.x, B0 = blockIdx.y * 128, kslice = blockIdx.z;
  const int nchunk = (g.nloc + 63) / 64;
  const int per = (nchunk + ksplit - 1) / ksplit;
  const int c0 = kslice * per, c1 = c0 + per < nchunk ? c0 + per : nchunk;
  const int kb = c0 * 64, ke = c1 * 64;   // reduction indices beyond nloc read as zero
  const T* Mc = M + (size_t)chunk * g.nloc * 64;
  acc_t acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  T ga[8], gb[16];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = tid + 256 * u, kk = t >> 6, row = t & 63, k = k0 + kk;
      ga[u] = k < g.nloc ? Mc[(size_t)k * 64 + row] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = tid + 256 * u, kk = t >> 7, c = t & 127, k = k0 + kk;
      gb[u] = k < g.nloc ? X[(size_t)k * nbp + B0 + c] : (T)0;
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = tid + 256 * u;
      As[t >> 6][t & 63] = ga[u];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = tid + 256 * u;
      Bs[t >> 7][t & 127] = gb[u];
    }
    __syncthreads();
    if (k0 + KC < ke) load(k0 + KC);   // in flight during the MFMAs below
#pragma unroll
    for (int st = 0; st < KC / 4; ++st) {
      const int kk = 4 * st + kq;
      const T a0 = As[kk][32 * wr + ln], a1 = As[kk][32 * wr + 16 + ln];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const T bv = Bs[kk][64 * wb + 16 * b + ln];
        acc[0][b] = Mfma<T>::mma(a0, bv, acc[0][b]);
        acc[1][b] = Mfma<T>::mma(a1, bv, acc[1][b]);
      }
    }
    __syncthreads();
  }
  const int nown_pad = g.nch * 64;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = chunk * 64 + 32 * wr + 16 * a + Mfma<T>::row(kq, v);
        const int box = B0 + 64 * wb + 16 * b + ln;
        if (row >= g.nown || box >= nlist) continue;
        if (ksplit == 1) {
          const size_t o = own_glob(g, boxes[box], row);
          z[o] = acc_mode ? z[o] + acc[a][b][v] : acc[a][b][v];
        } else {
          part[((size_t)kslice * nlist + box) * nown_pad + row] = acc[a][b][v];
        }
      }
}

// nloc x (boxes rounded up to 128): the gathered operand of the product
size_t int_gather_elems(const BoxGeom& g, int n_int) { return (size_t)g.nloc * (size_t)((n_int + 127) / 128 * 128); }

template <typename T>
void launch_ras_apply(const T* r, T* z, BoxGeom g, const T* inv, const int* ib_boxes, int n_ib,
                      const T* shared_inv, const int* int_boxes, int n_int, const int* loc_tab,
                      T* part, hipStream_t s, int parts, bool acc, int tb, T* xg, size_t xg_elems,
                      const SymIB* sym) {
  // slices of a split IB launch first in part, those of the interior product
  // after them; one sum launch finishes both (and the symmetric IB partials)
  const bool do_ib = (parts & 1) && n_ib > 0, do_int = (parts & 2) && n_int > 0;
  const bool use_sym = do_ib && sym != nullptr;
  const int ks_ib = do_ib && !use_sym ? ras_ib_ksplit(g, n_ib) : 1;
  const int ks_sym = use_sym ? ras_ib_ksplit(g, n_ib) : 1;
  const int ks_int = do_int ? ras_interior_ksplit(g, n_int) : 1;
  const size_t nown_pad = (size_t)g.nch * 64;
  T* ipart = part;
  T* tpart = part + (ks_ib > 1 ? (size_t)ks_ib * n_ib * nown_pad : 0);
  T* spart = use_sym ? static_cast<T*>(sym->part) : nullptr;
  if (use_sym) {
    if (g.nown % 64) throw Error(IBMG_ERR_ARG, "symmetric storage needs whole 64-row chunks");
    const size_t lds = ((((size_t)g.nloc + 3) & ~(size_t)3) + 256 + 64 * (size_t)(g.nch - 1)) * sizeof(T);
    IBMG_KLAUNCH((k_ras_ib_sym<T>), dim3(n_ib, g.nch, ks_sym), dim3(256), lds, s, r, g,
                 static_cast<const T*>(sym->inv), ib_boxes, sym->perm, spart);
    IBMG_LAUNCH_CHECK();
  } else if (do_ib) {
    const size_t lds = (((size_t)g.nloc + 3) & ~(size_t)3) * sizeof(T) + 256 * sizeof(T);
    IBMG_KLAUNCH((k_ras_ib<T>), dim3(n_ib, g.nch, ks_ib), dim3(256), lds, s, r, z, g, inv, ib_boxes, acc,
                       ipart);
    IBMG_LAUNCH_CHECK();
  }
  if (do_int) {
    const int ks = ks_int;
    if (tb == 128 && xg && xg_elems >= int_gather_elems(g, n_int)) {
      const int nbp = (n_int + 127) / 128 * 128;
      const size_t tot = (size_t)g.nloc * nbp;
      int grid = cdiv(tot, 256);
      if (grid > 8192) grid = 8192;
      IBMG_KLAUNCH((k_int_gather<T>), dim3(grid), dim3(256), 0, s, r, xg, g, int_boxes, n_int, nbp, loc_tab);
      IBMG_LAUNCH_CHECK();
      IBMG_KLAUNCH((k_int_gemm<T>), dim3(g.nch, nbp / 128, ks), dim3(256), 0, s, shared_inv, xg, z, g,
                         int_boxes, n_int, nbp, tpart, ks, acc);
    } else if (tb == kIntFormPipe) {
      const long long nwg = (long long)((n_int + 63) / 64) * g.nch * ks;
      if (nwg > 0x7fffffffLL) throw Error(IBMG_ERR_ARG, "interior product grid too large");
      IBMG_KLAUNCH((k_ras_interior_p<T>), dim3((unsigned)nwg), dim3(256), 0, s, r, z, g, shared_inv, int_boxes,
                   n_int, loc_tab, tpart, ks, acc);
    } else if (tb == 64)
      IBMG_KLAUNCH((k_ras_interior_g<T>), dim3((n_int + 63) / 64, g.nch, ks), dim3(256), 0, s, r, z, g,
                         shared_inv, int_boxes, n_int, loc_tab, tpart, ks, acc);
    else if (tb == 16)
      IBMG_KLAUNCH((k_ras_interior<T, 16>), dim3((n_int + 15) / 16, g.nch, ks), dim3(256), 0, s, r, z, g,
                         shared_inv, int_boxes, n_int, loc_tab, tpart, ks, acc);
    else
      IBMG_KLAUNCH((k_ras_interior<T, 32>), dim3((n_int + 31) / 32, g.nch, ks), dim3(256), 0, s, r, z, g,
                         shared_inv, int_boxes, n_int, loc_tab, tpart, ks, acc);
    IBMG_LAUNCH_CHECK();
  }
  const int na = ks_ib > 1 ? n_ib : 0, nb = ks_int > 1 ? n_int : 0, ns = use_sym ? n_ib : 0;
  if (na + nb + ns > 0) {
    int grid = cdiv((size_t)(na + nb + ns) * g.nown, 256);
    if (grid > 4096) grid = 4096;
    IBMG_KLAUNCH((k_ras_sum<T>), dim3(grid), dim3(256), 0, s, ipart, ib_boxes, na, ks_ib, tpart, int_boxes, nb,
                       ks_int, spart, ns, ks_sym, z, g, acc);
    IBMG_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// Summed additive Schwarz (the plain R_k^T combination).  First every box's
// whole local solution y_k = L_k^{-1} R_k r: a work-group per (box, 64-row
// chunk) streams that chunk of the box's full inverse as the IB-box kernel
// does (interior boxes share one inverse) and writes the 64 rows to
// Y[(box * nch + chunk) * 64 + row].  Then every unknown gathers its entries
// from the boxes whose index set holds it: no two work-groups write one
// unknown, and no atomics are needed.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_asm_local(const T* __restrict__ r, BoxGeom g, const T* __restrict__ inv,
                                                   const int* __restrict__ box_inv, T* __restrict__ Y) {
  extern __shared__ char smem_raw[];
  T* x = reinterpret_cast<T*>(smem_raw);
  T* part = x + ((g.nloc + 3) & ~3);
  const int pid = blockIdx.x, chunk = blockIdx.y;
  const T* Mc = inv + ((size_t)box_inv[pid] * g.nch + chunk) * g.nloc * 64;
  ras_ib_chunk<T, true>(r, nullptr, g, Mc, pid, chunk, x, part, false, 0, g.nloc,
                        Y + ((size_t)pid * g.nch + chunk) * 64);
}

// z[d] = sum of unknown d's entries over the boxes that hold it.  Along each
// axis the boxes holding a coordinate lie within reach (b + o) / b + 1 of its
// owner box (on levels with fewer boxes than that window, every box is
// tried); they are visited rows of boxes first, in increasing offset from
// the owner, a fixed order per unknown.
template <typename T>
__global__ void k_asm_gather(const T* __restrict__ Y, T* __restrict__ z, BoxGeom g) {
  const int N = g.N, m = g.m, nu = m * (m + 1), npd = g.npd;
  const size_t nn = (size_t)N * N, tot = 3 * nn;
  const int reach = (g.b + g.o) / g.b + 1;
  const bool every = 2 * reach + 1 >= npd;
  const int cnt = every ? npd : 2 * reach + 1;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int comp = (int)(t / nn);
    const size_t q = t - (size_t)comp * nn;
    const int i = (int)(q % N), j = (int)(q / N);
    const int ext_x = comp == 0 ? m + 1 : m, ext_y = comp == 1 ? m + 1 : m;
    const int ox = i / g.b, oy = j / g.b;
    T acc = 0;
    for (int ty = 0; ty < cnt; ++ty) {
      const int by = every ? ty : pmod(oy - reach + ty, npd);
      const int jj = pmod(j - (by * g.b - g.o), N);
      if (jj >= ext_y) continue;
      for (int tx = 0; tx < cnt; ++tx) {
        const int bx = every ? tx : pmod(ox - reach + tx, npd);
        const int ii = pmod(i - (bx * g.b - g.o), N);
        if (ii >= ext_x) continue;
        const int k = comp == 0 ? jj * (m + 1) + ii : (comp == 1 ? nu + jj * m + ii : 2 * nu + jj * m + ii);
        acc += Y[((size_t)(by * npd + bx) * g.nch + (k >> 6)) * 64 + (k & 63)];
      }
    }
    z[t] = acc;
  }
}

template <typename T>
void launch_asm_apply(const T* r, T* z, BoxGeom g, const T* inv, const int* box_inv, T* Y, hipStream_t s) {
  const int nbox = g.npd * g.npd;
  const size_t lds = (((size_t)g.nloc + 3) & ~(size_t)3) * sizeof(T) + 256 * sizeof(T);
  IBMG_KLAUNCH((k_asm_local<T>), dim3(nbox, g.nch), dim3(256), lds, s, r, g, inv, box_inv, Y);
  IBMG_LAUNCH_CHECK();
  const size_t tot = 3 * (size_t)g.N * g.N;
  int grid = cdiv(tot, 256);
  if (grid > 8192) grid = 8192;
  IBMG_KLAUNCH((k_asm_gather<T>), dim3(grid), dim3(256), 0, s, Y, z, g);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched RAS sweep: one persistent launch per sweep.  Items are interior
// tiles x row chunks (matrix cores, shared inverse) and (IB box, row chunk)
// pairs (streamed own inverses), interleaved evenly: item t is an IB item
// when floor((t + 1) B / total) > floor(t B / total), B = IB items, so every
// CU holds both kinds and the inverse streaming overlaps the products.
// Work-group w takes items w, w + grid, ...  Every item writes disjoint
// owned rows, so the result does not depend on the order.
// ---------------------------------------------------------------------------
template <typename T, int TB>
__global__ void __launch_bounds__(256) k_ras_batch(const T* __restrict__ r, T* __restrict__ z, BoxGeom g,
                                                   size_t sys_n, int nbox, const T* __restrict__ M,
                                                   const int* __restrict__ int_ents, int n_int,
                                                   const int* __restrict__ ib_ents, const T* const* __restrict__ ib_inv,
                                                   int n_ib, const int* __restrict__ loc_tab,
                                                   const int* __restrict__ active) {
  extern __shared__ char smem_raw[];
  const int n_tiles = (n_int + TB - 1) / TB;
  const long long int_items = (long long)n_tiles * g.nch;
  const long long ib_items = (long long)n_ib * g.nch;
  const long long total = int_items + ib_items;
  for (long long it = blockIdx.x; it < total; it += gridDim.x) {
    const long long before = it * ib_items / total;           // IB items among [0, it)
    const bool is_ib = (it + 1) * ib_items / total > before;
    if (!is_ib) {
      const int ti = (int)(it - before);
      if constexpr (TB == 64)
        ras_int_gemm<T>(r, z, g, sys_n, nbox, M, int_ents, n_int, ti / g.nch, ti % g.nch, 0, 1, loc_tab, active,
                        nullptr, *reinterpret_cast<GemmSmem<T>*>(smem_raw), false);
      else
        ras_int_tile<T, TB, false>(r, z, g, sys_n, nbox, M, int_ents, n_int, ti / g.nch, ti % g.nch, 0, 1,
                                   loc_tab, active, nullptr, *reinterpret_cast<IntTileSmem<T, TB>*>(smem_raw),
                                   false);
    } else {
      const int q = (int)before, e = q / g.nch, c = q % g.nch;
      const int ent = ib_ents[e], sy = ent / nbox;
      if (active && !active[sy]) continue;
      T* x = reinterpret_cast<T*>(smem_raw);
      ras_ib_chunk<T, false>(r + (size_t)sy * sys_n, z + (size_t)sy * sys_n, g,
                             ib_inv[e] + (size_t)c * g.nloc * 64, ent - sy * nbox, c, x,
                             x + ((g.nloc + 3) & ~3), false, 0, g.nloc, nullptr);
    }
    __syncthreads();
  }
}

int ras_batch_items(const BoxGeom& g, int n_int, int n_ib, int tb) {
  return ((n_int + tb - 1) / tb) * g.nch + n_ib * g.nch;
}

template <typename T>
void launch_ras_batch(const T* r, T* z, BoxGeom g, size_t sys_n, int nbox, const T* shared_inv,
                      const int* int_ents, int n_int, const int* ib_ents, const T* const* ib_inv, int n_ib,
                      const int* loc_tab, const int* active, RasBatchPlan plan, hipStream_t s) {
  const int tb = plan.tb == 16 ? 16 : (plan.tb == 64 ? 64 : 32);
  const int items = ras_batch_items(g, n_int, n_ib, tb);
  if (items <= 0) return;
  if (n_int > 0 && !shared_inv) throw Error(IBMG_ERR_ARG, "interior boxes without a shared inverse");
  int grid = plan.grid > 0 ? plan.grid : items;
  if (grid > items) grid = items;
  size_t lds = ((((size_t)g.nloc + 3) & ~(size_t)3) + 256) * sizeof(T);
  const size_t tile = tb == 16 ? sizeof(IntTileSmem<T, 16>)
                                : (tb == 64 ? sizeof(GemmSmem<T>) : sizeof(IntTileSmem<T, 32>));
  if (tile > lds) lds = tile;
  if (tb == 16)
    IBMG_KLAUNCH((k_ras_batch<T, 16>), dim3(grid), dim3(256), lds, s, r, z, g, sys_n, nbox, shared_inv,
                       int_ents, n_int, ib_ents, ib_inv, n_ib, loc_tab, active);
  else if (tb == 64)
    IBMG_KLAUNCH((k_ras_batch<T, 64>), dim3(grid), dim3(256), lds, s, r, z, g, sys_n, nbox, shared_inv,
                       int_ents, n_int, ib_ents, ib_inv, n_ib, loc_tab, active);
  else
    IBMG_KLAUNCH((k_ras_batch<T, 32>), dim3(grid), dim3(256), lds, s, r, z, g, sys_n, nbox, shared_inv,
                       int_ents, n_int, ib_ents, ib_inv, n_ib, loc_tab, active);
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
    for (int k = tv.ptr[q]; k < tv.ptr[q + 1]; ++k) Ar[tv.col[k]] += tv.val[k];
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
  IBMG_KLAUNCH(k_coarse_assemble, dim3(cdiv(nn, 64)), dim3(64), 0, s, N, c, tu, tv, nb, aug);
  IBMG_LAUNCH_CHECK();
}

// Gauss-Jordan with partial pivoting on [A | I] in one work-group of 1024
// threads.  Per pivot: the column's largest magnitude (ties to the lower
// row) by a butterfly within each wave and one pass over the 16 wave
// results; the row swap; the scaled pivot row and the column's factors
// staged in LDS; then the elimination over the whole matrix as one flat
// loop, so each thread keeps several independent loads in flight.
__global__ void __launch_bounds__(1024) k_coarse_invert(double* __restrict__ aug, int nn, size_t stride) {
  __shared__ double wmax[16];
  __shared__ int wimax[16];
  __shared__ double fac[1024];
  __shared__ double rowk[2048];   // the scaled pivot row (2 nn <= 2048)
  aug += blockIdx.x * stride;     // one system per work-group
  const int ld = 2 * nn;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  for (int k = 0; k < nn; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < nn; i += nt) {
      const double a = fabs(aug[(size_t)i * ld + k]);
      if (a > best) { best = a; bi = i; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (o > best || (o == best && oi < bi)) { best = o; bi = oi; }
    }
    if (lane == 0) {
      wmax[wave] = best;
      wimax[wave] = bi;
    }
    __syncthreads();
    double bv = wmax[0];
    int p = wimax[0];
    for (int q = 1; q < (nt >> 6); ++q) {
      const double o = wmax[q];
      const int oi = wimax[q];
      if (o > bv || (o == bv && oi < p)) { bv = o; p = oi; }
    }
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
    for (int j = tid; j < ld; j += nt) {
      const double v = aug[(size_t)k * ld + j] * ip;
      aug[(size_t)k * ld + j] = v;
      rowk[j] = v;
    }
    for (int i = tid; i < nn; i += nt) fac[i] = aug[(size_t)i * ld + k];
    __syncthreads();
    const int tot = nn * ld;
#pragma unroll 8
    for (int t = tid; t < tot; t += nt) {
      const int i = t / ld, j = t - i * ld;
      if (i != k) aug[(size_t)i * ld + j] -= fac[i] * rowk[j];
    }
    __syncthreads();
  }
}

void launch_coarse_invert(double* aug, int nn, int count, size_t stride, hipStream_t s) {
  if (nn > 1024) throw Error(IBMG_ERR_ARG, "coarsest system too large for one work-group");
  if (count < 1) return;
  IBMG_KLAUNCH(k_coarse_invert, dim3(count), dim3(1024), 0, s, aug, nn, stride);
  IBMG_LAUNCH_CHECK();
}

__global__ void k_coarse_extract(const double* __restrict__ aug, int nn, int n0, double* __restrict__ inv) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 * n0) return;
  const int i = t / n0, j = t % n0;
  inv[t] = aug[(size_t)i * 2 * nn + nn + j];
}

void launch_coarse_extract(const double* aug, int nn, int n0, double* inv, hipStream_t s) {
  IBMG_KLAUNCH(k_coarse_extract, dim3(cdiv((size_t)n0 * n0, 256)), dim3(256), 0, s, aug, nn, n0, inv);
  IBMG_LAUNCH_CHECK();
}

// z = inv r on the coarsest level, FP64 arithmetic whatever T is: one wave
// per row, the lanes reading the row (and r) contiguously, then a butterfly
// over the wave.
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_apply(const double* __restrict__ inv, int n0,
                                                      const T* __restrict__ r, T* __restrict__ z) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n0) return;
  // batched: system blockIdx.y, inverses n0^2 and vectors n0 apart
  inv += (size_t)blockIdx.y * n0 * n0;
  r += (size_t)blockIdx.y * n0;
  z += (size_t)blockIdx.y * n0;
  const double* row = inv + (size_t)i * n0;
  double a = 0.0;
  for (int j = lane; j < n0; j += 64) a += row[j] * (double)r[j];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
  if (lane == 0) z[i] = (T)a;
}

template <typename T>
void launch_coarse_apply_batch(const double* inv, int n0, const T* r, T* z, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH((k_coarse_apply<T>), dim3(cdiv(n0, 4), nsys), dim3(256), 0, s, inv, n0, r, z);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_coarse_apply(const double* inv, int n0, const T* r, T* z, hipStream_t s) {
  launch_coarse_apply_batch<T>(inv, n0, r, z, 1, s);
}

template void launch_extract_owned<double>(const double*, int, BoxGeom, double*, hipStream_t, bool);
template void launch_extract_owned<float>(const double*, int, BoxGeom, float*, hipStream_t, bool);
template void launch_asm_apply<double>(const double*, double*, BoxGeom, const double*, const int*, double*,
                                       hipStream_t);
template void launch_asm_apply<float>(const float*, float*, BoxGeom, const float*, const int*, float*, hipStream_t);
template void launch_ras_apply<double>(const double*, double*, BoxGeom, const double*, const int*, int,
                                       const double*, const int*, int, const int*, double*,
                                       hipStream_t, int, bool, int, double*, size_t, const SymIB*);
template void launch_ras_apply<float>(const float*, float*, BoxGeom, const float*, const int*, int,
                                      const float*, const int*, int, const int*, float*,
                                      hipStream_t, int, bool, int, float*, size_t, const SymIB*);
template void launch_extract_sym<double>(const double*, int, BoxGeom, const int*, double*, hipStream_t);
template void launch_extract_sym<float>(const double*, int, BoxGeom, const int*, float*, hipStream_t);
template void launch_coarse_apply<double>(const double*, int, const double*, double*, hipStream_t);
template void launch_coarse_apply<float>(const double*, int, const float*, float*, hipStream_t);
template void launch_coarse_apply_batch<double>(const double*, int, const double*, double*, int, hipStream_t);
template void launch_coarse_apply_batch<float>(const double*, int, const float*, float*, int, hipStream_t);
template void launch_ras_batch<double>(const double*, double*, BoxGeom, size_t, int, const double*, const int*,
                                       int, const int*, const double* const*, int, const int*, const int*,
                                       RasBatchPlan, hipStream_t);
template void launch_ras_batch<float>(const float*, float*, BoxGeom, size_t, int, const float*, const int*, int,
                                      const int*, const float* const*, int, const int*, const int*, RasBatchPlan,
                                      hipStream_t);

}  // namespace ibmg
