// Fused Gram-Schmidt and small least-squares kernels of the FGMRES iterations
// (outer solve and Sec. 3.3 smoothing).
//
// Classical Gram-Schmidt applied twice to t against V[0..k):
//   launch_dots        partial dots V_q . t                      (pass 1)
//   launch_upd_dots    h = sum partials; t -= V h; partial V_q . t (pass 2)
//   launch_upd_norm    h2 = sum partials; t -= V h2; partial |t|^2
//   launch_scale_red   |t| = sqrt(sum partials); v = t / |t|
// A consumer kernel reduces its producer's per-block partials itself, every
// block in the same fixed order, so the result is deterministic and no
// cross-block synchronisation or atomics are needed; block 0 also records the
// Hessenberg entries.
//
// Batched launches take the system from blockIdx.y: vectors are segments of
// a batch vector (BSeg), and partial sums, Hessenberg columns and norms sit
// at fixed per-system strides; systems whose active flag is 0 are skipped.
#include "internal.hpp"

namespace ibmg {

namespace {

constexpr int kThreads = 256;

// out[q] = sum_b partial[b * k + q], q < k (out in shared memory), eight
// sums at a time in a fixed order.
__device__ void reduce_partials(const double* __restrict__ partial, int nblk, int k, double* out,
                                double* red) {
  const int tid = threadIdx.x;
  for (int q0 = 0; q0 < k; q0 += 8) {
    const int nq = k - q0 < 8 ? k - q0 : 8;
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = 0.0;
    for (int b = tid; b < nblk; b += kThreads) {
      const double* pb = partial + (size_t)b * k + q0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nq) a[q] += pb[q];
    }
    block_sums256<8>(a, nq, red, out + q0, tid);
  }
}

// per-block partial sums of up to 8 products at a time, written as
// partial[blockIdx.x * k + q]
template <typename T>
__device__ void block_dots(const T* __restrict__ V, int k, size_t stride, const T* t, size_t n,
                           double* __restrict__ partial, double* red) {
  const int tid = threadIdx.x;
  for (int v0 = 0; v0 < k; v0 += 8) {
    const int nv = k - v0 < 8 ? k - v0 : 8;
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
#pragma unroll 4
    for (size_t i = blockIdx.x * (size_t)kThreads + tid; i < n; i += (size_t)gridDim.x * kThreads) {
      const double ti = (double)t[i];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nv) acc[q] += (double)V[(size_t)(v0 + q) * stride + i] * ti;
    }
    block_sums256<8>(acc, nv, red, partial + (size_t)blockIdx.x * k + v0, tid);
  }
}

}  // namespace

// t -= V h (h from pass-1 partials, stored into hcol by block 0), then the
// pass-2 partial dots of the updated t.  with_norm (k <= 8): each block's
// partials also carry |t|^2 of the updated t after its k dots (k + 1 values
// per block).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_upd_dots(T* t, const T* __restrict__ V, int k, size_t stride,
                                                       BSeg sg, const double* __restrict__ pin, int nblk_in,
                                                       size_t pstride, double* __restrict__ hcol,
                                                       size_t hstride, double* __restrict__ pout, bool with_norm) {
  __shared__ double red[36];
  __shared__ double h[64];
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  t += o;
  V += o;
  pin += sy * pstride;
  pout += sy * pstride;
  hcol += sy * hstride;
  reduce_partials(pin, nblk_in, k, h, red);
  if (blockIdx.x == 0 && threadIdx.x < k) hcol[threadIdx.x] = h[threadIdx.x];
  if (k <= 8) {
    // one pass: each basis value feeds the update and then the pass-2 dot
    // of the updated entry; every thread visits its entries in the order
    // block_dots would, so the sums are those of the two-pass form
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    double nn = 0.0;
#pragma unroll 2
    for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
      double vq[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) vq[q] = q < k ? (double)V[(size_t)q * stride + i] : 0.0;
      double a = (double)t[i];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < k) a -= h[q] * vq[q];
      const T tn = (T)a;
      t[i] = tn;
      const double ti = (double)tn;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < k) acc[q] += vq[q] * ti;
      nn += ti * ti;
    }
    if (with_norm) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
        if (q == k) acc[q] = nn;
      block_sums256<9>(acc, k + 1, red, pout + (size_t)blockIdx.x * (k + 1), threadIdx.x);
    } else {
      block_sums256<9>(acc, k, red, pout + (size_t)blockIdx.x * k, threadIdx.x);
    }
    return;
  }
#pragma unroll 4
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    double a = (double)t[i];
    for (int q = 0; q < k; ++q) a -= h[q] * (double)V[(size_t)q * stride + i];
    t[i] = (T)a;
  }
  __syncthreads();
  block_dots<T>(V, k, stride, t, n, pout, red);
}

// t -= V h2 (h2 from pass-2 partials, added into hcol by block 0), then the
// partial sums of |t|^2.  store = false leaves t as it was and only forms
// the norm's partial sums (the last basis vector of a smoothing step is
// never read: its norm alone enters the Hessenberg matrix).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_upd_norm(T* t, const T* __restrict__ V, int k, size_t stride,
                                                       BSeg sg, const double* __restrict__ pin, int nblk_in,
                                                       size_t pstride, double* __restrict__ hcol,
                                                       size_t hstride, double* __restrict__ pout, bool store) {
  __shared__ double red[32];
  __shared__ double h[64];
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  t += o;
  V += o;
  pin += sy * pstride;
  pout += sy * pstride;
  hcol += sy * hstride;
  reduce_partials(pin, nblk_in, k, h, red);
  if (blockIdx.x == 0 && threadIdx.x < k) hcol[threadIdx.x] += h[threadIdx.x];
  double acc = 0.0;
#pragma unroll 4
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    double a = (double)t[i];
    for (int q = 0; q < k; ++q) a -= h[q] * (double)V[(size_t)q * stride + i];
    const T tn = (T)a;
    if (store) t[i] = tn;
    acc += (double)tn * (double)tn;
  }
  const double a1[1] = {acc};
  block_sums256<1>(a1, 1, red, pout + blockIdx.x, threadIdx.x);
}

// v = t / sqrt(sum partials) (v = 0 on an exact breakdown); block 0 stores the
// norm into *hout.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_scale_red(const T* t, T* v, BSeg sg,
                                                        const double* __restrict__ pin, int nblk_in,
                                                        size_t pstride, double* __restrict__ hout,
                                                        size_t hstride) {
  __shared__ double red[32];
  __shared__ double nrm;
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  t += o;
  v += o;
  pin += sy * pstride;
  hout += sy * hstride;
  reduce_partials(pin, nblk_in, 1, &nrm, red);
  const double d = sqrt(nrm);
  if (blockIdx.x == 0 && threadIdx.x == 0) hout[0] = d;
  const double inv = d != 0.0 ? 1.0 / d : 0.0;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    v[i] = (T)((double)t[i] * inv);
}

// The second Gram-Schmidt pass finished with the normalisation, from
// k_upd_dots' with_norm partials (h2 = V^T t and |t|^2, k + 1 per block):
// t2 = t - V h2, whose norm is sqrt(|t|^2 - |h2|^2) (t2 is orthogonal to the
// orthonormal V), and t = t2 / |t2| (0 on an exact breakdown); block 0 adds
// h2 into hcol[0..k) and stores |t2| into hcol[k].
template <typename T>
__global__ void __launch_bounds__(kThreads) k_scale_upd(T* t, const T* __restrict__ V, int k, size_t stride,
                                                        BSeg sg, const double* __restrict__ pin, int nblk_in,
                                                        size_t pstride, double* __restrict__ hcol,
                                                        size_t hstride) {
  __shared__ double red[32];
  __shared__ double h[64];
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  t += o;
  V += o;
  pin += sy * pstride;
  hcol += sy * hstride;
  reduce_partials(pin, nblk_in, k + 1, h, red);
  double hh = 0.0;
  for (int q = 0; q < k; ++q) hh += h[q] * h[q];
  const double r2 = h[k] - hh;
  const double d = r2 > 0.0 ? sqrt(r2) : 0.0;
  if (blockIdx.x == 0) {
    if (threadIdx.x < k) hcol[threadIdx.x] += h[threadIdx.x];
    if (threadIdx.x == 0) hcol[k] = d;
  }
  const double inv = d != 0.0 ? 1.0 / d : 0.0;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    double a = (double)t[i];
    for (int q = 0; q < k; ++q) a -= h[q] * (double)V[(size_t)q * stride + i];
    t[i] = (T)((double)(T)a * inv);
  }
}

// Least squares min || beta e1 - H y || ((k+1) x k Hessenberg, column-major,
// leading dimension ldh) by Givens rotations in every block, then
// x += sum_q y_q Z_q (assign: x = sum_q y_q Z_q, the same bits as adding to
// a zeroed x); block 0 stores y.  npart != null: the last subdiagonal entry
// H[k][k-1] is the square root of the nnblk partial sums there (reduced as
// k_scale_red reduces them; block 0 stores it into H).  pass2: npart holds
// instead k_upd_dots' with_norm partials of the last column (h2 and |t|^2,
// k + 1 per block): the column gains h2 and its subdiagonal entry is
// sqrt(|t|^2 - |h2|^2), as k_scale_upd forms it (H itself keeps the first
// pass's coefficients of that column: no block writes what others read).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_combine_ls(T* __restrict__ x, const T* __restrict__ Z, int k,
                                                         size_t stride, BSeg sg, double* __restrict__ H,
                                                         int ldh, size_t hstride, const double* __restrict__ beta,
                                                         double* __restrict__ yout, size_t sstride, bool assign,
                                                         const double* __restrict__ npart, int nnblk,
                                                         size_t pstride, bool pass2) {
  __shared__ double y[16];
  __shared__ double red[32];
  __shared__ double nrm;
  __shared__ double h2[17];
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  x += o;
  Z += o;
  H += sy * hstride;
  beta += sy * sstride;
  yout += sy * sstride;
  double hlast = 0.0;
  if (npart && pass2) {
    reduce_partials(npart + sy * pstride, nnblk, k + 1, h2, red);
    double hh = 0.0;
    for (int q = 0; q < k; ++q) hh += h2[q] * h2[q];
    const double r2 = h2[k] - hh;
    hlast = r2 > 0.0 ? sqrt(r2) : 0.0;
  } else if (npart) {
    reduce_partials(npart + sy * pstride, nnblk, 1, &nrm, red);
    hlast = sqrt(nrm);
    if (blockIdx.x == 0 && threadIdx.x == 0) H[k + (size_t)(k - 1) * ldh] = hlast;
  }
  if (threadIdx.x == 0) {
    double R[17][16];
    double g[17], cs[16], sn[16];
    for (int j = 0; j < k; ++j)
      for (int i = 0; i <= k; ++i) R[i][j] = H[i + (size_t)j * ldh];
    if (npart && pass2)
      for (int i = 0; i < k; ++i) R[i][k - 1] += h2[i];
    if (npart) R[k][k - 1] = hlast;
    for (int i = 0; i <= k; ++i) g[i] = 0.0;
    g[0] = beta[0];
    for (int j = 0; j < k; ++j) {
      for (int i = 0; i < j; ++i) {
        const double a = R[i][j], b = R[i + 1][j];
        R[i][j] = cs[i] * a + sn[i] * b;
        R[i + 1][j] = -sn[i] * a + cs[i] * b;
      }
      const double a = R[j][j], b = R[j + 1][j];
      const double d = sqrt(a * a + b * b);
      double c = 1.0, s = 0.0;
      if (d != 0.0) {
        c = a / d;
        s = b / d;
      }
      cs[j] = c;
      sn[j] = s;
      R[j][j] = d;
      R[j + 1][j] = 0.0;
      const double gj = g[j];
      g[j] = c * gj;
      g[j + 1] = -s * gj;
    }
    for (int j = k - 1; j >= 0; --j) {
      double a = g[j];
      for (int m = j + 1; m < k; ++m) a -= R[j][m] * y[m];
      y[j] = R[j][j] != 0.0 ? a / R[j][j] : 0.0;
    }
    if (blockIdx.x == 0)
      for (int j = 0; j < k; ++j) yout[j] = y[j];
  }
  __syncthreads();
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    double a = assign ? 0.0 : (double)x[i];
    for (int q = 0; q < k; ++q) a += y[q] * (double)Z[(size_t)q * stride + i];
    x[i] = (T)a;
  }
}

static int stream_blocks(size_t n) {
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 1024) g = 1024;
  return (int)(g < 1 ? 1 : g);
}

template <typename T>
void launch_upd_dots_b(T* t, const T* V, int k, size_t stride, BSeg sg, int nsys, const double* pin,
                       int nblk, size_t pstride, double* hcol, size_t hstride, double* pout, hipStream_t s,
                       int nblk_in, bool with_norm) {
  if (nsys <= 0) return;
  if (with_norm && (k < 1 || k > 8))
    throw Error(IBMG_ERR_ARG, "the norm-carrying second pass takes 1..8 basis vectors");
  IBMG_KLAUNCH((k_upd_dots<T>), dim3(nblk, nsys), dim3(kThreads), 0, s, t, V, k, stride, sg, pin,
                     nblk_in > 0 ? nblk_in : nblk, pstride, hcol, hstride, pout, with_norm);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_upd_norm_b(T* t, const T* V, int k, size_t stride, BSeg sg, int nsys, const double* pin,
                       int nblk, size_t pstride, double* hcol, size_t hstride, double* pout, hipStream_t s,
                       int nblk_in, bool store) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH((k_upd_norm<T>), dim3(nblk, nsys), dim3(kThreads), 0, s, t, V, k, stride, sg, pin,
                     nblk_in > 0 ? nblk_in : nblk, pstride, hcol, hstride, pout, store);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_scale_red_b(const T* t, T* v, BSeg sg, int nsys, size_t nmax, const double* pin, int nblk,
                        size_t pstride, double* hout, size_t hstride, hipStream_t s) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH((k_scale_red<T>), dim3(stream_blocks(nmax), nsys), dim3(kThreads), 0, s, t, v, sg, pin,
                     nblk, pstride, hout, hstride);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_combine_ls_b(T* x, const T* Z, int k, size_t stride, BSeg sg, int nsys, size_t nmax,
                         double* H, int ldh, size_t hstride, const double* beta, double* yout,
                         size_t sstride, hipStream_t s, bool assign, const double* npart, int nnblk,
                         size_t pstride, bool pass2) {
  if (nsys <= 0) return;
  if (k < 1 || k > 16 || (pass2 && !npart))
    throw Error(IBMG_ERR_ARG, "the smoothing least squares takes 1..16 columns");
  IBMG_KLAUNCH((k_combine_ls<T>), dim3(stream_blocks(nmax), nsys), dim3(kThreads), 0, s, x, Z, k, stride,
                     sg, H, ldh, hstride, beta, yout, sstride, assign, npart, nnblk, pstride, pass2);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_scale_upd_b(T* t, const T* V, int k, size_t stride, BSeg sg, int nsys, size_t nmax,
                        const double* pin, int nblk_in, size_t pstride, double* hcol, size_t hstride,
                        hipStream_t s) {
  if (nsys <= 0) return;
  if (k < 1 || k > 8) throw Error(IBMG_ERR_ARG, "the norm-carrying second pass takes 1..8 basis vectors");
  IBMG_KLAUNCH((k_scale_upd<T>), dim3(stream_blocks(nmax), nsys), dim3(kThreads), 0, s, t, V, k, stride, sg, pin,
               nblk_in, pstride, hcol, hstride);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_upd_dots(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk,
                     double* hcol, double* pout, hipStream_t s, int nblk_in) {
  launch_upd_dots_b<T>(t, V, k, stride, seg1(n), 1, pin, nblk, 0, hcol, 0, pout, s, nblk_in);
}

template <typename T>
void launch_upd_norm(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk,
                     double* hcol, double* pout, hipStream_t s, int nblk_in, bool store) {
  launch_upd_norm_b<T>(t, V, k, stride, seg1(n), 1, pin, nblk, 0, hcol, 0, pout, s, nblk_in, store);
}

template <typename T>
void launch_scale_red(const T* t, T* v, size_t n, const double* pin, int nblk, double* hout, hipStream_t s) {
  // nblk: blocks of the producer of pin
  launch_scale_red_b<T>(t, v, seg1(n), 1, n, pin, nblk, 0, hout, 0, s);
}

template <typename T>
void launch_combine_ls(T* x, const T* Z, int k, size_t stride, size_t n, double* H, int ldh,
                       const double* beta, double* yout, hipStream_t s, bool assign, const double* npart,
                       int nnblk, bool pass2) {
  launch_combine_ls_b<T>(x, Z, k, stride, seg1(n), 1, n, H, ldh, 0, beta, yout, 0, s, assign, npart, nnblk, 0,
                         pass2);
}

template <typename T>
void launch_upd_dots_n(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk,
                       double* hcol, double* pout, hipStream_t s, int nblk_in) {
  launch_upd_dots_b<T>(t, V, k, stride, seg1(n), 1, pin, nblk, 0, hcol, 0, pout, s, nblk_in, true);
}

template <typename T>
void launch_scale_upd(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk_in,
                      double* hcol, hipStream_t s) {
  launch_scale_upd_b<T>(t, V, k, stride, seg1(n), 1, n, pin, nblk_in, 0, hcol, 0, s);
}

#define IBMG_INST_KRY(T)                                                                               \
  template void launch_upd_dots<T>(T*, const T*, int, size_t, size_t, const double*, int, double*,     \
                                   double*, hipStream_t, int);                                         \
  template void launch_upd_norm<T>(T*, const T*, int, size_t, size_t, const double*, int, double*,     \
                                   double*, hipStream_t, int, bool);                                   \
  template void launch_scale_red<T>(const T*, T*, size_t, const double*, int, double*, hipStream_t);   \
  template void launch_combine_ls<T>(T*, const T*, int, size_t, size_t, double*, int, const double*,   \
                                     double*, hipStream_t, bool, const double*, int, bool);            \
  template void launch_upd_dots_n<T>(T*, const T*, int, size_t, size_t, const double*, int, double*,   \
                                     double*, hipStream_t, int);                                       \
  template void launch_scale_upd<T>(T*, const T*, int, size_t, size_t, const double*, int, double*,    \
                                    hipStream_t);                                                      \
  template void launch_upd_dots_b<T>(T*, const T*, int, size_t, BSeg, int, const double*, int, size_t, \
                                     double*, size_t, double*, hipStream_t, int, bool);                \
  template void launch_scale_upd_b<T>(T*, const T*, int, size_t, BSeg, int, size_t, const double*, int, \
                                      size_t, double*, size_t, hipStream_t);                           \
  template void launch_upd_norm_b<T>(T*, const T*, int, size_t, BSeg, int, const double*, int, size_t, \
                                     double*, size_t, double*, hipStream_t, int, bool);                \
  template void launch_scale_red_b<T>(const T*, T*, BSeg, int, size_t, const double*, int, size_t,     \
                                      double*, size_t, hipStream_t);                                   \
  template void launch_combine_ls_b<T>(T*, const T*, int, size_t, BSeg, int, size_t, double*, int,     \
                                       size_t, const double*, double*, size_t, hipStream_t, bool,      \
                                       const double*, int, size_t, bool);

IBMG_INST_KRY(double)
IBMG_INST_KRY(float)

}  // namespace ibmg
