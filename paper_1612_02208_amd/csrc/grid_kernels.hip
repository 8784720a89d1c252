// Grid kernels: the MAC Stokes-IB operator (Eq. matrix-impib, App. A.1), its
// transpose, the inter-level transfers (Sec. 3.2) and the BLAS-1 / small
// dense pieces of the Krylov iterations (Sec. 3.3 smoothing, outer FGMRES).
#include "internal.hpp"

namespace ibmg {

static inline int cdiv(size_t a, int b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// L_IB w (or its transpose, or the residual b - L_IB w).  A thread computes
// the x-face, y-face and cell rows of the indices (i, j) of its rows of one
// column:
//   y_u = alpha u - mu Lap u + (p_ij - p_{i-1,j}) / h + dt/h^2 (J^T K' J u)
//   y_v = alpha v - mu Lap v + (p_ij - p_{i,j-1}) / h + dt/h^2 (J^T K' J v)
//   y_p = -(u_{i+1,j} - u_ij + v_{i,j+1} - v_ij) / h
// The IB term arrives as the nodal forces F = K' J u (k_ib_force) and is
// gathered through the face -> (point, slot) lists, so no atomics are used.
// The transposed form evaluates -D^T p and G^T u directly; the IB block is
// the same J^T K' J chain with J standing in for S^T (S = J^* / h^2).
// ---------------------------------------------------------------------------
// Rows per thread: grids below 2048 keep one point per thread (their fields
// stay in the caches, and more waves hide the latency); larger grids march
// four rows per thread with the vertical neighbours carried in registers and
// store with non-temporal hints (fields of 100 MB and more do not stay in
// cache), which brings the stencil close to the rate of a plain copy.
constexpr int kStripMinN = 2048;
static inline int apply_rows(int N) { return N >= kStripMinN ? 4 : 1; }
// work-group shape: 64 x 4 points for one row per thread, a 256-wide run of
// one row's columns for the marching form
static inline dim3 apply_block(int rows) { return rows > 1 ? dim3(256, 1) : dim3(64, 4); }

template <int RJ, typename T>
__device__ __forceinline__ void store_out(T* p, T v) {
  if constexpr (RJ > 1) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Rows j0 .. j0+RJ-1 (those below N) of column i; emit(c0, y_u, y_v, y_p)
// receives each point's three rows.
template <typename T, bool TRANS, bool RESID, int IBM, int RJ, typename Emit>
__device__ __forceinline__ void apply_strip(const T* __restrict__ w, const T* __restrict__ b,
                                            const T* __restrict__ F, const T* __restrict__ Gib,
                                            const FootView<T>& fx, const FootView<T>& fy, int N, int M,
                                            const StokesCoef<T>& c, int i, int j0, Emit emit) {
  const size_t n = (size_t)N * N;
  const T* u = w;
  const T* v = w + n;
  const T* p = w + 2 * n;
  const int im = i == 0 ? N - 1 : i - 1;
  const int ip = i == N - 1 ? 0 : i + 1;
  const int jm0 = j0 == 0 ? N - 1 : j0 - 1;
  T ud = u[(size_t)jm0 * N + i], vd = v[(size_t)jm0 * N + i], pd = p[(size_t)jm0 * N + i];
  T uc = u[(size_t)j0 * N + i], vc = v[(size_t)j0 * N + i], pc = p[(size_t)j0 * N + i];
  // the precomputed Galerkin rows already carry the factor dt/h^2
  const T ibs = IBM == 2 ? T(1) : c.ibs;
#pragma unroll
  for (int r = 0; r < RJ; ++r) {
    const int j = j0 + r;
    if (j >= N) break;
    const int jp = j == N - 1 ? 0 : j + 1;
    const size_t row = (size_t)j * N, c0 = row + i;
    const size_t ct = (size_t)jp * N + i;
    const T ut = u[ct], vt = v[ct];
    const T ul = u[row + im], ur = u[row + ip], vl = v[row + im], vr = v[row + ip], pl = p[row + im];
    T ibu = 0, ibv = 0;
    if (IBM == 2) {
      ibu = Gib[c0];
      ibv = Gib[n + c0];
    } else if (IBM == 1) {
      const int a0 = fx.sp_ptr[c0], a1 = fx.sp_ptr[c0 + 1];
      for (int e = a0; e < a1; ++e) ibu += fx.sw[e] * F[fx.sp_ent[e] >> 4];
      const int b0 = fy.sp_ptr[c0], b1 = fy.sp_ptr[c0 + 1];
      for (int e = b0; e < b1; ++e) ibv += fy.sw[e] * F[M + (fy.sp_ent[e] >> 4)];
    }
    const T lapu = ul + ur + ud + ut - T(4) * uc;
    const T lapv = vl + vr + vd + vt - T(4) * vc;
    T yu, yv, yp;
    if (!TRANS) {
      yu = c.alpha * uc - c.beta * lapu + c.gi * (pc - pl) + ibs * ibu;
      yv = c.alpha * vc - c.beta * lapv + c.gi * (pc - pd) + ibs * ibv;
      yp = -c.gi * (ur - uc + vt - vc);
    } else {
      // (-D^T p) on the x-face (i, j): D maps the face to cells (i, j) with -1/h
      // and (i-1, j) with +1/h.  G^T u on cell (i, j): G maps the cell to faces
      // (i, j) with +1/h and (i+1, j) with -1/h (likewise in y).
      yu = c.alpha * uc - c.beta * lapu - c.gi * (pl - pc) + ibs * ibu;
      yv = c.alpha * vc - c.beta * lapv - c.gi * (pd - pc) + ibs * ibv;
      yp = c.gi * (uc - ur + vc - vt);
    }
    if (RESID) {
      yu = b[c0] - yu;
      yv = b[n + c0] - yv;
      yp = b[2 * n + c0] - yp;
    }
    emit(c0, yu, yv, yp);
    if (r + 1 < RJ) {
      ud = uc;
      vd = vc;
      pd = pc;
      uc = ut;
      vc = vt;
      pc = p[ct];
    }
  }
}

template <typename T, bool TRANS, bool RESID, int IBM, int RJ>
__global__ void __launch_bounds__(256) k_apply(const T* __restrict__ w, T* __restrict__ y,
                                               const T* __restrict__ b, const T* __restrict__ F,
                                               const T* __restrict__ Gib, FootView<T> fx,
                                               FootView<T> fy, int N, int M, StokesCoef<T> c,
                                               size_t bs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = (blockIdx.y * blockDim.y + threadIdx.y) * RJ;
  if (i >= N || j0 >= N) return;
  // batched launches: system blockIdx.z, systems bs apart
  w += blockIdx.z * bs;
  y += blockIdx.z * bs;
  if (RESID) b += blockIdx.z * bs;
  const size_t n = (size_t)N * N;
  apply_strip<T, TRANS, RESID, IBM, RJ>(w, b, F, Gib, fx, fy, N, M, c, i, j0, [&](size_t c0, T yu, T yv, T yp) {
    store_out<RJ>(y + c0, yu);
    store_out<RJ>(y + n + c0, yv);
    store_out<RJ>(y + 2 * n + c0, yp);
  });
}

// The same (non-transposed) with the first Gram-Schmidt dot products fused:
// partial[blk * nvec + q] = this block's sum of V_q . y over its rows
// (V = null: nvec = 1 and the sum of y . y), each thread's points summed in
// row order, then reduced over the block's four waves by shuffles and shared
// memory in a fixed order; blk = the block's linear index.
template <typename T, bool RESID, int IBM, int RJ>
__global__ void __launch_bounds__(256) k_apply_dots(const T* __restrict__ w, T* __restrict__ y,
                                                    const T* __restrict__ b, const T* __restrict__ F,
                                                    const T* __restrict__ Gib, FootView<T> fx, FootView<T> fy,
                                                    int N, int M, StokesCoef<T> c, const T* __restrict__ V,
                                                    int nvec, size_t vstride, double* __restrict__ partial) {
  __shared__ double red[9][4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j0 = (blockIdx.y * blockDim.y + threadIdx.y) * RJ;
  const bool live = i < N && j0 < N;
  const size_t n = (size_t)N * N;
  double d[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) d[q] = 0.0;
  if (live)
    apply_strip<T, false, RESID, IBM, RJ>(w, b, F, Gib, fx, fy, N, M, c, i, j0, [&](size_t c0, T yu, T yv, T yp) {
      store_out<RJ>(y + c0, yu);
      store_out<RJ>(y + n + c0, yv);
      store_out<RJ>(y + 2 * n + c0, yp);
      if (V) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
          if (q < nvec) {
            const T* vq = V + (size_t)q * vstride;
            d[q] += (double)vq[c0] * (double)yu + (double)vq[n + c0] * (double)yv + (double)vq[2 * n + c0] * (double)yp;
          }
      } else {
        d[0] += (double)yu * (double)yu + (double)yv * (double)yv + (double)yp * (double)yp;
      }
    });
  const int tid = threadIdx.y * blockDim.x + threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if (q >= nvec) break;
    double a = d[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) red[q][wave] = a;
  }
  __syncthreads();
  if (tid < nvec)
    partial[(size_t)(blockIdx.y * gridDim.x + blockIdx.x) * nvec + tid] =
        (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
}


template <typename T, int IBM, int RJ>
static void launch_apply_r(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx,
                           FootView<T> fy, int N, int M, StokesCoef<T> c, bool transpose,
                           hipStream_t s, int nsys, size_t bs) {
  const dim3 blk = apply_block(RJ);
  dim3 grd((N + blk.x - 1) / blk.x, (N + blk.y * RJ - 1) / (blk.y * RJ), nsys);
  if (b) {
    if (transpose)
      IBMG_KLAUNCH((k_apply<T, true, true, IBM, RJ>), grd, blk, 0, s, w, y, b, F, G, fx, fy, N, M, c, bs);
    else
      IBMG_KLAUNCH((k_apply<T, false, true, IBM, RJ>), grd, blk, 0, s, w, y, b, F, G, fx, fy, N, M, c, bs);
  } else {
    if (transpose)
      IBMG_KLAUNCH((k_apply<T, true, false, IBM, RJ>), grd, blk, 0, s, w, y, b, F, G, fx, fy, N, M, c, bs);
    else
      IBMG_KLAUNCH((k_apply<T, false, false, IBM, RJ>), grd, blk, 0, s, w, y, b, F, G, fx, fy, N, M, c, bs);
  }
  IBMG_LAUNCH_CHECK();
}

template <typename T, int IBM>
static void launch_apply_m(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx,
                           FootView<T> fy, int N, int M, StokesCoef<T> c, bool transpose,
                           hipStream_t s, int nsys = 1, size_t bs = 0) {
  if (apply_rows(N) == 4) launch_apply_r<T, IBM, 4>(w, y, b, F, G, fx, fy, N, M, c, transpose, s, nsys, bs);
  else launch_apply_r<T, IBM, 1>(w, y, b, F, G, fx, fy, N, M, c, transpose, s, nsys, bs);
}

// IB source: G (precomputed dt/h^2 J^T K' J u rows) if non-null, else the
// forces F gathered through the spreading lists if non-null, else none.
template <typename T>
void launch_apply(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx,
                  FootView<T> fy, int N, int M, StokesCoef<T> c, bool transpose, hipStream_t s) {
  if (G)
    launch_apply_m<T, 2>(w, y, b, F, G, fx, fy, N, M, c, transpose, s);
  else if (F)
    launch_apply_m<T, 1>(w, y, b, F, G, fx, fy, N, M, c, transpose, s);
  else
    launch_apply_m<T, 0>(w, y, b, F, G, fx, fy, N, M, c, transpose, s);
}

template <typename T, int IBM, int RJ>
static void launch_apply_dots_r(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx,
                                FootView<T> fy, int N, int M, StokesCoef<T> c, const T* V, int nvec,
                                size_t vstride, double* partial, hipStream_t s) {
  const dim3 blk = apply_block(RJ);
  dim3 grd((N + blk.x - 1) / blk.x, (N + blk.y * RJ - 1) / (blk.y * RJ));
  if (b)
    IBMG_KLAUNCH((k_apply_dots<T, true, IBM, RJ>), grd, blk, 0, s, w, y, b, F, G, fx, fy, N, M, c, V, nvec,
                       vstride, partial);
  else
    IBMG_KLAUNCH((k_apply_dots<T, false, IBM, RJ>), grd, blk, 0, s, w, y, b, F, G, fx, fy, N, M, c, V, nvec,
                       vstride, partial);
  IBMG_LAUNCH_CHECK();
}

template <typename T, int IBM>
static void launch_apply_dots_m(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx,
                                FootView<T> fy, int N, int M, StokesCoef<T> c, const T* V, int nvec,
                                size_t vstride, double* partial, hipStream_t s) {
  if (apply_rows(N) == 4) launch_apply_dots_r<T, IBM, 4>(w, y, b, F, G, fx, fy, N, M, c, V, nvec, vstride, partial, s);
  else launch_apply_dots_r<T, IBM, 1>(w, y, b, F, G, fx, fy, N, M, c, V, nvec, vstride, partial, s);
}

int apply_blocks(int N) {
  const int rj = apply_rows(N);
  const dim3 blk = apply_block(rj);
  const int rows = (int)blk.y * rj;
  return ((N + (int)blk.x - 1) / (int)blk.x) * ((N + rows - 1) / rows);
}

template <typename T>
void launch_apply_dots(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx, FootView<T> fy,
                       int N, int M, StokesCoef<T> c, const T* V, int nvec, size_t vstride, double* partial,
                       hipStream_t s) {
  if (nvec < 1 || nvec > 9) throw Error(IBMG_ERR_ARG, "fused dots take 1..9 vectors");
  if (G)
    launch_apply_dots_m<T, 2>(w, y, b, F, G, fx, fy, N, M, c, V, nvec, vstride, partial, s);
  else if (F)
    launch_apply_dots_m<T, 1>(w, y, b, F, G, fx, fy, N, M, c, V, nvec, vstride, partial, s);
  else
    launch_apply_dots_m<T, 0>(w, y, b, F, G, fx, fy, N, M, c, V, nvec, vstride, partial, s);
}

// Stencil part of L_IB (or the residual) for nsys systems of one grid size,
// bs apart; the IB rows are added by launch_ib_rows.
template <typename T>
void launch_apply_batch(const T* w, T* y, const T* b, int N, StokesCoef<T> c, int nsys, size_t bs,
                        hipStream_t s) {
  if (nsys <= 0) return;
  FootView<T> none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  launch_apply_m<T, 0>(w, y, b, nullptr, nullptr, none, none, N, 0, c, false, s, nsys, bs);
}

// Explicit IB rows: one wave per listed row, lanes over its entries, the
// wave's sum formed by shuffles in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) k_ib_rows(const T* __restrict__ x, T* __restrict__ y,
                                                 const int* __restrict__ rows, const int* __restrict__ ptr,
                                                 const int* __restrict__ col, const T* __restrict__ val,
                                                 int nrows, T sign) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (q >= nrows) return;
  T a = 0;
  for (int k = ptr[q] + lane; k < ptr[q + 1]; k += 64) a += val[k] * x[col[k]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if (lane == 0) y[rows[q]] += sign * a;
}

template <typename T>
void launch_ib_rows(const T* x, T* y, const int* rows, const int* ptr, const int* col, const T* val,
                    int nrows, T sign, hipStream_t s) {
  if (nrows <= 0) return;
  IBMG_KLAUNCH((k_ib_rows<T>), dim3(cdiv(nrows, 4)), dim3(256), 0, s, x, y, rows, ptr, col, val, nrows, sign);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Restriction (Sec. 3.2): R_u = P_u^T / 4 (adjoint of the Raviart-Thomas
// prolongation), R_p = mean of the four fine cells.  With partial (single
// system, 64 x 4 blocks) each block also stores the sum of squares of its
// coarse values at partial[block], the first norm the coarse level's
// smoother needs: a wave butterfly, then (w0 + w1) + (w2 + w3).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void restrict_point(const T* __restrict__ f, T* __restrict__ cz, int Nc, int i, int j,
                                               double& sq) {
  const int Nf = 2 * Nc;
  const size_t nf = (size_t)Nf * Nf, nc = (size_t)Nc * Nc;
  f += blockIdx.z * 3 * nf;
  cz += blockIdx.z * 3 * nc;
  auto at = [&](int comp, int I, int J) -> T {
    I = I < 0 ? I + Nf : (I >= Nf ? I - Nf : I);
    J = J < 0 ? J + Nf : (J >= Nf ? J - Nf : J);
    return f[comp * nf + (size_t)J * Nf + I];
  };
  const int I = 2 * i, J = 2 * j;
  const T ru = T(0.25) * (at(0, I, J) + at(0, I, J + 1)) +
               T(0.125) * (at(0, I - 1, J) + at(0, I - 1, J + 1) + at(0, I + 1, J) + at(0, I + 1, J + 1));
  const T rv = T(0.25) * (at(1, I, J) + at(1, I + 1, J)) +
               T(0.125) * (at(1, I, J - 1) + at(1, I + 1, J - 1) + at(1, I, J + 1) + at(1, I + 1, J + 1));
  const T rp = T(0.25) * (at(2, I, J) + at(2, I + 1, J) + at(2, I, J + 1) + at(2, I + 1, J + 1));
  const size_t o = (size_t)j * Nc + i;
  cz[o] = ru;
  cz[nc + o] = rv;
  cz[2 * nc + o] = rp;
  sq = (double)ru * (double)ru + (double)rv * (double)rv + (double)rp * (double)rp;
}

template <typename T>
__global__ void k_restrict(const T* __restrict__ f, T* __restrict__ cz, int Nc, double* __restrict__ partial) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  double sq = 0.0;
  if (i < Nc && j < Nc) restrict_point<T>(f, cz, Nc, i, j, sq);
  if (!partial) return;
  __shared__ double red[4];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
  if (lane == 0) red[wave] = sq;
  __syncthreads();
  if (tid == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
void launch_restrict_batch(const T* fine, T* coarse, int Nc, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  dim3 blk(64, 4);
  dim3 grd((Nc + 63) / 64, (Nc + 3) / 4, nsys);
  IBMG_KLAUNCH((k_restrict<T>), grd, blk, 0, s, fine, coarse, Nc, nullptr);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_restrict(const T* fine, T* coarse, int Nc, hipStream_t s) {
  launch_restrict_batch<T>(fine, coarse, Nc, 1, s);
}

int restrict_blocks(int Nc) { return ((Nc + 63) / 64) * ((Nc + 3) / 4); }

template <typename T>
void launch_restrict_norm(const T* fine, T* coarse, int Nc, double* partial, hipStream_t s) {
  dim3 blk(64, 4);
  dim3 grd((Nc + 63) / 64, (Nc + 3) / 4, 1);
  IBMG_KLAUNCH((k_restrict<T>), grd, blk, 0, s, fine, coarse, Nc, partial);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Prolongation and correction, fine += P e (Sec. 3.2): lowest-order
// Raviart-Thomas for velocity (linear across the face normal, constant along
// it), bilinear cell-centred interpolation for pressure.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_prolong_add(const T* __restrict__ cz, T* __restrict__ f, int Nc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  const int Nf = 2 * Nc;
  if (I >= Nf || J >= Nf) return;
  const size_t nf = (size_t)Nf * Nf, nc = (size_t)Nc * Nc;
  f += blockIdx.z * 3 * nf;
  cz += blockIdx.z * 3 * nc;
  auto at = [&](int comp, int i, int j) -> T {
    i = i < 0 ? i + Nc : (i >= Nc ? i - Nc : i);
    j = j < 0 ? j + Nc : (j >= Nc ? j - Nc : j);
    return cz[comp * nc + (size_t)j * Nc + i];
  };
  const int i = I >> 1, j = J >> 1;
  const T eu = (I & 1) ? T(0.5) * (at(0, i, j) + at(0, i + 1, j)) : at(0, i, j);
  const T ev = (J & 1) ? T(0.5) * (at(1, i, j) + at(1, i, j + 1)) : at(1, i, j);
  const int di = (I & 1) ? 1 : -1, dj = (J & 1) ? 1 : -1;
  const T ep = T(9.0 / 16.0) * at(2, i, j) + T(3.0 / 16.0) * (at(2, i + di, j) + at(2, i, j + dj)) +
               T(1.0 / 16.0) * at(2, i + di, j + dj);
  const size_t o = (size_t)J * Nf + I;
  f[o] += eu;
  f[nf + o] += ev;
  f[2 * nf + o] += ep;
}

template <typename T>
void launch_prolong_add_batch(const T* coarse, T* fine, int Nc, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  const int Nf = 2 * Nc;
  dim3 blk(64, 4);
  dim3 grd((Nf + 63) / 64, (Nf + 3) / 4, nsys);
  IBMG_KLAUNCH((k_prolong_add<T>), grd, blk, 0, s, coarse, fine, Nc);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_prolong_add(const T* coarse, T* fine, int Nc, hipStream_t s) {
  launch_prolong_add_batch<T>(coarse, fine, Nc, 1, s);
}

// ---------------------------------------------------------------------------
// Elementwise helpers.
// ---------------------------------------------------------------------------
template <typename Ts, typename Td>
__global__ void k_cast(const Ts* __restrict__ a, Td* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (Td)a[i];
}

template <typename Ts, typename Td>
void launch_cast(const Ts* a, Td* b, size_t n, hipStream_t s) {
  if (!n) return;
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_cast<Ts, Td>), dim3(g), dim3(256), 0, s, a, b, n);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_fill(T* a, T v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] = v;
}

template <typename T>
void launch_fill(T* a, T v, size_t n, hipStream_t s) {
  if (!n) return;
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_fill<T>), dim3(g), dim3(256), 0, s, a, v, n);
  IBMG_LAUNCH_CHECK();
}

// y += x
template <typename T>
__global__ void k_axpy(T* __restrict__ y, const T* __restrict__ x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] += x[i];
}

template <typename T>
void launch_axpy(T* y, const T* x, size_t n, hipStream_t s) {
  if (!n) return;
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_axpy<T>), dim3(g), dim3(256), 0, s, y, x, n);
  IBMG_LAUNCH_CHECK();
}

// *flag = 1 if any of a[0..n) is NaN or infinite (every writer stores the
// same value, so the unsynchronised stores need no ordering)
template <typename T>
__global__ void k_count_nonfinite(const T* __restrict__ a, size_t n, int* __restrict__ flag) {
  bool bad = false;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    bad = bad || !isfinite(a[i]);
  if (bad) *flag = 1;
}

template <typename T>
void launch_count_nonfinite(const T* a, size_t n, int* flag, hipStream_t s) {
  if (!n) return;
  int g = cdiv(n, 256 * 8);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  IBMG_KLAUNCH((k_count_nonfinite<T>), dim3(g), dim3(256), 0, s, a, n, flag);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Deterministic multi-dot: partial[blk * nvec + q] = sum over the block's
// grid-stride slice of V_q . t, accumulated in double; the finishing kernel
// adds the partials in a fixed tree order.  The grid size depends only on n.
// ---------------------------------------------------------------------------
int dots_blocks(size_t n, int cap) {
  int g = cdiv(n, 256 * 4);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return g;
}

template <typename T>
__global__ void __launch_bounds__(256) k_dots(const T* __restrict__ V, int nvec, size_t stride,
                                              const T* __restrict__ t, BSeg sg,
                                              double* __restrict__ partial, size_t pstride) {
  __shared__ double red[32];
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  V += o;
  t += o;
  partial += sy * pstride;
  const int tid = threadIdx.x;
  for (int v0 = 0; v0 < nvec; v0 += 8) {
    const int nv = nvec - v0 < 8 ? nvec - v0 : 8;
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
#pragma unroll 4
    for (size_t i = blockIdx.x * (size_t)256 + tid; i < n; i += (size_t)gridDim.x * 256) {
      const double ti = (double)t[i];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nv) acc[q] += (double)V[(size_t)(v0 + q) * stride + i] * ti;
    }
    block_sums256<8>(acc, nv, red, partial + (size_t)blockIdx.x * nvec + v0, tid);
  }
}

template <typename T>
void launch_dots_b(const T* V, int nvec, size_t stride, const T* t, BSeg sg, int nsys, double* partial,
                   size_t pstride, int nblk, hipStream_t s) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH((k_dots<T>), dim3(nblk, nsys), dim3(256), 0, s, V, nvec, stride, t, sg, partial, pstride);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_dots(const T* V, int nvec, size_t stride, const T* t, size_t n, double* partial,
                 int nblk, hipStream_t s) {
  launch_dots_b<T>(V, nvec, stride, t, seg1(n), 1, partial, 0, nblk, s);
}

// mode 0: out1 = s; mode 1: out1 = s, out2 += s; mode 2: out1 = sqrt(s) (and out2 = sqrt(s)).
// Batched: system blockIdx.x, partials pstride and outputs ostride apart.
__global__ void __launch_bounds__(256) k_dots_finish(const double* __restrict__ partial, int nvec,
                                                     int nblk, size_t pstride, double* out1, double* out2,
                                                     size_t ostride, int mode) {
  __shared__ double red[32];
  __shared__ double sums[8];
  const int tid = threadIdx.x;
  partial += blockIdx.x * pstride;
  out1 += blockIdx.x * ostride;
  if (out2) out2 += blockIdx.x * ostride;
  for (int q0 = 0; q0 < nvec; q0 += 8) {
    const int nq = nvec - q0 < 8 ? nvec - q0 : 8;
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = 0.0;
    for (int b = tid; b < nblk; b += 256) {
      const double* pb = partial + (size_t)b * nvec + q0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nq) a[q] += pb[q];
    }
    block_sums256<8>(a, nq, red, sums, tid);
    if (tid < nq) {
      const int q = q0 + tid;
      const double sres = sums[tid];
      if (mode == 0) {
        out1[q] = sres;
      } else if (mode == 1) {
        out1[q] = sres;
        out2[q] += sres;
      } else {
        const double r = sqrt(sres);
        out1[q] = r;
        if (out2) out2[q] = r;
      }
    }
    __syncthreads();
  }
}

void launch_dots_finish_b(const double* partial, int nvec, int nblk, size_t pstride, double* out1,
                          double* out2, size_t ostride, int mode, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH(k_dots_finish, dim3(nsys), dim3(256), 0, s, partial, nvec, nblk, pstride, out1, out2,
                     ostride, mode);
  IBMG_LAUNCH_CHECK();
}

void launch_dots_finish(const double* partial, int nvec, int nblk, double* out1, double* out2,
                        int mode, hipStream_t s) {
  launch_dots_finish_b(partial, nvec, nblk, 0, out1, out2, 0, mode, 1, s);
}

// t += sign * sum_q coef[q] V_q
template <typename T>
__global__ void k_update(T* __restrict__ t, const T* __restrict__ V, int nvec, size_t stride,
                         const double* __restrict__ coef, double sign, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double a = (double)t[i];
    for (int q = 0; q < nvec; ++q) a += sign * coef[q] * (double)V[(size_t)q * stride + i];
    t[i] = (T)a;
  }
}

template <typename T>
void launch_update(T* t, const T* V, int nvec, size_t stride, const double* coef, double sign,
                   size_t n, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 8192) g = 8192;
  IBMG_KLAUNCH((k_update<T>), dim3(g), dim3(256), 0, s, t, V, nvec, stride, coef, sign, n);
  IBMG_LAUNCH_CHECK();
}

// v = t / denom (v = 0 when denom == 0: an exact Krylov breakdown).
// Batched: system blockIdx.y, denominators dstride apart.
template <typename T>
__global__ void k_scale(const T* t, T* v, const double* __restrict__ denom, size_t dstride, BSeg sg) {
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  const double d = denom[sy * dstride];
  const double inv = d != 0.0 ? 1.0 / d : 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[o + i] = (T)((double)t[o + i] * inv);
}

template <typename T>
void launch_scale_b(const T* t, T* v, const double* denom, size_t dstride, BSeg sg, int nsys, size_t nmax,
                    hipStream_t s) {
  if (nsys <= 0) return;
  int g = cdiv(nmax, 256);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  IBMG_KLAUNCH((k_scale<T>), dim3(g, nsys), dim3(256), 0, s, t, v, denom, dstride, sg);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_scale(const T* t, T* v, const double* denom, size_t n, hipStream_t s) {
  launch_scale_b<T>(t, v, denom, 0, seg1(n), 1, n, s);
}

// x += sum_q y[q] Z_q, q < k (batched: k = kcnt[s] per system when kcnt is
// given, y ystride apart)
template <typename T>
__global__ void k_combine(T* __restrict__ x, const T* __restrict__ Z, int k, size_t stride,
                          const double* __restrict__ y, size_t ystride, const int* __restrict__ kcnt, BSeg sg) {
  const int sy = blockIdx.y;
  if (!seg_on(sg, sy)) return;
  const size_t o = seg_begin(sg, sy), n = seg_len(sg, sy);
  if (kcnt) k = kcnt[sy];
  y += sy * ystride;
  x += o;
  Z += o;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double a = (double)x[i];
    for (int q = 0; q < k; ++q) a += y[q] * (double)Z[(size_t)q * stride + i];
    x[i] = (T)a;
  }
}

template <typename T>
void launch_combine_b(T* x, const T* Z, size_t stride, const double* y, size_t ystride, const int* kcnt,
                      BSeg sg, int nsys, size_t nmax, hipStream_t s) {
  if (nsys <= 0) return;
  int g = cdiv(nmax, 256);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  IBMG_KLAUNCH((k_combine<T>), dim3(g, nsys), dim3(256), 0, s, x, Z, 0, stride, y, ystride, kcnt, sg);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_combine(T* x, const T* Z, int k, size_t stride, const double* y, size_t n, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 8192) g = 8192;
  IBMG_KLAUNCH((k_combine<T>), dim3(g, 1), dim3(256), 0, s, x, Z, k, stride, y, (size_t)0,
                     (const int*)nullptr, seg1(n));
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Least squares min || beta e1 - H y || for a (k+1) x k Hessenberg matrix
// (column-major, leading dimension ldh) by Givens rotations; k <= 16.
// Zero pivots (exact breakdown) give zero components.
// ---------------------------------------------------------------------------
__global__ void k_small_ls(const double* __restrict__ H, int ldh, int k, const double* __restrict__ beta,
                           double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double R[17][16];
  double g[17];
  double cs[16], sn[16];
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= k; ++i) R[i][j] = H[i + (size_t)j * ldh];
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
    if (d != 0.0) { c = a / d; s = b / d; }
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
}

void launch_small_ls(double* H, int ldh, int k, const double* beta, double* y, hipStream_t s) {
  IBMG_KLAUNCH(k_small_ls, dim3(1), dim3(64), 0, s, H, ldh, k, beta, y);
  IBMG_LAUNCH_CHECK();
}

// Outer FGMRES: rotate column k of H (rows 0..k+1) by the stored rotations,
// form rotation k, update g and write |g[k+1]| to res.  Batched: system
// blockIdx.x (H hstride apart; cs, sn, g rstride apart; res[s]), inactive
// systems untouched.
__global__ void k_givens(double* __restrict__ H, int ldh, size_t hstride, int k, double* __restrict__ cs,
                         double* __restrict__ sn, double* __restrict__ g, size_t rstride,
                         double* __restrict__ res, const int* __restrict__ active) {
  const int sy = blockIdx.x;
  if (threadIdx.x != 0 || (active && !active[sy])) return;
  H += sy * hstride;
  cs += sy * rstride;
  sn += sy * rstride;
  g += sy * rstride;
  double* col = H + (size_t)k * ldh;
  for (int i = 0; i < k; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[k], b = col[k + 1];
  const double d = sqrt(a * a + b * b);
  double c = 1.0, s = 0.0;
  if (d != 0.0) { c = a / d; s = b / d; }
  cs[k] = c;
  sn[k] = s;
  col[k] = d;
  col[k + 1] = 0.0;
  const double gk = g[k];
  g[k] = c * gk;
  g[k + 1] = -s * gk;
  res[sy] = fabs(g[k + 1]);
}

void launch_givens_b(double* H, int ldh, size_t hstride, int k, double* cs, double* sn, double* g,
                     size_t rstride, double* res, const int* active, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH(k_givens, dim3(nsys), dim3(64), 0, s, H, ldh, hstride, k, cs, sn, g, rstride, res, active);
  IBMG_LAUNCH_CHECK();
}

void launch_givens(double* H, int ldh, int k, double* cs, double* sn, double* g, double* res,
                   hipStream_t s) {
  launch_givens_b(H, ldh, 0, k, cs, sn, g, 0, res, nullptr, 1, s);
}

// y = R^{-1} g (R: the rotated k x k upper triangle); batched: k = kcnt[s].
__global__ void k_backsolve(const double* __restrict__ H, int ldh, size_t hstride, int k,
                            const int* __restrict__ kcnt, const double* __restrict__ g,
                            double* __restrict__ y, size_t rstride) {
  const int sy = blockIdx.x;
  if (threadIdx.x != 0) return;
  if (kcnt) k = kcnt[sy];
  H += sy * hstride;
  g += sy * rstride;
  y += sy * rstride;
  for (int j = k - 1; j >= 0; --j) {
    double a = g[j];
    for (int m = j + 1; m < k; ++m) a -= H[j + (size_t)m * ldh] * y[m];
    const double d = H[j + (size_t)j * ldh];
    y[j] = d != 0.0 ? a / d : 0.0;
  }
}

void launch_backsolve_b(const double* H, int ldh, size_t hstride, const int* kcnt, const double* g,
                        double* y, size_t rstride, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH(k_backsolve, dim3(nsys), dim3(64), 0, s, H, ldh, hstride, 0, kcnt, g, y, rstride);
  IBMG_LAUNCH_CHECK();
}

void launch_backsolve(const double* H, int ldh, int k, const double* g, double* y, hipStream_t s) {
  IBMG_KLAUNCH(k_backsolve, dim3(1), dim3(64), 0, s, H, ldh, (size_t)0, k, (const int*)nullptr, g, y,
                     (size_t)0);
  IBMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Block sums of a level vector (u, v, p) for the null-space projection.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_block_sums(const T* __restrict__ a, size_t nn,
                                                    double* __restrict__ partial, size_t bs, size_t pstride) {
  __shared__ double red[12];
  a += blockIdx.y * bs;
  partial += blockIdx.y * pstride;
  const int tid = threadIdx.x;
  double s0 = 0, s1 = 0, s2 = 0;
  for (size_t i = blockIdx.x * (size_t)256 + tid; i < nn; i += (size_t)gridDim.x * 256) {
    s0 += (double)a[i];
    s1 += (double)a[nn + i];
    s2 += (double)a[2 * nn + i];
  }
  const double v[3] = {s0, s1, s2};
  block_sums256<3>(v, 3, red, partial + (size_t)blockIdx.x * 3, tid);
}

template <typename T>
void launch_block_sums_b(const T* a, int N, size_t bs, double* partial, int nblk, size_t pstride, int nsys,
                         hipStream_t s) {
  if (nsys <= 0) return;
  IBMG_KLAUNCH((k_block_sums<T>), dim3(nblk, nsys), dim3(256), 0, s, a, (size_t)N * N, partial, bs,
                     pstride);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_block_sums(const T* a, int N, double* partial, int nblk, hipStream_t s) {
  launch_block_sums_b<T>(a, N, 0, partial, nblk, 0, 1, s);
}

template <typename T>
__global__ void k_subtract_means(T* __restrict__ a, size_t nn, const double* __restrict__ sums,
                                 int nvel, size_t bs, size_t sstride) {
  a += blockIdx.y * bs;
  sums += blockIdx.y * sstride;
  const double inv = 1.0 / (double)nn;
  const double m0 = nvel ? sums[0] * inv : 0.0;
  const double m1 = nvel ? sums[1] * inv : 0.0;
  const double m2 = sums[2] * inv;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x) {
    if (nvel) {
      a[i] = (T)((double)a[i] - m0);
      a[nn + i] = (T)((double)a[nn + i] - m1);
    }
    a[2 * nn + i] = (T)((double)a[2 * nn + i] - m2);
  }
}

template <typename T>
void launch_subtract_means_b(T* a, int N, size_t bs, const double* sums, size_t sstride, int nvel, int nsys,
                             hipStream_t s) {
  if (nsys <= 0) return;
  size_t nn = (size_t)N * N;
  int g = cdiv(nn, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_subtract_means<T>), dim3(g, nsys), dim3(256), 0, s, a, nn, sums, nvel, bs, sstride);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_subtract_means(T* a, int N, const double* sums, int nvel, hipStream_t s) {
  launch_subtract_means_b<T>(a, N, 0, sums, 0, nvel, 1, s);
}

// ---------------------------------------------------------------------------
// Explicit instantiations.
// ---------------------------------------------------------------------------
#define IBMG_INST_GRID(T)                                                                         \
  template void launch_apply<T>(const T*, T*, const T*, const T*, const T*, FootView<T>,          \
                                FootView<T>, int, int, StokesCoef<T>, bool, hipStream_t);         \
  template void launch_restrict<T>(const T*, T*, int, hipStream_t);                               \
  template void launch_restrict_norm<T>(const T*, T*, int, double*, hipStream_t);                 \
  template void launch_prolong_add<T>(const T*, T*, int, hipStream_t);                            \
  template void launch_fill<T>(T*, T, size_t, hipStream_t);                                       \
  template void launch_axpy<T>(T*, const T*, size_t, hipStream_t);                                \
  template void launch_count_nonfinite<T>(const T*, size_t, int*, hipStream_t);                   \
  template void launch_dots<T>(const T*, int, size_t, const T*, size_t, double*, int, hipStream_t); \
  template void launch_update<T>(T*, const T*, int, size_t, const double*, double, size_t,        \
                                 hipStream_t);                                                    \
  template void launch_scale<T>(const T*, T*, const double*, size_t, hipStream_t);                \
  template void launch_combine<T>(T*, const T*, int, size_t, const double*, size_t, hipStream_t); \
  template void launch_block_sums<T>(const T*, int, double*, int, hipStream_t);                   \
  template void launch_subtract_means<T>(T*, int, const double*, int, hipStream_t);               \
  template void launch_apply_dots<T>(const T*, T*, const T*, const T*, const T*, FootView<T>,     \
                                     FootView<T>, int, int, StokesCoef<T>, const T*, int, size_t,  \
                                     double*, hipStream_t);                                        \
  template void launch_apply_batch<T>(const T*, T*, const T*, int, StokesCoef<T>, int, size_t,    \
                                      hipStream_t);                                               \
  template void launch_ib_rows<T>(const T*, T*, const int*, const int*, const int*, const T*, int, \
                                  T, hipStream_t);                                                \
  template void launch_restrict_batch<T>(const T*, T*, int, int, hipStream_t);                    \
  template void launch_prolong_add_batch<T>(const T*, T*, int, int, hipStream_t);                 \
  template void launch_dots_b<T>(const T*, int, size_t, const T*, BSeg, int, double*, size_t, int, \
                                 hipStream_t);                                                    \
  template void launch_scale_b<T>(const T*, T*, const double*, size_t, BSeg, int, size_t,         \
                                  hipStream_t);                                                   \
  template void launch_combine_b<T>(T*, const T*, size_t, const double*, size_t, const int*, BSeg, \
                                    int, size_t, hipStream_t);                                    \
  template void launch_block_sums_b<T>(const T*, int, size_t, double*, int, size_t, int,          \
                                       hipStream_t);                                              \
  template void launch_subtract_means_b<T>(T*, int, size_t, const double*, size_t, int, int,      \
                                           hipStream_t);

IBMG_INST_GRID(double)
IBMG_INST_GRID(float)
template void launch_cast<double, float>(const double*, float*, size_t, hipStream_t);
template void launch_cast<float, double>(const float*, double*, size_t, hipStream_t);
template void launch_cast<double, double>(const double*, double*, size_t, hipStream_t);
template void launch_fill<int>(int*, int, size_t, hipStream_t);

}  // namespace ibmg
