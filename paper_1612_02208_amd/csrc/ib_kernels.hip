// Immersed-boundary kernels: Peskin four-point weights (App. A.3), their
// Galerkin coarsening through the velocity prolongation (Sec. 3.1-3.2),
// interpolation J_h, spreading S_h = J_h^T / h^2 with unit nodal weights,
// the spring operator K' = sum_e B_e^T B_e (x) K_e with K_e = kappa_e I for
// zero-rest-length fibres (Sec. 5, App. A.2) or the 2x2 tangent block of a
// spring with a rest length (the linearised force of Sec. 6), the explicit
// Galerkin IB operator rows used to assemble dense box and coarsest-level
// matrices (columns over the level's [u | v] vector), and the stiffness
// gradient.
//
// Spreading is a gather: every face walks the (point, slot) entries sorted
// by face at set-up, so results are deterministic and use no atomics.
#include <mutex>

#include "internal.hpp"

namespace ibmg {

static inline int cdiv(size_t a, int b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ double phi4(double r) {
  const double a = fabs(r);
  if (a < 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a < 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

__device__ __forceinline__ int wrapi(int a, int N) { return a >= N ? a - N : a; }

// periodic difference t - k folded into (-N/2, N/2]
__device__ __forceinline__ double pdiff(double t, int k, int N) {
  double d = t - (double)k;
  if (d > 0.5 * N) d -= N;
  if (d <= -0.5 * N) d += N;
  return d;
}

// Finest-level weights phi(rx) phi(ry) on the 4 x 4 window (masked slots 0).
__global__ void k_fp_fine(const double* __restrict__ X, int M, int N, int comp,
                          const int* __restrict__ base, const int* __restrict__ mask,
                          double* __restrict__ w) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  const double sx = comp == 0 ? 0.0 : 0.5;
  const double sy = comp == 0 ? 0.5 : 0.0;
  const double tx = X[2 * l] * N - sx;
  const double ty = X[2 * l + 1] * N - sy;
  const int i0 = base[2 * l], j0 = base[2 * l + 1];
  const int mk = mask[l];
  double wx[4], wy[4];
  for (int a = 0; a < 4; ++a) {
    wx[a] = phi4(pdiff(tx, i0 + a, N));
    wy[a] = phi4(pdiff(ty, j0 + a, N));
  }
  for (int s = 0; s < 16; ++s)
    w[(size_t)l * 16 + s] = ((mk >> s) & 1) ? wx[s & 3] * wy[s >> 2] : 0.0;
}

void launch_fp_fine(const double* X, int M, int N, int comp, const int* base, const int* mask,
                    double* w, hipStream_t s) {
  if (!M) return;
  IBMG_KLAUNCH(k_fp_fine, dim3(cdiv(M, 128)), dim3(128), 0, s, X, M, N, comp, base, mask, w);
  IBMG_LAUNCH_CHECK();
}

// Coarse weights J_l = J_{l+1} P_u: every fine slot (I, J) is pushed to the
// coarse faces that P_u interpolates it from -- along the face normal an
// even fine index copies coarse I/2 and an odd one averages (I-1)/2 and
// (I+1)/2; tangentially the coarse index is floor(I/2).
__global__ void k_fp_coarsen(const int* __restrict__ fbase, const double* __restrict__ fw,
                             const int* __restrict__ cbase, int M, int comp,
                             double* __restrict__ cw) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  const int I0 = fbase[2 * l], J0 = fbase[2 * l + 1];
  const int ci0 = I0 >> 1, cj0 = J0 >> 1;
  double acc[16];
  for (int s = 0; s < 16; ++s) acc[s] = 0.0;
  for (int s = 0; s < 16; ++s) {
    const double wf = fw[(size_t)l * 16 + s];
    if (wf == 0.0) continue;
    const int I = I0 + (s & 3), J = J0 + (s >> 2);
    if (comp == 0) {
      const int cj = (J >> 1) - cj0;
      if ((I & 1) == 0) {
        acc[cj * 4 + ((I >> 1) - ci0)] += wf;
      } else {
        acc[cj * 4 + ((I - 1) / 2 - ci0)] += 0.5 * wf;
        acc[cj * 4 + ((I + 1) / 2 - ci0)] += 0.5 * wf;
      }
    } else {
      const int ci = (I >> 1) - ci0;
      if ((J & 1) == 0) {
        acc[((J >> 1) - cj0) * 4 + ci] += wf;
      } else {
        acc[((J - 1) / 2 - cj0) * 4 + ci] += 0.5 * wf;
        acc[((J + 1) / 2 - cj0) * 4 + ci] += 0.5 * wf;
      }
    }
  }
  (void)cbase;
  for (int s = 0; s < 16; ++s) cw[(size_t)l * 16 + s] = acc[s];
}

template <typename T>
__global__ void k_gather_weights(const double* __restrict__ w, const int* __restrict__ ent, size_t n,
                                 T* __restrict__ sw) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    sw[e] = (T)w[ent[e]];
}

template <typename T>
void launch_gather_weights(const double* w, const int* ent, size_t n, T* sw, hipStream_t s) {
  if (!n) return;
  const int g = (int)std::min<size_t>((n + 255) / 256, 65536);
  IBMG_KLAUNCH((k_gather_weights<T>), dim3(g), dim3(256), 0, s, w, ent, n, sw);
  IBMG_LAUNCH_CHECK();
}
template void launch_gather_weights<double>(const double*, const int*, size_t, double*, hipStream_t);
template void launch_gather_weights<float>(const double*, const int*, size_t, float*, hipStream_t);

void launch_fp_coarsen(const int* fbase, const double* fw, const int* cbase, int M, int comp,
                       int Nf, int Nc, double* cw, hipStream_t s) {
  (void)Nf;
  (void)Nc;
  if (!M) return;
  IBMG_KLAUNCH(k_fp_coarsen, dim3(cdiv(M, 128)), dim3(128), 0, s, fbase, fw, cbase, M, comp, cw);
  IBMG_LAUNCH_CHECK();
}

// (J u)_l for every point, both components: 8 lanes per point, lane
// 4 c + b taking row b of component c's 4 x 4 window (its four weights are
// contiguous; masked slots carry weight 0), the row sums added by shuffles in
// a fixed order.  Points are taken in cell order (f.order), so neighbouring
// lane groups read neighbouring faces, and their bases and weights are read
// from copies laid out in that order (obase, ow), so those reads are
// contiguous.  Output interleaved U[2 l + c]: a point's two values are
// stored side by side.
template <typename T>
__global__ void __launch_bounds__(256) k_interp_lanes(const T* __restrict__ u, const T* __restrict__ v,
                                                      FootView<T> fx, FootView<T> fy, int M, int N,
                                                      T* __restrict__ U) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int g = (int)(t / 8), comp = (int)(t / 4) & 1, b = (int)(t % 4);
  const bool live = g < M;
  T a = 0;
  int l = 0;
  if (live) {
    const FootView<T>& f = comp ? fy : fx;
    l = fx.order[g];
    const T* src = comp ? v : u;
    const int i0 = f.obase[2 * g];
    const T* row = src + (size_t)wrapi(f.obase[2 * g + 1] + b, N) * N;
    const T* w = f.ow + (size_t)g * 16 + 4 * b;
#pragma unroll
    for (int q = 0; q < 4; ++q) a += w[q] * row[wrapi(i0 + q, N)];
  }
  a += __shfl_xor(a, 1, 4);
  a += __shfl_xor(a, 2, 4);
  if (live && b == 0) U[2 * (size_t)l + comp] = a;
}

template <typename T>
__global__ void k_walk_order(const int* __restrict__ order, const int* __restrict__ base, const T* __restrict__ w,
                             int M, int* __restrict__ obase, T* __restrict__ ow) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= (size_t)M * 16) return;
  const int g = (int)(t / 16), s = (int)(t % 16);
  const int l = order[g];
  ow[t] = w[(size_t)l * 16 + s];
  if (s < 2) obase[2 * (size_t)g + s] = base[2 * (size_t)l + s];
}

template <typename T>
void launch_walk_order(const int* order, const int* base, const T* w, int M, int* obase, T* ow, hipStream_t s) {
  if (!M) return;
  IBMG_KLAUNCH((k_walk_order<T>), dim3(cdiv((size_t)M * 16, 256)), dim3(256), 0, s, order, base, w, M, obase, ow);
  IBMG_LAUNCH_CHECK();
}
template void launch_walk_order<double>(const int*, const int*, const double*, int, int*, double*, hipStream_t);
template void launch_walk_order<float>(const int*, const int*, const float*, int, int*, float*, hipStream_t);

// F_l = sum over springs e at l of K_e (U_l - U_{other end}), from U = J u
// (interleaved [M][2]); F is planar [2][M].  K_e = kappa_e I, or the tangent
// block when sv.adj_k2 is set.
template <typename T>
__global__ void k_spring_force(const T* __restrict__ U, SpringView<T> sv, T* __restrict__ F) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= sv.M) return;
  const int M = sv.M;
  const T U0 = U[2 * (size_t)l], U1 = U[2 * (size_t)l + 1];
  T f0 = 0, f1 = 0;
  if (sv.adj_k2) {
    for (int e = sv.adj_ptr[l]; e < sv.adj_ptr[l + 1]; ++e) {
      const int q = sv.adj_nbr[e];
      const T kxx = sv.adj_k[e], kxy = sv.adj_k2[2 * e], kyy = sv.adj_k2[2 * e + 1];
      const T d0 = U0 - U[2 * (size_t)q], d1 = U1 - U[2 * (size_t)q + 1];
      f0 += kxx * d0 + kxy * d1;
      f1 += kxy * d0 + kyy * d1;
    }
  } else {
    for (int e = sv.adj_ptr[l]; e < sv.adj_ptr[l + 1]; ++e) {
      const int q = sv.adj_nbr[e];
      const T k = sv.adj_k[e];
      f0 += k * (U0 - U[2 * (size_t)q]);
      f1 += k * (U1 - U[2 * (size_t)q + 1]);
    }
  }
  F[l] = f0;
  F[M + l] = f1;
}

template <typename T>
static void launch_interp_lanes(const T* u, const T* v, FootView<T> fx, FootView<T> fy, int M, int N, T* U,
                                hipStream_t s) {
  IBMG_KLAUNCH((k_interp_lanes<T>), dim3(cdiv((size_t)M * 8, 256)), dim3(256), 0, s, u, v, fx, fy, M, N, U);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_ib_force(const T* u, const T* v, FootView<T> fx, FootView<T> fy, SpringView<T> sv,
                     int N, T* U, T* F, hipStream_t s) {
  if (!sv.M) return;
  launch_interp_lanes<T>(u, v, fx, fy, sv.M, N, U, s);
  IBMG_KLAUNCH((k_spring_force<T>), dim3(cdiv(sv.M, 256)), dim3(256), 0, s, U, sv, F);
  IBMG_LAUNCH_CHECK();
}

template <typename T>
void launch_interp(const T* u, const T* v, FootView<T> fx, FootView<T> fy, int M, int N, T* U,
                   hipStream_t s) {
  if (!M) return;
  launch_interp_lanes<T>(u, v, fx, fy, M, N, U, s);
}

// Nodal spring forces on the periodic square (Sec. 5 fibres): spring e at l
// with separation d = X_q - X_l (minimum image) and rest length L_e pulls l
// by kappa_e (1 - L_e / |d|) d, i.e. kappa_e d for L_e = 0 (the linear model,
// F = K_h X); X and F interleaved [M][2], kappa_e = adj_k (the linear
// model's stiffness, also with tangent blocks), rest per incidence or null.
__global__ void k_fibre_force(const double* __restrict__ X, SpringView<double> sv, const double* __restrict__ kap,
                              const double* __restrict__ rest, double* __restrict__ F) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= sv.M) return;
  const double x0 = X[2 * l], y0 = X[2 * l + 1];
  double f0 = 0, f1 = 0;
  for (int e = sv.adj_ptr[l]; e < sv.adj_ptr[l + 1]; ++e) {
    const int q = sv.adj_nbr[e];
    double dx = X[2 * q] - x0, dy = X[2 * q + 1] - y0;
    dx -= rint(dx);
    dy -= rint(dy);
    double k = kap[e];
    if (rest && rest[e] != 0.0) k *= 1.0 - rest[e] / sqrt(dx * dx + dy * dy);
    f0 += k * dx;
    f1 += k * dy;
  }
  F[2 * l] = f0;
  F[2 * l + 1] = f1;
}

void launch_fibre_force(const double* X, SpringView<double> sv, const double* kap, const double* rest, double* F,
                        hipStream_t s) {
  if (!sv.M) return;
  IBMG_KLAUNCH(k_fibre_force, dim3(cdiv(sv.M, 256)), dim3(256), 0, s, X, sv, kap, rest, F);
  IBMG_LAUNCH_CHECK();
}

// rhs = [(rho/dt) u + f_u; (rho/dt) v + f_v; 0]  (f = S_h F on the faces)
__global__ void k_step_rhs(const double* __restrict__ w, const double* __restrict__ f, double a, size_t nn,
                           double* __restrict__ rhs) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < 3 * nn; i += (size_t)gridDim.x * blockDim.x)
    rhs[i] = i < 2 * nn ? a * w[i] + f[i] : 0.0;
}

void launch_step_rhs(const double* w, const double* f, double a, int N, double* rhs, hipStream_t s) {
  const size_t nn = (size_t)N * N;
  int g = cdiv(3 * nn, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH(k_step_rhs, dim3(g), dim3(256), 0, s, w, f, a, nn, rhs);
  IBMG_LAUNCH_CHECK();
}

// X <- X + dt U (U interleaved [M][2]), wrapped into [0, 1)
__global__ void k_advance(double* __restrict__ X, const double* __restrict__ U, double dt, int M) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * M) return;
  double x = X[t] + dt * U[t];
  x -= floor(x);
  X[t] = x < 1.0 ? x : 0.0;
}

void launch_advance(double* X, const double* U, double dt, int M, hipStream_t s) {
  if (!M) return;
  IBMG_KLAUNCH(k_advance, dim3(cdiv(2 * (size_t)M, 256)), dim3(256), 0, s, X, U, dt, M);
  IBMG_LAUNCH_CHECK();
}

// f_face = scale * sum_(l, slot) w F_l, F interleaved [M][2]; f = [2][N][N].
// One work-group per 256 consecutive faces, x-faces and then the y-faces of
// the same indices: their (point, slot) entries are contiguous in face
// order, so the work-group forms the entries' terms w F_l in chunks through
// LDS (every thread, in entry order, with coalesced reads of the weights and
// indices), and then each thread adds its face's terms in list order.  Long
// lists near a densely sampled structure are thereby spread over the
// work-group instead of one thread, and every face's sum keeps a fixed
// order.  The y-faces' entries mostly name the points the x-faces' entries
// just read, whose two force components share a cache line, so the second
// pass finds them in cache.
constexpr int kSpreadTile = 256, kSpreadChunk = 2048;

__global__ void __launch_bounds__(256) k_spread(const double* __restrict__ F, FootView<double> fx,
                                                FootView<double> fy, int N, double scale, double* __restrict__ f) {
  __shared__ double terms[kSpreadChunk];
  const int nf = N * N;
  const int f0 = blockIdx.x * kSpreadTile;
  const int face = f0 + threadIdx.x;
  const bool live = face < nf;
  const int fend = f0 + kSpreadTile < nf ? f0 + kSpreadTile : nf;
  for (int comp = 0; comp < 2; ++comp) {
    const FootView<double>& fv = comp ? fy : fx;
    const int e0 = fv.sp_ptr[f0], e1 = fv.sp_ptr[fend];
    const int my_lo = live ? fv.sp_ptr[face] : e1, my_hi = live ? fv.sp_ptr[face + 1] : e1;
    double a = 0.0;
    for (int c0 = e0; c0 < e1; c0 += kSpreadChunk) {
      const int c1 = c0 + kSpreadChunk < e1 ? c0 + kSpreadChunk : e1;
      for (int e = c0 + (int)threadIdx.x; e < c1; e += kSpreadTile)
        terms[e - c0] = fv.sw[e] * F[2 * (fv.sp_ent[e] >> 4) + comp];
      __syncthreads();
      const int lo = my_lo > c0 ? my_lo : c0, hi = my_hi < c1 ? my_hi : c1;
      for (int e = lo; e < hi; ++e) a += terms[e - c0];
      __syncthreads();
    }
    if (live) f[(size_t)comp * nf + face] = scale * a;
  }
}

void launch_spread(const double* F, FootView<double> fx, FootView<double> fy, int M, int N,
                   double scale, double* f, hipStream_t s) {
  (void)M;
  IBMG_KLAUNCH(k_spread, dim3(cdiv((size_t)N * N, kSpreadTile)), dim3(kSpreadTile), 0, s, F, fx, fy, N, scale, f);
  IBMG_LAUNCH_CHECK();
}

// Slot of face (i, j) in point q's window, or -1.
__device__ __forceinline__ int slot_of(const int* __restrict__ base, const int* __restrict__ mask,
                                       int q, int i, int j, int N) {
  int a = i - base[2 * q];
  if (a < 0) a += N;
  int b = j - base[2 * q + 1];
  if (b < 0) b += N;
  if (a > 3 || b > 3) return -1;
  const int s = b * 4 + a;
  return ((mask[q] >> s) & 1) ? s : -1;
}


// Weight of face (i, j) in point q's window of one component (0 outside).
__device__ __forceinline__ double window_weight(const FootView<double>& f, const int* __restrict__ mask, int q,
                                                int i, int j, int N) {
  const int s = slot_of(f.base, mask, q, i, j, N);
  return s >= 0 ? f.w[(size_t)q * 16 + s] : 0.0;
}

// Row r of component comp of the level IB operator dt/h^2 J^T K' J:
//   T(r, (c, col)) = ibs * sum_e g_e(r) K_e[comp][c] g^c_e(col),
//   g^c_e = J^c_{b_e} - J^c_{a_e},
// summing over the springs with an end whose comp-window holds r (a spring
// with both ends there is counted once, from its lower-numbered end), and
// over the components c that K_e couples (c = comp for the linear model).
// Columns index the level's [u | v] vector.  One wave per row and slice:
// every lane walks the slice's (point, spring) pairs in the same order and
// accumulates the columns it owns (pattern entries lane, lane + 64, ...), so
// each entry is a fixed-order sum.  With nslice > 1 the row's point list is
// cut into nslice contiguous slices (for coarse levels, whose faces carry
// thousands of points), slice s writes its sums to part[s * nnz + k], and
// k_t_sum adds the slices in order.
__global__ void __launch_bounds__(256) k_t_values(FootView<double> f0, FootView<double> f1,
                                                  const int* __restrict__ mask0, const int* __restrict__ mask1,
                                                  SpringView<double> sv, int comp, int N, double ibs,
                                                  const int* __restrict__ t_ptr, const int* __restrict__ t_col,
                                                  double* __restrict__ t_val, int nslice, size_t nnz,
                                                  double* __restrict__ part) {
  const size_t wv = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int NN = N * N;
  if (wv >= (size_t)NN * nslice) return;
  const int r = (int)(wv / nslice), sl = (int)(wv % nslice);
  const int lo = t_ptr[r], hi = t_ptr[r + 1];
  if (hi == lo) return;
  const FootView<double>& f = comp ? f1 : f0;
  const int* mask = comp ? mask1 : mask0;
  const int ri = r % N, rj = r / N;
  const int el = f.sp_ptr[r], elen = f.sp_ptr[r + 1] - el;
  const int e0 = el + (int)((long long)elen * sl / nslice), e1 = el + (int)((long long)elen * (sl + 1) / nslice);
  double* out = nslice > 1 ? part + (size_t)sl * nnz : t_val;
  for (int k = lo + lane; k - lane < hi; k += 64) {
    const bool live = k < hi;
    const int col = live ? t_col[k] : 0;
    const int c = col >= NN ? 1 : 0;
    const int face = col - c * NN;
    const int ci = face % N, cj = face / N;
    const FootView<double>& fc = c ? f1 : f0;
    const int* mc = c ? mask1 : mask0;
    double acc = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int l = f.sp_ent[e] >> 4;
      const double wl_r = f.sw[e];
      const int a0 = sv.adj_ptr[l], a1 = sv.adj_ptr[l + 1];
      if (a0 == a1) continue;
      const double wl_c = window_weight(fc, mc, l, ci, cj, N);
      for (int a = a0; a < a1; ++a) {
        const int q = sv.adj_nbr[a];
        const int sq = slot_of(f.base, mask, q, ri, rj, N);
        if (sq >= 0 && q < l) continue;  // counted from q's side
        const double g = (sq >= 0 ? f.w[(size_t)q * 16 + sq] : 0.0) - wl_r;
        double kc;
        if (sv.adj_k2) kc = comp == 0 ? (c == 0 ? sv.adj_k[a] : sv.adj_k2[2 * a]) : (c == 0 ? sv.adj_k2[2 * a] : sv.adj_k2[2 * a + 1]);
        else kc = c == comp ? sv.adj_k[a] : 0.0;
        const double coef = ibs * kc * g;
        if (coef == 0.0) continue;
        acc += coef * (window_weight(fc, mc, q, ci, cj, N) - wl_c);
      }
    }
    if (live) out[k] = acc;
  }
}

// t_val[k] = sum over the slices of part[s * nnz + k], slices in order
__global__ void k_t_sum(const double* __restrict__ part, int nslice, size_t nnz, double* __restrict__ t_val) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nnz; k += (size_t)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int sl = 0; sl < nslice; ++sl) a += part[(size_t)sl * nnz + k];
    t_val[k] = a;
  }
}

void launch_t_values(FootView<double> f0, FootView<double> f1, const int* mask0, const int* mask1,
                     SpringView<double> sv, int comp, int N, double ibs, const int* t_ptr, const int* t_col,
                     double* t_val, int nslice, size_t nnz, double* part, hipStream_t s) {
  if (nslice < 1 || (nslice > 1 && !part)) throw Error(IBMG_ERR_ARG, "IB-row slices need a partial buffer");
  const size_t n = (size_t)N * N;
  IBMG_KLAUNCH(k_t_values, dim3(cdiv(n * nslice * 64, 256)), dim3(256), 0, s, f0, f1, mask0, mask1, sv, comp,
                     N, ibs, t_ptr, t_col, t_val, nslice, nnz, part);
  IBMG_LAUNCH_CHECK();
  if (nslice > 1) {
    int grid = cdiv(nnz, 256);
    if (grid > 4096) grid = 4096;
    IBMG_KLAUNCH(k_t_sum, dim3(grid < 1 ? 1 : grid), dim3(256), 0, s, part, nslice, nnz, t_val);
    IBMG_LAUNCH_CHECK();
  }
}

// g_e = scale * (Ul_b - Ul_a)^T B_e (Uw_b - Uw_a), U interleaved [M][2],
// B_e = K_e / kappa_e = (B_xx, B_xy; B_xy, B_yy) per spring, or I when
// blocks is null.
__global__ void k_spring_grad(const double* __restrict__ Uw, const double* __restrict__ Ul,
                              const int* __restrict__ ends, const double* __restrict__ blocks, int n_springs,
                              double scale, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_springs) return;
  const int a = ends[2 * e], b = ends[2 * e + 1];
  const double l0 = Ul[2 * b] - Ul[2 * a], l1 = Ul[2 * b + 1] - Ul[2 * a + 1];
  const double w0 = Uw[2 * b] - Uw[2 * a], w1 = Uw[2 * b + 1] - Uw[2 * a + 1];
  double g;
  if (blocks) {
    const double bxx = blocks[3 * e], bxy = blocks[3 * e + 1], byy = blocks[3 * e + 2];
    g = l0 * (bxx * w0 + bxy * w1) + l1 * (bxy * w0 + byy * w1);
  } else {
    g = l0 * w0 + l1 * w1;
  }
  out[e] = scale * g;
}

void launch_spring_grad(const double* Uw, const double* Ul, const int* ends, const double* blocks,
                        int n_springs, double scale, double* out, hipStream_t s) {
  if (!n_springs) return;
  IBMG_KLAUNCH(k_spring_grad, dim3(cdiv(n_springs, 128)), dim3(128), 0, s, Uw, Ul, ends, blocks,
                     n_springs, scale, out);
  IBMG_LAUNCH_CHECK();
}

// Scratch of the allocation-free spring gradient: J w then J lambda, each
// [kStaticGradPoints][2] doubles.  Each GPU holds its own copy for the life
// of the process.  Host code never names the array in a launch or a copy: it
// asks the runtime for the array's device address once per device and uses
// that address.
static __device__ __align__(256) double scratch[4 * (size_t)kStaticGradPoints];

double* static_grad_scratch() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {};
  int dev = 0;
  IBMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(IBMG_ERR_STATE, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    IBMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(IBMG_ERR_HIP, "no device address for the gradient scratch");
    ptr[dev] = static_cast<double*>(p);
  }
  return ptr[dev];
}

template void launch_ib_force<double>(const double*, const double*, FootView<double>,
                                      FootView<double>, SpringView<double>, int, double*, double*, hipStream_t);
template void launch_ib_force<float>(const float*, const float*, FootView<float>, FootView<float>,
                                     SpringView<float>, int, float*, float*, hipStream_t);
template void launch_interp<double>(const double*, const double*, FootView<double>, FootView<double>,
                                    int, int, double*, hipStream_t);


// G = dt/h^2 J^T K' J x for both components from the explicit Galerkin rows:
// one wave per row, lanes stride the row, butterfly sum in a fixed order.
// Used on levels where many points share each face, so that a per-face
// gather would serialise on long lists.
template <typename T>
__global__ void __launch_bounds__(256) k_ib_spmv(const T* __restrict__ x, T* __restrict__ G,
                                                 CsrT<T> tu, CsrT<T> tv, int N) {
  const int NN = N * N;
  const int wave = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= 2 * NN) return;
  const int comp = wave >= NN ? 1 : 0;
  const int r = wave - comp * NN;
  const int* ptr = comp ? tv.ptr : tu.ptr;
  const int* col = comp ? tv.col : tu.col;
  const T* val = comp ? tv.val : tu.val;
  const int lo = ptr[r], hi = ptr[r + 1];
  T acc = 0;
  for (int k = lo + lane; k < hi; k += 64) acc += val[k] * x[col[k]];   // columns index [u | v]
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) G[wave] = acc;
}

template <typename T>
void launch_ib_spmv(const T* x, T* G, CsrT<T> tu, CsrT<T> tv, int N, hipStream_t s) {
  const size_t waves = 2 * (size_t)N * N;
  IBMG_KLAUNCH((k_ib_spmv<T>), dim3(cdiv(waves * 64, 256)), dim3(256), 0, s, x, G, tu, tv, N);
  IBMG_LAUNCH_CHECK();
}

template void launch_ib_spmv<double>(const double*, double*, CsrT<double>, CsrT<double>, int, hipStream_t);
template void launch_ib_spmv<float>(const float*, float*, CsrT<float>, CsrT<float>, int, hipStream_t);

}  // namespace ibmg
