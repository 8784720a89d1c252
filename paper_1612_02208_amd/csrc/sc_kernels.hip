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
// x given by a loader: xv(k) is entry k of [u | v]
template <typename T, typename Ld>
__device__ __forceinline__ T aib_row_l(Ld xv, int r, int N, const StokesCoef<T>& c, const CsrT<T>& tu,
                                       const CsrT<T>& tv) {
  const int NN = N * N;
  const int comp = r >= NN ? 1 : 0;
  const int q = r - comp * NN;
  const int i = q % N, j = q / N;
  const int o = comp * NN;
  const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
  const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
  const T xc = xv(o + q);
  T a = c.alpha * xc -
        c.beta * (xv(o + j * N + im) + xv(o + j * N + ip) + xv(o + jm * N + i) + xv(o + jp * N + i) - T(4) * xc);
  const CsrT<T>& t = comp ? tv : tu;
  for (int k = t.ptr[q]; k < t.ptr[q + 1]; ++k) a += t.val[k] * xv(t.col[k]);
  return a;
}
template <typename T>
__device__ __forceinline__ T aib_row(const T* __restrict__ x, int r, int N, const StokesCoef<T>& c,
                                     const CsrT<T>& tu, const CsrT<T>& tv) {
  return aib_row_l<T>([x](int k) { return x[k]; }, r, N, c, tu, tv);
}

// (-M^ p)_ij = (1/h^2) sum over the 4 faces of (p_ij - p_nb) / diag(A_IB)_face
template <typename T, typename Ld>
__device__ __forceinline__ T mhat_row_l(Ld pv, int q, int N, T ih2, const T* __restrict__ dinv) {
  const int NN = N * N;
  const int i = q % N, j = q / N;
  const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
  const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
  const T pc = pv(q);
  const T a = dinv[q] * (pc - pv(j * N + im)) + dinv[j * N + ip] * (pc - pv(j * N + ip)) +
              dinv[NN + q] * (pc - pv(jm * N + i)) + dinv[NN + jp * N + i] * (pc - pv(jp * N + i));
  return ih2 * a;
}
template <typename T>
__device__ __forceinline__ T mhat_row(const T* __restrict__ p, int q, int N, T ih2,
                                      const T* __restrict__ dinv) {
  return mhat_row_l<T>([p](int k) { return p[k]; }, q, N, ih2, dinv);
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

// The first colour of a sweep from x = 0: every row is written, colour 0's
// rows with b / diag (their whole update from a zero iterate), the others
// with 0 (the zero fill).
template <typename T>
__global__ void k_gs_init(T* __restrict__ x, const T* __restrict__ b, const int* __restrict__ colour, size_t n,
                          const T* __restrict__ diag) {
  for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < n; r += (size_t)gridDim.x * blockDim.x)
    x[r] = colour[r] == 0 ? (b[r] - T(0)) / diag[r] : T(0);
}

// The same for a velocity sweep whose right-hand side is b = G p: each face
// forms and stores its entry of G p (as k_grad does) before its update.
template <typename T>
__global__ void k_grad_init(T* __restrict__ x, T* __restrict__ b, const T* __restrict__ p,
                            const int* __restrict__ colour, int N, T gi, const T* __restrict__ diag) {
  const int NN = N * N;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < 2 * NN; r += gridDim.x * blockDim.x) {
    const int comp = r >= NN ? 1 : 0, q = r - comp * NN;
    const int i = q % N, j = q / N;
    const int im = i == 0 ? N - 1 : i - 1, jm = j == 0 ? N - 1 : j - 1;
    const T g = gi * (p[q] - p[comp ? jm * N + i : j * N + im]);
    b[r] = g;
    x[r] = colour[r] == 0 ? (g - T(0)) / diag[r] : T(0);
  }
}

// Colours sweep over a span of small colours inside one work-group: colours
// f0..f1 ascending, then g0..g1 descending (either part may be empty),
// colours separated by work-group barriers (all waves of a work-group share
// one CU, so global writes are visible to the group after the barrier).
__device__ __forceinline__ int span_steps(int f0, int f1, int g0, int g1) {
  return (f1 >= f0 ? f1 - f0 + 1 : 0) + (g0 >= g1 ? g0 - g1 + 1 : 0);
}
__device__ __forceinline__ int span_colour(int k, int f0, int f1, int g0) {
  const int na = f1 >= f0 ? f1 - f0 + 1 : 0;
  return k < na ? f0 + k : g0 - (k - na);
}

// pressure rows (-M^): one thread per row
template <typename T>
__global__ void __launch_bounds__(1024) k_gs_band_p(T* x, const T* __restrict__ b, const int* __restrict__ cptr,
                                                    const int* __restrict__ rows, int f0, int f1, int g0, int g1,
                                                    int N, const T* __restrict__ diag, const T* __restrict__ dinv,
                                                    T ih2) {
  const int ns = span_steps(f0, f1, g0, g1);
  for (int k = 0; k < ns; ++k) {
    const int col = span_colour(k, f0, f1, g0);
    for (int t = cptr[col] + threadIdx.x; t < cptr[col + 1]; t += blockDim.x) {
      const int r = rows[t];
      x[r] += (b[r] - mhat_row<T>(x, r, N, ih2, dinv)) / diag[r];
    }
    __syncthreads();
  }
}

// Velocity rows whose IB part is long (near the structure): groups of G
// lanes share a row, each lane summing every G-th IB entry, the group's
// partial sums combined by shuffles in a fixed order.  Every lane of the
// wave calls this (live = false for lanes without a row).
constexpr int kGsGroup = 16;

// xv(k): entry k of the iterate [u | v]; bv(r): the right-hand side
template <typename T, typename Ld, typename Bv>
__device__ __forceinline__ void gs_row_group_l(Ld xv, Bv bv, T* x, int r, bool live, int sub, int N,
                                               const StokesCoef<T>& c, const CsrT<T>& tu, const CsrT<T>& tv,
                                               const T* __restrict__ diag) {
  constexpr int G = kGsGroup;
  const int NN = N * N;
  const int comp = r >= NN ? 1 : 0;
  const int q = r - comp * NN;
  const int o = comp * NN;
  const CsrT<T>& tm = comp ? tv : tu;
  T a = 0;
  if (live)
    for (int k = tm.ptr[q] + sub; k < tm.ptr[q + 1]; k += G) a += tm.val[k] * xv(tm.col[k]);
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, G);
  if (live && sub == 0) {
    const int i = q % N, j = q / N;
    const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
    const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
    const T xc = xv(o + q);
    const T ax = c.alpha * xc -
                 c.beta * (xv(o + j * N + im) + xv(o + j * N + ip) + xv(o + jm * N + i) + xv(o + jp * N + i) -
                           T(4) * xc) + a;
    x[r] = xv(r) + (bv(r) - ax) / diag[r];
  }
}
template <typename T>
__device__ __forceinline__ void gs_row_group(T* x, const T* __restrict__ b, int r, bool live, int sub, int N,
                                             const StokesCoef<T>& c, const CsrT<T>& tu, const CsrT<T>& tv,
                                             const T* __restrict__ diag) {
  gs_row_group_l<T>([x](int k) { return x[k]; }, [b](int k) { return b[k]; }, x, r, live, sub, N, c, tu, tv, diag);
}

// One large colour over the grid: its nlong long rows (listed first) with a
// lane group per row in the first nbl work-groups, its other rows one
// thread per row in the rest.
template <typename T>
__global__ void k_gs_colour_split(T* x, const T* __restrict__ b, const int* __restrict__ rows, int nlong,
                                  int count, int nbl, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv,
                                  const T* __restrict__ diag) {
  if ((int)blockIdx.x < nbl) {
    const int g = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kGsGroup);
    const bool live = g < nlong;
    gs_row_group<T>(x, b, live ? rows[g] : 0, live, threadIdx.x % kGsGroup, N, c, tu, tv, diag);
    return;
  }
  const int t = nlong + (int)((blockIdx.x - nbl) * (size_t)blockDim.x + threadIdx.x);
  if (t >= count) return;
  const int r = rows[t];
  x[r] += (b[r] - aib_row<T>(x, r, N, c, tu, tv)) / diag[r];
}

// The sweep's first two colours in one launch, when colour 1 is a large
// colour: from x = 0, colour 0's rows take b / diag and colour 1's rows
// solve against those values, each formed where it is read (as the first
// launch would store it); every other row is zeroed.  The grid holds colour
// 1's long rows (lane groups, nbl blocks), then its other rows (nsb
// blocks), then every row for the fill.  GRAD (velocity sweeps): b = G p,
// formed on the fly and stored for the later colours.
template <typename T, bool GRAD>
__global__ void k_gs_init_c1(T* __restrict__ x, T* __restrict__ b, const T* __restrict__ p,
                             const int* __restrict__ colour, const int* __restrict__ rows, int nlong, int cnt,
                             int nbl, int nsb, int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv,
                             const T* __restrict__ diag) {
  const int NN = N * N;
  auto bv = [&](int r) -> T {
    if (!GRAD) return b[r];
    const int comp = r >= NN ? 1 : 0, q = r - comp * NN;
    const int i = q % N, j = q / N;
    const int im = i == 0 ? N - 1 : i - 1, jm = j == 0 ? N - 1 : j - 1;
    return c.gi * (p[q] - p[comp ? jm * N + i : j * N + im]);
  };
  auto xv = [&](int k) -> T { return colour[k] == 0 ? (bv(k) - T(0)) / diag[k] : T(0); };
  const int blk = blockIdx.x;
  if (blk < nbl) {
    const int gidx = (int)((blk * (size_t)blockDim.x + threadIdx.x) / kGsGroup);
    const bool live = gidx < nlong;
    gs_row_group_l<T>(xv, bv, x, live ? rows[gidx] : 0, live, threadIdx.x % kGsGroup, N, c, tu, tv, diag);
    return;
  }
  if (blk < nbl + nsb) {
    const int t = nlong + (int)((blk - nbl) * (size_t)blockDim.x + threadIdx.x);
    if (t >= cnt) return;
    const int r = rows[t];
    x[r] = xv(r) + (bv(r) - aib_row_l<T>(xv, r, N, c, tu, tv)) / diag[r];
    return;
  }
  const int r = (int)((blk - nbl - nsb) * (size_t)blockDim.x + threadIdx.x);
  if (r >= 2 * NN) return;
  const int cr = colour[r];
  if (GRAD) b[r] = bv(r);
  if (cr != 1) x[r] = cr == 0 ? (bv(r) - T(0)) / diag[r] : T(0);
}

// The same for a sweep on -M^ (cells; colour 1's rows one thread each).
template <typename T>
__global__ void k_gs_init_c1_m(T* __restrict__ x, const T* __restrict__ b, const int* __restrict__ colour,
                               const int* __restrict__ rows, int cnt, int nsb, int N, const T* __restrict__ diag,
                               const T* __restrict__ dinv, T ih2) {
  auto xv = [&](int k) -> T { return colour[k] == 0 ? (b[k] - T(0)) / diag[k] : T(0); };
  const int blk = blockIdx.x;
  if (blk < nsb) {
    const int t = (int)(blk * (size_t)blockDim.x + threadIdx.x);
    if (t >= cnt) return;
    const int r = rows[t];
    x[r] = xv(r) + (b[r] - mhat_row_l<T>(xv, r, N, ih2, dinv)) / diag[r];
    return;
  }
  const int r = (int)((blk - nsb) * (size_t)blockDim.x + threadIdx.x);
  if (r >= N * N) return;
  const int cr = colour[r];
  if (cr != 1) x[r] = cr == 0 ? (b[r] - T(0)) / diag[r] : T(0);
}

// a span of small velocity colours inside one work-group, lane groups per row
// (runs too large for the LDS kernel)
template <typename T>
__global__ void __launch_bounds__(1024) k_gs_band(T* x, const T* __restrict__ b, const int* __restrict__ cptr,
                                                  const int* __restrict__ rows, int f0, int f1, int g0, int g1,
                                                  int N, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv,
                                                  const T* __restrict__ diag) {
  constexpr int G = kGsGroup;
  const int grp = threadIdx.x / G, sub = threadIdx.x % G;
  const int ns = span_steps(f0, f1, g0, g1);
  for (int k = 0; k < ns; ++k) {
    const int col = span_colour(k, f0, f1, g0);
    const int r0 = cptr[col], r1 = cptr[col + 1];
    // uniform trip count across the work-group (shuffles inside)
    for (int base = r0; base < r1; base += blockDim.x / G) {
      const int t = base + grp;
      const bool live = t < r1;
      gs_row_group<T>(x, b, live ? rows[t] : 0, live, sub, N, c, tu, tv, diag);
    }
    __syncthreads();
  }
}

// LDS barrier: the work-group's LDS writes complete, then the barrier;
// global loads already issued stay in flight across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// A lane's value after a DPP move within its row of 16 lanes (CTRL: a
// quad_perm pattern here).
template <int CTRL>
__device__ __forceinline__ double quad_move(double x) {
  const long long bits = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float quad_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
// sum over the kBandG = 4 lanes of a row: lanes 2 apart, then neighbours
template <typename T>
__device__ __forceinline__ T quad_sum(T a) {
  a += quad_move<0x4E>(a);   // quad_perm [2,3,0,1]
  a += quad_move<0xB1>(a);   // quad_perm [1,0,3,2]
  return a;
}

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// A run of small velocity colours with the run's rows in LDS (BandRun).
// The prologue loads each slot's iterate and its right-hand side minus the
// outer entries (columns outside the run do not change while it is swept),
// a group of kBandG lanes per slot, the loads of four slot passes issued
// together; and the run's colour offsets.  Each colour then updates its
// slots from LDS, a group of kBandG lanes per row (a colour has fewer than
// kGsBigColour rows: one pass of the work-group); the epilogue stores the
// slots.  Band entries are read S colours ahead into S register stages
// (KP entry pairs per lane each), every load unconditional (lanes without
// a row, and steps past the span, read the last valid row), so the loads
// for the next S - 1 colours stay in flight while a colour is summed and
// across the barriers, which wait on LDS only.  A stage is refilled right
// after its colour's update, so its registers are reused in place.  Steps are padded to a
// multiple of S with empty ones.  Colours are run-relative: f0..f1
// ascending, then g0..g1 descending.  The sums run in the order of the
// row's entries per lane, then over lanes 2 apart and neighbours.
template <typename T, int KP, int S>
__global__ void __launch_bounds__(1024) k_gs_band_lds(T* x, const T* __restrict__ b, BandView<T> v, int f0, int f1,
                                                      int g0, int g1) {
  using T2 = typename Pair<T>::type;
  extern __shared__ char smem_raw[];
  T* xl = reinterpret_cast<T*>(smem_raw);
  T* cb = xl + v.nb;
  int* cp = reinterpret_cast<int*>(cb + v.nb);
  const char* xlb = reinterpret_cast<const char*>(xl);
  const int tid = threadIdx.x;
  const int grp = tid / kBandG, sub = tid % kBandG, ngrp = blockDim.x / kBandG;
  for (int i = tid; i <= v.ncol; i += blockDim.x) cp[i] = v.cptr[i];
  constexpr int U = 4, E = 3;   // slot passes per batch, outer entries per lane before the tail
  for (int base = 0; base < v.nb; base += U * ngrp) {
    int lo[U], hi[U], r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * ngrp + grp;
      const int ic = i < v.nb ? i : v.nb - 1;
      lo[u] = v.optr[ic];
      const int h = v.optr[ic + 1];
      hi[u] = i < v.nb ? h : lo[u];
      r[u] = v.brow[ic];
    }
    int oc[U][E];
    T ov[U][E];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int at = lo[u] + sub + kBandG * e;
        const bool ok = at < hi[u];
        const int c = v.ocol[ok ? at : 0];
        const T w = v.oval[ok ? at : 0];
        oc[u][e] = ok ? c : 0;
        ov[u][e] = ok ? w : T(0);
      }
    T a[U], br[U], xr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      br[u] = b[r[u]];
      xr[u] = x[r[u]];
      T xo[E];
#pragma unroll
      for (int e = 0; e < E; ++e) xo[e] = x[oc[u][e]];
      a[u] = T(0);
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (lo[u] + sub + kBandG * e < hi[u]) a[u] += ov[u][e] * xo[e];
      for (int at = lo[u] + sub + kBandG * E; at < hi[u]; at += kBandG) a[u] += v.oval[at] * x[v.ocol[at]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T s2 = quad_sum(a[u]);
      const int i = base + u * ngrp + grp;
      if (i < v.nb && sub == 0) {
        cb[i] = br[u] - s2;
        xl[i] = xr[u];
      }
    }
  }
  lds_barrier();
  const int ns = span_steps(f0, f1, g0, g1);
  if (ns > 0) {
    const unsigned* __restrict__ went = v.bent;
    const T2* __restrict__ wval = reinterpret_cast<const T2*>(v.bval);
    unsigned w[S][KP];
    T2 val[S][KP];
    T dg[S];
    int s0[S], n[S];
    auto fetch = [&](int st, int k) {
      const int col = span_colour(k < ns ? k : ns - 1, f0, f1, g0);
      const int c0 = cp[col], cn = cp[col + 1] - c0;
      s0[st] = k < ns ? c0 : 0;
      n[st] = k < ns ? cn : 0;
      const int li = grp < cn ? grp : cn - 1;
      dg[st] = v.bdiag[c0 + li];
      const size_t at = (size_t)c0 * (v.stride / 2) + (size_t)li * kBandG + sub;
      const size_t step = (size_t)cn * kBandG;
#pragma unroll
      for (int q = 0; q < KP; ++q) {
        w[st][q] = went[at + q * step];
        val[st][q] = wval[at + q * step];
      }
    };

    // the first stages' loads in stage order, as the loop refills them
#pragma unroll
    for (int st = 0; st < S; ++st) {
      fetch(st, st);
      asm volatile("" ::: "memory");
    }
    for (int k0 = 0; k0 < ns; k0 += S) {
#pragma unroll
      for (int st = 0; st < S; ++st) {
        T a = 0;
#pragma unroll
        for (int q = 0; q < KP; ++q) {
          a += val[st][q].x * *reinterpret_cast<const T*>(xlb + (w[st][q] & 0xffffu));
          a += val[st][q].y * *reinterpret_cast<const T*>(xlb + (w[st][q] >> 16));
        }
        a = quad_sum(a);
        const int myrow = grp < n[st] ? s0[st] + grp : -1;
        if (myrow >= 0 && sub == 0) xl[myrow] += (cb[myrow] - a) / dg[st];
        fetch(st, k0 + st + S);
        lds_barrier();
      }
    }
  }
  for (int i = tid; i < v.nb; i += blockDim.x) x[v.brow[i]] = xl[i];
}

// Values of a run's entries from their codes: (IB index + 1) * 4 + stencil
// kind, the IB index over the u rows' Galerkin entries, then the v rows'
// (padding: code 0, value 0); and each slot's diagonal.
template <typename T>
__device__ __forceinline__ T band_value(int code, const StokesCoef<T>& c, const CsrT<T>& tu, const CsrT<T>& tv,
                                        int nnz_u) {
  const int kind = code & 3, k = (code >> 2) - 1;
  T v = kind == 1 ? c.alpha + T(4) * c.beta : (kind == 2 ? -c.beta : T(0));
  if (k >= 0) v += k < nnz_u ? tu.val[k] : tv.val[k - nnz_u];
  return v;
}

template <typename T>
__global__ void k_band_values(const int* __restrict__ bcode, T* __restrict__ bval, size_t nbe,
                              const int* __restrict__ ocode, T* __restrict__ oval, size_t noe,
                              const int* __restrict__ brow, T* __restrict__ bdiag, int nb, const T* __restrict__ diag,
                              StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, int nnz_u) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nbe + noe + nb;
       e += (size_t)gridDim.x * blockDim.x) {
    if (e < nbe) bval[e] = band_value(bcode[e], c, tu, tv, nnz_u);
    else if (e < nbe + noe) oval[e - nbe] = band_value(ocode[e - nbe], c, tu, tv, nnz_u);
    else bdiag[e - nbe - noe] = diag[brow[e - nbe - noe]];
  }
}

template <typename T>
void launch_band_values(BandRun<T>& run, StokesCoef<T> c, CsrT<T> tu, CsrT<T> tv, int N, const T* diag,
                        hipStream_t s) {
  (void)N;
  if (!run.nb) return;
  const size_t nbe = run.hbcode.size(), noe = run.hocol.size(), tot = nbe + noe + run.nb;
  int grid = cdiv(tot, 256);
  if (grid > 4096) grid = 4096;
  IBMG_KLAUNCH((k_band_values<T>), dim3(grid), dim3(256), 0, s, run.bcode.p, run.bval.p, nbe, run.ocode.p,
               run.oval.p, noe, run.brow.p, run.bdiag.p, run.nb, diag, c, tu, tv, run.nnz_u);
  IBMG_LAUNCH_CHECK();
}

// One symmetric multicolour sweep from x = 0: colours 1 .. C-1 after the
// fused colour 0, then C-2 .. 0 (the last colour's second update is zero in
// exact arithmetic: its rows are mutually uncoupled, so after the first
// their residuals vanish).  Large colours run over the grid; each maximal
// span of small colours in that sequence runs in one work-group.
template <typename T>
void launch_gs_sweep(T* x, const T* b, const GsSweep<T>& g, hipStream_t s) {
  const ColourLists& cl = *g.cl;
  const int C = cl.ncol;
  const size_t n = cl.colour.size();
  if (!C) return;
  // colour 1 large: the first two colours in one launch
  const bool fuse1 = C >= 2 && cl.big(1);
  if (fuse1) {
    const int cnt = cl.ptr[2] - cl.ptr[1];
    const int* rows = cl.d_rows.p + cl.ptr[1];
    if (g.grad_p && (g.mhat || n != 2 * (size_t)g.N * g.N || g.grad_out != b))
      throw Error(IBMG_ERR_ARG, "the fused gradient start is for velocity sweeps on b = G p");
    if (g.mhat) {
      const int nsb = cdiv(cnt, 256);
      IBMG_KLAUNCH((k_gs_init_c1_m<T>), dim3(nsb + cdiv(n, 256)), dim3(256), 0, s, x, b, cl.d_colour.p, rows, cnt,
                   nsb, g.N, g.diag, g.dinv, g.ih2);
    } else {
      const int nl = cl.nlong[1];
      const int nbl = cdiv((size_t)nl * kGsGroup, 256), nsb = cdiv(cnt - nl, 256);
      const dim3 grid(nbl + nsb + cdiv(n, 256));
      if (g.grad_p)
        IBMG_KLAUNCH((k_gs_init_c1<T, true>), grid, dim3(256), 0, s, x, g.grad_out, g.grad_p, cl.d_colour.p, rows,
                     nl, cnt, nbl, nsb, g.N, g.c, g.tu, g.tv, g.diag);
      else
        IBMG_KLAUNCH((k_gs_init_c1<T, false>), grid, dim3(256), 0, s, x, const_cast<T*>(b), nullptr,
                     cl.d_colour.p, rows, nl, cnt, nbl, nsb, g.N, g.c, g.tu, g.tv, g.diag);
    }
    IBMG_LAUNCH_CHECK();
  } else {
    int grid = cdiv(n, 256);
    if (grid > 4096) grid = 4096;
    if (g.grad_p) {
      if (g.mhat || n != 2 * (size_t)g.N * g.N || g.grad_out != b)
        throw Error(IBMG_ERR_ARG, "the fused gradient start is for velocity sweeps on b = G p");
      IBMG_KLAUNCH((k_grad_init<T>), dim3(grid), dim3(256), 0, s, x, g.grad_out, g.grad_p, cl.d_colour.p, g.N,
                   g.c.gi, g.diag);
    } else {
      IBMG_KLAUNCH((k_gs_init<T>), dim3(grid), dim3(256), 0, s, x, b, cl.d_colour.p, n, g.diag);
    }
    IBMG_LAUNCH_CHECK();
  }
  std::vector<int> seq;
  for (int c = 1; c < C; ++c) seq.push_back(c);
  for (int c = C - 2; c >= 0; --c) seq.push_back(c);
  for (size_t a = fuse1 ? 1 : 0; a < seq.size();) {
    const int col = seq[a];
    if (cl.big(col)) {
      const int cnt = cl.ptr[col + 1] - cl.ptr[col];
      const int* rows = cl.d_rows.p + cl.ptr[col];
      if (g.mhat) {
        IBMG_KLAUNCH((k_gs_colour<T, true>), dim3(cdiv(cnt, 256)), dim3(256), 0, s, x, b, rows, cnt, g.N, g.c,
                     g.tu, g.tv, g.diag, g.dinv, g.ih2);
      } else {
        const int nl = cl.nlong[col];
        const int nbl = cdiv((size_t)nl * kGsGroup, 256);
        IBMG_KLAUNCH((k_gs_colour_split<T>), dim3(nbl + cdiv(cnt - nl, 256)), dim3(256), 0, s, x, b, rows, nl,
                     cnt, nbl, g.N, g.c, g.tu, g.tv, g.diag);
      }
      IBMG_LAUNCH_CHECK();
      ++a;
      continue;
    }
    // the span of small colours seq[a..z]: its entries up to the turnaround
    // (seq index C - 2, colour C - 1) ascend, the rest descend
    size_t z = a;
    while (z + 1 < seq.size() && !cl.big(seq[z + 1])) ++z;
    const size_t turn = (size_t)(C - 2);
    int f0 = 0, f1 = -1, g0 = -1, g1 = 0;
    if (a <= turn) {
      f0 = seq[a];
      f1 = seq[std::min(z, turn)];
    }
    if (z > turn) {
      g0 = seq[std::max(a, turn + 1)];
      g1 = seq[z];
    }
    const BandRun<T>* run = nullptr;
    if (g.runs)
      for (const BandRun<T>& rr : *g.runs)
        if (rr.cf <= seq[a] && seq[a] <= rr.cl) run = &rr;
    if (run && run->lds) {
      const int nc = run->cl - run->cf + 1;
      const BandView<T> v{run->nb,   nc,          run->stride, run->cptr.p, run->brow.p, run->optr.p,
                          run->ocol.p, run->bent.p, run->bval.p, run->oval.p, run->bdiag.p};
      const int o = run->cf;
      const size_t lds = 2 * (size_t)run->nb * sizeof(T) + (nc + 1) * sizeof(int);
      const int a0 = f0 - o, a1 = f1 - o, b0 = g0 - o, b1 = g1 - o;
      switch (run->kp) {
        case 1: IBMG_KLAUNCH((k_gs_band_lds<T, 1, 4>), dim3(1), dim3(1024), lds, s, x, b, v, a0, a1, b0, b1); break;
        case 2: IBMG_KLAUNCH((k_gs_band_lds<T, 2, 4>), dim3(1), dim3(1024), lds, s, x, b, v, a0, a1, b0, b1); break;
        case 3: IBMG_KLAUNCH((k_gs_band_lds<T, 3, 4>), dim3(1), dim3(1024), lds, s, x, b, v, a0, a1, b0, b1); break;
        case 4: IBMG_KLAUNCH((k_gs_band_lds<T, 4, 3>), dim3(1), dim3(1024), lds, s, x, b, v, a0, a1, b0, b1); break;
        case 6: IBMG_KLAUNCH((k_gs_band_lds<T, 6, 3>), dim3(1), dim3(1024), lds, s, x, b, v, a0, a1, b0, b1); break;
        default: IBMG_KLAUNCH((k_gs_band_lds<T, 8, 2>), dim3(1), dim3(1024), lds, s, x, b, v, a0, a1, b0, b1); break;
      }
    } else if (g.mhat) {
      IBMG_KLAUNCH((k_gs_band_p<T>), dim3(1), dim3(1024), 0, s, x, b, cl.d_ptr.p, cl.d_rows.p, f0, f1, g0, g1, g.N,
                   g.diag, g.dinv, g.ih2);
    } else {
      IBMG_KLAUNCH((k_gs_band<T>), dim3(1), dim3(1024), 0, s, x, b, cl.d_ptr.p, cl.d_rows.p, f0, f1, g0, g1, g.N,
                   g.c, g.tu, g.tv, g.diag);
    }
    IBMG_LAUNCH_CHECK();
    a = z + 1;
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

// Chebyshev start with the first residual update: d = theta_inv s, x = d,
// rc = r - A_IB d, the neighbours' d formed from s as the start forms it
template <typename T>
__global__ void k_cheb_init_sub(int N, T theta_inv, const T* __restrict__ sv, T* __restrict__ d, T* __restrict__ x,
                                const T* __restrict__ r, T* __restrict__ rc, StokesCoef<T> c, CsrT<T> tu,
                                CsrT<T> tv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * N * N) return;
  const T di = theta_inv * sv[i];
  d[i] = di;
  x[i] = di;
  rc[i] = r[i] - aib_row_l<T>([=](int k) { return theta_inv * sv[k]; }, i, N, c, tu, tv);
}

// A velocity iterate whose last Chebyshev step is still to be added:
// x + (c1 d + c2 s), rounded as k_cheb_step rounds it
template <typename T>
__device__ __forceinline__ T cheb_final(const T* __restrict__ x, const T* __restrict__ d, const T* __restrict__ sv,
                                        T c1, T c2, size_t k) {
  const T dk = c1 * d[k] + c2 * sv[k];
  return x[k] + dk;
}

// out = a D u + b y with u = x + (c1 d + c2 s) formed on the fly (u is not
// stored); out may be y
template <typename T>
__global__ void k_cheb_div(const T* __restrict__ x, const T* __restrict__ d, const T* __restrict__ sv, T c1, T c2,
                           const T* y, T* out, int N, T gi, T a, T b) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * N) return;
  const int i = q % N, j = q / N;
  const int ip = i == N - 1 ? 0 : i + 1, jp = j == N - 1 ? 0 : j + 1;
  const size_t NN = (size_t)N * N;
  const T dv = gi * (cheb_final(x, d, sv, c1, c2, (size_t)j * N + ip) - cheb_final(x, d, sv, c1, c2, q) +
                     cheb_final(x, d, sv, c1, c2, NN + (size_t)jp * N + i) - cheb_final(x, d, sv, c1, c2, NN + q));
  out[q] = a * dv + (y ? b * y[q] : T(0));
}

// z = w - (x + (c1 d + c2 s))
template <typename T>
__global__ void k_cheb_sub(size_t n, T c1, T c2, const T* __restrict__ sv, const T* __restrict__ d,
                           const T* __restrict__ x, const T* __restrict__ w, T* __restrict__ z) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    z[i] = w[i] - cheb_final(x, d, sv, c1, c2, i);
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
void launch_cheb_init_sub(int N, T theta_inv, const T* sv, T* d, T* x, const T* r, T* rc, StokesCoef<T> c,
                          CsrT<T> tu, CsrT<T> tv, hipStream_t s) {
  IBMG_KLAUNCH((k_cheb_init_sub<T>), dim3(cdiv(2 * (size_t)N * N, 256)), dim3(256), 0, s, N, theta_inv, sv, d, x, r,
               rc, c, tu, tv);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_cheb_div(const T* x, const T* d, const T* sv, T c1, T c2, const T* y, T* out, int N, T gi, T a, T b,
                     hipStream_t s) {
  IBMG_KLAUNCH((k_cheb_div<T>), dim3(cdiv((size_t)N * N, 256)), dim3(256), 0, s, x, d, sv, c1, c2, y, out, N, gi,
               a, b);
  IBMG_LAUNCH_CHECK();
}
template <typename T>
void launch_cheb_sub(size_t n, T c1, T c2, const T* sv, const T* d, const T* x, const T* w, T* z, hipStream_t s) {
  int g = cdiv(n, 256);
  if (g > 4096) g = 4096;
  IBMG_KLAUNCH((k_cheb_sub<T>), dim3(g), dim3(256), 0, s, n, c1, c2, sv, d, x, w, z);
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
  template void launch_gs_sweep<T>(T*, const T*, const GsSweep<T>&, hipStream_t);                          \
  template void launch_band_values<T>(BandRun<T>&, StokesCoef<T>, CsrT<T>, CsrT<T>, int, const T*,          \
                                      hipStream_t);                                                          \
  template void launch_aib_apply<T>(const T*, T*, int, StokesCoef<T>, CsrT<T>, CsrT<T>, hipStream_t);        \
  template void launch_grad<T>(const T*, T*, int, T, hipStream_t);                                           \
  template void launch_div_comb<T>(const T*, const T*, T*, int, T, T, T, hipStream_t);                       \
  template void launch_axpby<T>(size_t, T, const T*, T, const T*, T*, hipStream_t);                          \
  template void launch_weyl<T>(T*, size_t, hipStream_t);                                                     \
  template void launch_cheb_init<T>(size_t, T, const T*, T*, T*, const T*, T*, hipStream_t);                  \
  template void launch_cheb_step<T>(size_t, T, T, const T*, T*, T*, hipStream_t);                             \
  template void launch_cheb_init_sub<T>(int, T, const T*, T*, T*, const T*, T*, StokesCoef<T>, CsrT<T>, CsrT<T>, \
                                        hipStream_t);                                                        \
  template void launch_cheb_div<T>(const T*, const T*, const T*, T, T, const T*, T*, int, T, T, T, hipStream_t); \
  template void launch_cheb_sub<T>(size_t, T, T, const T*, const T*, const T*, const T*, T*, hipStream_t);      \
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
