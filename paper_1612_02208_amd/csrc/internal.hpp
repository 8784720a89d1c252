// Internal declarations shared by the host orchestration and the HIP kernels.
//
// Conventions (see include/ibmg.h): a level vector is [u | v | p], each block
// n*n in (j, i) row-major order; u[j][i] sits on the x-face (i h, (j+1/2) h),
// v[j][i] on the y-face ((i+1/2) h, j h), p[j][i] at the cell centre.
//
// Immersed-boundary footprints.  Each Lagrangian point owns, per velocity
// component and per level, a 4 x 4 window of faces starting at a wrapped base
// (i0, j0); slot s = 4*b + a addresses face (i0 + a, j0 + b).  A 16-bit mask
// marks the structurally coupled faces; the weights of the other slots are 0.
// On the finest level the weight is phi(rx) phi(ry) (App. A.3); on a coarser
// level it is the finer window pushed through the velocity prolongation,
// J_l = J_{l+1} P_u, so that dt/h_l^2 J_l^T K' J_l is the Galerkin product
// R_u [S K J]^{l+1} P_u of Sec. 3.1 (R_u = P_u^T / 4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <iterator>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ibmg.h"

namespace ibmg {

struct Error : public std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Sizing pass.  ibmg_workspace_bytes runs the whole set-up with this flag
// set: host planning and buffer placement happen as in ibmg_create, but no
// kernel is launched and no HIP runtime call is made, so the placement's
// high-water mark is the exact workspace the real set-up needs.
inline bool& dry_run_flag() {
  static thread_local bool f = false;
  return f;
}
inline bool dry_run() { return dry_run_flag(); }
struct DryScope {
  bool prev;
  DryScope() : prev(dry_run_flag()) { dry_run_flag() = true; }
  ~DryScope() { dry_run_flag() = prev; }
};

#define IBMG_HIP(expr)                                                                      \
  do {                                                                                      \
    if (!::ibmg::dry_run()) {                                                               \
      hipError_t e_ = (expr);                                                               \
      if (e_ != hipSuccess)                                                                 \
        throw ::ibmg::Error(IBMG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                                       \
  } while (0)

#define IBMG_LAUNCH_CHECK() IBMG_HIP(hipGetLastError())

// every kernel launch of the library (skipped in the sizing pass)
#define IBMG_KLAUNCH(...)                                    \
  do {                                                       \
    if (!::ibmg::dry_run()) hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)

inline void require(bool ok, const std::string& msg) {
  if (!ok) throw Error(IBMG_ERR_ARG, msg);
}

// Device memory of one handle: the single region the caller passes to
// ibmg_create.  Blocks are 256-byte aligned and placed first-fit from a
// free list ordered by offset; freed blocks merge with free neighbours and
// a freed block at the top lowers it.  The placement depends only on the
// sequence of sizes, so a sizing arena (no memory behind it: it hands out
// addresses of a virtual region that nothing dereferences) run through the
// same sequence reports the exact size needed as its high-water mark.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  Arena(void* base, size_t cap) : base_(static_cast<char*>(base)), cap_(cap) {}
  static Arena sizing() { return Arena(nullptr, ~(size_t)0); }
  bool is_sizing() const { return base_ == nullptr; }
  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_bytes_; }
  size_t peak() const { return peak_; }

  void* alloc(size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    if (bytes == 0) bytes = kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rem = it->second - bytes;
      free_.erase(it);
      if (rem) free_[off + bytes] = rem;
      return take(off, bytes);
    }
    if (bytes > cap_ - top_)
      throw Error(IBMG_ERR_WORKSPACE, "workspace too small: " + std::to_string(top_ + bytes) +
                                          " bytes needed at this point, " + std::to_string(cap_) + " given");
    const size_t off = top_;
    top_ += bytes;
    if (top_ > peak_) peak_ = top_;
    return take(off, bytes);
  }

  void release(void* p) {
    if (!p) return;
    size_t off = (size_t)(static_cast<char*>(p) - origin());
    auto it = used_.find(off);
    if (it == used_.end()) return;
    size_t sz = it->second;
    used_.erase(it);
    used_bytes_ -= sz;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + sz) {
      sz += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        sz += pv->second;
        free_.erase(pv);
      }
    }
    if (off + sz == top_) top_ = off;
    else free_[off] = sz;
  }

 private:
  // the virtual region of a sizing arena starts at a fixed non-null address
  char* origin() const { return base_ ? base_ : reinterpret_cast<char*>((uintptr_t)1 << 40); }
  void* take(size_t off, size_t bytes) {
    used_[off] = bytes;
    used_bytes_ += bytes;
    return origin() + off;
  }
  char* base_;
  size_t cap_;
  size_t top_ = 0, peak_ = 0, used_bytes_ = 0;
  std::map<size_t, size_t> free_, used_;   // offset -> size
};

// The arena the current ABI call allocates from (set per call by the entry
// points; a DBuf remembers its arena for the release).
inline Arena*& current_arena() {
  static thread_local Arena* a = nullptr;
  return a;
}
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(current_arena()) { current_arena() = a; }
  ~ArenaScope() { current_arena() = prev; }
};

// Owning device buffer (a block of the current arena).
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  Arena* a = nullptr;
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), a(o.a) {
    o.p = nullptr;
    o.n = 0;
    o.a = nullptr;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      a = o.a;
      o.p = nullptr;
      o.n = 0;
      o.a = nullptr;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (!count) return;
    Arena* ar = current_arena();
    if (!ar) throw Error(IBMG_ERR_STATE, "device buffer requested outside a handle's workspace");
    p = static_cast<T*>(ar->alloc(count * sizeof(T)));
    n = count;
    a = ar;
  }
  void release() {
    if (p && a) a->release(p);
    p = nullptr;
    n = 0;
    a = nullptr;
  }
  void upload(const T* h, size_t count, hipStream_t s) {
    if (count > n) alloc(count);
    if (count) IBMG_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T>& h, hipStream_t s) { upload(h.data(), h.size(), s); }
};

// ---------------------------------------------------------------------------
// Device-side views passed to kernels by value.
// ---------------------------------------------------------------------------
template <typename T>
struct FootView {       // one component of one level
  const int* base;      // [M][2] wrapped (i0, j0)
  const T* w;           // [M][16] weights
  const int* sp_ptr;    // [n*n + 1] faces -> entries
  const int* sp_ent;    // entries l*16 + slot
  const T* sw;          // weights in face-list order: sw[e] = w[sp_ent[e]]
  const int* order;     // [M] points in cell order (point-wise kernels walk it)
  const int* obase;     // [M][2] bases in walk order: obase[2 g] = base[2 order[g]]
  const T* ow;          // [M][16] weights in walk order
};

template <typename T>
struct SpringView {
  int M;
  const int* adj_ptr;   // [M + 1]
  const int* adj_nbr;   // neighbour node per incidence
  const T* adj_k;       // stiffness per incidence (K_e[0][0] with tangent blocks)
  const T* adj_k2;      // tangent blocks: (K_e[0][1], K_e[1][1]) per incidence,
                        // nullptr for the linear model (K_e = kappa_e I)
};

template <typename T>
struct StokesCoef {     // A = alpha I - mu Lap: alpha, beta = mu/h^2, gi = 1/h, ibs = dt/h^2
  T alpha, beta, gi, ibs;
};

struct BoxGeom {        // RAS boxes on one level
  int N, b, o, m, npd, nloc, nown, nch;  // nch = ceil(nown / 64) row chunks
};

// Segments of a batch vector: system s owns entries [begin(s), begin(s) +
// len(s)).  A single system is one segment at 0; a batch of equal systems
// has off = null and segment s = [s n, (s + 1) n); ragged batches (systems of
// different grid sizes) list their offsets.  Kernels take the system from a
// grid index and skip systems whose active flag is 0.
struct BSeg {
  const long long* off;  // [nsys + 1] device offsets, or null
  size_t n;              // segment length when off is null
  const int* active;     // [nsys] device flags, or null: every system active
};
inline BSeg seg1(size_t n) { return BSeg{nullptr, n, nullptr}; }
__device__ __forceinline__ size_t seg_begin(const BSeg& g, int s) {
  return g.off ? (size_t)g.off[s] : (size_t)s * g.n;
}
__device__ __forceinline__ size_t seg_len(const BSeg& g, int s) {
  return g.off ? (size_t)(g.off[s + 1] - g.off[s]) : g.n;
}
__device__ __forceinline__ bool seg_on(const BSeg& g, int s) { return !g.active || g.active[s] != 0; }

// Sums of nv <= K per-thread values over a block of 256 threads, in the same
// fixed order in every block (deterministic): a butterfly over the 64 lanes
// of each wave (every lane ends with identical bits), then the four wave
// sums as (w0 + w1) + (w2 + w3).  Threads tid < nv write sum q = tid to
// out[tid]; red holds 4 K doubles of shared memory.  Every thread of the
// block must call it (two barriers); out may be shared memory, visible to
// all threads on return.
template <int K>
__device__ __forceinline__ void block_sums256(const double (&v)[K], int nv, double* red, double* out, int tid) {
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (q < nv) {
      double a = v[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
      if (lane == 0) red[q * 4 + wave] = a;
    }
  }
  __syncthreads();
  if (tid < nv) out[tid] = (red[tid * 4] + red[tid * 4 + 1]) + (red[tid * 4 + 2] + red[tid * 4 + 3]);
  __syncthreads();
}

// Largest RAS box: b + 2 o <= 32 cells per side
constexpr int kMaxBoxSide = 32;
constexpr int kMaxNloc = 2 * kMaxBoxSide * (kMaxBoxSide + 1) + kMaxBoxSide * kMaxBoxSide;

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
// grid ops
template <typename T>
void launch_apply(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx,
                  FootView<T> fy, int N, int M, StokesCoef<T> c, bool transpose, hipStream_t s);
// L_IB w (b != null: b - L_IB w) with the first Gram-Schmidt pass fused:
// partial[blk * nvec + q] = block sums of V_q . y (V = null: nvec = 1, y . y)
// over apply_blocks(N) blocks; nvec <= 9
template <typename T>
void launch_apply_dots(const T* w, T* y, const T* b, const T* F, const T* G, FootView<T> fx, FootView<T> fy,
                       int N, int M, StokesCoef<T> c, const T* V, int nvec, size_t vstride, double* partial,
                       hipStream_t s);
int apply_blocks(int N);
template <typename T>
struct CsrT {
  const int* ptr;
  const int* col;
  const T* val;
};
template <typename T>
void launch_ib_spmv(const T* x, T* G, CsrT<T> tu, CsrT<T> tv, int N, hipStream_t s);
template <typename T>
void launch_restrict(const T* fine, T* coarse, int Nc, hipStream_t s);
// the same, and partial[0..restrict_blocks(Nc)) = per-block sums of the
// squared coarse values (launch_scale_red reduces them)
template <typename T>
void launch_restrict_norm(const T* fine, T* coarse, int Nc, double* partial, hipStream_t s);
int restrict_blocks(int Nc);
template <typename T>
void launch_prolong_add(const T* coarse, T* fine, int Nc, hipStream_t s);
template <typename Ts, typename Td>
void launch_cast(const Ts* a, Td* b, size_t n, hipStream_t s);
template <typename T>
void launch_fill(T* a, T v, size_t n, hipStream_t s);
// y += x
template <typename T>
void launch_axpy(T* y, const T* x, size_t n, hipStream_t s);
// *flag = 1 if a[0..n) holds NaN or Inf (flag is left alone otherwise)
template <typename T>
void launch_count_nonfinite(const T* a, size_t n, int* flag, hipStream_t s);

// Krylov helpers (T = vector type, reductions in double)
template <typename T>
void launch_dots(const T* V, int nvec, size_t stride, const T* t, size_t n, double* partial,
                 int nblk, hipStream_t s);
void launch_dots_finish(const double* partial, int nvec, int nblk, double* out1, double* out2,
                        int mode, hipStream_t s);
template <typename T>
void launch_update(T* t, const T* V, int nvec, size_t stride, const double* coef, double sign,
                   size_t n, hipStream_t s);
template <typename T>
void launch_scale(const T* t, T* v, const double* denom, size_t n, hipStream_t s);
template <typename T>
void launch_combine(T* x, const T* Z, int k, size_t stride, const double* y, size_t n,
                    hipStream_t s);
void launch_small_ls(double* H, int ldh, int k, const double* beta, double* y, hipStream_t s);
void launch_givens(double* H, int ldh, int k, double* cs, double* sn, double* g, double* res,
                   hipStream_t s);
void launch_backsolve(const double* H, int ldh, int k, const double* g, double* y, hipStream_t s);
template <typename T>
void launch_block_sums(const T* a, int N, double* partial, int nblk, hipStream_t s);
template <typename T>
void launch_subtract_means(T* a, int N, const double* sums, int nvel, hipStream_t s);

// blocks of the deterministic reductions (depends only on n and cap);
// consumers re-reduce blocks x vectors partials, so long bases use a lower cap
int dots_blocks(size_t n, int cap = 256);

// fused Gram-Schmidt passes (krylov_kernels.hip); nblk = producer blocks
// nblk_in: blocks of the producer of pin (<= 0: nblk)
template <typename T>
void launch_upd_dots(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk,
                     double* hcol, double* pout, hipStream_t s, int nblk_in = 0);
// store = false: only the partial sums of |t - V h2|^2, t left unchanged
template <typename T>
void launch_upd_norm(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk,
                     double* hcol, double* pout, hipStream_t s, int nblk_in = 0, bool store = true);
template <typename T>
void launch_scale_red(const T* t, T* v, size_t n, const double* pin, int nblk, double* hout,
                      hipStream_t s);
// npart != null: H[k][k-1] = sqrt(sum of the nnblk partials at npart),
// stored into H by the kernel.  pass2: npart holds launch_upd_dots_n's
// partials of the last column instead (its second-pass coefficients and the
// squared norm before them, k + 1 per block), added to that column inside
// the kernel
template <typename T>
void launch_combine_ls(T* x, const T* Z, int k, size_t stride, size_t n, double* H, int ldh,
                       const double* beta, double* yout, hipStream_t s, bool assign = false,
                       const double* npart = nullptr, int nnblk = 0, bool pass2 = false);
// launch_upd_dots whose partials also carry |t|^2 of the updated t (k + 1
// values per block, the norm last; k <= 8)
template <typename T>
void launch_upd_dots_n(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk,
                       double* hcol, double* pout, hipStream_t s, int nblk_in = 0);
// from those partials: t = (t - V h2) / |t - V h2| with the norm taken as
// sqrt(|t|^2 - |h2|^2); hcol[0..k) += h2, hcol[k] = the norm
template <typename T>
void launch_scale_upd(T* t, const T* V, int k, size_t stride, size_t n, const double* pin, int nblk_in,
                      double* hcol, hipStream_t s);

// immersed boundary
void launch_fp_fine(const double* X, int M, int N, int comp, const int* base, const int* mask,
                    double* w, hipStream_t s);
// sw[e] = w[ent[e]] for n entries (face-ordered copy of the weights)
template <typename T>
void launch_gather_weights(const double* w, const int* ent, size_t n, T* sw, hipStream_t s);
void launch_fp_coarsen(const int* fbase, const double* fw, const int* cbase, int M, int comp,
                       int Nf, int Nc, double* cw, hipStream_t s);
// walk-ordered copies of one component's window bases and weights
template <typename T>
void launch_walk_order(const int* order, const int* base, const T* w, int M, int* obase, T* ow, hipStream_t s);
template <typename T>
void launch_ib_force(const T* u, const T* v, FootView<T> fx, FootView<T> fy, SpringView<T> sv,
                     int N, T* U, T* F, hipStream_t s);   // U: [M][2] scratch (J u, interleaved)
template <typename T>
void launch_interp(const T* u, const T* v, FootView<T> fx, FootView<T> fy, int M, int N,
                   T* U, hipStream_t s);
void launch_spread(const double* F, FootView<double> fx, FootView<double> fy, int M, int N,
                   double scale, double* f, hipStream_t s);
// rows of component comp; f0/f1 and mask0/mask1 the level's two components.
// nslice > 1 splits each row's point list over that many waves, whose sums
// go to part (nslice x nnz doubles) and are added in slice order.
void launch_t_values(FootView<double> f0, FootView<double> f1, const int* mask0, const int* mask1,
                     SpringView<double> sv, int comp, int N, double ibs, const int* t_ptr,
                     const int* t_col, double* t_val, int nslice, size_t nnz, double* part, hipStream_t s);
// semi-implicit time step pieces (Sec. 2.2): spring forces on the periodic
// square, the step's right-hand side, the position update
// kap: kappa_e per incidence; rest: rest length per incidence, nullptr for
// zero rest lengths
void launch_fibre_force(const double* X, SpringView<double> sv, const double* kap, const double* rest, double* F,
                        hipStream_t s);
void launch_step_rhs(const double* w, const double* f, double a, int N, double* rhs, hipStream_t s);
void launch_advance(double* X, const double* U, double dt, int M, hipStream_t s);
// blocks: per spring (B_xx, B_xy, B_yy) of K_e / kappa_e, nullptr for B = I
void launch_spring_grad(const double* Uw, const double* Ul, const int* ends, const double* blocks,
                        int n_springs, double scale, double* out, hipStream_t s);
// The allocation-free gradient's scratch: a file-scope device array of
// 4 kStaticGradPoints doubles (J w and J lambda); its device address on the
// current device, looked up once per device.
constexpr int kStaticGradPoints = 1 << 18;
double* static_grad_scratch();

// dense boxes and coarsest solve
void launch_patch_assemble(const int* patch_ids, int count, BoxGeom g, StokesCoef<double> c,
                           const int* tptr_u, const int* tcol_u, const double* tval_u,
                           const int* tptr_v, const int* tcol_v, const double* tval_v,
                           double* mats, hipStream_t s);
// In-place block sweeps of count symmetric n x n matrices: afterwards the
// tiles on or below the diagonal (64 x 64, diagonal tiles in full) hold
// -A^{-1}; launch_extract_owned reads them.  work: count x 3 x n x 64 and
// dinv: count x 64 x 64 doubles of workspace.
void launch_gj_invert(double* mats, int n, int count, double* work, double* dinv, hipStream_t s);
constexpr int kGjNb = 128;  // block width of the batched inversion
// full: every row of the inverse (g.nown = nloc, the summed combination)
template <typename T>
void launch_extract_owned(const double* mats, int count, BoxGeom g, T* out, hipStream_t s, bool full = false);
// Summed additive Schwarz (IBMG_COMBINE_SUM): every box's whole local
// solution L_k^{-1} R_k r into Y (box id-major, g.nch chunks of 64 rows; inv
// holds full inverses, box_inv[box id] the inverse of each box), then every
// unknown z = the sum of its entries over the boxes whose index set holds it
// (boxes in a fixed order per unknown).
template <typename T>
void launch_asm_apply(const T* r, T* z, BoxGeom g, const T* inv, const int* box_inv, T* Y, hipStream_t s);
// parts: bit 0 = IB boxes (k_ras_ib), bit 1 = interior boxes
// (k_ras_interior); the smoother launches both, and one k_ras_sum adds the
// slices of whichever was split.
// acc: add the local solutions to z on the owned sets instead of storing them;
// tb: interior product form (16 or 32 boxes per tile, 64: register-blocked
// 64 x 64 tiles, 128: residuals gathered into xg (at least
// int_gather_elems(g, n_int) elements) and 64 x 128 tiles; results do not
// depend on it)
// Symmetric storage of the IB boxes' owned rows (restricted sweep): chunk c
// keeps the owned columns of tiles 0..c and every non-owned column, in the
// permuted local order perm (owned unknowns first, in owned order); the
// owned columns of later tiles are added as the transposed column sums of
// the chunks that hold them, through per-box partials.
struct SymIB {
  const void* inv;   // T[n_ib * sym_box_stride(g)]
  const int* perm;   // [nloc]
  void* part;        // T[n_ib * sym_part_len(g, n_ib)]
};
size_t sym_box_stride(const BoxGeom& g);
// partials per box (the column slices follow the IB-box kernel's split)
int sym_part_len(const BoxGeom& g, int n_ib);
template <typename T>
void launch_extract_sym(const double* mats, int count, BoxGeom g, const int* perm, T* out, hipStream_t s);

// sym != null: the IB boxes run from the symmetric storage (parts & 1),
// their rows summed with the interior slices in one launch
template <typename T>
void launch_ras_apply(const T* r, T* z, BoxGeom g, const T* inv, const int* ib_boxes, int n_ib,
                      const T* shared_inv, const int* int_boxes, int n_int, const int* loc_tab,
                      T* part, hipStream_t s, int parts = 3, bool acc = false, int tb = 32, T* xg = nullptr,
                      size_t xg_elems = 0, const SymIB* sym = nullptr);
size_t int_gather_elems(const BoxGeom& g, int n_int);
// reduction slices of the interior-box product (part holds ksplit * n_int * nch * 64)
int ras_interior_ksplit(const BoxGeom& g, int n_int);
// interior product forms (launch_ras_apply's tb): 16, 32 = boxes per tile of
// the narrow kernels, 64 = register-blocked tiles, 128 = gathered operand,
// kIntFormPipe = the pipelined XCD-ordered 64-box tiles
constexpr int kIntFormPipe = 1;
// column slices of the IB-box kernel (part holds ksplit * n_ib * nch * 64,
// followed by the interior product's slices when both are launched)
int ras_ib_ksplit(const BoxGeom& g, int n_ib);
void launch_coarse_assemble(int N, StokesCoef<double> c, const int* tptr_u, const int* tcol_u,
                            const double* tval_u, const int* tptr_v, const int* tcol_v,
                            const double* tval_v, int nb, double* aug, hipStream_t s);
// count augmented systems [A | I] (n x 2n each, stride doubles apart), a work-group each
void launch_coarse_invert(double* aug, int n, int count, size_t stride, hipStream_t s);
void launch_coarse_extract(const double* aug, int n, int n0, double* inv, hipStream_t s);
template <typename T>
void launch_coarse_apply(const double* inv, int n0, const T* r, T* z, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched forms: nsys systems of one grid size stored back to back (system
// stride bs), or ragged batches described by a BSeg.  Per-system scalars
// (partial sums, Hessenberg columns, norms) sit at fixed strides.
// ---------------------------------------------------------------------------
template <typename T>
void launch_apply_batch(const T* w, T* y, const T* b, int N, StokesCoef<T> c, int nsys, size_t bs,
                        hipStream_t s);
// y[rows[q]] += sign * sum_k val[k] x[col[k]], k in [ptr[q], ptr[q+1])
template <typename T>
void launch_ib_rows(const T* x, T* y, const int* rows, const int* ptr, const int* col, const T* val,
                    int nrows, T sign, hipStream_t s);
template <typename T>
void launch_restrict_batch(const T* fine, T* coarse, int Nc, int nsys, hipStream_t s);
template <typename T>
void launch_prolong_add_batch(const T* coarse, T* fine, int Nc, int nsys, hipStream_t s);
template <typename T>
void launch_dots_b(const T* V, int nvec, size_t stride, const T* t, BSeg sg, int nsys, double* partial,
                   size_t pstride, int nblk, hipStream_t s);
void launch_dots_finish_b(const double* partial, int nvec, int nblk, size_t pstride, double* out1,
                          double* out2, size_t ostride, int mode, int nsys, hipStream_t s);
template <typename T>
void launch_scale_b(const T* t, T* v, const double* denom, size_t dstride, BSeg sg, int nsys,
                    size_t nmax, hipStream_t s);
template <typename T>
void launch_combine_b(T* x, const T* Z, size_t stride, const double* y, size_t ystride, const int* kcnt,
                      BSeg sg, int nsys, size_t nmax, hipStream_t s);
void launch_givens_b(double* H, int ldh, size_t hstride, int k, double* cs, double* sn, double* g,
                     size_t rstride, double* res, const int* active, int nsys, hipStream_t s);
void launch_backsolve_b(const double* H, int ldh, size_t hstride, const int* kcnt, const double* g,
                        double* y, size_t rstride, int nsys, hipStream_t s);
template <typename T>
void launch_block_sums_b(const T* a, int N, size_t bs, double* partial, int nblk, size_t pstride, int nsys,
                         hipStream_t s);
template <typename T>
void launch_subtract_means_b(T* a, int N, size_t bs, const double* sums, size_t sstride, int nvel, int nsys,
                             hipStream_t s);
// with_norm: as launch_upd_dots_n (k + 1 partials per block, |t|^2 last)
template <typename T>
void launch_upd_dots_b(T* t, const T* V, int k, size_t stride, BSeg sg, int nsys, const double* pin,
                       int nblk, size_t pstride, double* hcol, size_t hstride, double* pout, hipStream_t s,
                       int nblk_in = 0, bool with_norm = false);
// launch_scale_upd on every active system
template <typename T>
void launch_scale_upd_b(T* t, const T* V, int k, size_t stride, BSeg sg, int nsys, size_t nmax,
                        const double* pin, int nblk_in, size_t pstride, double* hcol, size_t hstride,
                        hipStream_t s);
template <typename T>
void launch_upd_norm_b(T* t, const T* V, int k, size_t stride, BSeg sg, int nsys, const double* pin,
                       int nblk, size_t pstride, double* hcol, size_t hstride, double* pout, hipStream_t s,
                       int nblk_in = 0, bool store = true);
template <typename T>
void launch_scale_red_b(const T* t, T* v, BSeg sg, int nsys, size_t nmax, const double* pin, int nblk,
                        size_t pstride, double* hout, size_t hstride, hipStream_t s);
template <typename T>
void launch_combine_ls_b(T* x, const T* Z, int k, size_t stride, BSeg sg, int nsys, size_t nmax,
                         double* H, int ldh, size_t hstride, const double* beta, double* yout,
                         size_t sstride, hipStream_t s, bool assign = false, const double* npart = nullptr,
                         int nnblk = 0, size_t pstride = 0, bool pass2 = false);
template <typename T>
void launch_coarse_apply_batch(const double* inv, int n0, const T* r, T* z, int nsys, hipStream_t s);

// One persistent launch per smoother sweep over every (system, box) of a
// batch level: interior tiles of TB boxes on the matrix cores against the
// shared interior inverse, then (IB box, row chunk) items against each box's
// own inverse.  Box entries are s * nbox + box id; systems are sys_n apart.
struct RasBatchPlan {
  int tb = 32;      // interior tile width (16, 32, or 64: register-blocked)
  int grid = 0;     // work-groups of the persistent launch
};
template <typename T>
void launch_ras_batch(const T* r, T* z, BoxGeom g, size_t sys_n, int nbox, const T* shared_inv,
                      const int* int_ents, int n_int, const int* ib_ents, const T* const* ib_inv, int n_ib,
                      const int* loc_tab, const int* active, RasBatchPlan plan, hipStream_t s);
int ras_batch_items(const BoxGeom& g, int n_int, int n_ib, int tb);

}  // namespace ibmg
