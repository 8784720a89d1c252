// Host orchestration: hierarchy set-up, the V-cycle of Alg. 1 with
// FGMRES-wrapped smoothing (Sec. 3.3), and the outer flexible GMRES solve.
// Every arithmetic step runs in the kernels; the host builds index structures
// (footprint windows, face -> point lists, IB row patterns, box classes) and
// sequences launches on one stream.
#pragma once

#include <atomic>
#include <map>
#include <numeric>
#include <thread>
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <type_traits>

#include "sc_smoother.hpp"
#include "solver.hpp"

namespace ibmg {

namespace detail {

constexpr int kMaxNu = 8;
constexpr int kMaxRestart = 64;
constexpr int kScalY = 1;     // scal[1..16]: least-squares solution
constexpr int kScalTmp = 20;  // scal[20..]: second Gram-Schmidt pass
// Levels whose longest face -> point list exceeds this use the explicit
// Galerkin IB rows (one wave per row) for the IB term.
constexpr int kSpmvListThreshold = 24;
// partial-sum buffers: two of kPartStride doubles (blocks x vectors)
constexpr size_t kPartStride = (size_t)256 * 65;
// the outer solve's Gram-Schmidt passes: up to kOuterBlocks blocks of up to
// 65 vectors, folded by one block before their consumers
constexpr int kOuterBlocks = 1024;
constexpr size_t kOuterPartStride = (size_t)kOuterBlocks * 65;

inline int wrapn(int a, int N) {
  a %= N;
  return a < 0 ? a + N : a;
}

inline std::vector<int> level_sizes(int N, int coarse) {
  std::vector<int> s;
  for (int n = N; n >= coarse; n /= 2) {
    s.push_back(n);
    if (n == coarse) break;
  }
  std::reverse(s.begin(), s.end());
  return s;
}

inline void box_params(int N, int box, int overlap, int* b, int* o) {
  *b = std::min(box, N / 2);
  *o = std::min(overlap, (N - *b - 1) / 2);
  if (*o < 0) *o = 0;
}

}  // namespace detail

using namespace detail;

template <typename T>
struct Level {
  int N = 0;
  CompFoot f[2];
  // IB term from the explicit Galerkin rows (wave per row) instead of the
  // interpolate / spring / spread chain: chosen where points crowd the faces
  bool use_spmv = false;
  DBuf<double> Gd;
  DBuf<T> Gt;
  StokesCoef<double> cd{};
  StokesCoef<T> ct{};
  // restricted additive Schwarz
  BoxGeom g{};
  int n_unique = 0, n_ib = 0;
  std::vector<int> uniq;  // unique box ids (IB boxes, then one interior representative)
  std::vector<int> ib_list, int_list;
  std::vector<int> loc_tab;  // local unknown -> (comp << 24) | (jj << 12) | ii, then -> comp N^2 + jj N + ii
  DBuf<int> d_ib, d_int, d_loc;
  DBuf<T> inv;            // [n_unique][nch][nloc][64]
  DBuf<T> int_part;       // reduction slices of the interior-box product
  DBuf<T> int_x;          // gathered residuals of the interior boxes (product form 128)
  // symmetric storage of the IB boxes' owned rows (restricted additive
  // sweep): the permuted local order, the storage, the per-box partials
  bool use_sym = false;
  DBuf<int> d_perm;
  DBuf<T> inv_sym, sym_part;
  // restricted multiplicative Schwarz: box colours; ib_list and int_list
  // sorted by colour, colour c spanning [ib_off[c], ib_off[c+1]) and
  // [int_off[c], int_off[c+1])
  int ncolour = 0;
  std::vector<int> box_colour, ib_off, int_off;
  int int_tb = 32;        // interior tile width, picked by timing at set-up
  DBuf<T> rr;             // residual between colours
  // summed combination (IBMG_COMBINE_SUM): g.nown = nloc, every row of every
  // box inverse is kept; box_inv maps a box id to its inverse (IB boxes their
  // own, interior boxes the shared one), Y holds every box's local solution
  bool sum_mode = false;
  DBuf<int> d_box_inv;
  DBuf<T> Y;
  // work vectors
  DBuf<T> w, b, r, t, V, Z, F;
  DBuf<double> H, scal, part;
  // Schur-complement smoother
  std::unique_ptr<ScLevel<T>> sc;
};

template <typename T>
class BatchSolver;

template <typename T>
class Solver final : public SolverBase {
  friend class BatchSolver<T>;

 public:
  // defer_coarse: assemble the coarsest system but leave its inversion to
  // the caller (the batched form inverts every system's in one launch and
  // hands each back through finish_coarse)
  Solver(const ibmg_desc& d, hipStream_t s, bool defer_coarse = false) : d_(d), defer_coarse_(defer_coarse) {
    M_ = d.M;
    E_ = d.n_springs;
    X_.assign(d.X, d.X + 2 * (size_t)M_);
    ends_.assign(d.ends, d.ends + 2 * (size_t)E_);
    kappa_.assign(d.kappa, d.kappa + E_);
    tangent_ = d.spring_model == IBMG_SPRING_TANGENT;
    rest_.assign(E_, 0.0);
    if (d.rest) rest_.assign(d.rest, d.rest + E_);
    // the descriptor's host arrays belong to the caller
    d_.X = nullptr;
    d_.ends = nullptr;
    d_.kappa = nullptr;
    d_.rest = nullptr;
    nu_ = std::max(d.nu1, d.nu2);
    sizes_ = level_sizes(d.N, d.coarse_N);
    L_ = (int)sizes_.size() - 1;
    outer_cap_ = d.max_restart > 0 ? d.max_restart : 30;
    alloc_fixed(s);
    build_all(s);
  }

  // Buffers whose sizes do not depend on the structure's positions, placed
  // first in the workspace: a rebuild at moved positions releases everything
  // above them and lays it out again in the same order.  A member of a batch
  // keeps only its hierarchy (the batch has its own work and outer vectors).
  void alloc_fixed(hipStream_t s) {
    (void)s;
    if (defer_coarse_) return;
    const size_t n = 3 * (size_t)d_.N * d_.N, m2 = 2 * (size_t)std::max(M_, 1);
    const int R = outer_cap_;
    Vo_.alloc((size_t)(R + 1) * n);
    Zo_.alloc((size_t)R * n);
    Ho_.alloc((size_t)(R + 1) * R);
    cs_.alloc(R + 1);
    sn_.alloc(R + 1);
    g_.alloc(R + 2);
    y_.alloc(R + 1);
    osc_.alloc(256);
    opart_.alloc(2 * kOuterPartStride);
    ofold_.alloc(2 * 72);
    bp_.alloc(n);
    rr_.alloc(n);
    vin_.alloc(n);
    vout_.alloc(n);
    Fd_.alloc(2 * m2);   // forces [2][M] then J u [2][M]
    Uw_.alloc(m2);
    Ul_.alloc(m2);
    Fs_.alloc(m2);
    fs_.alloc(2 * (size_t)d_.N * d_.N);
    rhs_.alloc(n);
    if (!pinned_) IBMG_HIP(hipHostMalloc((void**)&pinned_, 8 * sizeof(double), hipHostMallocDefault));
  }

  // Every position-dependent part of the set-up, in workspace order.  With
  // IBMG_SETUP_TIMES set in the environment each phase waits for the device
  // and its wall time goes to stderr (a measurement aid; it serialises the
  // phases).
  void build_all(hipStream_t s) {
    const bool timed = std::getenv("IBMG_SETUP_TIMES") != nullptr;
    auto t = std::chrono::steady_clock::now();
    const auto t_begin = t;
    auto mark = [&](const char* what) {
      if (!timed) return;
      IBMG_HIP(hipStreamSynchronize(s));
      const auto now = std::chrono::steady_clock::now();
      std::fprintf(stderr, "[ibmg set-up] %-16s %8.3f ms\n", what,
                   std::chrono::duration<double, std::milli>(now - t).count());
      t = now;
    };
    build_structure(s, mark);
    if (!defer_coarse_) alloc_work(s);
    mark("work buffers");
    build_numeric(s, mark);
    check_breakdown(s);
    mark("breakdown scan");
    if (!defer_coarse_) tune_interior(s);
    mark("interior tuning");
    IBMG_HIP(hipStreamSynchronize(s));
    setup_ms_ = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
  }

  // Release everything alloc_fixed did not place (the whole hierarchy, the
  // structure's device arrays, the coarsest inverse and the set-up's slice
  // buffer), leaving the workspace as it was right after alloc_fixed.
  void release_dependent() {
    if (coarse_aug_.n) {   // a set-up that stopped before joining the coarsest inversion
      if (side_) IBMG_HIP(hipStreamSynchronize(side_));
      coarse_aug_.release();
    }
    levels_.clear();
    for (DBuf<int>* b : {&d_adj_ptr_, &d_adj_nbr_, &d_ends_, &d_order_}) b->release();
    for (DBuf<double>* b : {&d_adj_k_, &d_X_, &d_adj_k2_, &d_adj_kap_, &d_adj_rest_, &d_gblocks_, &inv0_, &tpart_,
                            &aug0_})
      b->release();
    d_adj_kf_.release();
    d_adj_k2f_.release();
  }

  // A set-up factorisation that broke down leaves non-finite entries in its
  // inverse (a zero pivot divides by zero); so does a non-finite operator.
  // The coarsest inverse and every level's box inverses are scanned once,
  // and the SC Chebyshev bounds must be finite and positive.
  void check_breakdown(hipStream_t s, bool coarse_only = false) {
    DBuf<int> flag(1);
    if (dry_run()) return;
    int bad = 0;
    auto scan = [&](const auto* a, size_t n, const char* what) {
      if (!n) return;
      launch_fill<int>(flag.p, 0, 1, s);
      launch_count_nonfinite(a, n, flag.p, s);
      IBMG_HIP(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
      IBMG_HIP(hipStreamSynchronize(s));
      if (bad) throw Error(IBMG_ERR_BREAKDOWN, std::string(what) + " has non-finite entries (singular or non-finite matrix)");
    };
    if (inv0_.n) scan(inv0_.p, inv0_.n, "the coarsest inverse");
    for (int l = 1; l <= L_ && !coarse_only; ++l) {
      Level<T>& lev = levels_[l];
      if (lev.inv.n) scan(lev.inv.p, lev.inv.n, ("the box inverses of level " + std::to_string(l)).c_str());
      if (lev.inv_sym.n) scan(lev.inv_sym.p, lev.inv_sym.n, ("the IB box inverses of level " + std::to_string(l)).c_str());
      if (lev.sc)
        if (!(std::isfinite(lev.sc->lamA) && lev.sc->lamA > 0.0 && std::isfinite(lev.sc->lamM) && lev.sc->lamM > 0.0))
          throw Error(IBMG_ERR_BREAKDOWN, "Schur-complement Chebyshev bound of level " + std::to_string(l) +
                                              " is not finite and positive");
    }
  }

  ~Solver() override {
    if (est_ev_) (void)hipEventDestroy(est_ev_);
    if (side_) {
      (void)hipStreamSynchronize(side_);
      (void)hipStreamDestroy(side_);
      (void)hipEventDestroy(ev_fork_);
      (void)hipEventDestroy(ev_join_);
    }
    drop_graph();
    if (gstream_) (void)hipStreamDestroy(gstream_);
    if (pinned_) (void)hipHostFree(pinned_);
  }

  int levels() const override { return L_ + 1; }
  int level_n(int l) const override { return sizes_.at(l); }

  // ---------------------------------------------------------------- set-up
  template <typename Mark>
  void build_structure(hipStream_t s, Mark& mark) {
    // spring adjacency (node -> incident springs in spring order)
    adj_ptr_.assign(M_ + 1, 0);
    for (int e = 0; e < E_; ++e) {
      adj_ptr_[ends_[2 * e] + 1]++;
      adj_ptr_[ends_[2 * e + 1] + 1]++;
    }
    for (int l = 0; l < M_; ++l) adj_ptr_[l + 1] += adj_ptr_[l];
    adj_nbr_.assign(adj_ptr_[M_], 0);
    adj_sid_.assign(adj_ptr_[M_], 0);
    {
      std::vector<int> fill(adj_ptr_.begin(), adj_ptr_.end() - 1);
      for (int e = 0; e < E_; ++e) {
        const int a = ends_[2 * e], b = ends_[2 * e + 1];
        adj_nbr_[fill[a]] = b;
        adj_sid_[fill[a]++] = e;
        adj_nbr_[fill[b]] = a;
        adj_sid_[fill[b]++] = e;
      }
    }
    d_adj_ptr_.upload(adj_ptr_, s);
    d_adj_nbr_.upload(adj_nbr_, s);
    d_ends_.upload(ends_, s);
    d_X_.upload(X_, s);
    levels_.resize(L_ + 1);
    for (int l = L_; l >= 0; --l) {
      Level<T>& lev = levels_[l];
      lev.N = sizes_[l];
      const double h = 1.0 / lev.N;
      lev.cd = StokesCoef<double>{d_.rho / d_.dt, d_.mu / (h * h), 1.0 / h, d_.dt / (h * h)};
      lev.ct = StokesCoef<T>{(T)lev.cd.alpha, (T)lev.cd.beta, (T)lev.cd.gi, (T)lev.cd.ibs};
      for (int c = 0; c < 2; ++c) {
        CompFoot& f = lev.f[c];
        if (l == L_) fine_windows(lev.N, c, f);
        else coarse_windows(levels_[l + 1].f[c], c, levels_[l + 1].N, lev.N, f);
        f.d_base.upload(f.base, s);
        f.d_mask.upload(f.mask, s);
        f.w.alloc((size_t)M_ * 16);
        if (l == L_)
          launch_fp_fine(d_X_.p, M_, lev.N, c, f.d_base.p, f.d_mask.p, f.w.p, s);
        else
          launch_fp_coarsen(levels_[l + 1].f[c].d_base.p, levels_[l + 1].f[c].w.p, f.d_base.p, M_, c,
                            levels_[l + 1].N, lev.N, f.w.p, s);
        if (std::is_same<T, float>::value) {
          f.wf.alloc((size_t)M_ * 16);
          launch_cast<double, float>(f.w.p, f.wf.p, (size_t)M_ * 16, s);
        }
        spread_lists(lev.N, f);
        f.d_sp_ptr.upload(f.sp_ptr, s);
        f.d_sp_ent.upload(f.sp_ent, s);
        f.sw.alloc(std::max<size_t>(f.sp_ent.size(), 1));
        launch_gather_weights<double>(f.w.p, f.d_sp_ent.p, f.sp_ent.size(), f.sw.p, s);
        if (std::is_same<T, float>::value) {
          f.swf.alloc(std::max<size_t>(f.sp_ent.size(), 1));
          launch_gather_weights<float>(f.w.p, f.d_sp_ent.p, f.sp_ent.size(), f.swf.p, s);
        }
        if (l == L_ && c == 0) point_order(lev.N, f, s);
        // the interpolation walks points in cell order and reads their
        // windows there, so it gets copies laid out in that order
        f.d_obase.alloc(2 * (size_t)M_);
        f.ow.alloc((size_t)M_ * 16);
        launch_walk_order<double>(d_order_.p, f.d_base.p, f.w.p, M_, f.d_obase.p, f.ow.p, s);
        if (std::is_same<T, float>::value) {
          f.owf.alloc((size_t)M_ * 16);
          launch_walk_order<float>(d_order_.p, f.d_base.p, f.wf.p, M_, f.d_obase.p, f.owf.p, s);
        }
      }
    }
    mark("windows, lists");
    ib_patterns();   // IB rows need both components' windows
    mark("IB row patterns");
    for (int l = L_; l >= 0; --l) {
      Level<T>& lev = levels_[l];
      for (int c = 0; c < 2; ++c) {
        CompFoot& f = lev.f[c];
        f.d_tptr.upload(f.tptr, s);
        f.d_tcol.upload(f.tcol, s);
        f.tval.alloc(f.tcol.size());
        if (std::is_same<T, float>::value) f.tvalf.alloc(f.tcol.size());
        f.max_list = 0;
        for (size_t r = 0; r + 1 < f.sp_ptr.size(); ++r)
          f.max_list = std::max(f.max_list, f.sp_ptr[r + 1] - f.sp_ptr[r]);
      }
      lev.use_spmv = std::max(lev.f[0].max_list, lev.f[1].max_list) > kSpmvListThreshold;
      if (l >= 1 && (d_.smoother == IBMG_RAS || d_.smoother == IBMG_RMS)) classify_boxes(lev);
      if (l >= 1 && d_.smoother == IBMG_RMS) colour_boxes(lev);
      if (l >= 1 && d_.smoother == IBMG_SC) sc_structure(lev, s);
    }
    mark("box classes");
  }

  // Points in cell order (row-major by the finest x-window base, ties in
  // index order), the order in which the point-wise kernels walk them.
  void point_order(int N, const CompFoot& f, hipStream_t s) {
    std::vector<int> ord(std::max(M_, 1), 0);
    std::iota(ord.begin(), ord.begin() + M_, 0);
    std::stable_sort(ord.begin(), ord.begin() + M_, [&](int a, int b) {
      const long long ka = (long long)f.base[2 * a + 1] * N + f.base[2 * a];
      const long long kb = (long long)f.base[2 * b + 1] * N + f.base[2 * b];
      return ka < kb;
    });
    d_order_.upload(ord, s);
  }

  // Finest windows: t = X N - shift, i0 = floor(t) - 1, slots with |t - k| < 2.
  void fine_windows(int N, int comp, CompFoot& f) {
    f.base.assign(2 * (size_t)M_, 0);
    f.mask.assign(M_, 0);
    const double sx = comp == 0 ? 0.0 : 0.5, sy = comp == 0 ? 0.5 : 0.0;
    for (int l = 0; l < M_; ++l) {
      const double tx = X_[2 * l] * N - sx, ty = X_[2 * l + 1] * N - sy;
      const int i0 = (int)std::floor(tx) - 1, j0 = (int)std::floor(ty) - 1;
      int mk = 0;
      for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a)
          if (std::fabs(tx - (i0 + a)) < 2.0 && std::fabs(ty - (j0 + b)) < 2.0) mk |= 1 << (b * 4 + a);
      f.base[2 * l] = wrapn(i0, N);
      f.base[2 * l + 1] = wrapn(j0, N);
      f.mask[l] = mk;
    }
  }

  // Coarse windows: base = fine base / 2; a coarse slot is structural when a
  // structural fine slot is interpolated from it by P_u.
  void coarse_windows(const CompFoot& ff, int comp, int Nf, int Nc, CompFoot& f) {
    (void)Nf;
    f.base.assign(2 * (size_t)M_, 0);
    f.mask.assign(M_, 0);
    for (int l = 0; l < M_; ++l) {
      const int I0 = ff.base[2 * l], J0 = ff.base[2 * l + 1];
      const int ci0 = I0 >> 1, cj0 = J0 >> 1;
      int mk = 0;
      for (int s = 0; s < 16; ++s) {
        if (!((ff.mask[l] >> s) & 1)) continue;
        const int I = I0 + (s & 3), J = J0 + (s >> 2);
        if (comp == 0) {
          const int cj = (J >> 1) - cj0;
          if ((I & 1) == 0) mk |= 1 << (cj * 4 + (I >> 1) - ci0);
          else mk |= (1 << (cj * 4 + ((I - 1) >> 1) - ci0)) | (1 << (cj * 4 + ((I + 1) >> 1) - ci0));
        } else {
          const int ci = (I >> 1) - ci0;
          if ((J & 1) == 0) mk |= 1 << (((J >> 1) - cj0) * 4 + ci);
          else mk |= (1 << ((((J - 1) >> 1) - cj0) * 4 + ci)) | (1 << ((((J + 1) >> 1) - cj0) * 4 + ci));
        }
      }
      f.base[2 * l] = wrapn(ci0, Nc);
      f.base[2 * l + 1] = wrapn(cj0, Nc);
      f.mask[l] = mk;
    }
  }

  static int face_of(const CompFoot& f, int l, int s, int N) {
    int i = f.base[2 * l] + (s & 3), j = f.base[2 * l + 1] + (s >> 2);
    if (i >= N) i -= N;
    if (j >= N) j -= N;
    return j * N + i;
  }

  // faces -> (point, slot) entries, entries of a face in increasing (l, s)
  void spread_lists(int N, CompFoot& f) {
    const size_t nf = (size_t)N * N;
    f.sp_ptr.assign(nf + 1, 0);
    for (int l = 0; l < M_; ++l)
      for (int s = 0; s < 16; ++s)
        if ((f.mask[l] >> s) & 1) f.sp_ptr[face_of(f, l, s, N) + 1]++;
    for (size_t r = 0; r < nf; ++r) f.sp_ptr[r + 1] += f.sp_ptr[r];
    f.sp_ent.assign(f.sp_ptr[nf], 0);
    std::vector<int> fill(f.sp_ptr.begin(), f.sp_ptr.end() - 1);
    for (int l = 0; l < M_; ++l)
      for (int s = 0; s < 16; ++s)
        if ((f.mask[l] >> s) & 1) f.sp_ent[fill[face_of(f, l, s, N)]++] = l * 16 + s;
  }

  // Pattern of the comp rows of dt/h^2 J^T K' J: row r couples to every face
  // of every point that shares a spring (or is itself) with a point whose
  // comp-window holds r, in the same component, and with tangent blocks also
  // in the other one.  Columns index [u | v] (v faces offset by N^2), sorted.
  // The IB rows' columns on every level and component (the Galerkin
  // pattern): one pool of worker threads takes chunks of rows of all (level,
  // component) pairs.  Each chunk keeps its own columns and the chunks join
  // in order, so the pattern does not depend on the thread count.  A worker
  // marks the columns of the row in hand with a tag it never reuses, so one
  // stamp array serves every pair without being cleared.
  void ib_patterns() {
    struct Task {
      int l, comp;
      size_t r0, r1;
    };
    constexpr size_t kChunk = 2048;
    std::vector<Task> tasks;
    std::vector<size_t> first(2 * (size_t)(L_ + 1) + 1, 0);   // first task of pair 2 l + comp
    for (int l = 0; l <= L_; ++l)
      for (int c = 0; c < 2; ++c) {
        first[2 * l + c] = tasks.size();
        const size_t nf = (size_t)levels_[l].N * levels_[l].N;
        for (size_t r0 = 0; r0 < nf; r0 += kChunk) tasks.push_back({l, c, r0, std::min(nf, r0 + kChunk)});
      }
    first[2 * (size_t)(L_ + 1)] = tasks.size();
    std::vector<std::vector<int>> ccols(tasks.size()), clen(tasks.size());
    const size_t nf_max = (size_t)levels_[L_].N * levels_[L_].N;
    std::atomic<size_t> next{0};
    auto worker = [&]() {
      std::vector<int> stamp(2 * nf_max, -1);
      std::vector<int> pstamp(std::max(M_, 1), -1);   // points already taken for this row
      std::vector<int> cols, pts;
      int tag = -1;
      for (;;) {
        const size_t ti = next++;
        if (ti >= tasks.size()) break;
        const Task& tk = tasks[ti];
        const Level<T>& lev = levels_[tk.l];
        const int N = lev.N;
        const size_t nf = (size_t)N * N;
        const CompFoot& f = lev.f[tk.comp];
        auto add_point = [&](int q) {
          for (int c = 0; c < 2; ++c) {
            if (c != tk.comp && !tangent_) continue;
            const CompFoot& fc = lev.f[c];
            for (int sl = 0; sl < 16; ++sl) {
              if (!((fc.mask[q] >> sl) & 1)) continue;
              const int col = c * (int)nf + face_of(fc, q, sl, N);
              if (stamp[col] != tag) {
                stamp[col] = tag;
                cols.push_back(col);
              }
            }
          }
        };
        std::vector<int>& out = ccols[ti];
        std::vector<int>& len = clen[ti];
        len.assign(tk.r1 - tk.r0, 0);
        // the points whose windows the row reaches: each spring-carrying
        // point in the face's list and its spring neighbours, each taken once
        auto take = [&](int q) {
          if (pstamp[q] != tag) {
            pstamp[q] = tag;
            pts.push_back(q);
          }
        };
        for (size_t r = tk.r0; r < tk.r1; ++r) {
          if (f.sp_ptr[r + 1] == f.sp_ptr[r]) continue;
          ++tag;
          cols.clear();
          pts.clear();
          for (int e = f.sp_ptr[r]; e < f.sp_ptr[r + 1]; ++e) {
            const int l = f.sp_ent[e] >> 4;
            if (adj_ptr_[l + 1] == adj_ptr_[l]) continue;
            take(l);
            for (int a = adj_ptr_[l]; a < adj_ptr_[l + 1]; ++a) take(adj_nbr_[a]);
          }
          for (int q : pts) add_point(q);
          std::sort(cols.begin(), cols.end());
          out.insert(out.end(), cols.begin(), cols.end());
          len[r - tk.r0] = (int)cols.size();
        }
      }
    };
    // each worker keeps a stamp over the finest [u | v]: at most 1 GiB in all
    const size_t by_mem = std::max<size_t>(1, ((size_t)1 << 30) / (2 * nf_max * sizeof(int)));
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nth = std::min({(size_t)16, hw, by_mem, tasks.size()});
    if (nth <= 1) {
      worker();
    } else {
      std::vector<std::thread> th;
      for (size_t t = 0; t < nth; ++t) th.emplace_back(worker);
      for (auto& t : th) t.join();
    }
    for (int l = 0; l <= L_; ++l)
      for (int c = 0; c < 2; ++c) {
        CompFoot& f = levels_[l].f[c];
        const size_t nf = (size_t)levels_[l].N * levels_[l].N;
        const size_t t0 = first[2 * l + c], t1 = first[2 * l + c + 1];
        f.tptr.assign(nf + 1, 0);
        size_t tot = 0;
        for (size_t t = t0; t < t1; ++t) tot += ccols[t].size();
        f.tcol.clear();
        f.tcol.reserve(tot);
        for (size_t t = t0; t < t1; ++t) {
          for (size_t i = 0; i < clen[t].size(); ++i) f.tptr[tasks[t].r0 + i + 1] = clen[t][i];
          f.tcol.insert(f.tcol.end(), ccols[t].begin(), ccols[t].end());
        }
        for (size_t r = 0; r < nf; ++r) f.tptr[r + 1] += f.tptr[r];
      }
  }

  // A box needs its own inverse when one of its faces carries an IB row;
  // every other box has the same (translation-invariant) matrix.
  void classify_boxes(Level<T>& lev) {
    int b, o;
    box_params(lev.N, d_.box, d_.overlap, &b, &o);
    const int m = b + 2 * o, N = lev.N;
    lev.g = BoxGeom{N, b, o, m, N / b, 2 * m * (m + 1) + m * m, 3 * b * b, (3 * b * b + 63) / 64};
    const int nbox = lev.g.npd * lev.g.npd;
    lev.uniq.clear();
    lev.ib_list.clear();
    lev.int_list.clear();
    for (int p = 0; p < nbox; ++p) {
      const int x0 = (p % lev.g.npd) * b - o, y0 = (p / lev.g.npd) * b - o;
      bool ib = false;
      for (int jj = 0; jj <= m && !ib; ++jj)
        for (int ii = 0; ii <= m && !ib; ++ii) {
          const int r = wrapn(y0 + jj, N) * N + wrapn(x0 + ii, N);
          if (jj < m && lev.f[0].tptr[r + 1] > lev.f[0].tptr[r]) ib = true;   // x-face (ii, jj)
          if (ii < m && lev.f[1].tptr[r + 1] > lev.f[1].tptr[r]) ib = true;   // y-face (ii, jj)
        }
      if (ib) lev.ib_list.push_back(p);
      else lev.int_list.push_back(p);
    }
    // codes, then linear offsets from the box's corner (the gathers' table)
    const int nloc = lev.g.nloc;
    lev.loc_tab.assign(2 * (size_t)nloc, 0);
    for (int k = 0; k < nloc; ++k) {
      const int nu = m * (m + 1);
      int comp, ii, jj;
      if (k < nu) { comp = 0; ii = k % (m + 1); jj = k / (m + 1); }
      else if (k < 2 * nu) { comp = 1; ii = (k - nu) % m; jj = (k - nu) / m; }
      else { comp = 2; ii = (k - 2 * nu) % m; jj = (k - 2 * nu) / m; }
      lev.loc_tab[k] = (comp << 24) | (jj << 12) | ii;
      lev.loc_tab[nloc + k] = (int)((int64_t)comp * N * N + (int64_t)jj * N + ii);
    }
    lev.n_ib = (int)lev.ib_list.size();
    lev.uniq = lev.ib_list;
    if (!lev.int_list.empty()) lev.uniq.push_back(lev.int_list.front());
    lev.n_unique = (int)lev.uniq.size();
    if (d_.combine == IBMG_COMBINE_SUM) {
      // every row of every box inverse: the whole local solution is summed
      lev.sum_mode = true;
      lev.g.nown = nloc;
      lev.g.nch = (nloc + 63) / 64;
    }
  }

  size_t box_stride(const Level<T>& lev) const { return (size_t)lev.g.nch * lev.g.nloc * 64; }

  // elements of the interior product's slice buffer for cnt boxes
  static size_t interior_part_need(const BoxGeom& g, int cnt) {
    if (cnt <= 0) return 0;
    const int ks = ras_interior_ksplit(g, cnt);
    return ks > 1 ? (size_t)ks * cnt * g.nch * 64 : 0;
  }

  // elements of the IB-box kernel's slice buffer for cnt boxes
  static size_t ib_part_need(const BoxGeom& g, int cnt) {
    if (cnt <= 0) return 0;
    const int ks = ras_ib_ksplit(g, cnt);
    return ks > 1 ? (size_t)ks * cnt * g.nch * 64 : 0;
  }

  // Every Schwarz launch goes through here: the slice buffer must hold the
  // launch's column slices (IB boxes) followed by its reduction slices
  // (interior).
  // sym: the IB boxes (the level's whole list) from the symmetric copy
  void ras_launch(Level<T>& lev, const T* r, T* z, const T* inv, const int* ib, int n_ib, const int* in, int n_int,
                  hipStream_t s, int parts, bool acc, int tb, bool sym = false) {
    require(lev.int_part.n >= ib_part_need(lev.g, (parts & 1) ? n_ib : 0) +
                                   interior_part_need(lev.g, (parts & 2) ? n_int : 0),
            "Schwarz slice buffer too small");
    require(!sym || (lev.use_sym && n_ib == lev.n_ib), "symmetric IB storage is for the whole IB list");
    const SymIB sy = sym_of(lev);
    require(sym || !lev.use_sym || !(parts & 1) || n_ib == 0, "the IB boxes of this level are in symmetric storage");
    launch_ras_apply<T>(r, z, lev.g, inv, ib, n_ib, shared_inv(lev), in, n_int, lev.d_loc.p, lev.int_part.p, s,
                        parts, acc, tb, lev.int_x.p, lev.int_x.n, sym ? &sy : nullptr);
  }

  // partial-sum buffers of a level: the reductions' blocks x vectors, and the
  // fused operator kernel's blocks x (nu + 1) vectors
  static size_t part_stride(const Level<T>& lev) {
    return std::max(kPartStride, (size_t)apply_blocks(lev.N) * (kMaxNu + 1));
  }

  // Interior product form per Schwarz level: time the pipelined XCD-ordered
  // 64-box tiles, the 16- and 32-box tiles, the register-blocked 64-box form
  // and the gathered 128-box form (HIP events, on the level's work vectors)
  // and keep the fastest.  All compute the same sums in the same order.
  // IBMG_INTERIOR_FORM=1|16|32|64|128 in the environment fixes the form
  // instead (1 = pipelined; where the level supports it).
  void tune_interior(hipStream_t s) {
    if (d_.smoother != IBMG_RAS && d_.smoother != IBMG_RMS) return;
    if (dry_run() || d_.combine == IBMG_COMBINE_SUM) return;
    int forced = 0;
    if (const char* e = std::getenv("IBMG_INTERIOR_FORM")) forced = std::atoi(e);
    for (int l = 1; l <= L_; ++l) {
      Level<T>& lev = levels_[l];
      const int n_int = (int)lev.int_list.size();
      if (n_int == 0) continue;
      if (forced == 16 || forced == 32 || forced == 64 || forced == kIntFormPipe ||
          (forced == 128 && lev.int_x.n >= int_gather_elems(lev.g, n_int))) {
        lev.int_tb = forced;
        continue;
      }
      // a rebuild at moved points keeps a level's earlier pick while its
      // interior box count stays within an eighth of the count it was timed
      // at (the forms give the same bits, so only speed is at stake)
      if ((int)int_forms_.size() > l && int_forms_[l].first > 0 &&
          8 * std::abs(n_int - int_forms_[l].first) <= int_forms_[l].first &&
          (int_forms_[l].second != 128 || lev.int_x.n >= int_gather_elems(lev.g, n_int))) {
        lev.int_tb = int_forms_[l].second;
        continue;
      }
      launch_fill<T>(lev.r.p, T(1), 3 * (size_t)lev.N * lev.N, s);
      double best = 1e300;
      for (int tb : {kIntFormPipe, 32, 16, 64, 128}) {
        if (tb == 128 && lev.int_x.n < int_gather_elems(lev.g, n_int)) continue;
        const double ms = time_launches([&] {
          ras_launch(lev, lev.r.p, lev.t.p, lev.inv.p, lev.d_ib.p, lev.n_ib, lev.d_int.p, n_int, s, 2, false, tb);
        }, 5, s);
        if (ms < best) {
          best = ms;
          lev.int_tb = tb;
        }
      }
      if ((int)int_forms_.size() <= l) int_forms_.resize(l + 1, {0, 0});
      int_forms_[l] = {n_int, lev.int_tb};
    }
  }

  // Colours of the multiplicative sweep (Alg. 3 in colour-major order).
  // Box p reaches box q when a row of p's enlarged box couples, through the
  // five-point stencil, the IB rows, G or D, to an unknown owned by q
  // (unknowns are owned by the box of their cell: left x-face, bottom
  // y-face, pressure); reaching in either direction is a conflict.  Boxes
  // take, in index order, the smallest colour unused by coloured conflicting
  // boxes; the box lists are then sorted by colour.
  void colour_boxes(Level<T>& lev) {
    const BoxGeom& g = lev.g;
    const int N = g.N, b = g.b, o = g.o, m = g.m, npd = g.npd, nb = npd * npd;
    std::vector<std::vector<int>> adj(nb);
    std::vector<int> stamp(nb, -1);
    auto owner = [&](int i, int j) { return (wrapn(j, N) / b) * npd + wrapn(i, N) / b; };
    for (int p = 0; p < nb; ++p) {
      const int x0 = (p % npd) * b - o, y0 = (p / npd) * b - o;
      auto touch = [&](int q) {
        if (q != p && stamp[q] != p) {
          stamp[q] = p;
          adj[p].push_back(q);
          adj[q].push_back(p);
        }
      };
      auto ib_cols = [&](int comp, int i, int j) {
        const CompFoot& f = lev.f[comp];
        const int r = wrapn(j, N) * N + wrapn(i, N);
        for (int k = f.tptr[r]; k < f.tptr[r + 1]; ++k) {
          const int face = f.tcol[k] % (N * N);   // columns index [u | v]
          touch(owner(face % N, face / N));
        }
      };
      for (int jj = 0; jj <= m; ++jj)
        for (int ii = 0; ii <= m; ++ii) {
          const int i = x0 + ii, j = y0 + jj;
          if (jj < m) {  // x-face (i, j): u stencil, G (cells (i, j), (i-1, j)), IB row
            touch(owner(i, j));
            touch(owner(i - 1, j));
            touch(owner(i + 1, j));
            touch(owner(i, j - 1));
            touch(owner(i, j + 1));
            ib_cols(0, i, j);
          }
          if (ii < m) {  // y-face (i, j): v stencil, G (cells (i, j), (i, j-1)), IB row
            touch(owner(i, j));
            touch(owner(i - 1, j));
            touch(owner(i + 1, j));
            touch(owner(i, j - 1));
            touch(owner(i, j + 1));
            ib_cols(1, i, j);
          }
          if (ii < m && jj < m) {  // cell (i, j): D (faces (i, j), (i+1, j), (i, j+1))
            touch(owner(i, j));
            touch(owner(i + 1, j));
            touch(owner(i, j + 1));
          }
        }
    }
    lev.box_colour.assign(nb, -1);
    std::vector<int> mark;
    lev.ncolour = 0;
    for (int p = 0; p < nb; ++p) {
      for (int q : adj[p])
        if (lev.box_colour[q] >= 0) {
          if ((int)mark.size() <= lev.box_colour[q]) mark.resize(lev.box_colour[q] + 1, -1);
          mark[lev.box_colour[q]] = p;
        }
      int c = 0;
      while (c < (int)mark.size() && mark[c] == p) ++c;
      lev.box_colour[p] = c;
      lev.ncolour = std::max(lev.ncolour, c + 1);
    }
    auto by_colour = [&](std::vector<int>& list, std::vector<int>& off) {
      std::stable_sort(list.begin(), list.end(),
                       [&](int a, int bb) { return lev.box_colour[a] < lev.box_colour[bb]; });
      off.assign(lev.ncolour + 1, 0);
      for (int q : list) off[lev.box_colour[q] + 1]++;
      for (int c = 0; c < lev.ncolour; ++c) off[c + 1] += off[c];
    };
    by_colour(lev.ib_list, lev.ib_off);
    by_colour(lev.int_list, lev.int_off);
    lev.uniq = lev.ib_list;
    if (!lev.int_list.empty()) lev.uniq.push_back(lev.int_list.front());
  }

  // Per spring the unit block B_e = K_e / kappa_e of the tangent model at the
  // current positions: (1 - L/l) I + (L/l) t t^T (B_xx, B_xy, B_yy), the
  // identity for L = 0.
  std::vector<double> unit_blocks() const {
    std::vector<double> B(3 * (size_t)E_);
    for (int e = 0; e < E_; ++e) {
      const double L = rest_[e];
      if (L == 0.0) {
        B[3 * e] = 1.0;
        B[3 * e + 1] = 0.0;
        B[3 * e + 2] = 1.0;
        continue;
      }
      const int a = ends_[2 * e], b = ends_[2 * e + 1];
      double dx = X_[2 * b] - X_[2 * a], dy = X_[2 * b + 1] - X_[2 * a + 1];
      dx -= std::nearbyint(dx);
      dy -= std::nearbyint(dy);
      const double len = std::hypot(dx, dy);
      require(len > 0.0, "spring " + std::to_string(e) + " has zero length and a non-zero rest length");
      const double tx = dx / len, ty = dy / len, g = L / len;
      B[3 * e] = (1.0 - g) + g * tx * tx;
      B[3 * e + 1] = g * tx * ty;
      B[3 * e + 2] = (1.0 - g) + g * ty * ty;
    }
    return B;
  }

  template <typename Mark>
  void build_numeric(hipStream_t s, Mark& mark) {
    // spring stiffness per incidence: kappa_e, or the tangent block K_e
    const size_t na = adj_nbr_.size();
    std::vector<double> ak(na);
    for (size_t a = 0; a < na; ++a) ak[a] = kappa_[adj_sid_[a]];
    if (tangent_) {
      const std::vector<double> B = unit_blocks();
      std::vector<double> k00(na), k2(2 * na), rest(na);
      for (size_t a = 0; a < na; ++a) {
        const int e = adj_sid_[a];
        k00[a] = kappa_[e] * B[3 * e];
        k2[2 * a] = kappa_[e] * B[3 * e + 1];
        k2[2 * a + 1] = kappa_[e] * B[3 * e + 2];
        rest[a] = rest_[e];
      }
      d_adj_kap_.upload(ak, s);
      d_adj_rest_.upload(rest, s);
      d_gblocks_.upload(B, s);
      ak.swap(k00);
      d_adj_k2_.upload(k2, s);
      if (std::is_same<T, float>::value) {
        std::vector<float> k2f(k2.begin(), k2.end());
        d_adj_k2f_.upload(k2f, s);
      }
    }
    d_adj_k_.upload(ak, s);
    if (std::is_same<T, float>::value) {
      std::vector<float> akf(ak.begin(), ak.end());
      d_adj_kf_.upload(akf, s);
    }
    for (int l = L_; l >= 0; --l) {
      Level<T>& lev = levels_[l];
      for (int c = 0; c < 2; ++c) {
        CompFoot& f = lev.f[c];
        if (!f.tcol.empty()) {
          // faces of coarse levels carry thousands of points: their rows'
          // point lists are shared out over several waves
          const size_t nnz = f.tcol.size();
          int nslice = std::min(32, std::max(1, f.max_list / 64));
          while (nslice > 1 && (size_t)nslice * nnz > ((size_t)1 << 27)) nslice /= 2;   // <= 1 GiB of slices
          if (nslice > 1 && tpart_.n < (size_t)nslice * nnz) tpart_.alloc((size_t)nslice * nnz);
          launch_t_values(fview<double>(lev.f[0]), fview<double>(lev.f[1]), lev.f[0].d_mask.p, lev.f[1].d_mask.p,
                          sview<double>(), c, lev.N, lev.cd.ibs, f.d_tptr.p, f.d_tcol.p, f.tval.p, nslice, nnz,
                          tpart_.p, s);
          if (std::is_same<T, float>::value)
            launch_cast<double, float>(f.tval.p, f.tvalf.p, f.tcol.size(), s);
        }
      }
    }
    mark("IB rows");
    build_coarse(s);
    mark("coarsest (queued)");
    if (d_.smoother == IBMG_RAS || d_.smoother == IBMG_RMS) build_boxes(s);
    if (d_.smoother == IBMG_SC)
      for (int l = 1; l <= L_; ++l) sc_numeric(levels_[l], s);
    join_coarse(s);
    mark("smoother data");
  }

  // ------------------------------------------------ Schur-complement set-up
  void sc_structure(Level<T>& lev, hipStream_t s) {
    const int N = lev.N, NN = N * N;
    lev.sc.reset(new ScLevel<T>());
    ScLevel<T>& sc = *lev.sc;
    sc.N = N;
    sc.its = d_.cheb_its;
    sc.rho_zero = d_.rho == 0.0;
    // velocity colours: five-point stencil plus IB rows, both components in
    // one greedy pass in row order (with uncoupled components this equals
    // colouring each component alone; tangent blocks couple u and v rows)
    std::vector<int> colv = greedy_colours(2 * NN, [&](int r, std::vector<int>& nb) {
      const int comp = r >= NN ? 1 : 0, q = r - comp * NN, o = comp * NN;
      const int i = q % N, j = q / N;
      nb.push_back(o + j * N + (i + 1) % N);
      nb.push_back(o + j * N + (i + N - 1) % N);
      nb.push_back(o + ((j + 1) % N) * N + i);
      nb.push_back(o + ((j + N - 1) % N) * N + i);
      const CompFoot& f = lev.f[comp];
      for (int k = f.tptr[q]; k < f.tptr[q + 1]; ++k) nb.push_back(f.tcol[k]);
    });
    sc.colu.build(colv, [&](int r) {
      const int comp = r >= NN ? 1 : 0, q = r - comp * NN;
      const CompFoot& f = lev.f[comp];
      return f.tptr[q + 1] - f.tptr[q] > kGsLongRow;
    }, s);
    build_band_runs<T>(sc.colu, lev.f[0].tptr, lev.f[0].tcol, lev.f[1].tptr, lev.f[1].tcol, N, sc.runs_u, s);
    std::vector<int> colp = greedy_colours(NN, [&](int r, std::vector<int>& nb) {
      const int i = r % N, j = r / N;
      nb.push_back(j * N + (i + 1) % N);
      nb.push_back(j * N + (i + N - 1) % N);
      nb.push_back(((j + 1) % N) * N + i);
      nb.push_back(((j + N - 1) % N) * N + i);
    });
    sc.colp.build(colp, [](int) { return false; }, s);
    const size_t n2 = 2 * (size_t)NN, n1 = NN;
    sc.diag.alloc(n2);
    sc.dinv.alloc(n2);
    sc.mdiag.alloc(n1);
    for (DBuf<T>* b : {&sc.yu, &sc.ga, &sc.gx, &sc.ad, &sc.ar, &sc.at, &sc.as}) b->alloc(n2);
    for (DBuf<T>* b : {&sc.md, &sc.mr, &sc.mt, &sc.ms, &sc.ones}) b->alloc(n1);
    sc.part.alloc(1024);
    launch_fill<T>(sc.ones.p, T(1), n1, s);
  }

  // Largest Ritz value of ten Arnoldi steps (classical Gram-Schmidt twice)
  // of op from v0 (overwritten).
  template <typename OP>
  double arnoldi_lambda(size_t n, T* v0, OP op, hipStream_t s) {
    constexpr int steps = 10;
    DBuf<T> V((size_t)(steps + 1) * n);
    DBuf<double> part(2 * kPartStride), hd(64);
    if (dry_run()) return 1.0;
    const int nblk = dots_blocks(n, 256);
    std::vector<double> H((steps + 1) * steps, 0.0), h(steps + 1), h2(steps + 1);
    auto norm_of = [&](const T* x) {
      launch_dots<T>(x, 1, n, x, n, part.p, nblk, s);
      launch_dots_finish(part.p, 1, nblk, hd.p, nullptr, 2, s);
      double v;
      IBMG_HIP(hipMemcpyAsync(&v, hd.p, sizeof(double), hipMemcpyDeviceToHost, s));
      IBMG_HIP(hipStreamSynchronize(s));
      return v;
    };
    const double b0 = norm_of(v0);
    launch_scale<T>(v0, V.p, hd.p, n, s);
    int k = steps;
    for (int j = 0; j < steps; ++j) {
      T* w = V.p + (size_t)(j + 1) * n;
      op(V.p + (size_t)j * n, w);
      for (int pass = 0; pass < 2; ++pass) {
        launch_dots<T>(V.p, j + 1, n, w, n, part.p, nblk, s);
        launch_dots_finish(part.p, j + 1, nblk, hd.p, nullptr, 0, s);
        launch_update<T>(w, V.p, j + 1, n, hd.p, -1.0, n, s);
        IBMG_HIP(hipMemcpyAsync(h2.data(), hd.p, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        IBMG_HIP(hipStreamSynchronize(s));
        for (int i = 0; i <= j; ++i) H[i * steps + j] += h2[i];
      }
      const double hn = norm_of(w);
      H[(j + 1) * steps + j] = hn;
      if (hn == 0.0) {
        k = j + 1;
        break;
      }
      launch_scale<T>(w, w, hd.p, n, s);
    }
    (void)b0;
    std::vector<double> Hk((size_t)k * k);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Hk[(size_t)i * k + j] = H[i * steps + j];
    return hessenberg_max_real_eig(Hk, k);
  }

  void sc_numeric(Level<T>& lev, hipStream_t s) {
    ScLevel<T>& sc = *lev.sc;
    const int N = lev.N, NN = N * N;
    const size_t n2 = 2 * (size_t)NN, n1 = NN;
    sc.c = coef<T>(lev);
    sc.tu = csr<T>(lev.f[0]);
    sc.tv = csr<T>(lev.f[1]);
    sc.ih2 = (T)((double)N * N);
    launch_sc_diag<T>(N, sc.c, sc.tu, sc.tv, sc.ih2, sc.diag.p, sc.dinv.p, sc.mdiag.p, s);
    for (BandRun<T>& run : sc.runs_u) launch_band_values<T>(run, sc.c, sc.tu, sc.tv, N, sc.diag.p, s);
    const int nb1 = dots_blocks(n1, 256);
    // lam for SGS(A_IB)^{-1} A_IB, start vector with the velocity means
    // removed when rho = 0
    DBuf<T> v0(n2);
    launch_weyl<T>(v0.p, n2, s);
    if (sc.rho_zero)
      for (int c = 0; c < 2; ++c) {
        launch_dots<T>(sc.ones.p, 1, n1, v0.p + (size_t)c * n1, n1, sc.part.p, nb1, s);
        launch_sub_mean<T>(v0.p + (size_t)c * n1, n1, sc.part.p, nb1, s);
      }
    sc.lamA = arnoldi_lambda(n2, v0.p, [&](const T* x, T* y) {
      launch_aib_apply<T>(x, sc.at.p, N, sc.c, sc.tu, sc.tv, s);
      sc.sgs_a(sc.at.p, y, s);
    }, s);
    ScLevel<T>::cheb_coefs(sc.lamA, sc.its, &sc.a_theta_inv, sc.a_c1, sc.a_c2);
    // lam for SGS(-M^)^{-1} (-D A~^{-1} G), mean-free start vector
    DBuf<T> q0(n1);
    launch_weyl<T>(q0.p, n1, s);
    launch_dots<T>(sc.ones.p, 1, n1, q0.p, n1, sc.part.p, nb1, s);
    launch_sub_mean<T>(q0.p, n1, sc.part.p, nb1, s);
    sc.lamM = arnoldi_lambda(n1, q0.p, [&](const T* x, T* y) {
      sc.schur_op(x, sc.mt.p, s);
      sc.sgs_m(sc.mt.p, y, s);
    }, s);
    ScLevel<T>::cheb_coefs(sc.lamM, sc.its, &sc.m_theta_inv, sc.m_c1, sc.m_c2);
    IBMG_HIP(hipStreamSynchronize(s));
  }

  void build_coarse(hipStream_t s) {
    Level<T>& lev = levels_[0];
    const int N = lev.N;
    const int nb = d_.rho == 0.0 ? 3 : 1;
    n0_ = 3 * N * N;
    const int nn = n0_ + nb;
    nn0_ = nn;
    DBuf<double> aug((size_t)nn * 2 * nn);
    launch_fill<double>(aug.p, 0.0, aug.n, s);
    launch_coarse_assemble(N, lev.cd, lev.f[0].d_tptr.p, lev.f[0].d_tcol.p, lev.f[0].tval.p,
                           lev.f[1].d_tptr.p, lev.f[1].d_tcol.p, lev.f[1].tval.p, nb, aug.p, s);
    if (defer_coarse_) {
      aug0_ = std::move(aug);
      IBMG_HIP(hipStreamSynchronize(s));
      return;
    }
    // The inversion is one work-group's latency-bound loop: it runs on a
    // second stream (default priority) beside the box inversions and is
    // joined by join_coarse before anything reads the inverse.
    inv0_.alloc((size_t)n0_ * n0_);
    if (!dry_run() && !side_) {
      IBMG_HIP(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
      IBMG_HIP(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
      IBMG_HIP(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming));
    }
    IBMG_HIP(hipEventRecord(ev_fork_, s));
    IBMG_HIP(hipStreamWaitEvent(side_, ev_fork_, 0));
    launch_coarse_invert(aug.p, nn, 1, 0, side_);
    launch_coarse_extract(aug.p, nn, n0_, inv0_.p, side_);
    IBMG_HIP(hipEventRecord(ev_join_, side_));
    coarse_aug_ = std::move(aug);
  }

  // The caller's stream waits for the coarsest inversion; its work matrix
  // is then released (later work on the stream is ordered after the join).
  void join_coarse(hipStream_t s) {
    if (!coarse_aug_.n) return;
    IBMG_HIP(hipStreamWaitEvent(s, ev_join_, 0));
    coarse_aug_.release();
  }

  // the coarsest inverse from the caller's inverted copy of aug0_
  void finish_coarse(const double* inverted, hipStream_t s) {
    inv0_.alloc((size_t)n0_ * n0_);
    launch_coarse_extract(inverted, nn0_, n0_, inv0_.p, s);
    aug0_.release();
    defer_coarse_ = false;
  }

  // Box lists, slice buffers and the inverse storage of one level.
  void prepare_boxes(Level<T>& lev, hipStream_t s) {
    const BoxGeom& g = lev.g;
    lev.d_ib.upload(lev.ib_list, s);
    lev.d_int.upload(lev.int_list, s);
    lev.d_loc.upload(lev.loc_tab, s);
    if (lev.sum_mode) {
      std::vector<int> bi((size_t)g.npd * g.npd, lev.n_ib);
      for (int i = 0; i < lev.n_ib; ++i) bi[lev.ib_list[i]] = i;
      lev.d_box_inv.upload(bi, s);
      lev.inv.alloc((size_t)lev.n_unique * box_stride(lev));
      lev.Y.alloc((size_t)g.npd * g.npd * g.nch * 64);
      return;
    }
    {
      // column slices of the IB boxes followed by the reduction slices of
      // the interior product: the whole lists (additive sweep, tuning,
      // single-kernel timing) and each colour's ranges (multiplicative sweep)
      size_t need = interior_part_need(g, (int)lev.int_list.size()) + ib_part_need(g, lev.n_ib);
      if (d_.smoother == IBMG_RMS)
        for (int c = 0; c < lev.ncolour; ++c)
          need = std::max(need, interior_part_need(g, lev.int_off[c + 1] - lev.int_off[c]) +
                                    ib_part_need(g, lev.ib_off[c + 1] - lev.ib_off[c]));
      if (lev.int_part.n < need) lev.int_part.alloc(need);
    }
    // the gathered operand of the 128-box product form, up to 512 MB a level
    const size_t xe = int_gather_elems(g, (int)lev.int_list.size());
    if (!lev.int_list.empty() && xe * sizeof(T) <= ((size_t)512 << 20)) lev.int_x.alloc(xe);
    // The additive sweep of a single system streams the IB boxes' owned
    // rows from a symmetric copy (lower owned tiles only; whole 64-row
    // chunks) on levels with enough IB boxes: at least 256 (box, chunk)
    // pairs, the IB-box kernel cut into at most four column slices in FP64,
    // two in FP32 (measured: below that the symmetric form's uneven slices
    // and longer sums cost more than its fewer bytes save).  The chunked
    // copy (lev.inv) serves the other levels, the multiplicative sweep and
    // the batched form; on a symmetric level it holds the interior boxes'
    // shared inverse alone.
    lev.use_sym = d_.smoother == IBMG_RAS && !defer_coarse_ && lev.n_ib > 0 && g.nown % 64 == 0 &&
                  lev.n_ib * g.nch >= 256 && ras_ib_ksplit(g, lev.n_ib) <= (sizeof(T) == 8 ? 4 : 2) &&
                  std::getenv("IBMG_NO_SYM") == nullptr;
    if (lev.use_sym) {
      std::vector<int> perm;
      perm.reserve(g.nloc);
      std::vector<char> owned(g.nloc, 0);
      const int bb = g.b * g.b, m = g.m;
      for (int r = 0; r < g.nown; ++r) {
        const int comp = r / bb, q = r % bb;
        const int oi = q % g.b + g.o, oj = q / g.b + g.o;
        const int k = comp == 0 ? oj * (m + 1) + oi : (comp == 1 ? m * (m + 1) + oj * m + oi : 2 * m * (m + 1) + oj * m + oi);
        perm.push_back(k);
        owned[k] = 1;
      }
      for (int k = 0; k < g.nloc; ++k)
        if (!owned[k]) perm.push_back(k);
      lev.d_perm.upload(perm, s);
      lev.inv_sym.alloc((size_t)lev.n_ib * sym_box_stride(g));
      lev.sym_part.alloc((size_t)lev.n_ib * sym_part_len(g, lev.n_ib));
    }
    lev.inv.alloc((size_t)(lev.n_unique - inv_base(lev)) * box_stride(lev));
  }

  SymIB sym_of(Level<T>& lev) { return SymIB{lev.inv_sym.p, lev.d_perm.p, lev.sym_part.p}; }

  // first unique box whose owned rows lev.inv holds in chunks (the IB boxes
  // of a symmetric level live in inv_sym only)
  static int inv_base(const Level<T>& lev) { return lev.use_sym ? lev.n_ib : 0; }
  // the interior boxes' shared inverse
  T* shared_inv(Level<T>& lev) { return lev.inv.p + (size_t)(lev.n_ib - inv_base(lev)) * box_stride(lev); }

  // The unique box inverses of every Schwarz level: assembled per level,
  // inverted in batches that mix levels whose boxes have the same number of
  // unknowns (one run of block sweeps serves them all), owned rows extracted
  // per level.  Batches hold at most 512 matrices and 8 GiB of them with
  // their sweep workspace (a set-up temporary of the handle's workspace).
  void build_boxes(hipStream_t s) {
    std::map<int, std::vector<std::pair<int, int>>> groups;   // nloc -> (level, unique index)
    std::vector<DBuf<int>> ids(L_ + 1);
    for (int l = 1; l <= L_; ++l) {
      Level<T>& lev = levels_[l];
      prepare_boxes(lev, s);
      ids[l].upload(lev.uniq, s);
      for (int u = 0; u < lev.n_unique; ++u) groups[lev.g.nloc].push_back({l, u});
    }
    // matrices of one size are inverted together, at most 10 GiB of them at
    // a time, split into equal batches
    const size_t budget = (size_t)10 << 30;
    for (auto& grp : groups) {
      const int n = grp.first;
      const auto& items = grp.second;
      const size_t per = ((size_t)n * n + 3 * (size_t)n * kGjNb + (size_t)kGjNb * kGjNb) * sizeof(double);
      const size_t cap = std::min<size_t>(std::max<size_t>(1, budget / per), 512);
      const size_t nbatch = (items.size() + cap - 1) / cap;
      const int batch = (int)((items.size() + nbatch - 1) / nbatch);
      DBuf<double> mats((size_t)batch * n * n), work(3 * (size_t)batch * n * kGjNb),
          dinv((size_t)batch * kGjNb * kGjNb);
      for (size_t b0 = 0; b0 < items.size(); b0 += batch) {
        const int cnt = (int)std::min<size_t>(batch, items.size() - b0);
        // runs of one level with consecutive unique indices
        auto for_runs = [&](auto fn) {
          size_t i = b0;
          while (i < b0 + cnt) {
            size_t j = i + 1;
            while (j < b0 + cnt && items[j].first == items[i].first && items[j].second == items[j - 1].second + 1) ++j;
            fn(items[i].first, items[i].second, (int)(j - i), i - b0);
            i = j;
          }
        };
        for_runs([&](int l, int u0, int count, size_t slot) {
          Level<T>& lev = levels_[l];
          launch_patch_assemble(ids[l].p + u0, count, lev.g, lev.cd, lev.f[0].d_tptr.p, lev.f[0].d_tcol.p,
                                lev.f[0].tval.p, lev.f[1].d_tptr.p, lev.f[1].d_tcol.p, lev.f[1].tval.p,
                                mats.p + slot * n * n, s);
        });
        launch_gj_invert(mats.p, n, cnt, work.p, dinv.p, s);
        for_runs([&](int l, int u0, int count, size_t slot) {
          Level<T>& lev = levels_[l];
          const int skip = std::min(count, std::max(0, inv_base(lev) - u0));
          if (count > skip)
            launch_extract_owned<T>(mats.p + (slot + skip) * n * n, count - skip, lev.g,
                                    lev.inv.p + (size_t)(u0 + skip - inv_base(lev)) * box_stride(lev), s,
                                    lev.sum_mode);
          // unique indices below n_ib are the IB boxes
          const int nsym = lev.use_sym ? std::min(count, std::max(0, lev.n_ib - u0)) : 0;
          if (nsym > 0)
            launch_extract_sym<T>(mats.p + slot * n * n, nsym, lev.g, lev.d_perm.p,
                                  lev.inv_sym.p + (size_t)u0 * sym_box_stride(lev.g), s);
        });
      }
      IBMG_HIP(hipStreamSynchronize(s));
    }
  }

  void alloc_work(hipStream_t s) {
    (void)s;
    for (int l = 0; l <= L_; ++l) {
      Level<T>& lev = levels_[l];
      const size_t n = 3 * (size_t)lev.N * lev.N;
      lev.w.alloc(n);
      lev.b.alloc(n);
      lev.r.alloc(n);
      lev.t.alloc(n);
      if (l >= 1) {
        lev.V.alloc((size_t)(nu_ + 1) * n);
        lev.Z.alloc((size_t)nu_ * n);
      }
      lev.F.alloc(4 * (size_t)std::max(M_, 1));   // forces [2][M] then J u [2][M]
      if (l >= 1 && d_.smoother == IBMG_RMS) lev.rr.alloc(n);
      if (lev.use_spmv) {
        lev.Gd.alloc(2 * (size_t)lev.N * lev.N);
        if (std::is_same<T, float>::value) lev.Gt.alloc(2 * (size_t)lev.N * lev.N);
      }
      lev.H.alloc((size_t)(kMaxNu + 1) * kMaxNu);
      lev.scal.alloc(64);
      lev.part.alloc(2 * part_stride(lev));
    }
  }

  // --------------------------------------------------------------- views
  template <typename U>
  FootView<U> fview(CompFoot& f) {
    if constexpr (std::is_same<U, double>::value)
      return FootView<double>{f.d_base.p, f.w.p, f.d_sp_ptr.p, f.d_sp_ent.p, f.sw.p, d_order_.p, f.d_obase.p,
                              f.ow.p};
    else
      return FootView<float>{f.d_base.p, f.wf.p, f.d_sp_ptr.p, f.d_sp_ent.p, f.swf.p, d_order_.p, f.d_obase.p,
                             f.owf.p};
  }
  template <typename U>
  SpringView<U> sview() {
    if constexpr (std::is_same<U, double>::value)
      return SpringView<double>{M_, d_adj_ptr_.p, d_adj_nbr_.p, d_adj_k_.p, tangent_ ? d_adj_k2_.p : nullptr};
    else
      return SpringView<float>{M_, d_adj_ptr_.p, d_adj_nbr_.p, d_adj_kf_.p, tangent_ ? d_adj_k2f_.p : nullptr};
  }
  template <typename U>
  StokesCoef<U> coef(Level<T>& lev) {
    if constexpr (std::is_same<U, double>::value) return lev.cd;
    else return StokesCoef<float>{(float)lev.cd.alpha, (float)lev.cd.beta, (float)lev.cd.gi, (float)lev.cd.ibs};
  }

  // y = L_IB^l x (b != null: y = b - L_IB^l x)
  template <typename U>
  void op(int l, const U* x, U* y, const U* b, bool trans, U* F, hipStream_t s) {
    Level<T>& lev = levels_[l];
    const size_t nn = (size_t)lev.N * lev.N;
    const U* Fp = nullptr;
    const U* Gp = nullptr;
    if (M_ > 0 && E_ > 0) {
      if (lev.use_spmv) {
        U* G = gbuf<U>(lev);
        launch_ib_spmv<U>(x, G, csr<U>(lev.f[0]), csr<U>(lev.f[1]), lev.N, s);
        Gp = G;
      } else {
        launch_ib_force<U>(x, x + nn, fview<U>(lev.f[0]), fview<U>(lev.f[1]), sview<U>(), lev.N,
                           F + 2 * (size_t)std::max(M_, 1), F, s);
        Fp = F;
      }
    }
    launch_apply<U>(x, y, b, Fp, Gp, fview<U>(lev.f[0]), fview<U>(lev.f[1]), lev.N, M_, coef<U>(lev),
                    trans, s);
  }

  // y = L_IB^l x (b != null: y = b - L_IB^l x) with the first Gram-Schmidt
  // pass fused into the operator kernel: partial holds apply_blocks(N)
  // blocks of the dots V_q . y, q < nvec (V = null: y . y)
  template <typename U>
  void op_dots(int l, const U* x, U* y, const U* b, const U* V, int nvec, size_t vstride, double* partial, U* F,
               hipStream_t s) {
    Level<T>& lev = levels_[l];
    const size_t nn = (size_t)lev.N * lev.N;
    const U* Fp = nullptr;
    const U* Gp = nullptr;
    if (M_ > 0 && E_ > 0) {
      if (lev.use_spmv) {
        U* G = gbuf<U>(lev);
        launch_ib_spmv<U>(x, G, csr<U>(lev.f[0]), csr<U>(lev.f[1]), lev.N, s);
        Gp = G;
      } else {
        launch_ib_force<U>(x, x + nn, fview<U>(lev.f[0]), fview<U>(lev.f[1]), sview<U>(), lev.N,
                           F + 2 * (size_t)std::max(M_, 1), F, s);
        Fp = F;
      }
    }
    launch_apply_dots<U>(x, y, b, Fp, Gp, fview<U>(lev.f[0]), fview<U>(lev.f[1]), lev.N, M_, coef<U>(lev), V, nvec,
                         vstride, partial, s);
  }

  template <typename U>
  CsrT<U> csr(CompFoot& f) {
    if constexpr (std::is_same<U, double>::value)
      return CsrT<double>{f.d_tptr.p, f.d_tcol.p, f.tval.p};
    else
      return CsrT<float>{f.d_tptr.p, f.d_tcol.p, f.tvalf.p};
  }
  template <typename U>
  U* gbuf(Level<T>& lev) {
    if constexpr (std::is_same<U, double>::value) return lev.Gd.p;
    else return lev.Gt.p;
  }

  // ------------------------------------------------------- V-cycle pieces
  void basic_smoother(int l, const T* v, T* z, hipStream_t s) {
    Level<T>& lev = levels_[l];
    if (lev.sc) {
      lev.sc->apply(v, z, s);
      return;
    }
    if (lev.sum_mode) {
      launch_asm_apply<T>(v, z, lev.g, lev.inv.p, lev.d_box_inv.p, lev.Y.p, s);
      return;
    }
    if (d_.smoother == IBMG_RMS) {
      // Alg. 3 colour by colour from z = 0: each colour's boxes add their
      // restricted local solutions of the residual of the current z
      launch_fill<T>(z, T(0), 3 * (size_t)lev.N * lev.N, s);
      for (int c = 0; c < lev.ncolour; ++c) {
        const T* rc = v;
        if (c > 0) {
          op<T>(l, z, lev.rr.p, v, false, lev.F.p, s);
          rc = lev.rr.p;
        }
        const int i0 = lev.ib_off[c], k0 = lev.int_off[c];
        ras_launch(lev, rc, z, lev.inv.p + (size_t)i0 * box_stride(lev), lev.d_ib.p + i0, lev.ib_off[c + 1] - i0,
                   lev.d_int.p + k0, lev.int_off[c + 1] - k0, s, 3, true, lev.int_tb);
      }
      return;
    }
    ras_launch(lev, v, z, lev.inv.p, lev.d_ib.p, lev.n_ib, lev.d_int.p, (int)lev.int_list.size(), s, 3, false,
               lev.int_tb, lev.use_sym);
  }

  // w <- w + e, e = nu FGMRES iterations (CGS2) on L e = b - L w from e = 0.
  // With w_zero, w is not read (the result is stored into it) and b_nblk > 0
  // says the level's partial-sum buffer already holds b_nblk block sums of
  // |b|^2 (left there by the restriction that produced b).
  void smooth_t(int l, T* w, const T* b, int nu, bool w_zero, hipStream_t s, int b_nblk = 0) {
    Level<T>& lev = levels_[l];
    const size_t n = 3 * (size_t)lev.N * lev.N;
    if (d_.sweep_kind == IBMG_SWEEP_RICHARDSON) {
      // nu undamped Richardson steps w <- w + B (b - L w); from w = 0 the
      // first step is w = B b
      for (int k = 0; k < nu; ++k) {
        if (k == 0 && w_zero) {
          basic_smoother(l, b, w, s);
          continue;
        }
        op<T>(l, w, lev.r.p, b, false, lev.F.p, s);
        basic_smoother(l, lev.r.p, lev.t.p, s);
        launch_axpy<T>(w, lev.t.p, n, s);
      }
      return;
    }
    const int nblk = dots_blocks(n, 1024);  // at most nu + 1 vectors
    const int ldh = kMaxNu + 1;
    const T* r0;
    if (w_zero) {
      r0 = b;
    } else {
      // r = b - L w with its squared norm's block sums
      op_dots<T>(l, w, lev.r.p, b, nullptr, 1, 0, lev.part.p, lev.F.p, s);
      r0 = lev.r.p;
    }
    double* beta = lev.scal.p;
    double* pa = lev.part.p;
    double* pb = lev.part.p + part_stride(lev);
    const int nab = apply_blocks(lev.N);  // blocks of the fused operator + dots kernel
    T* V = lev.V.p;
    T* Z = lev.Z.p;
    if (w_zero && b_nblk > 0) {
      launch_scale_red<T>(r0, V, n, pa, b_nblk, beta, s);
    } else if (w_zero) {
      launch_dots<T>(r0, 1, n, r0, n, pa, nblk, s);
      launch_scale_red<T>(r0, V, n, pa, nblk, beta, s);
    } else {
      launch_scale_red<T>(r0, V, n, pa, nab, beta, s);
    }
    for (int k = 0; k < nu; ++k) {
      T* vk = V + (size_t)k * n;
      T* zk = Z + (size_t)k * n;
      T* t = V + (size_t)(k + 1) * n;
      basic_smoother(l, vk, zk, s);
      // t = L z with the pass-1 dots V_q . t; pass 2 and the norm follow
      op_dots<T>(l, zk, t, nullptr, V, k + 1, n, pa, lev.F.p, s);
      double* hcol = lev.H.p + (size_t)k * ldh;
      // pass 2's dots with |t|^2 beside them: t - V h2 is orthogonal to the
      // orthonormal basis, so its norm is sqrt(|t|^2 - |h2|^2) and the
      // update, the norm and the normalisation take one more sweep
      launch_upd_dots_n<T>(t, V, k + 1, n, n, pa, nblk, hcol, pb, s, nab);
      // the last basis vector is never read: the least-squares kernel takes
      // its coefficients and norm from these partials
      if (k + 1 < nu) launch_scale_upd<T>(t, V, k + 1, n, n, pb, nblk, hcol, s);
    }
    launch_combine_ls<T>(w, Z, nu, n, n, lev.H.p, ldh, beta, lev.scal.p + kScalY, s, w_zero, pb, nblk, true);
  }

  // Classical Gram-Schmidt twice against V[0..k): h (first pass + second
  // pass) into hcol[0..k); the partial sums of ||t||^2 are left in pa for
  // launch_scale_red, which stores ||t|| and normalises t.
  template <typename U>
  void orthogonalise(const U* V, int k, size_t n, U* t, double* hcol, double* pa, double* pb,
                     int nblk, hipStream_t s) {
    launch_dots<U>(V, k, n, t, n, pa, nblk, s);
    launch_upd_dots<U>(t, V, k, n, n, pa, nblk, hcol, pb, s);
    launch_upd_norm<U>(t, V, k, n, n, pb, nblk, hcol, pa, s);
  }

  // The same for the outer solve's long vectors, on up to kOuterBlocks
  // blocks: one block folds each pass's partial sums (the pass-1 dots, then
  // the pass-2 dots) before the next kernel, so that kernel's blocks read k
  // values instead of every block's k partials.
  void orthogonalise_outer(const double* V, int k, size_t n, double* t, double* hcol, int nblk, hipStream_t s) {
    double* pa = opart_.p;
    double* pb = opart_.p + kOuterPartStride;
    launch_dots<double>(V, k, n, t, n, pa, nblk, s);
    launch_dots_finish(pa, k, nblk, ofold_.p, nullptr, 0, s);
    launch_upd_dots<double>(t, V, k, n, n, ofold_.p, nblk, hcol, pb, s, 1);
    launch_dots_finish(pb, k, nblk, ofold_.p + 72, nullptr, 0, s);
    launch_upd_norm<double>(t, V, k, n, n, ofold_.p + 72, nblk, hcol, pa, s, 1);
  }

  // w = MG(0, b) on level l (Alg. 1); b_nblk as for smooth_t
  void mg(int l, const T* b, T* w, hipStream_t s, int b_nblk = 0) {
    if (l == 0) {
      launch_coarse_apply<T>(inv0_.p, n0_, b, w, s);
      return;
    }
    Level<T>& lev = levels_[l];
    Level<T>& crs = levels_[l - 1];
    smooth_t(l, w, b, d_.nu1, true, s, b_nblk);
    op<T>(l, w, lev.r.p, b, false, lev.F.p, s);
    int c_nblk = 0;
    if (l - 1 >= 1 && restrict_blocks(crs.N) <= (int)part_stride(crs)) {
      launch_restrict_norm<T>(lev.r.p, crs.b.p, crs.N, crs.part.p, s);
      c_nblk = restrict_blocks(crs.N);
    } else {
      launch_restrict<T>(lev.r.p, crs.b.p, crs.N, s);
    }
    mg(l - 1, crs.b.p, crs.w.p, s, c_nblk);
    launch_prolong_add<T>(crs.w.p, w, crs.N, s);
    smooth_t(l, w, b, d_.nu2, false, s);
  }

  // ------------------------------------------------------------ ABI calls
  void apply(int level, const double* w, double* y, bool trans, hipStream_t s) override {
    op<double>(level, w, y, nullptr, trans, Fd_.p, s);
  }

  void spread(const double* F, double* f, hipStream_t s) override {
    Level<T>& lev = levels_[L_];
    const double h = 1.0 / lev.N;
    launch_spread(F, fview<double>(lev.f[0]), fview<double>(lev.f[1]), M_, lev.N, 1.0 / (h * h), f, s);
  }

  void interp(const double* u, double* U, hipStream_t s) override {
    Level<T>& lev = levels_[L_];
    launch_interp<double>(u, u + (size_t)lev.N * lev.N, fview<double>(lev.f[0]), fview<double>(lev.f[1]),
                          M_, lev.N, U, s);
  }

  void restrict_(int level, const double* fine, double* coarse, hipStream_t s) override {
    launch_restrict<double>(fine, coarse, levels_[level - 1].N, s);
  }

  void prolong_add(int level, const double* coarse, double* fine, hipStream_t s) override {
    launch_prolong_add<double>(coarse, fine, levels_[level - 1].N, s);
  }

  void smoother_apply(int level, const double* r, double* z, hipStream_t s) override {
    Level<T>& lev = levels_[level];
    const size_t n = 3 * (size_t)lev.N * lev.N;
    if constexpr (std::is_same<T, double>::value) {
      basic_smoother(level, r, z, s);
    } else {
      launch_cast<double, T>(r, lev.r.p, n, s);
      basic_smoother(level, lev.r.p, lev.t.p, s);
      launch_cast<T, double>(lev.t.p, z, n, s);
    }
  }

  void smooth(int level, double* w, const double* b, int nu, hipStream_t s) override {
    require(nu >= 1 && nu <= nu_, "nu must lie in [1, max(nu1, nu2)]");
    Level<T>& lev = levels_[level];
    const size_t n = 3 * (size_t)lev.N * lev.N;
    if constexpr (std::is_same<T, double>::value) {
      smooth_t(level, w, b, nu, false, s);
    } else {
      launch_cast<double, T>(w, lev.w.p, n, s);
      launch_cast<double, T>(b, lev.b.p, n, s);
      smooth_t(level, lev.w.p, lev.b.p, nu, false, s);
      launch_cast<T, double>(lev.w.p, w, n, s);
    }
  }

  void coarse_solve(const double* r, double* x, hipStream_t s) override {
    launch_coarse_apply<double>(inv0_.p, n0_, r, x, s);
  }

  void vcycle_body(const double* r, double* z, hipStream_t s) {
    Level<T>& top = levels_[L_];
    const size_t n = 3 * (size_t)top.N * top.N;
    if constexpr (std::is_same<T, double>::value) {
      mg(L_, r, z, s);
    } else {
      launch_cast<double, T>(r, top.b.p, n, s);
      mg(L_, top.b.p, top.w.p, s);
      launch_cast<T, double>(top.w.p, z, n, s);
    }
  }

  // The whole V-cycle (several hundred launches, no host synchronisation)
  // is captured once into a HIP graph reading vin_ and writing vout_, then
  // replayed; the graph holds kernel nodes only.
  void build_graph() {
    if (!gstream_) IBMG_HIP(hipStreamCreateWithFlags(&gstream_, hipStreamNonBlocking));
    IBMG_HIP(hipStreamBeginCapture(gstream_, hipStreamCaptureModeThreadLocal));
    try {
      vcycle_body(vin_.p, vout_.p, gstream_);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(gstream_, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    IBMG_HIP(hipStreamEndCapture(gstream_, &graph_));
    IBMG_HIP(hipGraphInstantiate(&gexec_, graph_, nullptr, nullptr, 0));
  }

  void drop_graph() {
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    gexec_ = nullptr;
    graph_ = nullptr;
  }

  void vcycle(const double* r, double* z, hipStream_t s) override {
    if (!use_graph_) {
      vcycle_body(r, z, s);
      return;
    }
    const size_t n = 3 * (size_t)d_.N * d_.N;
    if (!gexec_) build_graph();
    IBMG_HIP(hipMemcpyAsync(vin_.p, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipGraphLaunch(gexec_, s));
    IBMG_HIP(hipMemcpyAsync(z, vout_.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }

  double read_scalar(const double* dptr, hipStream_t s) {
    IBMG_HIP(hipMemcpyAsync(pinned_, dptr, sizeof(double), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
    return pinned_[0];
  }

  void project(double* a, hipStream_t s) {
    Level<T>& top = levels_[L_];
    launch_block_sums<double>(a, top.N, opart_.p, 64, s);
    launch_dots_finish(opart_.p, 3, 64, osc_.p + 8, nullptr, 0, s);
    launch_subtract_means<double>(a, top.N, osc_.p + 8, d_.rho == 0.0 ? 1 : 0, s);
  }

  double norm(const double* a, size_t n, hipStream_t s) {
    const int nblk = dots_blocks(n);
    launch_dots<double>(a, 1, n, a, n, opart_.p, nblk, s);
    launch_dots_finish(opart_.p, 1, nblk, osc_.p + 0, nullptr, 2, s);
    return read_scalar(osc_.p + 0, s);
  }

  int fgmres(const double* b, double* x, const ibmg_solve_opts& o, ibmg_solve_info* info,
             hipStream_t s) override {
    const auto t0 = std::chrono::steady_clock::now();
    require(o.restart >= 1 && o.restart <= outer_cap_,
            "restart must lie in [1, max_restart = " + std::to_string(outer_cap_) + "]");
    require(o.max_it >= 1, "max_it must be >= 1");
    require(std::isfinite(o.rtol) && o.rtol > 0.0, "rtol must be finite and > 0");
    // the adjoint system uses the transposed operator path; L_IB is
    // symmetric, so the same V-cycle preconditions it
    const bool trans = o.transpose != 0;
    const int N = d_.N;
    const size_t n = 3 * (size_t)N * N;
    const int gs_nblk = dots_blocks(n, kOuterBlocks);
    const int ldh = o.restart + 1;
    int hist_n = 0;
    auto push_hist = [&](double v) {
      if (info && info->history && hist_n < info->history_cap) info->history[hist_n] = v;
      ++hist_n;
    };
    // projected right-hand side and the removed null-space part
    IBMG_HIP(hipMemcpyAsync(bp_.p, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    project(bp_.p, s);
    IBMG_HIP(hipMemcpyAsync(pinned_, osc_.p + 8, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
    const double nn = (double)N * N;
    double null2 = pinned_[2] * pinned_[2] / nn;
    if (d_.rho == 0.0) null2 += (pinned_[0] * pinned_[0] + pinned_[1] * pinned_[1]) / nn;
    const double bnorm = norm(bp_.p, n, s);
    if (info) {
      info->iters = 0;
      info->restarts = 0;
      info->rhs_null_norm = std::sqrt(null2);
      info->setup_ms = setup_ms_;
      info->vcycles = 0;
    }
    if (!std::isfinite(bnorm) || !std::isfinite(null2)) throw Error(IBMG_ERR_NONFINITE, "right-hand side holds NaN/Inf");
    if (!o.use_x0) launch_fill<double>(x, 0.0, n, s);
    if (bnorm == 0.0) {
      launch_fill<double>(x, 0.0, n, s);
      IBMG_HIP(hipStreamSynchronize(s));
      if (info) {
        info->rel_res_est = info->rel_res_true = 0.0;
        info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      }
      return IBMG_OK;
    }
    const double target = o.rtol * bnorm;
    int its = 0, restarts = 0, vcycles = 0;
    bool converged = false;
    double est = bnorm, prev_est = 0.0;
    if (!est_ev_) IBMG_HIP(hipEventCreateWithFlags(&est_ev_, hipEventDisableTiming));
    while (its < o.max_it) {
      double* V0 = Vo_.p;
      op<double>(L_, x, V0, bp_.p, trans, Fd_.p, s);
      const double beta = norm(V0, n, s);
      if (!std::isfinite(beta)) throw Error(IBMG_ERR_NONFINITE, "residual is not finite");
      est = beta;
      if (beta <= target) { converged = true; break; }
      launch_scale<double>(V0, V0, osc_.p + 0, n, s);
      launch_fill<double>(g_.p, 0.0, (size_t)o.restart + 2, s);
      IBMG_HIP(hipMemcpyAsync(g_.p, osc_.p + 0, sizeof(double), hipMemcpyDeviceToDevice, s));
      int k = 0;
      bool queued = false;   // z_k's V-cycle already queued by the previous iteration
      for (; k < o.restart && its < o.max_it;) {
        double* vk = Vo_.p + (size_t)k * n;
        double* zk = Zo_.p + (size_t)k * n;
        double* t = Vo_.p + (size_t)(k + 1) * n;
        if (!queued) vcycle(vk, zk, s);
        queued = false;
        ++vcycles;
        op<double>(L_, zk, t, nullptr, trans, Fd_.p, s);
        double* hcol = Ho_.p + (size_t)k * ldh;
        orthogonalise_outer(Vo_.p, k + 1, n, t, hcol, gs_nblk, s);
        launch_scale_red<double>(t, t, n, opart_.p, gs_nblk, hcol + k + 1, s);
        launch_givens(Ho_.p, ldh, k, cs_.p, sn_.p, g_.p, osc_.p + 1, s);
        // The estimate is read on the host after this iteration's work.
        // While the last two estimates say that even one more step at their
        // rate would stay above the target, the next iteration's V-cycle
        // (its input, the normalised t, is already queued) is queued before
        // the host waits, so the device does not idle through the read.  A
        // wrong guess leaves one unused V-cycle behind the solve's tail; it
        // is not counted in vcycles.
        IBMG_HIP(hipMemcpyAsync(pinned_, osc_.p + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        IBMG_HIP(hipEventRecord(est_ev_, s));
        const double rate = prev_est > 0.0 ? std::min(1.0, est / prev_est) : 1.0;
        if (k + 1 < o.restart && its + 1 < o.max_it && its >= 2 && est * rate * rate > target) {
          vcycle(t, Zo_.p + (size_t)(k + 1) * n, s);
          queued = true;
        }
        IBMG_HIP(hipEventSynchronize(est_ev_));
        prev_est = est;
        est = pinned_[0];
        ++k;
        ++its;
        push_hist(est / bnorm);
        if (!std::isfinite(est)) throw Error(IBMG_ERR_NONFINITE, "iteration produced NaN/Inf");
        if (est <= target) { converged = true; break; }
      }
      launch_backsolve(Ho_.p, ldh, k, g_.p, y_.p, s);
      launch_combine<double>(x, Zo_.p, k, n, y_.p, n, s);
      ++restarts;
      if (converged) break;
    }
    project(x, s);
    op<double>(L_, x, rr_.p, bp_.p, trans, Fd_.p, s);
    const double tr = norm(rr_.p, n, s);
    if (info) {
      info->iters = its;
      info->restarts = restarts;
      info->rel_res_est = est / bnorm;
      info->rel_res_true = tr / bnorm;
      info->vcycles = vcycles;
      info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!std::isfinite(tr)) throw Error(IBMG_ERR_NONFINITE, "solution is not finite");
    return converged ? IBMG_OK : IBMG_NOT_CONVERGED;
  }

  void spring_gradient(const double* w, const double* lam, double* out, hipStream_t s) override {
    spring_gradient_in(w, lam, out, Uw_.p, Ul_.p, s);
  }

  void spring_gradient_in(const double* w, const double* lam, double* out, double* Uw, double* Ul,
                          hipStream_t s) override {
    Level<T>& lev = levels_[L_];
    const size_t nn = (size_t)lev.N * lev.N;
    const double h = 1.0 / lev.N;
    launch_interp<double>(w, w + nn, fview<double>(lev.f[0]), fview<double>(lev.f[1]), M_, lev.N, Uw, s);
    launch_interp<double>(lam, lam + nn, fview<double>(lev.f[0]), fview<double>(lev.f[1]), M_, lev.N, Ul, s);
    launch_spring_grad(Uw, Ul, d_ends_.p, tangent_ ? d_gblocks_.p : nullptr, E_, -d_.dt / (h * h), out, s);
  }

  int points() const override { return M_; }

  void set_kappa(const double* kappa, hipStream_t s) override {
    require(E_ == 0 || kappa != nullptr, "kappa is NULL");
    for (int e = 0; e < E_; ++e)
      require(std::isfinite(kappa[e]) && kappa[e] >= 0.0, "kappa must be finite and >= 0");
    kappa_.assign(kappa, kappa + E_);
    rebuild(s);
  }

  // ------------------------------------------- semi-implicit time step
  // rhs = [(rho/dt) u + S_h F(X); 0] on the finest grid (Eq. matrix-impib),
  // F the nodal spring forces (K_h X for the linear model)
  void step_rhs(const double* w, double* rhs, hipStream_t s) override {
    Level<T>& lev = levels_[L_];
    const double h = 1.0 / lev.N;
    const size_t m2 = 2 * (size_t)std::max(M_, 1);
    launch_fill<double>(Fs_.p, 0.0, m2, s);
    launch_fibre_force(d_X_.p, sview<double>(), tangent_ ? d_adj_kap_.p : d_adj_k_.p,
                       tangent_ ? d_adj_rest_.p : nullptr, Fs_.p, s);
    launch_spread(Fs_.p, fview<double>(lev.f[0]), fview<double>(lev.f[1]), M_, lev.N, 1.0 / (h * h), fs_.p, s);
    launch_step_rhs(w, fs_.p, d_.rho / d_.dt, lev.N, rhs, s);
  }

  // Solve L_IB(X^n) w^{n+1} = rhs, advance X^{n+1} = X^n + dt J_h u^{n+1}
  // (Eq. imp-X-new, wrapped into [0, 1)) and rebuild every level at X^{n+1}.
  int time_step(double* w, const ibmg_solve_opts& o, ibmg_solve_info* info, hipStream_t s) override {
    Level<T>& lev = levels_[L_];
    const size_t nn = (size_t)lev.N * lev.N;
    step_rhs(w, rhs_.p, s);
    const int st = fgmres(rhs_.p, w, o, info, s);
    launch_interp<double>(w, w + nn, fview<double>(lev.f[0]), fview<double>(lev.f[1]), M_, lev.N, Uw_.p, s);
    launch_advance(d_X_.p, Uw_.p, d_.dt, M_, s);
    if (M_ > 0)
      IBMG_HIP(hipMemcpyAsync(X_.data(), d_X_.p, 2 * (size_t)M_ * sizeof(double), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
    for (double x : X_)
      if (!std::isfinite(x) || x < 0.0 || x >= 1.0) throw Error(IBMG_ERR_NONFINITE, "updated positions are invalid");
    rebuild(s);
    if (info) info->setup_ms = setup_ms_;
    return st;
  }

  // Every level rebuilt for the current positions X_ (host copy) and
  // stiffnesses, laid out again above the fixed buffers.  If the rebuild
  // fails part-way (a workspace too small for the new layout), the handle
  // stays unusable.
  void rebuild(hipStream_t s) {
    drop_graph();
    valid_ = false;
    release_dependent();
    build_all(s);
    valid_ = true;
  }

  bool valid() const override { return valid_; }

  void positions(double* X) const override {
    std::copy(X_.begin(), X_.end(), X);
  }

  void sc_info(int level, double* lam, int32_t* colours) const override {
    require(level >= 1 && level <= L_, "level out of range");
    const Level<T>& lev = levels_[level];
    require(lev.sc != nullptr, "the handle does not use the Schur-complement smoother");
    lam[0] = lev.sc->lamA;
    lam[1] = lev.sc->lamM;
    colours[0] = lev.sc->colu.ncol;
    colours[1] = lev.sc->colp.ncol;
  }

  // One kernel of level `level`, launched alone on the level's work vectors
  // (filled with ones): IB-box Schwarz (k_ras_ib), interior-box Schwarz
  // (k_ras_interior, one reduction slice when the product is split) or the
  // stencil k_apply.  Algorithmic work per launch: every IB box streams its
  // owned rows of the inverse (nown x nloc), gathers nloc values and writes
  // nown; the interior product reads the shared inverse once and each box's
  // nloc values and writes nown, 2 nown nloc flops per box; the stencil reads
  // and writes the three fields once.
  double kernel_time(int kernel, int level, int reps, hipStream_t s, double* bytes, double* flops) override {
    require(level >= 0 && level <= L_, "level out of range");
    require(reps >= 1 && reps <= 100000, "reps must lie in [1, 100000]");
    Level<T>& lev = levels_[level];
    const size_t n = 3 * (size_t)lev.N * lev.N;
    const double ts = sizeof(T);
    launch_fill<T>(lev.r.p, T(1), n, s);
    launch_fill<T>(lev.t.p, T(0), n, s);
    double by = 0, fl = 0, ms = 0;
    const BoxGeom& g = lev.g;
    if (kernel == IBMG_KERNEL_RAS_IB || kernel == IBMG_KERNEL_RAS_INTERIOR) {
      require(level >= 1 && !lev.sc, "Schwarz kernels need a Schwarz smoother level >= 1");
      require(!lev.sum_mode, "the restricted Schwarz kernels do not run with the summed combination");
      const int n_int = (int)lev.int_list.size();
      if (kernel == IBMG_KERNEL_RAS_IB) {
        require(lev.n_ib > 0, "the level has no IB boxes");
        // the symmetric copy (as the additive sweep runs it, with the row
        // sums' launch) streams only its stored rows
        const double stored = lev.use_sym ? (double)sym_box_stride(g) : (double)g.nown * g.nloc;
        by = (double)lev.n_ib * (stored + g.nloc + g.nown) * ts;
        fl = 2.0 * lev.n_ib * g.nown * g.nloc;
      } else {
        require(n_int > 0, "the level has no interior boxes");
        by = ((double)g.nown * g.nloc + (double)n_int * (g.nloc + g.nown)) * ts;
        fl = 2.0 * n_int * g.nown * g.nloc;
      }
      const int part = kernel == IBMG_KERNEL_RAS_IB ? 1 : 2;
      ms = time_launches([&] {
        ras_launch(lev, lev.r.p, lev.t.p, lev.inv.p, lev.d_ib.p, lev.n_ib, lev.d_int.p, n_int, s, part, false,
                   lev.int_tb, part == 1 && lev.use_sym);
      }, reps, s);
    } else if (kernel == IBMG_KERNEL_STENCIL) {
      by = 2.0 * (double)n * ts;
      fl = 0;
      ms = time_launches([&] {
        launch_apply<T>(lev.r.p, lev.t.p, nullptr, nullptr, nullptr, fview<T>(lev.f[0]), fview<T>(lev.f[1]), lev.N,
                        M_, coef<T>(lev), false, s);
      }, reps, s);
    } else if (kernel == IBMG_KERNEL_RESTRICT || kernel == IBMG_KERNEL_PROLONG) {
      require(level >= 1, "transfers need a level >= 1");
      Level<T>& cl = levels_[level - 1];
      const size_t nc = 3 * (size_t)cl.N * cl.N;
      if (kernel == IBMG_KERNEL_RESTRICT) {
        by = (double)(n + nc) * ts;
        ms = time_launches([&] { launch_restrict<T>(lev.r.p, cl.t.p, cl.N, s); }, reps, s);
      } else {
        by = (double)(nc + 2 * n) * ts;
        launch_fill<T>(cl.r.p, T(1), nc, s);
        ms = time_launches([&] { launch_prolong_add<T>(cl.r.p, lev.t.p, cl.N, s); }, reps, s);
      }
    } else if (kernel == IBMG_KERNEL_SPREAD || kernel == IBMG_KERNEL_INTERP) {
      require(level == L_, "spreading and interpolation run on the finest level");
      require(M_ > 0, "the structure has no points");
      const size_t nn = (size_t)lev.N * lev.N;
      launch_fill<double>(fs_.p, 1.0, 2 * nn, s);
      launch_fill<double>(Fd_.p, 1.0, 2 * (size_t)M_, s);
      size_t ents = 0, touched = 0;
      for (int c = 0; c < 2; ++c) {
        ents += lev.f[c].sp_ent.size();
        for (size_t r = 0; r < nn; ++r) touched += lev.f[c].sp_ptr[r + 1] > lev.f[c].sp_ptr[r];
      }
      const double h = 1.0 / lev.N;
      if (kernel == IBMG_KERNEL_SPREAD) {
        by = (double)ents * 12.0 + (double)(2 * (nn + 1)) * 4.0 + 2.0 * M_ * 8.0 + 2.0 * nn * 8.0;
        ms = time_launches([&] {
          launch_spread(Fd_.p, fview<double>(lev.f[0]), fview<double>(lev.f[1]), M_, lev.N, 1.0 / (h * h), fs_.p, s);
        }, reps, s);
      } else {
        by = 2.0 * M_ * 16 * 8.0 + 2.0 * M_ * 2 * 4.0 + (double)touched * 8.0 + 2.0 * M_ * 8.0;
        ms = time_launches([&] {
          launch_interp<double>(fs_.p, fs_.p + nn, fview<double>(lev.f[0]), fview<double>(lev.f[1]), M_, lev.N,
                                Uw_.p, s);
        }, reps, s);
      }
    } else if (kernel >= IBMG_KERNEL_APPLY_DOTS && kernel <= IBMG_KERNEL_SCALE_UPD) {
      // one smoothing step's Krylov kernels with the basis at its largest
      // (k = nu vectors): zero first-pass dots leave t as it is, unit
      // partial norms give a unit scale, and a diagonal Hessenberg keeps the
      // least squares well posed, so repeated launches see the same values
      require(level >= 1, "the smoothing kernels run on levels >= 1");
      const int k = nu_;
      const int nblk = dots_blocks(n, 1024), nab = apply_blocks(lev.N), ldh = kMaxNu + 1;
      double* pa = lev.part.p;
      double* pb = lev.part.p + part_stride(lev);
      T* V = lev.V.p;
      T* Z = lev.Z.p;
      T* t = V + (size_t)k * n;
      launch_fill<T>(V, T(1), (size_t)(k + 1) * n, s);
      launch_fill<T>(Z, T(1), (size_t)k * n, s);
      launch_fill<double>(pa, 0.0, 2 * part_stride(lev), s);
      launch_fill<double>(lev.H.p, 0.0, (size_t)(kMaxNu + 1) * kMaxNu, s);
      launch_fill<double>(lev.scal.p, 1.0, 1, s);
      for (int q = 0; q < k; ++q) launch_fill<double>(lev.H.p + (size_t)q * ldh + q, 1.0, 1, s);
      double* hcol = lev.H.p + (size_t)(k - 1) * ldh;
      if (kernel == IBMG_KERNEL_APPLY_DOTS) {
        by = (double)(k + 2) * n * ts;
        ms = time_launches([&] { op_dots<T>(level, Z, lev.t.p, nullptr, V, k, n, pa, lev.F.p, s); }, reps, s);
      } else if (kernel == IBMG_KERNEL_UPD_DOTS) {
        by = (double)(k + 2) * n * ts;
        ms = time_launches([&] { launch_upd_dots_n<T>(t, V, k, n, n, pb, nblk, hcol, pa, s, nab); }, reps, s);
      } else if (kernel == IBMG_KERNEL_SCALE_UPD) {
        // zero second-pass dots and a unit |t|^2 in every block's partials:
        // t keeps its values and is scaled by the same factor each launch
        by = (double)(k + 2) * n * ts;
        launch_fill<double>(pb, 0.0, (size_t)nblk * (k + 1), s);
        launch_fill<double>(pb + k, 1.0, 1, s);
        ms = time_launches([&] { launch_scale_upd<T>(t, V, k, n, n, pb, nblk, hcol, s); }, reps, s);
      } else if (kernel == IBMG_KERNEL_UPD_NORM) {
        by = (double)(k + 2) * n * ts;
        ms = time_launches([&] { launch_upd_norm<T>(t, V, k, n, n, pb, nblk, hcol, pa, s); }, reps, s);
      } else if (kernel == IBMG_KERNEL_SCALE_RED) {
        by = 2.0 * n * ts;
        launch_fill<double>(pb, 1.0, (size_t)nblk, s);
        ms = time_launches([&] { launch_scale_red<T>(t, lev.t.p, n, pb, nblk, lev.scal.p + kScalTmp, s); },
                           reps, s);
      } else {
        by = (double)(k + 2) * n * ts;
        ms = time_launches([&] {
          launch_combine_ls<T>(lev.w.p, Z, k, n, n, lev.H.p, ldh, lev.scal.p, lev.scal.p + kScalY, s, false);
        }, reps, s);
      }
    } else {
      require(false, "unknown kernel");
    }
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    return ms;
  }

  std::vector<int64_t> stats() const override {
    std::vector<int64_t> v;
    v.push_back(L_ + 1);
    for (int l = 0; l <= L_; ++l) {
      const Level<T>& lev = levels_[l];
      v.push_back(lev.N);
      v.push_back((int64_t)lev.g.npd * lev.g.npd);
      v.push_back(lev.n_unique);
      v.push_back(lev.n_ib);
      v.push_back((int64_t)lev.f[0].tcol.size() + (int64_t)lev.f[1].tcol.size());
      v.push_back(lev.ncolour);
    }
    return v;
  }

 private:
  ibmg_desc d_;
  int M_ = 0, E_ = 0, nu_ = 2, L_ = 0, n0_ = 0;
  std::vector<double> X_, kappa_, rest_;
  bool tangent_ = false;   // IBMG_SPRING_TANGENT
  std::vector<int> ends_, sizes_;
  std::vector<int> adj_ptr_, adj_nbr_, adj_sid_;
  DBuf<int> d_adj_ptr_, d_adj_nbr_, d_ends_;
  DBuf<int> d_order_;   // points in cell order
  DBuf<double> d_adj_k_, d_X_;
  DBuf<float> d_adj_kf_;
  // tangent model: (K_e[0][1], K_e[1][1]) per incidence, kappa_e and L_e per
  // incidence (spring forces), unit blocks per spring (gradient)
  DBuf<double> d_adj_k2_, d_adj_kap_, d_adj_rest_, d_gblocks_;
  DBuf<float> d_adj_k2f_;
  std::vector<Level<T>> levels_;
  DBuf<double> inv0_;
  DBuf<double> Fd_, Uw_, Ul_;
  DBuf<double> Fs_, fs_, rhs_;   // time step: nodal forces, spread forces, right-hand side
  // outer FGMRES
  int outer_cap_ = 0;
  DBuf<double> Vo_, Zo_, Ho_, cs_, sn_, g_, y_, osc_, opart_, ofold_, bp_, rr_;
  double* pinned_ = nullptr;
  // V-cycle graph
  bool use_graph_ = graphs_enabled();
  hipStream_t gstream_ = nullptr;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t gexec_ = nullptr;
  DBuf<double> vin_, vout_;
  DBuf<double> tpart_;   // slice sums of the IB-row values on coarse levels
  std::vector<std::pair<int, int>> int_forms_;   // per level: interior boxes when timed, the form picked
  hipEvent_t est_ev_ = nullptr;   // the outer loop's estimate copy
  hipStream_t side_ = nullptr;    // the coarsest inversion beside the box inversions
  hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
  DBuf<double> coarse_aug_;       // its work matrix until the join
  bool defer_coarse_ = false;   // a member of a batch: the batch inverts the coarsest system
  bool valid_ = true;
  double setup_ms_ = 0.0;   // wall time of the latest build_all (device work included)
  int nn0_ = 0;          // size of the bordered coarsest system
  DBuf<double> aug0_;    // its assembled [A | I] while the inversion is deferred

  static bool graphs_enabled() {
    const char* e = std::getenv("IBMG_GRAPH");
    return !(e && e[0] == '0');
  }
};

}  // namespace ibmg
