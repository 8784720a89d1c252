// Batched form: many independent Stokes-IB systems (different grid sizes,
// structures and stiffnesses, one fluid and one box configuration) solved
// together.  Each system's hierarchy, IB rows, box inverses and coarsest
// inverse are built by its own single-system set-up; the batch then runs
// Alg. 1 on all of them in lockstep by level.  Level l has the same grid
// size 8 * 2^l (coarse_N * 2^l) in every system, so systems sorted by size,
// largest first, make level l's active systems a prefix [0, nact_l) and a
// level's batch vectors are nact_l level vectors back to back.  A system
// whose finest level is l joins the descent there and leaves the ascent
// there.  Per level and sweep: one stencil launch and one IB-row launch for
// L_IB, one persistent RAS launch over every (system, box) item, and the
// Gram-Schmidt kernels over all systems at once.  The outer FGMRES(m) runs
// per system in lockstep with one host read of all residual estimates per
// iteration; converged systems drop out through device-side active flags.
#include <numeric>

#include "solver_impl.hpp"

namespace ibmg {

namespace {

constexpr size_t kScalStride = 64;  // per-system smoother scalars (beta, y)

}  // namespace

// Host checks of a batch's descriptors (every one valid, the shared
// parameters equal, the options the batched form runs).
void validate_batch(int nsys, const ibmg_desc* d) {
  require(nsys >= 1 && nsys <= 4096, "nsys must lie in [1, 4096]");
  require(d != nullptr, "descs is NULL");
  const ibmg_desc& d0 = d[0];
  for (int i = 0; i < nsys; ++i) {
    validate_desc(d[i]);
    require(d[i].smoother == IBMG_RAS, "the batched form uses the additive Schwarz smoother");
    require(d[i].spring_model == IBMG_SPRING_LINEAR, "the batched form takes linear springs");
    require(d[i].combine == IBMG_COMBINE_RESTRICTED && d[i].sweep_kind == IBMG_SWEEP_FGMRES,
            "the batched form runs the restricted combination with FGMRES smoothing");
    require(d[i].coarse_N == d0.coarse_N && d[i].rho == d0.rho && d[i].mu == d0.mu && d[i].dt == d0.dt &&
                d[i].box == d0.box && d[i].overlap == d0.overlap && d[i].nu1 == d0.nu1 &&
                d[i].nu2 == d0.nu2 && d[i].precision == d0.precision && d[i].max_restart == d0.max_restart,
            "batched systems must share coarse_N, rho, mu, dt, box, overlap, nu1, nu2, precision and "
            "max_restart");
  }
}

template <typename T>
class BatchSolver final : public BatchBase {
 public:
  BatchSolver(int nsys, const ibmg_desc* d, hipStream_t s) : ns_(nsys) {
    const auto t_begin = std::chrono::steady_clock::now();
    validate_batch(nsys, d);
    const ibmg_desc& d0 = d[0];
    nu1_ = d0.nu1;
    nu2_ = d0.nu2;
    max_restart_ = d0.max_restart > 0 ? d0.max_restart : 30;
    rho_zero_ = d0.rho == 0.0;
    order_.resize(nsys);
    std::iota(order_.begin(), order_.end(), 0);
    std::stable_sort(order_.begin(), order_.end(), [&](int a, int b) { return d[a].N > d[b].N; });
    for (int p = 0; p < nsys; ++p) sys_.emplace_back(new Solver<T>(d[order_[p]], s, true));
    {
      // every system's bordered coarsest system has the same size (shared
      // coarse_N and rho): they are inverted a group at a time, one launch
      // per group of up to 1 GiB of augmented matrices
      const int nn = sys_[0]->nn0_;
      const size_t stride = (size_t)nn * 2 * nn;
      const int grp = (int)std::max<size_t>(1, std::min<size_t>(nsys, ((size_t)1 << 27) / stride));
      DBuf<double> augs(stride * grp);
      for (int p0 = 0; p0 < nsys; p0 += grp) {
        const int cnt = std::min(grp, nsys - p0);
        for (int p = p0; p < p0 + cnt; ++p) {
          require(sys_[p]->nn0_ == nn && sys_[p]->aug0_.n == stride, "coarsest systems differ in size");
          IBMG_HIP(hipMemcpyAsync(augs.p + (p - p0) * stride, sys_[p]->aug0_.p, stride * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
        }
        launch_coarse_invert(augs.p, nn, cnt, stride, s);
        for (int p = p0; p < p0 + cnt; ++p) sys_[p]->finish_coarse(augs.p + (p - p0) * stride, s);
        IBMG_HIP(hipStreamSynchronize(s));
      }
      for (int p = 0; p < nsys; ++p) sys_[p]->check_breakdown(s, true);
    }
    Lmax_ = sys_[0]->L_;
    nact_.assign(Lmax_ + 2, 0);
    for (int p = 0; p < nsys; ++p)
      for (int l = 0; l <= sys_[p]->L_; ++l) nact_[l]++;
    off_.assign(nsys + 1, 0);
    for (int p = 0; p < nsys; ++p) {
      const long long N = sys_[p]->d_.N;
      off_[p + 1] = off_[p] + 3 * N * N;
    }
    ntot_ = (size_t)off_[nsys];
    require(ntot_ < ((size_t)1 << 31), "batch too large for 32-bit indices");
    d_off_.upload(off_, s);
    std::vector<int> ones(nsys, 1);
    d_act_.upload(ones, s);
    IBMG_HIP(hipHostMalloc((void**)&pin_d_, (size_t)(2 * nsys + 8) * sizeof(double), hipHostMallocDefault));
    IBMG_HIP(hipHostMalloc((void**)&pin_i_, (size_t)(2 * nsys + 8) * sizeof(int), hipHostMallocDefault));
    build_levels(s);
    build_outer_rows(s);
    build_coarse(s);
    alloc_outer(max_restart_);
    tune(s);
    IBMG_HIP(hipStreamSynchronize(s));
    setup_ms_ = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
  }

  ~BatchSolver() override {
    drop_graph();
    if (gstream_) (void)hipStreamDestroy(gstream_);
    if (pin_d_) (void)hipHostFree(pin_d_);
    if (pin_i_) (void)hipHostFree(pin_i_);
  }

  int nsys() const override { return ns_; }

 private:
  struct BLevel {
    int N = 0, nact = 0, nblk = 1;
    size_t n = 0, pst = 0;
    StokesCoef<T> c{};
    DBuf<T> w, b, r, V, Z;
    DBuf<double> H, scal, pa, pb;
    // explicit IB rows of the level's systems, indices into the batch vector
    DBuf<int> rows, ptr, col;
    DBuf<T> val;
    int nrows = 0;
    // Schwarz boxes
    BoxGeom g{};
    int nbox = 0, n_int = 0, n_ib = 0;
    DBuf<int> int_ents, ib_ents, loc;
    DBuf<const T*> ib_inv;
    const T* shared_inv = nullptr;
    RasBatchPlan plan;
    double tuned_us = 0;
  };

  // ---------------------------------------------------------------- set-up
  template <typename U>
  static const U* tvals(const CompFoot& f) {
    if constexpr (std::is_same<U, double>::value) return f.tval.p;
    else return f.tvalf.p;
  }

  // Concatenate the IB rows of system positions [0, count) at level l (or
  // at each system's finest level when l < 0) with indices shifted by base.
  template <typename U>
  void gather_rows(int l, int count, const std::vector<size_t>& base, DBuf<int>& rows, DBuf<int>& ptr,
                   DBuf<int>& col, DBuf<U>& val, int* nrows, hipStream_t s) {
    std::vector<int> hr, hp(1, 0), hc;
    std::vector<std::pair<const U*, size_t>> pieces;
    for (int p = 0; p < count; ++p) {
      Solver<T>& S = *sys_[p];
      const int lv = l < 0 ? S.L_ : l;
      Level<T>& lev = S.levels_[lv];
      const size_t nn = (size_t)lev.N * lev.N;
      for (int c = 0; c < 2; ++c) {
        const CompFoot& f = lev.f[c];
        if (f.tcol.empty()) continue;
        const size_t b0 = base[p] + c * nn;
        for (size_t r = 0; r + 1 < f.tptr.size(); ++r) {
          if (f.tptr[r + 1] == f.tptr[r]) continue;
          hr.push_back((int)(b0 + r));
          hp.push_back(hp.back() + (f.tptr[r + 1] - f.tptr[r]));
        }
        // columns index the system's [u | v] vector
        for (int cc : f.tcol) hc.push_back((int)(base[p] + cc));
        pieces.emplace_back(tvals<U>(f), f.tcol.size());
      }
    }
    *nrows = (int)hr.size();
    rows.upload(hr, s);
    ptr.upload(hp, s);
    col.upload(hc, s);
    val.alloc(hc.size());
    size_t at = 0;
    for (auto& pc : pieces) {
      IBMG_HIP(hipMemcpyAsync(val.p + at, pc.first, pc.second * sizeof(U), hipMemcpyDeviceToDevice, s));
      at += pc.second;
    }
  }

  void build_levels(hipStream_t s) {
    lv_.resize(Lmax_ + 1);
    for (int l = 0; l <= Lmax_; ++l) {
      BLevel& L = lv_[l];
      Level<T>& l0 = sys_[0]->levels_[l];
      L.N = l0.N;
      L.n = 3 * (size_t)L.N * L.N;
      L.nact = nact_[l];
      L.c = sys_[0]->template coef<T>(l0);
      const size_t bn = (size_t)L.nact * L.n;
      L.w.alloc(bn);
      L.b.alloc(bn);
      L.r.alloc(bn);
      launch_fill<T>(L.w.p, T(0), bn, s);
      launch_fill<T>(L.b.p, T(0), bn, s);
      launch_fill<T>(L.r.p, T(0), bn, s);
      if (l == 0) continue;
      const int nv = std::max(nu1_, nu2_);
      L.V.alloc((size_t)(nv + 1) * bn);
      L.Z.alloc((size_t)nv * bn);
      launch_fill<T>(L.V.p, T(0), L.V.n, s);
      launch_fill<T>(L.Z.p, T(0), L.Z.n, s);
      L.nblk = dots_blocks(L.n, 1024);
      L.pst = (size_t)L.nblk * (kMaxNu + 1);
      L.pa.alloc((size_t)L.nact * L.pst);
      L.pb.alloc((size_t)L.nact * L.pst);
      L.H.alloc((size_t)L.nact * (kMaxNu + 1) * kMaxNu);
      L.scal.alloc((size_t)L.nact * kScalStride);
      std::vector<size_t> base(L.nact);
      for (int p = 0; p < L.nact; ++p) base[p] = (size_t)p * L.n;
      gather_rows<T>(l, L.nact, base, L.rows, L.ptr, L.col, L.val, &L.nrows, s);
      // Schwarz items: (system, box) entries, own inverses for IB boxes, the
      // first available interior inverse for every interior box (equal
      // fluid coefficients and box geometry give one interior matrix)
      L.g = l0.g;
      L.nbox = L.g.npd * L.g.npd;
      require((size_t)L.nact * L.nbox < ((size_t)1 << 31), "too many boxes");
      std::vector<int> ie, be;
      std::vector<const T*> bi;
      const size_t stride = sys_[0]->box_stride(l0);
      for (int p = 0; p < L.nact; ++p) {
        Level<T>& lev = sys_[p]->levels_[l];
        for (int i = 0; i < lev.n_ib; ++i) {
          be.push_back(p * L.nbox + lev.ib_list[i]);
          bi.push_back(lev.inv.p + (size_t)i * stride);
        }
        for (int q : lev.int_list) ie.push_back(p * L.nbox + q);
        if (!L.shared_inv && !lev.int_list.empty()) L.shared_inv = lev.inv.p + (size_t)lev.n_ib * stride;
      }
      L.n_int = (int)ie.size();
      L.n_ib = (int)be.size();
      L.int_ents.upload(ie, s);
      L.ib_ents.upload(be, s);
      L.ib_inv.upload(bi, s);
      L.loc.upload(l0.loc_tab, s);
    }
    n0_ = sys_[0]->n0_;
  }

  // IB rows of every system at its finest level, indexed into the ragged
  // outer vectors (FP64: the outer residual stays in double precision).
  void build_outer_rows(hipStream_t s) {
    std::vector<size_t> base(ns_);
    for (int p = 0; p < ns_; ++p) base[p] = (size_t)off_[p];
    gather_rows<double>(-1, ns_, base, orows_, optr_, ocol_, oval_, &onrows_, s);
  }

  void build_coarse(hipStream_t s) {
    inv0_.alloc((size_t)ns_ * n0_ * n0_);
    for (int p = 0; p < ns_; ++p)
      IBMG_HIP(hipMemcpyAsync(inv0_.p + (size_t)p * n0_ * n0_, sys_[p]->inv0_.p, (size_t)n0_ * n0_ * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
  }

  // Autotuner: time every (tile width, persistent grid) candidate of each
  // level's Schwarz launch with HIP events and keep the fastest.  All
  // candidates compute the same sums in the same order, so the choice
  // changes the time only.
  void tune(hipStream_t s) {
    if (dry_run()) return;
    hipEvent_t e0, e1;
    IBMG_HIP(hipEventCreate(&e0));
    IBMG_HIP(hipEventCreate(&e1));
    try {
      for (int l = 1; l <= Lmax_; ++l) {
        BLevel& L = lv_[l];
        launch_fill<T>(L.r.p, T(1), (size_t)L.nact * L.n, s);
        double best = 1e300;
        for (int tb : {16, 32, 64}) {
          const int items = ras_batch_items(L.g, L.n_int, L.n_ib, tb);
          if (items <= 0) continue;
          std::vector<int> grids;
          for (int gsz : {256, 512, 1024, 2048, 4096})
            if (gsz < items) grids.push_back(gsz);
          grids.push_back(items);
          for (int gsz : grids) {
            RasBatchPlan pl{tb, gsz};
            ras(l, L.r.p, L.w.p, pl, s);
            IBMG_HIP(hipEventRecord(e0, s));
            constexpr int reps = 5;
            for (int k = 0; k < reps; ++k) ras(l, L.r.p, L.w.p, pl, s);
            IBMG_HIP(hipEventRecord(e1, s));
            IBMG_HIP(hipEventSynchronize(e1));
            float ms = 0;
            IBMG_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1e3 * ms / reps;
            if (us < best) {
              best = us;
              L.plan = pl;
            }
          }
        }
        L.tuned_us = best < 1e300 ? best : 0.0;
        launch_fill<T>(L.r.p, T(0), (size_t)L.nact * L.n, s);
        launch_fill<T>(L.w.p, T(0), (size_t)L.nact * L.n, s);
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    IBMG_HIP(hipEventDestroy(e0));
    IBMG_HIP(hipEventDestroy(e1));
  }

  // --------------------------------------------------------- level pieces
  void ras(int l, const T* r, T* z, RasBatchPlan pl, hipStream_t s) {
    BLevel& L = lv_[l];
    launch_ras_batch<T>(r, z, L.g, L.n, L.nbox, L.shared_inv, L.int_ents.p, L.n_int, L.ib_ents.p, L.ib_inv.p,
                        L.n_ib, L.loc.p, d_act_.p, pl, s);
  }

  // y = L_IB x on level l for every active system (b != null: y = b - L_IB x)
  void op(int l, const T* x, T* y, const T* b, hipStream_t s) {
    BLevel& L = lv_[l];
    launch_apply_batch<T>(x, y, b, L.N, L.c, L.nact, L.n, s);
    launch_ib_rows<T>(x, y, L.rows.p, L.ptr.p, L.col.p, L.val.p, L.nrows, b ? T(-1) : T(1), s);
  }

  // Sec. 3.3 smoothing on every system of level l: w <- w + e, e from nu
  // FGMRES iterations (classical Gram-Schmidt twice) on L e = b - L w.
  void smooth(int l, T* w, const T* b, int nu, bool w_zero, hipStream_t s) {
    BLevel& L = lv_[l];
    const int ns = L.nact;
    const size_t n = L.n, bn = (size_t)ns * n;
    const BSeg sg{nullptr, n, d_act_.p};
    const int ldh = kMaxNu + 1;
    const size_t hst = (size_t)(kMaxNu + 1) * kMaxNu;
    const T* r0;
    if (w_zero) {
      launch_fill<T>(w, T(0), bn, s);
      r0 = b;
    } else {
      op(l, w, L.r.p, b, s);
      r0 = L.r.p;
    }
    launch_dots_b<T>(r0, 1, bn, r0, sg, ns, L.pa.p, L.pst, L.nblk, s);
    launch_scale_red_b<T>(r0, L.V.p, sg, ns, n, L.pa.p, L.nblk, L.pst, L.scal.p, kScalStride, s);
    for (int k = 0; k < nu; ++k) {
      T* vk = L.V.p + (size_t)k * bn;
      T* zk = L.Z.p + (size_t)k * bn;
      T* t = L.V.p + (size_t)(k + 1) * bn;
      ras(l, vk, zk, L.plan, s);
      op(l, zk, t, nullptr, s);
      double* hcol = L.H.p + (size_t)k * ldh;
      launch_dots_b<T>(L.V.p, k + 1, bn, t, sg, ns, L.pa.p, L.pst, L.nblk, s);
      // the second pass with |t|^2 beside its dots; one more sweep updates
      // and normalises (the norm from those sums), none for the last basis
      // vector, whose coefficients and norm go straight to the least squares
      launch_upd_dots_b<T>(t, L.V.p, k + 1, bn, sg, ns, L.pa.p, L.nblk, L.pst, hcol, hst, L.pb.p, s, 0, true);
      if (k + 1 < nu)
        launch_scale_upd_b<T>(t, L.V.p, k + 1, bn, sg, ns, n, L.pb.p, L.nblk, L.pst, hcol, hst, s);
    }
    launch_combine_ls_b<T>(w, L.Z.p, nu, bn, sg, ns, n, L.H.p, ldh, hst, L.scal.p, L.scal.p + kScalY,
                           kScalStride, s, false, L.pb.p, L.nblk, L.pst, true);
  }

  // Alg. 1 on every system: r and z are ragged batch vectors (FP64).
  void vcycle_body(const double* r, double* z, hipStream_t s) {
    for (int l = Lmax_; l >= 1; --l) {
      BLevel& L = lv_[l];
      const int p0 = nact_[l + 1], p1 = nact_[l];
      if (p1 > p0) launch_cast<double, T>(r + off_[p0], L.b.p + (size_t)p0 * L.n, (size_t)(p1 - p0) * L.n, s);
      smooth(l, L.w.p, L.b.p, nu1_, true, s);
      op(l, L.w.p, L.r.p, L.b.p, s);
      launch_restrict_batch<T>(L.r.p, lv_[l - 1].b.p, lv_[l - 1].N, p1, s);
    }
    launch_coarse_apply_batch<T>(inv0_.p, n0_, lv_[0].b.p, lv_[0].w.p, nact_[0], s);
    for (int l = 1; l <= Lmax_; ++l) {
      BLevel& L = lv_[l];
      const int p0 = nact_[l + 1], p1 = nact_[l];
      launch_prolong_add_batch<T>(lv_[l - 1].w.p, L.w.p, lv_[l - 1].N, p1, s);
      smooth(l, L.w.p, L.b.p, nu2_, false, s);
      if (p1 > p0) launch_cast<T, double>(L.w.p + (size_t)p0 * L.n, z + off_[p0], (size_t)(p1 - p0) * L.n, s);
    }
  }

  // The batched V-cycle is captured once into a HIP graph (kernel nodes
  // only) reading vin_ and writing vout_.
  void build_graph() {
    if (!gstream_) IBMG_HIP(hipStreamCreateWithFlags(&gstream_, hipStreamNonBlocking));
    launch_fill<double>(vin_.p, 0.0, ntot_, gstream_);
    launch_fill<double>(vout_.p, 0.0, ntot_, gstream_);
    IBMG_HIP(hipStreamSynchronize(gstream_));
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

  void vcycle_ragged(const double* r, double* z, hipStream_t s) {
    if (!use_graph_) {
      vcycle_body(r, z, s);
      return;
    }
    if (!gexec_) build_graph();
    IBMG_HIP(hipMemcpyAsync(vin_.p, r, ntot_ * sizeof(double), hipMemcpyDeviceToDevice, s));
    IBMG_HIP(hipGraphLaunch(gexec_, s));
    IBMG_HIP(hipMemcpyAsync(z, vout_.p, ntot_ * sizeof(double), hipMemcpyDeviceToDevice, s));
  }

  void gather(const double* const* src, double* dst, hipStream_t s) {
    for (int p = 0; p < ns_; ++p) {
      require(src[order_[p]] != nullptr, "NULL system vector");
      IBMG_HIP(hipMemcpyAsync(dst + off_[p], src[order_[p]], (size_t)(off_[p + 1] - off_[p]) * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    }
  }

  void scatter(const double* src, double* const* dst, hipStream_t s) {
    for (int p = 0; p < ns_; ++p) {
      require(dst[order_[p]] != nullptr, "NULL system vector");
      IBMG_HIP(hipMemcpyAsync(dst[order_[p]], src + off_[p], (size_t)(off_[p + 1] - off_[p]) * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    }
  }

 public:
  void vcycle(const double* const* r, double* const* z, hipStream_t s) override {
    require(r && z, "NULL pointer array");
    set_all_active(s);
    gather(r, io_in_.p, s);
    vcycle_ragged(io_in_.p, io_out_.p, s);
    scatter(io_out_.p, z, s);
  }

 private:

  void set_all_active(hipStream_t s) {
    for (int p = 0; p < ns_; ++p) pin_i_[p] = 1;
    IBMG_HIP(hipMemcpyAsync(d_act_.p, pin_i_, ns_ * sizeof(int), hipMemcpyHostToDevice, s));
    IBMG_HIP(hipStreamSynchronize(s));
  }

  // --------------------------------------------------------- outer solve
  // y = L_IB x (b != null: y = b - L_IB x) on every system's finest level,
  // FP64, over the ragged vectors: one stencil launch per grid size.
  void op_outer(const double* x, double* y, const double* b, hipStream_t s) {
    for (int l = Lmax_; l >= 1; --l) {
      const int p0 = nact_[l + 1], p1 = nact_[l];
      if (p1 <= p0) continue;
      Level<T>& lev = sys_[p0]->levels_[l];
      launch_apply_batch<double>(x + off_[p0], y + off_[p0], b ? b + off_[p0] : nullptr, lev.N, lev.cd, p1 - p0,
                                 lv_[l].n, s);
    }
    launch_ib_rows<double>(x, y, orows_.p, optr_.p, ocol_.p, oval_.p, onrows_, b ? -1.0 : 1.0, s);
  }

  // remove the null-space components of every system's vector; the block
  // sums are left at osums_ + 8 p
  void project(double* a, hipStream_t s) {
    for (int l = Lmax_; l >= 1; --l) {
      const int p0 = nact_[l + 1], p1 = nact_[l];
      if (p1 <= p0) continue;
      const int N = lv_[l].N;
      const size_t n = lv_[l].n;
      launch_block_sums_b<double>(a + off_[p0], N, n, ppart_.p + (size_t)p0 * 64 * 3, 64, 64 * 3, p1 - p0, s);
      launch_dots_finish_b(ppart_.p + (size_t)p0 * 64 * 3, 3, 64, 64 * 3, osums_.p + (size_t)p0 * 8, nullptr, 8,
                           0, p1 - p0, s);
      launch_subtract_means_b<double>(a + off_[p0], N, n, osums_.p + (size_t)p0 * 8, 8, rho_zero_ ? 1 : 0, p1 - p0,
                                      s);
    }
  }

  // per-system 2-norms into onorm_ and pin_d_[0..ns)
  void norms(const double* a, hipStream_t s) {
    const BSeg sg{d_off_.p, 0, nullptr};
    launch_dots_b<double>(a, 1, ntot_, a, sg, ns_, opa_.p, opst_, onblk_, s);
    launch_dots_finish_b(opa_.p, 1, onblk_, opst_, onorm_.p, nullptr, 1, 2, ns_, s);
    IBMG_HIP(hipMemcpyAsync(pin_d_, onorm_.p, ns_ * sizeof(double), hipMemcpyDeviceToHost, s));
    IBMG_HIP(hipStreamSynchronize(s));
  }

  // every buffer of the outer solve and the V-cycle's input and output,
  // for restarts up to max_restart (placed at creation)
  void alloc_outer(int restart) {
    io_in_.alloc(ntot_);
    io_out_.alloc(ntot_);
    vin_.alloc(ntot_);
    vout_.alloc(ntot_);
    Vo_.alloc((size_t)(restart + 1) * ntot_);
    Zo_.alloc((size_t)restart * ntot_);
    launch_fill<double>(Vo_.p, 0.0, Vo_.n, nullptr);
    launch_fill<double>(Zo_.p, 0.0, Zo_.n, nullptr);
    ldh_ = restart + 1;
    hst_ = (size_t)(restart + 1) * restart;
    rst_ = (size_t)restart + 2;
    Ho_.alloc((size_t)ns_ * hst_);
    cs_.alloc((size_t)ns_ * rst_);
    sn_.alloc((size_t)ns_ * rst_);
    g_.alloc((size_t)ns_ * rst_);
    y_.alloc((size_t)ns_ * rst_);
    est_.alloc(ns_);
    onorm_.alloc(ns_);
    osums_.alloc((size_t)ns_ * 8);
    ppart_.alloc((size_t)ns_ * 64 * 3);
    size_t nmax = 0;
    for (int p = 0; p < ns_; ++p) nmax = std::max(nmax, (size_t)(off_[p + 1] - off_[p]));
    onblk_ = dots_blocks(nmax, 256);
    opst_ = (size_t)onblk_ * (restart + 1);
    opa_.alloc((size_t)ns_ * opst_);
    opb_.alloc((size_t)ns_ * opst_);
    bp_.alloc(ntot_);
    xb_.alloc(ntot_);
    rr_.alloc(ntot_);
    kcnt_.alloc(ns_);
    nmax_ = nmax;
    outer_cap_ = restart;
  }

  void upload_flags(const std::vector<int>& act, hipStream_t s) {
    for (int p = 0; p < ns_; ++p) pin_i_[p] = act[p];
    IBMG_HIP(hipMemcpyAsync(d_act_.p, pin_i_, ns_ * sizeof(int), hipMemcpyHostToDevice, s));
  }

 public:
  int fgmres(const double* const* b, double* const* x, const ibmg_solve_opts& o, ibmg_solve_info* infos,
             hipStream_t s) override {
    const auto t0 = std::chrono::steady_clock::now();
    require(b && x, "NULL pointer array");
    require(o.restart >= 1 && o.restart <= outer_cap_,
            "restart must lie in [1, max_restart = " + std::to_string(outer_cap_) + "]");
    require(o.max_it >= 1, "max_it must be >= 1");
    require(std::isfinite(o.rtol) && o.rtol > 0.0, "rtol must be finite and > 0");
    require(o.transpose == 0, "the batched form solves with L_IB only");
    const int m = o.restart;
    set_all_active(s);
    gather(b, bp_.p, s);
    project(bp_.p, s);
    // removed null-space norms
    std::vector<double> sums((size_t)ns_ * 8);
    IBMG_HIP(hipMemcpyAsync(sums.data(), osums_.p, sums.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    norms(bp_.p, s);
    std::vector<double> bnorm(pin_d_, pin_d_ + ns_), target(ns_), est(ns_), null(ns_);
    for (int p = 0; p < ns_; ++p) {
      const double nn = (double)(off_[p + 1] - off_[p]) / 3.0;
      double n2 = sums[8 * p + 2] * sums[8 * p + 2] / nn;
      if (rho_zero_) n2 += (sums[8 * p] * sums[8 * p] + sums[8 * p + 1] * sums[8 * p + 1]) / nn;
      null[p] = std::sqrt(n2);
      if (!std::isfinite(bnorm[p]) || !std::isfinite(n2)) throw Error(IBMG_ERR_NONFINITE, "right-hand side holds NaN/Inf");
      target[p] = o.rtol * bnorm[p];
      est[p] = bnorm[p];
    }
    if (o.use_x0) gather(const_cast<const double* const*>(x), xb_.p, s);
    else launch_fill<double>(xb_.p, 0.0, ntot_, s);
    std::vector<int> its(ns_, 0), conv(ns_, 0), act(ns_, 0), kc(ns_, 0), restarts(ns_, 0), vcyc(ns_, 0);
    std::vector<int> hist_n(ns_, 0);
    auto push_hist = [&](int p, double v) {
      ibmg_solve_info* inf = infos ? &infos[order_[p]] : nullptr;
      if (inf && inf->history && hist_n[p] < inf->history_cap) inf->history[hist_n[p]] = v;
      ++hist_n[p];
    };
    for (int p = 0; p < ns_; ++p)
      if (bnorm[p] == 0.0) conv[p] = 1;
    const BSeg sga{d_off_.p, 0, d_act_.p};
    const BSeg sgall{d_off_.p, 0, nullptr};
    while (true) {
      // restart: V0 = (b - L x) / beta for the systems still running
      op_outer(xb_.p, Vo_.p, bp_.p, s);
      norms(Vo_.p, s);
      int nrun = 0;
      for (int p = 0; p < ns_; ++p) {
        act[p] = 0;
        if (conv[p]) continue;
        const double beta = pin_d_[p];
        if (!std::isfinite(beta)) throw Error(IBMG_ERR_NONFINITE, "residual is not finite");
        est[p] = beta;
        if (beta <= target[p]) {
          conv[p] = 1;
          continue;
        }
        if (its[p] >= o.max_it) continue;
        act[p] = 1;
        ++nrun;
      }
      if (nrun == 0) break;
      upload_flags(act, s);
      launch_scale_b<double>(Vo_.p, Vo_.p, onorm_.p, 1, sga, ns_, nmax_, s);
      launch_fill<double>(g_.p, 0.0, g_.n, s);
      IBMG_HIP(hipMemcpy2DAsync(g_.p, rst_ * sizeof(double), onorm_.p, sizeof(double), sizeof(double), ns_,
                                hipMemcpyDeviceToDevice, s));
      std::fill(kc.begin(), kc.end(), 0);
      for (int k = 0; k < m && nrun > 0; ++k) {
        double* vk = Vo_.p + (size_t)k * ntot_;
        double* zk = Zo_.p + (size_t)k * ntot_;
        double* t = Vo_.p + (size_t)(k + 1) * ntot_;
        vcycle_ragged(vk, zk, s);
        op_outer(zk, t, nullptr, s);
        double* hcol = Ho_.p + (size_t)k * ldh_;
        launch_dots_b<double>(Vo_.p, k + 1, ntot_, t, sga, ns_, opa_.p, opst_, onblk_, s);
        launch_upd_dots_b<double>(t, Vo_.p, k + 1, ntot_, sga, ns_, opa_.p, onblk_, opst_, hcol, hst_, opb_.p, s);
        launch_upd_norm_b<double>(t, Vo_.p, k + 1, ntot_, sga, ns_, opb_.p, onblk_, opst_, hcol, hst_, opa_.p, s);
        launch_scale_red_b<double>(t, t, sga, ns_, nmax_, opa_.p, onblk_, opst_, hcol + k + 1, hst_, s);
        launch_givens_b(Ho_.p, ldh_, hst_, k, cs_.p, sn_.p, g_.p, rst_, est_.p, d_act_.p, ns_, s);
        IBMG_HIP(hipMemcpyAsync(pin_d_, est_.p, ns_ * sizeof(double), hipMemcpyDeviceToHost, s));
        IBMG_HIP(hipStreamSynchronize(s));
        bool changed = false;
        for (int p = 0; p < ns_; ++p) {
          if (!act[p]) continue;
          const double e = pin_d_[p];
          if (!std::isfinite(e)) throw Error(IBMG_ERR_NONFINITE, "iteration produced NaN/Inf");
          est[p] = e;
          ++its[p];
          ++vcyc[p];
          kc[p] = k + 1;
          push_hist(p, e / bnorm[p]);
          if (e <= target[p]) conv[p] = 1;
          if (conv[p] || its[p] >= o.max_it) {
            act[p] = 0;
            --nrun;
            changed = true;
          }
        }
        if (changed && nrun > 0) upload_flags(act, s);
      }
      for (int p = 0; p < ns_; ++p) {
        pin_i_[ns_ + p] = kc[p];
        if (kc[p] > 0) ++restarts[p];
      }
      IBMG_HIP(hipMemcpyAsync(kcnt_.p, pin_i_ + ns_, ns_ * sizeof(int), hipMemcpyHostToDevice, s));
      launch_backsolve_b(Ho_.p, ldh_, hst_, kcnt_.p, g_.p, y_.p, rst_, ns_, s);
      launch_combine_b<double>(xb_.p, Zo_.p, ntot_, y_.p, rst_, kcnt_.p, sgall, ns_, nmax_, s);
      IBMG_HIP(hipStreamSynchronize(s));
      bool more = false;
      for (int p = 0; p < ns_; ++p)
        if (!conv[p] && its[p] < o.max_it) more = true;
      if (!more) break;
    }
    set_all_active(s);
    project(xb_.p, s);
    op_outer(xb_.p, rr_.p, bp_.p, s);
    norms(rr_.p, s);
    std::vector<double> tr(pin_d_, pin_d_ + ns_);
    scatter(xb_.p, x, s);
    IBMG_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    for (int p = 0; p < ns_; ++p) {
      if (!std::isfinite(tr[p])) throw Error(IBMG_ERR_NONFINITE, "solution is not finite");
      all = all && conv[p];
      if (!infos) continue;
      ibmg_solve_info& inf = infos[order_[p]];
      inf.iters = its[p];
      inf.restarts = restarts[p];
      inf.rel_res_est = bnorm[p] > 0 ? est[p] / bnorm[p] : 0.0;
      inf.rel_res_true = bnorm[p] > 0 ? tr[p] / bnorm[p] : 0.0;
      inf.rhs_null_norm = null[p];
      inf.setup_ms = setup_ms_;
      inf.solve_ms = ms;
      inf.vcycles = vcyc[p];
    }
    return all ? IBMG_OK : IBMG_NOT_CONVERGED;
  }

  // The persistent Schwarz launch of a batch level alone, on the level's
  // work vectors (filled with ones), with the tuned plan.  Algorithmic work:
  // each IB box streams its owned inverse rows, the interior product reads
  // the shared inverse once; every box gathers nloc values and writes nown.
  double kernel_time(int kernel, int level, int reps, hipStream_t s, double* bytes, double* flops) override {
    require(kernel == IBMG_KERNEL_RAS_BATCH, "batch handles time the batched Schwarz launch only");
    require(level >= 1 && level <= Lmax_, "level out of range");
    require(reps >= 1 && reps <= 100000, "reps must lie in [1, 100000]");
    BLevel& L = lv_[level];
    set_all_active(s);
    launch_fill<T>(L.r.p, T(1), (size_t)L.nact * L.n, s);
    const double ts = sizeof(T);
    const BoxGeom& g = L.g;
    double by = (double)L.n_ib * ((double)g.nown * g.nloc + g.nloc + g.nown) * ts +
                (double)L.n_int * (g.nloc + g.nown) * ts;
    if (L.n_int > 0) by += (double)g.nown * g.nloc * ts;
    const double ms = time_launches([&] { ras(level, L.r.p, L.w.p, L.plan, s); }, reps, s);
    if (bytes) *bytes = by;
    if (flops) *flops = 2.0 * (double)(L.n_ib + L.n_int) * g.nown * g.nloc;
    return ms;
  }

  // [nsys, levels, then per level: N, systems, interior boxes, IB boxes,
  //  IB rows, tile width, persistent grid, tuned sweep time (ns)]
  std::vector<int64_t> stats() const override {
    std::vector<int64_t> v{ns_, Lmax_ + 1};
    for (int l = 0; l <= Lmax_; ++l) {
      const BLevel& L = lv_[l];
      v.push_back(L.N);
      v.push_back(L.nact);
      v.push_back(L.n_int);
      v.push_back(L.n_ib);
      v.push_back(L.nrows);
      v.push_back(L.plan.tb);
      v.push_back(L.plan.grid);
      v.push_back((int64_t)(L.tuned_us * 1e3));
    }
    return v;
  }

 private:
  int ns_ = 0, Lmax_ = 0, nu1_ = 2, nu2_ = 2, n0_ = 0, max_restart_ = 30;
  double setup_ms_ = 0.0;   // wall time of the constructor's set-up (device work included)
  bool rho_zero_ = false;
  std::vector<int> order_, nact_;
  std::vector<std::unique_ptr<Solver<T>>> sys_;
  std::vector<BLevel> lv_;
  std::vector<long long> off_;
  size_t ntot_ = 0, nmax_ = 0;
  DBuf<long long> d_off_;
  DBuf<int> d_act_, kcnt_;
  DBuf<double> inv0_;
  DBuf<int> orows_, optr_, ocol_;
  DBuf<double> oval_;
  int onrows_ = 0;
  // outer FGMRES
  int outer_cap_ = 0, ldh_ = 0, onblk_ = 1;
  size_t hst_ = 0, rst_ = 0, opst_ = 0;
  DBuf<double> Vo_, Zo_, Ho_, cs_, sn_, g_, y_, est_, onorm_, osums_, ppart_, opa_, opb_, bp_, xb_, rr_;
  DBuf<double> io_in_, io_out_;
  double* pin_d_ = nullptr;
  int* pin_i_ = nullptr;
  // V-cycle graph
  bool use_graph_ = graphs_on();
  hipStream_t gstream_ = nullptr;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t gexec_ = nullptr;
  DBuf<double> vin_, vout_;

  static bool graphs_on() {
    const char* e = std::getenv("IBMG_GRAPH");
    return !(e && e[0] == '0');
  }
};

BatchBase* make_batch(int nsys, const ibmg_desc* d, hipStream_t s) {
  require(nsys >= 1 && d != nullptr, "nsys must be >= 1 and descs non-NULL");
  if (d[0].precision == IBMG_FP32_SMOOTHER) return new BatchSolver<float>(nsys, d, s);
  return new BatchSolver<double>(nsys, d, s);
}

}  // namespace ibmg
