// extern "C" entry points of libibmg (declared in include/ibmg.h): argument
// checks, error translation and dispatch to the solver object.
#include <cmath>
#include <mutex>

#include "solver.hpp"

struct ibmg_handle {
  // the caller's workspace: every device buffer of the handle lies in it
  std::unique_ptr<ibmg::Arena> arena;
  ibmg::SolverBase* s = nullptr;  // single system
  ibmg::BatchBase* b = nullptr;   // batched systems
  std::string err;
  ~ibmg_handle() {
    ibmg::ArenaScope as(arena.get());
    delete s;
    delete b;
  }
};

namespace {

thread_local std::string g_create_error;

template <typename F>
ibmg_status guarded(ibmg_handle* h, F&& f) {
  if (!h || !h->s) return IBMG_ERR_STATE;
  if (!h->s->valid()) {
    h->err = "the handle lost its set-up in a failed rebuild";
    return IBMG_ERR_STATE;
  }
  try {
    ibmg::ArenaScope as(h->arena.get());
    return (ibmg_status)f(h->s);
  } catch (const ibmg::Error& e) {
    h->err = e.what();
    return (ibmg_status)e.code;
  } catch (const std::exception& e) {
    h->err = e.what();
    return IBMG_ERR_HIP;
  }
}

template <typename F>
ibmg_status guarded_b(ibmg_handle* h, F&& f) {
  if (!h || !h->b) return IBMG_ERR_STATE;
  try {
    ibmg::ArenaScope as(h->arena.get());
    return (ibmg_status)f(h->b);
  } catch (const ibmg::Error& e) {
    h->err = e.what();
    return (ibmg_status)e.code;
  } catch (const std::exception& e) {
    h->err = e.what();
    return IBMG_ERR_HIP;
  }
}

hipStream_t S(ibmg_stream s) { return reinterpret_cast<hipStream_t>(s); }

void check_level(ibmg::SolverBase* s, int level, int lo) {
  ibmg::require(level >= lo && level < s->levels(), "level out of range");
}

// Runs make() with the thread's errors caught into g_create_error.
template <typename F>
ibmg_status creating(F&& make) {
  try {
    return make();
  } catch (const ibmg::Error& e) {
    g_create_error = e.what();
    return (ibmg_status)e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return IBMG_ERR_HIP;
  }
}

// The set-up's sizing pass: placement without device work.
template <typename F>
size_t sizing_pass(F&& build) {
  ibmg::Arena a = ibmg::Arena::sizing();
  {
    ibmg::ArenaScope as(&a);
    ibmg::DryScope dry;
    build();
  }
  return a.peak();
}

void check_workspace(void* ws, size_t bytes) {
  if (!ws || bytes == 0) throw ibmg::Error(IBMG_ERR_WORKSPACE, "workspace is NULL or empty");
  if ((uintptr_t)ws % ibmg::Arena::kAlign != 0)
    throw ibmg::Error(IBMG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
}

}  // namespace

extern "C" {

ibmg_status ibmg_workspace_bytes(const ibmg_desc* desc, size_t* bytes) {
  if (!desc || !bytes) {
    g_create_error = "desc or bytes is NULL";
    return IBMG_ERR_ARG;
  }
  return creating([&] {
    *bytes = sizing_pass([&] { std::unique_ptr<ibmg::SolverBase> s(ibmg::make_solver(*desc, nullptr)); });
    return IBMG_OK;
  });
}

ibmg_status ibmg_create(const ibmg_desc* desc, void* workspace, size_t bytes, ibmg_stream stream,
                        ibmg_handle** out) {
  if (!out) return IBMG_ERR_ARG;
  *out = nullptr;
  if (!desc) {
    g_create_error = "desc is NULL";
    return IBMG_ERR_ARG;
  }
  return creating([&] {
    ibmg::validate_desc(*desc);
    check_workspace(workspace, bytes);
    std::unique_ptr<ibmg_handle> h(new ibmg_handle());
    h->arena.reset(new ibmg::Arena(workspace, bytes));
    {
      ibmg::ArenaScope as(h->arena.get());
      h->s = ibmg::make_solver(*desc, S(stream));
    }
    *out = h.release();
    return IBMG_OK;
  });
}

ibmg_status ibmg_workspace_used(const ibmg_handle* h, size_t* in_use, size_t* peak) {
  if (!h || !h->arena) return IBMG_ERR_STATE;
  if (in_use) *in_use = h->arena->in_use();
  if (peak) *peak = h->arena->peak();
  return IBMG_OK;
}

ibmg_status ibmg_destroy(ibmg_handle* h) {
  if (!h) return IBMG_ERR_STATE;
  delete h;
  return IBMG_OK;
}

ibmg_status ibmg_batch_workspace_bytes(int32_t nsys, const ibmg_desc* descs, size_t* bytes) {
  if (!descs || !bytes || nsys < 1) {
    g_create_error = "descs or bytes is NULL, or nsys < 1";
    return IBMG_ERR_ARG;
  }
  return creating([&] {
    *bytes = sizing_pass([&] { std::unique_ptr<ibmg::BatchBase> b(ibmg::make_batch(nsys, descs, nullptr)); });
    return IBMG_OK;
  });
}

ibmg_status ibmg_batch_create(int32_t nsys, const ibmg_desc* descs, void* workspace, size_t bytes,
                              ibmg_stream stream, ibmg_handle** out) {
  if (!out) return IBMG_ERR_ARG;
  *out = nullptr;
  if (!descs || nsys < 1) {
    g_create_error = "descs is NULL or nsys < 1";
    return IBMG_ERR_ARG;
  }
  return creating([&] {
    ibmg::validate_batch(nsys, descs);
    check_workspace(workspace, bytes);
    std::unique_ptr<ibmg_handle> h(new ibmg_handle());
    h->arena.reset(new ibmg::Arena(workspace, bytes));
    {
      ibmg::ArenaScope as(h->arena.get());
      h->b = ibmg::make_batch(nsys, descs, S(stream));
    }
    *out = h.release();
    return IBMG_OK;
  });
}

ibmg_status ibmg_batch_size(const ibmg_handle* h, int32_t* nsys) {
  if (!h || !h->b) return IBMG_ERR_STATE;
  if (!nsys) return IBMG_ERR_ARG;
  *nsys = h->b->nsys();
  return IBMG_OK;
}

ibmg_status ibmg_batch_vcycle(ibmg_handle* h, const double* const* r, double* const* z, ibmg_stream st) {
  return guarded_b(h, [&](ibmg::BatchBase* b) {
    b->vcycle(r, z, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_batch_fgmres_solve(ibmg_handle* h, const double* const* b, double* const* x,
                                    const ibmg_solve_opts* opts, ibmg_solve_info* infos, ibmg_stream st) {
  return guarded_b(h, [&](ibmg::BatchBase* bs) {
    ibmg_solve_opts o{1e-8, 30, 100, 0, 0};
    if (opts) o = *opts;
    return bs->fgmres(b, x, o, infos, S(st));
  });
}

ibmg_status ibmg_kernel_time(ibmg_handle* h, int32_t kernel, int32_t level, int32_t reps, ibmg_stream st,
                             double* avg_ms, double* alg_bytes, double* alg_flops) {
  if (!h || (!h->s && !h->b)) return IBMG_ERR_STATE;
  if (!avg_ms) return IBMG_ERR_ARG;
  if (h->s && !h->s->valid()) return IBMG_ERR_STATE;
  try {
    ibmg::ArenaScope as(h->arena.get());
    *avg_ms = h->s ? h->s->kernel_time(kernel, level, reps, S(st), alg_bytes, alg_flops)
                   : h->b->kernel_time(kernel, level, reps, S(st), alg_bytes, alg_flops);
    return IBMG_OK;
  } catch (const ibmg::Error& e) {
    h->err = e.what();
    return (ibmg_status)e.code;
  } catch (const std::exception& e) {
    h->err = e.what();
    return IBMG_ERR_HIP;
  }
}

ibmg_status ibmg_batch_stats(const ibmg_handle* h, int64_t* out, int32_t cap, int32_t* written) {
  if (!h || !h->b) return IBMG_ERR_STATE;
  if (!written || (cap > 0 && !out)) return IBMG_ERR_ARG;
  std::vector<int64_t> v = h->b->stats();
  int n = 0;
  for (; n < (int)v.size() && n < cap; ++n) out[n] = v[n];
  *written = (int32_t)v.size();
  return IBMG_OK;
}

const char* ibmg_last_error(const ibmg_handle* h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

ibmg_status ibmg_levels(const ibmg_handle* h, int32_t* n_levels) {
  if (!h || !h->s) return IBMG_ERR_STATE;
  if (!n_levels) return IBMG_ERR_ARG;
  *n_levels = h->s->levels();
  return IBMG_OK;
}

ibmg_status ibmg_level_n(const ibmg_handle* h, int32_t level, int32_t* n) {
  if (!h || !h->s) return IBMG_ERR_STATE;
  if (!n || level < 0 || level >= h->s->levels()) return IBMG_ERR_ARG;
  *n = h->s->level_n(level);
  return IBMG_OK;
}

ibmg_status ibmg_apply_A_IB(ibmg_handle* h, int32_t level, const double* w, double* y, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    check_level(s, level, 0);
    ibmg::require(w && y && w != y, "w and y must be distinct device pointers");
    s->apply(level, w, y, false, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_apply_A_IB_T(ibmg_handle* h, int32_t level, const double* w, double* y, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    check_level(s, level, 0);
    ibmg::require(w && y && w != y, "w and y must be distinct device pointers");
    s->apply(level, w, y, true, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_spread(ibmg_handle* h, const double* F, double* f, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(f != nullptr, "f is NULL");
    s->spread(F, f, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_interp(ibmg_handle* h, const double* u, double* U, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(u != nullptr, "u is NULL");
    s->interp(u, U, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_restrict(ibmg_handle* h, int32_t level, const double* fine, double* coarse, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    check_level(s, level, 1);
    ibmg::require(fine && coarse, "NULL vector");
    s->restrict_(level, fine, coarse, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_prolong_add(ibmg_handle* h, int32_t level, const double* coarse, double* fine, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    check_level(s, level, 1);
    ibmg::require(fine && coarse, "NULL vector");
    s->prolong_add(level, coarse, fine, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_smoother_apply(ibmg_handle* h, int32_t level, const double* r, double* z, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    check_level(s, level, 1);
    ibmg::require(r && z && r != z, "r and z must be distinct device pointers");
    s->smoother_apply(level, r, z, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_smooth(ibmg_handle* h, int32_t level, double* w, const double* b, int32_t nu, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    check_level(s, level, 1);
    ibmg::require(w && b && w != b, "w and b must be distinct device pointers");
    s->smooth(level, w, b, nu, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_coarse_solve(ibmg_handle* h, const double* r, double* x, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(r && x && r != x, "r and x must be distinct device pointers");
    s->coarse_solve(r, x, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_vcycle(ibmg_handle* h, const double* r, double* z, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(r && z && r != z, "r and z must be distinct device pointers");
    s->vcycle(r, z, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_fgmres_solve(ibmg_handle* h, const double* b, double* x, const ibmg_solve_opts* opts,
                              ibmg_solve_info* info, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(b && x && b != x, "b and x must be distinct device pointers");
    ibmg_solve_opts o{1e-8, 30, 100, 0, 0};
    if (opts) o = *opts;
    return s->fgmres(b, x, o, info, S(st));
  });
}

ibmg_status ibmg_spring_gradient(ibmg_handle* h, const double* w, const double* lambda, double* out,
                                 ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(w && lambda, "NULL vector");
    s->spring_gradient(w, lambda, out, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_spring_gradient_static(ibmg_handle* h, const double* w, const double* lambda, double* out,
                                        ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(w && lambda, "NULL vector");
    ibmg::require(s->points() <= ibmg::kStaticGradPoints,
                  "the structure has " + std::to_string(s->points()) + " points; the allocation-free gradient holds " +
                      std::to_string(ibmg::kStaticGradPoints));
    double* scratch = ibmg::static_grad_scratch();
    s->spring_gradient_in(w, lambda, out, scratch, scratch + 2 * (size_t)ibmg::kStaticGradPoints, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_set_kappa(ibmg_handle* h, const double* kappa, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    s->set_kappa(kappa, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_step_rhs(ibmg_handle* h, const double* w, double* rhs, ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(w && rhs && w != rhs, "w and rhs must be distinct device pointers");
    s->step_rhs(w, rhs, S(st));
    return IBMG_OK;
  });
}

ibmg_status ibmg_time_step(ibmg_handle* h, double* w, const ibmg_solve_opts* opts, ibmg_solve_info* info,
                           ibmg_stream st) {
  return guarded(h, [&](ibmg::SolverBase* s) {
    ibmg::require(w != nullptr, "w is NULL");
    ibmg_solve_opts o{1e-8, 30, 100, 0, 0};
    if (opts) o = *opts;
    ibmg::require(o.transpose == 0, "the time step solves with L_IB");
    return s->time_step(w, o, info, S(st));
  });
}

ibmg_status ibmg_positions(const ibmg_handle* h, double* X) {
  if (!h || !h->s) return IBMG_ERR_STATE;
  if (!X) return IBMG_ERR_ARG;
  h->s->positions(X);
  return IBMG_OK;
}

ibmg_status ibmg_stats(const ibmg_handle* h, int64_t* out, int32_t cap, int32_t* written) {
  if (!h || !h->s) return IBMG_ERR_STATE;
  if (!written || (cap > 0 && !out)) return IBMG_ERR_ARG;
  std::vector<int64_t> v = h->s->stats();
  int n = 0;
  for (; n < (int)v.size() && n < cap; ++n) out[n] = v[n];
  *written = (int32_t)v.size();
  return IBMG_OK;
}

ibmg_status ibmg_sc_info(const ibmg_handle* h, int32_t level, double* lam, int32_t* colours) {
  if (!h || !h->s) return IBMG_ERR_STATE;
  if (!lam || !colours) return IBMG_ERR_ARG;
  try {
    h->s->sc_info(level, lam, colours);
    return IBMG_OK;
  } catch (const ibmg::Error& e) {
    return (ibmg_status)e.code;
  }
}

}  // extern "C"
