// Host orchestration of the Stokes-IB multigrid solver.
#pragma once

#include "internal.hpp"

namespace ibmg {

struct CompFoot {             // one velocity component on one level
  std::vector<int> base;      // [M][2] wrapped window base (i0, j0)
  std::vector<int> mask;      // [M] structural slots
  std::vector<int> sp_ptr, sp_ent;   // faces -> (point, slot) entries
  std::vector<int> tptr, tcol;       // Galerkin IB rows (pattern; columns index [u | v])
  DBuf<int> d_base, d_mask, d_sp_ptr, d_sp_ent, d_tptr, d_tcol;
  DBuf<double> w;             // [M][16]
  DBuf<float> wf;             // FP32 copy for the FP32 smoother
  DBuf<double> sw;            // weights in face-list order
  DBuf<float> swf;            // FP32 copy
  DBuf<int> d_obase;          // [M][2] window bases in walk (cell) order
  DBuf<double> ow;            // [M][16] weights in walk order
  DBuf<float> owf;            // FP32 copy
  DBuf<double> tval;
  DBuf<float> tvalf;          // FP32 copy for the FP32 smoother
  int max_list = 0;           // longest face -> point list
};

struct SolverBase {
  virtual ~SolverBase() = default;
  std::string last_error;
  virtual int levels() const = 0;
  virtual int level_n(int l) const = 0;
  virtual void apply(int level, const double* w, double* y, bool trans, hipStream_t s) = 0;
  virtual void spread(const double* F, double* f, hipStream_t s) = 0;
  virtual void interp(const double* u, double* U, hipStream_t s) = 0;
  virtual void restrict_(int level, const double* fine, double* coarse, hipStream_t s) = 0;
  virtual void prolong_add(int level, const double* coarse, double* fine, hipStream_t s) = 0;
  virtual void smoother_apply(int level, const double* r, double* z, hipStream_t s) = 0;
  virtual void smooth(int level, double* w, const double* b, int nu, hipStream_t s) = 0;
  virtual void coarse_solve(const double* r, double* x, hipStream_t s) = 0;
  virtual void vcycle(const double* r, double* z, hipStream_t s) = 0;
  virtual int fgmres(const double* b, double* x, const ibmg_solve_opts& o, ibmg_solve_info* info,
                     hipStream_t s) = 0;
  virtual void spring_gradient(const double* w, const double* lam, double* out, hipStream_t s) = 0;
  // the same with J w and J lambda in caller-given device scratch (2 M each)
  virtual void spring_gradient_in(const double* w, const double* lam, double* out, double* Uw, double* Ul,
                                  hipStream_t s) = 0;
  virtual int points() const = 0;
  virtual void set_kappa(const double* kappa, hipStream_t s) = 0;
  virtual std::vector<int64_t> stats() const = 0;
  virtual void sc_info(int level, double* lam, int32_t* colours) const = 0;
  // average duration (ms) of one launch of a single kernel, with its
  // algorithmic bytes and flops per launch
  virtual double kernel_time(int kernel, int level, int reps, hipStream_t s, double* bytes,
                             double* flops) = 0;
  // semi-implicit time step (Sec. 2.2)
  virtual void step_rhs(const double* w, double* rhs, hipStream_t s) = 0;
  virtual int time_step(double* w, const ibmg_solve_opts& o, ibmg_solve_info* info, hipStream_t s) = 0;
  virtual void positions(double* X) const = 0;
  // false after a rebuild failed part-way (the handle is then unusable)
  virtual bool valid() const { return true; }
};

// Many independent systems solved together (batched form): one launch per
// smoother sweep covers every system.
struct BatchBase {
  virtual ~BatchBase() = default;
  virtual int nsys() const = 0;
  virtual void vcycle(const double* const* r, double* const* z, hipStream_t s) = 0;
  virtual int fgmres(const double* const* b, double* const* x, const ibmg_solve_opts& o,
                     ibmg_solve_info* infos, hipStream_t s) = 0;
  virtual std::vector<int64_t> stats() const = 0;
  virtual double kernel_time(int kernel, int level, int reps, hipStream_t s, double* bytes,
                             double* flops) = 0;
};

// Time reps launches of fn on s with HIP events (after one untimed launch);
// returns the average in ms.
template <typename F>
double time_launches(F&& fn, int reps, hipStream_t s) {
  hipEvent_t e0, e1;
  IBMG_HIP(hipEventCreate(&e0));
  IBMG_HIP(hipEventCreate(&e1));
  float ms = 0;
  try {
    fn();
    IBMG_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) fn();
    IBMG_HIP(hipEventRecord(e1, s));
    IBMG_HIP(hipEventSynchronize(e1));
    IBMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  IBMG_HIP(hipEventDestroy(e0));
  IBMG_HIP(hipEventDestroy(e1));
  return (double)ms / reps;
}

SolverBase* make_solver(const ibmg_desc& d, hipStream_t s);
BatchBase* make_batch(int nsys, const ibmg_desc* d, hipStream_t s);
void validate_desc(const ibmg_desc& d);
void validate_batch(int nsys, const ibmg_desc* d);

}  // namespace ibmg
