// Descriptor validation and construction of the single-system solver.
#include "solver_impl.hpp"

namespace ibmg {

void validate_desc(const ibmg_desc& d) {
  require(d.coarse_N >= 4 && d.coarse_N <= 16, "coarse_N must lie in [4, 16]");
  require(d.N > d.coarse_N && d.N <= 8192, "N must exceed coarse_N and be at most 8192");
  {
    int n = d.N;
    while (n > d.coarse_N && n % 2 == 0) n /= 2;
    require(n == d.coarse_N, "N must be coarse_N * 2^k");
  }
  require(std::isfinite(d.rho) && d.rho >= 0.0, "rho must be finite and >= 0");
  require(std::isfinite(d.mu) && d.mu > 0.0, "mu must be finite and > 0");
  require(std::isfinite(d.dt) && d.dt > 0.0, "dt must be finite and > 0");
  require(d.M >= 0 && d.M <= (1 << 26), "M out of range");
  require(d.M == 0 || d.X != nullptr, "X is NULL");
  for (int l = 0; l < d.M; ++l)
    for (int c = 0; c < 2; ++c) {
      const double x = d.X[2 * l + c];
      require(std::isfinite(x) && x >= 0.0 && x < 1.0, "X must be finite and lie in [0, 1)");
    }
  require(d.n_springs >= 0, "n_springs < 0");
  require(d.n_springs == 0 || (d.ends != nullptr && d.kappa != nullptr), "ends/kappa is NULL");
  for (int e = 0; e < d.n_springs; ++e) {
    const int a = d.ends[2 * e], b = d.ends[2 * e + 1];
    require(a >= 0 && a < d.M && b >= 0 && b < d.M && a != b, "spring end out of range");
    require(std::isfinite(d.kappa[e]) && d.kappa[e] >= 0.0, "kappa must be finite and >= 0");
  }
  require(d.spring_model == IBMG_SPRING_LINEAR || d.spring_model == IBMG_SPRING_TANGENT, "unknown spring model");
  if (d.rest != nullptr)
    for (int e = 0; e < d.n_springs; ++e) {
      require(std::isfinite(d.rest[e]) && d.rest[e] >= 0.0, "rest lengths must be finite and >= 0");
      require(d.rest[e] == 0.0 || d.spring_model == IBMG_SPRING_TANGENT,
              "non-zero rest lengths need the tangent spring model");
      if (d.rest[e] == 0.0) continue;
      // the tangent block needs the spring's direction
      const int a = d.ends[2 * e], b = d.ends[2 * e + 1];
      double dx = d.X[2 * b] - d.X[2 * a], dy = d.X[2 * b + 1] - d.X[2 * a + 1];
      dx -= std::nearbyint(dx);
      dy -= std::nearbyint(dy);
      require(std::hypot(dx, dy) > 0.0, "a spring with a rest length has zero length");
    }
  require(d.smoother == IBMG_RAS || d.smoother == IBMG_SC || d.smoother == IBMG_RMS, "unknown smoother");
  require(d.nu1 >= 1 && d.nu1 <= kMaxNu && d.nu2 >= 1 && d.nu2 <= kMaxNu, "nu1/nu2 must lie in [1, 8]");
  require(d.precision == IBMG_FP64 || d.precision == IBMG_FP32_SMOOTHER, "unknown precision");
  require(d.combine == IBMG_COMBINE_RESTRICTED || d.combine == IBMG_COMBINE_SUM, "unknown combine");
  require(d.combine == IBMG_COMBINE_RESTRICTED || d.smoother == IBMG_RAS,
          "the summed combination applies to the additive Schwarz smoother only");
  require(d.sweep_kind == IBMG_SWEEP_FGMRES || d.sweep_kind == IBMG_SWEEP_RICHARDSON, "unknown sweep_kind");
  require(d.max_restart >= 0 && d.max_restart <= kMaxRestart, "max_restart must lie in [0, 64]");
  if (d.smoother == IBMG_SC) require(d.cheb_its >= 1 && d.cheb_its <= 8, "cheb_its must lie in [1, 8]");
  if (d.smoother == IBMG_RAS || d.smoother == IBMG_RMS) {
    require(d.box >= 1 && d.overlap >= 0, "box must be >= 1 and overlap >= 0");
    require(d.box + 2 * d.overlap <= 32, "box + 2 overlap must be <= 32");
    for (int n : level_sizes(d.N, d.coarse_N)) {
      if (n == d.coarse_N) continue;
      int b, o;
      box_params(n, d.box, d.overlap, &b, &o);
      require(b >= 1 && n % b == 0, "box size does not tile level " + std::to_string(n));
    }
  }
}

SolverBase* make_solver(const ibmg_desc& d, hipStream_t s) {
  validate_desc(d);
  if (d.precision == IBMG_FP32_SMOOTHER) return new Solver<float>(d, s);
  return new Solver<double>(d, s);
}

}  // namespace ibmg
