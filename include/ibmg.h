/* ibmg.h -- C ABI of the MI355X multigrid solver for the Stokes-IB system
 *
 *   L_IB [u; p] = [A_IB, G; -D, 0] [u; p] = b,
 *   A_IB = rho/dt I - mu Lap_h - dt S_h K_h J_h            (Eq. matrix-impib)
 *
 * on a periodic N x N staggered grid (App. A.1), preconditioned by the
 * geometric-multigrid V-cycle of Alg. 1 with a restricted additive Schwarz
 * (Alg. 2), restricted multiplicative Schwarz (Alg. 3) or Schur-complement
 * (Eq. approx-fact-Stokes-IB) smoother wrapped in a fixed number of FGMRES
 * iterations (Sec. 3.3), inside flexible GMRES.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vector layout.  A level vector w of an n x n level has 3 n^2 entries
 *   [u (j*n+i), v (j*n+i), p (j*n+i)],
 * u[j][i] the x-velocity on the face at (i h, (j+1/2) h), v[j][i] the
 * y-velocity on the face at ((i+1/2) h, j h), p[j][i] the pressure at the cell
 * centre ((i+1/2) h, (j+1/2) h), h = 1/n, all indices periodic.
 * Lagrangian arrays are [M][2] (x, y interleaved).
 * Memory.  Pointers named in a ``desc`` (X, ends, kappa, rest) are HOST pointers,
 * copied during ibmg_create.  Every vector argument of the other calls is a
 * DEVICE pointer (FP64 unless stated) owned by the caller; the library never
 * frees caller memory.  The library allocates no device memory: every device
 * buffer of a handle (operators, box inverses, work vectors, set-up
 * temporaries) lies in the one workspace region the caller passes to
 * ibmg_create / ibmg_batch_create (256-byte aligned, at least the size
 * ibmg_workspace_bytes / ibmg_batch_workspace_bytes report), which must stay
 * allocated and untouched until ibmg_destroy.  A handle also holds 64 bytes
 * of pinned host memory for its scalar reads.
 * Streams.  Calls enqueue work on the given HIP stream and return without
 * synchronising, except ibmg_create, ibmg_set_kappa and the *_solve calls,
 * which synchronise that stream.  A handle is not thread-safe; distinct
 * handles are independent.
 * Errors.  Every call returns an ibmg_status; nothing throws across the ABI.
 * Argument errors are detected on the host before any work is enqueued.  A
 * HIP error is returned by the call that observes it; ibmg_last_error gives
 * the message of the last failure on a handle (or of a failed create when
 * passed NULL).
 */
#ifndef IBMG_H
#define IBMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibmg_handle ibmg_handle;
typedef void* ibmg_stream; /* a hipStream_t; NULL means the null stream */

typedef enum {
  IBMG_OK = 0,
  IBMG_NOT_CONVERGED = 1, /* result valid, tolerance not reached in max_it */
  IBMG_ERR_ARG = -1,      /* invalid argument; nothing was enqueued */
  IBMG_ERR_HIP = -2,      /* HIP runtime error (launch, fault) */
  IBMG_ERR_WORKSPACE = -3,/* the caller's workspace is too small (or misaligned);
                             after a rebuild (ibmg_time_step, ibmg_set_kappa)
                             the handle is then unusable (IBMG_ERR_STATE)     */
  IBMG_ERR_BREAKDOWN = -4,/* a set-up factorisation broke down: a box matrix,
                             the coarsest bordered matrix or an SC Chebyshev
                             bound came out singular or non-finite            */
  IBMG_ERR_NONFINITE = -5,/* NaN/Inf in an input vector or in the iteration */
  IBMG_ERR_STATE = -6     /* call not valid for this handle */
} ibmg_status;

/* smoother: restricted additive Schwarz (Alg. 2), Schur complement
 * (Sec. 3.3.2), restricted multiplicative Schwarz (Alg. 3).  The
 * multiplicative sweep visits the boxes colour by colour: boxes are greedily
 * coloured in index order so that no box of a colour has a row coupled (by
 * the stencil, the IB term, G or D) to an owned unknown of another box of
 * that colour; each colour takes the residual of the current iterate, so the
 * sweep equals Alg. 3 with the boxes in colour-major order. */
enum { IBMG_RAS = 0, IBMG_SC = 1, IBMG_RMS = 2 };
enum { IBMG_FP64 = 0, IBMG_FP32_SMOOTHER = 1 };  /* precision */

/* combine: how the additive Schwarz smoother joins the boxes' local solutions
 * z_k = L_k^{-1} R_k r (Alg. 2):
 *   IBMG_COMBINE_RESTRICTED  each unknown takes the value of the one box that
 *                            owns it (R~_k^T, the paper's restricted form)
 *   IBMG_COMBINE_SUM         each unknown takes the sum over every box whose
 *                            index set holds it (R_k^T: plain additive
 *                            Schwarz), added in box-index order (deterministic,
 *                            no atomics).  IBMG_RAS only.
 * sweep_kind: what one of the nu1 / nu2 smoothing steps is (Sec. 3.3, Sec. 6):
 *   IBMG_SWEEP_FGMRES        nu FGMRES iterations on L e = b - L w from e = 0,
 *                            preconditioned by the basic smoother (default)
 *   IBMG_SWEEP_RICHARDSON    nu undamped Richardson steps w <- w + B (b - L w)
 *                            with the basic smoother B (the reading of Sec. 6,
 *                            where the large-box Vanka smoother is a Richardson
 *                            iteration).  Single-system handles only. */
enum { IBMG_COMBINE_RESTRICTED = 0, IBMG_COMBINE_SUM = 1 };
enum { IBMG_SWEEP_FGMRES = 0, IBMG_SWEEP_RICHARDSON = 1 };

/* Spring model.  Spring e = (a, b) has separation d = X_b - X_a (minimum
 * image on the periodic square), length l = |d| and unit vector t = d / l.
 *   IBMG_SPRING_LINEAR   zero rest length (the linear fibre force of Sec. 5,
 *                        App. A.2): node a feels kappa_e d, node b -kappa_e d,
 *                        the same operator on each velocity component.
 *   IBMG_SPRING_TANGENT  rest length L_e: node a feels kappa_e (l - L_e) t
 *                        (the Sec. 5 fibre model with a tension vanishing at
 *                        L_e), and the operator's stiffness is this force's
 *                        Jacobian at the handle's positions (the linearised
 *                        force of a Newton-Krylov step, Sec. 6): per spring
 *                        the 2x2 block K_e = kappa_e [(1 - L_e/l) I +
 *                        (L_e/l) t t^T], which couples the u and v rows of
 *                        A_IB.  L_e = 0 gives the linear model.  A spring of
 *                        zero length with L_e > 0 is rejected (IBMG_ERR_ARG).
 *                        The batched form takes linear springs only. */
enum { IBMG_SPRING_LINEAR = 0, IBMG_SPRING_TANGENT = 1 };

typedef struct {
  int32_t N;          /* finest grid size; N = coarse_N * 2^k, k >= 1        */
  int32_t coarse_N;   /* coarsest grid (Sec. 5 uses 8); 4 <= coarse_N <= 16   */
  double rho, mu, dt; /* A = rho/dt I - mu Lap_h (Eq. system-impib); rho >= 0,
                         mu > 0, dt > 0                                      */
  int32_t M;          /* Lagrangian points, >= 0                             */
  const double* X;    /* host [M][2], positions in [0,1)^2 (lagged X^n)      */
  int32_t n_springs;  /* >= 0                                                */
  const int32_t* ends;/* host [n_springs][2] node ids, a != b, in [0, M)     */
  const double* kappa;/* host [n_springs] spring stiffness >= 0             */
  int32_t smoother;   /* IBMG_RAS | IBMG_SC | IBMG_RMS                        */
  int32_t box;        /* RAS box size b (cells); must divide every level's
                         n >= 2b, levels below use min(b, n/2)               */
  int32_t overlap;    /* RAS overlap o (cells) >= 0                          */
  int32_t nu1, nu2;   /* pre/post smoothing: FGMRES iterations, 1..8         */
  int32_t cheb_its;   /* SC: Chebyshev iterations per inner solve, 1..8      */
  int32_t precision;  /* IBMG_FP64 | IBMG_FP32_SMOOTHER                       */
  int32_t spring_model;/* IBMG_SPRING_LINEAR | IBMG_SPRING_TANGENT (above)    */
  const double* rest; /* host [n_springs] rest lengths >= 0, or NULL (all
                         zero); non-zero values need IBMG_SPRING_TANGENT      */
  int32_t combine;    /* IBMG_COMBINE_RESTRICTED | IBMG_COMBINE_SUM (above)   */
  int32_t sweep_kind; /* IBMG_SWEEP_FGMRES | IBMG_SWEEP_RICHARDSON (above)    */
  int32_t max_restart;/* longest outer FGMRES restart the workspace holds,
                         1..64; 0 means 30                                    */
} ibmg_desc;

typedef struct {
  double rtol;        /* stop at ||b - L x|| <= rtol ||b|| (Arnoldi estimate) */
  int32_t restart;    /* FGMRES restart length, 1..max_restart (30)           */
  int32_t max_it;     /* total iteration cap (100, the paper's Sec. 5 cap)    */
  int32_t use_x0;     /* 1: x holds the initial guess; 0: start from zero     */
  int32_t transpose;  /* 1: solve L_IB^T x = b (adjoint system; the Krylov
                         operator is ibmg_apply_A_IB_T's transposed path)    */
} ibmg_solve_opts;

typedef struct {
  int32_t iters, restarts;
  double rel_res_est;   /* Arnoldi residual estimate / ||b||                 */
  double rel_res_true;  /* ||P b - L x|| / ||P b|| recomputed at the end      */
  double rhs_null_norm; /* ||b - P b||, the null-space part removed from b    */
  double setup_ms;      /* wall time of the handle's latest set-up, device
                           work included: ibmg_create / ibmg_batch_create,
                           ibmg_set_kappa, or the rebuild at X^{n+1} that
                           ibmg_time_step ends with (then that step's)       */
  double solve_ms;      /* wall time of the call (for ibmg_time_step: its
                           solve, without the rebuild)                       */
  double* history;      /* optional host array of residual estimates         */
  int32_t history_cap;  /* its capacity (0 if history is NULL)               */
  int32_t vcycles;      /* V-cycles applied                                  */
} ibmg_solve_info;

/* Bytes of device workspace ibmg_create needs for ``desc``: the exact
 * high-water mark of the set-up's buffers (every level's operators, box
 * inverses and work vectors, the outer FGMRES basis for max_restart, and the
 * set-up's temporaries, among them up to 8 GiB of box matrices inverted in
 * one batch).  Runs the set-up's host planning (no device work).  A rebuild
 * at moved positions (ibmg_time_step) re-lays the position-dependent buffers
 * and needs more when the structure touches more boxes, so time-stepping
 * callers add headroom.  Errors: IBMG_ERR_ARG as ibmg_create. */
ibmg_status ibmg_workspace_bytes(const ibmg_desc* desc, size_t* bytes);

/* Create a solver for one system: copies the structure, builds every level's
 * operators (rediscretised A, G, D; Galerkin IB operator, Sec. 3.1), the
 * smoother data (RAS box inverses, Alg. 2; or SC colourings and Chebyshev
 * bounds) and the coarsest direct solve, all inside ``workspace`` (a device
 * region of ``bytes`` bytes, 256-byte aligned, owned by the caller).
 * Synchronises ``stream``.
 * Errors: IBMG_ERR_ARG for an invalid desc (non-finite values, bad sizes,
 * out-of-range ids), IBMG_ERR_WORKSPACE if the workspace is NULL, misaligned
 * or smaller than ibmg_workspace_bytes, IBMG_ERR_BREAKDOWN if a box or the
 * coarsest system cannot be inverted, IBMG_ERR_HIP on kernel failure. */
ibmg_status ibmg_create(const ibmg_desc* desc, void* workspace, size_t bytes, ibmg_stream stream,
                        ibmg_handle** out);
/* Bytes of the handle's workspace in use now and the most ever in use. */
ibmg_status ibmg_workspace_used(const ibmg_handle* h, size_t* in_use, size_t* peak);
ibmg_status ibmg_destroy(ibmg_handle* h);
const char* ibmg_last_error(const ibmg_handle* h);

/* Number of levels and the grid size of a level (0 = coarsest). */
ibmg_status ibmg_levels(const ibmg_handle* h, int32_t* n_levels);
ibmg_status ibmg_level_n(const ibmg_handle* h, int32_t level, int32_t* n);

/* y = L_IB^l w on level l (Eq. matrix-h-impib; the finest level is
 * Eq. matrix-impib), FP64, w and y of length 3 n_l^2, must not alias. */
ibmg_status ibmg_apply_A_IB(ibmg_handle* h, int32_t level, const double* w, double* y,
                            ibmg_stream stream);
/* y = L_IB^T w on level l, computed by the transposed stencils and the
 * interpolation reused as the adjoint of spreading (S = J^*, App. A.3). */
ibmg_status ibmg_apply_A_IB_T(ibmg_handle* h, int32_t level, const double* w, double* y,
                              ibmg_stream stream);

/* f = S_h F on the finest grid (App. A.3 spreading, unit nodal weights):
 * F [M][2] -> f [2][N][N] (u-faces then v-faces). */
ibmg_status ibmg_spread(ibmg_handle* h, const double* F, double* f, ibmg_stream stream);
/* U = J_h u on the finest grid (App. A.3 interpolation): u [2][N][N] -> U [M][2]. */
ibmg_status ibmg_interp(ibmg_handle* h, const double* u, double* U, ibmg_stream stream);

/* Inter-level transfers (Sec. 3.2) between level l (fine) and l-1 (coarse):
 * coarse = [R_u; R_u; R_p] fine;  fine += [P_u; P_u; P_p] coarse. */
ibmg_status ibmg_restrict(ibmg_handle* h, int32_t level, const double* fine, double* coarse,
                          ibmg_stream stream);
ibmg_status ibmg_prolong_add(ibmg_handle* h, int32_t level, const double* coarse, double* fine,
                             ibmg_stream stream);

/* One application of the basic smoother on level l >= 1 from a zero guess:
 * z = RAS(0, r) (Alg. 2), RMS(0, r) (Alg. 3) or the SC approximate inverse
 * (Eq. approx-fact-Stokes-IB). */
ibmg_status ibmg_smoother_apply(ibmg_handle* h, int32_t level, const double* r, double* z,
                                ibmg_stream stream);
/* Sec. 3.3 smoothing on level l >= 1: w <- w + e, e from nu FGMRES iterations
 * on L e = b - L w (e0 = 0) preconditioned by the basic smoother. */
ibmg_status ibmg_smooth(ibmg_handle* h, int32_t level, double* w, const double* b, int32_t nu,
                        ibmg_stream stream);
/* Coarsest-level direct solve: x = L_IB^0+ r (bordered by the null vectors). */
ibmg_status ibmg_coarse_solve(ibmg_handle* h, const double* r, double* x, ibmg_stream stream);

/* z = MG(0, r): one V-cycle (Alg. 1) on the finest level from a zero guess. */
ibmg_status ibmg_vcycle(ibmg_handle* h, const double* r, double* z, ibmg_stream stream);

/* Solve L_IB x = b with FGMRES(restart) preconditioned by one V-cycle per
 * iteration.  b is projected onto range(L_IB) (block means removed: pressure
 * always, velocity components when rho = 0); the returned x has no null-space
 * component.  FGMRES orthogonalisation, the outer residual and the coarsest
 * solve are FP64 in both precisions.  Synchronises ``stream``.
 * Returns IBMG_NOT_CONVERGED if max_it is reached, IBMG_ERR_NONFINITE if b
 * holds NaN/Inf or the iteration produces it. */
ibmg_status ibmg_fgmres_solve(ibmg_handle* h, const double* b, double* x,
                              const ibmg_solve_opts* opts, ibmg_solve_info* info,
                              ibmg_stream stream);

/* dL/dkappa_e = -lambda^T (dL_IB/dkappa_e) w
 *             = -(dt/h^2) sum_c (B_e J lambda_c)(B_e J w_c),
 * B_e J x = (J x)_{b_e} - (J x)_{a_e}: the derivative of a loss through the
 * adjoint solution lambda of L_IB^T lambda = dL/dw (finest level, FP64).
 * With IBMG_SPRING_TANGENT the sum over c becomes
 * (B_e J lambda)^T (K_e / kappa_e) (B_e J w) with the spring's 2x2 block
 * (the operator is linear in kappa_e at fixed positions).
 * w, lambda: 3 N^2; out: [n_springs]. */
ibmg_status ibmg_spring_gradient(ibmg_handle* h, const double* w, const double* lambda,
                                 double* out, ibmg_stream stream);

/* ibmg_spring_gradient without the handle's workspace, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Its scratch (J w and J lambda per
 * point) is a fixed device array inside the library, 8 MiB per GPU, held
 * from the first call on a GPU until the process ends; it allocates nothing
 * and calls no allocating routine.  Structures of more than 2^18 points are
 * rejected (IBMG_ERR_ARG).  Every call on one GPU shares that array: calls
 * that overlap on one GPU (other streams, other threads, other handles)
 * race and must be ordered by the caller.  Same arguments and results as
 * ibmg_spring_gradient. */
ibmg_status ibmg_spring_gradient_static(ibmg_handle* h, const double* w, const double* lambda,
                                        double* out, ibmg_stream stream);

/* Replace the spring stiffnesses (host array [n_springs]) and rebuild every
 * level's IB operator and smoother data (tangent blocks at the current
 * positions).  Synchronises ``stream``. */
ibmg_status ibmg_set_kappa(ibmg_handle* h, const double* kappa, ibmg_stream stream);

/* The right-hand side of one semi-implicit time step (Sec. 2.2, Eq.
 * matrix-impib, without convection): rhs = [(rho/dt) u + S_h K_h X; 0] on the
 * finest grid, X the handle's current positions, K_h X the nodal spring
 * forces of the handle's spring model with minimum-image separations on the
 * periodic square (with IBMG_SPRING_TANGENT the nonlinear force F(X^n), so the
 * step is linearly implicit: F(X^{n+1}) ~ F(X^n) + dt K_tan J u^{n+1}).
 * w: [u | v | p] (the p part is not read); rhs: 3 N^2, distinct from w. */
ibmg_status ibmg_step_rhs(ibmg_handle* h, const double* w, double* rhs, ibmg_stream stream);

/* One semi-implicit time step (Sec. 2.2, Eqs. imp-momentum to imp-F without
 * convection): forms the right-hand side above from w = (u^n, .), solves
 * L_IB(X^n) w^{n+1} = rhs as ibmg_fgmres_solve does (opts, info; transpose
 * must be 0), moves the structure to X^{n+1} = X^n + dt J_h u^{n+1} (wrapped
 * into [0, 1)) and rebuilds every level at X^{n+1}, so the handle is ready
 * for the next step (tangent blocks re-evaluated there).  w is overwritten
 * with (u, p)^{n+1}.  Synchronises ``stream``.  IBMG_ERR_NONFINITE if the
 * positions become invalid; IBMG_ERR_ARG if a spring with a rest length
 * collapses to zero length. */
ibmg_status ibmg_time_step(ibmg_handle* h, double* w, const ibmg_solve_opts* opts, ibmg_solve_info* info,
                           ibmg_stream stream);

/* The handle's current structure positions, copied to the host array X [M][2]. */
ibmg_status ibmg_positions(const ibmg_handle* h, double* X);

/* Setup statistics.  Writes up to cap int64 values: [levels, then per
 * level: n, boxes, boxes with their own inverse (+1 for the shared interior
 * one), IB-touched boxes, entries of the explicit IB rows, box colours of the
 * multiplicative sweep (0 for the other smoothers)] and returns the full
 * count in *written. */
ibmg_status ibmg_stats(const ibmg_handle* h, int64_t* out, int32_t cap, int32_t* written);

/* Schur-complement smoother data of level l >= 1 (Sec. 3.3.2): lam[0], lam[1]
 * = the Chebyshev bounds' Ritz values for SGS(A_IB)^{-1} A_IB and for
 * SGS(-M^)^{-1}(-D A~^{-1} G); colours[0], colours[1] = Gauss-Seidel colours
 * of the velocity rows and of the cells.  IBMG_ERR_ARG if the handle uses the
 * Schwarz smoother. */
ibmg_status ibmg_sc_info(const ibmg_handle* h, int32_t level, double* lam, int32_t* colours);

/* Single-kernel timing, for benchmarks and profilers that price a kernel
 * against the hardware's roofline.  Launches one kernel of `level` alone,
 * once untimed and then `reps` times between two HIP events recorded on
 * ``stream`` (the stream the kernel runs on), on the handle's own work
 * vectors filled with ones, and returns the average duration of one launch in
 * *avg_ms with the kernel's algorithmic bytes and flops per launch (nullable
 * outputs).  Kernels:
 *   IBMG_KERNEL_RAS_IB        Schwarz boxes with their own inverse (k_ras_ib):
 *                             n_ib (nown nloc + nloc + nown) values, 2 n_ib nown
 *                             nloc flops
 *   IBMG_KERNEL_RAS_INTERIOR  interior boxes on the matrix cores
 *                             (k_ras_interior, one launch): the shared inverse
 *                             once plus n_int (nloc + nown) values, 2 n_int nown
 *                             nloc flops
 *   IBMG_KERNEL_STENCIL       the Stokes stencil k_apply (no IB term): 6 N^2
 *                             values
 *   IBMG_KERNEL_RAS_BATCH     (batch handles) the persistent batched Schwarz
 *                             launch of a level with its tuned plan
 *   IBMG_KERNEL_RESTRICT      restriction from `level` (>= 1) to the next
 *                             coarser level: 3 n_f^2 + 3 n_c^2 values
 *   IBMG_KERNEL_PROLONG       prolongation from the next coarser level added
 *                             into `level` (>= 1): 3 n_c^2 + 2 (3 n_f^2) values
 *   IBMG_KERNEL_SPREAD        spreading on the finest level (FP64): every
 *                             (point, slot) entry's weight and index, the face
 *                             list offsets, 2 M forces, 2 N^2 faces written
 *   IBMG_KERNEL_INTERP        interpolation on the finest level (FP64): 2 M x 16
 *                             weights, the window bases, every face some
 *                             window touches, 2 M values written
 * and the Krylov kernels of one smoothing step on `level` (>= 1), the basis
 * at its largest, k = max(nu1, nu2) vectors of n = 3 n_l^2 values (Sec. 3.3):
 *   IBMG_KERNEL_APPLY_DOTS    L_IB^l z with the first Gram-Schmidt pass fused:
 *                             z read, the product written, k vectors read
 *                             ((k + 2) n values)
 *   IBMG_KERNEL_UPD_DOTS      t -= V h, then the second pass's dots and |t|^2:
 *                             t read and written, k vectors read ((k + 2) n)
 *   IBMG_KERNEL_SCALE_UPD     t = (t - V h2) / |t - V h2|, the norm taken as
 *                             sqrt(|t|^2 - |h2|^2) from those sums: t read and
 *                             written, k vectors read ((k + 2) n)
 *   IBMG_KERNEL_COMBINE_LS    w += sum_q y_q Z_q after the small least squares:
 *                             k vectors and w read, w written ((k + 2) n)
 * and two kernels of the outer solve's (and the batched smoothing's) second
 * pass, timed on the same vectors:
 *   IBMG_KERNEL_UPD_NORM      t -= V h2, then |t|^2: (k + 2) n
 *   IBMG_KERNEL_SCALE_RED     v = t / |t|: 2 n
 * Synchronises ``stream``; IBMG_ERR_ARG if the level has no such work. */
typedef enum {
  IBMG_KERNEL_RAS_IB = 0,
  IBMG_KERNEL_RAS_INTERIOR = 1,
  IBMG_KERNEL_STENCIL = 2,
  IBMG_KERNEL_RAS_BATCH = 3,
  IBMG_KERNEL_RESTRICT = 4,
  IBMG_KERNEL_PROLONG = 5,
  IBMG_KERNEL_SPREAD = 6,
  IBMG_KERNEL_INTERP = 7,
  IBMG_KERNEL_APPLY_DOTS = 8,
  IBMG_KERNEL_UPD_DOTS = 9,
  IBMG_KERNEL_UPD_NORM = 10,
  IBMG_KERNEL_SCALE_RED = 11,
  IBMG_KERNEL_COMBINE_LS = 12,
  IBMG_KERNEL_SCALE_UPD = 13
} ibmg_kernel;
ibmg_status ibmg_kernel_time(ibmg_handle* h, int32_t kernel, int32_t level, int32_t reps,
                             ibmg_stream stream, double* avg_ms, double* alg_bytes,
                             double* alg_flops);

/* ------------------------------------------------------------------------
 * Batched form: nsys independent systems, each described by its own
 * ibmg_desc (grid size N, structure, stiffness), solved together.  All
 * systems must share coarse_N, rho, mu, dt, box, overlap, nu1, nu2 and
 * precision, and use the Schwarz smoother (IBMG_ERR_ARG otherwise).  The
 * V-cycle (Alg. 1) runs on every system in lockstep by level: each smoother
 * sweep is one persistent launch over all (system, box) items, tuned at
 * creation by timing the candidate tile widths and grid sizes; the V-cycle
 * is replayed from a HIP graph.  Vectors are passed as host arrays of nsys
 * device pointers in the order of descs, system i's vector holding 3 N_i^2
 * doubles in the single-system layout.  Single-system calls on a batch
 * handle (and batch calls on a single handle) return IBMG_ERR_STATE.
 * ---------------------------------------------------------------------- */
ibmg_status ibmg_batch_workspace_bytes(int32_t nsys, const ibmg_desc* descs, size_t* bytes);
ibmg_status ibmg_batch_create(int32_t nsys, const ibmg_desc* descs, void* workspace, size_t bytes,
                              ibmg_stream stream, ibmg_handle** out);

/* Number of systems of a batch handle. */
ibmg_status ibmg_batch_size(const ibmg_handle* h, int32_t* nsys);

/* z_i = MG(0, r_i) for every system (Alg. 1, zero initial guess). */
ibmg_status ibmg_batch_vcycle(ibmg_handle* h, const double* const* r, double* const* z,
                              ibmg_stream stream);

/* FGMRES(restart) on every system, right-preconditioned by the batched
 * V-cycle, each system stopping at its own tolerance (as ibmg_fgmres_solve;
 * opts->transpose must be 0).  The Krylov iterations run in lockstep with
 * one host read of all residual estimates per iteration; converged systems
 * stop doing work.  infos (nullable) receives one record per system, in the
 * order of descs.  Synchronises ``stream``.  Returns IBMG_NOT_CONVERGED if
 * any system reaches max_it. */
ibmg_status ibmg_batch_fgmres_solve(ibmg_handle* h, const double* const* b, double* const* x,
                                    const ibmg_solve_opts* opts, ibmg_solve_info* infos,
                                    ibmg_stream stream);

/* Batch statistics: [nsys, levels, then per level: n, systems on the level,
 * interior boxes, IB boxes, explicit IB rows, chosen tile width, chosen
 * persistent grid, tuned sweep time in ns]; count in *written. */
ibmg_status ibmg_batch_stats(const ibmg_handle* h, int64_t* out, int32_t cap, int32_t* written);

#ifdef __cplusplus
}
#endif
#endif
