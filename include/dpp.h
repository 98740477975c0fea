/*
 * dpp.h -- C ABI of the MI355X (gfx950) solver library for the four-field
 * double porosity/permeability (DPP) model discretised by the stabilised
 * continuous-Galerkin CG-VMS formulation with equal-order P1 elements.
 *
 * Problem (paper, governing equations eq. DG_GE_Darcy_BLM):
 *     mu k_i^-1 u_i + grad p_i = gamma b,   i = 1, 2
 *     div u_1 = -(beta/mu)(p_1 - p_2),  div u_2 = +(beta/mu)(p_1 - p_2)
 * with pressures p_i = p0_i imposed weakly on the whole boundary
 * (eq. DG_GE_Darcy_pBC, linear functional L_Gal).  The discrete system
 * K x = f (eq. S4_linear_problem) has the block entries of
 * eq. S4_cg_stiffness_matrix and eq. S4_cg_rhs.
 *
 * Conventions shared by every entry point:
 *   - All array arguments are DEVICE pointers on the current HIP device unless
 *     stated otherwise; the caller owns them.  The library owns the opaque
 *     handles (dpp_problem, dpp_precond) and their internal device memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Work
 *     is enqueued on it; calls that must return a scalar (solve statistics)
 *     synchronise that stream before returning.
 *   - Every function returns a dpp_status; nothing throws across the ABI.  On
 *     failure dpp_last_error() returns a thread-local message.
 *   - Mesh: box [0,L_x]x[0,L_y](x[0,L_z]) with n_x, n_y (, n_z) cells per side;
 *     node id = i + (n_x+1)(j + (n_y+1)k); hexahedron h = i + n_x(j + n_y k) is
 *     split into tetrahedra 6h+s (s = axis permutation, lexicographic; vertices
 *     = corner then unit steps along the permuted axes); square h into
 *     triangles 2h, 2h+1 (same rule).
 *   - Unknown vector layout (length n_dof = (2d+2) n_nodes):
 *       [u1 | p1 | u2 | p2], velocities node-major with the d components
 *       interleaved (u_i at node a, component c sits at d*a + c of its block).
 *     This is the field order 0..3 of the paper's solver listings.
 */
#ifndef DPP_H
#define DPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DPP_OK = 0,
  DPP_ERR_ARG = 1,           /* invalid argument (null pointer, bad size, bad option) */
  DPP_ERR_ALLOC = 2,         /* device allocation failed */
  DPP_ERR_HIP = 3,           /* a HIP runtime call failed */
  DPP_ERR_NOT_CONVERGED = 4, /* iteration limit reached; x holds the last iterate */
  DPP_ERR_NUMERIC = 5,       /* NaN/Inf met in the input or the iteration */
  DPP_ERR_BREAKDOWN = 6,     /* Krylov breakdown without convergence */
  DPP_ERR_UNSUPPORTED = 7,   /* valid request this version does not implement */
  DPP_ERR_STAGNATED = 8      /* restart cycles stopped reducing the residual (stag_cycles);
                                x holds the last iterate */
} dpp_status;

typedef struct dpp_problem_s *dpp_problem;
typedef struct dpp_precond_s *dpp_precond;
typedef struct dpp_batch_s *dpp_batch;

/* Structured box: dim 2 or 3, 1 <= n[a] <= 4096 cells per axis, L[a] > 0
 * extent; (2 dim + 2) x nodes must stay below 2^31 (DPP_ERR_ARG otherwise).
 * elem selects the element family of the element table (section "Finite
 * element discretizations", CG-VMS rows): 0 = P1 on the Kuhn simplices (the
 * numbering above), 1 = Q1 on the box cells themselves (quadrilaterals /
 * hexahedra; cell h = i + n_x(j + n_y k) is box h, and per-cell arrays have
 * one entry per box).  With Q1 the solver, mixed precision, velocity faces,
 * the adjoint solve with the parameter gradient (per box) and the L2-error
 * integrals are available; batched solves are P1 only (DPP_ERR_UNSUPPORTED).  2 = DG-VMS, discontinuous
 * P1 on the Kuhn simplices (section "Stabilized mixed discontinuous Galerkin
 * formulation (DG-VMS)", eq. VMS_DG_Weak_Form, eqs. S4_dg_stiffness_matrix and
 * S4_dg_rhs): every simplex e owns d + 1 vertex slots e (d+1) + v, the vector
 * is [u1 | p1 | u2 | p2] over slots and n_dof = (2d+2)(d+1) x simplices
 * (dpp_problem_sizes reports the slots as n_nodes).  DG-VMS problems take
 * pressure faces only (face_bc NULL or zero) and are solved with precision 0
 * or 2; the adjoint solve, the CSR export, the full product K x and the
 * L2-error integrals are available, while precision 1, the block products,
 * dpp_vcycle, the parameter gradient and batched solves return
 * DPP_ERR_UNSUPPORTED. */
typedef struct {
  int dim;
  int n[3];
  double L[3];
  int elem;
} dpp_box;

/* Coefficients and boundary data (section "Boundary conditions"; parameters of
 * the paper's data tables).  k1, k2: per-cell permeabilities [n_cells] (> 0).
 * beta: scalar mass-transfer coefficient (>= 0), used when beta_cells == NULL,
 * else beta_cells [n_cells] (>= 0; DPP_ERR_NUMERIC for a negative or
 * non-finite entry, as for k1, k2 <= 0).  body: gamma*b per cell [n_cells*dim] or NULL (b = 0).
 * p0_1, p0_2: nodal pressures on the box's grid nodes ((n_x+1)(n_y+1)(n_z+1),
 * also for DG-VMS); only boundary nodes are read, and the boundary integral
 * -(w.n; p0) uses their P1 interpolant exactly (on the pressure faces).
 * Velocity (flux) boundaries (eq. DG_GE_vBC): face_bc (host, int8 [2][2*dim])
 * or NULL (every box face a pressure boundary); face_bc[i][2a + s] = 1 makes
 * face s (0: x_a = 0, 1: x_a = L_a) a velocity boundary of network i, 0 a
 * pressure boundary.  On a velocity face the normal velocity component of
 * each node is prescribed (essential: identity row holding the value, the
 * value moved out of the other rows) from u_bc_i (device, [n_nodes*dim]
 * nodal velocities, node-major; required when network i has a velocity face,
 * else unread).  Batched instances take velocity faces too.  With velocity
 * faces on every face of both networks K is singular (kernel u = 0, p1 = p2 =
 * const, also its left kernel): the solves (single and batched) take the part
 * of the right-hand side in the range of K (its component along the kernel
 * removed) and return pressures normalised to int p1 = 0, the branch of the
 * constraint of the pressure space Q (int p1)(int p2) = 0 that this library
 * takes.  Such a box needs beta > 0 in some cell (without mass transfer each
 * network has its own constant-pressure kernel): DPP_ERR_UNSUPPORTED
 * otherwise. */
typedef struct {
  double mu;
  const double *k1;
  const double *k2;
  double beta;
  const double *beta_cells;
  const double *body;
  const double *p0_1;
  const double *p0_2;
  const int8_t *face_bc;
  const double *u_bc_1;
  const double *u_bc_2;
} dpp_params;

/* Solver options; dpp_default_opts() fills the defaults in brackets.
 *   restart [30]: flexible-GMRES restart length m (1..31).
 *   maxiter [500]: total Krylov iterations (inner iterations in mixed mode).
 *   rtol [1e-8]: stop when ||f - K x||_2 <= rtol ||f||_2 (true residual, FP64).
 *   precision [0]: 0 = FP64 throughout; 1 = mixed: an inner flexible GMRES
 *     with FP32 K and FP32 preconditioner (FP64 Arnoldi and coarse solve)
 *     inside FP64 iterative refinement on the true residual; 2 = FP64 K and
 *     Arnoldi with the FP32 preconditioner (FP64 coarse solve).
 *   inner_rtol [1e-4], max_refine [20]: mixed mode only.
 *   coarse_max [0]: coarsest multigrid level has at most this many nodes
 *     (1..4000); 0 = by dimension (2200 in 3D, 400 in 2D).
 *   cheb_degree [2], cheb_lo_frac [0], cheb_hi_factor [1.1], power_iters [15]:
 *     Chebyshev smoother (degree used where a level's degree below is -1) and
 *     its interval [cheb_lo_frac hi, hi], hi = cheb_hi_factor x the estimate
 *     from power_iters power steps; cheb_lo_frac 0 = by dimension (0.1 in 3D,
 *     0.3 in 2D).
 *   use_graph [0]: capture one Arnoldi step in a hipGraph and replay it.
 *   cheb_pre_fine [0], cheb_post_fine [2], cheb_pre_coarse [0],
 *   cheb_post_coarse [3]: Chebyshev degrees of the V-cycle's pre- and
 *     post-smoothing on the finest level and on the coarser smoothing levels;
 *     -1 = cheb_degree.  A pre degree of 0 skips pre-smoothing (the level
 *     restricts its right-hand side directly); post degrees are >= 1.  On
 *     DG-VMS problems they set the nodal cycle of the pressure solve; the
 *     smoothing on the slots after it takes 3 steps.
 *   inner_maxiter [0]: mixed mode: iteration limit of one inner solve
 *     (0 = what is left of maxiter).
 *   schedule [-1]: kernel schedule of the multigrid levels, fixed at setup:
 *     -1 = autotuned per level (timed candidates); s in 0..9 = one shape on
 *     every level: lanes per stencil row {two rows per lane, 1, 2, 4, 8}[s % 5],
 *     symmetric half storage when s >= 5.
 *   stag_cycles [3], stag_ratio [0.999]: the solve stops with
 *     DPP_ERR_STAGNATED once stag_cycles restart cycles in a row have each
 *     ended with the true residual above stag_ratio times its value at the
 *     start of the cycle (0 = no stagnation test; stag_ratio in (0, 1]).  In
 *     mixed mode the test applies to the refinement sweeps. */
typedef struct {
  int restart;
  int maxiter;
  double rtol;
  int precision;
  double inner_rtol;
  int max_refine;
  int coarse_max;
  int cheb_degree;
  double cheb_lo_frac;
  double cheb_hi_factor;
  int power_iters;
  int use_graph;
  int cheb_pre_fine, cheb_post_fine, cheb_pre_coarse, cheb_post_coarse;
  int inner_maxiter;
  int schedule;
  int stag_cycles;
  double stag_ratio;
} dpp_solve_opts;

typedef struct {
  int iters;        /* Krylov iterations (all refinement sweeps together) */
  int restarts;     /* GMRES restarts */
  int refinements;  /* outer refinement sweeps (mixed mode), else 0 */
  int converged;    /* 1 when the rtol test on the true residual passed */
  double rel_residual; /* ||f - K x|| / ||f|| in FP64 at exit */
  double ms_solve;  /* wall time of the call, milliseconds */
  double ms_setup;  /* wall time of the preconditioner's setup (dpp_setup_precond) */
} dpp_solve_stats;

void dpp_default_opts(dpp_solve_opts *opts);
const char *dpp_last_error(void);

/* Assemble K and f (eq. S4_cg_stiffness_matrix, eq. S4_cg_rhs) on the device.
 * Input arrays are read during the call only (copies are kept for the
 * parameter gradient).  *out receives a new handle. */
dpp_status dpp_assemble(const dpp_box *box, const dpp_params *params, void *stream,
                        dpp_problem *out);

/* Sizes of an assembled problem (host outputs; any may be NULL).  nnz is the
 * number of structurally nonzero entries of K (22 per node pair in 3D, 16 in 2D). */
dpp_status dpp_problem_sizes(dpp_problem prob, int64_t *n_dof, int64_t *n_nodes,
                             int64_t *n_cells, int64_t *nnz);

/* Copy the assembled right-hand side f into f_out [n_dof]. */
dpp_status dpp_rhs(dpp_problem prob, double *f_out, void *stream);

/* Test/inspection hook: write K in CSR form (columns ascending in each row)
 * into rowptr [n_dof+1] (int64), cols [nnz] (int32), vals [nnz]. */
dpp_status dpp_export_csr(dpp_problem prob, int64_t *rowptr, int32_t *cols, double *vals,
                          void *stream);

/* y = A x for a block of K (section "Proposed four-field solvers", the 2x2
 * block views of Method 1 / Method 2):
 *   which 0: A = K              x, y: [n_dof]
 *   which 1/2: A = K_up^1 / K_up^2   x: [n_nodes], y: [dim*n_nodes]
 *   which 3/4: A = K_pu^1 / K_pu^2   x: [dim*n_nodes], y: [n_nodes]
 * FP64. */
dpp_status dpp_spmv(dpp_problem prob, int which, const double *x, double *y, void *stream);

/* Build the Schur fieldsplit preconditioner (Method 2 of the solver section):
 * diag(K_uu^i)^-1, the selfp Schur blocks S_p^i = K_pp^i - K_pu^i
 * diag(K_uu^i)^-1 K_up^i (eqs. S4_sp1, S4_sp2) and one geometric multigrid
 * hierarchy per S_p^i.  opts may be NULL (defaults). */
dpp_status dpp_setup_precond(dpp_problem prob, const dpp_solve_opts *opts, void *stream,
                             dpp_precond *out);

/* Number of multigrid levels, cells per axis of each level (level_n[3*l+a]),
 * and the Chebyshev upper bound per level and network (hi[2*l+i]); host
 * outputs, arrays sized for 16 levels; any may be NULL. */
dpp_status dpp_precond_info(dpp_precond pc, int *n_levels, int *level_n, double *hi);

/* Kernel shape of multigrid level `level` (the autotuner's choice): lanes per
 * stencil row (1, 2, 4, 8, or 0 for two rows per lane with paired 16-byte
 * loads) and whether the symmetric half of the stencil is stored (1) or the
 * full stencil (0).  dpp_precond_set_shape overrides it (for tests and tuning
 * studies; the values must be one of those listed). */
dpp_status dpp_precond_shape(dpp_precond pc, int level, int *lanes, int *sym);
dpp_status dpp_precond_set_shape(dpp_precond pc, int level, int lanes, int sym);

/* z = P^-1 r: one application of the fieldsplit preconditioner
 * (Jacobi on the velocities, one V-cycle per S_p^i), FP64, x/z: [n_dof]. */
dpp_status dpp_precond_apply(dpp_precond pc, const double *r, double *z, void *stream);

/* One V-cycle on both pressure Schur blocks: b, x: [2*n_nodes], network 1
 * first.  Test hook. */
dpp_status dpp_vcycle(dpp_precond pc, const double *b, double *x, void *stream);

/* y = A_l x with the level-l operator of network net (level 0 = S_p^net);
 * x, y: [nodes of level l].  Test hook. */
dpp_status dpp_level_spmv(dpp_precond pc, int level, int net, const double *x, double *y,
                          void *stream);

/* Solve K x = rhs (rhs NULL = the assembled f) by flexible GMRES(m)
 * preconditioned with pc (the outer GMRES picks up the inter-network coupling
 * the preconditioner drops).  x: in = initial guess, out = solution.  stats may
 * be NULL.  Returns DPP_ERR_NOT_CONVERGED (x = last iterate, stats filled)
 * when maxiter is reached, DPP_ERR_STAGNATED (likewise) when the restart
 * cycles stop reducing the residual (stag_cycles, stag_ratio). */
dpp_status dpp_solve(dpp_problem prob, dpp_precond pc, const dpp_solve_opts *opts,
                     const double *rhs, double *x, dpp_solve_stats *stats, void *stream);

/* Adjoint solve K^T lambda = g.  Uses K^T = D K D with D = diag(I_u, -I_p)
 * (D K is symmetric because K_pu = -K_up^T and K_pp, K_uu are symmetric), so
 * lambda = D * solve(K, D g) with the same preconditioner.  lambda: [n_dof]
 * (zero initial guess).  CG-VMS and DG-VMS problems (the DG-VMS blocks of
 * eq. S4_dg_stiffness_matrix have the same structure). */
dpp_status dpp_solve_adjoint(dpp_problem prob, dpp_precond pc, const dpp_solve_opts *opts,
                             const double *g, double *lambda, dpp_solve_stats *stats,
                             void *stream);

/* Gradient of J(x(theta)) given x (K x = f) and lambda (K^T lambda = dJ/dx),
 * boundary data held fixed:  dJ/dtheta = -lambda^T (dK/dtheta) x, for
 * theta = ln k1_e, ln k2_e (outputs [n_cells]: per simplex, or per box with
 * Q1 elements) and the scalar beta (g_beta [1], or [n_cells] per-cell
 * derivatives when the problem was assembled with beta_cells).  Any output
 * may be NULL.  DG-VMS problems return DPP_ERR_UNSUPPORTED. */
dpp_status dpp_param_grad(dpp_problem prob, const double *x, const double *lambda,
                          double *g_logk1, double *g_logk2, double *g_beta, void *stream);

/* L2 errors ||u_h - u||_L2 (section "Performance spectrum modeling", mesh
 * convergence) of a solution x [n_dof] (device) against the manufactured
 * solution of the two- and three-dimensional studies (section "Representative
 * numerical results") with parameters mms = {k1, k2, beta, mu} (host, all
 * > 0), integrated over the problem's cells: on the simplices with the
 * q-point conical-product Gauss rule (q^d points per simplex, 1 <= q <= 16),
 * for DG-VMS problems each simplex taking the values of its own vertex slots;
 * on Q1 box cells with the tensor Gauss-Legendre rule of q points per axis
 * and the multilinear interpolation of the cell's corner values.  err
 * (host, [4]) receives the errors of u1, p1, u2, p2.  The 3D micro-pressure
 * uses mu/(beta k2) (the pair that solves the mass balances).  Synchronises
 * the stream; allocates its scratch per call. */
dpp_status dpp_mms_l2_errors(dpp_problem prob, const double *x, const double mms[4], int q,
                             double err[4], void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dpp_mms_l2_errors without
 * any device or host allocation.  The quadrature rule (simplices; the box
 * cells' tensor rule is passed by value) and the partial sums live in one
 * fixed device array of DPP_NOALLOC_SCRATCH_BYTES per GPU, which
 * the library holds on every GPU it runs on until the process ends (its
 * address is looked up once per device, on the first call there).  Same
 * arguments and result as dpp_mms_l2_errors; at most 2048 workgroups take
 * the cells in a grid-stride loop, so the sums are grouped differently
 * and agree with dpp_mms_l2_errors up to rounding.  q > 16 is DPP_ERR_ARG;
 * a device index of 64 or more is DPP_ERR_UNSUPPORTED.  Every call on a GPU
 * uses that GPU's one array and leaves its contents there: calls that
 * overlap on one GPU (other host threads, other streams) race and must be
 * serialised by the caller.  Synchronises the stream. */
#define DPP_NOALLOC_SCRATCH_BYTES (256 * 1024)
dpp_status dpp_mms_l2_errors_noalloc(dpp_problem prob, const double *x, const double mms[4], int q,
                                     double err[4], void *stream);

/* Host only (no GPU): the conical-product Gauss rule of dpp_mms_l2_errors on
 * the reference simplex of dimension dim (2 or 3): lam [q^dim][dim+1]
 * barycentric points and w [q^dim] weights (summing to 1/dim!), caller-owned
 * host arrays. */
dpp_status dpp_simplex_rule(int dim, int q, double *lam, double *w);

/* Kernel-family timing (instrumentation, for benchmarks): while enabled,
 * launches of the families below are bracketed by HIP events on the stream
 * they run on, and the algorithmic bytes each launch must move (matrix
 * entries inside the box, vectors read and written once) are accumulated.
 * dpp_profile_enable(on) also clears earlier records.  Families:
 *   0 y = K x / r = b - K x          1 Chebyshev step with S_p product (finest)
 *   2 residual b - S_p x (finest)    3 r_p - K_pu D^-1 r_u
 *   4 D^-1 (r_u - K_up z_p)          5 coarser multigrid levels + coarse solve
 *   6 finest-level vector steps (first Chebyshev step, restriction,
 *     prolongation)                  7 Arnoldi (CGS2 passes, norms, scaling)
 * and of batched solves (bytes summed over the instances still running):
 *   8 K products                     9 Chebyshev steps with the S_p products
 *                                      of the instances' finest levels
 *  10 Schur right-hand side and      11 coarser levels, grid transfers and
 *     velocity step                     coarse solves
 *  12 Arnoldi passes
 * and of the DG-VMS fieldsplit:
 *  13 velocity-block Chebyshev steps 14 pressure side (K_up products, S_q
 *     with the simplex-block Jacobi     Chebyshev steps, r_p - K_pu y_u)
 *  15 slot/node transfers around the nodal cycle
 * dpp_profile_read synchronises on the recorded events and returns the launch
 * count, total milliseconds and total algorithmic bytes of one family. */
dpp_status dpp_profile_enable(int on);
dpp_status dpp_profile_read(int family, int64_t *launches, double *total_ms, double *total_bytes);

/* ---- Batched solves: many independent instances, one launch per phase ----
 * dpp_assemble_batch assembles nb instances (boxes[i], params[i]; uneven
 * sizes allowed, all of one dimension), builds each one's fieldsplit
 * preconditioner (opts may be NULL) and autotunes the lanes per stencil row of
 * every multigrid level index over the whole batch.  The solution vector is
 * the concatenation of the instances' vectors (each in the single-problem
 * layout) at offsets given by dpp_batch_sizes.  All kernels of a solve phase
 * (operator products, Schur steps, every V-cycle level, the coarse solves,
 * the Arnoldi passes) are single launches over all instances; converged
 * instances are masked out.  opts->use_graph replays each Arnoldi step from a
 * captured hipGraph. */
dpp_status dpp_assemble_batch(int nb, const dpp_box *boxes, const dpp_params *params,
                              const dpp_solve_opts *opts, void *stream, dpp_batch *out);
/* total_dof (host, may be NULL); offsets: host [nb+1] or NULL. */
dpp_status dpp_batch_sizes(dpp_batch b, int64_t *total_dof, int64_t *offsets);
/* Lanes per row chosen by the autotuner per multigrid level index (host, [16]). */
dpp_status dpp_batch_lanes(dpp_batch b, int *n_levels, int *lanes);
/* Solve every instance: x_concat (device [total_dof]) in = initial guess,
 * out = solution; stats: host array [nb] or NULL.  precision 0, 1 (FP64
 * iterative refinement on every instance's true residual around one batched
 * inner FGMRES with the FP32 K product and FP32 preconditioner per sweep) or 2
 * (the FP32 preconditioner); the stagnation test applies per instance (to the
 * refinement sweeps with precision 1).  Returns DPP_ERR_STAGNATED when an
 * instance was stopped by it, else DPP_ERR_NOT_CONVERGED when an instance
 * stopped at maxiter (or max_refine). */
dpp_status dpp_solve_batch(dpp_batch b, const dpp_solve_opts *opts, double *x_concat,
                           dpp_solve_stats *stats, void *stream);
/* Test hooks on concatenated vectors (device [total_dof]): y = K x and
 * z = P^-1 r for every instance in one batched launch sequence (FP64). */
dpp_status dpp_batch_spmv(dpp_batch b, const double *x, double *y, void *stream);
dpp_status dpp_batch_precond_apply(dpp_batch b, const double *r, double *z, void *stream);
void dpp_destroy_batch(dpp_batch b);

void dpp_destroy_problem(dpp_problem prob);
void dpp_destroy_precond(dpp_precond pc);

#ifdef __cplusplus
}
#endif
#endif /* DPP_H */
