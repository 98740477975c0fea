// Library objects behind the opaque ABI handles and the cross-file launchers.
#pragma once

#include <map>
#include <memory>
#include <tuple>

#include "common.h"
#include "stagnation.h"

namespace dpp {

// Owning device buffer.
struct DBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  explicit DBuf(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    DPP_HIP(hipMalloc(&ptr, b));
    bytes = b;
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  ~DBuf() { release(); }
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) {
    o.ptr = nullptr;
    o.bytes = 0;
  }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) {
      release();
      ptr = o.ptr;
      bytes = o.bytes;
      o.ptr = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(ptr);
  }
};

}  // namespace dpp

// Assembled problem: K in node-pair stencil storage and f.
struct dpp_problem_s {
  dpp::Grid g;
  double mu = 1.0;
  int beta_per_cell = 0;
  double beta = 0.0;
  int ns = 0;           // K stencil size
  long nnz = 0;         // structural nonzeros of K in CSR terms
  dpp::DBuf kvals;      // [nv][ns][N] FP64, every kind on every offset (assembly, selfp, export)
  dpp::DBuf kh;         // half storage (layout KH<dim>) read by the hot kernels
  dpp::DBuf kh32;       // FP32 copy of kh (mixed precision), made on demand
  dpp::DBuf korder;     // [blocks] node block of each K-product workgroup (column order)
  dpp::DBuf upt, upt32; // K_up class table (UPT<dim>), FP64 and FP32 copies
  dpp::DBuf f;          // [n_dof]
  dpp::DBuf dinv;       // [2][N] 1/diag(K_uu^i)
  dpp::DBuf k1, k2, betac;  // coefficient copies [n_cells] for the gradient
  // DG-VMS (g is the node grid of the simplices; unknowns sit on vertex slots)
  int dg = 0;
  long nslot = 0;       // simplices x (dim + 1)
  dpp::DBuf dgA;        // [2][n_cells][dim+2][SB][SB] element blocks (SB = (dim+1)^2)
  dpp::DBuf dgB;        // [n_cells][dim+1][dim+1] inter-network transfer -(beta/mu) M
  dpp::DBuf dgnb;       // [n_cells][dim+1] facet neighbours (-1: boundary)
  long dgcoupled = 0;   // (simplex, simplex) blocks per network: self plus interior facets
  dpp::DBuf dgtab;      // per simplex type of a box: barycentric gradients, facet normals, facet weights
  long npos() const { return dg ? nslot : g.N; }  // positions per field component
  long ndof() const { return (long)(2 * g.dim + 2) * npos(); }
};

namespace dpp {

// Kernel shape of a multigrid level: lanes per stencil row (1, 2, 4, 8) and
// full or symmetric-half storage; chosen per level by the autotuner.
struct Shape {
  int lpr = 1;
  bool sym = false;
};

struct Level {
  Grid g;
  DBuf A;        // [2][nt][N] FP64 stencil values (network-major)
  DBuf A32;      // FP32 copy (mixed)
  DBuf Ah, Ah32; // symmetric half: zero offset + positive half of T
  DBuf dinv;     // [2][N]
  DBuf dinv32;
  double lo[2] = {0, 0}, hi[2] = {0, 0};
  Shape shape;     // level kernel shape (autotuned)
  // work vectors [2][N] each (FP64 and FP32 views share nothing)
  DBuf b, xa, xb, d, r, e;          // e: coarse-grid correction received from below
  DBuf b32, xa32, xb32, d32, r32, e32;
};

}  // namespace dpp

struct dpp_precond_s {
  dpp_problem prob = nullptr;
  dpp_solve_opts opts;
  std::vector<std::unique_ptr<dpp::Level>> lv;
  dpp::DBuf cinv;   // [2][nc][nc] FP64 inverse of the coarsest operator
  int ncoarse = 0;
  dpp::DBuf rhat;   // [2][N] level-0 right-hand side of the V-cycle
  dpp::DBuf bproj;  // [n_dof] consistent right-hand side (pure-flux problems)
  dpp::DBuf adjrhs; // [n_dof] D g of the adjoint solve, kept across calls
  dpp::DBuf rhat32;
  dpp::DBuf red;    // reduction scratch
  bool has32 = false;
  bool tune_shapes = true;  // autotune the level kernel shapes (off for batch members)
  double ms_setup = 0.0;    // wall time of dpp_setup_precond
  // Krylov workspace, kept across solves
  int ws_m = 0;
  dpp::DBuf V, Z, w, part, hdev, ydev, xtmp, rtmp;
  // Arnoldi steps captured as graphs, keyed by (step j, mode, smoothing
  // degrees); they hold the workspace pointers above, so any reallocation or
  // change of a level's kernel shape drops them.
  std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
  hipStream_t gstream = nullptr;  // capture/replay stream (default priority)
  double *hpin = nullptr;         // pinned host copy of one step's reductions
  hipEvent_t hev = nullptr;       // marks that copy
  // DG-VMS: the nodal CG-VMS problem of the same box and coefficients with its
  // own preconditioner (coarse level of the pressure blocks), and the DG
  // level's diagonals, Chebyshev bounds and work vectors
  std::unique_ptr<dpp_problem_s> dgcg;
  dpp_precond_s *dgpc = nullptr;
  dpp::DBuf dgzero, dgdu, dgds, dgrh, dgza, dgzb, dgd, dgtu, dgcb, dgcx, dgpart;
  dpp::DBuf dgbinv, dgva, dgvb, dgyu;  // velocity block: packed simplex-block inverses, Chebyshev work
  // FP32 copies (diagonals and block inverses rounded once) and FP32 work
  // vectors of the FP32 preconditioner (precision 2), made on demand
  dpp::DBuf dgdu32, dgds32, dgbinv32, dgrh32, dgza32, dgzb32, dgd32, dgtu32, dgcb32, dgcx32, dgva32, dgvb32, dgyu32;
  dpp::DBuf dgr32, dgz32;  // [n_dof] the residual and the correction
  bool dg32 = false;
  double dghi[2] = {0.0, 0.0}, dglo[2] = {0.0, 0.0};    // pressure-block Chebyshev interval
  double dgvhi[2] = {0.0, 0.0}, dgvlo[2] = {0.0, 0.0};  // velocity-block Chebyshev interval
  void drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
  }
  ~dpp_precond_s() {
    delete dgpc;  // before dgcg, the problem it belongs to
    drop_graphs();
    if (gstream) (void)hipStreamDestroy(gstream);
    if (hev) (void)hipEventDestroy(hev);
    if (hpin) (void)hipHostFree(hpin);
  }
};

namespace dpp {

// --- assemble.hip
void assemble_problem(dpp_problem P, const dpp_box *box, const dpp_params *prm, hipStream_t s);
void export_csr(dpp_problem P, int64_t *rowptr, int32_t *cols, double *vals, hipStream_t s);
long count_nnz(const Grid &g);

// --- ops.hip (operators on the ABI vector layout)
void spmv_K(dpp_problem P, const double *x, double *y, hipStream_t s, bool fp32 = false);
void residual_K(dpp_problem P, const double *b, const double *x, double *r, hipStream_t s,
                bool fp32 = false);
void spmv_block(dpp_problem P, int which, const double *x, double *y, hipStream_t s);
void make_dinv(dpp_problem P, hipStream_t s);
void make_selfp(dpp_problem P, double *S, hipStream_t s);
void make_kh(dpp_problem P, hipStream_t s);
void make_up_table(dpp_problem P, hipStream_t s);
void make_k32(dpp_problem P, hipStream_t s);
// algorithmic bytes of one K product (resid: r = b - K x) and of the K_up class table
double kbytes(const Grid &g, bool fp32, bool resid);
double upt_bytes(const Grid &g, bool fp32);
// Schur fieldsplit pieces: rhat_i = r_p_i - K_pu^i diag^-1 r_u_i ; z_u = diag^-1 (r_u - K_up z_p)
// With ldinv non-null it also writes the finest level's first Chebyshev step
// x = d = c2 ldinv rhat into xa and d (ldinv, xa, d in the level's precision).
void schur_rhs(dpp_problem P, const double *r, void *rhat, bool fp32, hipStream_t s,
               const void *ldinv = nullptr, void *xa = nullptr, void *d = nullptr,
               const double *c2 = nullptr);
void schur_velocity(dpp_problem P, const double *r, const void *zp, bool fp32, double *z,
                    hipStream_t s);

// --- mg.hip
void precond_setup(dpp_precond pc, hipStream_t s);
void precond_apply(dpp_precond pc, const double *r, double *z, bool fp32, hipStream_t s);
// L2 errors against the manufactured solution (err: u1, p1, u2, p2) and the
// conical-product Gauss rule they use
void mms_l2_errors(dpp_problem P, const double *x, const double mms[4], int q, double err[4],
                   hipStream_t s);
// the same without allocating: rule and partial sums in the fixed device array
void mms_l2_errors_noalloc(dpp_problem P, const double *x, const double mms[4], int q,
                           double err[4], hipStream_t s);
void simplex_rule(int dim, int q, std::vector<double> &lam, std::vector<double> &w);
// pure-flux case: velocity faces everywhere in both networks (singular K)
bool pure_flux(const Grid &g);
// DG-VMS (dg.hip)
void dg_assemble(dpp_problem P, const dpp_params *prm, hipStream_t s);
void dg_spmv(dpp_problem P, const double *x, const double *bsub, double *y, hipStream_t s);
void dg_export_csr(dpp_problem P, int64_t *rowptr, int32_t *cols, double *vals, hipStream_t s);
void dg_precond_setup(dpp_precond pc, hipStream_t s);
void dg_precond_apply(dpp_precond pc, const double *r, double *z, bool fp32, hipStream_t s);
void dg_make32(dpp_precond pc, hipStream_t s);
void consistent_rhs(dpp_problem P, double *b, hipStream_t s);
void normalize_pressures(dpp_problem P, double *x, hipStream_t s);
void vcycle(dpp_precond pc, const double *b, double *x, hipStream_t s);  // FP64, [2][N] in/out
void vcycle32(dpp_precond pc, const float *b, float *x, hipStream_t s);  // FP32 levels (precond_make32)
void level_spmv(dpp_precond pc, int level, int net, const double *x, double *y, hipStream_t s);
void precond_make32(dpp_precond pc, hipStream_t s);
// Chebyshev degrees of level l's pre- and post-smoothing (the finest level or
// a coarser one; -1 in the options means cheb_degree)
inline int cheb_pre(const dpp_solve_opts &o, int l) {
  const int v = l == 0 ? o.cheb_pre_fine : o.cheb_pre_coarse;
  return v < 0 ? o.cheb_degree : v;
}
inline int cheb_post(const dpp_solve_opts &o, int l) {
  const int v = l == 0 ? o.cheb_post_fine : o.cheb_post_coarse;
  return v < 0 ? o.cheb_degree : v;
}
// identifies the V-cycle's smoothing degrees (part of a captured graph's key)
inline int cycle_code(const dpp_solve_opts &o) {
  return ((cheb_pre(o, 0) * 16 + cheb_post(o, 0)) * 16 + cheb_pre(o, 1)) * 16 + cheb_post(o, 1);
}

// --- krylov.hip
struct SolveResult {
  int iters = 0, restarts = 0, converged = 0;
  double rel = 0.0;
  dpp_status status = DPP_OK;
};
double norm2(const double *x, long n, double *scratch, hipStream_t s);
void ensure_reduction(dpp_precond pc);
// mode 0: FP64 operator and preconditioner; 1: FP32 operator and
// preconditioner (inner solve of iterative refinement); 2: FP64 operator with
// the FP32 preconditioner.
SolveResult fgmres(dpp_problem P, dpp_precond pc, const dpp_solve_opts &o, const double *b,
                   double *x, int mode, double rtol, int maxiter, double bnorm_ref,
                   hipStream_t s);
void axpby(long n, double a, const double *x, double b, double *y, hipStream_t s);

// --- batch.hip
void batch_setup(dpp_batch B, hipStream_t s);
void batch_solve(dpp_batch B, const dpp_solve_opts &o, double *x, dpp_solve_stats *st, hipStream_t s);
void batch_apply(dpp_batch B, int what, const double *x, double *y, hipStream_t s);

// --- adjoint.hip
void param_grad(dpp_problem P, const double *x, const double *lam, double *g1, double *g2,
                double *gb, hipStream_t s);
void flip_pressure_sign(dpp_problem P, const double *in, double *out, hipStream_t s);

}  // namespace dpp
