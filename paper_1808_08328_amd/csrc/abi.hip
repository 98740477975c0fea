// extern "C" entry points: argument checks, status codes, the solve drivers
// (plain FP64, FP32-preconditioned, and FP64 iterative refinement around an
// FP32 inner flexible GMRES) and the adjoint solve.
#include <chrono>
#include <cmath>
#include <cstring>

#include "objects.h"
#include "profile.h"
#include "batch.h"

namespace {

thread_local std::string g_last_error;

template <typename F>
dpp_status guard(F &&f) {
  try {
    f();
    g_last_error.clear();
    return DPP_OK;
  } catch (const dpp::Error &e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return DPP_ERR_ALLOC;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return DPP_ERR_HIP;
  }
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

void check_opts(const dpp_solve_opts &o) {
  DPP_CHECK(o.restart >= 1 && o.restart <= 31, DPP_ERR_ARG, "restart must be in 1..31");
  DPP_CHECK(o.maxiter >= 0, DPP_ERR_ARG, "maxiter must be >= 0");
  DPP_CHECK(o.rtol > 0.0 && o.rtol < 1.0, DPP_ERR_ARG, "rtol must be in (0, 1)");
  DPP_CHECK(o.precision >= 0 && o.precision <= 2, DPP_ERR_ARG, "precision must be 0, 1 or 2");
  DPP_CHECK(o.inner_rtol > 0.0 && o.inner_rtol < 1.0, DPP_ERR_ARG, "inner_rtol must be in (0, 1)");
  DPP_CHECK(o.max_refine >= 1, DPP_ERR_ARG, "max_refine must be >= 1");
  DPP_CHECK(o.coarse_max >= 0 && o.coarse_max <= 4000, DPP_ERR_ARG, "coarse_max must be in 0..4000");
  DPP_CHECK(o.cheb_degree >= 1 && o.cheb_degree <= 8, DPP_ERR_ARG, "cheb_degree must be in 1..8");
  for (int v : {o.cheb_pre_fine, o.cheb_pre_coarse})
    DPP_CHECK(v >= -1 && v <= 8, DPP_ERR_ARG, "pre-smoothing degrees must be -1 or 0..8");
  for (int v : {o.cheb_post_fine, o.cheb_post_coarse})
    DPP_CHECK(v == -1 || (v >= 1 && v <= 8), DPP_ERR_ARG, "post-smoothing degrees must be -1 or 1..8");
  DPP_CHECK(o.cheb_lo_frac >= 0.0 && o.cheb_lo_frac < 1.0, DPP_ERR_ARG,
            "cheb_lo_frac must be 0 (by dimension) or in (0,1)");
  DPP_CHECK(o.cheb_hi_factor >= 1.0, DPP_ERR_ARG, "cheb_hi_factor must be >= 1");
  DPP_CHECK(o.power_iters >= 1, DPP_ERR_ARG, "power_iters must be >= 1");
  DPP_CHECK(o.inner_maxiter >= 0, DPP_ERR_ARG, "inner_maxiter must be >= 0");
  DPP_CHECK(o.schedule >= -1 && o.schedule <= 9, DPP_ERR_ARG, "schedule must be -1 or 0..9");
  DPP_CHECK(o.stag_cycles >= 0, DPP_ERR_ARG, "stag_cycles must be >= 0");
  DPP_CHECK(o.stag_ratio > 0.0 && o.stag_ratio <= 1.0, DPP_ERR_ARG, "stag_ratio must be in (0, 1]");
}

void set_device_of(const void *p) {
  hipPointerAttribute_t at;
  if (p && hipPointerGetAttributes(&at, p) == hipSuccess && at.type == hipMemoryTypeDevice)
    DPP_HIP(hipSetDevice(at.device));
}

}  // namespace

extern "C" {

void dpp_default_opts(dpp_solve_opts *o) {
  if (!o) return;
  o->restart = 30;
  o->maxiter = 500;
  o->rtol = 1e-8;
  o->precision = 0;
  o->inner_rtol = 1e-4;
  o->max_refine = 20;
  o->coarse_max = 0;  // by dimension: 2200 nodes in 3D, 400 in 2D
  o->cheb_degree = 2;
  // post-smoothing only, V(0,2) on the finest level and V(0,3) below it
  // (measured fastest to 1e-8 in 2D and 3D)
  o->cheb_pre_fine = 0;
  o->cheb_post_fine = 2;
  o->cheb_pre_coarse = 0;
  o->cheb_post_coarse = 3;
  o->cheb_lo_frac = 0.0;
  o->cheb_hi_factor = 1.1;
  o->power_iters = 15;
  o->use_graph = 0;
  o->inner_maxiter = 0;
  o->schedule = -1;
  o->stag_cycles = 3;
  o->stag_ratio = 0.999;
}

const char *dpp_last_error(void) { return g_last_error.c_str(); }

dpp_status dpp_assemble(const dpp_box *box, const dpp_params *params, void *stream,
                        dpp_problem *out) {
  return guard([&] {
    DPP_CHECK(out, DPP_ERR_ARG, "null output handle");
    *out = nullptr;
    DPP_CHECK(params, DPP_ERR_ARG, "null params");
    set_device_of(params->k1);
    auto *P = new dpp_problem_s();
    try {
      dpp::assemble_problem(P, box, params, S(stream));
      DPP_HIP(hipStreamSynchronize(S(stream)));
    } catch (...) {
      delete P;
      throw;
    }
    *out = P;
  });
}

dpp_status dpp_problem_sizes(dpp_problem P, int64_t *n_dof, int64_t *n_nodes, int64_t *n_cells,
                             int64_t *nnz) {
  return guard([&] {
    DPP_CHECK(P, DPP_ERR_ARG, "null problem");
    if (n_dof) *n_dof = P->ndof();
    if (n_nodes) *n_nodes = P->npos();
    if (n_cells) *n_cells = P->g.nc;
    if (nnz) *nnz = P->nnz;
  });
}

dpp_status dpp_rhs(dpp_problem P, double *f_out, void *stream) {
  return guard([&] {
    DPP_CHECK(P && f_out, DPP_ERR_ARG, "null argument");
    DPP_HIP(hipMemcpyAsync(f_out, P->f.ptr, sizeof(double) * P->ndof(), hipMemcpyDeviceToDevice,
                           S(stream)));
  });
}

dpp_status dpp_export_csr(dpp_problem P, int64_t *rowptr, int32_t *cols, double *vals, void *stream) {
  return guard([&] {
    DPP_CHECK(P && rowptr && cols && vals, DPP_ERR_ARG, "null argument");
    if (P->dg)
      dpp::dg_export_csr(P, rowptr, cols, vals, S(stream));
    else
      dpp::export_csr(P, rowptr, cols, vals, S(stream));
  });
}

dpp_status dpp_spmv(dpp_problem P, int which, const double *x, double *y, void *stream) {
  return guard([&] {
    DPP_CHECK(P && x && y, DPP_ERR_ARG, "null argument");
    DPP_CHECK(which >= 0 && which <= 4, DPP_ERR_ARG, "which must be 0..4");
    DPP_CHECK(x != y, DPP_ERR_ARG, "x and y must not alias");
    DPP_CHECK(!P->dg || which == 0, DPP_ERR_UNSUPPORTED, "DG-VMS problems have the full product only");
    if (which == 0)
      dpp::spmv_K(P, x, y, S(stream));
    else
      dpp::spmv_block(P, which, x, y, S(stream));
  });
}

dpp_status dpp_setup_precond(dpp_problem P, const dpp_solve_opts *opts, void *stream,
                             dpp_precond *out) {
  return guard([&] {
    DPP_CHECK(P && out, DPP_ERR_ARG, "null argument");
    *out = nullptr;
    auto *pc = new dpp_precond_s();
    pc->prob = P;
    if (opts)
      pc->opts = *opts;
    else
      dpp_default_opts(&pc->opts);
    try {
      check_opts(pc->opts);
      const auto t0 = std::chrono::steady_clock::now();
      if (P->dg)
        dpp::dg_precond_setup(pc, S(stream));
      else
        dpp::precond_setup(pc, S(stream));
      DPP_HIP(hipStreamSynchronize(S(stream)));
      pc->ms_setup =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    } catch (...) {
      delete pc;
      throw;
    }
    *out = pc;
  });
}

dpp_status dpp_precond_info(dpp_precond pc, int *n_levels, int *level_n, double *hi) {
  return guard([&] {
    DPP_CHECK(pc, DPP_ERR_ARG, "null preconditioner");
    const int nl = (int)pc->lv.size();
    if (n_levels) *n_levels = nl;
    for (int l = 0; l < nl && l < 16; ++l) {
      if (level_n)
        for (int a = 0; a < 3; ++a) level_n[3 * l + a] = pc->lv[l]->g.n[a];
      if (hi)
        for (int q = 0; q < 2; ++q) hi[2 * l + q] = pc->lv[l]->hi[q];
    }
  });
}

dpp_status dpp_precond_shape(dpp_precond pc, int level, int *lanes, int *sym) {
  return guard([&] {
    DPP_CHECK(pc, DPP_ERR_ARG, "null preconditioner");
    DPP_CHECK(level >= 0 && level < (int)pc->lv.size(), DPP_ERR_ARG, "level out of range");
    if (lanes) *lanes = pc->lv[level]->shape.lpr;
    if (sym) *sym = pc->lv[level]->shape.sym ? 1 : 0;
  });
}

dpp_status dpp_precond_set_shape(dpp_precond pc, int level, int lanes, int sym) {
  return guard([&] {
    DPP_CHECK(pc, DPP_ERR_ARG, "null preconditioner");
    DPP_CHECK(level >= 0 && level + 1 < (int)pc->lv.size(), DPP_ERR_ARG,
              "level out of range (the coarsest level has no stencil kernels)");
    DPP_CHECK(lanes == 0 || lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8, DPP_ERR_ARG,
              "lanes must be 0 (two rows per lane), 1, 2, 4 or 8");
    DPP_CHECK(sym == 0 || sym == 1, DPP_ERR_ARG, "sym must be 0 or 1");
    pc->lv[level]->shape.lpr = lanes;
    pc->lv[level]->shape.sym = sym != 0;
    pc->drop_graphs();
  });
}

dpp_status dpp_precond_apply(dpp_precond pc, const double *r, double *z, void *stream) {
  return guard([&] {
    DPP_CHECK(pc && r && z && r != z, DPP_ERR_ARG, "bad argument");
    dpp::precond_apply(pc, r, z, false, S(stream));
  });
}

dpp_status dpp_vcycle(dpp_precond pc, const double *b, double *x, void *stream) {
  return guard([&] {
    DPP_CHECK(pc && b && x && b != x, DPP_ERR_ARG, "bad argument");
    DPP_CHECK(!pc->prob->dg, DPP_ERR_UNSUPPORTED, "a DG-VMS preconditioner has no nodal V-cycle of its own");
    dpp::vcycle(pc, b, x, S(stream));
  });
}

dpp_status dpp_level_spmv(dpp_precond pc, int level, int net, const double *x, double *y,
                          void *stream) {
  return guard([&] {
    DPP_CHECK(pc && x && y, DPP_ERR_ARG, "null argument");
    DPP_CHECK(level >= 0 && level < (int)pc->lv.size(), DPP_ERR_ARG, "level out of range");
    DPP_CHECK(net == 0 || net == 1, DPP_ERR_ARG, "net must be 0 or 1");
    dpp::level_spmv(pc, level, net, x, y, S(stream));
  });
}

static dpp_status solve_common(dpp_problem P, dpp_precond pc, const dpp_solve_opts *opts,
                               const double *rhs, double *x, dpp_solve_stats *stats, void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  dpp::SolveResult res;
  int refine = 0;
  dpp_status st = guard([&] {
    DPP_CHECK(P && pc && x, DPP_ERR_ARG, "null argument");
    DPP_CHECK(pc->prob == P, DPP_ERR_ARG, "preconditioner belongs to another problem");
    dpp_solve_opts o = pc->opts;
    if (opts) {
      o = *opts;
      // the multigrid hierarchy is fixed at setup
      o.coarse_max = pc->opts.coarse_max;
      o.power_iters = pc->opts.power_iters;
      o.cheb_lo_frac = pc->opts.cheb_lo_frac;
      o.cheb_hi_factor = pc->opts.cheb_hi_factor;
      o.schedule = pc->opts.schedule;
    }
    // a rejected call leaves the handle as it was
    check_opts(o);
    DPP_CHECK(!P->dg || o.precision != 1, DPP_ERR_UNSUPPORTED,
              "DG-VMS problems are solved in FP64 or with the FP32 preconditioner (precision 0 or 2)");
    pc->opts.cheb_degree = o.cheb_degree;
    pc->opts.cheb_pre_fine = o.cheb_pre_fine;
    pc->opts.cheb_post_fine = o.cheb_post_fine;
    pc->opts.cheb_pre_coarse = o.cheb_pre_coarse;
    pc->opts.cheb_post_coarse = o.cheb_post_coarse;
    if (pc->dgpc) {
      // DG-VMS: the nodal cycle of the pressure solve takes the same degrees
      dpp_precond_s &nc = *pc->dgpc;
      nc.opts.cheb_degree = o.cheb_degree;
      nc.opts.cheb_pre_fine = o.cheb_pre_fine;
      nc.opts.cheb_post_fine = o.cheb_post_fine;
      nc.opts.cheb_pre_coarse = o.cheb_pre_coarse;
      nc.opts.cheb_post_coarse = o.cheb_post_coarse;
    }
    hipStream_t s = S(stream);
    if (o.use_graph && !dpp::prof_on()) {
      // Graphs are captured and replayed on a stream the library owns (the
      // caller's may be the legacy default stream, which cannot be captured),
      // ordered after the caller's stream; the solve ends with a host wait.
      if (!pc->gstream) DPP_HIP(hipStreamCreateWithFlags(&pc->gstream, hipStreamNonBlocking));
      hipEvent_t ev;
      DPP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      DPP_HIP(hipEventRecord(ev, s));
      DPP_HIP(hipStreamWaitEvent(pc->gstream, ev, 0));
      (void)hipEventDestroy(ev);
      s = pc->gstream;
    }
    const double *b = rhs ? rhs : P->f.as<double>();
    const long n = P->ndof();
    const bool singular = dpp::pure_flux(P->g);
    if (singular) {
      // pure flux: K is singular; solve for the consistent part of b
      if (!pc->bproj.ptr) pc->bproj.alloc(sizeof(double) * n);
      DPP_HIP(hipMemcpyAsync(pc->bproj.ptr, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      dpp::consistent_rhs(P, pc->bproj.as<double>(), s);
      b = pc->bproj.as<double>();
    }
    dpp::ensure_reduction(pc);
    const double bn = dpp::norm2(b, n, pc->part.as<double>(), s);
    DPP_CHECK(std::isfinite(bn), DPP_ERR_NUMERIC, "right-hand side holds NaN/Inf");
    if (o.precision != 1) {
      if (o.precision == 2) dpp::precond_make32(pc, s);
      res = dpp::fgmres(P, pc, o, b, x, o.precision == 2 ? 2 : 0, o.rtol, o.maxiter, bn, s);
    } else {
      dpp::precond_make32(pc, s);
      if (!pc->xtmp.ptr) {
        pc->xtmp.alloc(sizeof(double) * n);
        pc->rtmp.alloc(sizeof(double) * n);
      }
      double *e = pc->xtmp.as<double>(), *r = pc->rtmp.as<double>();
      dpp::Stagnation stag(o.stag_cycles, o.stag_ratio);
      // the inner solves stop at their own tolerance; stagnation is judged on
      // the refinement sweeps
      dpp_solve_opts oi = o;
      oi.stag_cycles = 0;
      while (true) {
        dpp::residual_K(P, b, x, r, s);
        const double rn = dpp::norm2(r, n, pc->part.as<double>(), s);
        res.rel = bn > 0 ? rn / bn : 0.0;
        DPP_CHECK(std::isfinite(rn), DPP_ERR_NUMERIC, "NaN/Inf in the refinement residual");
        if (rn <= o.rtol * bn) {
          res.converged = 1;
          res.status = DPP_OK;
          break;
        }
        if (res.iters >= o.maxiter || refine >= o.max_refine) {
          res.status = DPP_ERR_NOT_CONVERGED;
          break;
        }
        if (stag.stalled(rn)) {
          res.status = DPP_ERR_STAGNATED;
          break;
        }
        DPP_HIP(hipMemsetAsync(e, 0, sizeof(double) * n, s));
        const int left = o.maxiter - res.iters;
        const int lim = o.inner_maxiter > 0 ? std::min(o.inner_maxiter, left) : left;
        dpp::SolveResult in = dpp::fgmres(P, pc, oi, r, e, 1, o.inner_rtol, lim, rn, s);
        if (in.status == DPP_ERR_NUMERIC) {
          res.status = in.status;
          break;
        }
        dpp::axpby(n, 1.0, e, 1.0, x, s);
        res.iters += in.iters;
        res.restarts += in.restarts;
        ++refine;
      }
    }
    if (singular) dpp::normalize_pressures(P, x, s);  // int p1 = 0
    DPP_HIP(hipStreamSynchronize(s));
    if (res.status != DPP_OK) {
      throw dpp::Error(res.status,
                       res.status == DPP_ERR_NOT_CONVERGED ? "iteration limit reached before the tolerance"
                       : res.status == DPP_ERR_STAGNATED   ? "restart cycles stopped reducing the residual"
                       : res.status == DPP_ERR_NUMERIC     ? "NaN/Inf in the iteration"
                                                           : "Krylov breakdown");
    }
  });
  if (stats) {
    stats->refinements = refine;
    stats->iters = res.iters;
    stats->restarts = res.restarts;
    stats->converged = res.converged;
    stats->rel_residual = res.rel;
    stats->ms_solve =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->ms_setup = pc ? pc->ms_setup : 0.0;
  }
  return st;
}

dpp_status dpp_solve(dpp_problem P, dpp_precond pc, const dpp_solve_opts *opts, const double *rhs,
                     double *x, dpp_solve_stats *stats, void *stream) {
  return solve_common(P, pc, opts, rhs, x, stats, stream);
}

dpp_status dpp_solve_adjoint(dpp_problem P, dpp_precond pc, const dpp_solve_opts *opts,
                             const double *g, double *lambda, dpp_solve_stats *stats, void *stream) {
  double *dg = nullptr;
  dpp_status st = guard([&] {
    DPP_CHECK(P && pc && g && lambda && g != lambda, DPP_ERR_ARG, "bad argument");
    DPP_CHECK(pc->prob == P, DPP_ERR_ARG, "preconditioner belongs to another problem");
    const long n = P->ndof();
    // allocated on the first adjoint solve of this preconditioner, then reused
    if (!pc->adjrhs.ptr) pc->adjrhs.alloc(sizeof(double) * n);
    dg = pc->adjrhs.as<double>();
    dpp::flip_pressure_sign(P, g, dg, S(stream));
    DPP_HIP(hipMemsetAsync(lambda, 0, sizeof(double) * n, S(stream)));
  });
  if (st != DPP_OK) return st;
  st = solve_common(P, pc, opts, dg, lambda, stats, stream);
  if (st != DPP_OK && st != DPP_ERR_NOT_CONVERGED) return st;
  dpp_status st2 = guard([&] {
    dpp::flip_pressure_sign(P, lambda, lambda, S(stream));
    DPP_HIP(hipStreamSynchronize(S(stream)));
  });
  return st2 != DPP_OK ? st2 : st;
}

dpp_status dpp_param_grad(dpp_problem P, const double *x, const double *lambda, double *g_logk1,
                          double *g_logk2, double *g_beta, void *stream) {
  return guard([&] {
    DPP_CHECK(P && x && lambda, DPP_ERR_ARG, "null argument");
    dpp::param_grad(P, x, lambda, g_logk1, g_logk2, g_beta, S(stream));
  });
}

dpp_status dpp_mms_l2_errors(dpp_problem P, const double *x, const double mms[4], int q,
                             double err[4], void *stream) {
  return guard([&] {
    DPP_CHECK(P && x && mms && err, DPP_ERR_ARG, "null argument");
    dpp::mms_l2_errors(P, x, mms, q, err, S(stream));
  });
}

dpp_status dpp_mms_l2_errors_noalloc(dpp_problem P, const double *x, const double mms[4], int q,
                                     double err[4], void *stream) {
  return guard([&] {
    DPP_CHECK(P && x && mms && err, DPP_ERR_ARG, "null argument");
    dpp::mms_l2_errors_noalloc(P, x, mms, q, err, S(stream));
  });
}

dpp_status dpp_simplex_rule(int dim, int q, double *lam, double *w) {
  return guard([&] {
    DPP_CHECK(lam && w && (dim == 2 || dim == 3) && q >= 1 && q <= 16, DPP_ERR_ARG, "bad argument");
    std::vector<double> l, ww;
    dpp::simplex_rule(dim, q, l, ww);
    std::copy(l.begin(), l.end(), lam);
    std::copy(ww.begin(), ww.end(), w);
  });
}

dpp_status dpp_assemble_batch(int nb, const dpp_box *boxes, const dpp_params *params,
                              const dpp_solve_opts *opts, void *stream, dpp_batch *out) {
  return guard([&] {
    DPP_CHECK(out && boxes && params, DPP_ERR_ARG, "null argument");
    *out = nullptr;
    DPP_CHECK(nb >= 1 && nb <= 4096, DPP_ERR_ARG, "nb must be in 1..4096");
    auto *B = new dpp_batch_s();
    try {
      B->nb = nb;
      B->dim = boxes[0].dim;
      if (opts)
        B->opts = *opts;
      else
        dpp_default_opts(&B->opts);
      check_opts(B->opts);
      set_device_of(params[0].k1);
      for (int i = 0; i < nb; ++i) {
        DPP_CHECK(boxes[i].dim == B->dim, DPP_ERR_ARG, "all instances of a batch share one dimension");

        DPP_CHECK(boxes[i].elem == dpp::ELEM_P1, DPP_ERR_UNSUPPORTED,
                  "batched instances use P1 simplices");
        auto *P = new dpp_problem_s();
        B->P.push_back(P);
        dpp::assemble_problem(P, &boxes[i], &params[i], S(stream));
        B->any_bc = B->any_bc || (P->g.fix[0] | P->g.fix[1]) != 0;
        auto *pc = new dpp_precond_s();
        B->pc.push_back(pc);
        pc->prob = P;
        pc->opts = B->opts;
        pc->tune_shapes = false;
        dpp::precond_setup(pc, S(stream));
      }
      dpp::batch_setup(B, S(stream));
    } catch (...) {
      delete B;
      throw;
    }
    *out = B;
  });
}

dpp_status dpp_batch_sizes(dpp_batch B, int64_t *total_dof, int64_t *offsets) {
  return guard([&] {
    DPP_CHECK(B, DPP_ERR_ARG, "null batch");
    if (total_dof) *total_dof = B->ntot;
    if (offsets)
      for (int i = 0; i <= B->nb; ++i) offsets[i] = B->doff[i];
  });
}

dpp_status dpp_batch_lanes(dpp_batch B, int *n_levels, int *lanes) {
  return guard([&] {
    DPP_CHECK(B, DPP_ERR_ARG, "null batch");
    if (n_levels) *n_levels = B->nlev;
    if (lanes)
      for (int l = 0; l < B->nlev && l < 16; ++l) lanes[l] = B->lpr[l];
  });
}

dpp_status dpp_solve_batch(dpp_batch B, const dpp_solve_opts *opts, double *x, dpp_solve_stats *stats,
                           void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  std::vector<dpp_solve_stats> st;
  dpp_status status = guard([&] {
    DPP_CHECK(B && x, DPP_ERR_ARG, "null argument");
    dpp_solve_opts o = opts ? *opts : B->opts;
    o.coarse_max = B->opts.coarse_max;
    o.cheb_lo_frac = B->opts.cheb_lo_frac;
    o.cheb_hi_factor = B->opts.cheb_hi_factor;
    o.power_iters = B->opts.power_iters;
    o.cheb_degree = B->opts.cheb_degree;
    o.cheb_pre_fine = B->opts.cheb_pre_fine;
    o.cheb_post_fine = B->opts.cheb_post_fine;
    o.cheb_pre_coarse = B->opts.cheb_pre_coarse;
    o.cheb_post_coarse = B->opts.cheb_post_coarse;
    check_opts(o);
    st.resize(B->nb);
    dpp::batch_solve(B, o, x, st.data(), S(stream));
    for (int i = 0; i < B->nb; ++i)
      if (!st[i].converged && B->stalled.size() == st.size() && B->stalled[i])
        throw dpp::Error(DPP_ERR_STAGNATED, "an instance's restart cycles stopped reducing its residual");
    for (auto &s : st)
      if (!s.converged) throw dpp::Error(DPP_ERR_NOT_CONVERGED, "an instance reached maxiter");
  });
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats && B)
    for (int i = 0; i < (int)st.size(); ++i) {
      stats[i] = st[i];
      stats[i].ms_solve = ms;
      stats[i].ms_setup = 0.0;
    }
  return status;
}

dpp_status dpp_batch_spmv(dpp_batch B, const double *x, double *y, void *stream) {
  return guard([&] {
    DPP_CHECK(B && x && y && x != y, DPP_ERR_ARG, "bad argument");
    dpp::batch_apply(B, 0, x, y, S(stream));
  });
}

dpp_status dpp_batch_precond_apply(dpp_batch B, const double *r, double *z, void *stream) {
  return guard([&] {
    DPP_CHECK(B && r && z && r != z, DPP_ERR_ARG, "bad argument");
    dpp::batch_apply(B, 1, r, z, S(stream));
  });
}

void dpp_destroy_batch(dpp_batch B) { delete B; }

void dpp_destroy_problem(dpp_problem P) { delete P; }
void dpp_destroy_precond(dpp_precond pc) { delete pc; }

}  // extern "C"
