// Flexible GMRES(m) on the whole four-field system (the outer Krylov method
// of the solver section, which picks up the couplings the fieldsplit drops),
// right preconditioned so the preconditioner may change between iterations.
//
// Arnoldi in FP64 with classical Gram-Schmidt and delayed
// re-orthogonalisation (DCGS2: the second Gram-Schmidt pass of vector j is
// folded into step j + 1; Swirydowicz et al. 2020, Bielich et al. 2022).
// Step j holds v_0..v_{j-1} orthonormal and t = v~_j, the once-orthogonalised
// unnormalised vector of the previous step.  z_j = M^-1 t (any z_j is valid in
// flexible GMRES), w = K z_j, then two passes over the basis:
//   pass A  a = V^T t, b = V^T w, t.w                      (one reduction)
//   pass B  v_j = (t - V a) / rho,  rho^2 = ||t||^2 - |a|^2
//           v~_{j+1} = w - V b - hjj v_j,  hjj = (t.w - a.b) / rho,
//           and ||v~_{j+1}||^2                            (one reduction)
// Column j of the Hessenberg matrix is (b, hjj, ||v~_{j+1}||) until step
// j + 1 corrects it by a' = V^T v~_{j+1} and the exact subdiagonal rho_{j+1};
// the host keeps the unrotated columns, redoes the last Givens rotation when
// a column is corrected, and tests convergence on the provisional column.
// Reductions use per-block partials summed in a fixed order
// (bit-reproducible).  The next step is normally queued before the host reads
// the current one, so the GPU does not wait for the host's Givens update.
#include <cmath>

#include "objects.h"
#include "mvec.h"
#include "profile.h"

namespace dpp {

namespace {

constexpr int MAXK = MV_MAXK;  // basis vectors handled by the fused kernels (restart <= 31)
constexpr int BS = MV_BS;
// Layout of the per-step reduced values (device hdev and the pinned host copy):
// [a (nj) | b (nj) | t.w] from index 0, then ||t||^2 of two consecutive steps,
// rho and hjj of the current step.
constexpr int H_ALPHA = 2 * MAXK;
constexpr int H_RHO = H_ALPHA + 2;
constexpr int H_HJJ = H_RHO + 1;
constexpr int H_LEN = H_HJJ + 1;

__device__ inline double wave_sum(double v) { return mv_wave_sum(v); }

// out[k] = sum over the nb partials of slot k (one block per slot, fixed tree).
__global__ __launch_bounds__(BS) void k_finish(const double *__restrict__ part, int nb,
                                               double *__restrict__ out) {
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += BS) s += part[(size_t)k * nb + b];
  s = wave_sum(s);
  __shared__ double sh[BS / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < BS / 64; ++w) t += sh[w];
    out[k] = t;
  }
}

// part[k] = sum_i V_k[i] w[i], k < nk
template <int NKP>
__global__ __launch_bounds__(BS) void k_mdot(const double *__restrict__ V, long n, int nk,
                                             const double *__restrict__ w, double *__restrict__ part) {
  double acc[NKP];
#pragma unroll
  for (int k = 0; k < NKP; ++k) acc[k] = 0.0;
  mv_dot<NKP>(V, n, nk, w, (long)blockIdx.x * BS + threadIdx.x, n, (long)gridDim.x * BS, acc);
  mv_block_store<NKP>(acc, nk, 0.0, false, part, gridDim.x, blockIdx.x);
}

// DCGS2 pass A for t = V_nj (basis rows 0..nj-1 before it): partial rows
// [0, nj) = V_k . t, [nj, 2nj) = V_k . w, 2nj = t . w.
template <int NKP>
__global__ __launch_bounds__(BS) void k_dcgs_a(const double *__restrict__ V, long n, int nj,
                                               const double *__restrict__ w, double *__restrict__ part) {
  mv_dcgs_a_waves<NKP>(V, n, nj, V + (size_t)nj * n, w, (long)blockIdx.x * 64, n,
                       (long)gridDim.x * 64, part, gridDim.x, blockIdx.x);
}

// DCGS2 pass B of step j = nj: coefficients from the reduced sums in h (and
// alpha = ||t||^2 in h[HA_ALPHA + (j & 1)]); v_j replaces t, v~_{j+1} goes to
// V_{j+1}, its squared norm to partial row 0; block 0 publishes rho and hjj.
template <int NKP>
__global__ __launch_bounds__(BS) void k_dcgs_b(double *__restrict__ V, long n, int nj,
                                               const double *__restrict__ w, double *__restrict__ h,
                                               double *__restrict__ part) {
  double a[NKP], b[NKP], rho, inv, hjj;
  mv_dcgs_coefs<NKP>(h, h[H_ALPHA + (nj & 1)], nj, a, b, rho, inv, hjj);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h[H_RHO] = rho;
    h[H_HJJ] = hjj;
  }
  double nrm = 0.0;
  mv_dcgs_update<NKP>(V, n, nj, a, b, inv, hjj, V + (size_t)nj * n, w, V + (size_t)(nj + 1) * n,
                      (long)blockIdx.x * BS + threadIdx.x, n, (long)gridDim.x * BS, nrm);
  mv_block_store<NKP>(a, 0, nrm, true, part, gridDim.x, blockIdx.x);
}

__global__ void k_scale(double *__restrict__ v, long n, double a) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v[i] *= a;
}

// x <- x + Z y
template <int NKP>
__global__ __launch_bounds__(BS) void k_update(const double *__restrict__ Z, long n, int nk,
                                               const double *__restrict__ y, double *__restrict__ x) {
  double yk[NKP];
  mv_coefs<NKP>(y, nk, yk);
  mv_update<NKP>(Z, n, nk, yk, x, (long)blockIdx.x * BS + threadIdx.x, n, (long)gridDim.x * BS);
}

__global__ void k_axpby(long n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// Reduction grid: up to RED_MAX blocks, so every SIMD holds several waves
// (the vectors are streamed once; the partials stay small).
constexpr int RED_MAX = 2048;
int red_blocks(long n) { return (int)std::min<long>(RED_MAX, std::max<long>(1, (n + BS - 1) / BS)); }

void ensure_ws(dpp_precond pc, int m) {
  const long n = pc->prob->ndof();
  ensure_reduction(pc);
  if (pc->ws_m >= m && pc->V.ptr) return;
  pc->drop_graphs();
  pc->V.alloc(sizeof(double) * (size_t)(m + 1) * n);
  pc->Z.alloc(sizeof(double) * (size_t)m * n);
  pc->w.alloc(sizeof(double) * n);
  pc->hdev.alloc(sizeof(double) * H_LEN);
  pc->ydev.alloc(sizeof(double) * (MAXK + 2));
  if (!pc->hpin) DPP_HIP(hipHostMalloc((void **)&pc->hpin, sizeof(double) * H_LEN, hipHostMallocDefault));
  if (!pc->hev) DPP_HIP(hipEventCreateWithFlags(&pc->hev, hipEventDisableTiming));
  pc->ws_m = m;
}

}  // namespace

void ensure_reduction(dpp_precond pc) {
  if (!pc->part.ptr) pc->part.alloc(sizeof(double) * (size_t)MV_PART_ROWS * RED_MAX);
}

void axpby(long n, double a, const double *x, double b, double *y, hipStream_t s) {
  k_axpby<<<std::min<long>(2048, blocks_for(n, 256)), 256, 0, s>>>(n, a, x, b, y);
  check_launch("axpby");
}

double norm2(const double *x, long n, double *scratch, hipStream_t s) {
  const int nb = red_blocks(n);
  k_mdot<1><<<nb, BS, 0, s>>>(x, n, 1, x, scratch);
  k_finish<<<1, BS, 0, s>>>(scratch, nb, scratch + (size_t)(MV_PART_ROWS - 1) * RED_MAX);
  check_launch("norm2");
  double h = 0.0;
  DPP_HIP(hipMemcpyAsync(&h, scratch + (size_t)(MV_PART_ROWS - 1) * RED_MAX, sizeof(double),
                         hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  return std::sqrt(h);
}

// mode 0: FP64 operator and preconditioner; 1: FP32 operator and
// preconditioner (inner solve of iterative refinement); 2: FP64 operator,
// FP32 preconditioner.
SolveResult fgmres(dpp_problem P, dpp_precond pc, const dpp_solve_opts &o, const double *b,
                   double *x, int mode, double rtol, int maxiter, double bn, hipStream_t s) {
  SolveResult res;
  const long n = P->ndof();
  const int m = o.restart;
  ensure_ws(pc, m);
  const bool op32 = mode == 1, pre32 = mode != 0;
  double *V = pc->V.as<double>(), *Z = pc->Z.as<double>(), *w = pc->w.as<double>();
  double *part = pc->part.as<double>(), *hd = pc->hdev.as<double>();
  double *hh = pc->hpin;
  const int nb = red_blocks(n);
  // unrotated Hessenberg columns, rotated columns, Givens rotations, and the
  // right-hand side before rotation i is applied (gpre) / after it (g)
  std::vector<double> Hr((size_t)(m + 1) * m), Rr((size_t)(m + 1) * m), cs(m), sn(m),
      gpre(m + 1), g(m + 1), y(m);
  auto Hc = [&](int i, int j) -> double & { return Hr[(size_t)j * (m + 1) + i]; };
  auto Rc = [&](int i, int j) -> double & { return Rr[(size_t)j * (m + 1) + i]; };
  // Step j (launches only, so it can be captured): z_j = M^-1 v~_j, w = K z_j,
  // DCGS2 passes A and B.
  DPP_CHECK(2 * (m - 1) + 1 <= MV_PART_ROWS - 1 && (size_t)nb * MV_PART_ROWS * sizeof(double) <= pc->part.bytes,
            DPP_ERR_ARG, "Krylov reduction buffer too small for the restart length");
  auto step = [&](int j) {
    double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
    precond_apply(pc, vj, zj, pre32, s);
    spmv_K(P, zj, w, s, op32);
    {
      // A reads V_0..V_j and w; B reads them again, writes v_j (j > 0) and v~_{j+1}
      ProfScope ps(PF_ARNOLDI, 8.0 * n * (2.0 * j + 4.0 + (j > 0 ? 2.0 : 1.0)), s);
      DPP_NK_SWITCH(std::max(j, 1), k_dcgs_a<NKP><<<nb, BS, 0, s>>>(V, n, j, w, part));
      k_finish<<<2 * j + 1, BS, 0, s>>>(part, nb, hd);
      DPP_NK_SWITCH(std::max(j, 1), k_dcgs_b<NKP><<<nb, BS, 0, s>>>(V, n, j, w, hd, part));
      k_finish<<<1, BS, 0, s>>>(part, nb, hd + H_ALPHA + ((j + 1) & 1));
    }
    check_launch("arnoldi");
  };
  const bool graph = o.use_graph != 0 && !prof_on();
  auto enqueue = [&](int j) {
    if (!graph) {
      step(j);
      return;
    }
    const auto key = std::make_tuple(j, mode, cycle_code(pc->opts));
    auto it = pc->graphs.find(key);
    if (it == pc->graphs.end()) {
      hipGraph_t gr;
      DPP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      step(j);
      DPP_HIP(hipStreamEndCapture(s, &gr));
      hipGraphExec_t ex;
      const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      DPP_HIP(e);
      it = pc->graphs.emplace(key, ex).first;
    }
    DPP_HIP(hipGraphLaunch(it->second, s));
  };
  // applies the final rotations 0..j-1 to unrotated column j, into Rc(., j)
  auto rotate_column = [&](int j) {
    for (int i = 0; i <= j + 1; ++i) Rc(i, j) = Hc(i, j);
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * Rc(i, j) + sn[i] * Rc(i + 1, j);
      Rc(i + 1, j) = -sn[i] * Rc(i, j) + cs[i] * Rc(i + 1, j);
      Rc(i, j) = t;
    }
  };
  // rotation j from the rotated column j; false if the column is singular
  auto make_rotation = [&](int j) {
    const double den = std::hypot(Rc(j, j), Rc(j + 1, j));
    if (!std::isfinite(den)) throw Error(DPP_ERR_NUMERIC, "NaN/Inf in the Arnoldi process");
    if (den == 0.0) return false;
    cs[j] = Rc(j, j) / den;
    sn[j] = Rc(j + 1, j) / den;
    Rc(j, j) = den;
    Rc(j + 1, j) = 0.0;
    g[j] = cs[j] * gpre[j];
    gpre[j + 1] = -sn[j] * gpre[j];
    return true;
  };
  if (bn == 0.0) {
    DPP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    res.converged = 1;
    return res;
  }
  hipEvent_t ev = pc->hev;
  Stagnation stag(o.stag_cycles, o.stag_ratio);
  while (true) {
    // true residual r = b - K x into V_0
    residual_K(P, b, x, V, s, op32);
    const double beta = norm2(V, n, part, s);
    res.rel = beta / bn;
    if (!std::isfinite(beta)) {
      res.status = DPP_ERR_NUMERIC;
      return res;
    }
    if (beta <= rtol * bn) {
      res.converged = 1;
      return res;
    }
    if (res.iters >= maxiter) {
      res.status = DPP_ERR_NOT_CONVERGED;
      return res;
    }
    if (stag.stalled(beta)) {
      res.status = DPP_ERR_STAGNATED;
      return res;
    }
    k_scale<<<std::min(2048, blocks_for(n, 256)), 256, 0, s>>>(V, n, 1.0 / beta);
    gpre[0] = beta;
    int k_used = 0;
    bool breakdown = false;
    enqueue(0);
    for (int j = 0; j < m; ++j) {
      // Copy step j's reductions and queue step j + 1 behind them before
      // reading, unless the residual trend says step j is likely the last
      // (a queued step that is not used costs a whole step).
      DPP_HIP(hipMemcpyAsync(hh, hd, sizeof(double) * H_LEN, hipMemcpyDeviceToHost, s));
      DPP_HIP(hipEventRecord(ev, s));
      const bool more = j + 1 < m && res.iters + 1 < maxiter;
      const double predicted = j >= 1 ? gpre[j] * gpre[j] / std::fabs(gpre[j - 1]) : gpre[0];
      const bool queued = more && std::fabs(predicted) > 4.0 * rtol * bn;
      if (queued) enqueue(j + 1);
      DPP_HIP(hipEventSynchronize(ev));
      res.iters++;
      const double *a = hh, *bv = hh + j;
      if (j > 0) {
        // correct column j-1 by a = V^T v~_j and the exact subdiagonal rho_j
        const double rho = hh[H_RHO];
        const double alpha = hh[H_ALPHA + (j & 1)];
        for (int i = 0; i < j; ++i) Hc(i, j - 1) += a[i];
        Hc(j, j - 1) = rho;
        rotate_column(j - 1);
        if (!make_rotation(j - 1) || !(rho > 1e-2 * std::sqrt(alpha))) {
          // v~_j was (almost) inside the basis: column j - 1 ends the cycle
          k_used = j;
          breakdown = true;
          break;
        }
      }
      // provisional column j
      for (int i = 0; i < j; ++i) Hc(i, j) = bv[i];
      Hc(j, j) = hh[H_HJJ];
      const double hn = std::sqrt(std::max(0.0, hh[H_ALPHA + ((j + 1) & 1)]));
      Hc(j + 1, j) = hn;
      rotate_column(j);
      if (!make_rotation(j)) {
        k_used = j;
        breakdown = true;
        break;
      }
      k_used = j + 1;
      if (std::fabs(gpre[j + 1]) <= rtol * bn || !more) break;
      if (hn <= 1e-300) {  // exact (happy) breakdown: the solution lies in the space
        breakdown = true;
        break;
      }
      if (!queued) enqueue(j + 1);
    }
    // wait for a queued step that will not be used, then x += Z y
    DPP_HIP(hipStreamSynchronize(s));
    if (k_used > 0) {
      for (int i = k_used - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < k_used; ++l) t -= Rc(i, l) * y[l];
        y[i] = t / Rc(i, i);
      }
      DPP_HIP(hipMemcpyAsync(pc->ydev.ptr, y.data(), sizeof(double) * k_used, hipMemcpyHostToDevice, s));
      DPP_NK_SWITCH(k_used, k_update<NKP><<<nb, BS, 0, s>>>(Z, n, k_used, pc->ydev.as<double>(), x));
      check_launch("update");
    }
    res.restarts++;
    if (breakdown && k_used == 0) {
      res.status = DPP_ERR_BREAKDOWN;
      return res;
    }
  }
}

}  // namespace dpp
