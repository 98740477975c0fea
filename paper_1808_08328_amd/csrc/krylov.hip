// Flexible GMRES(m) on the whole four-field system (the outer Krylov method
// of the solver section, which picks up the couplings the fieldsplit drops),
// right preconditioned so the preconditioner may change between iterations.
//
// Arnoldi in FP64 with classical Gram-Schmidt applied twice (CGS2), organised
// to read the basis three times per step:
//   pass 1  h1 = V^T w                                (multi-dot)
//   pass 2  w' = w - V h1 and h2 = V^T w'            (fused multi-axpy + multi-dot)
//   pass 3  v_{j+1} = w' - V h2 with ||.||^2          (fused multi-axpy + norm)
// followed by a scaling that reads the norm from device memory.  Reductions
// use per-block partials summed in a fixed order (bit-reproducible).  The
// (m+1) x m Hessenberg system and its Givens rotations are kept on the host;
// one small copy per iteration returns the new column.
#include <cmath>

#include "objects.h"
#include "profile.h"

namespace dpp {

namespace {

constexpr int MAXK = 32;  // basis vectors handled by the fused kernels (restart <= 31)
constexpr int BS = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-reduce nk (<= MAXK) per-thread values, plus one extra value stored
// in slot nk when with_extra, into partials part[k*gridDim.x + block].
__device__ inline void block_store(const double *acc, int nk, double *part, double extra = 0.0,
                                   bool with_extra = false) {
  __shared__ double sh[BS / 64][MAXK + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    if (k < nk) {
      double v = wave_sum(acc[k]);
      if (lane == 0) sh[wv][k] = v;
    }
  }
  if (with_extra) {
    double v = wave_sum(extra);
    if (lane == 0) sh[wv][MAXK] = v;
  }
  __syncthreads();
  const int tot = nk + (with_extra ? 1 : 0);
  if ((int)threadIdx.x < tot) {
    const int slot = ((int)threadIdx.x == nk) ? MAXK : (int)threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += sh[w][slot];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

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
__global__ __launch_bounds__(BS) void k_mdot(const double *__restrict__ V, long n, int nk,
                                             const double *__restrict__ w, double *__restrict__ part) {
  double acc[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; ++k) acc[k] = 0.0;
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < MAXK; ++k)
      if (k < nk) acc[k] += V[(size_t)k * n + i] * wi;
  }
  block_store(acc, nk, part);
}

// w <- w - V h ; part[k] = V_k . w (k < nk), part[nk] = ||w||^2
__global__ __launch_bounds__(BS) void k_axpy_mdot(const double *__restrict__ V, long n, int nk,
                                                  const double *__restrict__ h,
                                                  double *__restrict__ w, double *__restrict__ part) {
  double acc[MAXK];
  double hk[MAXK], nrm = 0.0;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) acc[k] = 0.0;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) hk[k] = (k < nk) ? h[k] : 0.0;
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
    double v[MAXK];
    double s = w[i];
#pragma unroll
    for (int k = 0; k < MAXK; ++k) {
      v[k] = (k < nk) ? V[(size_t)k * n + i] : 0.0;
      s -= hk[k] * v[k];
    }
    w[i] = s;
#pragma unroll
    for (int k = 0; k < MAXK; ++k) acc[k] += v[k] * s;
    nrm += s * s;
  }
  block_store(acc, nk, part, nrm, true);
}

// out <- w - V h ; part[0] = ||out||^2
__global__ __launch_bounds__(BS) void k_axpy_norm(const double *__restrict__ V, long n, int nk,
                                                  const double *__restrict__ h,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ vout, double *__restrict__ part) {
  double hk[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; ++k) hk[k] = (k < nk) ? h[k] : 0.0;
  double nrm = 0.0;
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
    double s = w[i];
#pragma unroll
    for (int k = 0; k < MAXK; ++k)
      if (k < nk) s -= hk[k] * V[(size_t)k * n + i];
    vout[i] = s;
    nrm += s * s;
  }
  block_store(hk, 0, part, nrm, true);
}

// v <- v / sqrt(ss)   (ss read from device memory; zero norm leaves v as is)
__global__ void k_scale_rsqrt(double *__restrict__ v, long n, const double *__restrict__ ss) {
  const double s2 = ss[0];
  if (!(s2 > 0.0)) return;
  const double inv = 1.0 / sqrt(s2);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v[i] *= inv;
}

__global__ void k_scale(double *__restrict__ v, long n, double a) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v[i] *= a;
}

// x <- x + Z y
__global__ __launch_bounds__(BS) void k_update(const double *__restrict__ Z, long n, int nk,
                                               const double *__restrict__ y, double *__restrict__ x) {
  double yk[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; ++k) yk[k] = (k < nk) ? y[k] : 0.0;
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
    double s = x[i];
#pragma unroll
    for (int k = 0; k < MAXK; ++k)
      if (k < nk) s += yk[k] * Z[(size_t)k * n + i];
    x[i] = s;
  }
}

__global__ void k_axpby(long n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

int red_blocks(long n) { return (int)std::min<long>(1024, std::max<long>(1, (n + BS - 1) / BS)); }

void ensure_ws(dpp_precond pc, int m) {
  const long n = pc->prob->ndof();
  ensure_reduction(pc);
  if (pc->ws_m >= m && pc->V.ptr) return;
  pc->V.alloc(sizeof(double) * (size_t)(m + 1) * n);
  pc->Z.alloc(sizeof(double) * (size_t)m * n);
  pc->w.alloc(sizeof(double) * n);
  pc->hdev.alloc(sizeof(double) * 4 * (MAXK + 2));
  pc->ydev.alloc(sizeof(double) * (MAXK + 2));
  pc->ws_m = m;
}

}  // namespace

void ensure_reduction(dpp_precond pc) {
  if (!pc->part.ptr) pc->part.alloc(sizeof(double) * (size_t)(MAXK + 2) * 1024);
}

void axpby(long n, double a, const double *x, double b, double *y, hipStream_t s) {
  k_axpby<<<std::min<long>(2048, blocks_for(n, 256)), 256, 0, s>>>(n, a, x, b, y);
  check_launch("axpby");
}

double norm2(const double *x, long n, double *scratch, hipStream_t s) {
  const int nb = red_blocks(n);
  k_mdot<<<nb, BS, 0, s>>>(x, n, 1, x, scratch);
  k_finish<<<1, BS, 0, s>>>(scratch, nb, scratch + (size_t)(MAXK + 1) * 1024);
  check_launch("norm2");
  double h = 0.0;
  DPP_HIP(hipMemcpyAsync(&h, scratch + (size_t)(MAXK + 1) * 1024, sizeof(double),
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
  const int nb = red_blocks(n);
  std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), hh(2 * MAXK + 4), y(m);
  auto Hc = [&](int i, int j) -> double & { return H[(size_t)j * (m + 1) + i]; };
  if (bn == 0.0) {
    DPP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    res.converged = 1;
    return res;
  }
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
    k_scale<<<std::min(2048, blocks_for(n, 256)), 256, 0, s>>>(V, n, 1.0 / beta);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k_used = 0;
    bool breakdown = false;
    for (int j = 0; j < m; ++j) {
      double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
      precond_apply(pc, vj, zj, pre32, s);
      spmv_K(P, zj, w, s, op32);
      const int nk = j + 1;
      {
        // V read three times; w read 3x, written 1x; v_{j+1} written, then read+written
        ProfScope ps(PF_ARNOLDI, 8.0 * n * (3.0 * nk + 7.0), s);
        // pass 1: h1 = V^T w  -> hd[0..nk)
        k_mdot<<<nb, BS, 0, s>>>(V, n, nk, w, part);
        k_finish<<<nk, BS, 0, s>>>(part, nb, hd);
        // pass 2: w -= V h1 ; h2 = V^T w -> hd[MAXK+1 ..], ||w||^2
        k_axpy_mdot<<<nb, BS, 0, s>>>(V, n, nk, hd, w, part);
        k_finish<<<nk + 1, BS, 0, s>>>(part, nb, hd + MAXK + 1);
        // pass 3: v_{j+1} = w - V h2 and its squared norm -> hd[2 MAXK + 3]
        k_axpy_norm<<<nb, BS, 0, s>>>(V, n, nk, hd + MAXK + 1, w, vn, part);
        k_finish<<<1, BS, 0, s>>>(part, nb, hd + 2 * MAXK + 3);
        k_scale_rsqrt<<<std::min(2048, blocks_for(n, 256)), 256, 0, s>>>(vn, n, hd + 2 * MAXK + 3);
      }
      check_launch("arnoldi");
      DPP_HIP(hipMemcpyAsync(hh.data(), hd, sizeof(double) * (2 * MAXK + 4), hipMemcpyDeviceToHost, s));
      DPP_HIP(hipStreamSynchronize(s));
      res.iters++;
      for (int i = 0; i < nk; ++i) Hc(i, j) = hh[i] + hh[MAXK + 1 + i];
      const double hn = std::sqrt(std::max(0.0, hh[2 * MAXK + 3]));
      Hc(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
        Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
        Hc(i, j) = t;
      }
      const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
      if (!std::isfinite(den)) {
        res.status = DPP_ERR_NUMERIC;
        return res;
      }
      if (den == 0.0) {  // singular Hessenberg: no progress possible
        breakdown = true;
        break;
      }
      cs[j] = Hc(j, j) / den;
      sn[j] = Hc(j + 1, j) / den;
      Hc(j, j) = den;
      Hc(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k_used = j + 1;
      if (std::fabs(g[j + 1]) <= rtol * bn || res.iters >= maxiter) break;
      if (hn <= 1e-300) {  // exact (happy) breakdown: the solution lies in the space
        breakdown = true;
        break;
      }
    }
    if (k_used > 0) {
      for (int i = k_used - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < k_used; ++l) t -= Hc(i, l) * y[l];
        y[i] = t / Hc(i, i);
      }
      DPP_HIP(hipMemcpyAsync(pc->ydev.ptr, y.data(), sizeof(double) * k_used, hipMemcpyHostToDevice, s));
      k_update<<<nb, BS, 0, s>>>(Z, n, k_used, pc->ydev.as<double>(), x);
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
