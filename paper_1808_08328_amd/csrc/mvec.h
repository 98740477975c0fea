// Multi-vector streaming primitives of the Arnoldi process (classical
// Gram-Schmidt passes, norms, solution update), shared by the single-instance
// and the batched Krylov kernels.
//
// The number of basis vectors nk is a runtime value; each primitive is
// instantiated for a bucket NKP >= nk so that all loads of one element are
// unconditional and can be in flight together (a load behind a runtime
// `k < nk` branch would wait for the one before it).  Rows k >= nk read row
// nk - 1 again (a cache hit) and carry a zero coefficient or a discarded sum.
// Small buckets also unroll the element loop so every wave keeps several
// loads outstanding.
#pragma once

#include "common.h"

namespace dpp {

constexpr int MV_BS = 256;   // threads per block of every multi-vector kernel
constexpr int MV_MAXK = 32;  // largest bucket (restart length <= 31)
// Rows of the per-block partial-sum buffers: DCGS2 pass A reduces 2 nj + 1
// values (nj <= MV_MAXK - 1), the other kernels at most MV_MAXK + 1.
constexpr int MV_PART_ROWS = 2 * MV_MAXK + 2;

// 16-byte loads and stores of two consecutive doubles (the DCGS2 passes
// stream element pairs: every vector starts 16-byte aligned and has even
// length, (2d + 2) N unknowns per instance; an odd tail is still handled).
__device__ inline double2 mv_ld2(const double *p) {
  double2 t;
  __builtin_memcpy(&t, p, sizeof(t));
  return t;
}
__device__ inline void mv_st2(double *p, double v0, double v1) {
  const double2 t = {v0, v1};
  __builtin_memcpy(p, &t, sizeof(t));
}

template <int NKP>
constexpr int mv_unroll() {
  return NKP <= 2 ? 4 : (NKP <= 4 ? 2 : 1);
}

// Loads the first nk of a coefficient vector, zero beyond.
template <int NKP>
__device__ inline void mv_coefs(const double *__restrict__ c, int nk, double (&out)[NKP]) {
#pragma unroll
  for (int k = 0; k < NKP; ++k) out[k] = (k < nk) ? c[k] : 0.0;
}

__device__ inline double mv_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// acc[k] += sum_i V_k[i] w[i] over i = i0, i0 + stride, ... < n.
template <int NKP>
__device__ inline void mv_dot(const double *__restrict__ V, long ldv, int nk,
                              const double *__restrict__ w, long i0, long n, long stride,
                              double (&acc)[NKP]) {
  constexpr int U = mv_unroll<NKP>();
  long i = i0;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    double wv[U], vv[U][NKP];
#pragma unroll
    for (int u = 0; u < U; ++u) wv[u] = w[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NKP; ++k) vv[u][k] = V[(size_t)min(k, nk - 1) * ldv + i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NKP; ++k) acc[k] += vv[u][k] * wv[u];
  }
  for (; i < n; i += stride) {
    const double wi = w[i];
    double vv[NKP];
#pragma unroll
    for (int k = 0; k < NKP; ++k) vv[k] = V[(size_t)min(k, nk - 1) * ldv + i];
#pragma unroll
    for (int k = 0; k < NKP; ++k) acc[k] += vv[k] * wi;
  }
}

// s = w[i] - sum_k h[k] V_k[i]; then w[i] = s (or out[i] = s), nrm += s^2 and,
// when DOT, acc[k] += V_k[i] s.  h[k] = 0 for k >= nk.
template <int NKP, bool DOT>
__device__ inline void mv_axpy(const double *__restrict__ V, long ldv, int nk,
                               const double (&h)[NKP], const double *w, double *out, long i0,
                               long n, long stride, double (&acc)[NKP], double &nrm) {
  constexpr int U = mv_unroll<NKP>();
  long i = i0;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    double s[U], vv[U][NKP];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = w[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NKP; ++k) vv[u][k] = V[(size_t)min(k, nk - 1) * ldv + i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int k = 0; k < NKP; ++k) s[u] -= h[k] * vv[u][k];
      out[i + u * stride] = s[u];
      nrm += s[u] * s[u];
      if constexpr (DOT) {
#pragma unroll
        for (int k = 0; k < NKP; ++k) acc[k] += vv[u][k] * s[u];
      }
    }
  }
  for (; i < n; i += stride) {
    double s = w[i], vv[NKP];
#pragma unroll
    for (int k = 0; k < NKP; ++k) vv[k] = V[(size_t)min(k, nk - 1) * ldv + i];
#pragma unroll
    for (int k = 0; k < NKP; ++k) s -= h[k] * vv[k];
    out[i] = s;
    nrm += s * s;
    if constexpr (DOT) {
#pragma unroll
      for (int k = 0; k < NKP; ++k) acc[k] += vv[k] * s;
    }
  }
}

// x[i] += sum_k y[k] Z_k[i]  (y[k] = 0 for k >= nk)
template <int NKP>
__device__ inline void mv_update(const double *__restrict__ Z, long ldz, int nk,
                                 const double (&y)[NKP], double *__restrict__ x, long i0, long n,
                                 long stride) {
  constexpr int U = mv_unroll<NKP>();
  long i = i0;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    double s[U], zz[U][NKP];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = x[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NKP; ++k) zz[u][k] = Z[(size_t)min(k, nk - 1) * ldz + i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int k = 0; k < NKP; ++k) s[u] += y[k] * zz[u][k];
      x[i + u * stride] = s[u];
    }
  }
  for (; i < n; i += stride) {
    double s = x[i];
#pragma unroll
    for (int k = 0; k < NKP; ++k) s += y[k] * Z[(size_t)min(k, nk - 1) * ldz + i];
    x[i] = s;
  }
}

// Pass A of DCGS2 with the basis rows split over the block's waves: every
// wave streams the same 64 elements per step (t and w: one HBM read, the
// other waves hit in cache) and its own KG = NKP/4 rows, so each thread keeps
// 2 KG accumulators.  Partial row k < nj: V_k . t, row nj + k: V_k . w, row 2nj:
// t . w, one value per block (written by the owning wave, no block reduction).
// Element pair p (elements 2p, 2p + 1) runs over i0 + lane, + stride, ...
// (i0, stride multiples of 64, in pairs).
template <int NKP>
__device__ inline void mv_dcgs_a_waves(const double *__restrict__ V, long ldv, int nj,
                                       const double *__restrict__ t, const double *__restrict__ w,
                                       long i0, long n, long stride, double *__restrict__ part,
                                       long tb, long bid) {
  constexpr int KG = (NKP + MV_BS / 64 - 1) / (MV_BS / 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k0 = wv * KG;
  const int last = nj > 0 ? nj - 1 : 0;
  const double *rows[KG];
#pragma unroll
  for (int kk = 0; kk < KG; ++kk) rows[kk] = V + (size_t)min(k0 + kk, last) * ldv;
  double aa[KG], bb[KG], tw = 0.0;
#pragma unroll
  for (int kk = 0; kk < KG; ++kk) aa[kk] = bb[kk] = 0.0;
  // element pairs (2p, 2p + 1), p = i0 + lane, + stride, ...
  for (long p = i0 + lane; 2 * p + 1 < n; p += stride) {
    const double2 ti = mv_ld2(t + 2 * p), wi = mv_ld2(w + 2 * p);
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      const double2 v = mv_ld2(rows[kk] + 2 * p);
      aa[kk] += v.x * ti.x + v.y * ti.y;
      bb[kk] += v.x * wi.x + v.y * wi.y;
    }
    tw += ti.x * wi.x + ti.y * wi.y;
  }
  if ((n & 1) && i0 + lane == 0) {  // odd tail: the block's first lane
    const long i = n - 1;
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      aa[kk] += rows[kk][i] * t[i];
      bb[kk] += rows[kk][i] * w[i];
    }
    tw += t[i] * w[i];
  }
#pragma unroll
  for (int kk = 0; kk < KG; ++kk) {
    const double sa = mv_wave_sum(aa[kk]), sb = mv_wave_sum(bb[kk]);
    if (lane == 0 && k0 + kk < nj) {
      part[(size_t)(k0 + kk) * tb + bid] = sa;
      part[(size_t)(nj + k0 + kk) * tb + bid] = sb;
    }
  }
  if (wv == 0) {
    const double st = mv_wave_sum(tw);
    if (lane == 0) part[(size_t)(2 * nj) * tb + bid] = st;
  }
}

// Pass B of DCGS2: with per-row coefficients a, b (zero for k >= nj),
//   v = (t - sum_k a_k V_k) * inv      (written back over t when nj > 0)
//   w' = w - sum_k b_k V_k - hjj v     (written to wout),  nrm += w'^2.
template <int NKP>
__device__ inline void mv_dcgs_update(const double *__restrict__ V, long ldv, int nj,
                                      const double (&a)[NKP], const double (&b)[NKP], double inv,
                                      double hjj, double *__restrict__ t,
                                      const double *__restrict__ w, double *__restrict__ wout,
                                      long i0, long n, long stride, double &nrm) {
  const int last = nj > 0 ? nj - 1 : 0;
  // element pairs (2p, 2p + 1), p = i0, + stride, ...
  for (long p = i0; 2 * p + 1 < n; p += stride) {
    const long i = 2 * p;
    const double2 ti = mv_ld2(t + i), wi = mv_ld2(w + i);
    double2 vv[NKP];
#pragma unroll
    for (int k = 0; k < NKP; ++k) vv[k] = mv_ld2(V + (size_t)min(k, last) * ldv + i);
    double sa0 = 0.0, sb0 = 0.0, sa1 = 0.0, sb1 = 0.0;
#pragma unroll
    for (int k = 0; k < NKP; ++k) {
      sa0 += a[k] * vv[k].x;
      sb0 += b[k] * vv[k].x;
      sa1 += a[k] * vv[k].y;
      sb1 += b[k] * vv[k].y;
    }
    const double v0 = (ti.x - sa0) * inv, v1 = (ti.y - sa1) * inv;
    const double w0 = wi.x - sb0 - hjj * v0, w1 = wi.y - sb1 - hjj * v1;
    if (nj > 0) mv_st2(t + i, v0, v1);
    mv_st2(wout + i, w0, w1);
    nrm += w0 * w0 + w1 * w1;
  }
  if ((n & 1) && i0 == 0) {  // odd tail: the first thread
    const long i = n - 1;
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int k = 0; k < NKP; ++k) {
      const double vk = V[(size_t)min(k, last) * ldv + i];
      sa += a[k] * vk;
      sb += b[k] * vk;
    }
    const double v = (t[i] - sa) * inv;
    const double wp = w[i] - sb - hjj * v;
    if (nj > 0) t[i] = v;
    wout[i] = wp;
    nrm += wp * wp;
  }
}

// DCGS2 coefficients from the reduced sums h = [a (nj) | b (nj) | t.w] and
// alpha = ||t||^2: rho^2 = alpha - |a|^2 (t's norm after removing its
// components along V), hjj = (t.w - a.b) / rho (the new vector's coefficient
// of w).  nj = 0: t is already the normalised first vector (rho = 1).
template <int NKP>
__device__ inline void mv_dcgs_coefs(const double *__restrict__ h, double alpha, int nj,
                                     double (&a)[NKP], double (&b)[NKP], double &rho, double &inv,
                                     double &hjj) {
  mv_coefs<NKP>(h, nj, a);
  mv_coefs<NKP>(h + nj, nj, b);
  const double tw = h[2 * nj];
  if (nj == 0) {
    rho = 1.0;
    inv = 1.0;
    hjj = tw;
    return;
  }
  double r2 = alpha, ab = 0.0;
#pragma unroll
  for (int k = 0; k < NKP; ++k) {
    r2 -= a[k] * a[k];
    ab += a[k] * b[k];
  }
  rho = r2 > 0.0 ? sqrt(r2) : 0.0;
  inv = rho > 0.0 ? 1.0 / rho : 0.0;
  hjj = rho > 0.0 ? (tw - ab) / rho : 0.0;
}

// Block-reduce acc[0..nk) (and `extra` when with_extra) into per-block
// partials: part[k * tb + bid] for k < nk, the extra value in row nk.
template <int NKP>
__device__ inline void mv_block_store(const double (&acc)[NKP], int nk, double extra,
                                      bool with_extra, double *__restrict__ part, long tb,
                                      long bid) {
  __shared__ double sh[MV_BS / 64][NKP + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (nk > 0) {
    double v[NKP];
#pragma unroll
    for (int k = 0; k < NKP; ++k) v[k] = mv_wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NKP; ++k) sh[wv][k] = v[k];
    }
  }
  if (with_extra) {
    const double v = mv_wave_sum(extra);
    if (lane == 0) sh[wv][NKP] = v;
  }
  __syncthreads();
  const int tot = nk + (with_extra ? 1 : 0);
  if ((int)threadIdx.x < tot) {
    const int slot = ((int)threadIdx.x == nk) ? NKP : (int)threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < MV_BS / 64; ++w) s += sh[w][slot];
    part[(size_t)threadIdx.x * tb + bid] = s;
  }
}

}  // namespace dpp

// Dispatch a runtime basis count onto its bucket NKP.
#define DPP_NK_SWITCH(nk, ...)                                                     \
  do {                                                                             \
    const int nk_sw_ = (nk);                                                       \
    if (nk_sw_ <= 1) { constexpr int NKP = 1; __VA_ARGS__; }                       \
    else if (nk_sw_ <= 2) { constexpr int NKP = 2; __VA_ARGS__; }                  \
    else if (nk_sw_ <= 4) { constexpr int NKP = 4; __VA_ARGS__; }                  \
    else if (nk_sw_ <= 6) { constexpr int NKP = 6; __VA_ARGS__; }                  \
    else if (nk_sw_ <= 8) { constexpr int NKP = 8; __VA_ARGS__; }                  \
    else if (nk_sw_ <= 12) { constexpr int NKP = 12; __VA_ARGS__; }                \
    else if (nk_sw_ <= 16) { constexpr int NKP = 16; __VA_ARGS__; }                \
    else if (nk_sw_ <= 20) { constexpr int NKP = 20; __VA_ARGS__; }                \
    else if (nk_sw_ <= 24) { constexpr int NKP = 24; __VA_ARGS__; }                \
    else if (nk_sw_ <= 28) { constexpr int NKP = 28; __VA_ARGS__; }                \
    else { constexpr int NKP = 32; __VA_ARGS__; }                                  \
  } while (0)
