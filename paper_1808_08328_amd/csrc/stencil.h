// Device-side building blocks shared by the single-problem kernels and the
// batched multi-instance kernels: one node's worth of each operator.
#pragma once

#include "common.h"

namespace dpp {

struct Sc2 {
  double v[2];
};

__device__ inline void fine_to_coarse(int i, int n, int mc, int &lo, int &od) {
  if ((n & 1) && i == n) {
    lo = mc - 1;
    od = 0;
  } else {
    lo = i >> 1;
    od = i & 1;
  }
}

__device__ inline int exact_fine(int c, int n, int mc) { return ((n & 1) && c == mc - 1) ? n : 2 * c; }

// Stencil product of one row, split over LPR lanes (offsets t = sub, sub+LPR,
// ...); the lanes of a row are adjacent and reduce with shuffles.  LPR = 1 is
// the fully unrolled one-thread-per-row form used on large levels; smaller
// levels use more lanes per row so the launch still fills the GPU.
//
// SYM: the operators are symmetric, so only the zero offset and the positive
// half of T (linear offset > 0; T is sorted, so these are indices t0..NT-1)
// are stored, H[h][a] = A(a, a + o_{t0+h}); the entries of the negative
// half are read from the neighbour's row, A(a, a - o) = H[h][a - o].  That
// halves the matrix bytes streamed from HBM when the mirror reads hit in L2
// or the Infinity Cache (rows a and a - o are at most two planes apart).
template <int D, typename TV, typename TX, int LPR, bool SYM>
__device__ inline double row_product(const GridDev &g, const TV *__restrict__ Aq,
                                     const TX *__restrict__ xq, long a, int i, int j, int k, int sub) {
  // Entries of pairs that leave the box are stored as zeros, so the loads
  // need no guard: the vector index is clamped into range (the zero entry
  // multiplies a finite value) and only a mirror entry whose row index falls
  // outside [0, N) is masked.  Unguarded loads let every load of the row be
  // in flight at once.
  constexpr int NT = Tabs<D>::NT;
  constexpr int T0 = TAB<D>.t0;
  constexpr int NH = NT - T0;  // zero offset + positive half
  const long N = g.N, ld = g.ld;
  (void)i; (void)j; (void)k;
  double acc = 0.0;
  // Offsets are processed in unrolled groups of 8: each group's loads are
  // issued together without exhausting the register budget.
  if constexpr (!SYM) {
#pragma unroll 8
    for (int tt = 0; tt < (NT + LPR - 1) / LPR; ++tt) {
      const int t = tt * LPR + (LPR == 1 ? 0 : sub);
      if (LPR > 1 && t >= NT) continue;
      const int *o = TAB<D>.to[t];
      const long b = min(max(a + lin(g, o[0], o[1], o[2]), 0L), N - 1);
      acc += (double)Aq[(size_t)t * ld + a] * (double)xq[b];
    }
  } else {
#pragma unroll 8
    for (int hh = 0; hh < (NH + LPR - 1) / LPR; ++hh) {
      const int h = hh * LPR + (LPR == 1 ? 0 : sub);
      if (LPR > 1 && h >= NH) continue;
      const int *o = TAB<D>.to[T0 + h];
      const long lo = lin(g, o[0], o[1], o[2]);
      const long bp = min(a + lo, N - 1);
      acc += (double)Aq[(size_t)h * ld + a] * (double)xq[bp];
      if (h > 0) {
        const long bm = a - lo;
        const long bc = max(bm, 0L);
        const double v = (double)Aq[(size_t)h * ld + bc] * (double)xq[bc];
        acc += (bm >= 0) ? v : 0.0;
      }
    }
  }
  if constexpr (LPR > 1) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
  }
  return acc;
}

template <int D, bool SYM>
constexpr int stored_offsets() {
  return SYM ? Tabs<D>::NT - TAB<D>.t0 : Tabs<D>::NT;
}

// A x on a level, optionally returning b - A x and/or scaling by dinv.
// FINE only separates the finest-level instances from the coarse-level ones
// (distinct kernel names in profiles); the code is the same.

// y for the 2d+2 unknowns of node a: au[i][c] (velocity rows), ap[i]
// (pressure rows), from the node-pair stencil storage of K.  Out-of-box pairs
// hold zeros, so the neighbour index is clamped instead of guarded (all loads
// of an offset can be in flight together).
template <int D, typename TV>
__device__ inline void spmv_K_node(const GridDev &g, const TV *__restrict__ kv,
                                   const double *__restrict__ x, long a, double au[2][D],
                                   double ap[2]) {
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    ap[q] = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) au[q][c] = 0.0;
  }
  const size_t vs = (size_t)NS * g.ld;
  const long ou0 = off_u(D, N, 0), ou1 = off_u(D, N, 1), op0 = off_p(D, N, 0),
             op1 = off_p(D, N, 1);
  // one offset per trip: its 4d+5 value streams and 2d+2 neighbour unknowns
  // are loaded together
#pragma unroll 1
  for (int t = 0; t < NS; ++t) {
    const int *o = TAB<D>.so[t];
    const long b = min(max(a + lin(g, o[0], o[1], o[2]), 0L), N - 1);
    double xu[2][D], xp[2];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      xu[0][c] = x[ou0 + D * b + c];
      xu[1][c] = x[ou1 + D * b + c];
    }
    xp[0] = x[op0 + b];
    xp[1] = x[op1 + b];
    const TV *base = kv + (size_t)t * g.ld + a;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double uu = (double)base[kv_uu(D, q) * vs];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double up = (double)base[kv_up(D, q, c) * vs];
        const double pu = (double)base[kv_pu(D, q, c) * vs];
        au[q][c] += uu * xu[q][c] + up * xp[q];
        ap[q] += pu * xu[q][c];
      }
      ap[q] += (double)base[kv_pp(D, q) * vs] * xp[q];
    }
    const double k12 = (double)base[kv_12(D) * vs];
    ap[0] += k12 * xp[1];
    ap[1] += k12 * xp[0];
  }
}

// rhat_i(b) = r_p_i(b) - sum_t sum_c K_pu^i(b, (b+o_t, c)) dinv_i(b+o_t) r_u_i(b+o_t, c)
template <int D, typename TV>
__device__ inline double schur_rhs_node(const GridDev &g, const TV *__restrict__ kv,
                                        const double *__restrict__ dinv,
                                        const double *__restrict__ r, int q, long b) {
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  const size_t vs = (size_t)NS * g.ld;
  const long ou = off_u(D, N, q);
  double acc = r[off_p(D, N, q) + b];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int *o = TAB<D>.so[t];
    const long a = min(max(b + lin(g, o[0], o[1], o[2]), 0L), N - 1);
    const double di = dinv[q * N + a];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c)
      s += (double)kv[kv_pu(D, q, c) * vs + (size_t)t * g.ld + b] * r[ou + D * a + c];
    acc -= s * di;
  }
  return acc;
}

// z_u_i(a, c) = dinv_i(a) (r_u_i(a, c) - sum_t K_up^i((a,c), a+o_t) z_p_i(a+o_t))
template <int D, typename TV, typename TX>
__device__ inline void schur_vel_node(const GridDev &g, const TV *__restrict__ kv,
                                      const double *__restrict__ dinv,
                                      const double *__restrict__ r, const TX *__restrict__ zp,
                                      int q, long a, double out[D]) {
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  const size_t vs = (size_t)NS * g.ld;
  const long ou = off_u(D, N, q);
#pragma unroll
  for (int c = 0; c < D; ++c) out[c] = r[ou + D * a + c];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int *o = TAB<D>.so[t];
    const long b = min(max(a + lin(g, o[0], o[1], o[2]), 0L), N - 1);
    const double zb = (double)zp[q * N + b];
#pragma unroll
    for (int c = 0; c < D; ++c) out[c] -= (double)kv[kv_up(D, q, c) * vs + (size_t)t * g.ld + a] * zb;
  }
  const double di = dinv[q * N + a];
#pragma unroll
  for (int c = 0; c < D; ++c) out[c] *= di;
}

// b_c(C) = sum_f P(f, C) r(f) for one coarse node (one network's slice rq)
template <int D, typename TX>
__device__ inline double restrict_node(const GridDev &gf, const GridDev &gc,
                                       const TX *__restrict__ rq, long C) {
  int cc[3];
  node_ijk(gc, C, cc[0], cc[1], cc[2]);
  int ex[3];
  for (int ax = 0; ax < 3; ++ax) ex[ax] = exact_fine(cc[ax], gf.n[ax], gc.m[ax]);
  auto fid = [&](const int *f) { return f[0] + (long)gf.m[0] * (f[1] + (long)gf.m[1] * f[2]); };
  double acc = (double)rq[fid(ex)];
  for (int mask = 1; mask < (1 << D); ++mask) {
    int fu[3] = {ex[0], ex[1], ex[2]}, fd[3] = {ex[0], ex[1], ex[2]};
    bool uok = true, dok = true;
    for (int ax = 0; ax < D; ++ax) {
      if (!((mask >> ax) & 1)) continue;
      fu[ax] = 2 * cc[ax] + 1;
      fd[ax] = 2 * cc[ax] - 1;
      uok = uok && fu[ax] <= gf.n[ax] - 1;
      dok = dok && fd[ax] >= 1 && fd[ax] <= gf.n[ax] - 1;
    }
    if (uok) acc += 0.5 * (double)rq[fid(fu)];
    if (dok) acc += 0.5 * (double)rq[fid(fd)];
  }
  return acc;
}

// (P e)(f) for one fine node (one network's coarse slice eq)
template <int D, typename TX>
__device__ inline double prolong_node(const GridDev &gf, const GridDev &gc,
                                      const TX *__restrict__ eq, long f) {
  int fi[3];
  node_ijk(gf, f, fi[0], fi[1], fi[2]);
  int lo[3], od[3];
  bool any = false;
  for (int ax = 0; ax < 3; ++ax) {
    fine_to_coarse(fi[ax], gf.n[ax], gc.m[ax], lo[ax], od[ax]);
    any = any || od[ax];
  }
  const long c0 = lo[0] + (long)gc.m[0] * (lo[1] + (long)gc.m[1] * lo[2]);
  double v = (double)eq[c0];
  if (any) {
    const long c1 = (lo[0] + od[0]) + (long)gc.m[0] * ((lo[1] + od[1]) + (long)gc.m[1] * (lo[2] + od[2]));
    v = 0.5 * (v + (double)eq[c1]);
  }
  return v;
}

}  // namespace dpp
