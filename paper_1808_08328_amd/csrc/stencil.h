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
  // 32-bit node indices (N < 2^31)
  const int N = (int)g.N, ai = (int)a;
  const long ld = g.ld;
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
      const int b = min(max(ai + (int)lin(g, o[0], o[1], o[2]), 0), N - 1);
      acc += (double)Aq[(size_t)t * ld + a] * (double)xq[b];
    }
  } else {
#pragma unroll 8
    for (int hh = 0; hh < (NH + LPR - 1) / LPR; ++hh) {
      const int h = hh * LPR + (LPR == 1 ? 0 : sub);
      if (LPR > 1 && h >= NH) continue;
      const int *o = TAB<D>.to[T0 + h];
      // the linear offset of a stored offset is positive except on grids
      // with fewer than 3 nodes along an axis, where a Q1 offset such as
      // (-2, -2, 1) wraps to a negative one: clamp both ways
      const int lo = (int)lin(g, o[0], o[1], o[2]);
      const int bp = min(max(ai + lo, 0), N - 1);
      acc += (double)Aq[(size_t)h * ld + a] * (double)xq[bp];
      if (h > 0) {
        const int bm = ai - lo;
        const int bc = min(max(bm, 0), N - 1);
        const double v = (double)Aq[(size_t)h * ld + bc] * (double)xq[bc];
        acc += (bm >= 0 && bm < N) ? v : 0.0;
      }
    }
  }
  if constexpr (LPR > 1) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
  }
  return acc;
}

// Two consecutive values with one wide load / store (dword alignment is all
// the wide global accesses need, so odd element indices are fine).
__device__ inline void ld2(const double *p, double &v0, double &v1) {
  double2 t;
  __builtin_memcpy(&t, p, sizeof(t));
  v0 = t.x;
  v1 = t.y;
}
__device__ inline void ld2(const float *p, float &v0, float &v1) {
  float2 t;
  __builtin_memcpy(&t, p, sizeof(t));
  v0 = t.x;
  v1 = t.y;
}
__device__ inline void st2(double *p, double v0, double v1) {
  const double2 t = {v0, v1};
  __builtin_memcpy(p, &t, sizeof(t));
}
__device__ inline void st2(float *p, float v0, float v1) {
  const float2 t = {v0, v1};
  __builtin_memcpy(p, &t, sizeof(t));
}

// Stencil products of rows a and a + 1 (a even) with paired loads: every
// matrix and vector access reads two consecutive values in one 16-byte load
// (8 bytes in FP32), which halves the load instructions, the limit of these
// gather-heavy kernels.  A neighbour pair starting at b = a + o is read from
// c = clamp(b, 0, N - 2) and the lane values are picked by d = b - c: an
// index that falls outside [0, N) only ever meets a stored zero (own rows) or
// is masked (mirror rows).  Row a + 1 may be N (N odd): its result is
// meaningless and must not be stored; all its loads stay inside the arrays.
template <int D, typename TV, typename TX, bool SYM>
__device__ inline void row_product2(const GridDev &g, const TV *__restrict__ Aq,
                                    const TX *__restrict__ xq, long a, double &r0, double &r1) {
  constexpr int NT = Tabs<D>::NT;
  constexpr int T0 = TAB<D>.t0;
  constexpr int NH = NT - T0;
  // 32-bit node indices (N < 2^31) keep the per-offset index arithmetic short
  const int N = (int)g.N, ai = (int)a;
  const long ld = g.ld;
  double acc0 = 0.0, acc1 = 0.0;
  if constexpr (!SYM) {
#pragma unroll 8
    for (int t = 0; t < NT; ++t) {
      const int *o = TAB<D>.to[t];
      const int b = ai + (int)lin(g, o[0], o[1], o[2]);
      const int c = min(max(b, 0), N - 2);
      const int d = b - c;
      TV a0, a1;
      TX x0, x1;
      ld2(Aq + (size_t)t * ld + a, a0, a1);
      ld2(xq + c, x0, x1);
      acc0 += (double)a0 * (double)(d > 0 ? x1 : x0);
      acc1 += (double)a1 * (double)(d < 0 ? x0 : x1);
    }
  } else {
#pragma unroll 8
    for (int h = 0; h < NH; ++h) {
      const int *o = TAB<D>.to[T0 + h];
      const int lo = (int)lin(g, o[0], o[1], o[2]);
      const int b = ai + lo;
      // b < 0 only for a wrapped (negative) linear offset, whose pairs leave
      // the box for both rows (stored zeros): the clamp keeps the loads in range
      const int c = min(max(b, 0), N - 2);
      const int d = b - c;
      TV a0, a1;
      TX x0, x1;
      ld2(Aq + (size_t)h * ld + a, a0, a1);
      ld2(xq + c, x0, x1);
      // b >= a >= 0 but for wrapped offsets (both pairs leave the box); b + 1 >= N
      // means row a + 1's pair leaves the box (a1 = 0)
      acc0 += (double)a0 * (double)(d > 0 ? x1 : x0);
      acc1 += (double)a1 * (double)x1;
      if (h > 0) {
        // rows a - o and a + 1 - o hold the negative-half entries
        const int bm = ai - lo;
        const int cm = min(max(bm, 0), N - 2);
        const int dm = bm - cm;
        TV m0, m1;
        TX y0, y1;
        ld2(Aq + (size_t)h * ld + cm, m0, m1);
        ld2(xq + cm, y0, y1);
        const double p0 = (double)m0 * (double)y0, p1 = (double)m1 * (double)y1;
        acc0 += dm == 0 ? p0 : (dm == 1 ? p1 : 0.0);
        acc1 += dm == 0 ? p1 : (dm == -1 ? p0 : 0.0);
      }
    }
  }
  r0 = acc0;
  r1 = acc1;
}

template <int D, bool SYM>
constexpr int stored_offsets() {
  return SYM ? Tabs<D>::NT - TAB<D>.t0 : Tabs<D>::NT;
}

// A x on a level, optionally returning b - A x and/or scaling by dinv.
// FINE only separates the finest-level instances from the coarse-level ones
// (distinct kernel names in profiles); the code is the same.

// y for the 2d+2 unknowns of node a: au[i][c] (velocity rows), ap[i]
// (pressure rows), from the half storage kh of K (symmetric kinds) and the
// K_up class table ut (UPT<D>, staged in LDS by the caller).
//
// One trip per stored offset o = o_{s0+h} (h = 0 .. NH-1) covers the pairs
// (a, a + o) and (a, a - o).  The symmetric values of (a, a - o) are the ones
// node a - o stores for +o: every value read from a neighbour's row is one
// that the neighbour reads as its own in the same trip, so with all waves in
// step those reads hit L2.  K_up((a,c), a +- o) is ut at a's class and
// K_pu(a, (a +- o, c)) = -K_up((a +- o, c), a) is ut at the neighbour's class
// for -+o (zero when the neighbour is outside the box).  Own-row symmetric
// values of pairs that leave the box are stored zeros (the neighbour index is
// clamped, not guarded); neighbour-row values are masked when the neighbour's
// linear index falls outside [0, N) (a wrapped index inside [0, N) reads a
// pair that leaves the box from that node, a stored zero).
template <int D, typename TV, bool BC = false>
__device__ inline void spmv_K_node(const GridDev &g, const TV *__restrict__ kh, const TV *ut,
                                   const double *__restrict__ x, long a, double au[2][dim_of(D)],
                                   double ap[2]) {
  constexpr int d = dim_of(D);
  using L = KH<D>;
  using U = UPT<D>;
  const long N = g.N;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    ap[q] = 0.0;
#pragma unroll
    for (int c = 0; c < d; ++c) au[q][c] = 0.0;
  }
  const long ou[2] = {off_u(d, N, 0), off_u(d, N, 1)};
  const long op[2] = {off_p(d, N, 0), off_p(d, N, 1)};
  // with velocity faces (BC): prescribed velocity components are removed from
  // the columns, here through x (the table and kh hold the unmasked values)
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  const int ca = node_class<D>(g, ia[0], ia[1], ia[2]);
#pragma unroll 1
  for (int h = 0; h < L::NH; ++h) {
    const int tp = L::S0 + h, tn = L::S0 - h;
    const int *o = TAB<D>.so[tp];
    const long lo = lin(g, o[0], o[1], o[2]);
    const long bp = min(a + lo, N - 1);     // a + o (own-row values guard it)
    const long bnr = a - lo;
    const long bn = max(bnr, 0L);           // a - o
    const double mn = (bnr >= 0) ? 1.0 : 0.0;
    // K_up((a,c), a+o), K_up((a,c), a-o), and the neighbours' K_up toward a
    const int pb[3] = {ia[0] + o[0], ia[1] + o[1], ia[2] + o[2]};
    const int nb[3] = {ia[0] - o[0], ia[1] - o[1], ia[2] - o[2]};
    const bool ip = inside(g, pb[0], pb[1], pb[2]), im = inside(g, nb[0], nb[1], nb[2]);
    const int cp = ip ? node_class<D>(g, pb[0], pb[1], pb[2]) : 0;
    const int cm = im ? node_class<D>(g, nb[0], nb[1], nb[2]) : 0;
    double utp[d], utn[d], ptn[d], mtp[d];
#pragma unroll
    for (int c = 0; c < d; ++c) {
      utp[c] = (double)ut[U::at(ca, tp, c)];
      utn[c] = (double)ut[U::at(ca, tn, c)];
      ptn[c] = ip ? (double)ut[U::at(cp, tn, c)] : 0.0;
      mtp[c] = im ? (double)ut[U::at(cm, tp, c)] : 0.0;
    }
    // pair (a, a + o): symmetric kinds own
    double xu[d], xp[2], xo[2];
    const double uu0 = (double)kh[L::at(L::sym(L::UU0, h), a, g.ld)];
    const double uu1 = (double)kh[L::at(L::sym(L::UU1, h), a, g.ld)];
    const double pp0 = (double)kh[L::at(L::sym(L::PP0, h), a, g.ld)];
    const double pp1 = (double)kh[L::at(L::sym(L::PP1, h), a, g.ld)];
    const double s12 = (double)kh[L::at(L::sym(L::K12, h), a, g.ld)];
    xp[0] = x[op[0] + bp];
    xp[1] = x[op[1] + bp];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int c = 0; c < d; ++c) xu[c] = x[ou[q] + d * bp + c];
      if constexpr (BC) {
#pragma unroll
        for (int c = 0; c < d; ++c)
          if (u_fixed(g, q, c, pb)) xu[c] = 0.0;
      }
      const double uu = q ? uu1 : uu0, pp = q ? pp1 : pp0;
#pragma unroll
      for (int c = 0; c < d; ++c) {
        au[q][c] += uu * xu[c] + utp[c] * xp[q];
        ap[q] -= ptn[c] * xu[c];
      }
      ap[q] += pp * xp[q];
    }
    ap[0] += s12 * xp[1];
    ap[1] += s12 * xp[0];
    if (h == 0) continue;  // the zero offset has no mirror pair
    // pair (a, a - o): symmetric kinds stored at a - o
    const double vuu0 = mn * (double)kh[L::at(L::sym(L::UU0, h), bn, g.ld)];
    const double vuu1 = mn * (double)kh[L::at(L::sym(L::UU1, h), bn, g.ld)];
    const double vpp0 = mn * (double)kh[L::at(L::sym(L::PP0, h), bn, g.ld)];
    const double vpp1 = mn * (double)kh[L::at(L::sym(L::PP1, h), bn, g.ld)];
    const double v12 = mn * (double)kh[L::at(L::sym(L::K12, h), bn, g.ld)];
    xo[0] = x[op[0] + bn];
    xo[1] = x[op[1] + bn];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int c = 0; c < d; ++c) xu[c] = x[ou[q] + d * bn + c];
      if constexpr (BC) {
#pragma unroll
        for (int c = 0; c < d; ++c)
          if (u_fixed(g, q, c, nb)) xu[c] = 0.0;
      }
      const double uu = q ? vuu1 : vuu0, pp = q ? vpp1 : vpp0;
#pragma unroll
      for (int c = 0; c < d; ++c) {
        au[q][c] += uu * xu[c] + utn[c] * xo[q];
        ap[q] -= mtp[c] * xu[c];
      }
      ap[q] += pp * xo[q];
    }
    ap[0] += v12 * xo[1];
    ap[1] += v12 * xo[0];
  }
}

// spmv_K_node for the two nodes a and a + 1 (a even), with paired loads: the
// half-storage streams hold consecutive nodes next to each other, and the
// unknowns of two consecutive nodes are adjacent in x (2d velocity values, two
// pressures), so every value the product reads comes with one 16-byte load per
// pair of nodes (8 bytes for FP32 streams) instead of two narrow ones; the
// product issues half the load instructions, its limit.  The neighbour pair
// starting at b = a + o (b > a) is read from c = min(b, N - 2) and picked by
// b - c, the mirror pair starting at a - o from max(a - o, 0) and masked when
// it lies before node 0 (as in row_product2).  Node a + 1 may be N (N odd): its
// result is meaningless and must not be stored; all loads stay inside the
// arrays (streams have the leading dimension padded(N) > N for odd N).
// Problems without velocity faces only (their masks stay in spmv_K_node).
template <int D, typename TV>
__device__ inline void spmv_K_node2(const GridDev &g, const TV *__restrict__ kh, const TV *ut,
                                    const double *__restrict__ x, long a,
                                    double au[2][2][dim_of(D)], double ap[2][2]) {
  constexpr int d = dim_of(D);
  using L = KH<D>;
  using U = UPT<D>;
  // 32-bit node and unknown indices (the assembly keeps them below 2^31)
  const int N = (int)g.N, ai = (int)a;
  const long ld = g.ld;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ap[r][q] = 0.0;
#pragma unroll
      for (int c = 0; c < d; ++c) au[r][q][c] = 0.0;
    }
  const int ou[2] = {(int)off_u(d, N, 0), (int)off_u(d, N, 1)};
  const int op[2] = {(int)off_p(d, N, 0), (int)off_p(d, N, 1)};
  int ia[2][3];
  node_ijk(g, a, ia[0][0], ia[0][1], ia[0][2]);
  node_ijk(g, a + 1, ia[1][0], ia[1][1], ia[1][2]);
  const int ca[2] = {node_class<D>(g, ia[0][0], ia[0][1], ia[0][2]),
                     node_class<D>(g, ia[1][0], ia[1][1], ia[1][2])};
#pragma unroll 1
  for (int h = 0; h < L::NH; ++h) {
    const int tp = L::S0 + h, tn = L::S0 - h;
    const int *o = TAB<D>.so[tp];
    const int lo = (int)lin(g, o[0], o[1], o[2]);
    // neighbour classes and the K_up / K_pu table values of both nodes
    double utp[2][d], utn[2][d], ptn[2][d], mtp[2][d];
    int pb[2][3], nb[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        pb[r][e] = ia[r][e] + o[e];
        nb[r][e] = ia[r][e] - o[e];
      }
      const bool ip = inside(g, pb[r][0], pb[r][1], pb[r][2]);
      const bool im = inside(g, nb[r][0], nb[r][1], nb[r][2]);
      const int cp = ip ? node_class<D>(g, pb[r][0], pb[r][1], pb[r][2]) : 0;
      const int cm = im ? node_class<D>(g, nb[r][0], nb[r][1], nb[r][2]) : 0;
#pragma unroll
      for (int c = 0; c < d; ++c) {
        utp[r][c] = (double)ut[U::at(ca[r], tp, c)];
        utn[r][c] = (double)ut[U::at(ca[r], tn, c)];
        ptn[r][c] = ip ? (double)ut[U::at(cp, tn, c)] : 0.0;
        mtp[r][c] = im ? (double)ut[U::at(cm, tp, c)] : 0.0;
      }
    }
    // pairs (a, a + o) and (a + 1, a + 1 + o): symmetric kinds own
    {
      const int b = ai + lo;
      const int c0 = min(b, N - 2);
      const bool sh = b > c0;  // node a's neighbour is lane 1
      TV kv[5][2];
#pragma unroll
      for (int k = 0; k < 5; ++k) ld2(kh + L::at(L::sym(k, h), ai, ld), kv[k][0], kv[k][1]);
      double xp[2][2], xu[2][2][d];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double v0, v1;
        ld2(x + op[q] + c0, v0, v1);
        xp[q][0] = sh ? v1 : v0;
        xp[q][1] = v1;
        double w[2 * d];
#pragma unroll
        for (int e = 0; e < d; ++e) ld2(x + ou[q] + d * c0 + 2 * e, w[2 * e], w[2 * e + 1]);
#pragma unroll
        for (int c = 0; c < d; ++c) {
          xu[0][q][c] = sh ? w[d + c] : w[c];
          xu[1][q][c] = w[d + c];
        }
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const double uu = (double)kv[q ? L::UU1 : L::UU0][r], pp = (double)kv[q ? L::PP1 : L::PP0][r];
#pragma unroll
          for (int c = 0; c < d; ++c) {
            au[r][q][c] += uu * xu[r][q][c] + utp[r][c] * xp[q][r];
            ap[r][q] -= ptn[r][c] * xu[r][q][c];
          }
          ap[r][q] += pp * xp[q][r];
        }
        const double s12 = (double)kv[L::K12][r];
        ap[r][0] += s12 * xp[1][r];
        ap[r][1] += s12 * xp[0][r];
      }
    }
    if (h == 0) continue;  // the zero offset has no mirror pair
    // pairs (a, a - o) and (a + 1, a + 1 - o): symmetric kinds stored at the
    // mirror nodes a - o and a + 1 - o (masked before node 0)
    {
      const int bm = ai - lo;          // <= N - 2
      const int cm = max(bm, 0);
      const int dm = bm - cm;          // 0, or < 0 before node 0
      const double m0 = dm == 0 ? 1.0 : 0.0;
      TV kv[5][2];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        TV w0, w1;
        ld2(kh + L::at(L::sym(k, h), cm, ld), w0, w1);
        kv[k][0] = w0;
        kv[k][1] = dm == 0 ? w1 : (dm == -1 ? w0 : (TV)0);
      }
      double xo[2][2], xu[2][2][d];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double v0, v1;
        ld2(x + op[q] + cm, v0, v1);
        xo[q][0] = v0;
        xo[q][1] = dm == 0 ? v1 : v0;
        double w[2 * d];
#pragma unroll
        for (int e = 0; e < d; ++e) ld2(x + ou[q] + d * cm + 2 * e, w[2 * e], w[2 * e + 1]);
#pragma unroll
        for (int c = 0; c < d; ++c) {
          xu[0][q][c] = w[c];
          xu[1][q][c] = dm == 0 ? w[d + c] : w[c];
        }
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        // node a's mirror exists iff dm == 0; node a + 1's iff dm >= -1
        const double mr = r == 0 ? m0 : (dm >= -1 ? 1.0 : 0.0);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const double uu = mr * (double)kv[q ? L::UU1 : L::UU0][r];
          const double pp = mr * (double)kv[q ? L::PP1 : L::PP0][r];
#pragma unroll
          for (int c = 0; c < d; ++c) {
            au[r][q][c] += uu * xu[r][q][c] + utn[r][c] * xo[q][r];
            ap[r][q] -= mtp[r][c] * xu[r][q][c];
          }
          ap[r][q] += pp * xo[q][r];
        }
        const double v12 = mr * (double)kv[L::K12][r];
        ap[r][0] += v12 * xo[1][r];
        ap[r][1] += v12 * xo[0][r];
      }
    }
  }
}

// rhat_i(b) = r_p_i(b) - sum_t sum_c K_pu^i(b, (b+o_t, c)) dinv_i(b+o_t) r_u_i(b+o_t, c)
// with K_pu^i(b, (a, c)) = -K_up^i((a, c), b), ut at a's class for the mirror
// of t.  With BC the columns of prescribed velocity components are masked.
template <int D, typename TV, bool BC = false>
__device__ inline double schur_rhs_node(const GridDev &g, const TV *ut,
                                        const double *__restrict__ dinv,
                                        const double *__restrict__ r, int q, long b) {
  constexpr int d = dim_of(D);
  using U = UPT<D>;
  constexpr int NS = U::NS;
  // 32-bit node and unknown indices (the assembly keeps them below 2^31)
  const int N = (int)g.N, bi = (int)b;
  const int ou = (int)off_u(d, N, q);
  double acc = r[off_p(d, N, q) + bi];
  int ib[3];
  node_ijk(g, b, ib[0], ib[1], ib[2]);
  // offsets in unrolled groups of 5 (loads of a group in flight together)
#pragma unroll 5
  for (int t = 0; t < NS; ++t) {
    const int *o = TAB<D>.so[t];
    const int a = min(max(bi + (int)lin(g, o[0], o[1], o[2]), 0), N - 1);
    const int pa[3] = {ib[0] + o[0], ib[1] + o[1], ib[2] + o[2]};
    const bool in = inside(g, pa[0], pa[1], pa[2]);
    const int ca = in ? node_class<D>(g, pa[0], pa[1], pa[2]) : 0;
    const double di = in ? dinv[q * N + a] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < d; ++c) {
      double rv = r[ou + d * a + c];
      if constexpr (BC)
        if (u_fixed(g, q, c, pa)) rv = 0.0;
      s += (double)ut[U::at(ca, NS - 1 - t, c)] * rv;
    }
    acc += s * di;
  }
  return acc;
}

// z_u_i(a, c) = dinv_i(a) (r_u_i(a, c) - sum_t K_up^i((a,c), a+o_t) z_p_i(a+o_t)),
// K_up from the class table ut.
template <int D, typename TV, typename TX>
__device__ inline void schur_vel_node(const GridDev &g, const TV *ut,
                                      const double *__restrict__ dinv,
                                      const double *__restrict__ r, const TX *__restrict__ zp,
                                      int q, long a, double out[dim_of(D)]) {
  constexpr int d = dim_of(D);
  using U = UPT<D>;
  const long N = g.N;
  const long ou = off_u(d, N, q);
  int i, j, k;
  node_ijk(g, a, i, j, k);
  const int ca = node_class<D>(g, i, j, k);
#pragma unroll
  for (int c = 0; c < d; ++c) out[c] = r[ou + d * a + c];
#pragma unroll
  for (int t = 0; t < U::NS; ++t) {
    const int *o = TAB<D>.so[t];
    const long b = min(max(a + lin(g, o[0], o[1], o[2]), 0L), N - 1);
    const double zb = (double)zp[q * N + b];
#pragma unroll
    for (int c = 0; c < d; ++c) out[c] -= (double)ut[U::at(ca, t, c)] * zb;
  }
  const double di = dinv[q * N + a];
#pragma unroll
  for (int c = 0; c < d; ++c) out[c] *= di;
}

// schur_vel_node for rows a and a + 1 (a even, a + 1 < N), paired loads.
template <int D, typename TV, typename TX>
__device__ inline void schur_vel_node2(const GridDev &g, const TV *ut,
                                       const double *__restrict__ dinv,
                                       const double *__restrict__ r, const TX *__restrict__ zp,
                                       int q, long a, double out[2 * dim_of(D)]) {
  constexpr int d = dim_of(D);
  using U = UPT<D>;
  // 32-bit node and unknown indices (the assembly keeps them below 2^31)
  const int N = (int)g.N, ai = (int)a;
  const int ou = (int)off_u(d, N, q);
  int i, j, k;
  node_ijk(g, a, i, j, k);
  const int c0 = node_class<D>(g, i, j, k);
  node_ijk(g, a + 1, i, j, k);
  const int c1 = node_class<D>(g, i, j, k);
#pragma unroll
  for (int k2 = 0; k2 < d; ++k2) ld2(r + ou + d * ai + 2 * k2, out[2 * k2], out[2 * k2 + 1]);
#pragma unroll 5
  for (int t = 0; t < U::NS; ++t) {
    const int *o = TAB<D>.so[t];
    const int b = ai + (int)lin(g, o[0], o[1], o[2]);
    const int c = min(max(b, 0), N - 2);
    const int sh = b - c;
    TX z0, z1;
    ld2(zp + q * N + c, z0, z1);
    // the table is zero for pairs that leave the box, so a clamped z is harmless
    const double za = (double)(sh > 0 ? z1 : z0), zb = (double)(sh < 0 ? z0 : z1);
#pragma unroll
    for (int k2 = 0; k2 < d; ++k2) {
      out[k2] -= (double)ut[U::at(c0, t, k2)] * za;
      out[d + k2] -= (double)ut[U::at(c1, t, k2)] * zb;
    }
  }
  double di0, di1;
  ld2(dinv + q * N + ai, di0, di1);
#pragma unroll
  for (int k2 = 0; k2 < d; ++k2) {
    out[k2] *= di0;
    out[d + k2] *= di1;
  }
}

// Fine nodes f of one axis that coarse index c interpolates to (P(f, c) != 0)
// and their weights: the fine node at c's place (1), and the odd fine nodes
// beside it (1/2) -- at most 3.  Unused axes (n = 0) give the single node 0.
__device__ inline int axis_support(int c, int n, int mc, int *f, double *w) {
  int k = 0;
  f[k] = exact_fine(c, n, mc);
  w[k++] = 1.0;
  if (2 * c + 1 <= n - 1) {
    f[k] = 2 * c + 1;
    w[k++] = 0.5;
  }
  if (2 * c - 1 >= 1 && 2 * c - 1 <= n - 1) {
    f[k] = 2 * c - 1;
    w[k++] = 0.5;
  }
  return k;
}

// b_c(C) = sum_f P(f, C) r(f) for one coarse node (one network's slice rq).
// P1 (Kuhn simplices): a fine node with odd indices on the axes O lies on the
// Kuhn edge between lo and lo + 1_O and takes half of each; Q1 (box cells):
// the tensor product of the axes' linear interpolation.
template <int D, typename TX>
__device__ inline double restrict_node(const GridDev &gf, const GridDev &gc,
                                       const TX *__restrict__ rq, long C) {
  int cc[3];
  node_ijk(gc, C, cc[0], cc[1], cc[2]);
  if constexpr (is_q1(D)) {
    int f[3][3], k[3];
    double w[3][3];
    for (int ax = 0; ax < 3; ++ax) k[ax] = axis_support(cc[ax], gf.n[ax], gc.m[ax], f[ax], w[ax]);
    double acc = 0.0;
    for (int z = 0; z < k[2]; ++z)
      for (int y = 0; y < k[1]; ++y) {
        const int row = gf.m[0] * (f[1][y] + gf.m[1] * f[2][z]);  // < 2^31
        double s = 0.0;
        for (int x = 0; x < k[0]; ++x) s += w[0][x] * (double)rq[f[0][x] + row];
        acc += w[2][z] * w[1][y] * s;
      }
    return acc;
  }
  int ex[3];
  for (int ax = 0; ax < 3; ++ax) ex[ax] = exact_fine(cc[ax], gf.n[ax], gc.m[ax]);
  auto fid = [&](const int *f) { return f[0] + gf.m[0] * (f[1] + gf.m[1] * f[2]); };  // < 2^31
  double acc = (double)rq[fid(ex)];
  for (int mask = 1; mask < (1 << dim_of(D)); ++mask) {
    int fu[3] = {ex[0], ex[1], ex[2]}, fd[3] = {ex[0], ex[1], ex[2]};
    bool uok = true, dok = true;
    for (int ax = 0; ax < dim_of(D); ++ax) {
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
  if constexpr (is_q1(D)) {
    // tensor product: half of each end on every axis where f is odd
    double v = 0.0;
    for (int z = 0; z <= od[2]; ++z)
      for (int y = 0; y <= od[1]; ++y)
        for (int x = 0; x <= od[0]; ++x)
          v += (double)eq[(lo[0] + x) + gc.m[0] * ((lo[1] + y) + gc.m[1] * (lo[2] + z))];
    return v * (od[0] ? 0.5 : 1.0) * (od[1] ? 0.5 : 1.0) * (od[2] ? 0.5 : 1.0);
  }
  // 32-bit node indices (the assembly keeps every level below 2^31 nodes)
  const int c0 = lo[0] + gc.m[0] * (lo[1] + gc.m[1] * lo[2]);
  double v = (double)eq[c0];
  if (any) {
    const int c1 = (lo[0] + od[0]) + gc.m[0] * ((lo[1] + od[1]) + gc.m[1] * (lo[2] + od[2]));
    v = 0.5 * (v + (double)eq[c1]);
  }
  return v;
}

}  // namespace dpp
