// Internal definitions of the DPP library: errors, the structured box, the
// stencil tables of the node-pair storage of K and of the pressure operators.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dpp.h"

// fixed scratch of the allocation-free entry point, per GPU, and the largest
// device index it keeps an address for
constexpr size_t NOALLOC_SCRATCH_BYTES = DPP_NOALLOC_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;

namespace dpp {

// Template tag of the stencil code: D = 2, 3 for the Kuhn simplices with P1
// elements, D = 12, 13 for box cells (quadrilaterals, hexahedra) with Q1
// elements -- the [P1 + P1]^2 and [Q1 + Q1]^2 rows of the paper's element
// table for CG-VMS.  dim_of(D) is the spatial dimension.
__host__ __device__ constexpr int dim_of(int D) { return D % 10; }
__host__ __device__ constexpr bool is_q1(int D) { return D >= 10; }
// ELEM_DG: the DG-VMS form, discontinuous P1 on the Kuhn simplices (its own
// element-block storage, not the stencil code)
enum Elem { ELEM_P1 = 0, ELEM_Q1 = 1, ELEM_DG = 2 };

struct Error : std::runtime_error {
  dpp_status status;
  Error(dpp_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define DPP_HIP(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::dpp::Error(e_ == hipErrorOutOfMemory ? DPP_ERR_ALLOC : DPP_ERR_HIP,  \
                         std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define DPP_CHECK(cond, status, msg)              \
  do {                                            \
    if (!(cond)) throw ::dpp::Error(status, msg); \
  } while (0)

inline void check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(DPP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- grid ----
// Structured box: m[a] = n[a] + 1 nodes per axis (axis 2 unused in 2D:
// n = 0, m = 1).
struct Grid {
  int dim = 3;
  int elem = ELEM_P1;  // element family (ELEM_P1: Kuhn simplices, ELEM_Q1: box cells)
  int n[3] = {1, 1, 0};
  int m[3] = {2, 2, 1};
  double h[3] = {1, 1, 1};
  long N = 0;   // nodes
  long nc = 0;  // cells (simplices, or boxes with Q1)
  // velocity (flux) faces of network q: bit 2a + s set when face s (0: x_a = 0,
  // 1: x_a = L_a) prescribes the normal velocity (finest grid only)
  int fix[2] = {0, 0};
};

inline Grid make_grid(int dim, const int *n, const double *L, int elem = ELEM_P1) {
  Grid g;
  g.dim = dim;
  g.elem = elem;
  g.N = 1;
  g.nc = elem == ELEM_Q1 ? 1 : (dim == 3) ? 6 : 2;
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      g.n[a] = n[a];
      g.m[a] = n[a] + 1;
      g.h[a] = (L ? L[a] : 1.0) / n[a];
      g.N *= g.m[a];
      g.nc *= n[a];
    } else {
      g.n[a] = 0;
      g.m[a] = 1;
      g.h[a] = 1.0;
    }
  }
  return g;
}

// Coarse box of the multigrid hierarchy: ceil(n/2) cells per axis.
inline Grid coarse_grid(const Grid &f) {
  Grid g = f;
  g.N = 1;
  g.fix[0] = g.fix[1] = 0;
  for (int a = 0; a < f.dim; ++a) {
    g.n[a] = (f.n[a] + 1) / 2;
    g.m[a] = g.n[a] + 1;
    g.N *= g.m[a];
  }
  return g;
}

// Leading dimension of the structure-of-arrays operator storage: every
// offset's value stream starts on a 256-byte boundary (no partial cache
// lines at the stream ends).
inline long padded(long N) { return (N + 31) / 32 * 32; }

struct GridDev {
  int n[3];
  int m[3];
  long N;
  long ld;
  int fix[2];
};
inline GridDev dev(const Grid &g) {
  return GridDev{{g.n[0], g.n[1], g.n[2]}, {g.m[0], g.m[1], g.m[2]}, g.N, padded(g.N),
                 {g.fix[0], g.fix[1]}};
}

// Velocity component c of the node with indices ijk is prescribed for
// network q: the node lies on a velocity face of q whose normal is axis c.
__host__ __device__ inline bool u_fixed(const GridDev &g, int q, int c, const int *ijk) {
  const int bits = g.fix[q] >> (2 * c);
  return ((bits & 1) && ijk[c] == 0) || ((bits & 2) && ijk[c] == g.n[c]);
}

// ---------------------------------------------------------- stencils ----
// Boundary class of a node: per axis 0 (first node), 1 (interior) or 2 (last
// node); class = cx + 3 cy (+ 9 cz).
__host__ __device__ inline int axis_class(int i, int n) { return i == 0 ? 0 : (i == n ? 2 : 1); }
// K couples node a with node a + o for o in the node stencil St.  With P1 on
// the Kuhn simplices: 0 and +-every nonzero binary vector (15 offsets in 3D, 7
// in 2D); with Q1 on box cells: the full 3 x 3 (x 3) box of offsets (27, 9).
// The pressure operators (selfp Schur blocks and every Galerkin coarse level)
// share the stencil T = St - St (components in [-2, 2]: 65 and 19 offsets for
// P1, the full 5 x 5 (x 5) box, 125 and 25, for Q1).  Both lists are ordered
// by (dz, dy, dx), i.e. by linear node offset, so valid neighbours of a node
// come out in ascending node id.
template <int D>
struct Tabs {
  static constexpr int NS = is_q1(D) ? (dim_of(D) == 3 ? 27 : 9) : (dim_of(D) == 3 ? 15 : 7);
  static constexpr int NT = is_q1(D) ? (dim_of(D) == 3 ? 125 : 25) : (dim_of(D) == 3 ? 65 : 19);
  int so[NS][3];
  int to[NT][3];
  int sidx[27];   // (dx+1) + 3(dy+1) + 9(dz+1) -> index in St or -1
  int tidx[125];  // (dx+2) + 5(dy+2) + 25(dz+2) -> index in T or -1
  int s0;         // index of the zero offset in St
  int t0;         // index of the zero offset in T
};

constexpr bool in_st(int dx, int dy, int dz) {
  bool pos = dx >= 0 && dy >= 0 && dz >= 0 && dx <= 1 && dy <= 1 && dz <= 1;
  bool neg = dx <= 0 && dy <= 0 && dz <= 0 && dx >= -1 && dy >= -1 && dz >= -1;
  return pos || neg;
}

// membership of St for the element family of tag D
template <int D>
constexpr bool st_member(int dx, int dy, int dz) {
  const bool box = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
  return (is_q1(D) ? box : in_st(dx, dy, dz)) && (dim_of(D) == 3 || dz == 0);
}

template <int D>
constexpr Tabs<D> make_tabs() {
  Tabs<D> t{};
  const int zr = (dim_of(D) == 3) ? 1 : 0;
  int k = 0;
  for (int i = 0; i < 27; ++i) t.sidx[i] = -1;
  for (int i = 0; i < 125; ++i) t.tidx[i] = -1;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx)
        if (st_member<D>(dx, dy, dz)) {
          t.so[k][0] = dx;
          t.so[k][1] = dy;
          t.so[k][2] = dz;
          if (dx == 0 && dy == 0 && dz == 0) t.s0 = k;
          t.sidx[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] = k;
          ++k;
        }
  int q = 0;
  const int z2 = (dim_of(D) == 3) ? 2 : 0;
  for (int dz = -z2; dz <= z2; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        bool any = false;
        for (int s = 0; s < Tabs<D>::NS; ++s) {
          int ex = dx + t.so[s][0], ey = dy + t.so[s][1], ez = dz + t.so[s][2];
          // t = s1 - s2 with s1 = t + s2 in St
          if (st_member<D>(ex, ey, ez)) any = true;
        }
        if (any) {
          t.to[q][0] = dx;
          t.to[q][1] = dy;
          t.to[q][2] = dz;
          if (dx == 0 && dy == 0 && dz == 0) t.t0 = q;
          t.tidx[(dx + 2) + 5 * (dy + 2) + 25 * (dz + 2)] = q;
          ++q;
        }
      }
  return t;
}

template <int D>
inline constexpr Tabs<D> TAB = make_tabs<D>();

// Number of distinct value kinds stored per (offset, node) of K:
// per network i: kuu (one scalar; the uu block is delta_cc' times it), kup[c],
// kpu[c], kpp; plus k12 (the K12 = K21^T entry).  4d + 5 kinds.
__host__ __device__ constexpr int nv_kinds(int dim) { return 4 * dim + 5; }
__host__ __device__ constexpr int kv_uu(int dim, int net) { return net * (2 * dim + 2); }
__host__ __device__ constexpr int kv_up(int dim, int net, int c) {
  return net * (2 * dim + 2) + 1 + c;
}
__host__ __device__ constexpr int kv_pu(int dim, int net, int c) {
  return net * (2 * dim + 2) + 1 + dim + c;
}
__host__ __device__ constexpr int kv_pp(int dim, int net) { return net * (2 * dim + 2) + 1 + 2 * dim; }
__host__ __device__ constexpr int kv_12(int dim) { return 4 * dim + 4; }

// Half storage of K used by the hot kernels.  D K is symmetric (D = diag(I_u,
// -I_p)): K_uu^i, K_pp^i and K12 are symmetric and K_pu^i = -(K_up^i)^T.  The
// K_up values come from the class table UPT<D> (below), so per node a the
// half storage keeps only the symmetric kinds (kuu0, kuu1, kpp0, kpp1, k12)
// for the zero offset and the positive half of St (t >= s0; NH = NS - s0
// offsets), stream sym(kind, t - s0); for t < s0 the value of (a, a + o_t) is
// the one stored at a + o_t for the mirrored offset (St is sorted by linear
// offset and symmetric, so the mirror of t is NS-1-t).  40 streams in 3D, 20
// in 2D.  The storage is sliced: the values of 64 consecutive nodes form one
// run per stream and the runs of all streams of a slice are contiguous, so a
// wave reads one contiguous block of DRAM pages instead of one page per
// stream.  Streams are ordered by trip h = |t - s0| of the K product (the 5
// kinds of h together), so the values one trip reads from a row sit next to
// each other and share one address register.
template <int D>
struct KH {
  static constexpr int NS = Tabs<D>::NS;
  static constexpr int S0 = (NS - 1) / 2;
  static constexpr int NH = NS - S0;
  static constexpr int NSYM = 5;
  static constexpr int streams = NSYM * NH;
  // sym kind ids
  static constexpr int UU0 = 0, UU1 = 1, PP0 = 2, PP1 = 3, K12 = 4;
  __host__ __device__ static constexpr int sym(int kind, int h) { return h * NSYM + kind; }
  // element of stream s at node a: structure of arrays with the leading
  // dimension ld = padded(N) of the operator storage, so that the values of
  // two consecutive nodes are adjacent in every stream (paired loads)
  __host__ __device__ static size_t at(int s, long a, long ld) { return (size_t)s * ld + a; }
  __host__ __device__ static size_t size(long N) { return (size_t)streams * padded(N); }
};

// Table of the K_up values by boundary class.  The velocity-pressure
// couplings of the CG-VMS form carry no coefficient: the Galerkin term
// -(div w; p) has none and in the stabilisation -1/2 (mu k^-1 w; (k/mu) grad p)
// the permeabilities cancel (eq. CG_VMS_Weak_form).  On the uniform box the
// value of K_up^i((a, c), a + o_t) is then a sum over the cells around a that
// exist, i.e. a function of (class of a, t, c), the same for both networks
// and bit-identical for every node of a class (the cell sums run in the same
// order).  UPT<D> lays the table out as [class][t][c].
template <int D>
struct UPT {
  static constexpr int d = dim_of(D);
  static constexpr int NS = Tabs<D>::NS;
  static constexpr int NCLS = d == 3 ? 27 : 9;
  static constexpr int size = NCLS * NS * d;
  __host__ __device__ static constexpr int at(int cls, int t, int c) { return (cls * NS + t) * d + c; }
};

template <int D>
constexpr bool kh_layout_ok() {
  for (int t = 0; t < KH<D>::NS; ++t)
    for (int a = 0; a < 3; ++a)
      if (TAB<D>.so[KH<D>::NS - 1 - t][a] != -TAB<D>.so[t][a]) return false;
  return TAB<D>.s0 == KH<D>::S0 && Tabs<D>::NS == KH<D>::NS;
}
static_assert(kh_layout_ok<2>() && kh_layout_ok<3>() && kh_layout_ok<12>() && kh_layout_ok<13>(),
              "St must be symmetric and sorted");

template <int D>
constexpr bool kh_streams_bijective() {
  using L = KH<D>;
  int seen[L::streams] = {};
  for (int k = 0; k < L::NSYM; ++k)
    for (int h = 0; h < L::NH; ++h) seen[L::sym(k, h)] += 1;
  for (int s = 0; s < L::streams; ++s)
    if (seen[s] != 1) return false;
  return true;
}
static_assert(kh_streams_bijective<2>() && kh_streams_bijective<3>() && kh_streams_bijective<12>() &&
                  kh_streams_bijective<13>(),
              "kh streams must be a bijection");

// Field offsets of the ABI vector layout [u1 | p1 | u2 | p2].
__host__ __device__ inline long off_u(int dim, long N, int net) {
  return net ? (long)(dim + 1) * N : 0;
}
__host__ __device__ inline long off_p(int dim, long N, int net) {
  return net ? (long)(2 * dim + 1) * N : (long)dim * N;
}

// Node coordinates from its id.
__device__ inline void node_ijk(const GridDev &g, long a, int &i, int &j, int &k) {
  i = (int)(a % g.m[0]);
  long r = a / g.m[0];
  j = (int)(r % g.m[1]);
  k = (int)(r / g.m[1]);
}

__device__ inline bool inside(const GridDev &g, int i, int j, int k) {
  return i >= 0 && i < g.m[0] && j >= 0 && j < g.m[1] && k >= 0 && k < g.m[2];
}

__device__ inline long lin(const GridDev &g, int dx, int dy, int dz) {
  return (long)dx + (long)g.m[0] * ((long)dy + (long)g.m[1] * dz);
}

// Boundary class (UPT) of the node with indices i, j, k (inside the box).
template <int D>
__device__ inline int node_class(const GridDev &g, int i, int j, int k) {
  const int c = axis_class(i, g.n[0]) + 3 * axis_class(j, g.n[1]);
  return dim_of(D) == 3 ? c + 9 * axis_class(k, g.n[2]) : c;
}

// --------------------------------------------------------- XCD mapping ----
// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2.  The remap gives every XCD one contiguous range of tiles
// so that stencil neighbours mostly share an L2.
__device__ inline int xcd_block(int bid, int nblk) {
  const int nx = 8;
  int per = (nblk + nx - 1) / nx;
  int x = bid % nx, q = bid / nx;
  int full = (nblk % nx == 0) ? nx : nblk % nx;  // XCDs that receive `per` blocks
  int base = (x < full) ? x * per : full * per + (x - full) * (per - 1);
  return base + q;
}

inline int blocks_for(long n, int bs) { return (int)((n + bs - 1) / bs); }

// Runs KCALL with `constexpr int D_` set to the stencil tag of grid g (its
// dimension, plus 10 for Q1 box cells).
#define DPP_TAG_SWITCH(g, KCALL)                                        \
  do {                                                                  \
    switch (((g).elem == ::dpp::ELEM_Q1 ? 10 : 0) + (g).dim) {          \
      case 2: { constexpr int D_ = 2; KCALL; } break;                   \
      case 3: { constexpr int D_ = 3; KCALL; } break;                   \
      case 12: { constexpr int D_ = 12; KCALL; } break;                 \
      default: { constexpr int D_ = 13; KCALL; } break;                 \
    }                                                                   \
  } while (0)

// Column order of workgroups over node blocks [j*bs, (j+1)*bs), j < ceil(N/bs):
// returns order[i] = the node block of workgroup i.  MI355X deals consecutive
// workgroups round-robin to its 8 XCDs, each with its own 4 MB L2.  A stencil
// product that reads values of the nodes a +- o (up to one node plane away)
// finds them in L2 when both nodes are processed on the same XCD, so XCD x
// (workgroups i with i % 8 == x) is given the blocks that start in the x-th
// eighth of a node plane, in plane order.  Bands that hold more blocks than
// their XCD's share pass the surplus to the free places.  plane = N gives one
// contiguous range per XCD.
inline std::vector<int> block_column_order(long N, int bs, long plane) {
  const long nb = (N + bs - 1) / bs;
  std::vector<std::vector<int>> band(8);
  for (long j = 0; j < nb; ++j)
    band[std::min(7L, ((j * bs) % plane) * 8 / plane)].push_back((int)j);
  std::vector<int> order(nb, -1), rest;
  std::vector<size_t> taken(8, 0);
  for (long i = 0; i < nb; ++i) {
    const size_t q = (size_t)(i / 8);
    const std::vector<int> &b = band[i % 8];
    if (q < b.size()) {
      order[i] = b[q];
      taken[i % 8] = q + 1;
    }
  }
  for (int x = 0; x < 8; ++x) rest.insert(rest.end(), band[x].begin() + taken[x], band[x].end());
  size_t k = 0;
  for (long i = 0; i < nb; ++i)
    if (order[i] < 0) {
      DPP_CHECK(k < rest.size(), DPP_ERR_ARG, "internal: workgroup order is not a permutation");
      order[i] = rest[k++];
    }
  DPP_CHECK(k == rest.size(), DPP_ERR_ARG, "internal: workgroup order is not a permutation");
  return order;
}

// Two per-network pointers, passed by value.
template <typename T>
struct P2 {
  T *p[2];
};

}  // namespace dpp
