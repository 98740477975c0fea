// DG-VMS on the Kuhn simplices: assembly, operator products and CSR export.
//
// The discontinuous Galerkin form of section "Stabilized mixed discontinuous
// Galerkin formulation (DG-VMS)" (eq. VMS_DG_Weak_Form; block entries eq.
// S4_dg_stiffness_matrix; right-hand side eq. S4_dg_rhs) with discontinuous
// P1 for u1, p1, u2, p2.  Every simplex e owns its d + 1 vertex slots; the
// unknown vector is [u1 | p1 | u2 | p2] over slots, so the unknowns of one
// simplex are contiguous within each field: u at off_u + e (d+1) d + l (l <
// (d+1) d, vertex-major, components interleaved), p at off_p + e (d+1) + v.
//
// Storage: per network q and simplex e, one dense block per coupled simplex,
// SB = (d+1)^2 local unknowns square (16 x 16 in 3D): block 0 couples e with
// itself (volume terms and the own-own facet terms), block 1 + k with the
// neighbour across the facet opposite local vertex k (own-neighbour facet
// terms; zero when the facet is on the boundary), plus one (d+1) x (d+1)
// block per simplex for the inter-network transfer -(beta/mu)(q1; p2).
// Every thread computes the rows of its own simplex, so assembly needs no
// atomics, and the row of one unknown in a block is SB contiguous values.
//
// Facet neighbours follow the Freudenthal (Kuhn) adjacency: the simplex of
// corner c and axis permutation pi has the vertices v_0 = c, v_k = v_(k-1) +
// e_(pi(k-1)); across the facet opposite v_0 lies (c + e_(pi(0)), pi rotated
// left), across the facet opposite v_d lies (c - e_(pi(d-1)), pi rotated
// right), and across the facet opposite v_k (0 < k < d) lies (c, pi with
// entries k-1 and k swapped).
#include <vector>

#include "objects.h"
#include "profile.h"
#include "stencil.h"

namespace dpp {

namespace {

constexpr double ETA_U = 10.0;  // velocity-jump penalty (data tables)
constexpr double ETA_P = 10.0;  // pressure-jump penalty

__host__ __device__ constexpr int dg_nper(int d) { return d == 3 ? 6 : 2; }
__host__ __device__ constexpr int dg_sb(int d) { return (d + 1) * (d + 1); }

// permutations of the axes in lexicographic order (the simplex index within
// its box, as in the numbering spec)
__device__ inline void dg_perm(int d, int s, int *p) {
  if (d == 2) {
    p[0] = s;
    p[1] = 1 - s;
    return;
  }
  const int P3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int a = 0; a < 3; ++a) p[a] = P3[s][a];
}
__device__ inline int dg_perm_index(int d, const int *p) {
  if (d == 2) return p[0];
  // lexicographic rank of a permutation of {0, 1, 2}
  const int first = p[0];
  const int second_rank = p[1] > p[2] ? 1 : 0;
  return 2 * first + second_rank;
}

// Geometry of simplex e: box cell indices, permutation, local vertex node
// ids, barycentric gradients G[v][c], volume, and its facet neighbours with
// the vertex maps.
struct DGSimplex {
  int cell[3];
  int perm[3];
  long node[4];
  double G[4][3];
  double vol;
  long nb[4];        // neighbour across the facet opposite local vertex k, -1 on the boundary
  int map[4][4];     // map[k][v]: the neighbour's local index of own vertex v (v != k)
};

template <int d>
__device__ inline void dg_simplex(const GridDev &g, const double *h, long e, DGSimplex &S) {
  constexpr int NP = dg_nper(d);
  const long box = e / NP;
  const int s = (int)(e % NP);
  long r = box;
  for (int a = 0; a < d; ++a) {
    S.cell[a] = (int)(r % g.n[a]);
    r /= g.n[a];
  }
  dg_perm(d, s, S.perm);
  const long stride[3] = {1, g.m[0], (long)g.m[0] * g.m[1]};
  long c0 = 0;
  for (int a = 0; a < d; ++a) c0 += (long)S.cell[a] * stride[a];
  S.node[0] = c0;
  for (int k = 1; k <= d; ++k) S.node[k] = S.node[k - 1] + stride[S.perm[k - 1]];
  // phi_0 = 1 - t_pi0, phi_k = t_pi(k-1) - t_pi(k), phi_d = t_pi(d-1), t_a = (x_a - c_a)/h_a
  for (int v = 0; v <= d; ++v)
    for (int c = 0; c < d; ++c) S.G[v][c] = 0.0;
  S.G[0][S.perm[0]] = -1.0 / h[S.perm[0]];
  for (int k = 1; k < d; ++k) {
    S.G[k][S.perm[k - 1]] = 1.0 / h[S.perm[k - 1]];
    S.G[k][S.perm[k]] = -1.0 / h[S.perm[k]];
  }
  S.G[d][S.perm[d - 1]] = 1.0 / h[S.perm[d - 1]];
  double v = 1.0;
  for (int a = 0; a < d; ++a) v *= h[a];
  S.vol = v / (d == 3 ? 6.0 : 2.0);
  // neighbours
  for (int k = 0; k <= d; ++k) {
    int ncell[3] = {S.cell[0], S.cell[1], S.cell[2]};
    int np[3];
    bool inside = true;
    for (int v2 = 0; v2 <= d; ++v2) S.map[k][v2] = -1;
    if (k == 0) {
      ncell[S.perm[0]] += 1;
      inside = ncell[S.perm[0]] < g.n[S.perm[0]];
      for (int j = 0; j < d - 1; ++j) np[j] = S.perm[j + 1];
      np[d - 1] = S.perm[0];
      for (int j = 1; j <= d; ++j) S.map[k][j] = j - 1;
    } else if (k == d) {
      ncell[S.perm[d - 1]] -= 1;
      inside = ncell[S.perm[d - 1]] >= 0;
      np[0] = S.perm[d - 1];
      for (int j = 1; j < d; ++j) np[j] = S.perm[j - 1];
      for (int j = 0; j < d; ++j) S.map[k][j] = j + 1;
    } else {
      for (int j = 0; j < d; ++j) np[j] = S.perm[j];
      np[k - 1] = S.perm[k];
      np[k] = S.perm[k - 1];
      for (int j = 0; j <= d; ++j)
        if (j != k) S.map[k][j] = j;
    }
    if (!inside) {
      S.nb[k] = -1;
      continue;
    }
    long nbox = 0, mul = 1;
    for (int a = 0; a < d; ++a) {
      nbox += ncell[a] * mul;
      mul *= g.n[a];
    }
    S.nb[k] = nbox * NP + dg_perm_index(d, np);
  }
}

// local unknown l of a simplex: velocity (vertex l / d, component l % d) for
// l < (d+1) d, else pressure at vertex l - (d+1) d
__device__ inline bool dg_is_u(int d, int l) { return l < (d + 1) * d; }

// Assembly: one thread per (simplex, network) writes the rows of its own
// unknowns in every block, the transfer block (network 0 thread) and the
// simplex's part of f.
template <int d>
__global__ __launch_bounds__(128) void k_dg_assemble(GridDev g, double hx, double hy, double hz,
                                                     const double *__restrict__ k1,
                                                     const double *__restrict__ k2, double beta,
                                                     const double *__restrict__ betac, double mu,
                                                     const double *__restrict__ body, const double *__restrict__ p01,
                                                     const double *__restrict__ p02, long nc, long nslot,
                                                     double *__restrict__ A, double *__restrict__ B,
                                                     int *__restrict__ nbr, double *__restrict__ f) {
  constexpr int SB = dg_sb(d);
  constexpr int NB = d + 2;
  constexpr int NU = (d + 1) * d;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (e >= nc) return;
  const double h[3] = {hx, hy, hz};
  DGSimplex S;
  dg_simplex<d>(g, h, e, S);
  const double *kq = q ? k2 : k1;
  const double alpha = mu / kq[e], kappa = kq[e] / mu;
  const double be = betac ? betac[e] : beta;
  double hd = 0.0;
  for (int a = 0; a < d; ++a) hd += h[a] * h[a];
  hd = sqrt(hd);  // twice the circumradius: the box-cell diagonal
  const double mc = S.vol / ((d + 1) * (d + 2));  // M[v][w] = mc (1 + delta_vw)
  const double vm = S.vol / (d + 1);
  // facet data
  double nrm[4][3], area[4], aavg[4], kavg[4];
  for (int k = 0; k <= d; ++k) {
    double gn = 0.0;
    for (int c = 0; c < d; ++c) gn += S.G[k][c] * S.G[k][c];
    gn = sqrt(gn);
    area[k] = d * S.vol * gn;
    for (int c = 0; c < d; ++c) nrm[k][c] = -S.G[k][c] / gn;
    aavg[k] = kavg[k] = 0.0;
    if (S.nb[k] >= 0) {
      const double kn = kq[S.nb[k]];
      aavg[k] = 0.5 * (alpha + mu / kn);
      kavg[k] = 0.5 * (kappa + kn / mu);
    }
  }
  const double mf0 = 1.0 / (d * (d + 1));  // Mf[a][b] = area mf0 (1 + delta_ab)
  // facet term of own row (vertex a, unknown kind of r) and a column of side
  // sigma (vertex b in own numbering) on facet k
  auto facet = [&](int k, int r, int b, int cu, bool col_u, double sigma) -> double {
    const int a = dg_is_u(d, r) ? r / d : r - NU;
    const double Mf = area[k] * mf0 * (a == b ? 2.0 : 1.0);
    if (dg_is_u(d, r)) {
      const int c1 = r % d;
      if (col_u) return ETA_U * hd * aavg[k] * sigma * nrm[k][c1] * nrm[k][cu] * Mf;
      return 0.5 * nrm[k][c1] * Mf;
    }
    if (col_u) return -0.5 * sigma * nrm[k][cu] * Mf;
    return (ETA_P / hd) * kavg[k] * sigma * Mf;
  };
  double *Aq = A + ((size_t)q * nc + e) * NB * SB * SB;
  for (int r = 0; r < SB; ++r) {
    const bool ru = dg_is_u(d, r);
    const int va = ru ? r / d : r - NU;
    // block 0: volume terms and own-own facet terms
    for (int c = 0; c < SB; ++c) {
      const bool cu = dg_is_u(d, c);
      const int vb = cu ? c / d : c - NU;
      const double M = mc * (va == vb ? 2.0 : 1.0);
      double v = 0.0;
      if (ru && cu) {
        if (r % d == c % d) v = 0.5 * alpha * M;
      } else if (ru) {
        const int cc = r % d;
        v = -vm * (S.G[va][cc] + 0.5 * S.G[vb][cc]);
      } else if (cu) {
        const int cc = c % d;
        v = vm * (S.G[vb][cc] + 0.5 * S.G[va][cc]);
      } else {
        double gg = 0.0;
        for (int cc = 0; cc < d; ++cc) gg += S.G[va][cc] * S.G[vb][cc];
        v = 0.5 * kappa * S.vol * gg + (be / mu) * M;
      }
      for (int k = 0; k <= d; ++k)
        if (S.nb[k] >= 0 && k != va && k != vb) v += facet(k, r, vb, cu ? c % d : 0, cu, 1.0);
      Aq[(size_t)r * SB + c] = v;
    }
    // blocks 1 + k: own rows, neighbour columns (the neighbour's numbering)
    for (int k = 0; k <= d; ++k) {
      double *Ab = Aq + (size_t)(1 + k) * SB * SB + (size_t)r * SB;
      for (int c = 0; c < SB; ++c) {
        double v = 0.0;
        if (S.nb[k] >= 0 && va != k) {
          const bool cu = dg_is_u(d, c);
          const int wn = cu ? c / d : c - NU;  // neighbour's local vertex
          int vb = -1;                         // that vertex in own numbering
          for (int j = 0; j <= d; ++j)
            if (j != k && S.map[k][j] == wn) vb = j;
          if (vb >= 0) v = facet(k, r, vb, cu ? c % d : 0, cu, -1.0);
        }
        Ab[c] = v;
      }
    }
  }
  if (q == 0) {
    // inter-network transfer block -(beta/mu) M and the neighbour table
    double *Be = B + (size_t)e * (d + 1) * (d + 1);
    for (int a = 0; a <= d; ++a)
      for (int b = 0; b <= d; ++b) Be[a * (d + 1) + b] = -(be / mu) * mc * (a == b ? 2.0 : 1.0);
    for (int k = 0; k <= d; ++k) nbr[e * (d + 1) + k] = (int)S.nb[k];
  }
  // right-hand side of the simplex's own unknowns
  const double *p0 = q ? p02 : p01;
  const long ou = off_u(d, nslot, q) + e * NU, op = off_p(d, nslot, q) + e * (d + 1);
  double bf[3] = {0.0, 0.0, 0.0};
  if (body)
    for (int c = 0; c < d; ++c) bf[c] = body[e * d + c];
  for (int v = 0; v <= d; ++v) {
    double fu[3];
    for (int c = 0; c < d; ++c) fu[c] = 0.5 * vm * bf[c];
    for (int k = 0; k <= d; ++k) {
      if (S.nb[k] >= 0 || k == v) continue;
      // boundary facet k holds vertex v: -(w.n; p0) with p0 linear on the facet
      double tr = 0.0;
      for (int b = 0; b <= d; ++b)
        if (b != k) tr += area[k] * mf0 * (b == v ? 2.0 : 1.0) * p0[S.node[b]];
      for (int c = 0; c < d; ++c) fu[c] -= nrm[k][c] * tr;
    }
    for (int c = 0; c < d; ++c) f[ou + v * d + c] = fu[c];
    double gb = 0.0;
    for (int c = 0; c < d; ++c) gb += S.G[v][c] * bf[c];
    f[op + v] = 0.5 * kappa * S.vol * gb;
  }
}

// ------------------------------------------------------ matrix-free rows --
// The solve applies K and its blocks from the simplex geometry and the
// coefficients instead of reading the stored blocks: on the uniform Kuhn
// mesh a simplex's barycentric gradients, facet normals and facet areas
// follow from its axis permutation and the box sizes, and every term of
// eq. S4_dg_stiffness_matrix is a short sum over the simplex's vertices
// (volume terms) or over the vertices of one facet (jump and average terms).
// A product then moves the vectors and the coefficients instead of (d + 2)
// SB^2 block values per simplex (facet neighbours follow from the Freudenthal
// rule, dg_neighbours).  The entries are those of the assembly above, summed
// in another order.

struct DGGeo {
  double h[3];
  double hd;  // twice the circumradius (the box-cell diagonal)
  double mu;
  double mc;  // M[a][b] = mc (1 + delta_ab), the same for every simplex of the box
  int n[3];   // boxes per axis
};

// Per-type shape table (one row per simplex type of a box, built on the
// host with the arithmetic of dg_shape): G[v][c], then nrm[k][c], then wf[k].
constexpr int DG_TAB_NRM = 1;  // nrm starts at DG_TAB_NRM (d + 1) d
__host__ __device__ constexpr int dg_tabsz(int d) { return 2 * (d + 1) * d + (d + 1); }

template <int d>
struct DGShape {
  double G[d + 1][d];    // barycentric gradients
  double nrm[d + 1][d];  // outward unit normal of the facet opposite each vertex
  double wf[d + 1];      // facet mass weight: Mf[a][b] = wf (1 + delta_ab)
  double mc, vm, vol;    // M[a][b] = mc (1 + delta_ab); vm = vol / (d + 1)
};

// Shape data of simplex e (its type is e mod the simplices per box; the
// permutation is formed without a lookup table so that it stays in registers)
template <int d>
__device__ inline void dg_shape(const DGGeo &geo, long e, DGShape<d> &S) {
  const int s = (int)(e % dg_nper(d));
  int p[d];
  if constexpr (d == 2) {
    p[0] = s;
    p[1] = 1 - s;
  } else {  // lexicographic permutations of {0, 1, 2}
    const int f = s >> 1, lo = f == 0 ? 1 : 0, hi = f == 2 ? 1 : 2;
    p[0] = f;
    p[1] = (s & 1) ? hi : lo;
    p[2] = (s & 1) ? lo : hi;
  }
#pragma unroll
  for (int c = 0; c < d; ++c) {
    const double ih = 1.0 / geo.h[c];
    S.G[0][c] = p[0] == c ? -ih : 0.0;
#pragma unroll
    for (int k = 1; k < d; ++k) S.G[k][c] = p[k - 1] == c ? ih : (p[k] == c ? -ih : 0.0);
    S.G[d][c] = p[d - 1] == c ? ih : 0.0;
  }
  double v = 1.0;
#pragma unroll
  for (int a = 0; a < d; ++a) v *= geo.h[a];
  S.vol = v / (d == 3 ? 6.0 : 2.0);
  S.mc = S.vol / ((d + 1) * (d + 2));
  S.vm = S.vol / (d + 1);
  const double mf0 = 1.0 / (d * (d + 1));
#pragma unroll
  for (int k = 0; k <= d; ++k) {
    double gn = 0.0;
#pragma unroll
    for (int c = 0; c < d; ++c) gn += S.G[k][c] * S.G[k][c];
    gn = sqrt(gn);
    S.wf[k] = d * S.vol * gn * mf0;
#pragma unroll
    for (int c = 0; c < d; ++c) S.nrm[k][c] = -S.G[k][c] / gn;
  }
}

// Volume terms of the selected blocks of one simplex: yu += K_uu xu (UU) +
// K_up xp (UP), yp += K_pu xu (PU) + K_pp xp (PP, without the transfer).
template <int d, bool UU, bool UP, bool PU, bool PP>
__device__ inline void dg_volume(const DGShape<d> &S, double alpha, double kappa, double bm, const double *xu,
                                 const double *xp, double *yu, double *yp) {
  double su[d], gp[d], sp = 0.0, divu = 0.0;
#pragma unroll
  for (int c = 0; c < d; ++c) su[c] = gp[c] = 0.0;
  if constexpr (UU || PU) {
#pragma unroll
    for (int b = 0; b <= d; ++b)
#pragma unroll
      for (int c = 0; c < d; ++c) {
        su[c] += xu[b * d + c];
        if constexpr (PU) divu += S.G[b][c] * xu[b * d + c];
      }
  }
  if constexpr (UP || PP) {
#pragma unroll
    for (int b = 0; b <= d; ++b) {
      sp += xp[b];
#pragma unroll
      for (int c = 0; c < d; ++c) gp[c] += S.G[b][c] * xp[b];
    }
  }
#pragma unroll
  for (int a = 0; a <= d; ++a) {
#pragma unroll
    for (int c = 0; c < d; ++c) {
      if constexpr (UU) yu[a * d + c] += 0.5 * alpha * S.mc * (xu[a * d + c] + su[c]);
      if constexpr (UP) yu[a * d + c] -= S.vm * (S.G[a][c] * sp + 0.5 * gp[c]);
    }
    if constexpr (PU) {
      double g = 0.0;
#pragma unroll
      for (int c = 0; c < d; ++c) g += S.G[a][c] * su[c];
      yp[a] += S.vm * (divu + 0.5 * g);
    }
    if constexpr (PP) {
      double g = 0.0;
#pragma unroll
      for (int c = 0; c < d; ++c) g += S.G[a][c] * gp[c];
      yp[a] += 0.5 * kappa * S.vol * g + bm * S.mc * (xp[a] + sp);
    }
  }
}

// Terms of the interior facet opposite own vertex k, with the neighbour's
// values nu, np in its own numbering (own vertex b is its vertex m(b)):
// cu = ETA_U hd {mu/k}, cp = (ETA_P / hd) {k/mu} (averages over the facet).
// With the normal jump [x_u.n], the pressure jump [x_p] and the pressure sum
// at the facet vertices, own rows a != k take
//   y_u(a, c) += cu n_c (Mf [x_u.n])_a + (1/2) n_c (Mf (x_p + x_p'))_a
//   y_p(a)    += -(1/2) (Mf [x_u.n])_a + cp (Mf [x_p])_a
template <int d, bool UU, bool UP, bool PU, bool PP>
__device__ inline void dg_facet(const DGShape<d> &S, int k, double cu, double cp, const double *xu, const double *xp,
                                const double *nu, const double *np, double *yu, double *yp) {
  double Jn[d + 1], Jp[d + 1], Sp[d + 1], sJn = 0.0, sJp = 0.0, sSp = 0.0;
#pragma unroll
  for (int b = 0; b <= d; ++b) {
    Jn[b] = Jp[b] = Sp[b] = 0.0;
    if (b == k) continue;
    const int m = k == 0 ? b - 1 : (k == d ? b + 1 : b);
    if constexpr (UU || PU) {
      double j = 0.0;
#pragma unroll
      for (int c = 0; c < d; ++c) j += S.nrm[k][c] * (xu[b * d + c] - nu[m * d + c]);
      Jn[b] = j;
      sJn += j;
    }
    if constexpr (PP) {
      Jp[b] = xp[b] - np[m];
      sJp += Jp[b];
    }
    if constexpr (UP) {
      Sp[b] = xp[b] + np[m];
      sSp += Sp[b];
    }
  }
  const double w = S.wf[k];
#pragma unroll
  for (int a = 0; a <= d; ++a) {
    if (a == k) continue;
    const double mjn = w * (Jn[a] + sJn), mjp = w * (Jp[a] + sJp), msp = w * (Sp[a] + sSp);
#pragma unroll
    for (int c = 0; c < d; ++c) {
      if constexpr (UU) yu[a * d + c] += cu * S.nrm[k][c] * mjn;
      if constexpr (UP) yu[a * d + c] += 0.5 * S.nrm[k][c] * msp;
    }
    if constexpr (PU) yp[a] -= 0.5 * mjn;
    if constexpr (PP) yp[a] += cp * mjp;
  }
}

// Facet neighbours of simplex e by the Freudenthal rule of the Kuhn split (as
// dg_simplex builds the neighbour table), computed in registers so that the
// neighbours' values can be fetched without waiting for the table: nb[k] is
// the simplex across the facet opposite local vertex k, -1 on the boundary.
template <int d>
__device__ inline void dg_neighbours(const DGGeo &g, long e, int *nb) {
  constexpr int NP = dg_nper(d);
  const long box = e / NP;
  const int s = (int)(e - box * NP);
  int cell[3] = {0, 0, 0}, p[3] = {0, 0, 0};
  long rr = box;
#pragma unroll
  for (int a = 0; a < d; ++a) {
    const long t = rr / g.n[a];
    cell[a] = (int)(rr - t * g.n[a]);
    rr = t;
  }
  if constexpr (d == 2) {
    p[0] = s;
    p[1] = 1 - s;
  } else {
    const int f = s >> 1, lo = f == 0 ? 1 : 0, hi = f == 2 ? 1 : 2;
    p[0] = f;
    p[1] = (s & 1) ? hi : lo;
    p[2] = (s & 1) ? lo : hi;
  }
#pragma unroll
  for (int k = 0; k <= d; ++k) {
    // the neighbour's box: one step along p[0] (k = 0) or back along p[d-1] (k = d)
    const int ax = k == 0 ? p[0] : (k == d ? p[d - 1] : -1);
    const int step = k == 0 ? 1 : -1;
    bool inside = true;
    long nbox = 0, mul = 1;
#pragma unroll
    for (int a = 0; a < d; ++a) {
      const int c = cell[a] + (ax == a ? step : 0);
      inside = inside && c >= 0 && c < g.n[a];
      nbox += c * mul;
      mul *= g.n[a];
    }
    // its axis permutation: p rotated left (k = 0), right (k = d), or with
    // entries k-1 and k swapped
    int q0, q1, q2 = 0;
    if (k == 0) {
      q0 = p[1];
      q1 = d == 3 ? p[2] : p[0];
      if (d == 3) q2 = p[0];
    } else if (k == d) {
      q0 = p[d - 1];
      q1 = p[0];
      if (d == 3) q2 = p[1];
    } else {
      q0 = k == 1 ? p[1] : p[0];
      q1 = k == 1 ? p[0] : p[2];
      if (d == 3) q2 = k == 1 ? p[2] : p[1];
    }
    const int pidx = d == 2 ? q0 : 2 * q0 + (q1 > q2 ? 1 : 0);
    nb[k] = inside ? (int)(nbox * NP + pidx) : -1;
  }
}

template <int n, typename T>
__device__ inline void dg_ld(const T *__restrict__ p, double *v) {
#pragma unroll
  for (int j = 0; j < n; ++j) v[j] = (double)p[j];
}

// y = K x (bsub null) or y = bsub - K x: one thread per (network, simplex)
// computes the (d + 1)^2 rows of its simplex.
template <int d>
__global__ __launch_bounds__(256) void k_dg_spmv(DGGeo geo, long nc, long nslot, const double *__restrict__ k1,
                                                 const double *__restrict__ k2, const double *__restrict__ betac,
                                                 double beta, const double *__restrict__ x,
                                                 const double *__restrict__ bsub,
                                                 double *__restrict__ y) {
  constexpr int NU = (d + 1) * d, NV = d + 1;
  const int q = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  DGShape<d> S;
  dg_shape<d>(geo, e, S);
  const double *kq = q ? k2 : k1;
  const double ke = kq[e], alpha = geo.mu / ke, kappa = ke / geo.mu;
  const double bm = (betac ? betac[e] : beta) / geo.mu;
  const double *xuq = x + off_u(d, nslot, q), *xpq = x + off_p(d, nslot, q);
  double xu[NU], xp[NV], xo[NV], yu[NU], yp[NV];
  dg_ld<NU>(xuq + e * NU, xu);
  dg_ld<NV>(xpq + e * NV, xp);
  dg_ld<NV>(x + off_p(d, nslot, 1 - q) + e * NV, xo);
#pragma unroll
  for (int j = 0; j < NU; ++j) yu[j] = 0.0;
#pragma unroll
  for (int j = 0; j < NV; ++j) yp[j] = 0.0;
  dg_volume<d, true, true, true, true>(S, alpha, kappa, bm, xu, xp, yu, yp);
  // transfer -(beta/mu) M to the other network's pressures
  double so = 0.0;
#pragma unroll
  for (int b = 0; b <= d; ++b) so += xo[b];
#pragma unroll
  for (int a = 0; a <= d; ++a) yp[a] -= bm * S.mc * (xo[a] + so);
  int nb[NV];
  dg_neighbours<d>(geo, e, nb);
#pragma unroll
  for (int k = 0; k <= d; ++k) {
    if (nb[k] < 0) continue;
    double nu[NU], np[NV];
    dg_ld<NU>(xuq + (long)nb[k] * NU, nu);
    dg_ld<NV>(xpq + (long)nb[k] * NV, np);
    const double kn = kq[nb[k]];
    dg_facet<d, true, true, true, true>(S, k, ETA_U * geo.hd * 0.5 * (alpha + geo.mu / kn),
                                        (ETA_P / geo.hd) * 0.5 * (kappa + kn / geo.mu), xu, xp, nu, np, yu, yp);
  }
  const long ou = off_u(d, nslot, q) + e * NU, op = off_p(d, nslot, q) + e * NV;
#pragma unroll
  for (int j = 0; j < NU; ++j) y[ou + j] = bsub ? bsub[ou + j] - yu[j] : yu[j];
#pragma unroll
  for (int j = 0; j < NV; ++j) y[op + j] = bsub ? bsub[op + j] - yp[j] : yp[j];
}

// CSR export: row r of simplex e lists its blocks' columns (self, then the
// neighbours in facet order), then the transfer columns of pressure rows.
template <int d>
__global__ void k_dg_export(long nc, long nslot, const double *__restrict__ A, const double *__restrict__ B,
                            const int *__restrict__ nbr, const int64_t *__restrict__ rowptr,
                            int32_t *__restrict__ cols, double *__restrict__ vals) {
  constexpr int SB = dg_sb(d);
  constexpr int NB = d + 2;
  constexpr int NU = (d + 1) * d;
  const int q = blockIdx.y;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * SB) return;
  const long e = t / SB;
  const int r = (int)(t % SB);
  const long ou = off_u(d, nslot, q), op = off_p(d, nslot, q);
  const long row = r < NU ? ou + e * NU + r : op + e * (d + 1) + (r - NU);
  int64_t w = rowptr[row];
  const double *Ar = A + ((size_t)q * nc + e) * NB * SB * SB + (size_t)r * SB;
  for (int b = 0; b < NB; ++b) {
    const long s = b == 0 ? e : nbr[e * (d + 1) + b - 1];
    if (s < 0) continue;
    for (int c = 0; c < SB; ++c) {
      cols[w] = (int32_t)(c < NU ? ou + s * NU + c : op + s * (d + 1) + (c - NU));
      vals[w++] = Ar[(size_t)b * SB * SB + c];
    }
  }
  if (r >= NU) {
    const int a = r - NU;
    const long oo = off_p(d, nslot, 1 - q);
    for (int c = 0; c <= d; ++c) {
      cols[w] = (int32_t)(oo + e * (d + 1) + c);
      vals[w++] = B[(size_t)e * (d + 1) * (d + 1) + a * (d + 1) + c];
    }
  }
}

// ------------------------------------------------------------ fieldsplit --
// The Schur fieldsplit of the solver section (Method 2, selfp) on the DG
// blocks, per network q (both networks in one launch, blockIdx.y = q):
//   rhat = r_p - K_pu V(r_u),  z_p ~ S_q^-1 rhat,  z_u = V(r_u - K_up z_p)
// with V the velocity solve (Chebyshev steps with the simplex-block Jacobi,
// k_dg_vcheb) and S_q = K_pp - K_pu D_u^-1 K_up, D_u = diag(K_uu), applied
// without forming it.  z_p comes from a two-level cycle: the nodal CG-VMS hierarchy
// of the same box and coefficients corrects the restricted residual (node
// values = sums over the node's slots; back by copying node values to the
// slots), then Chebyshev steps on S_q with its diagonal smooth on the slots.

// 1 / diag(K_uu): one thread per (network, simplex, velocity row)
template <int d>
__global__ void k_dg_diag_u(long nc, const double *__restrict__ A, double *__restrict__ du) {
  constexpr int SB = dg_sb(d), NB = d + 2, NU = (d + 1) * d;
  const int q = blockIdx.y;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * NU) return;
  const long e = t / NU;
  const int r = (int)(t % NU);
  du[(size_t)q * nc * NU + t] = 1.0 / A[(((size_t)q * nc + e) * NB * SB + r) * SB + r];
}

// 1 / diag(S_q) = 1 / (K_pp[i][i] + sum_j K_pu[i][j]^2 / K_uu[j][j]) (K_up = -K_pu^T)
template <int d>
__global__ void k_dg_diag_s(long nc, const double *__restrict__ A, const int *__restrict__ nbr,
                            const double *__restrict__ du, double *__restrict__ ds) {
  constexpr int SB = dg_sb(d), NB = d + 2, NU = (d + 1) * d;
  const int q = blockIdx.y;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * (d + 1)) return;
  const long e = t / (d + 1);
  const int a = (int)(t % (d + 1));
  const double *Ar = A + (((size_t)q * nc + e) * NB * SB + NU + a) * SB;
  const double *duq = du + (size_t)q * nc * NU;
  double v = Ar[NU + a];
  for (int b = 0; b < NB; ++b) {
    const long s2 = b == 0 ? e : nbr[e * (d + 1) + b - 1];
    if (s2 < 0) continue;
    for (int c = 0; c < NU; ++c) {
      const double w = Ar[(size_t)b * SB * SB + c];
      v += w * w * duq[s2 * NU + c];
    }
  }
  ds[(size_t)q * nc * (d + 1) + t] = 1.0 / v;
}

// The fieldsplit kernels below store their vectors (and the block inverses
// and diagonals) in T: double, or float for the FP32 preconditioner; they
// compute in double.

// rhat = r_p - K_pu y_u (y_u [2][n_cells NU], the velocity solve's output):
// one thread per (network, simplex)
template <int d, typename T>
__global__ __launch_bounds__(256) void k_dg_rhat(DGGeo geo, long nc, long nslot,
                                                 const T *__restrict__ yu, const T *__restrict__ r,
                                                 T *__restrict__ rh) {
  constexpr int NU = (d + 1) * d, NV = d + 1;
  const int q = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  DGShape<d> S;
  dg_shape<d>(geo, e, S);
  const T *yq = yu + (size_t)q * nc * NU;
  double xu[NU], yp[NV];
  dg_ld<NU>(yq + e * NU, xu);
#pragma unroll
  for (int j = 0; j < NV; ++j) yp[j] = 0.0;
  dg_volume<d, false, false, true, false>(S, 0.0, 0.0, 0.0, xu, nullptr, nullptr, yp);
  int nb[NV];
  dg_neighbours<d>(geo, e, nb);
#pragma unroll
  for (int k = 0; k <= d; ++k) {
    if (nb[k] < 0) continue;
    double nu[NU];
    dg_ld<NU>(yq + (long)nb[k] * NU, nu);
    dg_facet<d, false, false, true, false>(S, k, 0.0, 0.0, xu, nullptr, nu, nullptr, nullptr, yp);
  }
  const T *rp = r + off_p(d, nslot, q) + e * NV;
  T *o = rh + (size_t)q * nslot + e * NV;
#pragma unroll
  for (int j = 0; j < NV; ++j) o[j] = (T)((double)rp[j] - yp[j]);
}

// tu = K_up zp, or w = D_u^-1 K_up zp when du is given: one thread per
// (network, simplex)
template <int d, typename T>
__global__ __launch_bounds__(256) void k_dg_tu(DGGeo geo, long nc, long nslot,
                                               const T *__restrict__ zp, const T *__restrict__ du,
                                               T *__restrict__ tu) {
  constexpr int NU = (d + 1) * d, NV = d + 1;
  const int q = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  DGShape<d> S;
  dg_shape<d>(geo, e, S);
  const T *z = zp + (size_t)q * nslot;
  double xp[NV], yu[NU];
  dg_ld<NV>(z + e * NV, xp);
#pragma unroll
  for (int j = 0; j < NU; ++j) yu[j] = 0.0;
  dg_volume<d, false, true, false, false>(S, 0.0, 0.0, 0.0, nullptr, xp, yu, nullptr);
  int nb[NV];
  dg_neighbours<d>(geo, e, nb);
#pragma unroll
  for (int k = 0; k <= d; ++k) {
    if (nb[k] < 0) continue;
    double np[NV];
    dg_ld<NV>(z + (long)nb[k] * NV, np);
    dg_facet<d, false, true, false, false>(S, k, 0.0, 0.0, nullptr, xp, nullptr, np, yu, nullptr);
  }
  const size_t o = (size_t)q * nc * NU + e * NU;
  if (du) {
#pragma unroll
    for (int j = 0; j < NU; ++j) tu[o + j] = (T)((double)du[o + j] * yu[j]);
  } else {
#pragma unroll
    for (int j = 0; j < NU; ++j) tu[o + j] = (T)yu[j];
  }
}

// y = S_q x = K_pp x - K_pu w with w = D_u^-1 K_up x (from k_dg_tu); with
// cheb, one Chebyshev step instead: r = D_S^-1 (b - S_q x), dd = c1 dd + c2 r,
// xout = x + dd.  One thread per (network, simplex).
template <int d, typename T>
__global__ __launch_bounds__(256) void k_dg_sp(DGGeo geo, long nc, long nslot, const double *__restrict__ k1,
                                               const double *__restrict__ k2, const double *__restrict__ betac,
                                               double beta, const T *__restrict__ w,
                                               const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ ds,
                                               const T *__restrict__ b, T *__restrict__ dd, Sc2 c1, Sc2 c2,
                                               bool cheb) {
  constexpr int NU = (d + 1) * d, NV = d + 1;
  const int q = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  DGShape<d> S;
  dg_shape<d>(geo, e, S);
  const double *kq = q ? k2 : k1;
  const double ke = kq[e], alpha = geo.mu / ke, kappa = ke / geo.mu;
  const double bm = (betac ? betac[e] : beta) / geo.mu;
  const T *xq = x + (size_t)q * nslot, *wq = w + (size_t)q * nc * NU;
  double xp[NV], wu[NU], ypp[NV], ypu[NV];
  dg_ld<NV>(xq + e * NV, xp);
  dg_ld<NU>(wq + e * NU, wu);
#pragma unroll
  for (int j = 0; j < NV; ++j) ypp[j] = ypu[j] = 0.0;
  dg_volume<d, false, false, false, true>(S, alpha, kappa, bm, nullptr, xp, nullptr, ypp);
  dg_volume<d, false, false, true, false>(S, alpha, kappa, bm, wu, nullptr, nullptr, ypu);
  int nb[NV];
  dg_neighbours<d>(geo, e, nb);
#pragma unroll
  for (int k = 0; k <= d; ++k) {
    if (nb[k] < 0) continue;
    double np[NV], nw[NU];
    dg_ld<NV>(xq + (long)nb[k] * NV, np);
    dg_ld<NU>(wq + (long)nb[k] * NU, nw);
    const double kn = kq[nb[k]];
    dg_facet<d, false, false, false, true>(S, k, 0.0, (ETA_P / geo.hd) * 0.5 * (kappa + kn / geo.mu), nullptr, xp,
                                           nullptr, np, nullptr, ypp);
    dg_facet<d, false, false, true, false>(S, k, 0.0, 0.0, wu, nullptr, nw, nullptr, nullptr, ypu);
  }
  const size_t i0 = (size_t)q * nslot + e * NV;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const size_t i = i0 + j;
    const double acc = ypp[j] - ypu[j];
    if (!cheb) {
      y[i] = (T)(ds ? (double)ds[i] * acc : acc);
      continue;
    }
    const double rr = (double)ds[i] * ((double)b[i] - acc);
    const double dn = (c1.v[q] != 0.0 ? c1.v[q] * (double)dd[i] : 0.0) + c2.v[q] * rr;
    dd[i] = (T)dn;
    y[i] = (T)(xp[j] + dn);
  }
}

// Inverses of the diagonal velocity blocks of K_uu (one per simplex and
// network, NU x NU, symmetric positive definite): Gauss-Jordan without
// pivoting, one thread per (network, simplex).  Stored packed: the upper
// triangle of the symmetric part, row by row (dg_packed), NU (NU + 1) / 2
// values per block.
__host__ __device__ constexpr int dg_npk(int d) { return (d + 1) * d * ((d + 1) * d + 1) / 2; }
// packed position of entry (i, j), i <= j, of an n x n symmetric matrix
__host__ __device__ constexpr int dg_packed(int n, int i, int j) { return i * n - i * (i - 1) / 2 + (j - i); }
template <int d>
__global__ void k_dg_binv(long nc, const double *__restrict__ A, double *__restrict__ Bi) {
  constexpr int SB = dg_sb(d), NB = d + 2, NU = (d + 1) * d;
  const int q = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  double M[NU][NU], X[NU][NU];
  const double *Ae = A + ((size_t)q * nc + e) * NB * SB * SB;
  for (int r = 0; r < NU; ++r)
    for (int c = 0; c < NU; ++c) {
      M[r][c] = Ae[r * SB + c];
      X[r][c] = r == c ? 1.0 : 0.0;
    }
  for (int k = 0; k < NU; ++k) {
    const double piv = 1.0 / M[k][k];
    for (int c = 0; c < NU; ++c) {
      M[k][c] *= piv;
      X[k][c] *= piv;
    }
    for (int r = 0; r < NU; ++r) {
      if (r == k) continue;
      const double f = M[r][k];
      for (int c = 0; c < NU; ++c) {
        M[r][c] -= f * M[k][c];
        X[r][c] -= f * X[k][c];
      }
    }
  }
  double *Be = Bi + ((size_t)q * nc + e) * dg_npk(d);
  for (int r = 0; r < NU; ++r)
    for (int c = r; c < NU; ++c) Be[dg_packed(NU, r, c)] = 0.5 * (X[r][c] + X[c][r]);
}

// Strided view of per-network velocity vectors: network q's value of
// simplex e, row r sits at base[q * stride + e NU + r].
template <typename T>
struct DGVec {
  const T *base;
  long stride;
};
template <typename T>
struct DGOut {
  T *base;
  long stride;
};

// Velocity-block Chebyshev step with the simplex-block Jacobi (Saad, Alg.
// 12.1): res = b - K_uu x (b less tu when given; x = 0 when xin is null),
// r' = Binv res, xout = x + c1 (x - xprev) + c2 r' (the three-term form of
// dd = c1 dd + c2 r', xout = x + dd; xprev null: 0; xout may be xprev, each
// thread reading its own entry first).  power: xout = Binv (K_uu x) (the
// power steps of the interval).  Workgroups of whole simplices (192
// threads: 16 simplices in 3D, 32 in 2D), in three phases: every thread
// stages one value of its simplex and of each facet neighbour in LDS (and
// fetches its b, x_(k-1) entries); one thread per (simplex, vertex) forms the
// d K_uu x rows of that vertex from LDS and the simplex type's shape table;
// one thread per row applies its row of Binv.  The step is bound by the
// latency of these dependent phases more than by its bytes, so the launch
// bound asks for 7 waves per SIMD (72 VGPRs in 3D, no spills; 8 spill).
constexpr int DGV_BS = 192;
template <int d, typename T>
__global__ __launch_bounds__(DGV_BS, 7) void k_dg_vcheb(DGGeo geo, const double *__restrict__ tab, long nc,
                                                     const double *__restrict__ k1,
                                                     const double *__restrict__ k2, const T *__restrict__ Bi,
                                                     DGVec<T> b, const T *__restrict__ tu, DGVec<T> xin,
                                                     DGOut<T> xout, DGVec<T> xprev, Sc2 c1, Sc2 c2, bool power) {
  constexpr int NU = (d + 1) * d, NV = d + 1;
  constexpr int EPB = DGV_BS / NU;
  // per-simplex LDS stride: odd in doubles, so that the simplices of a wave
  // spread over the banks
  constexpr int XS = (NV + 1) * NU + 1, TS = dg_tabsz(d) * dg_nper(d);
  static_assert(EPB * NU == DGV_BS && NU > NV && TS <= DGV_BS, "whole simplices per workgroup");
  __shared__ double xs[EPB * XS];   // own values, then the facet neighbours' (NU each)
  __shared__ double sa[EPB][NV + 1];  // mu/k of the facet neighbours (0 across the boundary), own last
  __shared__ double sh[DGV_BS];
  __shared__ double st[TS];           // the shape table
  const int q = blockIdx.y;
  const int loc = threadIdx.x / NU, r = threadIdx.x % NU;
  const long e = (long)blockIdx.x * EPB + loc;
  const bool live = e < nc;
  const T *xq = xin.base ? xin.base + (size_t)q * xin.stride : nullptr;
  // operands of the last phase, fetched first: b less tu, x_(k-1)
  double bv = 0.0, xp = 0.0;
  if (live) {
    if (!power) {
      bv = (double)b.base[(size_t)q * b.stride + e * NU + r] -
           (tu ? (double)tu[(size_t)q * nc * NU + e * NU + r] : 0.0);
      if (xprev.base) xp = (double)xprev.base[(size_t)q * xprev.stride + e * NU + r];
    }
  }
  if (xq) {  // uniform over the launch
    const double *kq = q ? k2 : k1;
    if (threadIdx.x < TS) st[threadIdx.x] = tab[threadIdx.x];
    if (live) {
      double *xl = xs + loc * XS;
      int nb[NV];
      dg_neighbours<d>(geo, e, nb);
      xl[r] = (double)xq[e * NU + r];
#pragma unroll
      for (int k = 0; k <= d; ++k) xl[(1 + k) * NU + r] = nb[k] >= 0 ? (double)xq[(long)nb[k] * NU + r] : 0.0;
      if (r < NV) {
        int nr = nb[0];
#pragma unroll
        for (int k = 1; k <= d; ++k) nr = r == k ? nb[k] : nr;
        sa[loc][r] = nr >= 0 ? geo.mu / kq[nr] : 0.0;
      } else if (r == NV) {
        sa[loc][NV] = geo.mu / kq[e];
      }
    }
    __syncthreads();
    if (threadIdx.x < EPB * NV) {
      const int l2 = threadIdx.x / NV, a = threadIdx.x % NV;
      const long e2 = (long)blockIdx.x * EPB + l2;
      if (e2 < nc) {
        const double *tb = st + (e2 % dg_nper(d)) * dg_tabsz(d);
        const double alpha = sa[l2][NV];
        const double *x0 = xs + l2 * XS;
        double su[d], y[d];
#pragma unroll
        for (int c = 0; c < d; ++c) {
          double t = 0.0;
#pragma unroll
          for (int v = 0; v <= d; ++v) t += x0[v * d + c];
          su[c] = t;
        }
        // volume: (1/2) (mu/k) M, M[a][b] = mc (1 + delta_ab), per component
#pragma unroll
        for (int c = 0; c < d; ++c) y[c] = 0.5 * alpha * geo.mc * (x0[a * d + c] + su[c]);
#pragma unroll
        for (int k = 0; k <= d; ++k) {
          const double an = sa[l2][k];
          if (an == 0.0 || k == a) continue;
          const double *xk = x0 + (1 + k) * NU;
          double n[d];
#pragma unroll
          for (int c = 0; c < d; ++c) n[c] = tb[DG_TAB_NRM * NV * d + k * d + c];
          // normal jumps at the facet vertices: all of them, then own vertex a
          double sj = 0.0;
#pragma unroll
          for (int v = 0; v <= d; ++v) {
            if (v == k) continue;
            const int m = k == 0 ? v - 1 : (k == d ? v + 1 : v);
#pragma unroll
            for (int c = 0; c < d; ++c) sj += n[c] * (x0[v * d + c] - xk[m * d + c]);
          }
          const int ma = k == 0 ? a - 1 : (k == d ? a + 1 : a);
          double ja = 0.0;
#pragma unroll
          for (int c = 0; c < d; ++c) ja += n[c] * (x0[a * d + c] - xk[ma * d + c]);
          const double cu = ETA_U * geo.hd * 0.5 * (alpha + an);
          const double mjn = tb[2 * NV * d + k] * (ja + sj);
#pragma unroll
          for (int c = 0; c < d; ++c) y[c] += cu * n[c] * mjn;
        }
#pragma unroll
        for (int c = 0; c < d; ++c) sh[l2 * NU + a * d + c] = y[c];
      }
    }
    __syncthreads();
  }
  double res = 0.0, xr = 0.0;
  if (live) {
    const double acc = xq ? sh[threadIdx.x] : 0.0;
    if (xq) xr = xs[loc * XS + r];
    res = power ? acc : bv - acc;
  }
  __syncthreads();
  sh[threadIdx.x] = res;
  __syncthreads();
  if (!live) return;
  // row r of the packed symmetric block: (r, c) for c >= r, (c, r) below
  const T *Be = Bi + ((size_t)q * nc + e) * dg_npk(d);
  const int rb = dg_packed(NU, r, 0);
  double rp = 0.0;
#pragma unroll
  for (int c = 0; c < NU; ++c) rp += (double)Be[r <= c ? rb + c : dg_packed(NU, c, 0) + r] * sh[loc * NU + c];
  T *out = xout.base + (size_t)q * xout.stride + e * NU + r;
  if (power) {
    *out = (T)rp;
    return;
  }
  *out = (T)(xr + (c1.v[q] != 0.0 ? c1.v[q] * (xr - xp) : 0.0) + c2.v[q] * rp);
}

// z_p = zp (the pressure part of the fieldsplit's output)
template <int d, typename T>
__global__ void k_dg_copyp(long nslot, const T *__restrict__ zp, T *__restrict__ z) {
  const int q = blockIdx.y;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslot) return;
  z[off_p(d, nslot, q) + i] = zp[(size_t)q * nslot + i];
}

// node value = sum over the slots on the node: for each box around the node
// and each simplex of it, the node is local vertex |delta| when the axes of
// its offset delta from the box corner are the first |delta| axes of pi
template <int d, typename T>
__global__ void k_dg_restrict(GridDev g, long nslot, const T *__restrict__ xs, T *__restrict__ xn) {
  constexpr int NP = dg_nper(d);
  const int q = blockIdx.y;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= g.N) return;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  double acc = 0.0;
  for (int m = 0; m < (1 << d); ++m) {  // delta bits: the node sits at corner + delta
    int cell[3];
    bool ok = true;
    for (int ax = 0; ax < d; ++ax) {
      cell[ax] = ia[ax] - ((m >> ax) & 1);
      ok = ok && cell[ax] >= 0 && cell[ax] < g.n[ax];
    }
    if (!ok) continue;
    long box = 0, mul = 1;
    for (int ax = 0; ax < d; ++ax) {
      box += cell[ax] * mul;
      mul *= g.n[ax];
    }
    const int v = __popc(m);
    for (int s = 0; s < NP; ++s) {
      int p[3];
      dg_perm(d, s, p);
      int pre = 0;
      for (int j = 0; j < v; ++j) pre |= 1 << p[j];
      if (pre == m) acc += (double)xs[(size_t)q * nslot + (box * NP + s) * (d + 1) + v];
    }
  }
  xn[(size_t)q * g.N + a] = (T)acc;
}

// slot value = value of its node
template <int d, typename T>
__global__ void k_dg_prolong(GridDev g, long nc, long nslot, const T *__restrict__ xn, T *__restrict__ xs) {
  constexpr int NP = dg_nper(d);
  const int q = blockIdx.y;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslot) return;
  const long e = t / (d + 1);
  const int v = (int)(t % (d + 1));
  const long box = e / NP;
  int p[3];
  dg_perm(d, (int)(e % NP), p);
  long r = box, node = 0;
  const long stride[3] = {1, g.m[0], (long)g.m[0] * g.m[1]};
  for (int ax = 0; ax < d; ++ax) {
    node += (r % g.n[ax]) * stride[ax];
    r /= g.n[ax];
  }
  for (int j = 0; j < v; ++j) node += stride[p[j]];
  xs[(size_t)q * nslot + t] = xn[(size_t)q * g.N + node];
}

__global__ void k_dg_hash(double *__restrict__ x, long n) {
  const int q = blockIdx.y;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long h = ((unsigned long long)i * 2654435761ull) & 0xffffffffull;
  x[(size_t)q * n + i] = (double)h / 4294967296.0 - 0.5;
}

// per-network sums of squares in a fixed order: partials, then one block
constexpr int DG_RB = 256;
__global__ __launch_bounds__(256) void k_dg_sumsq(const double *__restrict__ x, long n, double *__restrict__ part) {
  const int q = blockIdx.y;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double v = x[(size_t)q * n + i];
    acc += v * v;
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[q * DG_RB + blockIdx.x] = sh[0];
}
__global__ __launch_bounds__(256) void k_dg_sumsq_fin(const double *__restrict__ part, double *__restrict__ ss) {
  __shared__ double sh[256];
  for (int q = 0; q < 2; ++q) {
    sh[threadIdx.x] = part[q * DG_RB + threadIdx.x];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) ss[q] = sh[0];
    __syncthreads();
  }
}
__global__ void k_dg_scale(double *__restrict__ x, long n, const double *__restrict__ ss) {
  const int q = blockIdx.y;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[(size_t)q * n + i] /= sqrt(ss[q]);
}

}  // namespace

namespace {
DGGeo dg_geo(dpp_problem P) {
  DGGeo geo{};
  double hd = 0.0;
  for (int a = 0; a < P->g.dim; ++a) {
    geo.h[a] = P->g.h[a];
    hd += P->g.h[a] * P->g.h[a];
  }
  geo.hd = std::sqrt(hd);
  geo.mu = P->mu;
  for (int a = 0; a < 3; ++a) geo.n[a] = P->g.n[a];
  double v = 1.0;
  for (int a = 0; a < P->g.dim; ++a) v *= P->g.h[a];
  const int d = P->g.dim;
  geo.mc = v / (d == 3 ? 6.0 : 2.0) / ((d + 1) * (d + 2));
  return geo;
}

// the per-type shape table (dg_tabsz values per type), with dg_shape's arithmetic
std::vector<double> dg_shape_table(const Grid &g) {
  const int d = g.dim, NP = dg_nper(d), NV = d + 1;
  std::vector<double> tab((size_t)NP * dg_tabsz(d), 0.0);
  double v = 1.0;
  for (int a = 0; a < d; ++a) v *= g.h[a];
  const double vol = v / (d == 3 ? 6.0 : 2.0), mf0 = 1.0 / (d * (d + 1));
  for (int t = 0; t < NP; ++t) {
    int p[3] = {0, 0, 0};
    if (d == 2) {
      p[0] = t;
      p[1] = 1 - t;
    } else {
      const int f = t >> 1, lo = f == 0 ? 1 : 0, hi = f == 2 ? 1 : 2;
      p[0] = f;
      p[1] = (t & 1) ? hi : lo;
      p[2] = (t & 1) ? lo : hi;
    }
    double G[4][3] = {};
    for (int c = 0; c < d; ++c) {
      const double ih = 1.0 / g.h[c];
      G[0][c] = p[0] == c ? -ih : 0.0;
      for (int k = 1; k < d; ++k) G[k][c] = p[k - 1] == c ? ih : (p[k] == c ? -ih : 0.0);
      G[d][c] = p[d - 1] == c ? ih : 0.0;
    }
    double *T = tab.data() + (size_t)t * dg_tabsz(d);
    for (int k = 0; k <= d; ++k) {
      double gn = 0.0;
      for (int c = 0; c < d; ++c) gn += G[k][c] * G[k][c];
      gn = std::sqrt(gn);
      T[2 * NV * d + k] = d * vol * gn * mf0;
      for (int c = 0; c < d; ++c) {
        T[k * d + c] = G[k][c];
        T[DG_TAB_NRM * NV * d + k * d + c] = -G[k][c] / gn;
      }
    }
  }
  return tab;
}
const double *dg_betac(dpp_problem P) { return P->beta_per_cell ? P->betac.as<double>() : nullptr; }
// coefficient bytes a product reads per network: k (and beta per simplex)
double dg_coef_bytes(dpp_problem P) { return 8.0 * P->g.nc * (P->beta_per_cell ? 2.0 : 1.0); }
}  // namespace

void dg_assemble(dpp_problem P, const dpp_params *prm, hipStream_t s) {
  const Grid &g = P->g;
  const int d = g.dim;
  const long nc = g.nc;
  const long nslot = nc * (d + 1);
  const int SB = (d + 1) * (d + 1);
  P->dg = 1;
  P->nslot = nslot;
  P->dgA.alloc(sizeof(double) * 2 * (size_t)nc * (d + 2) * SB * SB);
  P->dgB.alloc(sizeof(double) * (size_t)nc * (d + 1) * (d + 1));
  P->dgnb.alloc(sizeof(int) * (size_t)nc * (d + 1));
  {
    const std::vector<double> tab = dg_shape_table(g);
    P->dgtab.alloc(sizeof(double) * tab.size());
    DPP_HIP(hipMemcpyAsync(P->dgtab.ptr, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s));
    DPP_HIP(hipStreamSynchronize(s));  // the host table is freed on return
  }
  P->f.alloc(sizeof(double) * P->ndof());
  // coefficient copies: the preconditioner assembles the nodal problem of the
  // same box and coefficients
  P->k1.alloc(sizeof(double) * nc);
  P->k2.alloc(sizeof(double) * nc);
  DPP_HIP(hipMemcpyAsync(P->k1.ptr, prm->k1, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
  DPP_HIP(hipMemcpyAsync(P->k2.ptr, prm->k2, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
  if (prm->beta_cells) {
    P->betac.alloc(sizeof(double) * nc);
    DPP_HIP(hipMemcpyAsync(P->betac.ptr, prm->beta_cells, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
  }
  const dim3 grid(blocks_for(nc, 128), 2);
  if (d == 3)
    k_dg_assemble<3><<<grid, 128, 0, s>>>(dev(g), g.h[0], g.h[1], g.h[2], prm->k1, prm->k2, prm->beta, prm->beta_cells,
                                          prm->mu, prm->body, prm->p0_1, prm->p0_2, nc, nslot, P->dgA.as<double>(),
                                          P->dgB.as<double>(), P->dgnb.as<int>(), P->f.as<double>());
  else
    k_dg_assemble<2><<<grid, 128, 0, s>>>(dev(g), g.h[0], g.h[1], g.h[2], prm->k1, prm->k2, prm->beta, prm->beta_cells,
                                          prm->mu, prm->body, prm->p0_1, prm->p0_2, nc, nslot, P->dgA.as<double>(),
                                          P->dgB.as<double>(), P->dgnb.as<int>(), P->f.as<double>());
  check_launch("DG assembly");
  // structural nonzeros: SB per coupled simplex and row, plus d + 1 transfer
  // columns per pressure row; the interior facets are counted on the host
  long interior = 0;  // (simplex, facet) pairs with a neighbour, from the neighbour table
  {
    std::vector<int> nb((size_t)nc * (d + 1));
    DPP_HIP(hipMemcpyAsync(nb.data(), P->dgnb.ptr, sizeof(int) * nb.size(), hipMemcpyDeviceToHost, s));
    DPP_HIP(hipStreamSynchronize(s));
    for (int v : nb) interior += v >= 0;
  }
  P->dgcoupled = nc + interior;
  P->nnz = 2 * (P->dgcoupled * (long)SB * SB + nc * (long)(d + 1) * (d + 1));
}

void dg_spmv(dpp_problem P, const double *x, const double *bsub, double *y, hipStream_t s) {
  const Grid &g = P->g;
  const int d = g.dim;
  const long nc = g.nc;
  const dim3 grid(blocks_for(nc, 256), 2);
  // algorithmic bytes (matrix-free, neighbours from the Freudenthal rule): x
  // and y (and b) once, the coefficients of both networks
  ProfScope ps(PF_SPMV_K, 8.0 * P->ndof() * (bsub ? 3.0 : 2.0) + 2.0 * dg_coef_bytes(P), s);
  const DGGeo geo = dg_geo(P);
  if (d == 3)
    k_dg_spmv<3><<<grid, 256, 0, s>>>(geo, nc, P->nslot, P->k1.as<double>(), P->k2.as<double>(), dg_betac(P),
                                      P->beta, x, bsub, y);
  else
    k_dg_spmv<2><<<grid, 256, 0, s>>>(geo, nc, P->nslot, P->k1.as<double>(), P->k2.as<double>(), dg_betac(P),
                                      P->beta, x, bsub, y);
  check_launch("DG spmv");
}

void dg_export_csr(dpp_problem P, int64_t *rowptr, int32_t *cols, double *vals, hipStream_t s) {
  const Grid &g = P->g;
  const int d = g.dim;
  const long nc = g.nc;
  const int SB = (d + 1) * (d + 1), NU = (d + 1) * d;
  // row lengths on the host from the neighbour table
  std::vector<int> nb((size_t)nc * (d + 1));
  DPP_HIP(hipMemcpyAsync(nb.data(), P->dgnb.ptr, sizeof(int) * nb.size(), hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  const long n = P->ndof(), nslot = P->nslot;
  std::vector<int64_t> rp(n + 1, 0);
  for (int q = 0; q < 2; ++q)
    for (long e = 0; e < nc; ++e) {
      int coupled = 1;
      for (int k = 0; k <= d; ++k) coupled += nb[e * (d + 1) + k] >= 0;
      for (int l = 0; l < SB; ++l) {
        const long row = l < NU ? off_u(d, nslot, q) + e * NU + l : off_p(d, nslot, q) + e * (d + 1) + (l - NU);
        rp[row + 1] = (int64_t)coupled * SB + (l < NU ? 0 : d + 1);
      }
    }
  for (long i = 0; i < n; ++i) rp[i + 1] += rp[i];
  DPP_CHECK(rp[n] == P->nnz, DPP_ERR_ARG, "internal: DG nonzero count");
  DPP_HIP(hipMemcpyAsync(rowptr, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
  const dim3 grid(blocks_for(nc * SB, 256), 2);
  if (d == 3)
    k_dg_export<3><<<grid, 256, 0, s>>>(nc, nslot, P->dgA.as<double>(), P->dgB.as<double>(), P->dgnb.as<int>(),
                                        rowptr, cols, vals);
  else
    k_dg_export<2><<<grid, 256, 0, s>>>(nc, nslot, P->dgA.as<double>(), P->dgB.as<double>(), P->dgnb.as<int>(),
                                        rowptr, cols, vals);
  check_launch("DG export");
  DPP_HIP(hipStreamSynchronize(s));
}


// ------------------------------------------------------------ fieldsplit --
namespace {

template <int d>
void dg_s_apply(dpp_precond pc, const double *x, double *y, const double *ds, hipStream_t s) {
  dpp_problem P = pc->prob;
  const long nc = P->g.nc, nslot = P->nslot;
  const DGGeo geo = dg_geo(P);
  const dim3 gs(blocks_for(nc, 256), 2);
  k_dg_tu<d, double><<<gs, 256, 0, s>>>(geo, nc, nslot, x, pc->dgdu.as<double>(),
                                        pc->dgtu.as<double>());
  k_dg_sp<d, double><<<gs, 256, 0, s>>>(geo, nc, nslot, P->k1.as<double>(), P->k2.as<double>(), dg_betac(P), P->beta,
                                        pc->dgtu.as<double>(), x, y, ds, nullptr, nullptr,
                                        Sc2{{0, 0}}, Sc2{{0, 0}}, false);
}

// Work buffers of the fieldsplit in one precision: FP64, or FP32 (the block
// inverses and diagonals rounded once, dg_make32) for the FP32 preconditioner.
template <typename T>
struct DGWork {
  const T *du, *ds, *binv;
  T *rh, *za, *zb, *dd, *tu, *cb, *cx, *va, *vb, *yu;
};
DGWork<double> dg_work(dpp_precond pc, double) {
  return {pc->dgdu.as<double>(), pc->dgds.as<double>(), pc->dgbinv.as<double>(), pc->dgrh.as<double>(),
          pc->dgza.as<double>(), pc->dgzb.as<double>(),  pc->dgd.as<double>(),     pc->dgtu.as<double>(),
          pc->dgcb.as<double>(), pc->dgcx.as<double>(),  pc->dgva.as<double>(),    pc->dgvb.as<double>(),
          pc->dgyu.as<double>()};
}
DGWork<float> dg_work(dpp_precond pc, float) {
  return {pc->dgdu32.as<float>(), pc->dgds32.as<float>(), pc->dgbinv32.as<float>(), pc->dgrh32.as<float>(),
          pc->dgza32.as<float>(), pc->dgzb32.as<float>(),  pc->dgd32.as<float>(),     pc->dgtu32.as<float>(),
          pc->dgcb32.as<float>(), pc->dgcx32.as<float>(),  pc->dgva32.as<float>(),    pc->dgvb32.as<float>(),
          pc->dgyu32.as<float>()};
}
// the nodal CG-VMS cycle in the fieldsplit's precision
void dg_vcycle(dpp_precond pc, const double *b, double *x, hipStream_t s) { vcycle(pc, b, x, s); }
void dg_vcycle(dpp_precond pc, const float *b, float *x, hipStream_t s) { vcycle32(pc, b, x, s); }

constexpr int DG_VEL_DEGREE = 8;      // Chebyshev steps of the velocity-block solve
constexpr int DG_NODAL_COARSE_2D = 1800;  // default coarsest size of the 2D nodal cycle
constexpr double DG_VEL_LO_FRAC = 0.01;  // its interval [0.01 hi, hi]
constexpr int DG_PRES_DEGREE = 3;     // Chebyshev steps on S_q after the nodal correction

// out ~ K_uu^-1 (b - tu) per network: DG_VEL_DEGREE Chebyshev steps from
// zero with the simplex-block Jacobi (intermediate iterates in w.va / w.vb)
template <int d, typename T>
void dg_vsolve(dpp_precond pc, const DGWork<T> &w, DGVec<T> b, const T *tu, DGOut<T> out, hipStream_t s) {
  dpp_problem P = pc->prob;
  const long nc = P->g.nc, NU = (d + 1) * d;
  const dim3 gv(blocks_for(nc, DGV_BS / NU), 2);
  const DGGeo geo = dg_geo(P);
  double th[2], de[2], sig[2], rho[2];
  for (int q = 0; q < 2; ++q) {
    th[q] = 0.5 * (pc->dgvhi[q] + pc->dgvlo[q]);
    de[q] = 0.5 * (pc->dgvhi[q] - pc->dgvlo[q]);
    sig[q] = th[q] / de[q];
    rho[q] = 1.0 / sig[q];
  }
  T *buf[2] = {w.va, w.vb};
  DGVec<T> xin{nullptr, 0}, xprev{nullptr, 0};
  for (int k = 0; k < DG_VEL_DEGREE; ++k) {
    Sc2 c1{{0, 0}}, c2{{0, 0}};
    for (int q = 0; q < 2; ++q) {
      if (k == 0) {
        c2.v[q] = 1.0 / th[q];
      } else {
        const double rn = 1.0 / (2.0 * sig[q] - rho[q]);
        c1.v[q] = rn * rho[q];
        c2.v[q] = 2.0 * rn / de[q];
        rho[q] = rn;
      }
    }
    // x_(k+1) overwrites x_(k-1) (buf alternates), the last one goes to out
    const DGOut<T> o = k + 1 == DG_VEL_DEGREE ? out : DGOut<T>{buf[k & 1], nc * NU};
    // bytes: the packed block inverses; b (less tu) read, x' written; x read
    // after the first step (x_0 = 0), x_(k-1) after the second, with the
    // coefficients
    const double vecs = 2.0 + (tu ? 1.0 : 0.0) + (k > 0 ? 1.0 : 0.0) + (k > 1 ? 1.0 : 0.0);
    ProfScope ps(PF_DG_VEL,
                 2.0 * sizeof(T) * ((double)nc * dg_npk(d) + vecs * nc * NU) +
                     (k > 0 ? 2.0 * 8.0 * nc : 0.0), s);
    k_dg_vcheb<d, T><<<gv, DGV_BS, 0, s>>>(geo, P->dgtab.as<double>(), nc, P->k1.as<double>(),
                                           P->k2.as<double>(), w.binv, b, tu, xin, o, xprev, c1, c2, false);
    xprev = xin;
    xin = DGVec<T>{o.base, o.stride};
  }
  check_launch("DG velocity solve");
}

void dg_sumsq(dpp_precond pc, const double *x, long n, double *ssd, hipStream_t s) {
  k_dg_sumsq<<<dim3(DG_RB, 2), 256, 0, s>>>(x, n, pc->dgpart.as<double>());
  k_dg_sumsq_fin<<<1, 256, 0, s>>>(pc->dgpart.as<double>(), ssd);
}

template <int d>
void dg_setup_impl(dpp_precond pc, hipStream_t s) {
  dpp_problem P = pc->prob;
  const Grid &g = P->g;
  const long nc = g.nc, nslot = P->nslot, NU = (d + 1) * d;
  // the nodal CG-VMS problem of the same box and coefficients (pressure data
  // do not enter the operator) and its preconditioner: the coarse level
  dpp_box box{};
  box.dim = d;
  for (int a = 0; a < d; ++a) {
    box.n[a] = g.n[a];
    box.L[a] = g.h[a] * g.n[a];
  }
  box.elem = ELEM_P1;
  pc->dgzero.alloc(sizeof(double) * g.N);
  DPP_HIP(hipMemsetAsync(pc->dgzero.ptr, 0, sizeof(double) * g.N, s));
  dpp_params prm{};
  prm.mu = P->mu;
  prm.k1 = P->k1.as<double>();
  prm.k2 = P->k2.as<double>();
  prm.beta = P->beta;
  prm.beta_cells = P->beta_per_cell ? P->betac.as<double>() : nullptr;
  prm.p0_1 = prm.p0_2 = pc->dgzero.as<double>();
  pc->dgcg.reset(new dpp_problem_s());
  assemble_problem(pc->dgcg.get(), &box, &prm, s);
  pc->dgpc = new dpp_precond_s();
  pc->dgpc->prob = pc->dgcg.get();
  pc->dgpc->opts = pc->opts;
  // in 2D the nodal cycle's small levels are launch-bound: by default its
  // coarsest level takes up to DG_NODAL_COARSE_2D nodes (solved exactly)
  if (pc->opts.coarse_max == 0 && d == 2) pc->dgpc->opts.coarse_max = DG_NODAL_COARSE_2D;
  precond_setup(pc->dgpc, s);
  // DG level: diagonals, work vectors, Chebyshev bounds from power steps
  pc->dgdu.alloc(sizeof(double) * 2 * nc * NU);
  pc->dgds.alloc(sizeof(double) * 2 * nslot);
  for (DBuf *b : {&pc->dgrh, &pc->dgza, &pc->dgzb, &pc->dgd}) b->alloc(sizeof(double) * 2 * nslot);
  pc->dgtu.alloc(sizeof(double) * 2 * nc * NU);
  for (DBuf *b : {&pc->dgva, &pc->dgvb, &pc->dgyu}) b->alloc(sizeof(double) * 2 * nc * NU);
  pc->dgbinv.alloc(sizeof(double) * 2 * nc * dg_npk(d));
  pc->dgcb.alloc(sizeof(double) * 2 * g.N);
  pc->dgcx.alloc(sizeof(double) * 2 * g.N);
  pc->dgpart.alloc(sizeof(double) * 2 * DG_RB + 2 * sizeof(double));
  k_dg_diag_u<d><<<dim3(blocks_for(nc * NU, 256), 2), 256, 0, s>>>(nc, P->dgA.as<double>(), pc->dgdu.as<double>());
  k_dg_diag_s<d><<<dim3(blocks_for(nslot, 256), 2), 256, 0, s>>>(nc, P->dgA.as<double>(), P->dgnb.as<int>(),
                                                                pc->dgdu.as<double>(), pc->dgds.as<double>());
  check_launch("DG diagonals");
  double *x = pc->dgza.as<double>(), *y = pc->dgzb.as<double>();
  double *ssd = pc->dgpart.as<double>() + 2 * DG_RB;
  const dim3 gv(blocks_for(nslot, 256), 2);
  k_dg_hash<<<gv, 256, 0, s>>>(x, nslot);
  dg_sumsq(pc, x, nslot, ssd, s);
  k_dg_scale<<<gv, 256, 0, s>>>(x, nslot, ssd);
  const dpp_solve_opts &o = pc->opts;
  for (int it = 0; it < o.power_iters; ++it) {
    dg_s_apply<d>(pc, x, y, pc->dgds.as<double>(), s);
    dg_sumsq(pc, y, nslot, ssd, s);
    k_dg_scale<<<gv, 256, 0, s>>>(y, nslot, ssd);
    std::swap(x, y);
  }
  check_launch("DG power steps");
  double ss[2] = {0.0, 0.0};
  DPP_HIP(hipMemcpyAsync(ss, ssd, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  // velocity block: simplex-block inverses and the interval of Binv K_uu
  k_dg_binv<d><<<dim3(blocks_for(nc, 64), 2), 64, 0, s>>>(nc, P->dgA.as<double>(), pc->dgbinv.as<double>());
  check_launch("DG velocity blocks");
  {
    const long nu = nc * NU;
    double *vx = pc->dgva.as<double>(), *vy = pc->dgvb.as<double>();
    const dim3 gu(blocks_for(nu, 256), 2), gb(blocks_for(nc, DGV_BS / NU), 2);
    k_dg_hash<<<gu, 256, 0, s>>>(vx, nu);
    dg_sumsq(pc, vx, nu, ssd, s);
    k_dg_scale<<<gu, 256, 0, s>>>(vx, nu, ssd);
    for (int it = 0; it < o.power_iters; ++it) {
      k_dg_vcheb<d, double><<<gb, DGV_BS, 0, s>>>(
          dg_geo(P), P->dgtab.as<double>(), nc, P->k1.as<double>(), P->k2.as<double>(),
          pc->dgbinv.as<double>(), DGVec<double>{nullptr, 0}, nullptr, DGVec<double>{vx, nu}, DGOut<double>{vy, nu},
          DGVec<double>{nullptr, 0}, Sc2{{0, 0}}, Sc2{{0, 0}}, true);
      dg_sumsq(pc, vy, nu, ssd, s);
      k_dg_scale<<<gu, 256, 0, s>>>(vy, nu, ssd);
      std::swap(vx, vy);
    }
    check_launch("DG velocity power steps");
    double sv[2] = {0.0, 0.0};
    DPP_HIP(hipMemcpyAsync(sv, ssd, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    DPP_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < 2; ++q) {
      pc->dgvhi[q] = o.cheb_hi_factor * std::sqrt(sv[q]);
      pc->dgvlo[q] = DG_VEL_LO_FRAC * pc->dgvhi[q];
      DPP_CHECK(std::isfinite(pc->dgvhi[q]) && pc->dgvhi[q] > 0.0, DPP_ERR_NUMERIC,
                "DG velocity-block eigenvalue estimate is not positive");
    }
  }
  const double lo_frac = o.cheb_lo_frac > 0.0 ? o.cheb_lo_frac : (d == 3 ? 0.1 : 0.3);
  for (int q = 0; q < 2; ++q) {
    pc->dghi[q] = o.cheb_hi_factor * std::sqrt(ss[q]);
    pc->dglo[q] = lo_frac * pc->dghi[q];
    DPP_CHECK(std::isfinite(pc->dghi[q]) && pc->dghi[q] > 0.0, DPP_ERR_NUMERIC,
              "DG Schur eigenvalue estimate is not positive");
  }
}

template <int d, typename T>
void dg_apply_impl(dpp_precond pc, const T *r, T *z, hipStream_t s) {
  dpp_problem P = pc->prob;
  const Grid &g = P->g;
  const long nc = g.nc, nslot = P->nslot;
  const DGWork<T> w = dg_work(pc, T());
  const double *k1 = P->k1.as<double>(), *k2 = P->k2.as<double>(), *bc = dg_betac(P);
  const DGGeo geo = dg_geo(P);
  const dim3 gp(blocks_for(nslot, 256), 2), gs(blocks_for(nc, 256), 2);
  const long NU = (d + 1) * d, vstride = (d + 1) * nslot;  // network stride of the ABI vector
  const double vb = sizeof(T);                               // bytes per stored vector value
  dg_vsolve<d, T>(pc, w, DGVec<T>{r + off_u(d, nslot, 0), vstride}, nullptr, DGOut<T>{w.yu, nc * NU}, s);
  // algorithmic bytes of the pressure-side launches (2 networks, matrix-free):
  // vectors once, the coefficients where they enter
  const double b_tu = 2.0 * vb * ((double)nslot + (double)nc * NU);  // zp in, tu out
  {
    ProfScope ps(PF_DG_PRES, 2.0 * vb * ((double)nc * NU + 2.0 * nslot), s);
    k_dg_rhat<d, T><<<gs, 256, 0, s>>>(geo, nc, nslot, w.yu, r, w.rh);
  }
  // coarse correction on the nodes, back to the slots
  {
    ProfScope ps(PF_DG_TRANSFER, 2.0 * vb * ((double)nslot + (double)g.N), s);
    k_dg_restrict<d, T><<<dim3(blocks_for(g.N, 256), 2), 256, 0, s>>>(dev(g), nslot, w.rh, w.cb);
  }
  dg_vcycle(pc->dgpc, w.cb, w.cx, s);
  T *cur = w.za, *oth = w.zb;
  {
    ProfScope ps(PF_DG_TRANSFER, 2.0 * vb * ((double)nslot + (double)g.N), s);
    k_dg_prolong<d, T><<<gp, 256, 0, s>>>(dev(g), nc, nslot, w.cx, cur);
  }
  // Chebyshev post-smoothing on S_q (Saad, Alg. 12.1 with the diagonal of S_q)
  const int deg = DG_PRES_DEGREE;
  double sig[2], rho[2], th[2], de[2];
  for (int q = 0; q < 2; ++q) {
    th[q] = 0.5 * (pc->dghi[q] + pc->dglo[q]);
    de[q] = 0.5 * (pc->dghi[q] - pc->dglo[q]);
    sig[q] = th[q] / de[q];
    rho[q] = 1.0 / sig[q];
  }
  for (int k = 0; k < deg; ++k) {
    Sc2 c1{{0, 0}}, c2{{0, 0}};
    for (int q = 0; q < 2; ++q) {
      if (k == 0) {
        c2.v[q] = 1.0 / th[q];
      } else {
        const double rn = 1.0 / (2.0 * sig[q] - rho[q]);
        c1.v[q] = rn * rho[q];
        c2.v[q] = 2.0 * rn / de[q];
        rho[q] = rn;
      }
    }
    {
      // w = D_u^-1 K_up x: x and D_u^-1 in, w out
      ProfScope ps(PF_DG_PRES, b_tu + 2.0 * vb * nc * NU, s);
      k_dg_tu<d, T><<<gs, 256, 0, s>>>(geo, nc, nslot, cur, w.du, w.tu);
    }
    {
      // S_q rows: w, x, diag, b, dd (read after the first step), dd and x'
      // written, the coefficients
      ProfScope ps(PF_DG_PRES,
                   2.0 * vb * ((double)nc * NU + (k > 0 ? 6.0 : 5.0) * nslot) + 2.0 * dg_coef_bytes(P), s);
      k_dg_sp<d, T><<<gs, 256, 0, s>>>(geo, nc, nslot, k1, k2, bc, P->beta, w.tu, cur, oth, w.ds, w.rh, w.dd, c1,
                                       c2, true);
    }
    std::swap(cur, oth);
  }
  // z_u ~ K_uu^-1 (r_u - K_up z_p), z_p
  {
    ProfScope ps(PF_DG_PRES, b_tu, s);
    k_dg_tu<d, T><<<gs, 256, 0, s>>>(geo, nc, nslot, cur, nullptr, w.tu);
  }
  dg_vsolve<d, T>(pc, w, DGVec<T>{r + off_u(d, nslot, 0), vstride}, w.tu, DGOut<T>{z + off_u(d, nslot, 0), vstride},
                  s);
  {
    ProfScope ps(PF_DG_PRES, 2.0 * 2.0 * vb * nslot, s);
    k_dg_copyp<d, T><<<gp, 256, 0, s>>>(nslot, cur, z);
  }
  check_launch("DG fieldsplit");
}

__global__ void k_dg_to32(const double *__restrict__ x, float *__restrict__ y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void k_dg_to64(const float *__restrict__ x, double *__restrict__ y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

}  // namespace

void dg_precond_setup(dpp_precond pc, hipStream_t s) {
  if (pc->prob->g.dim == 3)
    dg_setup_impl<3>(pc, s);
  else
    dg_setup_impl<2>(pc, s);
}

void dg_make32(dpp_precond pc, hipStream_t s) {
  if (pc->dg32) return;
  dpp_problem P = pc->prob;
  const int d = P->g.dim;
  const long nc = P->g.nc, nslot = P->nslot, NU = (d + 1) * d, N = P->g.N;
  auto conv = [&](const DBuf &src, DBuf &dst, long n) {
    dst.alloc(sizeof(float) * n);
    k_dg_to32<<<std::min(2048, blocks_for(n, 256)), 256, 0, s>>>(src.as<double>(), dst.as<float>(), n);
  };
  conv(pc->dgdu, pc->dgdu32, 2 * nc * NU);
  conv(pc->dgds, pc->dgds32, 2 * nslot);
  conv(pc->dgbinv, pc->dgbinv32, 2 * nc * dg_npk(d));
  for (DBuf *b : {&pc->dgrh32, &pc->dgza32, &pc->dgzb32, &pc->dgd32}) b->alloc(sizeof(float) * 2 * nslot);
  for (DBuf *b : {&pc->dgtu32, &pc->dgva32, &pc->dgvb32, &pc->dgyu32}) b->alloc(sizeof(float) * 2 * nc * NU);
  for (DBuf *b : {&pc->dgcb32, &pc->dgcx32}) b->alloc(sizeof(float) * 2 * N);
  for (DBuf *b : {&pc->dgr32, &pc->dgz32}) b->alloc(sizeof(float) * P->ndof());
  check_launch("DG fp32 copies");
  precond_make32(pc->dgpc, s);
  pc->dg32 = true;
}

void dg_precond_apply(dpp_precond pc, const double *r, double *z, bool fp32, hipStream_t s) {
  const int d = pc->prob->g.dim;
  if (!fp32) {
    if (d == 3)
      dg_apply_impl<3, double>(pc, r, z, s);
    else
      dg_apply_impl<2, double>(pc, r, z, s);
    return;
  }
  // FP32 preconditioner: the residual rounded once, the correction widened once
  DPP_CHECK(pc->dg32, DPP_ERR_ARG, "internal: DG FP32 preconditioner not set up");
  const long n = pc->prob->ndof();
  const int nb = std::min(2048, blocks_for(n, 256));
  k_dg_to32<<<nb, 256, 0, s>>>(r, pc->dgr32.as<float>(), n);
  if (d == 3)
    dg_apply_impl<3, float>(pc, pc->dgr32.as<float>(), pc->dgz32.as<float>(), s);
  else
    dg_apply_impl<2, float>(pc, pc->dgr32.as<float>(), pc->dgz32.as<float>(), s);
  k_dg_to64<<<nb, 256, 0, s>>>(pc->dgz32.as<float>(), z, n);
  check_launch("DG fieldsplit (fp32)");
}

}  // namespace dpp
