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

// y = K x (bsub null) or y = bsub - K x: one thread per (network, simplex,
// local unknown); row r of every block is SB contiguous values.
template <int d>
__global__ __launch_bounds__(256) void k_dg_spmv(long nc, long nslot, const double *__restrict__ A,
                                                 const double *__restrict__ B, const int *__restrict__ nbr,
                                                 const double *__restrict__ x, const double *__restrict__ bsub,
                                                 double *__restrict__ y) {
  constexpr int SB = dg_sb(d);
  constexpr int NB = d + 2;
  constexpr int NU = (d + 1) * d;
  const int q = blockIdx.y;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * SB) return;
  const long e = t / SB;
  const int r = (int)(t % SB);
  const long ou = off_u(d, nslot, q), op = off_p(d, nslot, q);
  const double *Ar = A + ((size_t)q * nc + e) * NB * SB * SB + (size_t)r * SB;
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const long s = b == 0 ? e : nbr[e * (d + 1) + b - 1];
    if (s < 0) continue;
    const double *Ab = Ar + (size_t)b * SB * SB;
    const double *xu = x + ou + s * NU, *xp = x + op + s * (d + 1);
#pragma unroll
    for (int c = 0; c < NU; c += 2) {
      double a0, a1, x0, x1;
      ld2(Ab + c, a0, a1);
      ld2(xu + c, x0, x1);
      acc += a0 * x0 + a1 * x1;
    }
#pragma unroll
    for (int c = 0; c <= d; ++c) acc += Ab[NU + c] * xp[c];
  }
  long row;
  if (r < NU) {
    row = ou + e * NU + r;
  } else {
    const int a = r - NU;
    row = op + e * (d + 1) + a;
    // transfer to the other network's pressures of the same simplex
    const double *Be = B + (size_t)e * (d + 1) * (d + 1) + a * (d + 1);
    const double *xo = x + off_p(d, nslot, 1 - q) + e * (d + 1);
#pragma unroll
    for (int c = 0; c <= d; ++c) acc += Be[c] * xo[c];
  }
  y[row] = bsub ? bsub[row] - acc : acc;
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
  P->f.alloc(sizeof(double) * P->ndof());
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
  P->nnz = 2 * ((nc + interior) * (long)SB * SB + nc * (long)(d + 1) * (d + 1));
}

void dg_spmv(dpp_problem P, const double *x, const double *bsub, double *y, hipStream_t s) {
  const Grid &g = P->g;
  const int d = g.dim;
  const long nc = g.nc;
  const int SB = (d + 1) * (d + 1);
  const dim3 grid(blocks_for(nc * SB, 256), 2);
  ProfScope ps(PF_SPMV_K, 2.0 * 8.0 * ((double)nc * (d + 2) * SB * SB + (double)nc * (d + 1) * (d + 1)) +
                              8.0 * P->ndof() * (bsub ? 3.0 : 2.0), s);
  if (d == 3)
    k_dg_spmv<3><<<grid, 256, 0, s>>>(nc, P->nslot, P->dgA.as<double>(), P->dgB.as<double>(), P->dgnb.as<int>(),
                                      x, bsub, y);
  else
    k_dg_spmv<2><<<grid, 256, 0, s>>>(nc, P->nslot, P->dgA.as<double>(), P->dgB.as<double>(), P->dgnb.as<int>(),
                                      x, bsub, y);
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

}  // namespace dpp
