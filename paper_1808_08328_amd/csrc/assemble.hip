// Assembly of the CG-VMS four-field DPP system on the device.
//
// K entries follow eq. S4_cg_stiffness_matrix (CG-VMS weak form
// eq. CG_VMS_Weak_form, P1 on the Kuhn simplices of a structured box); f
// follows eq. S4_cg_rhs with the pressure data imposed weakly,
// -(w.n ; p0) over the boundary, p0 the P1 nodal interpolant.
//
// Storage: for every node a and every offset t of the node stencil St the
// 4d+5 distinct values of the node-pair block (a, a+o_t) are kept in
// structure-of-arrays form, kv[(v*NS + t)*ld + a] (v = value kind, see
// common.h; ld = N rounded up to 32).  Entries of pairs leaving the box are
// zero.  Each (a, t) is
// computed by one thread that sums the contributions of the simplices holding
// both nodes in a fixed order: no atomics, bit-reproducible.
#include "objects.h"

namespace dpp {

namespace {

// Axis permutations in lexicographic order: simplex s of a box cell visits
// the corner, then steps along perm[s][0], perm[s][1] (, perm[s][2]).
__device__ inline int perm_axis(int D, int s, int k) {
  if (D == 2) return (s == 0) ? k : 1 - k;
  const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  return P[s][k];
}

// Local vertex index of the corner-relative binary offset `bits` in simplex s,
// or -1 when it is not a vertex of that simplex.
template <int D>
__device__ inline int local_vertex(int s, int bits) {
  int mask = 0;
  if (bits == 0) return 0;
  for (int k = 0; k < D; ++k) {
    mask |= 1 << perm_axis(D, s, k);
    if (mask == bits) return k + 1;
  }
  return -1;
}

// Component c of grad(lambda_k) on simplex s with cell sizes h:
// lambda_0 = 1 - y_{p0}, lambda_k = y_{p(k-1)} - y_{pk}, lambda_D = y_{p(D-1)}.
template <int D>
__device__ inline double grad_lambda(int s, int k, int c, const double *h) {
  double g = 0.0;
  if (k >= 1 && perm_axis(D, s, k - 1) == c) g += 1.0 / h[c];
  if (k < D && perm_axis(D, s, k) == c) g -= 1.0 / h[c];
  return g;
}

struct Coef {
  const double *k1, *k2, *betac;
  double beta, mu;
  double h[3];
};

template <int D>
__global__ __launch_bounds__(256) void k_assemble(GridDev g, Coef cf, double *__restrict__ kv) {
  constexpr int NS = Tabs<D>::NS;
  constexpr int NV = nv_kinds(D);
  const long N = g.N;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * NS) return;
  const int t = (int)(idx / N);
  const long a = idx - (long)t * N;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  const int *o = TAB<D>.so[t];
  double uu[2] = {0, 0}, up[2][D], pu[2][D], pp[2] = {0, 0}, k12 = 0.0;
  for (int q = 0; q < 2; ++q)
    for (int c = 0; c < D; ++c) up[q][c] = pu[q][c] = 0.0;
  const bool valid = inside(g, ia[0] + o[0], ia[1] + o[1], ia[2] + o[2]);
  if (valid) {
    const double vol = (D == 3) ? cf.h[0] * cf.h[1] * cf.h[2] / 6.0 : cf.h[0] * cf.h[1] / 2.0;
    const double avg = vol / (D + 1);
    const double moff = vol / ((D + 1.0) * (D + 2.0));
    const int nper = (D == 3) ? 6 : 2;
    for (int sb = 0; sb < (1 << D); ++sb) {       // box cells around a
      int cc[3] = {0, 0, 0}, sa = sb, sbb = 0;
      bool ok = true;
      for (int ax = 0; ax < D; ++ax) {
        int bit = (sb >> ax) & 1;
        cc[ax] = ia[ax] - bit;
        if (cc[ax] < 0 || cc[ax] >= g.n[ax]) ok = false;
        int ob = bit + o[ax];                       // offset of b from the corner
        if (ob < 0 || ob > 1) ok = false;
        sbb |= (ob & 1) << ax;
      }
      if (!ok) continue;
      long hexid = cc[0] + (long)g.n[0] * (cc[1] + (long)g.n[1] * cc[2]);
      for (int s = 0; s < nper; ++s) {
        int la = local_vertex<D>(s, sa), lb = local_vertex<D>(s, sbb);
        if (la < 0 || lb < 0) continue;
        long e = hexid * nper + s;
        double ga[D], gb[D], gg = 0.0;
        for (int c = 0; c < D; ++c) {
          ga[c] = grad_lambda<D>(s, la, c, cf.h);
          gb[c] = grad_lambda<D>(s, lb, c, cf.h);
          gg += ga[c] * gb[c];
        }
        const double M = moff * (la == lb ? 2.0 : 1.0);
        const double bm = (cf.betac ? cf.betac[e] : cf.beta) / cf.mu;
        for (int q = 0; q < 2; ++q) {
          const double kk = q ? cf.k2[e] : cf.k1[e];
          uu[q] += 0.5 * (cf.mu / kk) * M;                 // 1/2 (w; mu/k u)
          for (int c = 0; c < D; ++c) {
            up[q][c] += -ga[c] * avg - 0.5 * gb[c] * avg;   // -(div w;p) - 1/2 (w;grad p)
            pu[q][c] += gb[c] * avg + 0.5 * ga[c] * avg;    // (q;div u) + 1/2 (grad q;u)
          }
          pp[q] += 0.5 * (kk / cf.mu) * vol * gg + bm * M;  // 1/2 (grad q;k/mu grad p) + (q;beta/mu p)
        }
        k12 += -bm * M;                                     // -(q1; beta/mu p2)
      }
    }
  }
  const size_t vs = (size_t)NS * g.ld;
  double *base = kv + (size_t)t * g.ld + a;
  for (int q = 0; q < 2; ++q) {
    base[kv_uu(D, q) * vs] = uu[q];
    for (int c = 0; c < D; ++c) {
      base[kv_up(D, q, c) * vs] = up[q][c];
      base[kv_pu(D, q, c) * vs] = pu[q][c];
    }
    base[kv_pp(D, q) * vs] = pp[q];
  }
  base[kv_12(D) * vs] = k12;
  (void)NV;
}

// Right-hand side, one thread per node: body-force terms
// 1/2 (w; gamma b) and 1/2 (grad q; k/mu gamma b) over the incident simplices,
// and -(w.n; p0) over the boundary facets holding the node.  On every face of
// the box the facets are the 2D Kuhn triangles of that face's grid (in-plane
// axes in ascending order).
template <int D>
__global__ __launch_bounds__(256) void k_rhs(GridDev g, Coef cf, const double *__restrict__ body,
                                             const double *__restrict__ p01,
                                             const double *__restrict__ p02, double *__restrict__ f) {
  const long N = g.N;
  long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  double fu[2][D], fp[2] = {0, 0};
  for (int q = 0; q < 2; ++q)
    for (int c = 0; c < D; ++c) fu[q][c] = 0.0;
  const long stride[3] = {1, (long)g.m[0], (long)g.m[0] * g.m[1]};
  if (body) {
    const double vol = (D == 3) ? cf.h[0] * cf.h[1] * cf.h[2] / 6.0 : cf.h[0] * cf.h[1] / 2.0;
    const double avg = vol / (D + 1);
    const int nper = (D == 3) ? 6 : 2;
    for (int sb = 0; sb < (1 << D); ++sb) {
      int cc[3] = {0, 0, 0};
      bool ok = true;
      for (int ax = 0; ax < D; ++ax) {
        cc[ax] = ia[ax] - ((sb >> ax) & 1);
        if (cc[ax] < 0 || cc[ax] >= g.n[ax]) ok = false;
      }
      if (!ok) continue;
      long hexid = cc[0] + (long)g.n[0] * (cc[1] + (long)g.n[1] * cc[2]);
      for (int s = 0; s < nper; ++s) {
        int la = local_vertex<D>(s, sb);
        if (la < 0) continue;
        long e = hexid * nper + s;
        for (int q = 0; q < 2; ++q) {
          const double kk = q ? cf.k2[e] : cf.k1[e];
          double acc = 0.0;
          for (int c = 0; c < D; ++c) {
            const double gb = body[e * D + c];
            fu[q][c] += 0.5 * gb * avg;                     // (w;gb) - 1/2 (mu/k w; k/mu gb)
            acc += grad_lambda<D>(s, la, c, cf.h) * gb;
          }
          fp[q] += 0.5 * (kk / cf.mu) * vol * acc;          // 1/2 (grad q; k/mu gb)
        }
      }
    }
  }
  for (int ax = 0; ax < D; ++ax) {
    for (int side = 0; side < 2; ++side) {
      if (ia[ax] != (side ? g.n[ax] : 0)) continue;
      const double nrm = side ? 1.0 : -1.0;
      double s1 = 0.0, s2 = 0.0;
      if (D == 2) {
        const int qa = 1 - ax;
        for (int dn = -1; dn <= 1; dn += 2) {
          int jq = ia[qa] + dn;
          if (jq < 0 || jq > g.n[qa]) continue;
          long b = a + dn * stride[qa];
          const double w = cf.h[qa] / 6.0;                  // |F| (1 + delta) / (d (d+1))
          s1 += w * (2.0 * p01[a] + p01[b]);
          s2 += w * (2.0 * p02[a] + p02[b]);
        }
      } else {
        const int pa = (ax == 0) ? 1 : 0, qa = (ax == 2) ? 1 : 2;
        const double w = cf.h[pa] * cf.h[qa] / 2.0 / 12.0;
        for (int sp = 0; sp < 2; ++sp)
          for (int sq = 0; sq < 2; ++sq) {
            int cp = ia[pa] - sp, cq = ia[qa] - sq;
            if (cp < 0 || cp >= g.n[pa] || cq < 0 || cq >= g.n[qa]) continue;
            long corner = a - sp * stride[pa] - sq * stride[qa];
            // triangle 0: (0,0),(1,0),(1,1); triangle 1: (0,0),(0,1),(1,1)
            for (int tri = 0; tri < 2; ++tri) {
              int vp[3] = {0, tri == 0 ? 1 : 0, 1}, vq[3] = {0, tri == 0 ? 0 : 1, 1};
              bool has = false;
              for (int v = 0; v < 3; ++v)
                if (vp[v] == sp && vq[v] == sq) has = true;
              if (!has) continue;
              for (int v = 0; v < 3; ++v) {
                long b = corner + vp[v] * stride[pa] + vq[v] * stride[qa];
                double wv = (b == a) ? 2.0 : 1.0;
                s1 += w * wv * p01[b];
                s2 += w * wv * p02[b];
              }
            }
          }
      }
      fu[0][ax] -= nrm * s1;
      fu[1][ax] -= nrm * s2;
    }
  }
  for (int q = 0; q < 2; ++q) {
    for (int c = 0; c < D; ++c) f[off_u(D, N, q) + (long)D * a + c] = fu[q][c];
    f[off_p(D, N, q) + a] = fp[q];
  }
}

// ---- Q1 elements on box cells (stencil tags 12, 13): the [Q1 + Q1]^2 rows
// of the element table with the same block entries, integrated exactly.  The
// integrals over a cell are products of one-dimensional integrals on its
// edges (length h, phi_0 = 1 - t, phi_1 = t): mass h (1 + delta_ij)/6,
// stiffness (2 delta_ij - 1)/h, int phi_i' phi_j = i - 1/2, int phi_i = h/2,
// int phi_i' = 2i - 1.  A node's local coordinate in a cell is one bit per axis.
__device__ inline double q1_mass1(int i, int j, double h) { return h * (i == j ? 2.0 : 1.0) / 6.0; }
__device__ inline double q1_stiff1(int i, int j, double h) { return (i == j ? 1.0 : -1.0) / h; }

template <int D>
__global__ __launch_bounds__(256) void k_assemble_q1(GridDev g, Coef cf, double *__restrict__ kv) {
  constexpr int d = dim_of(D);
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * NS) return;
  const int t = (int)(idx / N);
  const long a = idx - (long)t * N;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  const int *o = TAB<D>.so[t];
  double uu[2] = {0, 0}, up[2][d], pu[2][d], pp[2] = {0, 0}, k12 = 0.0;
  for (int q = 0; q < 2; ++q)
    for (int c = 0; c < d; ++c) up[q][c] = pu[q][c] = 0.0;
  if (inside(g, ia[0] + o[0], ia[1] + o[1], ia[2] + o[2])) {
    for (int sb = 0; sb < (1 << d); ++sb) {  // box cells around a, fixed order
      int cc[3] = {0, 0, 0}, la[3] = {0, 0, 0}, lb[3] = {0, 0, 0};
      bool ok = true;
      for (int ax = 0; ax < d; ++ax) {
        la[ax] = (sb >> ax) & 1;          // a's local coordinate in the cell
        cc[ax] = ia[ax] - la[ax];
        lb[ax] = la[ax] + o[ax];          // the neighbour's
        if (cc[ax] < 0 || cc[ax] >= g.n[ax] || lb[ax] < 0 || lb[ax] > 1) ok = false;
      }
      if (!ok) continue;
      const long e = cc[0] + (long)g.n[0] * (cc[1] + (long)g.n[1] * cc[2]);
      double m1[3], M = 1.0;
      for (int ax = 0; ax < d; ++ax) {
        m1[ax] = q1_mass1(la[ax], lb[ax], cf.h[ax]);
        M *= m1[ax];
      }
      double St = 0.0, cab[d], cba[d];
      for (int c = 0; c < d; ++c) {
        double rest = 1.0;
        for (int x = 0; x < d; ++x)
          if (x != c) rest *= m1[x];
        St += q1_stiff1(la[c], lb[c], cf.h[c]) * rest;
        cab[c] = (la[c] ? 0.5 : -0.5) * rest;   // int (d_c psi_a) psi_b
        cba[c] = (lb[c] ? 0.5 : -0.5) * rest;   // int psi_a (d_c psi_b)
      }
      const double bm = (cf.betac ? cf.betac[e] : cf.beta) / cf.mu;
      for (int q = 0; q < 2; ++q) {
        const double kk = q ? cf.k2[e] : cf.k1[e];
        uu[q] += 0.5 * (cf.mu / kk) * M;                 // 1/2 (w; mu/k u)
        for (int c = 0; c < d; ++c) {
          up[q][c] += -cab[c] - 0.5 * cba[c];            // -(div w;p) - 1/2 (w;grad p)
          pu[q][c] += cba[c] + 0.5 * cab[c];             // (q;div u) + 1/2 (grad q;u)
        }
        pp[q] += 0.5 * (kk / cf.mu) * St + bm * M;       // 1/2 (grad q;k/mu grad p) + (q;beta/mu p)
      }
      k12 += -bm * M;                                    // -(q1; beta/mu p2)
    }
  }
  const size_t vs = (size_t)NS * g.ld;
  double *base = kv + (size_t)t * g.ld + a;
  for (int q = 0; q < 2; ++q) {
    base[kv_uu(d, q) * vs] = uu[q];
    for (int c = 0; c < d; ++c) {
      base[kv_up(d, q, c) * vs] = up[q][c];
      base[kv_pu(d, q, c) * vs] = pu[q][c];
    }
    base[kv_pp(d, q) * vs] = pp[q];
  }
  base[kv_12(d) * vs] = k12;
}

// Right-hand side with Q1 box cells, one thread per node: body-force terms
// 1/2 (w; gamma b) and 1/2 (grad q; k/mu gamma b) over the cells around the
// node, and -(w.n; p0) over the cell faces on the box boundary that hold it
// (p0 by its Q1 interpolant on the face: the face mass of the other axes).
template <int D>
__global__ __launch_bounds__(256) void k_rhs_q1(GridDev g, Coef cf, const double *__restrict__ body,
                                                const double *__restrict__ p01,
                                                const double *__restrict__ p02,
                                                double *__restrict__ f) {
  constexpr int d = dim_of(D);
  const long N = g.N;
  long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  double fu[2][d], fp[2] = {0, 0};
  for (int q = 0; q < 2; ++q)
    for (int c = 0; c < d; ++c) fu[q][c] = 0.0;
  const long stride[3] = {1, (long)g.m[0], (long)g.m[0] * g.m[1]};
  double mean = 1.0;  // int psi_a over a cell
  for (int ax = 0; ax < d; ++ax) mean *= 0.5 * cf.h[ax];
  for (int sb = 0; sb < (1 << d); ++sb) {
    int cc[3] = {0, 0, 0}, la[3] = {0, 0, 0};
    bool ok = true;
    for (int ax = 0; ax < d; ++ax) {
      la[ax] = (sb >> ax) & 1;
      cc[ax] = ia[ax] - la[ax];
      if (cc[ax] < 0 || cc[ax] >= g.n[ax]) ok = false;
    }
    if (!ok) continue;
    const long e = cc[0] + (long)g.n[0] * (cc[1] + (long)g.n[1] * cc[2]);
    if (body) {
      for (int q = 0; q < 2; ++q) {
        const double kk = q ? cf.k2[e] : cf.k1[e];
        double acc = 0.0;
        for (int c = 0; c < d; ++c) {
          const double gb = body[e * d + c];
          fu[q][c] += 0.5 * gb * mean;                   // (w;gb) - 1/2 (mu/k w; k/mu gb)
          double dm = la[c] ? 1.0 : -1.0;                // int d_c psi_a
          for (int x = 0; x < d; ++x)
            if (x != c) dm *= 0.5 * cf.h[x];
          acc += dm * gb;
        }
        fp[q] += 0.5 * (kk / cf.mu) * acc;               // 1/2 (grad q; k/mu gb)
      }
    }
    const long corner = a - la[0] * stride[0] - la[1] * stride[1] - la[2] * stride[2];
    for (int ax = 0; ax < d; ++ax) {
      const int side = la[ax];
      if (cc[ax] != (side ? g.n[ax] - 1 : 0)) continue;  // face not on the box boundary
      const double nrm = side ? 1.0 : -1.0;
      double s1 = 0.0, s2 = 0.0;
      for (int vb = 0; vb < (1 << d); ++vb) {
        if (((vb >> ax) & 1) != side) continue;          // vertices of that face
        double w = 1.0;
        long b = corner;
        for (int x = 0; x < d; ++x) {
          const int lbx = (vb >> x) & 1;
          b += lbx * stride[x];
          if (x != ax) w *= q1_mass1(la[x], lbx, cf.h[x]);
        }
        s1 += w * p01[b];
        s2 += w * p02[b];
      }
      fu[0][ax] -= nrm * s1;
      fu[1][ax] -= nrm * s2;
    }
  }
  for (int q = 0; q < 2; ++q) {
    for (int c = 0; c < d; ++c) f[off_u(d, N, q) + (long)d * a + c] = fu[q][c];
    f[off_p(d, N, q) + a] = fp[q];
  }
}

// Velocity faces (section "Boundary conditions", eq. DG_GE_vBC): the
// prescribed normal velocities are essential conditions (w.n = 0 in the test
// space), imposed by elimination.  k_lift moves the known values out of the
// other rows, f -= K g over the prescribed DOFs (K_uu couples equal
// components, K_pu every component), and writes the data into their rows; it
// reads K before k_mask_bc.  One thread per node.
template <int D>
__global__ void k_lift(GridDev g, const double *__restrict__ kv, const double *__restrict__ ub1,
                       const double *__restrict__ ub2, double *__restrict__ f) {
  constexpr int d = dim_of(D);
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  const size_t vs = (size_t)NS * g.ld;
  for (int q = 0; q < 2; ++q) {
    if (!g.fix[q]) continue;
    const double *ub = q ? ub2 : ub1;
    const long ou = off_u(d, N, q), op = off_p(d, N, q);
    double fp = 0.0, fu[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < NS; ++t) {
      const int *o = TAB<D>.so[t];
      const int ib[3] = {ia[0] + o[0], ia[1] + o[1], ia[2] + o[2]};
      if (!inside(g, ib[0], ib[1], ib[2])) continue;
      const long b = a + lin(g, o[0], o[1], o[2]);
      for (int c = 0; c < d; ++c) {
        if (!u_fixed(g, q, c, ib)) continue;
        const double gv = ub[(long)d * b + c];
        fu[c] += kv[kv_uu(d, q) * vs + (size_t)t * g.ld + a] * gv;
        fp += kv[kv_pu(d, q, c) * vs + (size_t)t * g.ld + a] * gv;
      }
    }
    for (int c = 0; c < d; ++c)
      f[ou + d * a + c] = u_fixed(g, q, c, ia) ? ub[(long)d * a + c] : f[ou + d * a + c] - fu[c];
    f[op + a] -= fp;
  }
}

// Removes the prescribed velocity DOFs from the coupling blocks of the stored
// K: their K_up rows and K_pu columns become zeros (K_pu = -K_up^T still
// holds), so the Schur blocks, selfp and the half storage see the masked
// operator.  K_uu keeps its values (one scalar per node pair serves every
// component); the kernels that apply it mask the prescribed components.
template <int D>
__global__ void k_mask_bc(GridDev g, double *__restrict__ kv) {
  constexpr int d = dim_of(D);
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  const size_t vs = (size_t)NS * g.ld;
  for (int q = 0; q < 2; ++q) {
    if (!g.fix[q]) continue;
    for (int t = 0; t < NS; ++t) {
      const int *o = TAB<D>.so[t];
      const int ib[3] = {ia[0] + o[0], ia[1] + o[1], ia[2] + o[2]};
      for (int c = 0; c < d; ++c) {
        if (u_fixed(g, q, c, ia)) kv[kv_up(d, q, c) * vs + (size_t)t * g.ld + a] = 0.0;
        if (u_fixed(g, q, c, ib)) kv[kv_pu(d, q, c) * vs + (size_t)t * g.ld + a] = 0.0;
      }
    }
  }
}

// CSR export (test hook): one thread per node writes all 2d+2 rows of it.
// Prescribed velocity DOFs have identity rows and zero K_uu columns (their
// coupling values are stored zeros).
template <int D>
__global__ void k_export(GridDev g, const double *__restrict__ kv, const int64_t *__restrict__ rowptr,
                         int32_t *__restrict__ cols, double *__restrict__ vals) {
  constexpr int d = dim_of(D);
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  const size_t vs = (size_t)NS * g.ld;
  auto val = [&](int v, int t) { return kv[v * vs + (size_t)t * g.ld + a]; };
  auto nb = [&](int t, long &b) {
    const int *o = TAB<D>.so[t];
    if (!inside(g, ia[0] + o[0], ia[1] + o[1], ia[2] + o[2])) return false;
    b = a + lin(g, o[0], o[1], o[2]);
    return true;
  };
  for (int q = 0; q < 2; ++q) {
    for (int c = 0; c < d; ++c) {
      long row = off_u(d, N, q) + (long)d * a + c;
      int64_t w = rowptr[row];
      long b;
      const bool fixed_row = u_fixed(g, q, c, ia);
      for (int t = 0; t < NS; ++t)
        if (nb(t, b)) {
          const int *o = TAB<D>.so[t];
          const int ib[3] = {ia[0] + o[0], ia[1] + o[1], ia[2] + o[2]};
          double v = val(kv_uu(d, q), t);
          if (fixed_row) v = (b == a) ? 1.0 : 0.0;
          else if (u_fixed(g, q, c, ib)) v = 0.0;
          cols[w] = (int32_t)(off_u(d, N, q) + d * b + c);
          vals[w++] = v;
        }
      for (int t = 0; t < NS; ++t)
        if (nb(t, b)) { cols[w] = (int32_t)(off_p(d, N, q) + b); vals[w++] = val(kv_up(d, q, c), t); }
    }
    long row = off_p(d, N, q) + a;
    int64_t w = rowptr[row];
    long b;
    if (q == 1)
      for (int t = 0; t < NS; ++t)
        if (nb(t, b)) { cols[w] = (int32_t)(off_p(d, N, 0) + b); vals[w++] = val(kv_12(d), t); }
    for (int t = 0; t < NS; ++t)
      if (nb(t, b))
        for (int c = 0; c < d; ++c) {
          cols[w] = (int32_t)(off_u(d, N, q) + d * b + c);
          vals[w++] = val(kv_pu(d, q, c), t);
        }
    for (int t = 0; t < NS; ++t)
      if (nb(t, b)) { cols[w] = (int32_t)(off_p(d, N, q) + b); vals[w++] = val(kv_pp(d, q), t); }
    if (q == 0)
      for (int t = 0; t < NS; ++t)
        if (nb(t, b)) { cols[w] = (int32_t)(off_p(d, N, 1) + b); vals[w++] = val(kv_12(d), t); }
  }
}

template <int D>
int count_neighbours_host(const Grid &g, long a) {
  int ia[3] = {(int)(a % g.m[0]), (int)((a / g.m[0]) % g.m[1]), (int)(a / ((long)g.m[0] * g.m[1]))};
  int cnt = 0;
  for (int t = 0; t < Tabs<D>::NS; ++t) {
    const int *o = TAB<D>.so[t];
    bool ok = true;
    for (int ax = 0; ax < 3; ++ax) {
      int v = ia[ax] + o[ax];
      if (v < 0 || v >= g.m[ax]) ok = false;
    }
    cnt += ok;
  }
  return cnt;
}

// bad[0] = 1 when an entry is not finite, or (kind 1) not > 0, or (kind 2) < 0
__global__ void k_check_values(const double *v, long n, int kind, int *bad) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = v[i];
  const bool ok = fabs(x) < INFINITY && (kind != 1 || x > 0.0) && (kind != 2 || x >= 0.0);
  if (!ok) bad[0] = 1;
}

}  // namespace

long count_nnz(const Grid &g) {
  // node pairs (a, a+o) inside the box, summed over the stencil offsets
  long pairs = 0;
  auto count = [&](const int *o) {
    long c = 1;
    for (int ax = 0; ax < g.dim; ++ax) c *= (g.m[ax] - std::abs(o[ax]));
    return c;
  };
  DPP_TAG_SWITCH(g, (({ for (int t = 0; t < Tabs<D_>::NS; ++t) pairs += count(TAB<D_>.so[t]); })));
  return pairs * (g.dim == 3 ? 22 : 16);
}

__global__ void k_any_positive(const double *v, long n, int *hit) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && v[i] > 0.0) hit[0] = 1;
}

static bool any_positive(const double *p, long n, hipStream_t s) {
  DBuf flag(sizeof(int));
  DPP_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(int), s));
  k_any_positive<<<blocks_for(n, 256), 256, 0, s>>>(p, n, flag.as<int>());
  check_launch("any_positive");
  int h = 0;
  DPP_HIP(hipMemcpyAsync(&h, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  return h != 0;
}

enum CheckKind { FINITE = 0, POSITIVE = 1, NONNEGATIVE = 2 };

static void check_input(const double *p, long n, CheckKind kind, const char *name, hipStream_t s) {
  DBuf flag(sizeof(int));
  DPP_HIP(hipMemsetAsync(flag.ptr, 0, sizeof(int), s));
  k_check_values<<<blocks_for(n, 256), 256, 0, s>>>(p, n, (int)kind, flag.as<int>());
  check_launch("check_input");
  int h = 0;
  DPP_HIP(hipMemcpyAsync(&h, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  static const char *what[] = {"a non-finite value", "a non-finite or non-positive value",
                               "a non-finite or negative value"};
  DPP_CHECK(!h, DPP_ERR_NUMERIC, std::string(name) + " holds " + what[kind]);
}

void assemble_problem(dpp_problem P, const dpp_box *box, const dpp_params *prm, hipStream_t s) {
  DPP_CHECK(box && prm, DPP_ERR_ARG, "null box or params");
  DPP_CHECK(box->dim == 2 || box->dim == 3, DPP_ERR_ARG, "dim must be 2 or 3");
  DPP_CHECK(box->elem == ELEM_P1 || box->elem == ELEM_Q1 || box->elem == ELEM_DG, DPP_ERR_ARG,
            "elem must be 0 (P1 simplices), 1 (Q1 box cells) or 2 (DG-VMS on simplices)");
  for (int a = 0; a < box->dim; ++a) {
    DPP_CHECK(box->n[a] >= 1 && box->n[a] <= 4096, DPP_ERR_ARG, "cells per axis must be in 1..4096");
    DPP_CHECK(box->L[a] > 0.0, DPP_ERR_ARG, "box extent must be positive");
  }
  DPP_CHECK(prm->k1 && prm->k2 && prm->p0_1 && prm->p0_2, DPP_ERR_ARG, "null coefficient array");
  DPP_CHECK(prm->mu > 0.0, DPP_ERR_ARG, "mu must be positive");
  const bool dg = box->elem == ELEM_DG;
  // DG-VMS keeps the node grid of the simplices (boundary data, coefficients)
  Grid g = make_grid(box->dim, box->n, box->L, dg ? ELEM_P1 : box->elem);
  const int D = g.dim;
  // the stencil kernels index nodes and unknowns with 32-bit integers
  DPP_CHECK((2L * D + 2L) * g.N <= 2147483647L, DPP_ERR_ARG,
            "box too large: (2 dim + 2) x nodes must stay below 2^31");
  int NS = 0;
  DPP_TAG_SWITCH(g, (NS = Tabs<D_>::NS));
  DPP_CHECK((double)g.N * (2 * D + 2) < 2.0e9, DPP_ERR_ARG, "problem too large for 32-bit indices");
  check_input(prm->k1, g.nc, POSITIVE, "k1", s);
  check_input(prm->k2, g.nc, POSITIVE, "k2", s);
  check_input(prm->p0_1, g.N, FINITE, "p0_1", s);
  check_input(prm->p0_2, g.N, FINITE, "p0_2", s);
  if (prm->beta_cells) check_input(prm->beta_cells, g.nc, NONNEGATIVE, "beta_cells", s);
  if (prm->body) check_input(prm->body, g.nc * D, FINITE, "body", s);
  DPP_CHECK(std::isfinite(prm->beta) && prm->beta >= 0.0, DPP_ERR_ARG, "beta must be >= 0");

  if (dg) {
    if (prm->face_bc)
      for (int i = 0; i < 4 * D; ++i)
        DPP_CHECK(prm->face_bc[i] == 0, DPP_ERR_UNSUPPORTED, "DG-VMS problems take pressure faces only");
    // unknowns on vertex slots, 32-bit indices in the block kernels
    DPP_CHECK((2L * D + 2L) * (D + 1) * g.nc <= 2147483647L, DPP_ERR_ARG,
              "box too large: (2 dim + 2) x slots must stay below 2^31");
    P->g = g;
    P->mu = prm->mu;
    P->beta = prm->beta;
    P->beta_per_cell = prm->beta_cells != nullptr;
    dg_assemble(P, prm, s);
    return;
  }
  if (prm->face_bc) {
    for (int q = 0; q < 2; ++q)
      for (int fa = 0; fa < 2 * D; ++fa) {
        const int8_t v = prm->face_bc[q * 2 * D + fa];
        DPP_CHECK(v == 0 || v == 1, DPP_ERR_ARG, "face_bc entries must be 0 or 1");
        g.fix[q] |= v << fa;
      }
    DPP_CHECK((!g.fix[0] || prm->u_bc_1) && (!g.fix[1] || prm->u_bc_2), DPP_ERR_ARG,
              "u_bc_i is required for a network with velocity faces");
    if (g.fix[0]) check_input(prm->u_bc_1, g.N * D, FINITE, "u_bc_1", s);
    if (g.fix[1]) check_input(prm->u_bc_2, g.N * D, FINITE, "u_bc_2", s);
    // With velocity faces everywhere and no mass transfer the two networks
    // decouple and K has a constant-pressure kernel per network; the
    // pure-flux solve removes one shared constant only.
    if (pure_flux(g)) {
      const bool coupled = prm->beta_cells ? any_positive(prm->beta_cells, g.nc, s) : prm->beta > 0.0;
      DPP_CHECK(coupled, DPP_ERR_UNSUPPORTED,
                "velocity faces on every face of both networks need beta > 0 somewhere");
    }
  }
  P->g = g;
  P->mu = prm->mu;
  P->beta = prm->beta;
  P->beta_per_cell = prm->beta_cells != nullptr;
  P->ns = NS;
  P->nnz = count_nnz(g);
  P->kvals.alloc(sizeof(double) * (size_t)nv_kinds(D) * NS * padded(g.N));
  P->f.alloc(sizeof(double) * P->ndof());
  P->dinv.alloc(sizeof(double) * 2 * g.N);
  P->k1.alloc(sizeof(double) * g.nc);
  P->k2.alloc(sizeof(double) * g.nc);
  DPP_HIP(hipMemcpyAsync(P->k1.ptr, prm->k1, sizeof(double) * g.nc, hipMemcpyDeviceToDevice, s));
  DPP_HIP(hipMemcpyAsync(P->k2.ptr, prm->k2, sizeof(double) * g.nc, hipMemcpyDeviceToDevice, s));
  if (prm->beta_cells) {
    P->betac.alloc(sizeof(double) * g.nc);
    DPP_HIP(hipMemcpyAsync(P->betac.ptr, prm->beta_cells, sizeof(double) * g.nc,
                           hipMemcpyDeviceToDevice, s));
  }
  Coef cf{P->k1.as<double>(), P->k2.as<double>(), P->betac.as<double>(), prm->beta, prm->mu,
          {g.h[0], g.h[1], g.h[2]}};
  GridDev gd = dev(g);
  long work = g.N * NS;
  const int wb = blocks_for(work, 256), nbk = blocks_for(g.N, 256);
  double *kv = P->kvals.as<double>(), *fv = P->f.as<double>();
  switch (g.elem == ELEM_Q1 ? 10 + D : D) {
    case 3:
      k_assemble<3><<<wb, 256, 0, s>>>(gd, cf, kv);
      k_rhs<3><<<nbk, 256, 0, s>>>(gd, cf, prm->body, prm->p0_1, prm->p0_2, fv);
      break;
    case 2:
      k_assemble<2><<<wb, 256, 0, s>>>(gd, cf, kv);
      k_rhs<2><<<nbk, 256, 0, s>>>(gd, cf, prm->body, prm->p0_1, prm->p0_2, fv);
      break;
    case 13:
      k_assemble_q1<13><<<wb, 256, 0, s>>>(gd, cf, kv);
      k_rhs_q1<13><<<nbk, 256, 0, s>>>(gd, cf, prm->body, prm->p0_1, prm->p0_2, fv);
      break;
    default:
      k_assemble_q1<12><<<wb, 256, 0, s>>>(gd, cf, kv);
      k_rhs_q1<12><<<nbk, 256, 0, s>>>(gd, cf, prm->body, prm->p0_1, prm->p0_2, fv);
      break;
  }
  check_launch("assemble");
  make_up_table(P, s);
  if (g.fix[0] | g.fix[1]) {
    // essential normal velocities: lift with the full K, then mask its couplings
    DPP_TAG_SWITCH(g, (k_lift<D_><<<blocks_for(g.N, 256), 256, 0, s>>>(gd, P->kvals.as<double>(), prm->u_bc_1,
                                                                    prm->u_bc_2, P->f.as<double>())));
    DPP_TAG_SWITCH(g, (k_mask_bc<D_><<<blocks_for(g.N, 256), 256, 0, s>>>(gd, P->kvals.as<double>())));
    check_launch("velocity boundaries");
  }
  make_dinv(P, s);
  make_kh(P, s);
}

void export_csr(dpp_problem P, int64_t *rowptr, int32_t *cols, double *vals, hipStream_t s) {
  const Grid &g = P->g;
  const int D = g.dim;
  const long N = g.N, nd = P->ndof();
  std::vector<int64_t> rp(nd + 1, 0);
  std::vector<int> m(N);
  DPP_TAG_SWITCH(g, (({ for (long a = 0; a < N; ++a) m[a] = count_neighbours_host<D_>(g, a); })));
  long row = 0;
  for (int q = 0; q < 2; ++q) {
    for (long a = 0; a < N; ++a)
      for (int c = 0; c < D; ++c, ++row) rp[row + 1] = rp[row] + 2 * m[a];
    for (long a = 0; a < N; ++a, ++row) rp[row + 1] = rp[row] + (D + 2) * m[a];
  }
  DPP_CHECK(rp[nd] == P->nnz, DPP_ERR_HIP, "internal: CSR size mismatch");
  DPP_HIP(hipMemcpyAsync(rowptr, rp.data(), sizeof(int64_t) * (nd + 1), hipMemcpyHostToDevice, s));
  GridDev gd = dev(g);
  DPP_TAG_SWITCH(g, (k_export<D_><<<blocks_for(N, 256), 256, 0, s>>>(gd, P->kvals.as<double>(), rowptr,
                                                                   cols, vals)));
  check_launch("export_csr");
  DPP_HIP(hipStreamSynchronize(s));
}

}  // namespace dpp
