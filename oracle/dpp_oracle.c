/*
 * dpp_oracle.c -- CPU oracle for the CG-VMS four-field DPP system.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this code; the GPU library never does,
 * and this file shares no source with it.
 *
 * Plain FP64 C, written from the paper:
 *   - governing equations: two Darcy laws and two mass balances coupled by the
 *     mass-transfer term beta/mu (p1 - p2)   (eq. DG_GE_Darcy_BLM);
 *   - CG-VMS weak form B_stab = B_Gal - 1/2 (mu k^-1 w - grad q ;
 *     (k/mu)(mu k^-1 u + grad p)) per network, L_stab likewise
 *     (eq. CG_VMS_Weak_form; Galerkin part eq. VMS_classical_mixed_formulation);
 *   - resulting block entries of K and f (eqs. S4_cg_stiffness_matrix and
 *     S4_cg_rhs), pressures imposed weakly through -(w.n ; p0) on the boundary.
 *
 * Mesh: structured box, nodes i + (nx+1)(j + (ny+1)k); hexahedron h split into
 * 6 tetrahedra 6h+s (s = axis permutation in lexicographic order, vertices =
 * corner followed by unit steps along the permuted axes); square h split into
 * triangles 2h, 2h+1 with the same rule.
 *
 * Global unknown ordering: [u1 | p1 | u2 | p2], velocities node-major with the
 * d components interleaved (dof of u_i at node a, component c = d*a + c).
 *
 * Assembly is node-owned: each node sums, in a fixed order, the element
 * contributions of its incident cells into its own rows (deterministic).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXADJ 32

static const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int PERM2[2][2] = {{0, 1}, {1, 0}};

long or_num_nodes(int d, const int *n) {
  long N = 1;
  for (int a = 0; a < d; ++a) N *= (long)(n[a] + 1);
  return N;
}

long or_num_cells(int d, const int *n) {
  long c = (d == 3) ? 6 : 2;
  for (int a = 0; a < d; ++a) c *= (long)n[a];
  return c;
}

/* Node coordinates X[N*d] and cell vertex lists cells[nc*(d+1)]. */
void or_mesh(int d, const int *n, const double *L, double *X, int32_t *cells) {
  long N = or_num_nodes(d, n);
  int s1[3] = {1, n[0] + 1, (d == 3) ? (n[0] + 1) * (n[1] + 1) : 0};
  for (long id = 0; id < N; ++id) {
    long r = id;
    for (int a = 0; a < d; ++a) {
      long ia = r % (n[a] + 1);
      r /= (n[a] + 1);
      X[id * d + a] = (double)ia * (L[a] / n[a]);
    }
  }
  long nbox = 1;
  for (int a = 0; a < d; ++a) nbox *= n[a];
  int nper = (d == 3) ? 6 : 2;
  for (long h = 0; h < nbox; ++h) {
    int ijk[3] = {0, 0, 0};
    long r = h;
    for (int a = 0; a < d; ++a) {
      ijk[a] = (int)(r % n[a]);
      r /= n[a];
    }
    long corner = 0;
    for (int a = 0; a < d; ++a) corner += (long)ijk[a] * s1[a];
    for (int s = 0; s < nper; ++s) {
      const int *perm = (d == 3) ? PERM3[s] : PERM2[s];
      int32_t *cv = cells + (h * nper + s) * (d + 1);
      long v = corner;
      cv[0] = (int32_t)v;
      for (int st = 0; st < d; ++st) {
        v += s1[perm[st]];
        cv[st + 1] = (int32_t)v;
      }
    }
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* node -> cell incidence (incptr[N+1], inc[nc*nv]) and sorted node adjacency
 * (nodes sharing at least one cell, the node itself included); nv vertices per
 * cell (d + 1 for simplices, 2^d for box cells). */
void or_adjacency(int d, int nv, long N, long nc, const int32_t *cells, int64_t *incptr,
                  int32_t *inc, int32_t *adjcnt, int32_t *adj) {
  (void)d;
  memset(incptr, 0, sizeof(int64_t) * (N + 1));
  for (long e = 0; e < nc; ++e)
    for (int a = 0; a < nv; ++a) incptr[cells[e * nv + a] + 1]++;
  for (long i = 0; i < N; ++i) incptr[i + 1] += incptr[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * N);
  for (long i = 0; i < N; ++i) fill[i] = incptr[i];
  for (long e = 0; e < nc; ++e)
    for (int a = 0; a < nv; ++a) inc[fill[cells[e * nv + a]]++] = (int32_t)e;
  free(fill);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    int32_t buf[256];
    int m = 0;
    for (int64_t q = incptr[i]; q < incptr[i + 1]; ++q)
      for (int a = 0; a < nv; ++a) buf[m++] = cells[(long)inc[q] * nv + a];
    qsort(buf, m, sizeof(int32_t), cmp_i32);
    int u = 0;
    for (int t = 0; t < m; ++t)
      if (u == 0 || buf[t] != buf[u - 1]) buf[u++] = buf[t];
    adjcnt[i] = u;
    for (int t = 0; t < u; ++t) adj[i * MAXADJ + t] = buf[t];
  }
}

/* Row pointers of K for the pattern the bilinear form couples:
 * u_i row (a,c): u_i (b,c) and p_i (b) for b adjacent to a  -> 2m entries;
 * p_1 row a: u_1 (b,*), p_1 (b), p_2 (b)                    -> (d+2)m;
 * p_2 row a: p_1 (b), u_2 (b,*), p_2 (b)                    -> (d+2)m.
 * Returns nnz. */
int64_t or_rowptr(int d, long N, const int32_t *adjcnt, int64_t *rowptr) {
  long ndof = (long)(2 * d + 2) * N;
  rowptr[0] = 0;
  long row = 0;
  for (int net = 0; net < 2; ++net) {
    for (long a = 0; a < N; ++a)
      for (int c = 0; c < d; ++c, ++row) rowptr[row + 1] = rowptr[row] + 2 * adjcnt[a];
    for (long a = 0; a < N; ++a, ++row) rowptr[row + 1] = rowptr[row] + (d + 2) * adjcnt[a];
  }
  (void)ndof;
  return rowptr[row];
}

static inline long dof_u(int d, long N, int net, long a, int c) {
  return (net == 0 ? 0 : (long)(d + 1) * N) + (long)d * a + c;
}
static inline long dof_p(int d, long N, int net, long a) {
  return (net == 0 ? (long)d * N : (long)(2 * d + 1) * N) + a;
}

/* Column pattern, ascending within each row. */
void or_cols(int d, long N, const int32_t *adjcnt, const int32_t *adj, const int64_t *rowptr,
             int32_t *cols) {
#pragma omp parallel for schedule(static)
  for (long a = 0; a < N; ++a) {
    int m = adjcnt[a];
    const int32_t *nb = adj + a * MAXADJ;
    for (int net = 0; net < 2; ++net) {
      for (int c = 0; c < d; ++c) {
        int32_t *q = cols + rowptr[dof_u(d, N, net, a, c)];
        for (int t = 0; t < m; ++t) *q++ = (int32_t)dof_u(d, N, net, nb[t], c);
        for (int t = 0; t < m; ++t) *q++ = (int32_t)dof_p(d, N, net, nb[t]);
      }
      int32_t *q = cols + rowptr[dof_p(d, N, net, a)];
      if (net == 1)
        for (int t = 0; t < m; ++t) *q++ = (int32_t)dof_p(d, N, 0, nb[t]);
      for (int t = 0; t < m; ++t)
        for (int c = 0; c < d; ++c) *q++ = (int32_t)dof_u(d, N, net, nb[t], c);
      for (int t = 0; t < m; ++t) *q++ = (int32_t)dof_p(d, N, net, nb[t]);
      if (net == 0)
        for (int t = 0; t < m; ++t) *q++ = (int32_t)dof_p(d, N, 1, nb[t]);
    }
  }
}

/* P1 simplex geometry: volume |e| and barycentric gradients G[a][c]. */
static double simplex_geometry(int d, const double *X, const int32_t *cv, double G[4][3]) {
  double J[3][3] = {{0.0}}, Ji[3][3] = {{0.0}}, det;
  for (int r = 0; r < d; ++r)      /* J[r][a-1] = X_a[r] - X_0[r] */
    for (int a = 1; a <= d; ++a) J[r][a - 1] = X[(long)cv[a] * d + r] - X[(long)cv[0] * d + r];
  if (d == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
          J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  /* lambda_a (a >= 1) = row a-1 of J^-1 applied to (x - X_0) */
  for (int c = 0; c < d; ++c) G[0][c] = 0.0;
  for (int a = 1; a <= d; ++a)
    for (int c = 0; c < d; ++c) {
      G[a][c] = Ji[a - 1][c];
      G[0][c] -= Ji[a - 1][c];
    }
  double fact = (d == 2) ? 2.0 : 6.0;
  return fabs(det) / fact;
}

/* Add v to K(row, col): binary search of col in the sorted row. */
static inline void add_entry(const int64_t *rowptr, const int32_t *cols, double *vals, long row,
                             long col, double v) {
  int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) >> 1;
    if (cols[mid] == col) { vals[mid] += v; return; }
    if (cols[mid] < col) lo = mid + 1; else hi = mid - 1;
  }
  /* a missing slot means the pattern is wrong: poison the row */
  vals[rowptr[row]] = NAN;
}

/* Node index along axis a. */
static inline int node_axis(int d, const int *n, long id, int a) {
  for (int q = 0; q < a; ++q) id /= (n[q] + 1);
  (void)d;
  return (int)(id % (n[a] + 1));
}

/*
 * Assemble K (values into the given pattern) and f.
 * k1, k2: per cell; beta: per cell; body: gamma*b per cell [nc*d] or NULL;
 * p0_1, p0_2: nodal boundary pressures (P1 interpolant, integrated exactly).
 */
void or_assemble(int d, const int *n, long N, long nc, const double *X, const int32_t *cells,
                 const int64_t *incptr, const int32_t *inc, const int64_t *rowptr,
                 const int32_t *cols, double *vals, double *f, const double *k1,
                 const double *k2, const double *beta, double mu, const double *body,
                 const double *p0_1, const double *p0_2) {
  int nv = d + 1;
  memset(vals, 0, sizeof(double) * rowptr[(long)(2 * d + 2) * N]);
  memset(f, 0, sizeof(double) * (long)(2 * d + 2) * N);
#pragma omp parallel for schedule(dynamic, 256)
  for (long a = 0; a < N; ++a) {
    for (int64_t q = incptr[a]; q < incptr[a + 1]; ++q) {
      long e = inc[q];
      const int32_t *cv = cells + e * nv;
      int la = 0;
      while (cv[la] != a) ++la;
      double G[4][3];
      double vol = simplex_geometry(d, X, cv, G);
      double mass_off = vol / ((d + 1.0) * (d + 2.0)); /* int psi_a psi_b, a != b */
      double avg = vol / (d + 1.0);                    /* int psi_a */
      double bm = beta[e] / mu;
      for (int net = 0; net < 2; ++net) {
        double k = (net == 0) ? k1[e] : k2[e];
        for (int lb = 0; lb < nv; ++lb) {
          long b = cv[lb];
          double M = mass_off * (la == lb ? 2.0 : 1.0);
          double gg = 0.0;
          for (int c = 0; c < d; ++c) gg += G[la][c] * G[lb][c];
          /* velocity rows of node a */
          for (int c = 0; c < d; ++c) {
            long ra = dof_u(d, N, net, a, c);
            /* (w; mu/k u) - 1/2 (mu/k w; k/mu mu/k u)  -> 1/2 mu/k M */
            double gal_uu = (mu / k) * M, stab_uu = -0.5 * (mu / k) * M;
            add_entry(rowptr, cols, vals, ra, dof_u(d, N, net, b, c), gal_uu + stab_uu);
            /* -(div w; p) - 1/2 (mu/k w; k/mu grad p) */
            double gal_up = -G[la][c] * avg, stab_up = -0.5 * G[lb][c] * avg;
            add_entry(rowptr, cols, vals, ra, dof_p(d, N, net, b), gal_up + stab_up);
          }
          /* pressure row of node a */
          long rp = dof_p(d, N, net, a);
          for (int c = 0; c < d; ++c) {
            /* (q; div u) - 1/2 (-grad q; k/mu mu/k u) */
            double gal_pu = G[lb][c] * avg, stab_pu = 0.5 * G[la][c] * avg;
            add_entry(rowptr, cols, vals, rp, dof_u(d, N, net, b, c), gal_pu + stab_pu);
          }
          /* (q_i; beta/mu p_i) - 1/2 (-grad q; k/mu grad p) */
          double gal_pp = bm * M, stab_pp = 0.5 * (k / mu) * vol * gg;
          add_entry(rowptr, cols, vals, rp, dof_p(d, N, net, b), gal_pp + stab_pp);
          /* (q1 - q2; beta/mu (p1 - p2)): cross terms -beta/mu M */
          add_entry(rowptr, cols, vals, rp, dof_p(d, N, 1 - net, b), -bm * M);
        }
        /* right-hand side, body force part:
         * (w; gamma b) - 1/2 (mu/k w; k/mu gamma b) and -1/2 (-grad q; k/mu gamma b) */
        if (body) {
          double fp = 0.0;
          for (int c = 0; c < d; ++c) {
            double gb = body[e * d + c];
            f[dof_u(d, N, net, a, c)] += gb * avg - 0.5 * gb * avg;
            fp += 0.5 * (k / mu) * vol * G[la][c] * gb;
          }
          f[dof_p(d, N, net, a)] += fp;
        }
      }
      /* boundary part -(w.n; p0) over facets of this cell lying on the box
       * boundary that contain node a (facet = face opposite vertex lf). */
      for (int lf = 0; lf < nv; ++lf) {
        if (lf == la) continue;
        int fv[3], k = 0;
        for (int t = 0; t < nv; ++t)
          if (t != lf) fv[k++] = cv[t];
        for (int ax = 0; ax < d; ++ax) {
          for (int side = 0; side < 2; ++side) {
            int target = side ? n[ax] : 0;
            int on = 1;
            for (int t = 0; t < d; ++t)
              if (node_axis(d, n, fv[t], ax) != target) on = 0;
            if (!on) continue;
            double area;
            if (d == 2) {
              double dx = X[fv[1] * 2] - X[fv[0] * 2], dy = X[fv[1] * 2 + 1] - X[fv[0] * 2 + 1];
              area = sqrt(dx * dx + dy * dy);
            } else {
              double u[3], w[3], cr[3];
              for (int c = 0; c < 3; ++c) {
                u[c] = X[fv[1] * 3 + c] - X[fv[0] * 3 + c];
                w[c] = X[fv[2] * 3 + c] - X[fv[0] * 3 + c];
              }
              cr[0] = u[1] * w[2] - u[2] * w[1];
              cr[1] = u[2] * w[0] - u[0] * w[2];
              cr[2] = u[0] * w[1] - u[1] * w[0];
              area = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            }
            double nrm = side ? 1.0 : -1.0;
            /* int_F psi_a psi_b = |F| (1 + delta_ab) / (d (d+1)) on a (d-1)-simplex */
            double s1 = 0.0, s2 = 0.0;
            for (int t = 0; t < d; ++t) {
              double w = area * ((fv[t] == a) ? 2.0 : 1.0) / (d * (d + 1.0));
              s1 += w * p0_1[fv[t]];
              s2 += w * p0_2[fv[t]];
            }
            f[dof_u(d, N, 0, a, ax)] -= nrm * s1;
            f[dof_u(d, N, 1, a, ax)] -= nrm * s2;
          }
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------
 * Q1 elements on box cells (the [Q1 + Q1]^2 rows of the element table: the
 * same CG-VMS forms on quadrilaterals / hexahedra with (bi/tri)linear
 * functions).  Cell h = i + n_x(j + n_y k) is the box itself; its local
 * vertex v (bits v_a for the axes) is the node corner + sum_a v_a e_a.
 * ------------------------------------------------------------------------ */
long or_num_cells_q1(int d, const int *n) {
  long c = 1;
  for (int a = 0; a < d; ++a) c *= (long)n[a];
  return c;
}

void or_mesh_q1(int d, const int *n, const double *L, double *X, int32_t *cells) {
  long N = or_num_nodes(d, n);
  int s1[3] = {1, n[0] + 1, (d == 3) ? (n[0] + 1) * (n[1] + 1) : 0};
  for (long id = 0; id < N; ++id) {
    long r = id;
    for (int a = 0; a < d; ++a) {
      long ia = r % (n[a] + 1);
      r /= (n[a] + 1);
      X[id * d + a] = (double)ia * (L[a] / n[a]);
    }
  }
  long nbox = or_num_cells_q1(d, n);
  int nv = 1 << d;
  for (long h = 0; h < nbox; ++h) {
    long r = h, corner = 0;
    for (int a = 0; a < d; ++a) {
      corner += (r % n[a]) * s1[a];
      r /= n[a];
    }
    for (int v = 0; v < nv; ++v) {
      long id = corner;
      for (int a = 0; a < d; ++a)
        if ((v >> a) & 1) id += s1[a];
      cells[h * nv + v] = (int32_t)id;
    }
  }
}

/* One-dimensional integrals on an interval of length h with the linear
 * functions phi_0 = 1 - t, phi_1 = t (t = (x - x_0)/h):
 *   mass      int phi_i phi_j     = h (1 + delta_ij) / 6
 *   stiffness int phi_i' phi_j'   = (2 delta_ij - 1) / h
 *   mixed     int phi_i' phi_j    = (2 i - 1) / 2        (no h)
 *   mean      int phi_i           = h / 2
 *   slope     int phi_i'          = 2 i - 1 */
static double m1(int i, int j, double h) { return h * (i == j ? 2.0 : 1.0) / 6.0; }
static double s1d(int i, int j, double h) { return (i == j ? 1.0 : -1.0) / h; }
static double c1d(int i) { return i ? 0.5 : -0.5; }

/* Tensor-product integrals over the cell of local vertices a, b (bits per axis). */
static double q1_mass(int d, int a, int b, const double *h) {
  double v = 1.0;
  for (int x = 0; x < d; ++x) v *= m1((a >> x) & 1, (b >> x) & 1, h[x]);
  return v;
}
static double q1_stiff(int d, int a, int b, const double *h) {
  double v = 0.0;
  for (int c = 0; c < d; ++c) {
    double t = s1d((a >> c) & 1, (b >> c) & 1, h[c]);
    for (int x = 0; x < d; ++x)
      if (x != c) t *= m1((a >> x) & 1, (b >> x) & 1, h[x]);
    v += t;
  }
  return v;
}
/* int (d_c psi_a) psi_b */
static double q1_dmix(int d, int c, int a, int b, const double *h) {
  double v = c1d((a >> c) & 1);
  for (int x = 0; x < d; ++x)
    if (x != c) v *= m1((a >> x) & 1, (b >> x) & 1, h[x]);
  return v;
}
static double q1_mean(int d, const double *h) {
  double v = 1.0;
  for (int x = 0; x < d; ++x) v *= 0.5 * h[x];
  return v;
}
/* int d_c psi_a */
static double q1_dmean(int d, int c, int a, const double *h) {
  double v = ((a >> c) & 1) ? 1.0 : -1.0;
  for (int x = 0; x < d; ++x)
    if (x != c) v *= 0.5 * h[x];
  return v;
}

/*
 * Assemble K and f for Q1 box cells into the pattern of or_rowptr / or_cols
 * (same block entries as or_assemble, eq. S4_cg_stiffness_matrix and
 * eq. S4_cg_rhs, integrated exactly); p0 enters through its Q1 interpolant on
 * the boundary faces.  k1, k2, beta: per box cell; body: [nc*d] or NULL.
 */
void or_assemble_q1(int d, const int *n, const double *L, long N, const int32_t *cells,
                    const int64_t *incptr, const int32_t *inc, const int64_t *rowptr,
                    const int32_t *cols, double *vals, double *f, const double *k1,
                    const double *k2, const double *beta, double mu, const double *body,
                    const double *p0_1, const double *p0_2) {
  int nv = 1 << d;
  double h[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < d; ++a) h[a] = L[a] / n[a];
  memset(vals, 0, sizeof(double) * rowptr[(long)(2 * d + 2) * N]);
  memset(f, 0, sizeof(double) * (long)(2 * d + 2) * N);
  const double mean = q1_mean(d, h);
#pragma omp parallel for schedule(dynamic, 256)
  for (long a = 0; a < N; ++a) {
    for (int64_t q = incptr[a]; q < incptr[a + 1]; ++q) {
      long e = inc[q];
      const int32_t *cv = cells + e * nv;
      int la = 0;
      while (cv[la] != a) ++la;
      double bm = beta[e] / mu;
      for (int net = 0; net < 2; ++net) {
        double k = (net == 0) ? k1[e] : k2[e];
        for (int lb = 0; lb < nv; ++lb) {
          long b = cv[lb];
          double M = q1_mass(d, la, lb, h), St = q1_stiff(d, la, lb, h);
          for (int c = 0; c < d; ++c) {
            long ra = dof_u(d, N, net, a, c);
            /* (w; mu/k u) - 1/2 (mu/k w; k/mu mu/k u) */
            add_entry(rowptr, cols, vals, ra, dof_u(d, N, net, b, c), 0.5 * (mu / k) * M);
            /* -(div w; p) - 1/2 (w; grad p) */
            add_entry(rowptr, cols, vals, ra, dof_p(d, N, net, b),
                      -q1_dmix(d, c, la, lb, h) - 0.5 * q1_dmix(d, c, lb, la, h));
          }
          long rp = dof_p(d, N, net, a);
          for (int c = 0; c < d; ++c)
            /* (q; div u) + 1/2 (grad q; u) */
            add_entry(rowptr, cols, vals, rp, dof_u(d, N, net, b, c),
                      q1_dmix(d, c, lb, la, h) + 0.5 * q1_dmix(d, c, la, lb, h));
          /* (q; beta/mu p) + 1/2 (grad q; k/mu grad p); cross -beta/mu M */
          add_entry(rowptr, cols, vals, rp, dof_p(d, N, net, b), bm * M + 0.5 * (k / mu) * St);
          add_entry(rowptr, cols, vals, rp, dof_p(d, N, 1 - net, b), -bm * M);
        }
        if (body) {
          double fp = 0.0;
          for (int c = 0; c < d; ++c) {
            double gb = body[e * d + c];
            f[dof_u(d, N, net, a, c)] += 0.5 * gb * mean;
            fp += 0.5 * (k / mu) * q1_dmean(d, c, la, h) * gb;
          }
          f[dof_p(d, N, net, a)] += fp;
        }
      }
      /* -(w.n; p0) over the faces of this cell on the box boundary holding a:
       * face (axis ax, side s) = local vertices with bit ax equal to s */
      long r = e;
      int ce[3] = {0, 0, 0};
      for (int x = 0; x < d; ++x) {
        ce[x] = (int)(r % n[x]);
        r /= n[x];
      }
      for (int ax = 0; ax < d; ++ax) {
        int s = (la >> ax) & 1;
        if (ce[ax] != (s ? n[ax] - 1 : 0)) continue;
        double nrm = s ? 1.0 : -1.0, t1 = 0.0, t2 = 0.0;
        for (int lb = 0; lb < nv; ++lb) {
          if (((lb >> ax) & 1) != s) continue;
          double w = 1.0;   /* int_F psi_a psi_b: the mass of the other axes */
          for (int x = 0; x < d; ++x)
            if (x != ax) w *= m1((la >> x) & 1, (lb >> x) & 1, h[x]);
          t1 += w * p0_1[cv[lb]];
          t2 += w * p0_2[cv[lb]];
        }
        f[dof_u(d, N, 0, a, ax)] -= nrm * t1;
        f[dof_u(d, N, 1, a, ax)] -= nrm * t2;
      }
    }
  }
}

/* Threads the OpenMP loops of this file use. */
int or_max_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    t = omp_get_num_threads();
  }
  return t;
}

/* y = A x for a CSR matrix (OpenMP over rows). */
void or_spmv(long nrows, const int64_t *rowptr, const int32_t *cols, const double *vals,
             const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (long r = 0; r < nrows; ++r) {
    double s = 0.0;
    for (int64_t q = rowptr[r]; q < rowptr[r + 1]; ++q) s += vals[q] * x[cols[q]];
    y[r] = s;
  }
}
