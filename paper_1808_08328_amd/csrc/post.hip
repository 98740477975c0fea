// Post-processing for the time-accuracy-size study (section "Performance
// spectrum modeling"): L2 errors ||u_h - u||_L2 of a discrete solution against
// the manufactured solutions of the two- and three-dimensional studies
// (section "Representative numerical results"), per field u1, p1, u2, p2.
//
// The error integral is taken over the cells of the assembly: on the Kuhn
// simplices with a conical-product Gauss rule (Stroud 1971), Gauss-Legendre
// nodes on [0, 1] in each collapsed coordinate of the simplex, q^d points per
// simplex; on Q1 box cells with the tensor Gauss-Legendre rule of q points per
// axis and the multilinear interpolation of the cell's corner values.  One
// thread per cell loops over the points; per-workgroup partial sums are added
// in a fixed order (bit-reproducible).
#include <cmath>
#include <mutex>
#include <vector>

#include "objects.h"

namespace dpp {

namespace {

constexpr int PBS = 256;   // threads per workgroup of the error kernel
constexpr int QMAX = 16;   // largest rule order (16^3 points per simplex)

struct MMS {
  double k1, k2, beta, mu, eta;
};

// Gauss-Legendre nodes and weights on [0, 1], passed by value
struct GL01 {
  double t[QMAX], w[QMAX];
};

// Manufactured solution at X: pressures p1, p2 and velocities u_i = -(k_i/mu)
// grad p_i.  2D:  p_{1,2} = (mu/pi) e^{pi x} sin(pi y) -+ mu/(beta k_{1,2}) e^{eta y};
// 3D:  p_{1,2} = (mu/pi) e^{pi x} (sin(pi y) + sin(pi z))
//                -+ mu/(beta k_{1,2}) (e^{eta y} + e^{eta z}),
// eta = sqrt(beta (k1 + k2) / (k1 k2)).  The 3D micro-pressure uses
// mu/(beta k2), the value for which the pair solves the mass balances.
template <int D>
__device__ inline void mms_exact(const MMS &m, const double *X, double &p1, double &p2,
                                 double *u1, double *u2) {
  const double pi = 3.14159265358979323846;
  const double ex = exp(pi * X[0]);
  const double a1 = m.mu / (m.beta * m.k1), a2 = m.mu / (m.beta * m.k2);
  double sy, cy, sz = 0.0, cz = 0.0;
  sincos(pi * X[1], &sy, &cy);
  const double ey = exp(m.eta * X[1]);
  double ez = 0.0;
  if constexpr (D == 3) {
    sincos(pi * X[2], &sz, &cz);
    ez = exp(m.eta * X[2]);
  }
  const double harm = ex * (sy + sz);
  p1 = (m.mu / pi) * harm - a1 * (ey + ez);
  p2 = (m.mu / pi) * harm + a2 * (ey + ez);
  // grad p_i = mu [e^{pi x}(sy + sz), e^{pi x} cy -+ eta/(beta k_i) e^{eta y}, ...] / mu
  u1[0] = -m.k1 * harm;
  u2[0] = -m.k2 * harm;
  u1[1] = -m.k1 * (ex * cy - m.eta / (m.beta * m.k1) * ey);
  u2[1] = -m.k2 * (ex * cy + m.eta / (m.beta * m.k2) * ey);
  if constexpr (D == 3) {
    u1[2] = -m.k1 * (ex * cz - m.eta / (m.beta * m.k1) * ez);
    u2[2] = -m.k2 * (ex * cz + m.eta / (m.beta * m.k2) * ez);
  }
}

// Simplex s of box cell (ci, cj, ck) starts at the cell corner and steps along
// the axes of permutation s (the ordering of the assembly).
__device__ inline int perm_of(int D, int s, int k) {
  if (D == 2) return (s == 0) ? k : 1 - k;
  const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  return P[s][k];
}

// Squared errors of simplex e, summed over the rule (lam: [nq][D+1], w: [nq]).
template <int D>
__global__ __launch_bounds__(PBS) void k_l2_error(GridDev g, const double *__restrict__ x,
                                                  MMS m, const double *__restrict__ lam,
                                                  const double *__restrict__ w, int nq,
                                                  double hx, double hy, double hz, long nslot,
                                                  double *__restrict__ part) {
  constexpr int NPER = D == 3 ? 6 : 2;
  // CG-VMS: the fields live on the nodes; DG-VMS (nslot > 0): on the vertex
  // slots, slot e (D+1) + k being vertex k of simplex e
  const long N = nslot > 0 ? nslot : g.N;
  const long ncell = (long)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1) * NPER;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // u1, p1, u2, p2
  // grid-stride over the simplices (one pass when the grid covers them all)
  for (long e = (long)blockIdx.x * PBS + threadIdx.x; e < ncell; e += (long)gridDim.x * PBS) {
    double se[4] = {0.0, 0.0, 0.0, 0.0};
    const int s = (int)(e % NPER);
    long hex = e / NPER;
    const int ci = (int)(hex % g.n[0]);
    hex /= g.n[0];
    const int cj = (int)(hex % g.n[1]);
    const int ck = D == 3 ? (int)(hex / g.n[1]) : 0;
    const double h[3] = {hx, hy, hz};
    // vertices: node ids and coordinates
    long vid[D + 1];
    double vx[D + 1][D];
    int ijk[3] = {ci, cj, ck};
    for (int k = 0; k <= D; ++k) {
      if (k > 0) ijk[perm_of(D, s, k - 1)] += 1;
      vid[k] = ijk[0] + (long)g.m[0] * (ijk[1] + (long)g.m[1] * ijk[2]);
      for (int c = 0; c < D; ++c) vx[k][c] = ijk[c] * h[c];
    }
    // nodal values of the discrete fields at the vertices
    const long ou1 = off_u(D, N, 0), ou2 = off_u(D, N, 1);
    const long op1 = off_p(D, N, 0), op2 = off_p(D, N, 1);
    double vp1[D + 1], vp2[D + 1], vu1[D + 1][D], vu2[D + 1][D];
    for (int k = 0; k <= D; ++k) {
      const long at = nslot > 0 ? e * (D + 1) + k : vid[k];
      vp1[k] = x[op1 + at];
      vp2[k] = x[op2 + at];
      for (int c = 0; c < D; ++c) {
        vu1[k][c] = x[ou1 + D * at + c];
        vu2[k][c] = x[ou2 + D * at + c];
      }
    }
    for (int iq = 0; iq < nq; ++iq) {
      const double *l = lam + (size_t)iq * (D + 1);
      double X[D], hp1 = 0.0, hp2 = 0.0, hu1[D], hu2[D];
      for (int c = 0; c < D; ++c) X[c] = hu1[c] = hu2[c] = 0.0;
      for (int k = 0; k <= D; ++k) {
        for (int c = 0; c < D; ++c) {
          X[c] += l[k] * vx[k][c];
          hu1[c] += l[k] * vu1[k][c];
          hu2[c] += l[k] * vu2[k][c];
        }
        hp1 += l[k] * vp1[k];
        hp2 += l[k] * vp2[k];
      }
      double p1, p2, u1[3], u2[3];
      mms_exact<D>(m, X, p1, p2, u1, u2);
      double e1 = 0.0, e2 = 0.0;
      for (int c = 0; c < D; ++c) {
        e1 += (hu1[c] - u1[c]) * (hu1[c] - u1[c]);
        e2 += (hu2[c] - u2[c]) * (hu2[c] - u2[c]);
      }
      se[0] += w[iq] * e1;
      se[1] += w[iq] * (hp1 - p1) * (hp1 - p1);
      se[2] += w[iq] * e2;
      se[3] += w[iq] * (hp2 - p2) * (hp2 - p2);
    }
    // |det J| of the simplex: the product of the cell sizes (the reference
    // simplex has volume 1/d!, carried by the weights)
    const double detj = D == 3 ? hx * hy * hz : hx * hy;
    for (int f = 0; f < 4; ++f) acc[f] += se[f] * detj;
  }
  // fixed-order workgroup sum
  __shared__ double red[4][PBS];
  for (int f = 0; f < 4; ++f) red[f][threadIdx.x] = acc[f];
  __syncthreads();
  for (int st = PBS / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int f = 0; f < 4; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

// Squared errors of Q1 box cell e over the tensor rule gl (q points per axis,
// x fastest): the fields at a point are the multilinear interpolation of the
// 2^D corner values, corner v taking the upper node on axis a when bit a of v
// is set.
template <int D>
__global__ __launch_bounds__(PBS) void k_l2_error_box(GridDev g, const double *__restrict__ x,
                                                      MMS m, GL01 gl, int q, double hx, double hy,
                                                      double hz, double *__restrict__ part) {
  constexpr int NV = 1 << D;
  const long N = g.N;
  const long ncell = (long)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
  const int nq = D == 3 ? q * q * q : q * q;
  const double h[3] = {hx, hy, hz};
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // u1, p1, u2, p2
  for (long e = (long)blockIdx.x * PBS + threadIdx.x; e < ncell; e += (long)gridDim.x * PBS) {
    long r = e;
    int c[3] = {(int)(r % g.n[0]), 0, 0};
    r /= g.n[0];
    c[1] = (int)(r % g.n[1]);
    c[2] = D == 3 ? (int)(r / g.n[1]) : 0;
    const long ou1 = off_u(D, N, 0), ou2 = off_u(D, N, 1);
    const long op1 = off_p(D, N, 0), op2 = off_p(D, N, 1);
    double vp1[NV], vp2[NV], vu1[NV][D], vu2[NV][D];
    for (int v = 0; v < NV; ++v) {
      const long at = (c[0] + (v & 1)) +
                      (long)g.m[0] * ((c[1] + ((v >> 1) & 1)) + (long)g.m[1] * (c[2] + ((v >> 2) & 1)));
      vp1[v] = x[op1 + at];
      vp2[v] = x[op2 + at];
      for (int a = 0; a < D; ++a) {
        vu1[v][a] = x[ou1 + D * at + a];
        vu2[v][a] = x[ou2 + D * at + a];
      }
    }
    double se[4] = {0.0, 0.0, 0.0, 0.0};
    for (int iq = 0; iq < nq; ++iq) {
      const int ia[3] = {iq % q, (iq / q) % q, D == 3 ? iq / (q * q) : 0};
      double xi[D], X[D], wq = 1.0;
      for (int a = 0; a < D; ++a) {
        xi[a] = gl.t[ia[a]];
        wq *= gl.w[ia[a]];
        X[a] = c[a] * h[a] + xi[a] * h[a];
      }
      double hp1 = 0.0, hp2 = 0.0, hu1[D], hu2[D];
      for (int a = 0; a < D; ++a) hu1[a] = hu2[a] = 0.0;
      for (int v = 0; v < NV; ++v) {
        double sh = 1.0;
        for (int a = 0; a < D; ++a) sh *= ((v >> a) & 1) ? xi[a] : 1.0 - xi[a];
        hp1 += sh * vp1[v];
        hp2 += sh * vp2[v];
        for (int a = 0; a < D; ++a) {
          hu1[a] += sh * vu1[v][a];
          hu2[a] += sh * vu2[v][a];
        }
      }
      double p1, p2, u1[3], u2[3];
      mms_exact<D>(m, X, p1, p2, u1, u2);
      double e1 = 0.0, e2 = 0.0;
      for (int a = 0; a < D; ++a) {
        e1 += (hu1[a] - u1[a]) * (hu1[a] - u1[a]);
        e2 += (hu2[a] - u2[a]) * (hu2[a] - u2[a]);
      }
      se[0] += wq * e1;
      se[1] += wq * (hp1 - p1) * (hp1 - p1);
      se[2] += wq * e2;
      se[3] += wq * (hp2 - p2) * (hp2 - p2);
    }
    // the rule's weights sum to 1 on the unit box: scale by the cell volume
    const double vol = D == 3 ? hx * hy * hz : hx * hy;
    for (int f = 0; f < 4; ++f) acc[f] += se[f] * vol;
  }
  __shared__ double red[4][PBS];
  for (int f = 0; f < 4; ++f) red[f][threadIdx.x] = acc[f];
  __syncthreads();
  for (int st = PBS / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int f = 0; f < 4; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

// Pure-flux case (velocity faces on every face of both networks): K has the
// kernel u = 0, p1 = p2 = const, which is also its left kernel (K^T = D K D).
// mode 0: per-workgroup sums of p1 + p2 over the nodes (the right-hand side's
// component along the kernel); mode 1: of the cell means of p1 (int p1, up to
// the constant cell volume of the box; cells are the Kuhn simplices, or the
// boxes themselves with Q1 elements, where a cell's mean is its vertex mean).
template <int D>
__global__ __launch_bounds__(PBS) void k_pressure_sums(GridDev g, const double *__restrict__ v,
                                                       int mode, int boxcells,
                                                       double *__restrict__ part) {
  constexpr int NPER = D == 3 ? 6 : 2;
  const long N = g.N;
  double acc = 0.0;
  if (mode == 0) {
    const long op1 = off_p(D, N, 0), op2 = off_p(D, N, 1);
    for (long a = (long)blockIdx.x * PBS + threadIdx.x; a < N; a += (long)gridDim.x * PBS)
      acc += v[op1 + a] + v[op2 + a];
  } else if (boxcells) {
    const long ncell = (long)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
    const long op1 = off_p(D, N, 0);
    for (long e = (long)blockIdx.x * PBS + threadIdx.x; e < ncell; e += (long)gridDim.x * PBS) {
      long r = e;
      const int i = (int)(r % g.n[0]);
      r /= g.n[0];
      const int j = (int)(r % g.n[1]);
      const int k = D == 3 ? (int)(r / g.n[1]) : 0;
      double sv = 0.0;
      for (int vb = 0; vb < (1 << D); ++vb)
        sv += v[op1 + (i + (vb & 1)) + (long)g.m[0] * ((j + ((vb >> 1) & 1)) + (long)g.m[1] * (k + ((vb >> 2) & 1)))];
      acc += sv / (1 << D);
    }
  } else {
    const long ncell = (long)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1) * NPER;
    const long op1 = off_p(D, N, 0);
    for (long e = (long)blockIdx.x * PBS + threadIdx.x; e < ncell; e += (long)gridDim.x * PBS) {
      const int s = (int)(e % NPER);
      long hex = e / NPER;
      int ijk[3] = {(int)(hex % g.n[0]), 0, 0};
      hex /= g.n[0];
      ijk[1] = (int)(hex % g.n[1]);
      ijk[2] = D == 3 ? (int)(hex / g.n[1]) : 0;
      double sv = 0.0;
      for (int k = 0; k <= D; ++k) {
        if (k > 0) ijk[perm_of(D, s, k - 1)] += 1;
        sv += v[op1 + ijk[0] + (long)g.m[0] * (ijk[1] + (long)g.m[1] * ijk[2])];
      }
      acc += sv / (D + 1);
    }
  }
  __shared__ double red[PBS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = PBS / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <int D>
__global__ void k_shift_pressures(GridDev g, double *__restrict__ v, double c) {
  const long N = g.N;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  v[off_p(D, N, 0) + a] -= c;
  v[off_p(D, N, 1) + a] -= c;
}

// out[f] = sum over workgroups of part[f][.], in a fixed order
__global__ __launch_bounds__(PBS) void k_l2_finish(const double *__restrict__ part, int nb,
                                                   double *__restrict__ out) {
  __shared__ double red[PBS];
  const int f = blockIdx.x;
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += PBS) a += part[(size_t)f * nb + i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = PBS / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[f] = red[0];
}

}  // namespace

bool pure_flux(const Grid &g) {
  const int all = (1 << (2 * g.dim)) - 1;
  return g.fix[0] == all && g.fix[1] == all;
}

// sum of p1 + p2 over the nodes (mode 0) or the mean of p1 over the box
// (mode 1), reduced in a fixed order; synchronises the stream
static double pressure_reduce(dpp_problem P, const double *v, int mode, hipStream_t s) {
  const Grid &g = P->g;
  constexpr int NB = 512;
  DBuf part(sizeof(double) * (NB + 1));
  double *dp = part.as<double>();
  const int box = g.elem == ELEM_Q1 ? 1 : 0;
  if (g.dim == 3)
    k_pressure_sums<3><<<NB, PBS, 0, s>>>(dev(g), v, mode, box, dp);
  else
    k_pressure_sums<2><<<NB, PBS, 0, s>>>(dev(g), v, mode, box, dp);
  k_l2_finish<<<1, PBS, 0, s>>>(dp, NB, dp + NB);
  check_launch("pressure sums");
  double h = 0.0;
  DPP_HIP(hipMemcpyAsync(&h, dp + NB, sizeof(double), hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  return mode == 0 ? h : h / (double)g.nc;
}

static void shift_pressures(dpp_problem P, double *v, double c, hipStream_t s) {
  const Grid &g = P->g;
  if (g.dim == 3)
    k_shift_pressures<3><<<blocks_for(g.N, 256), 256, 0, s>>>(dev(g), v, c);
  else
    k_shift_pressures<2><<<blocks_for(g.N, 256), 256, 0, s>>>(dev(g), v, c);
  check_launch("shift pressures");
}

// The part of b in the range of K: b minus its component along the kernel
// (the interpolated boundary fluxes are compatible only up to O(h^2)).
void consistent_rhs(dpp_problem P, double *b, hipStream_t s) {
  shift_pressures(P, b, pressure_reduce(P, b, 0, s) / (2.0 * P->g.N), s);
}

// The pressure space Q asks (int p1)(int p2) = 0; of its two branches the
// solution is normalised to int p1 = 0 (both pressures shifted alike).
void normalize_pressures(dpp_problem P, double *x, hipStream_t s) {
  shift_pressures(P, x, pressure_reduce(P, x, 1, s), s);
}

// Gauss-Legendre nodes and weights on [0, 1]: Newton iteration on P_q from the
// Chebyshev-like guesses cos(pi (i + 3/4) / (q + 1/2)), with P_q and P_q' from
// the three-term recurrence.
static void gauss_legendre01(int q, double *t, double *w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < q; ++i) {
    double z = std::cos(pi * (i + 0.75) / (q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      const double pq = q == 1 ? z : p1, pq1 = q == 1 ? 1.0 : p0;
      dp = q * (z * pq - pq1) / (z * z - 1.0);
      const double dz = pq / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute P_q' at the converged node for the weight
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    const double pq = q == 1 ? z : p1, pq1 = q == 1 ? 1.0 : p0;
    dp = q * (z * pq - pq1) / (z * z - 1.0);
    t[q - 1 - i] = 0.5 * (z + 1.0);                        // ascending on [0, 1]
    w[q - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);        // 2/((1-z^2)P'^2), halved
  }
}

// Conical-product rule on the reference simplex {lambda_1 + ... + lambda_d <= 1}:
// collapsed coordinates s = lambda_1 + .. + lambda_d, then the share of the
// later vertices at each stage, with Jacobian s^(d-1) (and e in 3D).
// Writes q^dim points: lam [q^dim][dim+1] and wt [q^dim] (caller-sized).
static void simplex_rule_into(int dim, int q, double *lam, double *wt) {
  double t[QMAX], w[QMAX];
  gauss_legendre01(q, t, w);
  int k = 0;
  if (dim == 2) {
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b, ++k) {
        const double s = t[a], e = t[b];
        double *l = lam + 3 * k;
        l[0] = 1.0 - s;
        l[1] = s * (1.0 - e);
        l[2] = s * e;
        wt[k] = w[a] * w[b] * s;
      }
    return;
  }
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b)
      for (int c = 0; c < q; ++c, ++k) {
        const double s = t[a], e = t[b], gq = t[c];
        double *l = lam + 4 * k;
        l[0] = 1.0 - s;
        l[1] = s * (1.0 - e);
        l[2] = s * e * (1.0 - gq);
        l[3] = s * e * gq;
        wt[k] = w[a] * w[b] * w[c] * s * s * e;
      }
}

void simplex_rule(int dim, int q, std::vector<double> &lam, std::vector<double> &wt) {
  int nq = 1;
  for (int a = 0; a < dim; ++a) nq *= q;
  lam.assign((size_t)nq * (dim + 1), 0.0);
  wt.assign(nq, 0.0);
  simplex_rule_into(dim, q, lam.data(), wt.data());
}

// Fixed-order sum of the nb partials per field (dp: 4 nb partials, then the 4
// results), returned to the host as square roots in the order u1, p1, u2, p2.
static void l2_finish(double *dp, int nb, double err[4], hipStream_t s) {
  double *dout = dp + 4 * (size_t)nb;
  k_l2_finish<<<4, PBS, 0, s>>>(dp, nb, dout);
  check_launch("l2 error finish");
  double h4[4];
  DPP_HIP(hipMemcpyAsync(h4, dout, sizeof(h4), hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  for (int f = 0; f < 4; ++f) err[f] = std::sqrt(std::max(h4[f], 0.0));
}

// The error integral with the rule at dl/dw (device), nb workgroups writing
// their partial sums to dp (device, 4 nb + 4 doubles); err on the host.
static void l2_errors_on(dpp_problem P, const double *x, const double mms[4], int nq,
                         const double *dl, const double *dw, int nb, double *dp, double err[4],
                         hipStream_t s) {
  const Grid &g = P->g;
  MMS m{mms[0], mms[1], mms[2], mms[3], std::sqrt(mms[2] * (mms[0] + mms[1]) / (mms[0] * mms[1]))};
  const long nslot = P->dg ? P->nslot : 0;
  if (g.dim == 3)
    k_l2_error<3><<<nb, PBS, 0, s>>>(dev(g), x, m, dl, dw, nq, g.h[0], g.h[1], g.h[2], nslot, dp);
  else
    k_l2_error<2><<<nb, PBS, 0, s>>>(dev(g), x, m, dl, dw, nq, g.h[0], g.h[1], 1.0, nslot, dp);
  check_launch("l2 error");
  l2_finish(dp, nb, err, s);
}

// The error integral over Q1 box cells with the tensor rule of q points per
// axis, nb workgroups writing their partial sums to dp (4 nb + 4 doubles).
static void l2_errors_box_on(dpp_problem P, const double *x, const double mms[4], int q, int nb,
                             double *dp, double err[4], hipStream_t s) {
  const Grid &g = P->g;
  MMS m{mms[0], mms[1], mms[2], mms[3], std::sqrt(mms[2] * (mms[0] + mms[1]) / (mms[0] * mms[1]))};
  GL01 gl{};
  gauss_legendre01(q, gl.t, gl.w);
  if (g.dim == 3)
    k_l2_error_box<3><<<nb, PBS, 0, s>>>(dev(g), x, m, gl, q, g.h[0], g.h[1], g.h[2], dp);
  else
    k_l2_error_box<2><<<nb, PBS, 0, s>>>(dev(g), x, m, gl, q, g.h[0], g.h[1], 1.0, dp);
  check_launch("l2 error (box cells)");
  l2_finish(dp, nb, err, s);
}

static void check_mms_args(int q, const double mms[4]) {
  DPP_CHECK(q >= 1 && q <= QMAX, DPP_ERR_ARG, "quadrature order must be in 1..16");
  DPP_CHECK(mms[0] > 0.0 && mms[1] > 0.0 && mms[2] > 0.0 && mms[3] > 0.0, DPP_ERR_ARG,
            "manufactured-solution parameters must be positive");
}

void mms_l2_errors(dpp_problem P, const double *x, const double mms[4], int q, double err[4],
                   hipStream_t s) {
  check_mms_args(q, mms);
  const Grid &g = P->g;
  if (g.elem == ELEM_Q1) {
    const long ncell = (long)g.nc;
    const int nb = (int)((ncell + PBS - 1) / PBS);  // one box cell per thread
    DBuf part(sizeof(double) * 4 * (size_t)nb + sizeof(double) * 4);
    l2_errors_box_on(P, x, mms, q, nb, part.as<double>(), err, s);
    return;
  }
  std::vector<double> lam, wt;
  simplex_rule(g.dim, q, lam, wt);
  const int nq = (int)wt.size();
  const long ncell = (long)g.nc;
  const int nb = (int)((ncell + PBS - 1) / PBS);  // one simplex per thread
  DBuf rule(sizeof(double) * (lam.size() + wt.size()));
  DBuf part(sizeof(double) * 4 * (size_t)nb + sizeof(double) * 4);
  double *dl = rule.as<double>(), *dw = dl + lam.size();
  DPP_HIP(hipMemcpyAsync(dl, lam.data(), sizeof(double) * lam.size(), hipMemcpyHostToDevice, s));
  DPP_HIP(hipMemcpyAsync(dw, wt.data(), sizeof(double) * wt.size(), hipMemcpyHostToDevice, s));
  l2_errors_on(P, x, mms, nq, dl, dw, nb, part.as<double>(), err, s);
}

// ---- the same integral with no allocation: the rule and the partial sums
// live in one fixed device array per GPU (`scratch`), whose address is taken
// once per device with hipGetSymbolAddress and used from then on.
namespace {
constexpr int NA_BLOCKS = 2048;                              // workgroups (grid-stride)
constexpr size_t NA_RULE = (size_t)QMAX * QMAX * QMAX * 5;   // lam [q^3][4] + w [q^3]
constexpr size_t NA_DOUBLES = NA_RULE + 4 * (size_t)NA_BLOCKS + 4;
static_assert(NA_DOUBLES * sizeof(double) <= NOALLOC_SCRATCH_BYTES, "scratch too small");
__device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

std::mutex na_mu;
double *na_ptr[MAX_DEVICES] = {};

// The conical-product rule of simplex_rule_into, expanded on the device from
// the one-dimensional nodes (same products in the same order).
__global__ void k_expand_rule(int dim, int q, GL01 gl, double *__restrict__ lam,
                              double *__restrict__ wt) {
  const int nq = dim == 2 ? q * q : q * q * q;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nq) return;
  if (dim == 2) {
    const int a = k / q, b = k % q;
    const double s = gl.t[a], e = gl.t[b];
    lam[3 * k] = 1.0 - s;
    lam[3 * k + 1] = s * (1.0 - e);
    lam[3 * k + 2] = s * e;
    wt[k] = gl.w[a] * gl.w[b] * s;
    return;
  }
  const int a = k / (q * q), b = (k / q) % q, c = k % q;
  const double s = gl.t[a], e = gl.t[b], gq = gl.t[c];
  lam[4 * k] = 1.0 - s;
  lam[4 * k + 1] = s * (1.0 - e);
  lam[4 * k + 2] = s * e * (1.0 - gq);
  lam[4 * k + 3] = s * e * gq;
  wt[k] = gl.w[a] * gl.w[b] * gl.w[c] * s * s * e;
}

double *scratch_of_current_device() {
  int dv = 0;
  DPP_HIP(hipGetDevice(&dv));
  DPP_CHECK(dv >= 0 && dv < MAX_DEVICES, DPP_ERR_UNSUPPORTED, "device index beyond the table");
  std::lock_guard<std::mutex> lk(na_mu);
  if (!na_ptr[dv]) {
    void *p = nullptr;
    DPP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    na_ptr[dv] = static_cast<double *>(p);
  }
  return na_ptr[dv];
}
}  // namespace

void mms_l2_errors_noalloc(dpp_problem P, const double *x, const double mms[4], int q,
                           double err[4], hipStream_t s) {
  check_mms_args(q, mms);
  const Grid &g = P->g;
  if (g.elem == ELEM_Q1) {
    // the rule goes by value; only the partial sums use the fixed array
    const long ncell = (long)g.nc;
    const int nb = (int)std::min<long>(NA_BLOCKS, (ncell + PBS - 1) / PBS);
    DPP_CHECK(4 * (size_t)nb + 4 <= NA_DOUBLES, DPP_ERR_ARG, "partial sums larger than the fixed scratch");
    l2_errors_box_on(P, x, mms, q, nb, scratch_of_current_device(), err, s);
    return;
  }
  int nq = 1;
  for (int a = 0; a < g.dim; ++a) nq *= q;
  const size_t nl = (size_t)nq * (g.dim + 1);
  DPP_CHECK(nl + nq <= NA_RULE, DPP_ERR_ARG, "quadrature rule larger than the fixed scratch");
  const long ncell = (long)g.nc;
  const int nb = (int)std::min<long>(NA_BLOCKS, (ncell + PBS - 1) / PBS);
  DPP_CHECK(4 * (size_t)nb + 4 <= NA_DOUBLES - NA_RULE, DPP_ERR_ARG,
            "partial sums larger than the fixed scratch");
  double *base = scratch_of_current_device();
  double *dl = base, *dw = base + nl, *dp = base + NA_RULE;
  GL01 gl{};
  gauss_legendre01(q, gl.t, gl.w);
  k_expand_rule<<<(nq + 255) / 256, 256, 0, s>>>(g.dim, q, gl, dl, dw);
  check_launch("quadrature rule");
  // every workgroup writes its partial sums and the finish kernel the result,
  // so nothing left by an earlier call is read
  l2_errors_on(P, x, mms, nq, dl, dw, nb, dp, err, s);
}

}  // namespace dpp
