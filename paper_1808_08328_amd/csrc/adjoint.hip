// Adjoint support: the sign map D = diag(I_u, -I_p) (D K is symmetric for
// the CG-VMS operator, so K^T = D K D and the adjoint system reuses the
// forward solver), and the element-local parameter gradient
//   dJ/dtheta = -lambda^T (dK/dtheta) x,
// theta = ln k1_e, ln k2_e (entering the uu block through mu/(2k) and the pp
// block through k/(2 mu), eq. S4_cg_stiffness_matrix) and beta (the mass
// transfer (q1 - q2; beta/mu (p1 - p2))).
#include "objects.h"

namespace dpp {

namespace {

__global__ void k_flip(long nu, long N, int dim, const double *__restrict__ in, double *__restrict__ out) {
  const long n = (long)(2 * dim + 2) * N;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const bool pres = (i >= (long)dim * N && i < (long)(dim + 1) * N) || i >= (long)(2 * dim + 1) * N;
    out[i] = pres ? -in[i] : in[i];
  }
  (void)nu;
}

__device__ inline int perm_axis_g(int D, int s, int k) {
  if (D == 2) return (s == 0) ? k : 1 - k;
  const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  return P[s][k];
}

// One thread per simplex: gathers x and lambda at its d+1 vertices.
template <int D>
__global__ __launch_bounds__(256) void k_grad(GridDev g, double h0, double h1, double h2, double mu,
                                              const double *__restrict__ k1,
                                              const double *__restrict__ k2,
                                              const double *__restrict__ x,
                                              const double *__restrict__ lam,
                                              double *__restrict__ g1, double *__restrict__ g2,
                                              double *__restrict__ gbc) {
  const long N = g.N;
  const int nper = (D == 3) ? 6 : 2;
  const long ncell = (long)nper * g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const double h[3] = {h0, h1, h2};
  const int s = (int)(e % nper);
  long hex = e / nper;
  int c[3] = {0, 0, 0};
  c[0] = (int)(hex % g.n[0]);
  hex /= g.n[0];
  c[1] = (int)(hex % g.n[1]);
  c[2] = (D == 3) ? (int)(hex / g.n[1]) : 0;
  long v[D + 1];
  int pos[3] = {c[0], c[1], c[2]};
  v[0] = pos[0] + (long)g.m[0] * (pos[1] + (long)g.m[1] * pos[2]);
  for (int k = 0; k < D; ++k) {
    pos[perm_axis_g(D, s, k)] += 1;
    v[k + 1] = pos[0] + (long)g.m[0] * (pos[1] + (long)g.m[1] * pos[2]);
  }
  double G[D + 1][D];
  for (int k = 0; k <= D; ++k)
    for (int cc = 0; cc < D; ++cc) {
      double gv = 0.0;
      if (k >= 1 && perm_axis_g(D, s, k - 1) == cc) gv += 1.0 / h[cc];
      if (k < D && perm_axis_g(D, s, k) == cc) gv -= 1.0 / h[cc];
      G[k][cc] = gv;
    }
  const double vol = (D == 3) ? h[0] * h[1] * h[2] / 6.0 : h[0] * h[1] / 2.0;
  const double moff = vol / ((D + 1.0) * (D + 2.0));
  double gnet[2], dpl[D + 1], dpx[D + 1];
  for (int q = 0; q < 2; ++q) {
    const double kk = q ? k2[e] : k1[e];
    const long ou = off_u(D, N, q), op = off_p(D, N, q);
    double uu = 0.0, pp = 0.0;
    for (int a = 0; a <= D; ++a)
      for (int b = 0; b <= D; ++b) {
        const double M = moff * (a == b ? 2.0 : 1.0);
        double lx = 0.0, gg = 0.0;
        for (int cc = 0; cc < D; ++cc) {
          lx += lam[ou + D * v[a] + cc] * x[ou + D * v[b] + cc];
          gg += G[a][cc] * G[b][cc];
        }
        uu += M * lx;
        pp += gg * lam[op + v[a]] * x[op + v[b]];
      }
    gnet[q] = -(-(mu / (2.0 * kk)) * uu + (kk / (2.0 * mu)) * vol * pp);
  }
  for (int a = 0; a <= D; ++a) {
    dpl[a] = lam[off_p(D, N, 0) + v[a]] - lam[off_p(D, N, 1) + v[a]];
    dpx[a] = x[off_p(D, N, 0) + v[a]] - x[off_p(D, N, 1) + v[a]];
  }
  double gb = 0.0;
  for (int a = 0; a <= D; ++a)
    for (int b = 0; b <= D; ++b) gb += moff * (a == b ? 2.0 : 1.0) * dpl[a] * dpx[b];
  if (g1) g1[e] = gnet[0];
  if (g2) g2[e] = gnet[1];
  gbc[e] = -gb / mu;
}

// Q1 box cells: one thread per box gathers x and lambda at its 2^D corners
// (corner v on the upper side of axis a when bit a of v is set).  The cell's
// mass and stiffness matrices are tensor products of the one-dimensional
// linear-element matrices (h/6)[[2, 1], [1, 2]] and (1/h)[[1, -1], [-1, 1]].
template <int D>
__global__ __launch_bounds__(256) void k_grad_q1(GridDev g, double h0, double h1, double h2,
                                                 double mu, const double *__restrict__ k1,
                                                 const double *__restrict__ k2,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ lam,
                                                 double *__restrict__ g1, double *__restrict__ g2,
                                                 double *__restrict__ gbc) {
  constexpr int NV = 1 << D;
  const long N = g.N;
  const long ncell = (long)g.n[0] * g.n[1] * (D == 3 ? g.n[2] : 1);
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const double h[3] = {h0, h1, h2};
  long r = e;
  int c[3] = {(int)(r % g.n[0]), 0, 0};
  r /= g.n[0];
  c[1] = (int)(r % g.n[1]);
  c[2] = D == 3 ? (int)(r / g.n[1]) : 0;
  long v[NV];
  for (int k = 0; k < NV; ++k)
    v[k] = (c[0] + (k & 1)) + (long)g.m[0] * ((c[1] + ((k >> 1) & 1)) + (long)g.m[1] * (c[2] + ((k >> 2) & 1)));
  // M(a, b) and S(a, b) of the cell from the corner bits
  auto mass = [&](int a, int b) {
    double m = 1.0;
    for (int ax = 0; ax < D; ++ax) m *= (((a ^ b) >> ax) & 1) ? h[ax] / 6.0 : h[ax] / 3.0;
    return m;
  };
  auto stiff = [&](int a, int b) {
    double sv = 0.0;
    for (int ax = 0; ax < D; ++ax) {
      double t = (((a ^ b) >> ax) & 1) ? -1.0 / h[ax] : 1.0 / h[ax];
      for (int bx = 0; bx < D; ++bx)
        if (bx != ax) t *= (((a ^ b) >> bx) & 1) ? h[bx] / 6.0 : h[bx] / 3.0;
      sv += t;
    }
    return sv;
  };
  double gnet[2];
  for (int q = 0; q < 2; ++q) {
    const double kk = q ? k2[e] : k1[e];
    const long ou = off_u(D, N, q), op = off_p(D, N, q);
    double uu = 0.0, pp = 0.0;
    for (int a = 0; a < NV; ++a)
      for (int b = 0; b < NV; ++b) {
        double lx = 0.0;
        for (int cc = 0; cc < D; ++cc) lx += lam[ou + D * v[a] + cc] * x[ou + D * v[b] + cc];
        uu += mass(a, b) * lx;
        pp += stiff(a, b) * lam[op + v[a]] * x[op + v[b]];
      }
    gnet[q] = -(-(mu / (2.0 * kk)) * uu + (kk / (2.0 * mu)) * pp);
  }
  double dpl[NV], dpx[NV];
  for (int a = 0; a < NV; ++a) {
    dpl[a] = lam[off_p(D, N, 0) + v[a]] - lam[off_p(D, N, 1) + v[a]];
    dpx[a] = x[off_p(D, N, 0) + v[a]] - x[off_p(D, N, 1) + v[a]];
  }
  double gb = 0.0;
  for (int a = 0; a < NV; ++a)
    for (int b = 0; b < NV; ++b) gb += mass(a, b) * dpl[a] * dpx[b];
  if (g1) g1[e] = gnet[0];
  if (g2) g2[e] = gnet[1];
  gbc[e] = -gb / mu;
}

__global__ void k_sum_fixed(const double *__restrict__ v, long n, double *__restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace

void flip_pressure_sign(dpp_problem P, const double *in, double *out, hipStream_t s) {
  const long n = P->ndof();
  k_flip<<<std::min(2048, blocks_for(n, 256)), 256, 0, s>>>(0, P->npos(), P->g.dim, in, out);
  check_launch("flip");
}

// lam with the prescribed velocity components zeroed (velocity faces)
template <int D>
__global__ void k_mask_fixed(GridDev g, const double *__restrict__ lam, double *__restrict__ out) {
  const long N = g.N;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
  for (int q = 0; q < 2; ++q) {
    const long ou = off_u(D, N, q), op = off_p(D, N, q);
    for (int c = 0; c < D; ++c) out[ou + D * a + c] = u_fixed(g, q, c, ia) ? 0.0 : lam[ou + D * a + c];
    out[op + a] = lam[op + a];
  }
}

void param_grad(dpp_problem P, const double *x, const double *lam, double *g1, double *g2,
                double *gb, hipStream_t s) {
  DPP_CHECK(!P->dg, DPP_ERR_UNSUPPORTED,
            "the parameter gradient is implemented for CG-VMS (P1 simplices, Q1 box cells)");
  const Grid &g = P->g;
  // With velocity faces K~ = P_f K P_f + P_c and f~ = P_f (f - K P_c g) + P_c g,
  // so dJ/dtheta = lam^T (df~ - dK~ x) = -(P_f lam)^T (dK/dtheta) x (x = g on
  // the prescribed DOFs): the gradient takes lam with those entries zeroed.
  DBuf lmask;
  if (g.fix[0] | g.fix[1]) {
    lmask.alloc(sizeof(double) * P->ndof());
    if (g.dim == 3)
      k_mask_fixed<3><<<blocks_for(g.N, 256), 256, 0, s>>>(dev(g), lam, lmask.as<double>());
    else
      k_mask_fixed<2><<<blocks_for(g.N, 256), 256, 0, s>>>(dev(g), lam, lmask.as<double>());
    lam = lmask.as<double>();
  }
  DBuf tmp;
  double *gbc = gb;
  if (!P->beta_per_cell || !gb) {
    tmp.alloc(sizeof(double) * g.nc);
    gbc = tmp.as<double>();
  }
  const int nb = blocks_for(g.nc, 256);
  if (g.elem == ELEM_Q1) {
    if (g.dim == 3)
      k_grad_q1<3><<<nb, 256, 0, s>>>(dev(g), g.h[0], g.h[1], g.h[2], P->mu, P->k1.as<double>(),
                                      P->k2.as<double>(), x, lam, g1, g2, gbc);
    else
      k_grad_q1<2><<<nb, 256, 0, s>>>(dev(g), g.h[0], g.h[1], g.h[2], P->mu, P->k1.as<double>(),
                                      P->k2.as<double>(), x, lam, g1, g2, gbc);
  } else if (g.dim == 3)
    k_grad<3><<<nb, 256, 0, s>>>(dev(g), g.h[0], g.h[1], g.h[2], P->mu, P->k1.as<double>(),
                                 P->k2.as<double>(), x, lam, g1, g2, gbc);
  else
    k_grad<2><<<nb, 256, 0, s>>>(dev(g), g.h[0], g.h[1], g.h[2], P->mu, P->k1.as<double>(),
                                 P->k2.as<double>(), x, lam, g1, g2, gbc);
  if (gb && !P->beta_per_cell) k_sum_fixed<<<1, 256, 0, s>>>(gbc, g.nc, gb);
  check_launch("param_grad");
  DPP_HIP(hipStreamSynchronize(s));
}

}  // namespace dpp
