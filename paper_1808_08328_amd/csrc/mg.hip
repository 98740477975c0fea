// Multigrid V-cycle on the two pressure Schur blocks S_p^1, S_p^2 and the
// Schur-complement fieldsplit application.
//
// The solver section applies one multigrid V-cycle to each diagonal block of
// the selfp Schur approximation (eqs. S4_sp1, S4_sp2), relying on S_p being
// spectrally equivalent to a Laplacian.  Here the cycle is geometric on the
// structured box:
//   * P: P1 interpolation from the box with ceil(n/2) cells per axis (coarse
//     node C at fine index 2C, the last one at n when n is odd; a fine node
//     with odd indices on the axes O averages the coarse nodes lo and lo+1_O,
//     the ends of the Kuhn edge it sits on);
//   * Galerkin coarse operators P^T A P, which keep the 65-point (19 in 2D)
//     stencil of S_p on every level, so all levels share one index-free
//     storage A[(i*NT + t)*ld + a] (ld = N rounded up to 32);
//   * Chebyshev smoothing (degree `cheb_degree`, diagonal preconditioning,
//     interval [lo_frac*hi, hi], hi = hi_factor * ||D^-1 A x_k|| after
//     `power_iters` power steps from a fixed integer-hash start vector);
//   * exact FP64 solve on the coarsest level through its inverse.
// Both networks are processed by the same launches (blockIdx.y = network).
#include <map>
#include <mutex>
#include <tuple>

#include "objects.h"
#include "profile.h"
#include "stencil.h"

namespace dpp {

namespace {

// Occupancy floor of the stencil kernels: at least 4 waves per SIMD (<= 128
// VGPRs), which still leaves a whole row's loads in flight per wave.
template <int D, typename TV, typename TX, int LPR, bool SYM, bool FINE>
__global__ __launch_bounds__(256, 4) void k_lspmv(GridDev g, const TV *__restrict__ A,
                                               const TX *__restrict__ x, TX *__restrict__ y,
                                               const TX *__restrict__ b,
                                               const TV *__restrict__ dinv) {
  constexpr int NT = Tabs<D>::NT;
  const long N = g.N;
  const int q = blockIdx.y;
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  constexpr int NA = stored_offsets<D, SYM>();
  if constexpr (LPR == 0) {
    // rows a, a + 1 per thread (paired loads)
    const long a = 2 * gid;
    if (a >= N) return;
    double r0, r1;
    row_product2<D, TV, TX, SYM>(g, A + (size_t)q * NA * g.ld, x + (size_t)q * N, a, r0, r1);
    const size_t ia = (size_t)q * N + a;
    if (a + 1 < N) {
      if (b) {
        TX b0, b1;
        ld2(b + ia, b0, b1);
        r0 = (double)b0 - r0;
        r1 = (double)b1 - r1;
      }
      if (dinv) {
        TV d0, d1;
        ld2(dinv + ia, d0, d1);
        r0 *= (double)d0;
        r1 *= (double)d1;
      }
      st2(y + ia, (TX)r0, (TX)r1);
    } else {
      if (b) r0 = (double)b[ia] - r0;
      if (dinv) r0 *= (double)dinv[ia];
      y[ia] = (TX)r0;
    }
    return;
  }
  const long a = gid / (LPR > 0 ? LPR : 1);
  const int sub = (int)(gid % (LPR > 0 ? LPR : 1));
  if (a >= N) return;
  int i, j, k;
  node_ijk(g, a, i, j, k);
  double acc = row_product<D, TV, TX, (LPR > 0 ? LPR : 1), SYM>(g, A + (size_t)q * NA * g.ld, x + (size_t)q * N, a, i, j, k, sub);
  if (sub != 0) return;
  if (b) acc = (double)b[(size_t)q * N + a] - acc;
  if (dinv) acc *= (double)dinv[(size_t)q * N + a];
  y[(size_t)q * N + a] = (TX)acc;
}

// Chebyshev step k (Saad, Alg. 12.1 with diagonal preconditioning):
//   r = D^-1 (b - A xin);  d = c1 d + c2 r;  xout = xin + d.
// (The first step from a zero guess has no product: k_cheb_first.)
template <int D, typename TV, typename TX, int LPR, bool SYM, bool FINE>
__global__ __launch_bounds__(256, 4) void k_cheb(GridDev g, const TV *__restrict__ A,
                                              const TV *__restrict__ dinv,
                                              const TX *__restrict__ b, const TX *__restrict__ xin,
                                              TX *__restrict__ xout, TX *__restrict__ d, Sc2 c1,
                                              Sc2 c2) {
  constexpr int NT = Tabs<D>::NT;
  const long N = g.N;
  const int q = blockIdx.y;
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  constexpr int NA = stored_offsets<D, SYM>();
  if constexpr (LPR == 0) {
    // rows a, a + 1 per thread (paired loads)
    const long a = 2 * gid;
    if (a >= N) return;
    double ax0, ax1;
    row_product2<D, TV, TX, SYM>(g, A + (size_t)q * NA * g.ld, xin + (size_t)q * N, a, ax0, ax1);
    const size_t ia = (size_t)q * N + a;
    const bool first = c1.v[q] == 0.0;
    if (a + 1 < N) {
      TX x0, x1, b0, b1, d0 = 0, d1 = 0;
      TV i0, i1;
      ld2(xin + ia, x0, x1);
      ld2(b + ia, b0, b1);
      ld2(dinv + ia, i0, i1);
      if (!first) ld2(d + ia, d0, d1);
      const double r0 = (double)i0 * ((double)b0 - ax0), r1 = (double)i1 * ((double)b1 - ax1);
      const double n0 = (first ? 0.0 : c1.v[q] * (double)d0) + c2.v[q] * r0;
      const double n1 = (first ? 0.0 : c1.v[q] * (double)d1) + c2.v[q] * r1;
      st2(d + ia, (TX)n0, (TX)n1);
      st2(xout + ia, (TX)((double)x0 + n0), (TX)((double)x1 + n1));
    } else {
      const double r0 = (double)dinv[ia] * ((double)b[ia] - ax0);
      const double n0 = (first ? 0.0 : c1.v[q] * (double)d[ia]) + c2.v[q] * r0;
      d[ia] = (TX)n0;
      xout[ia] = (TX)((double)xin[ia] + n0);
    }
    return;
  }
  const long a = gid / (LPR > 0 ? LPR : 1);
  const int sub = (int)(gid % (LPR > 0 ? LPR : 1));
  if (a >= N) return;
  const size_t ia = (size_t)q * N + a;
  int i, j, k;
  node_ijk(g, a, i, j, k);
  const double ax =
      row_product<D, TV, TX, (LPR > 0 ? LPR : 1), SYM>(g, A + (size_t)q * NA * g.ld, xin + (size_t)q * N, a, i, j, k, sub);
  if (sub != 0) return;
  const double xa = (double)xin[ia];
  const double r = (double)dinv[ia] * ((double)b[ia] - ax);
  const double dn = (c1.v[q] != 0.0 ? c1.v[q] * (double)d[ia] : 0.0) + c2.v[q] * r;
  d[ia] = (TX)dn;
  xout[ia] = (TX)(xa + dn);
}

#define DPP_SHAPE_SWITCH(sh, KCALL)                         \
  do {                                                      \
    if (sh.sym) {                                           \
      switch (sh.lpr) {                                     \
        case 0: { constexpr int L_ = 0; constexpr bool S_ = true; KCALL; } break; \
        case 1: { constexpr int L_ = 1; constexpr bool S_ = true; KCALL; } break; \
        case 2: { constexpr int L_ = 2; constexpr bool S_ = true; KCALL; } break; \
        case 4: { constexpr int L_ = 4; constexpr bool S_ = true; KCALL; } break; \
        default: { constexpr int L_ = 8; constexpr bool S_ = true; KCALL; } break; \
      }                                                     \
    } else {                                                \
      switch (sh.lpr) {                                     \
        case 0: { constexpr int L_ = 0; constexpr bool S_ = false; KCALL; } break; \
        case 1: { constexpr int L_ = 1; constexpr bool S_ = false; KCALL; } break; \
        case 2: { constexpr int L_ = 2; constexpr bool S_ = false; KCALL; } break; \
        case 4: { constexpr int L_ = 4; constexpr bool S_ = false; KCALL; } break; \
        default: { constexpr int L_ = 8; constexpr bool S_ = false; KCALL; } break; \
      }                                                     \
    }                                                       \
  } while (0)

// Level stencil kernels run in one-wave workgroups: at 64^3 the finest level
// is a single round of workgroups, and small workgroups spread it (and the
// much smaller coarse levels) evenly over the 256 CUs.
constexpr int LBS = 64;

// threads of a level launch: lpr lanes per row, or one thread per row pair (lpr = 0)
inline long shape_threads(Shape sh, long N) { return sh.lpr > 0 ? N * sh.lpr : (N + 1) / 2; }

template <int D, typename TV, typename TX>
void launch_lspmv(Shape sh, const Grid &gl, hipStream_t s, const TV *A, const TX *x, TX *y,
                  const TX *b, const TV *dinv, bool fine = false) {
  const dim3 grid(blocks_for(shape_threads(sh, gl.N), LBS), 2);
  if (fine)
    DPP_SHAPE_SWITCH(sh, (k_lspmv<D, TV, TX, L_, S_, true><<<grid, LBS, 0, s>>>(dev(gl), A, x, y, b, dinv)));
  else
    DPP_SHAPE_SWITCH(sh, (k_lspmv<D, TV, TX, L_, S_, false><<<grid, LBS, 0, s>>>(dev(gl), A, x, y, b, dinv)));
}

template <int D, typename TV, typename TX>
void launch_cheb(Shape sh, const Grid &gl, hipStream_t s, const TV *A, const TV *di, const TX *b,
                 const TX *xin, TX *xout, TX *d, Sc2 c1, Sc2 c2, bool fine) {
  const dim3 grid(blocks_for(shape_threads(sh, gl.N), LBS), 2);
  if (fine)
    DPP_SHAPE_SWITCH(sh, (k_cheb<D, TV, TX, L_, S_, true><<<grid, LBS, 0, s>>>(dev(gl), A, di, b, xin,
                                                                                xout, d, c1, c2)));
  else
    DPP_SHAPE_SWITCH(sh, (k_cheb<D, TV, TX, L_, S_, false><<<grid, LBS, 0, s>>>(dev(gl), A, di, b, xin,
                                                                                 xout, d, c1, c2)));
}

// Ah[q][h][a] = A[q][t0 + h][a]: the zero offset and positive half of T.
template <int D, typename TV>
__global__ void k_pack_half(const TV *__restrict__ A, long N, long ld, TV *__restrict__ Ah) {
  constexpr int NT = Tabs<D>::NT;
  constexpr int T0 = TAB<D>.t0;
  constexpr int NH = NT - T0;
  const int q = blockIdx.y;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)NH * N) return;
  const int h = (int)(idx / N);
  const long a = idx - (long)h * N;
  Ah[((size_t)q * NH + h) * ld + a] = A[((size_t)q * NT + T0 + h) * ld + a];
}

// First Chebyshev step from a zero guess: x = d = c2 D^-1 b (no product).
template <typename TV, typename TX>
__global__ __launch_bounds__(256) void k_cheb_first(long N, const TV *__restrict__ dinv,
                                                    const TX *__restrict__ b, TX *__restrict__ x,
                                                    TX *__restrict__ d, Sc2 c2) {
  const int q = blockIdx.y;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  const size_t ia = (size_t)q * N + a;
  const double v = c2.v[q] * (double)dinv[ia] * (double)b[ia];
  d[ia] = (TX)v;
  x[ia] = (TX)v;
}

// b_c(C) = sum_f P(f, C) r(f)
template <int D, typename TX>
__global__ __launch_bounds__(256) void k_restrict(GridDev gf, GridDev gc, const TX *__restrict__ r,
                                                  TX *__restrict__ bc) {
  const int q = blockIdx.y;
  const long C = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= gc.N) return;
  bc[(size_t)q * gc.N + C] = (TX)restrict_node<D, TX>(gf, gc, r + (size_t)q * gf.N, C);
}

// Restriction fused with the coarse level's first Chebyshev step (which needs
// only its own node): bc = R r, xc = dc = c2 D_c^-1 bc.
template <int D, typename TV, typename TX>
__global__ __launch_bounds__(256) void k_restrict_first(GridDev gf, GridDev gc,
                                                        const TX *__restrict__ r,
                                                        TX *__restrict__ bc,
                                                        const TV *__restrict__ dinvc,
                                                        TX *__restrict__ xc, TX *__restrict__ dc,
                                                        Sc2 c2) {
  const int q = blockIdx.y;
  const long C = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= gc.N) return;
  const size_t ic = (size_t)q * gc.N + C;
  const TX bv = (TX)restrict_node<D, TX>(gf, gc, r + (size_t)q * gf.N, C);
  bc[ic] = bv;
  const double v = c2.v[q] * (double)dinvc[ic] * (double)bv;
  dc[ic] = (TX)v;
  xc[ic] = (TX)v;
}

// x(f) += (P e)(f), or x(f) = (P e)(f) when assign (no pre-smoothing: x was 0)
template <int D, typename TX>
__global__ __launch_bounds__(256) void k_prolong(GridDev gf, GridDev gc, const TX *__restrict__ e,
                                                 TX *__restrict__ x, int assign) {
  const long N = gf.N;
  const int q = blockIdx.y;
  const long f = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (f >= N) return;
  const double v = prolong_node<D, TX>(gf, gc, e + (size_t)q * gc.N, f);
  x[(size_t)q * N + f] = (TX)(assign ? v : (double)x[(size_t)q * N + f] + v);
}

// Galerkin coarse operator A_c(C, C+t) = sum_{f, g} P(f,C) A(f,g) P(g,C+t).
template <int D>
__device__ inline int fine_support(const GridDev &gf, const GridDev &gc, const int *cc, int fs[][3],
                                   double *w) {
  if constexpr (is_q1(D)) {
    // box cells: the tensor product of the axes' supports (at most 27 nodes)
    int f[3][3], k[3];
    double wa[3][3];
    for (int ax = 0; ax < 3; ++ax) k[ax] = axis_support(cc[ax], gf.n[ax], gc.m[ax], f[ax], wa[ax]);
    int n = 0;
    for (int z = 0; z < k[2]; ++z)
      for (int y = 0; y < k[1]; ++y)
        for (int x = 0; x < k[0]; ++x, ++n) {
          fs[n][0] = f[0][x];
          fs[n][1] = f[1][y];
          fs[n][2] = f[2][z];
          w[n] = wa[0][x] * wa[1][y] * wa[2][z];
        }
    return n;
  }
  int ex[3];
  for (int ax = 0; ax < 3; ++ax) ex[ax] = exact_fine(cc[ax], gf.n[ax], gc.m[ax]);
  int k = 0;
  for (int ax = 0; ax < 3; ++ax) fs[0][ax] = ex[ax];
  w[k++] = 1.0;
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
    if (uok) {
      for (int ax = 0; ax < 3; ++ax) fs[k][ax] = fu[ax];
      w[k++] = 0.5;
    }
    if (dok) {
      for (int ax = 0; ax < 3; ++ax) fs[k][ax] = fd[ax];
      w[k++] = 0.5;
    }
  }
  return k;
}

template <int D>
__global__ __launch_bounds__(256) void k_galerkin(GridDev gf, GridDev gc, const double *__restrict__ A,
                                                  double *__restrict__ Ac) {
  constexpr int NT = Tabs<D>::NT;
  constexpr int NS = Tabs<D>::NS;
  const long Nc = gc.N;
  const int q = blockIdx.y;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Nc * NT) return;
  const int t = (int)(idx / Nc);
  const long C = idx - (long)t * Nc;
  int cc[3], c2[3];
  node_ijk(gc, C, cc[0], cc[1], cc[2]);
  const int *o = TAB<D>.to[t];
  for (int ax = 0; ax < 3; ++ax) c2[ax] = cc[ax] + o[ax];
  double acc = 0.0;
  if (inside(gc, c2[0], c2[1], c2[2])) {
    int fs[NS][3], gs[NS][3];
    double wf[NS], wg[NS];
    const int nf = fine_support<D>(gf, gc, cc, fs, wf);
    const int ng = fine_support<D>(gf, gc, c2, gs, wg);
    const double *Aq = A + (size_t)q * NT * gf.ld;
    for (int u = 0; u < nf; ++u) {
      const long fidx = fs[u][0] + (long)gf.m[0] * (fs[u][1] + (long)gf.m[1] * fs[u][2]);
      double s = 0.0;
      for (int v = 0; v < ng; ++v) {
        const int dx = gs[v][0] - fs[u][0], dy = gs[v][1] - fs[u][1], dz = gs[v][2] - fs[u][2];
        if (dx < -2 || dx > 2 || dy < -2 || dy > 2 || dz < -2 || dz > 2) continue;
        const int tt = TAB<D>.tidx[(dx + 2) + 5 * (dy + 2) + 25 * (dz + 2)];
        if (tt < 0) continue;
        s += wg[v] * Aq[(size_t)tt * gf.ld + fidx];
      }
      acc += wf[u] * s;
    }
  }
  Ac[((size_t)q * NT + t) * gc.ld + C] = acc;
}

template <int D>
__global__ void k_diag_inv(GridDev g, const double *__restrict__ A, double *__restrict__ dinv) {
  constexpr int NT = Tabs<D>::NT;
  const long N = g.N;
  const int q = blockIdx.y;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  dinv[(size_t)q * N + a] = 1.0 / A[((size_t)q * NT + TAB<D>.t0) * g.ld + a];
}

template <int D>
__global__ void k_dense_fill(GridDev g, const double *__restrict__ A, double *__restrict__ M) {
  constexpr int NT = Tabs<D>::NT;
  const long N = g.N;
  const int q = blockIdx.y;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int i, j, k;
  node_ijk(g, a, i, j, k);
  double *Mq = M + (size_t)q * N * N + (size_t)a * N;
  for (long c = 0; c < N; ++c) Mq[c] = 0.0;
  for (int t = 0; t < NT; ++t) {
    const int *o = TAB<D>.to[t];
    if (!inside(g, i + o[0], j + o[1], k + o[2])) continue;
    Mq[a + lin(g, o[0], o[1], o[2])] = A[((size_t)q * NT + t) * g.ld + a];
  }
}

// In-place Gauss-Jordan inversion of the coarsest operators, without pivoting
// (they are symmetric positive definite), blocked: the pivots of block
// I = [k0, k0 + nb) in one step of three launches over both networks.  With
// P = A[I,I] and the snapshots R = A[I,:], C = A[:,I] of the current matrix,
// the nb scalar steps amount to
//   A[I,I] = P^-1,  A[I,J] = P^-1 R[:,J],  A[J,I] = -C[J,:] P^-1,
//   A[J,J] = A[J,J] - C[J,:] P^-1 R[:,J]       (J = the other indices).
constexpr int GJB = 32;

// (1) snapshots R, C and the inverse of P (scalar Gauss-Jordan in LDS, block 0).
__global__ __launch_bounds__(256) void k_bgj_panel(const double *__restrict__ M, int n, int k0,
                                                   int nb, double *__restrict__ rbuf,
                                                   double *__restrict__ cbuf,
                                                   double *__restrict__ pinv,
                                                   int *__restrict__ bad) {
  const int q = blockIdx.y;
  const double *A = M + (size_t)q * n * n;
  if (blockIdx.x == 0) {
    __shared__ double P[GJB][GJB + 1];
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x)
      P[e / nb][e % nb] = A[(size_t)(k0 + e / nb) * n + k0 + e % nb];
    __syncthreads();
    constexpr int PER = GJB * GJB / 256;
    for (int k = 0; k < nb; ++k) {
      double v[PER];
      // an SPD matrix has positive pivots; anything else is reported
      if (threadIdx.x == 0 && !(P[k][k] > 0.0 && P[k][k] < INFINITY)) bad[q] = 1;
      const double ip = 1.0 / P[k][k];
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * 256, i = e / nb, j = e % nb;
        if (e >= nb * nb) continue;
        v[u] = (i == k && j == k) ? ip
             : (i == k) ? P[k][j] * ip
             : (j == k) ? -P[i][k] * ip
             : P[i][j] - P[i][k] * P[k][j] * ip;
      }
      __syncthreads();
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * 256;
        if (e < nb * nb) P[e / nb][e % nb] = v[u];
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x)
      pinv[(size_t)q * GJB * GJB + e] = P[e / nb][e % nb];
    return;
  }
  // the other blocks copy the block rows and columns
  const long tot = 2L * nb * n;
  for (long e = (long)(blockIdx.x - 1) * blockDim.x + threadIdx.x; e < tot;
       e += (long)(gridDim.x - 1) * blockDim.x) {
    if (e < (long)nb * n) {
      const int m = (int)(e / n), j = (int)(e % n);
      rbuf[(size_t)q * GJB * n + (size_t)m * n + j] = A[(size_t)(k0 + m) * n + j];
    } else {
      const long f = e - (long)nb * n;
      const int i = (int)(f / nb), m = (int)(f % nb);
      cbuf[(size_t)q * n * GJB + (size_t)i * GJB + m] = A[(size_t)i * n + k0 + m];
    }
  }
}

// (2) T = P^-1 R  (nb x n), into tbuf.
__global__ __launch_bounds__(256) void k_bgj_rows(int n, int nb, const double *__restrict__ rbuf,
                                                  const double *__restrict__ pinv,
                                                  double *__restrict__ tbuf) {
  const int q = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)nb * n) return;
  const int m = (int)(e / n), j = (int)(e % n);
  const double *R = rbuf + (size_t)q * GJB * n, *Pi = pinv + (size_t)q * GJB * GJB;
  double acc = 0.0;
  for (int l = 0; l < nb; ++l) acc += Pi[m * nb + l] * R[(size_t)l * n + j];
  tbuf[(size_t)q * GJB * n + (size_t)m * n + j] = acc;
}

// (3) every entry of the matrix from the snapshots, P^-1 and T.
__global__ __launch_bounds__(256) void k_bgj_update(double *__restrict__ M, int n, int k0, int nb,
                                                    const double *__restrict__ cbuf,
                                                    const double *__restrict__ pinv,
                                                    const double *__restrict__ tbuf) {
  const int q = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  double *A = M + (size_t)q * n * n;
  const double *C = cbuf + (size_t)q * n * GJB + (size_t)i * GJB;
  const double *Pi = pinv + (size_t)q * GJB * GJB, *T = tbuf + (size_t)q * GJB * n;
  const bool ii = i >= k0 && i < k0 + nb, jj = j >= k0 && j < k0 + nb;
  double v;
  if (ii) {
    v = jj ? Pi[(i - k0) * nb + (j - k0)] : T[(size_t)(i - k0) * n + j];
  } else if (jj) {
    v = 0.0;
    for (int m = 0; m < nb; ++m) v -= C[m] * Pi[m * nb + (j - k0)];
  } else {
    v = A[e];
    for (int m = 0; m < nb; ++m) v -= C[m] * T[(size_t)m * n + j];
  }
  A[e] = v;
}

// x = Cinv b on the coarsest level (FP64 arithmetic); one wavefront per row.
template <typename TX>
__global__ __launch_bounds__(256) void k_coarse(const double *__restrict__ Cinv, int n,
                                                const TX *__restrict__ b, TX *__restrict__ x) {
  const int q = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  const double *Mr = Cinv + (size_t)q * n * n + (size_t)row * n;
  const TX *bq = b + (size_t)q * n;
  // four independent partial sums, so four loads per lane are in flight
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int c = lane;
  for (; c + 192 < n; c += 256) {
    s0 += Mr[c] * (double)bq[c];
    s1 += Mr[c + 64] * (double)bq[c + 64];
    s2 += Mr[c + 128] * (double)bq[c + 128];
    s3 += Mr[c + 192] * (double)bq[c + 192];
  }
  for (; c < n; c += 64) s0 += Mr[c] * (double)bq[c];
  double s = (s0 + s1) + (s2 + s3);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) x[(size_t)q * n + row] = (TX)s;
}

// Per-network sum of squares: partials [2][nblk], then a fixed-order final sum.
__global__ __launch_bounds__(256) void k_sumsq2(const double *__restrict__ x, long n,
                                                double *__restrict__ part) {
  const int q = blockIdx.y;
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double v = x[(size_t)q * n + i];
    s += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ double w[4];
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[q * gridDim.x + blockIdx.x] = w[0] + w[1] + w[2] + w[3];
}

// out[q] = sum of the nb partials of network q; one 256-thread block,
// fixed order (strided per-thread sums, wave trees, then the four waves).
__global__ __launch_bounds__(256) void k_sum2(const double *__restrict__ part, int nb,
                                              double *__restrict__ out) {
  __shared__ double w[2][4];
  for (int q = 0; q < 2; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[q * nb + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) w[q][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < 2) out[threadIdx.x] = w[threadIdx.x][0] + w[threadIdx.x][1] + w[threadIdx.x][2] + w[threadIdx.x][3];
}

__global__ void k_hash_start(double *__restrict__ x, long n) {
  const int q = blockIdx.y;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long h = ((unsigned long long)i * 2654435761ull) & 0xffffffffull;
  x[(size_t)q * n + i] = (double)h / 4294967296.0 - 0.5;
}

__global__ void k_scale2(double *__restrict__ x, long n, const double *__restrict__ ss) {
  const int q = blockIdx.y;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[(size_t)q * n + i] /= sqrt(ss[q]);
}

__global__ void k_f64_to_f32(const double *__restrict__ x, float *__restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

constexpr int RED_BLOCKS = 512;

// Autotuner for the kernel shape of the level stencil kernels (lanes per
// row 1/2/4/8 or two rows per lane, full or symmetric-half storage): each
// candidate is timed with HIP events on the level's own operator and the
// fastest wins; results are cached per (dim, nodes, value bytes) for the
// process.
std::mutex g_tune_mu;
std::map<std::tuple<int, long, int>, Shape> g_tune_cache;

template <int D>
Shape tune_shape(Level &L, hipStream_t s) {
  const auto key = std::make_tuple(D, L.g.N, 8);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) return it->second;
  }
  hipEvent_t e0, e1;
  DPP_HIP(hipEventCreate(&e0));
  DPP_HIP(hipEventCreate(&e1));
  Shape best;
  float best_ms = 1e30f;
  const double *x = L.xa.as<double>();
  double *y = L.xb.as<double>();
  DPP_HIP(hipMemsetAsync(L.xa.ptr, 0, L.xa.bytes, s));
  for (int sym = 0; sym < 2; ++sym)
    for (int cand : {1, 0, 2, 4, 8}) {
      const Shape sh{cand, sym != 0};
      const double *A = sh.sym ? L.Ah.as<double>() : L.A.as<double>();
      launch_lspmv<D, double, double>(sh, L.g, s, A, x, y, nullptr, nullptr);
      DPP_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 5; ++r) launch_lspmv<D, double, double>(sh, L.g, s, A, x, y, nullptr, nullptr);
      DPP_HIP(hipEventRecord(e1, s));
      DPP_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      DPP_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms * 0.97f) {  // prefer the simpler shape unless clearly faster
        best_ms = ms;
        best = sh;
      }
    }
  check_launch("tune_shape");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best;
  return best;
}

template <int D>
void pack_half(Level &L, hipStream_t s) {
  constexpr int NH = Tabs<D>::NT - TAB<D>.t0;
  L.Ah.alloc(sizeof(double) * 2 * NH * padded(L.g.N));
  k_pack_half<D, double><<<dim3(blocks_for((long)NH * L.g.N, 256), 2), 256, 0, s>>>(
      L.A.as<double>(), L.g.N, padded(L.g.N), L.Ah.as<double>());
  check_launch("pack_half");
}

// Per-network sums of squares of x into red[2 RED_BLOCKS .. +2) (device only).
template <int D>
void sumsq2(dpp_precond pc, const double *x, long n, hipStream_t s) {
  double *part = pc->red.as<double>();
  k_sumsq2<<<dim3(RED_BLOCKS, 2), 256, 0, s>>>(x, n, part);
  k_sum2<<<1, 256, 0, s>>>(part, RED_BLOCKS, part + 2 * RED_BLOCKS);
  check_launch("sumsq2");
}

template <int D>
void setup_impl(dpp_precond pc, hipStream_t s) {
  constexpr int NT = Tabs<D>::NT;
  dpp_problem P = pc->prob;
  const dpp_solve_opts &o = pc->opts;
  pc->red.alloc(sizeof(double) * (2 * RED_BLOCKS + 4));
  Grid g = P->g;
  auto lev0 = std::make_unique<Level>();
  lev0->g = g;
  lev0->A.alloc(sizeof(double) * 2 * NT * padded(g.N));
  make_selfp(P, lev0->A.as<double>(), s);
  pc->lv.push_back(std::move(lev0));
  while (true) {
    Level &L = *pc->lv.back();
    const Grid &gl = L.g;
    L.dinv.alloc(sizeof(double) * 2 * gl.N);
    dim3 grid(blocks_for(gl.N, 256), 2);
    k_diag_inv<D><<<grid, 256, 0, s>>>(dev(gl), L.A.as<double>(), L.dinv.as<double>());
    check_launch("diag_inv");
    for (DBuf *b : {&L.b, &L.xa, &L.xb, &L.d, &L.r, &L.e}) b->alloc(sizeof(double) * 2 * gl.N);
    Grid gc = coarse_grid(gl);
    // coarsest size: given, or by dimension.  In 3D an exact solve on a level
    // of up to 2200 nodes (13^3 below 97^3) applies its dense inverse faster
    // than the V-cycle over the two levels under it, and being exact one level
    // higher also saves FGMRES iterations (96^3 log-normal: 27 -> 23); in 2D
    // the dense inverses of ~1000-node levels cost more than one more cheap level.
    const long cmax = o.coarse_max > 0 ? o.coarse_max : (dim_of(D) == 3 ? 2200 : 400);
    const bool last = gl.N <= cmax || gc.N == gl.N || (int)pc->lv.size() >= 16;
    if (last) break;
    // Chebyshev bounds from normalised power steps on D^-1 A; the norms stay
    // on the device, only the last one comes back to the host
    double *x = L.xa.as<double>(), *y = L.xb.as<double>();
    const double *ssd = pc->red.as<double>() + 2 * RED_BLOCKS;
    k_hash_start<<<grid, 256, 0, s>>>(x, gl.N);
    sumsq2<D>(pc, x, gl.N, s);
    k_scale2<<<grid, 256, 0, s>>>(x, gl.N, ssd);
    for (int it = 0; it < o.power_iters; ++it) {
      launch_lspmv<D, double, double>(Shape{}, gl, s, L.A.as<double>(), x, y, nullptr, L.dinv.as<double>());
      sumsq2<D>(pc, y, gl.N, s);
      k_scale2<<<grid, 256, 0, s>>>(y, gl.N, ssd);
      std::swap(x, y);
    }
    double ss[2] = {0.0, 0.0}, lam[2] = {0.0, 0.0};
    if (o.power_iters > 0) {
      DPP_HIP(hipMemcpyAsync(ss, ssd, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      DPP_HIP(hipStreamSynchronize(s));
      lam[0] = std::sqrt(ss[0]);
      lam[1] = std::sqrt(ss[1]);
    }
    for (int q = 0; q < 2; ++q) {
      DPP_CHECK(std::isfinite(lam[q]) && lam[q] > 0.0, DPP_ERR_NUMERIC,
                "multigrid eigenvalue estimate failed");
      L.hi[q] = o.cheb_hi_factor * lam[q];
      // lower end of the interval: given, or by dimension (0.1 in 3D, 0.3 in 2D)
      const double lof = o.cheb_lo_frac > 0.0 ? o.cheb_lo_frac : (dim_of(D) == 3 ? 0.1 : 0.3);
      L.lo[q] = lof * L.hi[q];
    }
    auto C = std::make_unique<Level>();
    C->g = gc;
    C->A.alloc(sizeof(double) * 2 * NT * padded(gc.N));
    dim3 gg(blocks_for(gc.N * NT, 256), 2);
    k_galerkin<D><<<gg, 256, 0, s>>>(dev(gl), dev(gc), L.A.as<double>(), C->A.as<double>());
    check_launch("galerkin");
    pc->lv.push_back(std::move(C));
  }
  for (size_t l = 0; l + 1 < pc->lv.size(); ++l) {
    pack_half<D>(*pc->lv[l], s);
    // members of a batch run the batched kernels, whose lanes are tuned over
    // the whole batch: their own shapes are never used.  A fixed schedule
    // s in 0..9 puts lanes {pairs, 1, 2, 4, 8}[s % 5] (symmetric half storage
    // for s >= 5) on every level.
    static constexpr int kLanes[5] = {0, 1, 2, 4, 8};
    const int sch = pc->opts.schedule;
    if (!pc->tune_shapes)
      pc->lv[l]->shape = Shape{};
    else if (sch >= 0)
      pc->lv[l]->shape = Shape{kLanes[sch % 5], sch >= 5};
    else
      pc->lv[l]->shape = tune_shape<D>(*pc->lv[l], s);
  }
  Level &Lc = *pc->lv.back();
  const int n = (int)Lc.g.N;
  DPP_CHECK(n <= 4000, DPP_ERR_ARG, "coarsest multigrid level too large (lower coarse_max)");
  pc->ncoarse = n;
  pc->cinv.alloc(sizeof(double) * 2 * (size_t)n * n);
  k_dense_fill<D><<<dim3(blocks_for(n, 64), 2), 64, 0, s>>>(dev(Lc.g), Lc.A.as<double>(),
                                                             pc->cinv.as<double>());
  {
    // blocked Gauss-Jordan, GJB pivots per step
    DBuf rb(sizeof(double) * 2 * GJB * n), cb(sizeof(double) * 2 * GJB * n),
        tb(sizeof(double) * 2 * GJB * n), pb(sizeof(double) * 2 * GJB * GJB), bad(sizeof(int) * 2);
    DPP_HIP(hipMemsetAsync(bad.ptr, 0, sizeof(int) * 2, s));
    const dim3 gp(1 + std::min(1024, blocks_for(2L * GJB * n, 256)), 2);
    const dim3 gr(blocks_for((long)GJB * n, 256), 2), gu(blocks_for((long)n * n, 256), 2);
    for (int k0 = 0; k0 < n; k0 += GJB) {
      const int nb = std::min(GJB, n - k0);
      k_bgj_panel<<<gp, 256, 0, s>>>(pc->cinv.as<double>(), n, k0, nb, rb.as<double>(),
                                     cb.as<double>(), pb.as<double>(), bad.as<int>());
      k_bgj_rows<<<gr, 256, 0, s>>>(n, nb, rb.as<double>(), pb.as<double>(), tb.as<double>());
      k_bgj_update<<<gu, 256, 0, s>>>(pc->cinv.as<double>(), n, k0, nb, cb.as<double>(),
                                      pb.as<double>(), tb.as<double>());
    }
    check_launch("coarse inverse");
    int hbad[2] = {0, 0};
    DPP_HIP(hipMemcpyAsync(hbad, bad.ptr, sizeof(hbad), hipMemcpyDeviceToHost, s));
    DPP_HIP(hipStreamSynchronize(s));
    DPP_CHECK(!hbad[0] && !hbad[1], DPP_ERR_NUMERIC,
              "coarsest multigrid operator is not positive definite (non-positive or "
              "non-finite pivot in its inverse)");
  }
  pc->rhat.alloc(sizeof(double) * 2 * P->g.N);
  DPP_HIP(hipStreamSynchronize(s));
}

// Chebyshev coefficients of step k: k = 0 -> (0, 1/theta); k >= 1 ->
// (rho_k rho_{k-1}, 2 rho_k / delta), rho_0 = delta/theta,
// rho_k = 1/(2 sigma - rho_{k-1}), sigma = theta/delta.
void cheb_coefs(const Level &L, int deg, std::vector<Sc2> &c1, std::vector<Sc2> &c2) {
  c1.assign(deg, Sc2{{0, 0}});
  c2.assign(deg, Sc2{{0, 0}});
  for (int q = 0; q < 2; ++q) {
    const double theta = 0.5 * (L.hi[q] + L.lo[q]), delta = 0.5 * (L.hi[q] - L.lo[q]);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    c1[0].v[q] = 0.0;
    c2[0].v[q] = 1.0 / theta;
    for (int k = 1; k < deg; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1[k].v[q] = rn * rho;
      c2[k].v[q] = 2.0 * rn / delta;
      rho = rn;
    }
  }
}

template <typename TX>
struct LevelBufs {
  TX *b, *xa, *xb, *d, *r, *e;
  const void *A, *dinv;
};

template <typename TX>
LevelBufs<TX> bufs(Level &L);
template <>
LevelBufs<double> bufs<double>(Level &L) {
  return {L.b.as<double>(), L.xa.as<double>(), L.xb.as<double>(), L.d.as<double>(),
          L.r.as<double>(), L.e.as<double>(), L.shape.sym ? L.Ah.ptr : L.A.ptr, L.dinv.ptr};
}
template <>
LevelBufs<float> bufs<float>(Level &L) {
  return {L.b32.as<float>(), L.xa32.as<float>(), L.xb32.as<float>(), L.d32.as<float>(),
          L.r32.as<float>(), L.e32.as<float>(), L.shape.sym ? L.Ah32.ptr : L.A32.ptr,
          L.dinv32.ptr};
}

// V-cycle from level l.  first_done: the producer of b already wrote the
// first Chebyshev step (x = d = c2 D^-1 b) into the level's xa and d.
template <int D, typename TX>
void vcyc(dpp_precond pc, int l, const TX *b, TX *xout, hipStream_t s, bool first_done = false) {
  using TV = TX;  // FP64 levels in FP64 mode, FP32 levels in mixed mode
  const int nl = (int)pc->lv.size();
  Level &L = *pc->lv[l];
  const GridDev gd = dev(L.g);
  const dim3 grid(blocks_for(L.g.N, 256), 2);
  const double tv = sizeof(TV), tx = sizeof(TX), Nl = (double)L.g.N;
  // stored matrix entries the format must stream: the full stencil, or with
  // symmetric storage the zero offset plus the positive half
  const double pairs_full = valid_pairs<D, true>(L.g);
  const double pairs = L.shape.sym ? 0.5 * (pairs_full + Nl) : pairs_full;
  if (l == nl - 1) {
    const int n = pc->ncoarse;
    ProfScope ps(PF_COARSE, 2.0 * n * (n * 8.0 + 2 * tx), s);
    k_coarse<TX><<<dim3(blocks_for(n, 4), 2), 256, 0, s>>>(pc->cinv.as<double>(), n, b, xout);
    check_launch("coarse solve");
    return;
  }
  LevelBufs<TX> B = bufs<TX>(L);
  const TV *A = (const TV *)B.A, *di = (const TV *)B.dinv;
  const int pre = cheb_pre(pc->opts, l), post = cheb_post(pc->opts, l);
  std::vector<Sc2> c1, c2;
  cheb_coefs(L, std::max(pre, post), c1, c2);  // step k's coefficients do not depend on the degree
  TX *cur = B.xa, *oth = B.xb;
  const bool fine = l == 0;
  const int fam_cheb = fine ? PF_CHEB_L0 : PF_COARSE;
  const int fam_res = fine ? PF_RESID_L0 : PF_COARSE;
  const int fam_vec = fine ? PF_VECTOR_L0 : PF_COARSE;
  // Chebyshev step bytes: matrix entries + dinv, b, x_in, d_in (k>=1), d, x_out
  auto cheb_bytes = [&](bool zero_x, bool dread) {
    return 2.0 * ((zero_x ? 0.0 : pairs * tv) + Nl * (tv + tx * (zero_x ? 3.0 : 4.0) +
                                                     (dread ? tx : 0.0)));
  };
  const Shape lpr = L.shape;
  // what is restricted: the residual after pre-smoothing, or b itself (x = 0)
  const TX *rr = b;
  if (pre > 0) {
    // pre-smoothing from x = 0
    if (!first_done) {
      ProfScope ps(fam_vec, cheb_bytes(true, false), s);
      k_cheb_first<TV, TX><<<dim3(blocks_for(L.g.N, 256), 2), 256, 0, s>>>(L.g.N, di, b, cur, B.d, c2[0]);
    }
    for (int k = 1; k < pre; ++k) {
      ProfScope ps(fam_cheb, cheb_bytes(false, true), s);
      launch_cheb<D, TV, TX>(lpr, L.g, s, A, di, b, cur, oth, B.d, c1[k], c2[k], fine);
      std::swap(cur, oth);
    }
    ProfScope ps(fam_res, 2.0 * (pairs * tv + 3.0 * Nl * tx), s);
    launch_lspmv<D, TV, TX>(lpr, L.g, s, A, cur, B.r, b, (const TV *)nullptr, fine);
    rr = B.r;
  }
  // restriction and coarse correction
  Level &Cl = *pc->lv[l + 1];
  LevelBufs<TX> CB = bufs<TX>(Cl);
  // the coarse level pre-smooths: fuse its first step into the restriction
  const bool fuse = l + 1 < nl - 1 && cheb_pre(pc->opts, l + 1) > 0;
  if (fuse) {
    std::vector<Sc2> cc1, cc2;
    cheb_coefs(Cl, 1, cc1, cc2);
    ProfScope ps(fam_vec, 2.0 * (tx * (Nl + 3.0 * Cl.g.N) + tv * Cl.g.N), s);
    k_restrict_first<D, TV, TX><<<dim3(blocks_for(Cl.g.N, 256), 2), 256, 0, s>>>(
        gd, dev(Cl.g), rr, CB.b, (const TV *)CB.dinv, CB.xa, CB.d, cc2[0]);
  } else {
    ProfScope ps(fam_vec, 2.0 * tx * (Nl + Cl.g.N), s);
    k_restrict<D, TX><<<dim3(blocks_for(Cl.g.N, 256), 2), 256, 0, s>>>(gd, dev(Cl.g), rr, CB.b);
  }
  vcyc<D, TX>(pc, l + 1, CB.b, CB.e, s, fuse);
  {
    ProfScope ps(fam_vec, 2.0 * tx * ((pre > 0 ? 2.0 : 1.0) * Nl + Cl.g.N), s);
    k_prolong<D, TX><<<grid, 256, 0, s>>>(gd, dev(Cl.g), CB.e, cur, pre > 0 ? 0 : 1);
  }
  // post-smoothing
  for (int k = 0; k < post; ++k) {
    TX *out = (k == post - 1) ? xout : oth;
    ProfScope ps(fam_cheb, cheb_bytes(false, k > 0), s);
    launch_cheb<D, TV, TX>(lpr, L.g, s, A, di, b, cur, out, B.d, c1[k], c2[k], fine);
    oth = cur;
    cur = out;
  }
  check_launch("vcycle");
}

}  // namespace

void precond_setup(dpp_precond pc, hipStream_t s) {
  DPP_TAG_SWITCH(pc->prob->g, (setup_impl<D_>(pc, s)));
}

void precond_make32(dpp_precond pc, hipStream_t s) {
  if (pc->prob->dg) {
    dg_make32(pc, s);
    return;
  }
  if (pc->has32) return;
  make_k32(pc->prob, s);
  for (auto &lp : pc->lv) {
    Level &L = *lp;
    const size_t nA = L.A.bytes / sizeof(double), nv = 2 * (size_t)L.g.N;
    L.A32.alloc(nA * sizeof(float));
    k_f64_to_f32<<<2048, 256, 0, s>>>(L.A.as<double>(), L.A32.as<float>(), nA);
    if (L.Ah.ptr) {
      const size_t nH = L.Ah.bytes / sizeof(double);
      L.Ah32.alloc(nH * sizeof(float));
      k_f64_to_f32<<<2048, 256, 0, s>>>(L.Ah.as<double>(), L.Ah32.as<float>(), nH);
    }
    if (L.dinv.ptr) {
      L.dinv32.alloc(nv * sizeof(float));
      k_f64_to_f32<<<256, 256, 0, s>>>(L.dinv.as<double>(), L.dinv32.as<float>(), nv);
    }
    for (DBuf *b : {&L.b32, &L.xa32, &L.xb32, &L.d32, &L.r32, &L.e32}) b->alloc(nv * sizeof(float));
  }
  pc->rhat32.alloc(sizeof(float) * 2 * pc->prob->g.N);
  check_launch("precond fp32");
  pc->has32 = true;
}

void vcycle(dpp_precond pc, const double *b, double *x, hipStream_t s) {
  DPP_TAG_SWITCH(pc->prob->g, (vcyc<D_, double>(pc, 0, b, x, s)));
}

void vcycle32(dpp_precond pc, const float *b, float *x, hipStream_t s) {
  DPP_CHECK(pc->has32, DPP_ERR_ARG, "internal: FP32 levels not set up");
  DPP_TAG_SWITCH(pc->prob->g, (vcyc<D_, float>(pc, 0, b, x, s)));
}

void precond_apply(dpp_precond pc, const double *r, double *z, bool fp32, hipStream_t s) {
  dpp_problem P = pc->prob;
  if (P->dg) {
    dg_precond_apply(pc, r, z, fp32, s);
    return;
  }
  Level &L0 = *pc->lv[0];
  // the Schur right-hand side kernel also writes the finest level's first
  // Chebyshev step when that level smooths
  const bool fuse = pc->lv.size() > 1 && cheb_pre(pc->opts, 0) > 0;
  const Grid &g = P->g;
  double c2q[2] = {0.0, 0.0};
  if (fuse) {
    std::vector<Sc2> c1, c2;
    cheb_coefs(L0, 1, c1, c2);
    c2q[0] = c2[0].v[0];
    c2q[1] = c2[0].v[1];
  }
  if (fp32) {
    schur_rhs(P, r, pc->rhat32.ptr, true, s, fuse ? L0.dinv32.ptr : nullptr, L0.xa32.ptr, L0.d32.ptr, c2q);
    DPP_TAG_SWITCH(g, (vcyc<D_, float>(pc, 0, pc->rhat32.as<float>(), L0.e32.as<float>(), s, fuse)));
    schur_velocity(P, r, L0.e32.ptr, true, z, s);
  } else {
    schur_rhs(P, r, pc->rhat.ptr, false, s, fuse ? L0.dinv.ptr : nullptr, L0.xa.ptr, L0.d.ptr, c2q);
    DPP_TAG_SWITCH(g, (vcyc<D_, double>(pc, 0, pc->rhat.as<double>(), L0.e.as<double>(), s, fuse)));
    schur_velocity(P, r, L0.e.ptr, false, z, s);
  }
}

void level_spmv(dpp_precond pc, int level, int net, const double *x, double *y, hipStream_t s) {
  Level &L = *pc->lv[level];
  const long N = L.g.N;
  // run both networks through the scratch vectors, copy the requested one
  DPP_HIP(hipMemsetAsync(L.r.ptr, 0, sizeof(double) * 2 * N, s));
  DPP_HIP(hipMemcpyAsync(L.r.as<double>() + net * N, x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  const double *A = L.shape.sym ? L.Ah.as<double>() : L.A.as<double>();
  DPP_TAG_SWITCH(L.g, (launch_lspmv<D_, double, double>(L.shape, L.g, s, A, L.r.as<double>(),
                                                        L.d.as<double>(), nullptr, nullptr)));
  check_launch("level_spmv");
  DPP_HIP(hipMemcpyAsync(y, L.d.as<double>() + net * N, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
}

}  // namespace dpp
