// Operators on the unknown vector [u1 | p1 | u2 | p2]: y = K x, residuals,
// the block views K_up^i / K_pu^i, the selfp Schur blocks and the two
// velocity-side steps of the Schur fieldsplit.
//
// The K product is bandwidth bound.  It reads the half storage of K (the
// symmetric kinds on the zero offset and the positive half of the stencil;
// structure-of-arrays, coalesced), takes the other half from the neighbours'
// rows, which are at most one node plane away and mostly served from L2, and
// takes every K_up / K_pu value from the class table (UPT), which each
// workgroup stages in LDS.  The two velocity-side steps of the fieldsplit read
// only that table for their K blocks.  Assembly, selfp and the CSR export
// read the full node-pair storage.
#include <algorithm>
#include <vector>

#include "objects.h"
#include "profile.h"
#include "stencil.h"

namespace dpp {

namespace {

// One workgroup of KBS threads per block of 2 KBS nodes (a node pair per
// thread), or of KBS nodes with velocity faces (one node per thread: the
// masked pair form needs 170 registers and ran 30% slower at 64^3); order[]
// gives the node block of each workgroup (band order, below).
constexpr int KBS = 128;
inline int k_block_nodes(const Grid &g) { return (g.fix[0] | g.fix[1]) != 0 ? KBS : 2 * KBS; }

// The K_up class table (UPT<D>) copied into LDS by every workgroup.
template <int D, typename TV>
__device__ inline void stage_upt(TV *sut, const TV *__restrict__ upt) {
  for (int i = threadIdx.x; i < UPT<D>::size; i += blockDim.x) sut[i] = upt[i];
  __syncthreads();
}

// One node per thread, for problems with velocity faces (BC): their
// prescribed components have identity rows (y_u = x_u there).
template <int D, typename TV>
__global__ __launch_bounds__(256) void k_spmv_K1(GridDev g, const TV *__restrict__ kv,
                                                 const TV *__restrict__ upt,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ bsub,
                                                 double *__restrict__ y,
                                                 const int *__restrict__ order) {
  constexpr int d = dim_of(D);
  __shared__ TV sut[UPT<D>::size];
  stage_upt<D>(sut, upt);
  const long N = g.N;
  const long a = (long)order[blockIdx.x] * KBS + threadIdx.x;
  if (a >= N) return;
  double au[2][d], ap[2];
  spmv_K_node<D, TV, true>(g, kv, sut, x, a, au, ap);
  int ia[3];
  node_ijk(g, a, ia[0], ia[1], ia[2]);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const long ou = off_u(d, N, q), op = off_p(d, N, q);
#pragma unroll
    for (int c = 0; c < d; ++c) {
      const long r = ou + d * a + c;
      const double v = u_fixed(g, q, c, ia) ? x[r] : au[q][c];
      y[r] = bsub ? bsub[r] - v : v;
    }
    y[op + a] = bsub ? bsub[op + a] - ap[q] : ap[q];
  }
}

// Node pairs, for problems without velocity faces.
template <int D, typename TV>
__global__ __launch_bounds__(256) void k_spmv_K(GridDev g, const TV *__restrict__ kv,
                                                const TV *__restrict__ upt,
                                                const double *__restrict__ x,
                                                const double *__restrict__ bsub,
                                                double *__restrict__ y,
                                                const int *__restrict__ order) {
  constexpr int d = dim_of(D);
  __shared__ TV sut[UPT<D>::size];
  stage_upt<D>(sut, upt);
  const long N = g.N;
  const long a = 2 * ((long)order[blockIdx.x] * KBS + threadIdx.x);
  if (a >= N) return;
  double au[2][2][d], ap[2][2];
  spmv_K_node2<D, TV>(g, kv, sut, x, a, au, ap);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const long ou = off_u(d, N, q), op = off_p(d, N, q);
    if (a + 1 < N) {
#pragma unroll
      for (int e = 0; e < d; ++e) {
        // values 2e, 2e + 1 of the pair's 2d velocity unknowns
        const double v0 = au[(2 * e) / d][q][(2 * e) % d], v1 = au[(2 * e + 1) / d][q][(2 * e + 1) % d];
        double b0 = 0.0, b1 = 0.0;
        if (bsub) ld2(bsub + ou + d * a + 2 * e, b0, b1);
        st2(y + ou + d * a + 2 * e, bsub ? b0 - v0 : v0, bsub ? b1 - v1 : v1);
      }
      double b0 = 0.0, b1 = 0.0;
      if (bsub) ld2(bsub + op + a, b0, b1);
      st2(y + op + a, bsub ? b0 - ap[0][q] : ap[0][q], bsub ? b1 - ap[1][q] : ap[1][q]);
    } else {  // node a + 1 = N has no row
#pragma unroll
      for (int c = 0; c < d; ++c) {
        const long r = ou + d * a + c;
        y[r] = bsub ? bsub[r] - au[0][q][c] : au[0][q][c];
      }
      y[op + a] = bsub ? bsub[op + a] - ap[0][q] : ap[0][q];
    }
  }
}

// which: 1/2 -> y_u = K_up^i x_p ; 3/4 -> y_p = K_pu^i x_u
template <int D>
__global__ void k_spmv_block(GridDev g, const double *__restrict__ kv, int which,
                             const double *__restrict__ x, double *__restrict__ y) {
  constexpr int d = dim_of(D);
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int i, j, k;
  node_ijk(g, a, i, j, k);
  const int q = (which - 1) & 1;
  const bool up = which <= 2;
  const size_t vs = (size_t)NS * g.ld;
  double acc[d], accp = 0.0;
  for (int c = 0; c < d; ++c) acc[c] = 0.0;
  for (int t = 0; t < NS; ++t) {
    const int *o = TAB<D>.so[t];
    if (!inside(g, i + o[0], j + o[1], k + o[2])) continue;
    const long b = a + lin(g, o[0], o[1], o[2]);
    const double *base = kv + (size_t)t * g.ld + a;
    for (int c = 0; c < d; ++c) {
      if (up)
        acc[c] += base[kv_up(d, q, c) * vs] * x[b];
      else
        accp += base[kv_pu(d, q, c) * vs] * x[d * b + c];
    }
  }
  if (up)
    for (int c = 0; c < d; ++c) y[d * a + c] = acc[c];
  else
    y[a] = accp;
}

template <int D>
__global__ void k_dinv(GridDev g, const double *__restrict__ kv, double *__restrict__ dinv) {
  constexpr int d = dim_of(D);
  constexpr int NS = Tabs<D>::NS;
  const long N = g.N;
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= N) return;
  const size_t vs = (size_t)NS * g.ld;
  const int t0 = TAB<D>.s0;
  for (int q = 0; q < 2; ++q) dinv[q * N + a] = 1.0 / kv[kv_uu(d, q) * vs + (size_t)t0 * g.ld + a];
}

// Half storage of K (layout KH<D>: the symmetric kinds on the zero offset and
// the positive half of St) from the full node-pair storage.  One thread per
// (stream, node).
template <int D>
__global__ void k_pack_kh(GridDev g, const double *__restrict__ kv, double *__restrict__ kh) {
  constexpr int d = dim_of(D);
  using L = KH<D>;
  const long N = g.N;
  const size_t ld = g.ld, vs = (size_t)L::NS * ld;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)L::streams * N) return;
  const int st = (int)(idx / N);
  const long a = idx - (long)st * N;
  const int k = st / L::NH, h = st % L::NH;
  const int kind = k == L::UU0 ? kv_uu(d, 0) : k == L::UU1 ? kv_uu(d, 1) : k == L::PP0 ? kv_pp(d, 0)
                 : k == L::PP1 ? kv_pp(d, 1) : kv_12(d);
  kh[L::at(L::sym(k, h), a, ld)] = kv[kind * vs + (size_t)(h + L::S0) * ld + a];
}

// K_up class table (UPT<D>) read from the assembled values of one node of
// each class (first network; both networks hold the same values).  Classes with
// no node (an axis with a single cell has no interior node) are zero.  Must
// run before the velocity faces mask K.
template <int D>
__global__ void k_up_table(GridDev g, const double *__restrict__ kv, double *__restrict__ upt) {
  constexpr int d = dim_of(D);
  using U = UPT<D>;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= U::size) return;
  const int c = idx % d, t = (idx / d) % U::NS, cls = idx / (d * U::NS);
  int ijk[3] = {0, 0, 0}, cc = cls;
  bool exists = true;
  for (int ax = 0; ax < d; ++ax) {
    const int k = cc % 3;
    cc /= 3;
    ijk[ax] = k == 0 ? 0 : (k == 2 ? g.n[ax] : 1);
    if (k == 1 && g.n[ax] < 2) exists = false;
  }
  const long a = ijk[0] + (long)g.m[0] * (ijk[1] + (long)g.m[1] * ijk[2]);
  const size_t vs = (size_t)U::NS * g.ld;
  upt[idx] = exists ? kv[kv_up(d, 0, c) * vs + (size_t)t * g.ld + a] : 0.0;
}

// selfp Schur block (eqs. S4_sp1, S4_sp2):
//   S_i(b, b+t) = K_pp^i(b, b+t) - sum_{a, c} K_pu^i(b, (a,c)) dinv_i(a) K_up^i((a,c), b+t)
// with a = b + s (s in St) and b + t - a in St.  One thread per (t, b, i).
template <int D>
__global__ __launch_bounds__(256) void k_selfp(GridDev g, const double *__restrict__ kv,
                                               const double *__restrict__ dinv,
                                               double *__restrict__ S) {
  constexpr int d = dim_of(D);
  constexpr int NS = Tabs<D>::NS;
  constexpr int NT = Tabs<D>::NT;
  const long N = g.N;
  const int q = blockIdx.y;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * NT) return;
  const int t = (int)(idx / N);
  const long b = idx - (long)t * N;
  int ib[3];
  node_ijk(g, b, ib[0], ib[1], ib[2]);
  const int *to = TAB<D>.to[t];
  double acc = 0.0;
  if (inside(g, ib[0] + to[0], ib[1] + to[1], ib[2] + to[2])) {
    const size_t vs = (size_t)NS * g.ld;
    const bool small = to[0] >= -1 && to[0] <= 1 && to[1] >= -1 && to[1] <= 1 && to[2] >= -1 &&
                       to[2] <= 1;
    const int st = small ? TAB<D>.sidx[(to[0] + 1) + 3 * (to[1] + 1) + 9 * (to[2] + 1)] : -1;
    if (st >= 0) acc = kv[kv_pp(d, q) * vs + (size_t)st * g.ld + b];
    for (int s = 0; s < NS; ++s) {
      const int *so = TAB<D>.so[s];
      if (!inside(g, ib[0] + so[0], ib[1] + so[1], ib[2] + so[2])) continue;
      const int rx = to[0] - so[0], ry = to[1] - so[1], rz = to[2] - so[2];
      if (rx < -1 || rx > 1 || ry < -1 || ry > 1 || rz < -1 || rz > 1) continue;
      const int r = TAB<D>.sidx[(rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)];
      if (r < 0) continue;
      const long a = b + lin(g, so[0], so[1], so[2]);
      double sum = 0.0;
      for (int c = 0; c < d; ++c)
        sum += kv[kv_pu(d, q, c) * vs + (size_t)s * g.ld + b] *
               kv[kv_up(d, q, c) * vs + (size_t)r * g.ld + a];
      acc -= sum * dinv[q * N + a];
    }
  }
  S[((size_t)q * NT + t) * g.ld + b] = acc;
}

// rhat = r_p - K_pu D^-1 r_u; with ldinv non-null also the multigrid's first
// Chebyshev step on rhat (pointwise): xa = d = c2 ldinv rhat.
template <int D, typename TV, typename TX, bool BC>
__global__ __launch_bounds__(256) void k_schur_rhs(GridDev g, const TV *__restrict__ upt,
                                                   const double *__restrict__ dinv,
                                                   const double *__restrict__ r,
                                                   TX *__restrict__ rhat,
                                                   const TX *__restrict__ ldinv,
                                                   TX *__restrict__ xa, TX *__restrict__ dd,
                                                   Sc2 c2) {
  constexpr int d = dim_of(D);
  __shared__ TV sut[UPT<D>::size];
  stage_upt<D>(sut, upt);
  const int q = blockIdx.y;
  const long b = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (b >= g.N) return;
  const size_t ib = (size_t)q * g.N + b;
  const TX v = (TX)schur_rhs_node<D, TV, BC>(g, sut, dinv, r, q, b);
  rhat[ib] = v;
  if (ldinv) {
    const double x0 = c2.v[q] * (double)ldinv[ib] * (double)v;
    xa[ib] = (TX)x0;
    dd[ib] = (TX)x0;
  }
}

// BC: prescribed velocity components (velocity faces) keep z_u = r_u, the
// identity rows of the masked velocity block.
template <int D, typename TV, typename TX, bool BC>
__global__ __launch_bounds__(256) void k_schur_vel(GridDev g, const TV *__restrict__ upt,
                                                   const double *__restrict__ dinv,
                                                   const double *__restrict__ r,
                                                   const TX *__restrict__ zp,
                                                   double *__restrict__ z) {
  constexpr int d = dim_of(D);
  __shared__ TV sut[UPT<D>::size];
  stage_upt<D>(sut, upt);
  const long N = g.N;
  const int q = blockIdx.y;
  const long a = 2 * ((long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
  if (a >= N) return;
  const long ou = off_u(d, N, q);
  if (a + 1 < N) {
    double out[2 * d];
    schur_vel_node2<D, TV, TX>(g, sut, dinv, r, zp, q, a, out);
    if constexpr (BC) {
      int ia[3], ib[3];
      node_ijk(g, a, ia[0], ia[1], ia[2]);
      node_ijk(g, a + 1, ib[0], ib[1], ib[2]);
#pragma unroll
      for (int c = 0; c < d; ++c) {
        if (u_fixed(g, q, c, ia)) out[c] = r[ou + d * a + c];
        if (u_fixed(g, q, c, ib)) out[d + c] = r[ou + d * (a + 1) + c];
      }
    }
#pragma unroll
    for (int k = 0; k < d; ++k) st2(z + ou + d * a + 2 * k, out[2 * k], out[2 * k + 1]);
    TX p0, p1;
    ld2(zp + q * N + a, p0, p1);
    st2(z + off_p(d, N, q) + a, (double)p0, (double)p1);
  } else {
    double out[d];
    schur_vel_node<D, TV, TX>(g, sut, dinv, r, zp, q, a, out);
    if constexpr (BC) {
      int ia[3];
      node_ijk(g, a, ia[0], ia[1], ia[2]);
#pragma unroll
      for (int c = 0; c < d; ++c)
        if (u_fixed(g, q, c, ia)) out[c] = r[ou + d * a + c];
    }
#pragma unroll
    for (int c = 0; c < d; ++c) z[ou + d * a + c] = out[c];
    z[off_p(d, N, q) + a] = (double)zp[q * N + a];
  }
}

__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) y[i] = (float)x[i];
}

}  // namespace

// Algorithmic bytes of y = K x (or r = b - K x): the five symmetric kinds of
// the half storage (zero offset and positive half) once, the K_up class
// table once, and the vectors.
double upt_bytes(const Grid &g, bool fp32) {
  int n = 0;
  DPP_TAG_SWITCH(g, (n = UPT<D_>::size));
  return n * (fp32 ? 4.0 : 8.0);
}
double kbytes(const Grid &g, bool fp32, bool resid) {
  double pairs = 0.0;
  DPP_TAG_SWITCH(g, (pairs = valid_pairs<D_, false>(g)));
  const double half = 0.5 * (pairs + g.N);
  const double nd = (2.0 * g.dim + 2.0) * g.N;
  return half * 5.0 * (fp32 ? 4.0 : 8.0) + upt_bytes(g, fp32) + nd * 8.0 * (resid ? 3.0 : 2.0);
}

// y = K x, or y = bsub - K x when bsub is non-null
static void launch_K(dpp_problem P, const double *x, const double *bsub, double *y, hipStream_t s,
                     bool fp32) {
  const Grid &g = P->g;
  const int nb = blocks_for(g.N, k_block_nodes(g));
  const int *ord = P->korder.as<int>();
  const bool bc = (g.fix[0] | g.fix[1]) != 0;
  if (fp32)
    DPP_TAG_SWITCH(g, ((bc ? k_spmv_K1<D_, float> : k_spmv_K<D_, float>)<<<nb, KBS, 0, s>>>(
                          dev(g), P->kh32.as<float>(), P->upt32.as<float>(), x, bsub, y, ord)));
  else
    DPP_TAG_SWITCH(g, ((bc ? k_spmv_K1<D_, double> : k_spmv_K<D_, double>)<<<nb, KBS, 0, s>>>(
                          dev(g), P->kh.as<double>(), P->upt.as<double>(), x, bsub, y, ord)));
}

void spmv_K(dpp_problem P, const double *x, double *y, hipStream_t s, bool fp32) {
  if (P->dg) {
    DPP_CHECK(!fp32, DPP_ERR_UNSUPPORTED, "DG-VMS problems are solved in FP64");
    dg_spmv(P, x, nullptr, y, s);
    return;
  }
  ProfScope ps(PF_SPMV_K, kbytes(P->g, fp32, false), s);
  launch_K(P, x, nullptr, y, s, fp32);
  check_launch("spmv_K");
}

void residual_K(dpp_problem P, const double *b, const double *x, double *r, hipStream_t s,
                bool fp32) {
  if (P->dg) {
    DPP_CHECK(!fp32, DPP_ERR_UNSUPPORTED, "DG-VMS problems are solved in FP64");
    dg_spmv(P, x, b, r, s);
    return;
  }
  ProfScope ps(PF_SPMV_K, kbytes(P->g, fp32, true), s);
  launch_K(P, x, b, r, s, fp32);
  check_launch("residual_K");
}

void spmv_block(dpp_problem P, int which, const double *x, double *y, hipStream_t s) {
  const Grid &g = P->g;
  DPP_TAG_SWITCH(g, (k_spmv_block<D_><<<blocks_for(g.N, 256), 256, 0, s>>>(dev(g), P->kvals.as<double>(),
                                                                        which, x, y)));
  check_launch("spmv_block");
}

void make_dinv(dpp_problem P, hipStream_t s) {
  const Grid &g = P->g;
  DPP_TAG_SWITCH(g, (k_dinv<D_><<<blocks_for(g.N, 256), 256, 0, s>>>(dev(g), P->kvals.as<double>(),
                                                                  P->dinv.as<double>())));
  check_launch("dinv");
}

void make_selfp(dpp_problem P, double *S, hipStream_t s) {
  const Grid &g = P->g;
  DPP_TAG_SWITCH(g, (k_selfp<D_><<<dim3(blocks_for(g.N * Tabs<D_>::NT, 256), 2), 256, 0, s>>>(
                        dev(g), P->kvals.as<double>(), P->dinv.as<double>(), S)));
  check_launch("selfp");
}

void make_up_table(dpp_problem P, hipStream_t s) {
  const Grid &g = P->g;
  int n = 0;
  DPP_TAG_SWITCH(g, (n = UPT<D_>::size));
  P->upt.alloc(sizeof(double) * n);
  DPP_TAG_SWITCH(g, (k_up_table<D_><<<blocks_for(n, 256), 256, 0, s>>>(dev(g), P->kvals.as<double>(),
                                                                    P->upt.as<double>())));
  check_launch("K_up class table");
}

void make_kh(dpp_problem P, hipStream_t s) {
  const Grid &g = P->g;
  int streams = 0;
  size_t size = 0;
  DPP_TAG_SWITCH(g, (streams = KH<D_>::streams, size = KH<D_>::size(g.N)));
  P->kh.alloc(sizeof(double) * size);
  // the stream padding is read (never used) by the pair loads of the last node
  DPP_HIP(hipMemsetAsync(P->kh.ptr, 0, sizeof(double) * size, s));
  const long work = (long)streams * g.N;
  DPP_TAG_SWITCH(g, (k_pack_kh<D_><<<blocks_for(work, 256), 256, 0, s>>>(dev(g), P->kvals.as<double>(),
                                                                      P->kh.as<double>())));
  check_launch("pack K half storage");
  // K product workgroups in band order (block_column_order)
  const long plane = g.dim == 3 ? (long)g.m[0] * g.m[1] : g.N;
  const std::vector<int> order = block_column_order(g.N, k_block_nodes(g), plane);
  const long nb = (long)order.size();
  P->korder.alloc(sizeof(int) * nb);
  DPP_HIP(hipMemcpyAsync(P->korder.ptr, order.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
  DPP_HIP(hipStreamSynchronize(s));
}

void make_k32(dpp_problem P, hipStream_t s) {
  if (P->kh32.ptr) return;
  size_t n = P->kh.bytes / sizeof(double);
  P->kh32.alloc(n * sizeof(float));
  k_to_f32<<<2048, 256, 0, s>>>(P->kh.as<double>(), P->kh32.as<float>(), n);
  n = P->upt.bytes / sizeof(double);
  P->upt32.alloc(n * sizeof(float));
  k_to_f32<<<blocks_for((long)n, 256), 256, 0, s>>>(P->upt.as<double>(), P->upt32.as<float>(), n);
  check_launch("k32");
}

void schur_rhs(dpp_problem P, const double *r, void *rhat, bool fp32, hipStream_t s,
               const void *ldinv, void *xa, void *dd, const double *c2) {
  const Grid &g = P->g;
  const double tx = fp32 ? 4.0 : 8.0;
  ProfScope ps(PF_SCHUR_RHS,
               2.0 * (upt_bytes(g, fp32) + g.N * (g.dim + 2.0) * 8.0 + g.N * tx +
                      (ldinv ? 3.0 * g.N * tx : 0.0)), s);
  dim3 grid(blocks_for(g.N, 256), 2);
  const double *di = P->dinv.as<double>();
  const Sc2 c{{c2 ? c2[0] : 0.0, c2 ? c2[1] : 0.0}};
  const bool bc = (g.fix[0] | g.fix[1]) != 0;
  const float *u32 = P->upt32.as<float>();
  const double *u64 = P->upt.as<double>();
  if (fp32)
    DPP_TAG_SWITCH(g, ((bc ? k_schur_rhs<D_, float, float, true> : k_schur_rhs<D_, float, float, false>)
                          <<<grid, 256, 0, s>>>(dev(g), u32, di, r, (float *)rhat, (const float *)ldinv,
                                                (float *)xa, (float *)dd, c)));
  else
    DPP_TAG_SWITCH(g, ((bc ? k_schur_rhs<D_, double, double, true> : k_schur_rhs<D_, double, double, false>)
                          <<<grid, 256, 0, s>>>(dev(g), u64, di, r, (double *)rhat, (const double *)ldinv,
                                                (double *)xa, (double *)dd, c)));
  check_launch("schur_rhs");
}

void schur_velocity(dpp_problem P, const double *r, const void *zp, bool fp32, double *z,
                    hipStream_t s) {
  const Grid &g = P->g;
  ProfScope ps(PF_SCHUR_VEL,
               2.0 * (upt_bytes(g, fp32) + g.N * (2.0 * g.dim + 2.0) * 8.0 +
                      g.N * (fp32 ? 4.0 : 8.0)), s);
  dim3 grid(blocks_for((g.N + 1) / 2, 256), 2);
  const double *di = P->dinv.as<double>();
  const bool bc = (g.fix[0] | g.fix[1]) != 0;
  if (fp32)
    DPP_TAG_SWITCH(g, ((bc ? k_schur_vel<D_, float, float, true> : k_schur_vel<D_, float, float, false>)
                          <<<grid, 256, 0, s>>>(dev(g), P->upt32.as<float>(), di, r, (const float *)zp, z)));
  else
    DPP_TAG_SWITCH(g, ((bc ? k_schur_vel<D_, double, double, true> : k_schur_vel<D_, double, double, false>)
                          <<<grid, 256, 0, s>>>(dev(g), P->upt.as<double>(), di, r, (const double *)zp, z)));
  check_launch("schur_velocity");
}

}  // namespace dpp
