// Batched solve of many independent DPP instances (uneven boxes): one launch
// per phase covers every instance.
//
// Each launch walks a table of per-instance descriptors; a workgroup finds
// its instance by binary search on the descriptors' first-block indices.
// The V-cycle is level-synchronous: going down, level l of every instance
// deeper than l+1 is smoothed in one launch; the coarsest levels (which sit at
// different depths) are solved in one launch; going up mirrors the descent.
// The Krylov method is the same flexible GMRES(m) with CGS2 as the single
// solve, run in lockstep with per-instance Hessenberg systems; an instance
// that has converged is masked out of every later launch.  One Arnoldi step
// can be captured in a hipGraph per step index and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>

#include "objects.h"
#include "profile.h"
#include "stencil.h"
#include "batch.h"
#include "mvec.h"

namespace dpp {

template <typename Desc>
__device__ inline int find_desc(const Desc *__restrict__ d, int nd, int bid, int Desc::*first) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].*first <= bid)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline double bwave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

namespace {

// ---------------------------------------------------------------- K level --
// The instance's K_up class table (UPT<D>) copied into LDS.
template <int D, typename TV>
__device__ inline void stage_upt_b(TV *sut, const double *__restrict__ upt) {
  for (int i = threadIdx.x; i < UPT<D>::size; i += blockDim.x) sut[i] = (TV)upt[i];
  __syncthreads();
}

// BC: some instance has velocity faces (masked velocity gathers, identity rows
// on the prescribed components; the face bits of each instance are in k.g).
template <int D, typename TV, bool BC>
__global__ __launch_bounds__(256) void kb_spmv_K(const KDesc *__restrict__ kd, int nd,
                                                 const int *__restrict__ active,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ bsub,
                                                 double *__restrict__ y) {
  const int di = find_desc(kd, nd, (int)blockIdx.x, &KDesc::blk0);
  const KDesc &k = kd[di];
  if (!active[k.inst]) return;  // uniform over the workgroup
  __shared__ TV sut[UPT<D>::size];
  stage_upt_b<D>(sut, k.upt);
  const long a = (long)(blockIdx.x - k.blk0) * blockDim.x + threadIdx.x;
  const GridDev g = k.g;
  if (a >= g.N) return;
  double au[2][D], ap[2];
  spmv_K_node<D, TV, BC>(g, (const TV *)k.kv, sut, x + k.off, a, au, ap);
  const long N = g.N;
  int ia[3] = {0, 0, 0};
  if constexpr (BC) node_ijk(g, a, ia[0], ia[1], ia[2]);
  for (int q = 0; q < 2; ++q) {
    const long ou = k.off + off_u(D, N, q), op = k.off + off_p(D, N, q);
    for (int c = 0; c < D; ++c) {
      const long r = ou + D * a + c;
      double v = au[q][c];
      if constexpr (BC)
        if (u_fixed(g, q, c, ia)) v = x[r];
      y[r] = bsub ? bsub[r] - v : v;
    }
    y[op + a] = bsub ? bsub[op + a] - ap[q] : ap[q];
  }
}

template <int D, typename TV, typename TX, bool BC>
__global__ __launch_bounds__(256) void kb_schur_rhs(const KDesc *__restrict__ kd, int nd,
                                                    const int *__restrict__ active,
                                                    const double *__restrict__ r) {
  const int di = find_desc(kd, nd, (int)blockIdx.x, &KDesc::blk0);
  const KDesc &k = kd[di];
  if (!active[k.inst]) return;  // uniform over the workgroup
  __shared__ TV sut[UPT<D>::size];
  stage_upt_b<D>(sut, k.upt);
  const int q = blockIdx.y;
  const long b = (long)(blockIdx.x - k.blk0) * blockDim.x + threadIdx.x;
  if (b >= k.g.N) return;
  ((TX *)k.rhat)[q * k.g.N + b] =
      (TX)schur_rhs_node<D, TV, BC>(k.g, sut, k.dinv, r + k.off, q, b);
}

template <int D, typename TV, typename TX, bool BC>
__global__ __launch_bounds__(256) void kb_schur_vel(const KDesc *__restrict__ kd, int nd,
                                                    const int *__restrict__ active,
                                                    const double *__restrict__ r,
                                                    double *__restrict__ z) {
  const int di = find_desc(kd, nd, (int)blockIdx.x, &KDesc::blk0);
  const KDesc &k = kd[di];
  if (!active[k.inst]) return;  // uniform over the workgroup
  __shared__ TV sut[UPT<D>::size];
  stage_upt_b<D>(sut, k.upt);
  const int q = blockIdx.y;
  const long a = (long)(blockIdx.x - k.blk0) * blockDim.x + threadIdx.x;
  const long N = k.g.N;
  if (a >= N) return;
  double out[D];
  const TX *zp = (const TX *)k.zp;
  schur_vel_node<D, TV, TX>(k.g, sut, k.dinv, r + k.off, zp, q, a, out);
  const long ou = k.off + off_u(D, N, q);
  if constexpr (BC) {
    int ia[3];
    node_ijk(k.g, a, ia[0], ia[1], ia[2]);
    for (int c = 0; c < D; ++c)
      if (u_fixed(k.g, q, c, ia)) out[c] = r[ou + D * a + c];  // identity rows
  }
  for (int c = 0; c < D; ++c) z[ou + D * a + c] = out[c];
  z[k.off + off_p(D, N, q) + a] = (double)zp[q * N + a];
}

// ---------------------------------------------------------- level kernels --
template <typename TX>
__device__ inline TX *lbuf(const LDesc &l, int which) {
  return (TX *)(which == 0 ? l.xa : which == 1 ? l.xb : l.e);
}

template <typename TV, typename TX>
__global__ __launch_bounds__(256) void kb_cheb_first(const LDesc *__restrict__ ld, int nd,
                                                     const int *__restrict__ active, int out_w) {
  const int di = find_desc(ld, nd, (int)blockIdx.x, &LDesc::blk0);
  const LDesc &l = ld[di];
  if (!active[l.inst]) return;
  const int q = blockIdx.y;
  const long a = (long)(blockIdx.x - l.blk0) * blockDim.x + threadIdx.x;
  if (a >= l.g.N) return;
  const size_t ia = (size_t)q * l.g.N + a;
  const double v = l.c2[0][q] * (double)((const TV *)l.dinv)[ia] * (double)((const TX *)l.b)[ia];
  ((TX *)l.d)[ia] = (TX)v;
  lbuf<TX>(l, out_w)[ia] = (TX)v;
}

// Chebyshev step `step` (>= 0, nonzero guess): in -> out, d updated.  With
// resid_only, writes r = b - A in instead.
template <int D, typename TV, typename TX, int LPR>
__global__ __launch_bounds__(256, 4) void kb_cheb(const LDesc *__restrict__ ld, int nd,
                                                  const int *__restrict__ active, int step,
                                                  int in_w, int out_w, int resid_only) {
  const int di = find_desc(ld, nd, (int)blockIdx.x, &LDesc::blk0);
  const LDesc &l = ld[di];
  if (!active[l.inst]) return;
  const int q = blockIdx.y;
  const long gid = (long)(blockIdx.x - l.blk0) * blockDim.x + threadIdx.x;
  const long a = gid / LPR;
  const int sub = (int)(gid % LPR);
  const GridDev g = l.g;
  if (a >= g.N) return;
  constexpr int NA = stored_offsets<D, true>();
  const TX *xin = lbuf<TX>(l, in_w);
  const double ax = row_product<D, TV, TX, LPR, true>(g, (const TV *)l.A + (size_t)q * NA * g.ld,
                                                      xin + (size_t)q * g.N, a, 0, 0, 0, sub);
  if (sub != 0) return;
  const size_t ia = (size_t)q * g.N + a;
  const double bb = (double)((const TX *)l.b)[ia];
  if (resid_only) {
    ((TX *)l.r)[ia] = (TX)(bb - ax);
    return;
  }
  const double r = (double)((const TV *)l.dinv)[ia] * (bb - ax);
  const double c1 = l.c1[step][q], c2 = l.c2[step][q];
  const double dn = (c1 != 0.0 ? c1 * (double)((TX *)l.d)[ia] : 0.0) + c2 * r;
  ((TX *)l.d)[ia] = (TX)dn;
  lbuf<TX>(l, out_w)[ia] = (TX)((double)xin[ia] + dn);
}

// bc = R r (or R b when the level does not pre-smooth)
template <int D, typename TX>
__global__ __launch_bounds__(256) void kb_restrict(const LDesc *__restrict__ ld, int nd,
                                                   const int *__restrict__ active, int from_b) {
  const int di = find_desc(ld, nd, (int)blockIdx.x, &LDesc::cblk0);
  const LDesc &l = ld[di];
  if (!active[l.inst]) return;
  const int q = blockIdx.y;
  const long C = (long)(blockIdx.x - l.cblk0) * blockDim.x + threadIdx.x;
  if (C >= l.gc.N) return;
  const TX *src = (const TX *)(from_b ? l.b : l.r);
  ((TX *)l.bc)[(size_t)q * l.gc.N + C] = (TX)restrict_node<D, TX>(l.g, l.gc, src + (size_t)q * l.g.N, C);
}

// x += P ec (x = P ec when assign: the level did not pre-smooth)
template <int D, typename TX>
__global__ __launch_bounds__(256) void kb_prolong(const LDesc *__restrict__ ld, int nd,
                                                  const int *__restrict__ active, int x_w, int assign) {
  const int di = find_desc(ld, nd, (int)blockIdx.x, &LDesc::blk0);
  const LDesc &l = ld[di];
  if (!active[l.inst]) return;
  const int q = blockIdx.y;
  // node blocks were sized for LPR lanes; one thread per node here
  const long f = (long)(blockIdx.x - l.blk0) * blockDim.x + threadIdx.x;
  if (f >= l.g.N) return;
  const double v = prolong_node<D, TX>(l.g, l.gc, (const TX *)l.ec + (size_t)q * l.gc.N, f);
  TX *x = lbuf<TX>(l, x_w);
  x[(size_t)q * l.g.N + f] = (TX)(assign ? v : (double)x[(size_t)q * l.g.N + f] + v);
}

template <typename TX>
__global__ __launch_bounds__(256) void kb_coarse(const CDesc *__restrict__ cd, int nd,
                                                 const int *__restrict__ active) {
  const int di = find_desc(cd, nd, (int)blockIdx.x, &CDesc::blk0);
  const CDesc &c = cd[di];
  if (!active[c.inst]) return;
  const int q = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int row = (blockIdx.x - c.blk0) * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= c.n) return;
  const double *Mr = c.Cinv + (size_t)q * c.n * c.n + (size_t)row * c.n;
  const TX *bq = (const TX *)c.b + (size_t)q * c.n;
  // four independent partial sums, so four loads per lane are in flight
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = lane;
  for (; k + 192 < c.n; k += 256) {
    s0 += Mr[k] * (double)bq[k];
    s1 += Mr[k + 64] * (double)bq[k + 64];
    s2 += Mr[k + 128] * (double)bq[k + 128];
    s3 += Mr[k + 192] * (double)bq[k + 192];
  }
  for (; k < c.n; k += 64) s0 += Mr[k] * (double)bq[k];
  double s = (s0 + s1) + (s2 + s3);
  s = bwave_sum(s);
  if (lane == 0) ((TX *)c.x)[(size_t)q * c.n + row] = (TX)s;
}

// ---------------------------------------------------------------- Krylov --
// Every block works on its instance's slice [off, off + n) with the
// instance's own grid stride; partials are indexed by the global block.
template <int NKP>
__global__ __launch_bounds__(BBS) void kb_mdot(const VDesc *__restrict__ vd, int nd,
                                               const int *__restrict__ active,
                                               const double *__restrict__ V, long ldv, int nk,
                                               const double *__restrict__ w, double *__restrict__ part) {
  const int di = find_desc(vd, nd, (int)blockIdx.x, &VDesc::blk0);
  const VDesc &v = vd[di];
  if (!active[v.inst]) return;
  double acc[NKP];
#pragma unroll
  for (int k = 0; k < NKP; ++k) acc[k] = 0.0;
  mv_dot<NKP>(V + v.off, ldv, nk, w + v.off, (long)(blockIdx.x - v.blk0) * BBS + threadIdx.x, v.n,
              (long)v.nblk * BBS, acc);
  mv_block_store<NKP>(acc, nk, 0.0, false, part, gridDim.x, blockIdx.x);
}

// DCGS2 pass A per instance (t = V_nj of the instance): partial rows
// [0, nj) = V_k . t, [nj, 2nj) = V_k . w, 2nj = t . w.
template <int NKP>
__global__ __launch_bounds__(BBS) void kb_dcgs_a(const VDesc *__restrict__ vd, int nd,
                                                 const int *__restrict__ active,
                                                 const double *__restrict__ V, long ldv, int nj,
                                                 const double *__restrict__ w, double *__restrict__ part) {
  const int di = find_desc(vd, nd, (int)blockIdx.x, &VDesc::blk0);
  const VDesc &v = vd[di];
  if (!active[v.inst]) return;
  mv_dcgs_a_waves<NKP>(V + v.off, ldv, nj, V + (size_t)nj * ldv + v.off, w + v.off,
                       (long)(blockIdx.x - v.blk0) * 64, v.n, (long)v.nblk * 64, part, gridDim.x,
                       blockIdx.x);
}

// DCGS2 pass B per instance, coefficients from the instance's reduced sums in
// hb; the instance's first block publishes rho and hjj.
template <int NKP>
__global__ __launch_bounds__(BBS) void kb_dcgs_b(const VDesc *__restrict__ vd, int nd,
                                                 const int *__restrict__ active,
                                                 double *__restrict__ V, long ldv, int nj,
                                                 const double *__restrict__ w,
                                                 double *__restrict__ hb, double *__restrict__ part) {
  const int di = find_desc(vd, nd, (int)blockIdx.x, &VDesc::blk0);
  const VDesc &v = vd[di];
  if (!active[v.inst]) return;
  double *h = hb + (size_t)v.inst * HS;
  double a[NKP], b[NKP], rho, inv, hjj;
  mv_dcgs_coefs<NKP>(h, h[HB_ALPHA + (nj & 1)], nj, a, b, rho, inv, hjj);
  if ((int)blockIdx.x == v.blk0 && threadIdx.x == 0) {
    h[HB_RHO] = rho;
    h[HB_HJJ] = hjj;
  }
  double nrm = 0.0;
  mv_dcgs_update<NKP>(V + v.off, ldv, nj, a, b, inv, hjj, V + (size_t)nj * ldv + v.off, w + v.off,
                      V + (size_t)(nj + 1) * ldv + v.off, (long)(blockIdx.x - v.blk0) * BBS + threadIdx.x,
                      v.n, (long)v.nblk * BBS, nrm);
  mv_block_store<NKP>(a, 0, nrm, true, part, gridDim.x, blockIdx.x);
}

// hb[inst*HS + hslot + k] = sum of instance inst's partials of slot k
__global__ __launch_bounds__(BBS) void kb_finish(const VDesc *__restrict__ vd,
                                                 const int *__restrict__ active,
                                                 const double *__restrict__ part, int tb,
                                                 double *__restrict__ hb, int hslot) {
  const int k = blockIdx.x, di = blockIdx.y;
  const VDesc &v = vd[di];
  if (!active[v.inst]) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < v.nblk; b += BBS) s += part[(size_t)k * tb + v.blk0 + b];
  s = bwave_sum(s);
  __shared__ double sh[BBS / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < BBS / 64; ++w) t += sh[w];
    hb[(size_t)v.inst * HS + hslot + k] = t;
  }
}

// v <- v / sqrt(hb[inst*HS + slot]) (or times fac[inst] when fac != null)
__global__ __launch_bounds__(BBS) void kb_scale(const VDesc *__restrict__ vd, int nd,
                                                const int *__restrict__ active, double *__restrict__ v,
                                                const double *__restrict__ hb, int slot,
                                                const double *__restrict__ fac) {
  const int di = find_desc(vd, nd, (int)blockIdx.x, &VDesc::blk0);
  const VDesc &d = vd[di];
  if (!active[d.inst]) return;
  double a;
  if (fac) {
    a = fac[d.inst];
  } else {
    const double s2 = hb[(size_t)d.inst * HS + slot];
    if (!(s2 > 0.0)) return;
    a = 1.0 / sqrt(s2);
  }
  for (long i = (long)(blockIdx.x - d.blk0) * BBS + threadIdx.x; i < d.n; i += (long)d.nblk * BBS)
    v[d.off + i] *= a;
}

// x_i <- x_i + Z_i y_i (y per instance, nk_i <= NKP columns; nk_i = 0 skips)
template <int NKP>
__global__ __launch_bounds__(BBS) void kb_update(const VDesc *__restrict__ vd, int nd,
                                                 const double *__restrict__ Z, long ldz,
                                                 const double *__restrict__ y,
                                                 const int *__restrict__ nks, double *__restrict__ x) {
  const int di = find_desc(vd, nd, (int)blockIdx.x, &VDesc::blk0);
  const VDesc &d = vd[di];
  const int nk = nks[d.inst];
  if (nk == 0) return;
  double yk[NKP];
  mv_coefs<NKP>(y + (size_t)d.inst * BMAXK, nk, yk);
  mv_update<NKP>(Z + d.off, ldz, nk, yk, x + d.off, (long)(blockIdx.x - d.blk0) * BBS + threadIdx.x,
                 d.n, (long)d.nblk * BBS);
}

}  // namespace

}  // namespace dpp

namespace dpp {

namespace {

void cheb_coefs_l(const Level &L, int deg, LDesc &d) {
  for (int q = 0; q < 2; ++q) {
    const double theta = 0.5 * (L.hi[q] + L.lo[q]), delta = 0.5 * (L.hi[q] - L.lo[q]);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    d.c1[0][q] = 0.0;
    d.c2[0][q] = 1.0 / theta;
    for (int k = 1; k < deg; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      d.c1[k][q] = rn * rho;
      d.c2[k][q] = 2.0 * rn / delta;
      rho = rn;
    }
  }
}

void build_level_tables(dpp_batch B, int l, int lanes, bool fp32, DTable<LDesc> &out) {
  std::vector<LDesc> v;
  int blk = 0, cblk = 0;
  std::vector<LDesc> tmp;
  for (int i = 0; i < B->nb; ++i) {
    dpp_precond pc = B->pc[i];
    if ((int)pc->lv.size() - 1 <= l) continue;  // level l is this instance's coarsest (or absent)
    Level &L = *pc->lv[l];
    Level &C = *pc->lv[l + 1];
    LDesc d{};
    d.g = dev(L.g);
    d.gc = dev(C.g);
    d.inst = i;
    d.blk0 = blk;
    d.nblk = blocks_for(L.g.N * lanes, 256);
    blk += d.nblk;
    d.cblk0 = cblk;
    d.cnblk = blocks_for(C.g.N, 256);
    cblk += d.cnblk;
    if (fp32) {
      d.A = L.Ah32.ptr;
      d.dinv = L.dinv32.ptr;
      d.b = L.b32.ptr; d.xa = L.xa32.ptr; d.xb = L.xb32.ptr; d.d = L.d32.ptr; d.r = L.r32.ptr; d.e = L.e32.ptr;
      d.bc = C.b32.ptr; d.ec = C.e32.ptr;
    } else {
      d.A = L.Ah.ptr;
      d.dinv = L.dinv.ptr;
      d.b = L.b.ptr; d.xa = L.xa.ptr; d.xb = L.xb.ptr; d.d = L.d.ptr; d.r = L.r.ptr; d.e = L.e.ptr;
      d.bc = C.b.ptr; d.ec = C.e.ptr;
    }
    cheb_coefs_l(L, 8, d);  // step k's coefficients do not depend on the degree
    v.push_back(d);
  }
  // restriction blocks are looked up through cblk0: keep both orders valid
  out.upload(v, blk);
  (void)cblk;
}

int level_cblocks(dpp_batch B, int l) {
  int c = 0;
  for (int i = 0; i < B->nb; ++i) {
    dpp_precond pc = B->pc[i];
    if ((int)pc->lv.size() - 1 <= l) continue;
    c += blocks_for(pc->lv[l + 1]->g.N, 256);
  }
  return c;
}

// Algorithmic bytes of the batched launches, summed over the running
// instances (instrumentation only): stored matrix entries inside each box
// once, each vector read or written once, as for the single-instance kernels.
bool running(dpp_batch B, int i) { return i < (int)B->hact.size() && B->hact[i]; }

double bytes_spmv(dpp_batch B, bool resid, bool fp32) {
  double t = 0.0;
  for (int i = 0; i < B->nb; ++i)
    if (running(B, i)) t += kbytes(B->P[i]->g, fp32, resid);
  return t;
}

template <int D>
double bytes_cheb(dpp_batch B, int l, double tx, int step, bool resid_only) {
  double t = 0.0;
  for (int i = 0; i < B->nb; ++i) {
    dpp_precond pc = B->pc[i];
    if (!running(B, i) || (int)pc->lv.size() - 1 <= l) continue;
    const Grid &g = pc->lv[l]->g;
    const double N = (double)g.N, pairs = 0.5 * (valid_pairs<D, true>(g) + N);
    t += resid_only ? 2.0 * (pairs * tx + 3.0 * N * tx)
                    : 2.0 * (pairs * tx + N * (5.0 * tx + (step > 0 ? tx : 0.0)));
  }
  return t;
}

// restriction (w = 0), prolongation (w = 1) or the coarse solves (w = 2)
double bytes_transfer(dpp_batch B, int l, double tx, int w, bool assign) {
  double t = 0.0;
  for (int i = 0; i < B->nb; ++i) {
    dpp_precond pc = B->pc[i];
    if (!running(B, i)) continue;
    if (w == 2) {
      const double n = pc->ncoarse;
      t += 2.0 * n * (n * 8.0 + 2.0 * tx);
      continue;
    }
    if ((int)pc->lv.size() - 1 <= l) continue;
    const double N = (double)pc->lv[l]->g.N, Nc = (double)pc->lv[l + 1]->g.N;
    t += w == 0 ? 2.0 * tx * (N + Nc) : 2.0 * tx * ((assign ? 1.0 : 2.0) * N + Nc);
  }
  return t;
}

double bytes_schur(dpp_batch B, double tx, bool vel) {
  double t = 0.0;
  for (int i = 0; i < B->nb; ++i) {
    if (!running(B, i)) continue;
    const Grid &g = B->P[i]->g;
    t += 2.0 * (upt_bytes(g, tx == 4.0) + g.N * (vel ? 2.0 * g.dim + 2.0 : g.dim + 2.0) * 8.0 + g.N * tx);
  }
  return t;
}

double running_dof(dpp_batch B) {
  double t = 0.0;
  for (int i = 0; i < B->nb; ++i)
    if (running(B, i)) t += (double)B->P[i]->ndof();
  return t;
}

template <int D, typename TV, typename TX>
void launch_cheb_b(dpp_batch B, int l, const DTable<LDesc> &t, hipStream_t s, int step, int in_w,
                   int out_w, int resid_only) {
  if (!t.count) return;
  ProfScope ps(l == 0 ? PF_B_CHEB_L0 : PF_B_LEVELS,
               prof_on() ? bytes_cheb<D>(B, l, sizeof(TX), step, resid_only != 0) : 0.0, s);
  const dim3 grid(t.blocks, 2);
  const int *act = B->active.as<int>();
  switch (B->lpr[l]) {
    case 1: kb_cheb<D, TV, TX, 1><<<grid, 256, 0, s>>>(t.get(), t.count, act, step, in_w, out_w, resid_only); break;
    case 2: kb_cheb<D, TV, TX, 2><<<grid, 256, 0, s>>>(t.get(), t.count, act, step, in_w, out_w, resid_only); break;
    case 4: kb_cheb<D, TV, TX, 4><<<grid, 256, 0, s>>>(t.get(), t.count, act, step, in_w, out_w, resid_only); break;
    default: kb_cheb<D, TV, TX, 8><<<grid, 256, 0, s>>>(t.get(), t.count, act, step, in_w, out_w, resid_only); break;
  }
}

// Level-synchronous V-cycle over every instance (finest-level input and output
// are each instance's level-0 b and e buffers).
template <int D, typename TV, typename TX>
void vcycle_b(dpp_batch B, bool fp32, hipStream_t s) {
  const int *act = B->active.as<int>();
  auto &tabs = fp32 ? B->ld32 : B->ld;
  std::vector<int> cur_after_pre(B->nlev, 0);
  for (int l = 0; l < B->nlev; ++l) {
    const DTable<LDesc> &t = tabs[l];
    if (!t.count) continue;
    const int pre = cheb_pre(B->opts, l);
    const dim3 g1(t.blocks, 2);
    int cur = 0, oth = 1;
    if (pre > 0) {
      {
        ProfScope ps(PF_B_LEVELS, prof_on() ? bytes_transfer(B, l, sizeof(TX), 1, false) : 0.0, s);
        kb_cheb_first<TV, TX><<<g1, 256, 0, s>>>(t.get(), t.count, act, 0);
      }
      for (int k = 1; k < pre; ++k) {
        launch_cheb_b<D, TV, TX>(B, l, t, s, k, cur, oth, 0);
        std::swap(cur, oth);
      }
      launch_cheb_b<D, TV, TX>(B, l, t, s, 0, cur, 0, 1);  // r = b - A x
    }
    cur_after_pre[l] = cur;
    const int cb = level_cblocks(B, l);
    // restriction of r (or of b without pre-smoothing): grid over coarse-node
    // blocks, descriptors found through cblk0
    ProfScope ps(PF_B_LEVELS, prof_on() ? bytes_transfer(B, l, sizeof(TX), 0, false) : 0.0, s);
    kb_restrict<D, TX><<<dim3(cb, 2), 256, 0, s>>>(t.get(), t.count, act, pre > 0 ? 0 : 1);
  }
  const DTable<CDesc> &c = fp32 ? B->cd32 : B->cd;
  {
    ProfScope ps(PF_B_LEVELS, prof_on() ? bytes_transfer(B, 0, sizeof(TX), 2, false) : 0.0, s);
    kb_coarse<TX><<<dim3(c.blocks, 2), 256, 0, s>>>(c.get(), c.count, act);
  }
  for (int l = B->nlev - 1; l >= 0; --l) {
    const DTable<LDesc> &t = tabs[l];
    if (!t.count) continue;
    const int pre = cheb_pre(B->opts, l), post = cheb_post(B->opts, l);
    const dim3 g1(t.blocks, 2);
    int cur = cur_after_pre[l], oth = 1 - cur;
    {
      ProfScope ps(PF_B_LEVELS, prof_on() ? bytes_transfer(B, l, sizeof(TX), 1, pre == 0) : 0.0, s);
      kb_prolong<D, TX><<<g1, 256, 0, s>>>(t.get(), t.count, act, cur, pre > 0 ? 0 : 1);
    }
    for (int k = 0; k < post; ++k) {
      const int out = (k == post - 1) ? 2 : oth;
      launch_cheb_b<D, TV, TX>(B, l, t, s, k, cur, out, 0);
      oth = cur;
      cur = out;
    }
  }
  check_launch("batched vcycle");
}

template <int D>
void precond_b(dpp_batch B, const double *r, double *z, bool fp32, hipStream_t s) {
  const DTable<KDesc> &k = fp32 ? B->kd32 : B->kd;
  const int *act = B->active.as<int>();
  const dim3 g(k.blocks, 2);
  const double tx = fp32 ? 4.0 : 8.0;
  if (fp32) {
    {
      ProfScope ps(PF_B_SCHUR, prof_on() ? bytes_schur(B, tx, false) : 0.0, s);
      (B->any_bc ? kb_schur_rhs<D, double, float, true> : kb_schur_rhs<D, double, float, false>)
          <<<g, 256, 0, s>>>(k.get(), k.count, act, r);
    }
    vcycle_b<D, float, float>(B, true, s);
    ProfScope ps(PF_B_SCHUR, prof_on() ? bytes_schur(B, tx, true) : 0.0, s);
    (B->any_bc ? kb_schur_vel<D, double, float, true> : kb_schur_vel<D, double, float, false>)
        <<<g, 256, 0, s>>>(k.get(), k.count, act, r, z);
  } else {
    {
      ProfScope ps(PF_B_SCHUR, prof_on() ? bytes_schur(B, tx, false) : 0.0, s);
      (B->any_bc ? kb_schur_rhs<D, double, double, true> : kb_schur_rhs<D, double, double, false>)
          <<<g, 256, 0, s>>>(k.get(), k.count, act, r);
    }
    vcycle_b<D, double, double>(B, false, s);
    ProfScope ps(PF_B_SCHUR, prof_on() ? bytes_schur(B, tx, true) : 0.0, s);
    (B->any_bc ? kb_schur_vel<D, double, double, true> : kb_schur_vel<D, double, double, false>)
        <<<g, 256, 0, s>>>(k.get(), k.count, act, r, z);
  }
  check_launch("batched precond");
}

// y = K x (or bsub - K x) for the active instances; op32 reads the FP32 copy
// of the half storage (the inner solves of iterative refinement)
template <int D>
void spmv_b(dpp_batch B, const double *x, const double *bsub, double *y, hipStream_t s,
            bool op32 = false) {
  ProfScope ps(PF_B_SPMV_K, prof_on() ? bytes_spmv(B, bsub != nullptr, op32) : 0.0, s);
  if (op32)
    (B->any_bc ? kb_spmv_K<D, float, true> : kb_spmv_K<D, float, false>)
        <<<B->kd32.blocks, 256, 0, s>>>(B->kd32.get(), B->kd32.count, B->active.as<int>(), x, bsub, y);
  else
    (B->any_bc ? kb_spmv_K<D, double, true> : kb_spmv_K<D, double, false>)
        <<<B->kd.blocks, 256, 0, s>>>(B->kd.get(), B->kd.count, B->active.as<int>(), x, bsub, y);
  check_launch("batched spmv");
}

// one Arnoldi step j for every active instance: z_j = M^-1 v~_j, w = K z_j and
// the two DCGS2 passes (graph-capturable: launches only)
template <int D>
void arnoldi_step_b(dpp_batch B, int j, bool fp32, bool op32, hipStream_t s) {
  const long n = B->ntot;
  double *V = B->V.as<double>(), *Z = B->Z.as<double>(), *w = B->w.as<double>();
  double *part = B->part.as<double>(), *hb = B->hb.as<double>();
  const int *act = B->active.as<int>();
  const VDesc *vd = B->vd.get();
  const int nvd = B->vd.count, tb = B->vd.blocks;
  precond_b<D>(B, V + (size_t)j * n, Z + (size_t)j * n, fp32, s);
  spmv_b<D>(B, Z + (size_t)j * n, nullptr, w, s, op32);
  // A reads V_0..V_j and w; B reads them again, writes v_j (j > 0) and v~_{j+1}
  ProfScope ps(PF_B_ARNOLDI, prof_on() ? 8.0 * running_dof(B) * (2.0 * j + 4.0 + (j > 0 ? 2.0 : 1.0)) : 0.0,
               s);
  DPP_NK_SWITCH(std::max(j, 1), kb_dcgs_a<NKP><<<tb, BBS, 0, s>>>(vd, nvd, act, V, n, j, w, part));
  kb_finish<<<dim3(2 * j + 1, nvd), BBS, 0, s>>>(vd, act, part, tb, hb, 0);
  DPP_NK_SWITCH(std::max(j, 1), kb_dcgs_b<NKP><<<tb, BBS, 0, s>>>(vd, nvd, act, V, n, j, w, hb, part));
  kb_finish<<<dim3(1, nvd), BBS, 0, s>>>(vd, act, part, tb, hb, HB_ALPHA + ((j + 1) & 1));
  check_launch("batched arnoldi");
}

// per-instance sums of squares of v (into hb slot `slot`), copied to host
void norms_b(dpp_batch B, const double *v, int slot, std::vector<double> &out, hipStream_t s) {
  const int tb = B->vd.blocks;
  kb_mdot<1><<<tb, BBS, 0, s>>>(B->vd.get(), B->vd.count, B->active.as<int>(), v, 0, 1, v, B->part.as<double>());
  kb_finish<<<dim3(1, B->vd.count), BBS, 0, s>>>(B->vd.get(), B->active.as<int>(), B->part.as<double>(), tb,
                                                 B->hb.as<double>(), slot);
  check_launch("batched norms");
  std::vector<double> h((size_t)B->nb * HS);
  DPP_HIP(hipMemcpyAsync(h.data(), B->hb.ptr, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  DPP_HIP(hipStreamSynchronize(s));
  out.resize(B->nb);
  for (int i = 0; i < B->nb; ++i) out[i] = std::sqrt(std::max(0.0, h[(size_t)i * HS + slot]));
}

template <int D>
void tune_batch_lanes(dpp_batch B, hipStream_t s) {
  B->lpr.assign(B->nlev, 1);
  hipEvent_t e0, e1;
  DPP_HIP(hipEventCreate(&e0));
  DPP_HIP(hipEventCreate(&e1));
  std::vector<int> ones(B->nb, 1);
  DPP_HIP(hipMemcpy(B->active.ptr, ones.data(), sizeof(int) * B->nb, hipMemcpyHostToDevice));
  for (int l = 0; l < B->nlev; ++l) {
    float best_ms = 1e30f;
    int best = 1;
    for (int cand : {1, 2, 4, 8}) {
      B->lpr[l] = cand;
      DTable<LDesc> t;
      build_level_tables(B, l, cand, false, t);
      if (!t.count) break;
      launch_cheb_b<D, double, double>(B, l, t, s, 0, 0, 0, 1);
      DPP_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 5; ++r) launch_cheb_b<D, double, double>(B, l, t, s, 0, 0, 0, 1);
      DPP_HIP(hipEventRecord(e1, s));
      DPP_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      DPP_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms * 0.97f) {
        best_ms = ms;
        best = cand;
      }
    }
    B->lpr[l] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace

// ---------------------------------------------------------------- set-up --
void batch_setup(dpp_batch B, hipStream_t s) {
  const int nb = B->nb;
  const bool d3 = B->dim == 3;
  B->doff.assign(nb + 1, 0);
  for (int i = 0; i < nb; ++i) B->doff[i + 1] = B->doff[i] + B->P[i]->ndof();
  B->ntot = B->doff[nb];
  B->nlev = 0;
  for (auto pc : B->pc) B->nlev = std::max(B->nlev, (int)pc->lv.size() - 1);
  B->active.alloc(sizeof(int) * nb);
  B->fac.alloc(sizeof(double) * nb);
  B->nks.alloc(sizeof(int) * nb);
  B->ydev.alloc(sizeof(double) * (size_t)nb * BMAXK);
  B->hb.alloc(sizeof(double) * (size_t)nb * HS);
  // K-level and Krylov descriptors
  std::vector<KDesc> kv;
  std::vector<VDesc> vv;
  int kb = 0, vb = 0;
  for (int i = 0; i < nb; ++i) {
    dpp_problem P = B->P[i];
    Level &L0 = *B->pc[i]->lv[0];
    KDesc k{};
    k.g = dev(P->g);
    k.blk0 = kb;
    k.nblk = blocks_for(P->g.N, 256);
    kb += k.nblk;
    k.kv = P->kh.ptr;
    k.upt = P->upt.as<double>();
    k.dinv = P->dinv.as<double>();
    k.off = B->doff[i];
    k.rhat = L0.b.ptr;
    k.zp = L0.e.ptr;
    k.inst = i;
    kv.push_back(k);
    VDesc v{};
    v.off = B->doff[i];
    v.n = P->ndof();
    v.blk0 = vb;
    v.nblk = (int)std::min<long>(256, std::max<long>(1, v.n / 2048));
    vb += v.nblk;
    v.inst = i;
    vv.push_back(v);
  }
  B->kd.upload(kv, kb);
  B->vd.upload(vv, vb);
  B->part.alloc(sizeof(double) * (size_t)MV_PART_ROWS * vb);
  std::vector<CDesc> cv;
  int cb = 0;
  for (int i = 0; i < nb; ++i) {
    dpp_precond pc = B->pc[i];
    Level &Lc = *pc->lv.back();
    CDesc c{};
    c.Cinv = pc->cinv.as<double>();
    c.n = pc->ncoarse;
    c.blk0 = cb;
    c.nblk = blocks_for(c.n, 4);
    cb += c.nblk;
    c.b = Lc.b.ptr;
    c.x = Lc.e.ptr;
    c.inst = i;
    cv.push_back(c);
  }
  B->cd.upload(cv, cb);
  if (d3)
    tune_batch_lanes<3>(B, s);
  else
    tune_batch_lanes<2>(B, s);
  B->ld.clear();
  B->ld.resize(B->nlev);
  for (int l = 0; l < B->nlev; ++l) build_level_tables(B, l, B->lpr[l], false, B->ld[l]);
  DPP_HIP(hipStreamSynchronize(s));
}

void batch_make32(dpp_batch B, hipStream_t s) {
  if (B->has32) return;
  for (auto pc : B->pc) precond_make32(pc, s);
  std::vector<KDesc> kv;
  for (int i = 0; i < B->nb; ++i) {
    KDesc k = {};
    DPP_HIP(hipMemcpy(&k, B->kd.get() + i, sizeof(KDesc), hipMemcpyDeviceToHost));
    k.rhat = B->pc[i]->lv[0]->b32.ptr;
    k.zp = B->pc[i]->lv[0]->e32.ptr;
    k.kv = B->P[i]->kh32.ptr;  // FP32 half storage (made by precond_make32)
    kv.push_back(k);
  }
  B->kd32.upload(kv, B->kd.blocks);
  std::vector<CDesc> cv;
  for (int i = 0; i < B->nb; ++i) {
    CDesc c = {};
    DPP_HIP(hipMemcpy(&c, B->cd.get() + i, sizeof(CDesc), hipMemcpyDeviceToHost));
    c.b = B->pc[i]->lv.back()->b32.ptr;
    c.x = B->pc[i]->lv.back()->e32.ptr;
    cv.push_back(c);
  }
  B->cd32.upload(cv, B->cd.blocks);
  B->ld32.clear();
  B->ld32.resize(B->nlev);
  for (int l = 0; l < B->nlev; ++l) build_level_tables(B, l, B->lpr[l], true, B->ld32[l]);
  DPP_HIP(hipStreamSynchronize(s));
  B->has32 = true;
}

// ---------------------------------------------------------------- solve --
// Batched flexible GMRES(m) on K x = rhs (rhs NULL: the assembled f, with the
// consistent part for pure-flux instances) to rtol, at most maxiter iterations
// per instance.  mode 0: FP64 operator and preconditioner; 1: FP32 operator
// and preconditioner (inner solves of iterative refinement); 2: FP64 operator,
// FP32 preconditioner.  Instances with skip[i] set do not run (x_i unchanged).
// stall[i] is set for instances stopped by the stagnation test.
template <int D>
void batch_fgmres(dpp_batch B, const dpp_solve_opts &o, const double *rhs, double *x,
                  dpp_solve_stats *st, double rtol, int maxiter, int mode,
                  const std::vector<int> *skip, std::vector<int> &stall, hipStream_t s) {
  const int nb = B->nb, m = o.restart;
  const bool use_graph = o.use_graph != 0 && !prof_on();
  // Graphs are captured on a stream the library owns (the caller's stream may
  // be the legacy default stream, which cannot be captured); it is ordered
  // after the caller's stream on entry and the caller's stream after it on exit.
  hipStream_t caller = s;
  if (use_graph) {
    if (!B->gstream) DPP_HIP(hipStreamCreateWithFlags(&B->gstream, hipStreamNonBlocking));
    hipEvent_t ev;
    DPP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    DPP_HIP(hipEventRecord(ev, caller));
    DPP_HIP(hipStreamWaitEvent(B->gstream, ev, 0));
    (void)hipEventDestroy(ev);
    s = B->gstream;
  }
  const long n = B->ntot;
  const bool fp32 = mode != 0, op32 = mode == 1;
  DPP_CHECK(2 * (m - 1) + 1 <= MV_PART_ROWS - 1 && m <= BMAXK - 1 &&
                (size_t)B->vd.blocks * MV_PART_ROWS * sizeof(double) <= B->part.bytes,
            DPP_ERR_ARG, "batched Krylov reduction buffer too small for the restart length");
  if (!B->hpin) DPP_HIP(hipHostMalloc((void **)&B->hpin, sizeof(double) * (size_t)nb * HS, hipHostMallocDefault));
  if (!B->hev) DPP_HIP(hipEventCreateWithFlags(&B->hev, hipEventDisableTiming));
  if (B->ws_m < m) {
    B->V.alloc(sizeof(double) * (size_t)(m + 1) * n);
    B->Z.alloc(sizeof(double) * (size_t)m * n);
    B->w.alloc(sizeof(double) * n);
    B->rtmp.alloc(sizeof(double) * n);
    B->ws_m = m;
    for (auto &g : B->graphs) (void)hipGraphExecDestroy(g.second);
    B->graphs.clear();
  }
  double *V = B->V.as<double>();
  const double *f = rhs;
  if (!f) {
    // concatenated right-hand side; a pure-flux instance (singular K) solves
    // for the consistent part of its f, as the single-instance solve does
    double *fc = B->rtmp.as<double>();
    for (int i = 0; i < nb; ++i) {
      DPP_HIP(hipMemcpyAsync(fc + B->doff[i], B->P[i]->f.ptr, sizeof(double) * B->P[i]->ndof(),
                             hipMemcpyDeviceToDevice, s));
      if (pure_flux(B->P[i]->g)) consistent_rhs(B->P[i], fc + B->doff[i], s);
    }
    f = fc;
  }
  std::vector<int> act(nb, 1), conv(nb, 0), its(nb, 0), rest(nb, 0);
  std::vector<Stagnation> stg(nb, Stagnation(o.stag_cycles, o.stag_ratio));
  stall.assign(nb, 0);
  // skipped instances count as finished from the start
  if (skip)
    for (int i = 0; i < nb; ++i) conv[i] = (*skip)[i] ? 1 : 0;
  std::vector<double> bn, rn(nb, 0.0);
  auto upload_active = [&]() {
    B->hact = act;
    DPP_HIP(hipMemcpyAsync(B->active.ptr, act.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
  };
  upload_active();
  norms_b(B, f, 0, bn, s);
  // per instance: unrotated and rotated Hessenberg columns, Givens rotations,
  // right-hand side before (gpre) and after (g) each rotation
  std::vector<double> Hr((size_t)nb * (m + 1) * m), Rr((size_t)nb * (m + 1) * m), cs((size_t)nb * m),
      sn((size_t)nb * m), gpre((size_t)nb * (m + 1)), g((size_t)nb * (m + 1)), y((size_t)nb * BMAXK), fac(nb);
  std::vector<int> kused(nb), stop(nb);
  double *hh = B->hpin;
  auto Hc = [&](int i, int r, int c) -> double & { return Hr[((size_t)i * m + c) * (m + 1) + r]; };
  auto Rc = [&](int i, int r, int c) -> double & { return Rr[((size_t)i * m + c) * (m + 1) + r]; };
  auto rotate_column = [&](int i, int j) {
    for (int r = 0; r <= j + 1; ++r) Rc(i, r, j) = Hc(i, r, j);
    for (int r = 0; r < j; ++r) {
      const double c = cs[(size_t)i * m + r], sr = sn[(size_t)i * m + r];
      const double t = c * Rc(i, r, j) + sr * Rc(i, r + 1, j);
      Rc(i, r + 1, j) = -sr * Rc(i, r, j) + c * Rc(i, r + 1, j);
      Rc(i, r, j) = t;
    }
  };
  auto make_rotation = [&](int i, int j) {
    const double den = std::hypot(Rc(i, j, j), Rc(i, j + 1, j));
    DPP_CHECK(std::isfinite(den), DPP_ERR_NUMERIC, "NaN/Inf in a batched Arnoldi step");
    if (den == 0.0) return false;
    double &c = cs[(size_t)i * m + j], &sr = sn[(size_t)i * m + j];
    c = Rc(i, j, j) / den;
    sr = Rc(i, j + 1, j) / den;
    Rc(i, j, j) = den;
    Rc(i, j + 1, j) = 0.0;
    double *gp = &gpre[(size_t)i * (m + 1)];
    g[(size_t)i * (m + 1) + j] = c * gp[j];
    gp[j + 1] = -sr * gp[j];
    return true;
  };
  auto enqueue = [&](int j) {
    if (!use_graph) {
      arnoldi_step_b<D>(B, j, fp32, op32, s);
      return;
    }
    auto key = std::make_pair(j, mode + 3 * cycle_code(B->opts));
    auto itg = B->graphs.find(key);
    if (itg == B->graphs.end()) {
      hipGraph_t graph;
      DPP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      arnoldi_step_b<D>(B, j, fp32, op32, s);
      DPP_HIP(hipStreamEndCapture(s, &graph));
      hipGraphExec_t ex;
      const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      DPP_HIP(e);
      itg = B->graphs.emplace(key, ex).first;
    }
    DPP_HIP(hipGraphLaunch(itg->second, s));
  };
  int total_iters = 0;
  while (true) {
    // true residuals of the instances still running
    for (int i = 0; i < nb; ++i) act[i] = !conv[i];
    for (int i = 0; i < nb; ++i)
      if (stall[i]) act[i] = 0;
    upload_active();
    spmv_b<D>(B, x, f, V, s, op32);
    norms_b(B, V, 1, rn, s);
    bool any = false;
    for (int i = 0; i < nb; ++i) {
      if (conv[i] || stall[i]) continue;
      DPP_CHECK(std::isfinite(rn[i]), DPP_ERR_NUMERIC, "NaN/Inf in a batched residual");
      if (bn[i] == 0.0 || rn[i] <= rtol * bn[i]) {
        conv[i] = 1;
        act[i] = 0;
      } else if (its[i] >= maxiter) {
        act[i] = 0;
      } else if (stg[i].stalled(rn[i])) {
        stall[i] = 1;
        act[i] = 0;
      } else {
        any = true;
      }
      fac[i] = rn[i] > 0 ? 1.0 / rn[i] : 0.0;
    }
    if (!any) break;
    upload_active();
    DPP_HIP(hipMemcpyAsync(B->fac.ptr, fac.data(), sizeof(double) * nb, hipMemcpyHostToDevice, s));
    kb_scale<<<B->vd.blocks, BBS, 0, s>>>(B->vd.get(), B->vd.count, B->active.as<int>(), V, nullptr, 0,
                                          B->fac.as<double>());
    std::fill(kused.begin(), kused.end(), 0);
    std::fill(stop.begin(), stop.end(), 0);
    for (int i = 0; i < nb; ++i) gpre[(size_t)i * (m + 1)] = rn[i];
    enqueue(0);
    for (int j = 0; j < m; ++j) {
      // copy step j's reductions; queue step j + 1 behind them unless every
      // running instance's residual trend says step j is its last
      DPP_HIP(hipMemcpyAsync(hh, B->hb.ptr, sizeof(double) * (size_t)nb * HS, hipMemcpyDeviceToHost, s));
      DPP_HIP(hipEventRecord(B->hev, s));
      bool want = false;
      for (int i = 0; i < nb; ++i) {
        if (!act[i]) continue;
        const double *gp = &gpre[(size_t)i * (m + 1)];
        const double pred = j >= 1 ? gp[j] * gp[j] / std::fabs(gp[j - 1]) : gp[0];
        if (its[i] + 1 < maxiter && std::fabs(pred) > 4.0 * rtol * bn[i]) want = true;
      }
      const bool queued = j + 1 < m && want;
      if (queued) enqueue(j + 1);
      DPP_HIP(hipEventSynchronize(B->hev));
      ++total_iters;
      bool still = false, changed = false;
      for (int i = 0; i < nb; ++i) {
        if (!act[i]) continue;
        its[i]++;
        const double *h = &hh[(size_t)i * HS];
        bool end = false;
        if (j > 0) {
          // correct column j-1 by a = V^T v~_j and the exact subdiagonal rho_j
          const double rho = h[HB_RHO], alpha = h[HB_ALPHA + (j & 1)];
          for (int r = 0; r < j; ++r) Hc(i, r, j - 1) += h[r];
          Hc(i, j, j - 1) = rho;
          rotate_column(i, j - 1);
          if (!make_rotation(i, j - 1) || !(rho > 1e-2 * std::sqrt(alpha))) {
            kused[i] = j;  // v~_j (almost) inside the basis: column j - 1 ends the cycle
            end = true;
          }
        }
        if (!end) {
          for (int r = 0; r < j; ++r) Hc(i, r, j) = h[j + r];
          Hc(i, j, j) = h[HB_HJJ];
          const double hn = std::sqrt(std::max(0.0, h[HB_ALPHA + ((j + 1) & 1)]));
          Hc(i, j + 1, j) = hn;
          rotate_column(i, j);
          if (!make_rotation(i, j)) {
            kused[i] = j;
            end = true;
          } else {
            kused[i] = j + 1;
            const double res = std::fabs(gpre[(size_t)i * (m + 1) + j + 1]);
            end = res <= rtol * bn[i] || its[i] >= maxiter || hn <= 1e-300 || j + 1 == m;
          }
        }
        if (end) {
          act[i] = 0;
          changed = true;
        } else {
          still = true;
        }
      }
      if (!still) break;
      if (changed) upload_active();
      if (!queued) enqueue(j + 1);
    }
    // wait for a queued step that will not be used, then x_i += Z_i y_i
    DPP_HIP(hipStreamSynchronize(s));
    std::vector<int> nk(nb, 0);
    for (int i = 0; i < nb; ++i) {
      const int k = kused[i];
      nk[i] = k;
      double *yi = &y[(size_t)i * BMAXK];
      const double *gi = &g[(size_t)i * (m + 1)];
      for (int r = k - 1; r >= 0; --r) {
        double t = gi[r];
        for (int c = r + 1; c < k; ++c) t -= Rc(i, r, c) * yi[c];
        yi[r] = t / Rc(i, r, r);
      }
      if (k) rest[i]++;
    }
    DPP_HIP(hipMemcpyAsync(B->ydev.ptr, y.data(), sizeof(double) * y.size(), hipMemcpyHostToDevice, s));
    DPP_HIP(hipMemcpyAsync(B->nks.ptr, nk.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
    const int nkmax = *std::max_element(nk.begin(), nk.end());
    if (nkmax > 0)
      DPP_NK_SWITCH(nkmax, kb_update<NKP><<<B->vd.blocks, BBS, 0, s>>>(B->vd.get(), B->vd.count, B->Z.as<double>(), n,
                                                                      B->ydev.as<double>(), B->nks.as<int>(), x));
    check_launch("batched update");
    bool progress = false;
    for (int i = 0; i < nb; ++i)
      if (!conv[i] && !stall[i] && its[i] < maxiter) progress = true;
    if (!progress) {
      // final residuals for the report
      for (int i = 0; i < nb; ++i) act[i] = 1;
      upload_active();
      spmv_b<D>(B, x, f, V, s, op32);
      norms_b(B, V, 1, rn, s);
      for (int i = 0; i < nb; ++i)
        if (!conv[i] && bn[i] > 0 && rn[i] <= rtol * bn[i]) conv[i] = 1;
      break;
    }
  }
  // pure-flux instances: normalise the pressures (int p1 = 0)
  for (int i = 0; i < nb; ++i)
    if (pure_flux(B->P[i]->g)) normalize_pressures(B->P[i], x + B->doff[i], s);
  DPP_HIP(hipStreamSynchronize(s));
  if (use_graph) DPP_HIP(hipStreamSynchronize(caller));
  for (int i = 0; i < nb; ++i) {
    st[i].iters = its[i];
    st[i].restarts = rest[i];
    st[i].refinements = 0;
    st[i].converged = conv[i];
    st[i].rel_residual = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
    st[i].ms_solve = 0.0;
  }
  (void)total_iters;
}

void batch_apply(dpp_batch B, int what, const double *x, double *y, hipStream_t s) {
  std::vector<int> ones(B->nb, 1);
  B->hact = ones;
  DPP_HIP(hipMemcpyAsync(B->active.ptr, ones.data(), sizeof(int) * B->nb, hipMemcpyHostToDevice, s));
  DPP_HIP(hipStreamSynchronize(s));
  if (B->dim == 3) {
    if (what == 0) spmv_b<3>(B, x, nullptr, y, s); else precond_b<3>(B, x, y, false, s);
  } else {
    if (what == 0) spmv_b<2>(B, x, nullptr, y, s); else precond_b<2>(B, x, y, false, s);
  }
  DPP_HIP(hipStreamSynchronize(s));
}

// Iterative refinement of the batch (precision 1): FP64 true residuals of
// every instance, inner batched FGMRES with the FP32 operator and FP32
// preconditioner to inner_rtol on the instances still running, x += e.
template <int D>
void batch_refine(dpp_batch B, const dpp_solve_opts &o, double *x, dpp_solve_stats *st,
                  std::vector<int> &stall, hipStream_t s) {
  const int nb = B->nb;
  const long n = B->ntot;
  if (!B->fref.ptr) {
    B->fref.alloc(sizeof(double) * n);
    B->rref.alloc(sizeof(double) * n);
    B->eref.alloc(sizeof(double) * n);
  }
  double *f = B->fref.as<double>(), *r = B->rref.as<double>(), *e = B->eref.as<double>();
  for (int i = 0; i < nb; ++i) {
    DPP_HIP(hipMemcpyAsync(f + B->doff[i], B->P[i]->f.ptr, sizeof(double) * B->P[i]->ndof(),
                           hipMemcpyDeviceToDevice, s));
    if (pure_flux(B->P[i]->g)) consistent_rhs(B->P[i], f + B->doff[i], s);
  }
  std::vector<int> ones(nb, 1);
  B->hact = ones;
  DPP_HIP(hipMemcpyAsync(B->active.ptr, ones.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
  std::vector<double> bn, rn;
  norms_b(B, f, 0, bn, s);
  std::vector<int> conv(nb, 0), done(nb, 0), its(nb, 0), rest(nb, 0), refs(nb, 0), inner_stall;
  std::vector<Stagnation> stg(nb, Stagnation(o.stag_cycles, o.stag_ratio));
  std::vector<dpp_solve_stats> sti(nb);
  stall.assign(nb, 0);
  // the inner solves stop at their own tolerance; stagnation is judged on
  // the refinement sweeps
  dpp_solve_opts oi = o;
  oi.stag_cycles = 0;
  for (int sweep = 0;; ++sweep) {
    B->hact = ones;
    DPP_HIP(hipMemcpyAsync(B->active.ptr, ones.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
    spmv_b<D>(B, x, f, r, s);
    norms_b(B, r, 1, rn, s);
    bool any = false;
    for (int i = 0; i < nb; ++i) {
      if (done[i]) continue;
      DPP_CHECK(std::isfinite(rn[i]), DPP_ERR_NUMERIC, "NaN/Inf in a batched refinement residual");
      if (bn[i] == 0.0 || rn[i] <= o.rtol * bn[i]) {
        conv[i] = 1;
        done[i] = 1;
      } else if (its[i] >= o.maxiter || sweep >= o.max_refine) {
        done[i] = 1;
      } else if (stg[i].stalled(rn[i])) {
        stall[i] = 1;
        done[i] = 1;
      } else {
        any = true;
      }
    }
    if (!any) break;
    DPP_HIP(hipMemsetAsync(e, 0, sizeof(double) * n, s));
    const int lim = o.inner_maxiter > 0 ? o.inner_maxiter : o.maxiter;
    batch_fgmres<D>(B, oi, r, e, sti.data(), o.inner_rtol, lim, 1, &done, inner_stall, s);
    axpby(n, 1.0, e, 1.0, x, s);
    for (int i = 0; i < nb; ++i)
      if (!done[i]) {
        its[i] += sti[i].iters;
        rest[i] += sti[i].restarts;
        refs[i]++;
      }
  }
  for (int i = 0; i < nb; ++i)
    if (pure_flux(B->P[i]->g)) normalize_pressures(B->P[i], x + B->doff[i], s);
  DPP_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < nb; ++i) {
    st[i].iters = its[i];
    st[i].restarts = rest[i];
    st[i].refinements = refs[i];
    st[i].converged = conv[i];
    st[i].rel_residual = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
    st[i].ms_solve = 0.0;
  }
}

void batch_solve(dpp_batch B, const dpp_solve_opts &o, double *x, dpp_solve_stats *st, hipStream_t s) {
  if (o.precision != 0) batch_make32(B, s);
  std::vector<int> &stall = B->stalled;
  if (o.precision == 1) {
    if (B->dim == 3)
      batch_refine<3>(B, o, x, st, stall, s);
    else
      batch_refine<2>(B, o, x, st, stall, s);
    return;
  }
  const int mode = o.precision == 2 ? 2 : 0;
  if (B->dim == 3)
    batch_fgmres<3>(B, o, nullptr, x, st, o.rtol, o.maxiter, mode, nullptr, stall, s);
  else
    batch_fgmres<2>(B, o, nullptr, x, st, o.rtol, o.maxiter, mode, nullptr, stall, s);
}

}  // namespace dpp
