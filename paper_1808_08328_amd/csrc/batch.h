// Batched-solve descriptors and the object behind the dpp_batch handle.
#pragma once

#include <map>

#include "objects.h"

namespace dpp {

constexpr int BMAXK = 32;           // basis vectors per instance in the fused kernels
constexpr int HS = 2 * BMAXK + 4;   // per-instance slots of the Hessenberg scratch
// per-instance slot layout: [a (nj) | b (nj) | t.w] from 0, ||v~||^2 of two
// consecutive steps, rho and hjj of the current step
constexpr int HB_ALPHA = 2 * BMAXK;
constexpr int HB_RHO = HB_ALPHA + 2;
constexpr int HB_HJJ = HB_RHO + 1;
constexpr int BBS = 256;

struct KDesc {
  GridDev g;
  int blk0, nblk;           // node blocks (one network per grid row)
  const void *kv;           // K storage (FP64 or FP32 copy)
  const double *upt;        // K_up class table (UPT<dim>)
  const double *dinv;       // [2][N]
  long off;                 // offset of the instance in concatenated vectors
  void *rhat;               // finest-level V-cycle input  [2][N]
  void *zp;                 // finest-level V-cycle output [2][N]
  int inst;
};

struct LDesc {
  GridDev g, gc;            // this level, next coarser level
  int blk0, nblk;           // node blocks of this level (x LPR lanes)
  int cblk0, cnblk;         // coarse-node blocks (restriction)
  const void *A;            // symmetric-half storage of the level operator
  const void *dinv;
  void *b, *xa, *xb, *d, *r, *e;
  void *bc, *ec;            // coarser level's right-hand side and correction
  double c1[8][2], c2[8][2];
  int inst;
};

struct CDesc {
  const double *Cinv;
  int n, blk0, nblk, inst;
  void *b, *x;
};

struct VDesc {
  long off, n;
  int blk0, nblk, inst;
};

template <typename T>
struct DTable {
  DBuf buf;
  int count = 0, blocks = 0;
  void upload(const std::vector<T> &v, int nblocks) {
    count = (int)v.size();
    blocks = nblocks;
    buf.alloc(sizeof(T) * std::max<size_t>(1, v.size()));
    if (!v.empty()) DPP_HIP(hipMemcpy(buf.ptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  }
  const T *get() const { return buf.as<T>(); }
};

}  // namespace dpp

struct dpp_batch_s {
  int nb = 0, dim = 3;
  bool any_bc = false;                   // some instance has velocity faces
  std::vector<dpp_problem> P;
  std::vector<dpp_precond> pc;
  std::vector<long> doff;
  long ntot = 0;
  dpp_solve_opts opts;
  int nlev = 0;                          // max smoothing levels over instances
  std::vector<int> lpr;                  // lanes per row per level index (autotuned)
  dpp::DTable<dpp::KDesc> kd, kd32;
  std::vector<dpp::DTable<dpp::LDesc>> ld, ld32;
  dpp::DTable<dpp::CDesc> cd, cd32;
  dpp::DTable<dpp::VDesc> vd;
  dpp::DBuf active, fac, nks, ydev;
  std::vector<int> hact;                 // host copy of the active flags (profiling bytes)
  dpp::DBuf V, Z, w, part, hb, rtmp;
  dpp::DBuf fref, rref, eref;            // iterative refinement: f, residual, correction
  std::vector<int> stalled;              // instances the last solve stopped for stagnation
  int ws_m = 0;
  bool has32 = false;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  hipStream_t gstream = nullptr;  // capture/replay stream (default priority)
  double *hpin = nullptr;         // pinned host copy of one step's reductions [nb][HS]
  hipEvent_t hev = nullptr;       // marks that copy
  ~dpp_batch_s() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (hev) (void)hipEventDestroy(hev);
    if (hpin) (void)hipHostFree(hpin);
    for (auto p : pc) delete p;
    for (auto p : P) delete p;
  }
};

