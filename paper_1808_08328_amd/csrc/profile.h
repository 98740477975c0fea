// Kernel-family timing: when enabled, launches of the instrumented families
// are bracketed by HIP events on their own stream, and the algorithmic bytes
// each launch must move are accumulated next to the measured time.
#pragma once

#include "common.h"

namespace dpp {

enum ProfFamily {
  PF_SPMV_K = 0,     // y = K x and r = b - K x (node-pair stencil)
  PF_CHEB_L0 = 1,    // Chebyshev step with S_p product, finest level
  PF_RESID_L0 = 2,   // residual b - S_p x, finest level
  PF_SCHUR_RHS = 3,  // r_p - K_pu D^-1 r_u
  PF_SCHUR_VEL = 4,  // D^-1 (r_u - K_up z_p)
  PF_COARSE = 5,     // every kernel of the coarser levels and the coarse solve
  PF_VECTOR_L0 = 6,  // finest level: first Chebyshev step (no product), restriction, prolongation
  PF_ARNOLDI = 7,    // CGS2 passes, norms, scaling, solution update
  // batched solves (every running instance in one launch)
  PF_B_SPMV_K = 8,   // y = K x, r = b - K x
  PF_B_CHEB_L0 = 9,  // Chebyshev step (or residual) with the S_p product, finest levels
  PF_B_SCHUR = 10,   // Schur right-hand side and velocity step
  PF_B_LEVELS = 11,  // coarser levels, restriction, prolongation, coarse solves
  PF_B_ARNOLDI = 12, // DCGS2 passes and their finish kernels
  // DG-VMS fieldsplit (both networks in one launch)
  PF_DG_VEL = 13,    // velocity-block Chebyshev step with the simplex-block Jacobi
  PF_DG_PRES = 14,   // pressure side: K_up products, S_q Chebyshev steps, r_p - K_pu y_u, z_p copy
  PF_DG_TRANSFER = 15,  // slots to nodes and back around the nodal cycle
  PF_COUNT = 16
};

bool prof_on();
void prof_begin(int fam, hipStream_t s);
void prof_end(int fam, double bytes, hipStream_t s);

struct ProfScope {
  int fam;
  double bytes;
  hipStream_t s;
  bool on;
  ProfScope(int f, double b, hipStream_t st) : fam(f), bytes(b), s(st), on(prof_on()) {
    if (on) prof_begin(fam, s);
  }
  ~ProfScope() {
    if (on) prof_end(fam, bytes, s);
  }
};

// Number of (node, offset) pairs of a stencil that stay inside the box.
template <int D, bool PRESSURE>
inline double valid_pairs(const Grid &g) {
  double tot = 0.0;
  constexpr int n = PRESSURE ? Tabs<D>::NT : Tabs<D>::NS;
  for (int t = 0; t < n; ++t) {
    const int *o = PRESSURE ? TAB<D>.to[t] : TAB<D>.so[t];
    double c = 1.0;
    for (int a = 0; a < dim_of(D); ++a) c *= std::max(0, g.m[a] - std::abs(o[a]));
    tot += c;
  }
  return tot;
}

}  // namespace dpp
