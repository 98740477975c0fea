// Stagnation test across restart cycles of flexible GMRES (or across the
// sweeps of iterative refinement).  Host code only, no HIP: the decision is
// a pure function of the residual norms the solver sees.
#pragma once

namespace dpp {

// stalled(r) is called with the true residual norm at the start of every
// cycle.  It counts the cycles in a row whose end residual (the start of the
// next one) stayed above ratio times their start residual, and reports
// stagnation once that count reaches limit (limit 0: never).
struct Stagnation {
  int limit;
  double ratio;
  int count = 0;
  double prev = -1.0;
  Stagnation(int limit_, double ratio_) : limit(limit_), ratio(ratio_) {}
  bool stalled(double r) {
    if (limit <= 0) return false;
    if (prev >= 0.0) count = r > ratio * prev ? count + 1 : 0;
    prev = r;
    return count >= limit;
  }
};

}  // namespace dpp
