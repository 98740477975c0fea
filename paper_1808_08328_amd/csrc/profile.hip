// Kernel-family timing with HIP events (instrumentation mode only).
#include <mutex>

#include "objects.h"
#include "profile.h"

namespace dpp {

namespace {

struct Rec {
  int fam;
  hipEvent_t a, b;
  double bytes;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<hipEvent_t> g_open[PF_COUNT];

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  DPP_HIP(hipEventCreate(&e));
  return e;
}

}  // namespace

bool prof_on() { return g_on; }

void prof_begin(int fam, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = take();
  DPP_HIP(hipEventRecord(e, s));
  g_open[fam].push_back(e);
}

void prof_end(int fam, double bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_open[fam].empty()) return;
  hipEvent_t a = g_open[fam].back();
  g_open[fam].pop_back();
  hipEvent_t b = take();
  DPP_HIP(hipEventRecord(b, s));
  g_recs.push_back(Rec{fam, a, b, bytes});
}

}  // namespace dpp

extern "C" {

// Instrumentation hook (declared in dpp.h): enable/disable and reset.
dpp_status dpp_profile_enable(int on) {
  try {
    std::lock_guard<std::mutex> lk(dpp::g_mu);
    for (auto &r : dpp::g_recs) {
      dpp::g_pool.push_back(r.a);
      dpp::g_pool.push_back(r.b);
    }
    dpp::g_recs.clear();
    dpp::g_on = on != 0;
    return DPP_OK;
  } catch (...) {
    return DPP_ERR_HIP;
  }
}

dpp_status dpp_profile_read(int family, int64_t *launches, double *total_ms, double *total_bytes) {
  if (family < 0 || family >= dpp::PF_COUNT) return DPP_ERR_ARG;
  std::lock_guard<std::mutex> lk(dpp::g_mu);
  int64_t n = 0;
  double ms = 0.0, by = 0.0;
  for (auto &r : dpp::g_recs) {
    if (r.fam != family) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return DPP_ERR_HIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return DPP_ERR_HIP;
    ++n;
    ms += t;
    by += r.bytes;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (total_bytes) *total_bytes = by;
  return DPP_OK;
}

}  // extern "C"
