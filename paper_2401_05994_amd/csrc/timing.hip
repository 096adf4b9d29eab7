// Optional per-kernel timing with HIP events on the launch stream.
//
// When enabled (mgard_timing(1)), every launch wrapped by KernelTimer records
// a start and an end event on its stream; mgard_timing_report() resolves the
// pairs and returns "name launches total_ms" lines.  Disabled, the wrappers
// cost one branch.
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mg {

namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
thread_local bool g_paused = false;  // set while a graph is being captured on this thread
}  // namespace

bool timing_enabled() { return g_on; }

void timing_pause(bool paused) { g_paused = paused; }

KernelTimer::KernelTimer(const char* name, hipStream_t st) : st_(st), idx_(-1) {
  if (!g_on || g_paused) return;
  Rec r;
  r.name = name;
  MG_HIP(hipEventCreate(&r.a));
  MG_HIP(hipEventCreate(&r.b));
  MG_HIP(hipEventRecord(r.a, st));
  std::lock_guard<std::mutex> lk(g_mu);
  idx_ = (int)g_recs.size();
  g_recs.push_back(r);
}

KernelTimer::~KernelTimer() {
  if (idx_ < 0) return;
  hipEvent_t b;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    b = g_recs[idx_].b;
  }
  (void)hipEventRecord(b, st_);
}

void timing_set(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
  g_on = on != 0;
}

std::string timing_report() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::map<std::string, std::pair<long, double>> acc;
  for (auto& r : g_recs) {
    MG_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    MG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    auto& e = acc[r.name];
    e.first += 1;
    e.second += ms;
  }
  std::string out;
  char line[256];
  for (auto& kv : acc) {
    std::snprintf(line, sizeof line, "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  return out;
}

}  // namespace mg
