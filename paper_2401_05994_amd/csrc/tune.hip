// Registry of autotuned launch shapes.
//
// Key: (knob, dtype, fine level shape n0 x n1 x n2); value: the launch
// parameter the tuner found fastest.  Knobs: TUNE_COEFF_SEG (coarse intervals
// of dim 0 per block of the decomposition's plane-marching kernel) and
// TUNE_SCATTER_PLANES (fine planes per block of the recomposition's scatter
// kernel).  Every value of either knob gives the same results; only the
// launch shape changes.  The table persists as a flat JSON object
// {"knob:dtype:n0xn1xn2": value, ...} in the file named by MGARD_TUNE_FILE.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace mg {

namespace {

struct TuneKey {
  int knob, f64, n0, n1, n2;
  bool operator<(const TuneKey& o) const {
    if (knob != o.knob) return knob < o.knob;
    if (f64 != o.f64) return f64 < o.f64;
    if (n0 != o.n0) return n0 < o.n0;
    if (n1 != o.n1) return n1 < o.n1;
    return n2 < o.n2;
  }
};

std::mutex g_mu;
std::map<TuneKey, int> g_table;
bool g_loaded = false;
thread_local int g_force[TUNE_KNOBS] = {0, 0};

const char* knob_name(int k) { return k == TUNE_COEFF_SEG ? "coeff_seg" : "scatter_planes"; }

const char* tune_file() {
  const char* f = std::getenv("MGARD_TUNE_FILE");
  return (f && *f) ? f : nullptr;
}

// Reads entries "name:f32|f64:AxBxC": V from the file; anything else is skipped.
void load_locked() {
  g_loaded = true;
  const char* path = tune_file();
  if (!path) return;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, got);
  std::fclose(fp);
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = text.substr(pos + 1, end - pos - 1);
    pos = end + 1;
    const size_t colon = text.find(':', pos);
    if (colon == std::string::npos) break;
    const int value = std::atoi(text.c_str() + colon + 1);
    char name[32] = {0}, dt[8] = {0};
    int a = 0, b = 0, c = 0;
    if (std::sscanf(key.c_str(), "%31[a-z_]:%7[f0-9]:%dx%dx%d", name, dt, &a, &b, &c) != 5 || value < 1) continue;
    int knob = -1;
    for (int k = 0; k < TUNE_KNOBS; ++k)
      if (std::string(name) == knob_name(k)) knob = k;
    if (knob < 0) continue;
    g_table[TuneKey{knob, std::string(dt) == "f64" ? 1 : 0, a, b, c}] = value;
  }
}

void save_locked() {
  const char* path = tune_file();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return;
  std::fprintf(fp, "{");
  bool first = true;
  for (const auto& kv : g_table) {
    std::fprintf(fp, "%s\n  \"%s:%s:%dx%dx%d\": %d", first ? "" : ",", knob_name(kv.first.knob),
                 kv.first.f64 ? "f64" : "f32", kv.first.n0, kv.first.n1, kv.first.n2, kv.second);
    first = false;
  }
  std::fprintf(fp, "\n}\n");
  std::fclose(fp);
  std::rename(tmp.c_str(), path);
}

}  // namespace

int tune_get(int knob, bool f64, int n0, int n1, int n2, int fallback) {
  if (g_force[knob] > 0) return g_force[knob];
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_loaded) load_locked();
  auto it = g_table.find(TuneKey{knob, f64 ? 1 : 0, n0, n1, n2});
  return it == g_table.end() ? fallback : it->second;
}

bool tune_known(int knob, bool f64, int n0, int n1, int n2) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_loaded) load_locked();
  return g_table.count(TuneKey{knob, f64 ? 1 : 0, n0, n1, n2}) != 0;
}

void tune_set(int knob, bool f64, int n0, int n1, int n2, int value) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_loaded) load_locked();
  g_table[TuneKey{knob, f64 ? 1 : 0, n0, n1, n2}] = value;
}

void tune_force(int knob, int value) { g_force[knob] = value; }

void tune_save() {
  std::lock_guard<std::mutex> lk(g_mu);
  save_locked();
}

}  // namespace mg
