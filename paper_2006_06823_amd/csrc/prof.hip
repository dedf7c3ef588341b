// Event-based per-kernel timing (see prof.h).
#include "prof.h"

#include <map>
#include <mutex>
#include <vector>

namespace lddmm {
namespace prof {

namespace {

struct Record {
  std::string name;
  double bytes, flops;
  hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Record> g_rec;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool enabled() { return g_on; }

bool take_events(hipEvent_t* start, hipEvent_t* stop) {
  std::lock_guard<std::mutex> lk(g_mu);
  *start = take_event();
  *stop = take_event();
  return *start != nullptr && *stop != nullptr;
}

void record(const std::string& name, double bytes, double flops, hipEvent_t start, hipEvent_t stop) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_rec.push_back(Record{name, bytes, flops, start, stop});
}

void set_enabled(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on;
}

std::string collect() {
  std::lock_guard<std::mutex> lk(g_mu);
  struct Agg {
    long count = 0;
    double ms = 0, bytes = 0, flops = 0;
  };
  std::map<std::string, Agg> agg;
  for (auto& r : g_rec) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      Agg& a = agg[r.name];
      a.count += 1;
      a.ms += ms;
      a.bytes += r.bytes;
      a.flops += r.flops;
    }
    g_pool.push_back(r.start);
    g_pool.push_back(r.stop);
  }
  g_rec.clear();
  std::string out;
  char line[512];
  for (auto& kv : agg) {
    snprintf(line, sizeof(line), "%s\t%ld\t%.6f\t%.0f\t%.0f\n", kv.first.c_str(), kv.second.count, kv.second.ms,
             kv.second.bytes, kv.second.flops);
    out += line;
  }
  return out;
}

}  // namespace prof
}  // namespace lddmm
