// Autotuner cache and timing (see tune.h).
#include "tune.h"

#include <map>
#include <mutex>

#include "common.h"

namespace lddmm {
namespace tune {

namespace {
std::mutex g_mu;
std::map<std::string, int> g_choice;
}  // namespace

int get(const std::string& key, int fallback) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_choice.find(key);
  return it == g_choice.end() ? fallback : it->second;
}

void set(const std::string& key, int choice) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_choice[key] = choice;
}

int pick(int ncand, const std::function<void(int)>& run, hipStream_t s, int reps) {
  hipEvent_t a, b;
  LDDMM_HIP(hipEventCreate(&a));
  LDDMM_HIP(hipEventCreate(&b));
  int best = 0;
  float best_ms = 1e30f;
  for (int c = 0; c < ncand; ++c) {
    run(c);  // warm-up
    float mn = 1e30f;
    for (int r = 0; r < reps; ++r) {
      LDDMM_HIP(hipEventRecord(a, s));
      run(c);
      LDDMM_HIP(hipEventRecord(b, s));
      LDDMM_HIP(hipEventSynchronize(b));
      float ms = 0.f;
      LDDMM_HIP(hipEventElapsedTime(&ms, a, b));
      if (ms < mn) mn = ms;
    }
    if (mn < best_ms) {
      best_ms = mn;
      best = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

namespace {
thread_local int t_collect = 0;
}

Collect::Collect() { ++t_collect; }
Collect::~Collect() { --t_collect; }

bool collecting(hipStream_t s) {
  if (t_collect == 0) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
  return cs == hipStreamCaptureStatusNone;
}

int choose(const std::string& key, const int* cand, int n, int dflt, const std::function<void(int)>& run,
           hipStream_t s) {
  const int c = get(key, -1);
  if (c >= 0 && c < n) return cand[c];
  if (!collecting(s)) return dflt;
  const int best = pick(n, [&](int i) { run(cand[i]); }, s);
  set(key, best);
  return cand[best];
}

std::vector<std::pair<std::string, int>> table() {
  std::lock_guard<std::mutex> lk(g_mu);
  return {g_choice.begin(), g_choice.end()};
}

}  // namespace tune
}  // namespace lddmm
