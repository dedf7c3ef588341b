// Project autotuner: picks a kernel variant (tile shape, contraction kernel) per
// problem shape by timing every candidate on the real shapes, and caches the
// choice process-wide under a key such as "brick:128x128x128:gs2".
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <utility>
#include <vector>

namespace lddmm {
namespace tune {

int get(const std::string& key, int fallback);
void set(const std::string& key, int choice);
// Launches candidate c (c < ncand) through run(c) on stream s; returns the fastest (min over reps).
int pick(int ncand, const std::function<void(int)>& run, hipStream_t s, int reps = 3);
// All cached choices, for reporting.
std::vector<std::pair<std::string, int>> table();

// Launch parameters that are tuned lazily (the workgroup caps of the DFT contractions) are timed only
// inside a Collect scope on the calling thread (the solver's set-up pass), never while the stream is
// being captured into a graph; elsewhere an unseen key takes its default.
bool collecting(hipStream_t s);
struct Collect {
  Collect();
  ~Collect();
};
// Choice for key among candidates cand[0..n): cached, or timed through run(value) inside a Collect
// scope, or dflt.
int choose(const std::string& key, const int* cand, int n, int dflt, const std::function<void(int)>& run,
           hipStream_t s);

}  // namespace tune
}  // namespace lddmm
