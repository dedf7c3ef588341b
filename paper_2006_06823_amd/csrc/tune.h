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

}  // namespace tune
}  // namespace lddmm
