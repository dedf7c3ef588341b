// Optional per-launch timing of the library's kernels with HIP events.
// When enabled, every launcher brackets its kernel with two events from a pool
// and records the algorithmic bytes and flops of that launch; a read-out
// aggregates them per kernel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>

namespace lddmm {
namespace prof {

bool enabled();
void set_enabled(bool on);
template <typename T>
inline const char* tname() {
  return sizeof(T) == 4 ? "float" : "double";
}
// per-kernel lines "name\tcount\ttotal_ms\tbytes\tflops\n"; clears the records
std::string collect();

// event pair from the pool and bookkeeping of one timed dispatch
bool take_events(hipEvent_t* start, hipEvent_t* stop);
void record(const std::string& name, double bytes, double flops, hipEvent_t start, hipEvent_t stop);

// Launch a kernel; while profiling is on, the dispatch itself carries the start and
// stop events (hipExtLaunchKernelGGL), so host-side gaps do not enter the timing.
template <typename F, typename... Args>
inline void launch(const std::string& name, double bytes, double flops, F kernel, dim3 grid, dim3 block,
                   uint32_t shm, hipStream_t s, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (enabled() && take_events(&e0, &e1)) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e0, e1, 0, args...);
    record(name, bytes, flops, e0, e1);
  } else {
    kernel<<<grid, block, shm, s>>>(args...);
  }
}

}  // namespace prof
}  // namespace lddmm
