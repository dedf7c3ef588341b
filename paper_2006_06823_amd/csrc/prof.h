// Optional per-launch timing of the library's kernels with HIP events.
// When enabled, every launcher brackets its kernel with two events from a pool
// and records the algorithmic bytes and flops of that launch; a read-out
// aggregates them per kernel.
#pragma once

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

class Scope {
 public:
  Scope(hipStream_t s, const std::string& name, double bytes, double flops);
  ~Scope();
  Scope(const Scope&) = delete;
  Scope& operator=(const Scope&) = delete;

 private:
  hipStream_t s_;
  int slot_ = -1;
};

}  // namespace prof
}  // namespace lddmm
