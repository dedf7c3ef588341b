// Staging of global-memory tiles into LDS with the loads batched ahead of the stores.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lddmm {

// Copies a rows x cols float tile from global memory (row stride gstride) into LDS (row stride
// lstride); elements with r >= vrows or c >= vcols are written as zeros.  Each thread issues U
// loads before its first LDS store, so a tile of up to NTHR * U elements costs one memory
// latency instead of one per element the thread moves.
template <int NTHR, int U>
__device__ __forceinline__ void stage_tile(float* __restrict__ lds, int lstride, const float* __restrict__ g,
                                           int64_t gstride, int rows, int cols, int vrows, int vcols) {
  const int tid = threadIdx.x;
  const int tot = rows * cols;
  for (int base = 0; base < tot; base += NTHR * U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NTHR + tid;
      v[u] = 0.f;
      if (e < tot) {
        const int r = e / cols, c = e - r * cols;
        if (r < vrows && c < vcols) v[u] = g[(int64_t)r * gstride + c];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NTHR + tid;
      if (e < tot) {
        const int r = e / cols, c = e - r * cols;
        lds[r * lstride + c] = v[u];
      }
    }
  }
}

}  // namespace lddmm
