// Staging of global-memory tiles into LDS with the loads batched ahead of the stores.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lddmm {

// Walks the elements e = tid, tid + NTHR, tid + 2 NTHR, ... of a row-major rows x cols index space
// keeping (row, column) and the row-major offsets into two arrays of row strides s1 and s2 without
// an integer division per element (a division is a sequence of some 25 instructions on the vector
// unit): the step of NTHR elements is split once into whole rows and a column remainder.  The
// offsets are 32-bit: a staged tile spans less than 2^31 elements of either array.
struct TileWalk {
  int r, c, cols, dr, dc;
  int o1, o2, st1, st2, w1, w2;
  __device__ __forceinline__ TileWalk(int nthr, int tid, int cols_, int s1, int s2) : cols(cols_) {
    dr = nthr / cols;
    dc = nthr - dr * cols;
    r = tid / cols;
    c = tid - r * cols;
    o1 = r * s1 + c, o2 = r * s2 + c;
    st1 = dr * s1 + dc, st2 = dr * s2 + dc;
    w1 = s1 - cols, w2 = s2 - cols;
  }
  __device__ __forceinline__ void next() {
    r += dr, c += dc, o1 += st1, o2 += st2;
    if (c >= cols) c -= cols, ++r, o1 += w1, o2 += w2;
  }
};

// Copies a rows x cols float tile from global memory (row stride gstride) into LDS (row stride
// lstride); elements with r >= vrows or c >= vcols are written as zeros.  Each thread issues U
// loads before its first LDS store, so a tile of up to NTHR * U elements costs one memory
// latency instead of one per element the thread moves.
// Loads are branch-free (an element outside the valid region reads the tile's first element and
// is replaced by zero), and a batch that lies wholly inside the tile stores without per-element
// tests, so the compiler emits no divergent branch per element.
template <int NTHR, int U>
__device__ __forceinline__ void stage_tile(float* __restrict__ lds, int lstride, const float* __restrict__ g,
                                           int64_t gstride, int rows, int cols, int vrows, int vcols) {
  TileWalk w(NTHR, threadIdx.x, cols, static_cast<int>(gstride), lstride);
  const int tot = rows * cols;
  for (int base = 0; base < tot; base += NTHR * U) {
    const bool full = base + NTHR * U <= tot;  // uniform across the block
    const TileWalk w0 = w;
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = (full || w.r < rows) && w.r < vrows && w.c < vcols;
      const float t = g[ok ? w.o1 : 0];
      v[u] = ok ? t : 0.f;
      w.next();
    }
    w = w0;
    if (full) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        lds[w.o2] = v[u];
        w.next();
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (w.r < rows) lds[w.o2] = v[u];
        w.next();
      }
    }
  }
}

}  // namespace lddmm
