// Shared definitions of the gfx950 band-limited PDE-LDDMM library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace lddmm {

// Internal representation: every problem is held as a 3D grid (n0, n1, n2)
// with 3 vector components.  A 2D problem of size N1 x N2 sits in the planes
// n0 = 1 (band k0 = 1, the constant only), with vector component 0 kept at
// zero; the API maps its d = 2 arrays onto components 1 and 2.
struct Dims {
  int n[3];
  int k[3];
  int64_t P;  // grid points
  int64_t Q;  // band coefficients per component
};

class HipError : public std::runtime_error {
 public:
  explicit HipError(const std::string& s) : std::runtime_error(s) {}
};

class ArgError : public std::runtime_error {
 public:
  explicit ArgError(const std::string& s) : std::runtime_error(s) {}
};

#define LDDMM_HIP(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::lddmm::HipError(std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define LDDMM_LAUNCH_CHECK() LDDMM_HIP(hipGetLastError())

// Maximum number of fields in one batched transform.
constexpr int kMaxFields = 12;

template <typename T>
struct FieldMats {
  const T* w[kMaxFields];
};

template <typename T>
struct FieldPtrs {
  const T* p[kMaxFields];
};

// Cubic B-spline weights for the four nodes base-1 .. base+2 around a point at
// fractional offset t in [0,1) from node `base`; each weight is one piece of the
// centred cubic B-spline evaluated at the node's distance.
template <typename T>
__device__ __forceinline__ void bspline_weights(T t, T w[4]) {
  const T t2 = t * t, t3 = t2 * t, u = T(1) - t;
  w[0] = u * u * u * T(1.0 / 6.0);
  w[1] = (T(3) * t3 - T(6) * t2 + T(4)) * T(1.0 / 6.0);
  w[2] = (T(-3) * t3 + T(3) * t2 + T(3) * t + T(1)) * T(1.0 / 6.0);
  w[3] = t3 * T(1.0 / 6.0);
}

// Derivatives of the weights with respect to t.
template <typename T>
__device__ __forceinline__ void bspline_dweights(T t, T w[4]) {
  const T t2 = t * t, u = T(1) - t;
  w[0] = T(-0.5) * u * u;
  w[1] = T(1.5) * t2 - T(2) * t;
  w[2] = T(-1.5) * t2 + t + T(0.5);
  w[3] = T(0.5) * t2;
}

// Split a coordinate (grid units) into the periodic indices of its 4 taps and
// the fractional offset.
template <typename T>
__device__ __forceinline__ T tap_indices(T x, int n, int idx[4]) {
  const T f = floor(x);
  int b = static_cast<int>(f);
  b %= n;
  if (b < 0) b += n;
  int i = b - 1;
  if (i < 0) i += n;
  idx[0] = i;
  for (int o = 1; o < 4; ++o) {
    ++i;
    if (i >= n) i -= n;
    idx[o] = i;
  }
  return x - f;
}

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

}  // namespace lddmm
