// FP64 reductions on the device: PCG inner products and norms, the data term
// of the objective, the regulariser, the gradient infinity norm and the
// Jacobian extrema.  Two passes with a fixed block count keep the summation
// order deterministic: each block reduces a strided slice to one double (wave
// shuffles, then LDS across the block's waves), a single block adds the partials.
#include "kernels.h"

namespace lddmm {

namespace {

constexpr int kRBlocks = 512;
constexpr int kRThreads = 256;

enum class Op { Sum, Max, Min };

template <Op op>
__device__ __forceinline__ double combine(double a, double b) {
  if constexpr (op == Op::Sum) return a + b;
  // NaN-propagating: a NaN operand wins, so a non-finite input shows in max / min
  if constexpr (op == Op::Max) return (a > b || a != a) ? a : b;
  return (a < b || a != a) ? a : b;
}

template <Op op>
__device__ __forceinline__ double identity() {
  if constexpr (op == Op::Sum) return 0.0;
  if constexpr (op == Op::Max) return -1.0 / 0.0;
  return 1.0 / 0.0;
}

template <Op op>
__device__ double block_reduce(double v) {
  __shared__ double part[kRThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v = combine<op>(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = part[0];
    for (int w = 1; w < kRThreads / 64; ++w) r = combine<op>(r, part[w]);
    v = r;
  }
  return v;
}

enum class Kind { Dot, SqDiff, MaxAbs, SymDot, Max, Min };

template <typename T, Kind kind>
__global__ __launch_bounds__(kRThreads) void k_reduce_pass1(const T* a, const T* b, const double* sym,
                                                            int64_t Q, int64_t n, double* work) {
  constexpr Op op = (kind == Kind::MaxAbs || kind == Kind::Max) ? Op::Max : (kind == Kind::Min ? Op::Min : Op::Sum);
  double acc = identity<op>();
  for (int64_t i = blockIdx.x * (int64_t)kRThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRThreads) {
    double x;
    if constexpr (kind == Kind::Dot) {
      x = static_cast<double>(a[i]) * static_cast<double>(b[i]);
    } else if constexpr (kind == Kind::SqDiff) {
      const double dd = static_cast<double>(a[i]) - static_cast<double>(b[i]);
      x = dd * dd;
    } else if constexpr (kind == Kind::MaxAbs) {
      x = fabs(static_cast<double>(a[i]));
    } else if constexpr (kind == Kind::SymDot) {
      x = sym[i % Q] * static_cast<double>(a[i]) * static_cast<double>(b[i]);
    } else {
      x = static_cast<double>(a[i]);
    }
    acc = combine<op>(acc, x);
  }
  acc = block_reduce<op>(acc);
  if (threadIdx.x == 0) work[blockIdx.x] = acc;
}

template <Op op>
__global__ __launch_bounds__(kRThreads) void k_reduce_pass2(double* work, int nparts, int slot) {
  double acc = identity<op>();
  for (int i = threadIdx.x; i < nparts; i += kRThreads) acc = combine<op>(acc, work[i]);
  acc = block_reduce<op>(acc);
  if (threadIdx.x == 0) work[kRBlocks + slot] = acc;
}

template <typename T, Kind kind>
void launch(const T* a, const T* b, const double* sym, int64_t Q, int64_t n, double* work, hipStream_t s,
            int slot) {
  constexpr Op op = (kind == Kind::MaxAbs || kind == Kind::Max) ? Op::Max : (kind == Kind::Min ? Op::Min : Op::Sum);
  int blocks = ceil_div(n, kRThreads);
  if (blocks > kRBlocks) blocks = kRBlocks;
  if (blocks < 1) blocks = 1;
  k_reduce_pass1<T, kind><<<blocks, kRThreads, 0, s>>>(a, b, sym, Q, n, work);
  LDDMM_LAUNCH_CHECK();
  k_reduce_pass2<op><<<1, kRThreads, 0, s>>>(work, blocks, slot);
  LDDMM_LAUNCH_CHECK();
}

double fetch(double* work, double* host, int count, hipStream_t s) {
  LDDMM_HIP(hipMemcpyAsync(host, work + kRBlocks, count * sizeof(double), hipMemcpyDeviceToHost, s));
  LDDMM_HIP(hipStreamSynchronize(s));
  return host[0];
}

}  // namespace

int64_t reduce_work_size() { return kRBlocks + kRedSlots; }

double* reduce_slots(double* work) { return work + kRBlocks; }

template <typename T>
double dot(const T* a, const T* b, int64_t n, double* work, double* host, hipStream_t s) {
  launch<T, Kind::Dot>(a, b, nullptr, 1, n, work, s, 0);
  return fetch(work, host, 1, s);
}

template <typename T>
double sqdiff(const T* a, const T* b, int64_t n, double* work, double* host, hipStream_t s) {
  launch<T, Kind::SqDiff>(a, b, nullptr, 1, n, work, s, 0);
  return fetch(work, host, 1, s);
}

template <typename T>
double maxabs(const T* a, int64_t n, double* work, double* host, hipStream_t s) {
  launch<T, Kind::MaxAbs>(a, nullptr, nullptr, 1, n, work, s, 0);
  return fetch(work, host, 1, s);
}

template <typename T>
double sym_dot(const T* x, const T* y, const double* sym, int ncomp, int64_t Q, double* work, double* host,
               hipStream_t s) {
  launch<T, Kind::SymDot>(x, y, sym, Q, Q * ncomp, work, s, 0);
  return fetch(work, host, 1, s);
}

void minmax_f64(const double* a, int64_t n, double* work, double* host2, hipStream_t s) {
  launch<double, Kind::Min>(a, nullptr, nullptr, 1, n, work, s, 0);
  launch<double, Kind::Max>(a, nullptr, nullptr, 1, n, work, s, 1);
  fetch(work, host2, 2, s);
}

template <typename T>
void reduce_launch(RedKind kind, const T* a, const T* b, int64_t n, double* work, int slot, hipStream_t s) {
  if (slot < 0 || slot >= kRedSlots) throw ArgError("reduce_launch: result slot out of range");
  switch (kind) {
    case RedKind::Dot:
      launch<T, Kind::Dot>(a, b, nullptr, 1, n, work, s, slot);
      break;
    case RedKind::SqDiff:
      launch<T, Kind::SqDiff>(a, b, nullptr, 1, n, work, s, slot);
      break;
    case RedKind::MaxAbs:
      launch<T, Kind::MaxAbs>(a, nullptr, nullptr, 1, n, work, s, slot);
      break;
  }
}

template <typename T>
void sym_dot_launch(const T* x, const T* y, const double* sym, int ncomp, int64_t Q, double* work, int slot,
                    hipStream_t s) {
  if (slot < 0 || slot >= kRedSlots) throw ArgError("sym_dot_launch: result slot out of range");
  launch<T, Kind::SymDot>(x, y, sym, Q, Q * ncomp, work, s, slot);
}

void fetch_async(double* work, double* host, int count, hipStream_t s) {
  LDDMM_HIP(hipMemcpyAsync(host, work + kRBlocks, count * sizeof(double), hipMemcpyDeviceToHost, s));
}

// ---- PCG steps with their scalars on the device (result slots sc = reduce_slots(work))
namespace {
// x += a p, r -= a Ap with a = rz / pAp, applied only when pAp > 0 (a non-positive curvature leaves
// every vector as it was, for the caller's truncation)
template <typename T>
__global__ void k_pcg_step(T* x, T* r, const T* p, const T* Ap, const double* sc, int irz, int ipap, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double pap = sc[ipap];
  if (i >= n || !(pap > 0.0)) return;
  const T a = static_cast<T>(sc[irz] / pap);
  x[i] = T(1) * x[i] + a * p[i];
  r[i] = T(1) * r[i] + (-a) * Ap[i];
}
// p = z + beta p, only when pAp > 0: beta = rz_new / rz, or with ixz >= 0 (flexible CG, the slot holding
// r_new . z_old) beta = (rz_new - r_new . z_old) / rz
template <typename T>
__global__ void k_pcg_dir(T* p, const T* z, const double* sc, int irz, int irzn, int ipap, int ixz, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || !(sc[ipap] > 0.0)) return;
  const T b = static_cast<T>((sc[irzn] - (ixz >= 0 ? sc[ixz] : 0.0)) / sc[irz]);
  p[i] = T(1) * z[i] + b * p[i];
}
// z += sum_i y_i Z_i with y = Minv c, c_i = sc[ic + i] (r <= 16 directions of length n, Minv r x r)
template <typename T>
__global__ void k_lowrank_add(T* z, const T* Z, const double* Minv, const double* sc, int ic, int r, int64_t n) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  double acc = 0.0;
  for (int i = 0; i < r; ++i) {
    double yi = 0.0;
    for (int j = 0; j < r; ++j) yi += Minv[i * r + j] * sc[ic + j];
    acc += yi * static_cast<double>(Z[(int64_t)i * n + k]);
  }
  z[k] = z[k] + static_cast<T>(acc);
}
}  // namespace

template <typename T>
void pcg_step(T* x, T* r, const T* p, const T* Ap, double* work, int irz, int ipap, int64_t n, hipStream_t s) {
  k_pcg_step<T><<<ceil_div(n, 256), 256, 0, s>>>(x, r, p, Ap, work + kRBlocks, irz, ipap, n);
  LDDMM_LAUNCH_CHECK();
}
template <typename T>
void pcg_dir(T* p, const T* z, double* work, int irz, int irzn, int ipap, int64_t n, hipStream_t s, int ixz) {
  k_pcg_dir<T><<<ceil_div(n, 256), 256, 0, s>>>(p, z, work + kRBlocks, irz, irzn, ipap, ixz, n);
  LDDMM_LAUNCH_CHECK();
}
template <typename T>
void lowrank_add(T* z, const T* Z, const double* Minv, double* work, int ic, int r, int64_t n, hipStream_t s) {
  k_lowrank_add<T><<<ceil_div(n, 256), 256, 0, s>>>(z, Z, Minv, work + kRBlocks, ic, r, n);
  LDDMM_LAUNCH_CHECK();
}
template void pcg_step<float>(float*, float*, const float*, const float*, double*, int, int, int64_t, hipStream_t);
template void pcg_step<double>(double*, double*, const double*, const double*, double*, int, int, int64_t,
                               hipStream_t);
template void pcg_dir<float>(float*, const float*, double*, int, int, int, int64_t, hipStream_t, int);
template void pcg_dir<double>(double*, const double*, double*, int, int, int, int64_t, hipStream_t, int);
template void lowrank_add<float>(float*, const float*, const double*, double*, int, int, int64_t, hipStream_t);
template void lowrank_add<double>(double*, const double*, const double*, double*, int, int, int64_t, hipStream_t);

template void reduce_launch<float>(RedKind, const float*, const float*, int64_t, double*, int, hipStream_t);
template void reduce_launch<double>(RedKind, const double*, const double*, int64_t, double*, int, hipStream_t);
template void sym_dot_launch<float>(const float*, const float*, const double*, int, int64_t, double*, int,
                                    hipStream_t);
template void sym_dot_launch<double>(const double*, const double*, const double*, int, int64_t, double*, int,
                                     hipStream_t);
template double dot<float>(const float*, const float*, int64_t, double*, double*, hipStream_t);
template double dot<double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template double sqdiff<float>(const float*, const float*, int64_t, double*, double*, hipStream_t);
template double sqdiff<double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template double maxabs<float>(const float*, int64_t, double*, double*, hipStream_t);
template double maxabs<double>(const double*, int64_t, double*, double*, hipStream_t);
template double sym_dot<float>(const float*, const float*, const double*, int, int64_t, double*, double*,
                               hipStream_t);
template double sym_dot<double>(const double*, const double*, const double*, int, int64_t, double*, double*,
                                hipStream_t);

}  // namespace lddmm
