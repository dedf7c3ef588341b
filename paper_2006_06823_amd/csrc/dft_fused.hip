// Fused inner-axis stages of the truncated DFT (float, matrix cores).
//
// iota: band [f][a0][a1][a2] -> plane slab [f][a0][x1][x2] in one kernel per
//   (field, a0, 64-row block of x1):  t = S W2^T  (a2 contracted, kept in LDS),
//   then out = W1 t (a1 contracted).  A prologue forms the input as x + alpha y
//   (the BL combinations of the SL steps) so no separate axpy pass is needed.
// pi: grid slab [f][a0][x1][x2] -> band [f][a0][a1][a2] in one kernel per
//   (field, a0): t = P1 slab (x1 contracted, the slab streamed from global
//   memory straight into the matrix-core operands), then r = t P2^T (x2
//   contracted; partial sums of the waves reduced in LDS), and an epilogue
//   out = beta out + alpha r per field (plain store or accumulation).
// Both replace two launches of the separable scheme and keep the K x N
// intermediate on chip.
#include "kernels.h"
#include "prof.h"

namespace lddmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ void zero16(f32x16& a) {
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = 0.f;
}

constexpr int kMaxN = 192, kMaxK = 64;

__global__ __launch_bounds__(256) void k_iota_ab(IotaABArgs a) {
  extern __shared__ float smem[];
  const int f = blockIdx.z, a0 = blockIdx.y, x1b = blockIdx.x * 64;
  const int k0 = a.k0, k1 = a.k1, k2 = a.k2, n1 = a.n1, n2 = a.n2;
  const int lds = k2 + 1, ldt = n2 + 4;
  float* S = smem;             // [a1][a2]
  float* T = smem + k1 * lds;  // [a1][x2]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kh = lane >> 5, li = lane & 31;
  // prologue: slab = x + alpha y
  {
    const int64_t off = (int64_t)a0 * k1 * k2;
    const float* x = a.x[f] + off;
    const float* y = a.y[f] ? a.y[f] + off : nullptr;
    const float al = a.alpha[f];
    for (int e = tid; e < k1 * k2; e += 256) {
      const int r = e / k2, c = e - r * k2;
      float v = x[e];
      if (y) v += al * y[e];
      S[r * lds + c] = v;
    }
  }
  __syncthreads();
  // stage 1: T[a1][x2] = sum_a2 S[a1][a2] W2[x2][a2]
  const float* __restrict__ W2t = a.w2t[f];  // [k2][n2]
  const int mb1 = (k1 + 31) / 32, nb = (n2 + 31) / 32;
  for (int tile = wave; tile < mb1 * nb; tile += 4) {
    const int mb = tile / nb, cb = tile - mb * nb;
    f32x16 acc;
    zero16(acc);
    const int arow = mb * 32 + li, x2 = cb * 32 + li;
    for (int kk = 0; kk < k2; kk += 2) {
      const int l = kk + kh;
      const float av = (arow < k1 && l < k2) ? S[arow * lds + l] : 0.f;
      const float bv = (x2 < n2 && l < k2) ? W2t[(int64_t)l * n2 + x2] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int a1 = mb * 32 + acc_row(r, lane);
      if (a1 < k1 && x2 < n2) T[a1 * ldt + x2] = acc[r];
    }
  }
  __syncthreads();
  // stage 2: out[x1][x2] = sum_a1 W1[x1][a1] T[a1][x2], x1 in [x1b, x1b + 64)
  const float* __restrict__ W1t = a.w1t[f];  // [k1][n1]
  float* out = a.out + ((int64_t)f * k0 + a0) * n1 * n2;
  for (int tile = wave; tile < 2 * nb; tile += 4) {
    const int mb = tile / nb, cb = tile - mb * nb;
    const int x1 = x1b + mb * 32 + li, x2 = cb * 32 + li;
    if (x1b + mb * 32 >= n1) continue;
    f32x16 acc;
    zero16(acc);
    for (int kk = 0; kk < k1; kk += 2) {
      const int l = kk + kh;
      const float av = (x1 < n1 && l < k1) ? W1t[(int64_t)l * n1 + x1] : 0.f;
      const float bv = (x2 < n2 && l < k1) ? T[l * ldt + x2] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
    if (x2 < n2) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int xr = x1b + mb * 32 + acc_row(r, lane);
        if (xr < n1) out[(int64_t)xr * n2 + x2] = acc[r];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_pi_ba(PiBAArgs a) {
  extern __shared__ float smem[];
  const int f = blockIdx.z, a0 = blockIdx.y;
  const int k0 = a.k0, k1 = a.k1, k2 = a.k2, n1 = a.n1, n2 = a.n2;
  const int ldt = n2 + 4;
  float* R = smem;         // [4][1024] partial 32x32 blocks of the waves
  float* T = smem + 4096;  // [a1][x2]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kh = lane >> 5, li = lane & 31;
  const float* __restrict__ in = a.in + ((int64_t)f * k0 + a0) * n1 * n2;
  const float* __restrict__ P1t = a.p1t;  // [n1][k1]
  const float* __restrict__ P2t = a.p2t;  // [n2][k2]
  // stage 1: T[a1][x2] = sum_x1 P1[a1][x1] in[x1][x2]
  const int mb1 = (k1 + 31) / 32, nb = (n2 + 31) / 32;
  for (int tile = wave; tile < mb1 * nb; tile += 4) {
    const int mb = tile / nb, cb = tile - mb * nb;
    const int arow = mb * 32 + li, x2 = cb * 32 + li;
    f32x16 acc;
    zero16(acc);
#pragma unroll 8
    for (int kk = 0; kk < n1; kk += 2) {
      const int l = kk + kh;
      const float av = (arow < k1 && l < n1) ? P1t[(int64_t)l * k1 + arow] : 0.f;
      const float bv = (x2 < n2 && l < n1) ? in[(int64_t)l * n2 + x2] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int a1 = mb * 32 + acc_row(r, lane);
      if (a1 < k1 && x2 < n2) T[a1 * ldt + x2] = acc[r];
    }
  }
  __syncthreads();
  // stage 2: r[a1][a2] = sum_x2 T[a1][x2] P2[a2][x2]; ntile (1, 2 or 4) tiles, 4/ntile waves per tile
  const int mb2 = (k1 + 31) / 32, cb2 = (k2 + 31) / 32, ntile = mb2 * cb2;
  const int wpt = 4 / ntile;  // waves per tile
  const int tile = wave / wpt, part = wave - tile * wpt;
  const int mb = tile / cb2, cb = tile - mb * cb2;
  const int arow = mb * 32 + li, a2 = cb * 32 + li;
  const int seg = ((n2 + 2 * wpt - 1) / (2 * wpt)) * 2;
  const int lb = part * seg, le = min(n2, lb + seg);
  f32x16 acc;
  zero16(acc);
  for (int kk = lb; kk < le; kk += 2) {
    const int l = kk + kh;
    const float av = (arow < k1 && l < le) ? T[arow * ldt + l] : 0.f;
    const float bv = (a2 < k2 && l < le) ? P2t[(int64_t)l * k2 + a2] : 0.f;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) R[wave * 1024 + r * 64 + lane] = acc[r];
  __syncthreads();
  // epilogue: one thread per output coefficient of this (field, a0) slab
  float* dst = a.out[f] + (int64_t)a0 * k1 * k2;
  const float al = a.alpha[f], be = a.beta[f];
  for (int e = tid; e < k1 * k2; e += 256) {
    const int r1 = e / k2, r2 = e - r1 * k2;
    const int tm = r1 >> 5, tc = r2 >> 5, t = tm * cb2 + tc;
    const int rr = r1 & 31, ln = r2 & 31;
    // register index and lane of (rr, ln) in the 32x32 accumulator layout
    const int reg = ((rr >> 3) << 2) + (rr & 3), lanei = ln + 32 * ((rr >> 2) & 1);
    float sum = 0.f;
    for (int w = 0; w < wpt; ++w) sum += R[(t * wpt + w) * 1024 + reg * 64 + lanei];
    dst[e] = be == 0.f ? al * sum : be * dst[e] + al * sum;
  }
}

}  // namespace

bool fused_dft_ok(int n1, int n2, int k1, int k2) {
  const size_t lds_iota = ((size_t)k1 * (k2 + 1) + (size_t)k1 * (n2 + 4)) * sizeof(float);
  const size_t lds_pi = (4096 + (size_t)k1 * (n2 + 4)) * sizeof(float);
  return n1 <= kMaxN && n2 <= kMaxN && k1 <= kMaxK && k2 <= kMaxK && k1 >= 2 && k2 >= 2 && lds_iota <= 65536 &&
         lds_pi <= 65536;
}

void iota_ab(const IotaABArgs& a, int nf, hipStream_t s) {
  const double bytes = 4.0 * nf * ((double)a.k0 * a.k1 * a.k2 + (double)a.k0 * a.n1 * a.n2);
  const double flops = 2.0 * nf * a.k0 * ((double)a.k1 * a.k2 * a.n2 + (double)a.n1 * a.k1 * a.n2);
  dim3 g(ceil_div(a.n1, 64), a.k0, nf);
  const uint32_t sm = (uint32_t)(a.k1 * (a.k2 + 1) + a.k1 * (a.n2 + 4)) * sizeof(float);
  prof::launch("k_iota_ab", bytes, flops, k_iota_ab, g, dim3(256), sm, s, a);
  LDDMM_LAUNCH_CHECK();
}

void pi_ba(const PiBAArgs& a, int nf, hipStream_t s) {
  const double bytes = 4.0 * nf * ((double)a.k0 * a.n1 * a.n2 + (double)a.k0 * a.k1 * a.k2);
  const double flops = 2.0 * nf * a.k0 * ((double)a.k1 * a.n1 * a.n2 + (double)a.k1 * a.n2 * a.k2);
  dim3 g(1, a.k0, nf);
  const uint32_t sm = (uint32_t)(4096 + a.k1 * (a.n2 + 4)) * sizeof(float);
  prof::launch("k_pi_ba", bytes, flops, k_pi_ba, g, dim3(256), sm, s, a);
  LDDMM_LAUNCH_CHECK();
}

}  // namespace lddmm
