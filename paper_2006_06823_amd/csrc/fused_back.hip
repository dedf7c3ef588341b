// Fused grid pass of the image-transport backward sweeps (incremental adjoint,
// Table 1 row 6, and the Hessian term of Section 2.3.1), float.
//
// Given the inner-axis slab T2 = (iota stages on axes 2, 1)(dl~) of the band
// adjoint, one kernel per 32-column block of the (x1, x2) plane
//   1. expands the last axis: e[x0][c] = sum_a0 B0[x0][a0] T2[a0][c]   (e = iota(dl~) on the grid);
//   2. forms the four products p_f = e * {div v, G_0, G_1, G_2} in registers;
//   3. contracts axis 0 of each product: out_f[a0][c] = (1/n0) sum_x0 B0[x0][a0] p_f[x0][c],
//      the first projection stage, feeding each product straight from the matrix-core
//      accumulator registers back in as operand (the contraction order is permuted to
//      match the accumulator layout), partial sums of the waves reduced in LDS.
// e and the products never reach HBM: per step this reads T2 (F/4), div v and G (4F)
// and writes 4 x F/4, instead of writing and re-reading e and the products.
#include "kernels.h"
#include "prof.h"
#include "stage.h"

namespace lddmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

template <int MBO>
__global__ __launch_bounds__(256) void k_back_v1(BackV1Args a) {
  extern __shared__ float smem[];
  const int n0 = a.n0, k0 = a.k0, C = a.C;
  const int ldb = k0 + 1;
  float* B0s = smem;             // [n0][k0 + 1]
  float* red = smem + n0 * ldb;  // [4 waves][MBO][16][64]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kh = lane >> 5, li = lane & 31;
  stage_tile<256, 16>(B0s, ldb, a.B0, k0, n0, k0, n0, k0);
  __syncthreads();
  const int c0 = blockIdx.x * 32, c = c0 + li;
  const bool cok = c < C;
  const int MB = (n0 + 31) / 32;
  f32x16 acc[4][MBO];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int m = 0; m < MBO; ++m)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[f][m][r] = 0.f;
  // 32-bit element offsets (the grid stays below 2^31 nodes) keep one address register per load
  for (int mb = wave; mb < MB; mb += 4) {
    // software pipeline: T2 and the first product field are requested before the expansion,
    // each further field one product ahead of its use
    float fcur[16], fnext[16];
    auto load_field = [&](int f, float* dst) {
      const float* __restrict__ F = f == 0 ? a.divv : a.G + (int64_t)(f - 1) * n0 * C;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int x0 = mb * 32 + acc_row(r, lane);
        dst[r] = (cok && x0 < n0) ? F[x0 * C + c] : 0.f;
      }
    };
    float tv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int l = 2 * q + kh;
      tv[q] = (cok && l < k0) ? a.t2[l * C + c] : 0.f;
    }
    load_field(0, fcur);
    // 1. e for rows x0 in [32 mb, 32 mb + 32)
    f32x16 ev;
#pragma unroll
    for (int r = 0; r < 16; ++r) ev[r] = 0.f;
    const int xr = mb * 32 + li;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int l = 2 * q + kh;
      const float av = (xr < n0 && l < k0) ? B0s[xr * ldb + l] : 0.f;
      ev = __builtin_amdgcn_mfma_f32_32x32x2f32(av, tv[q], ev, 0, 0, 0);
    }
    for (int kk = 32; kk < k0; kk += 2) {  // k0 > 32 (second output tile)
      const int l = kk + kh;
      const float av = (xr < n0 && l < k0) ? B0s[xr * ldb + l] : 0.f;
      const float bv = (cok && l < k0) ? a.t2[l * C + c] : 0.f;
      ev = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, ev, 0, 0, 0);
    }
    // 2-3. products and the axis-0 contraction
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (f < 3) load_field(f + 1, fnext);
      float p[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) p[r] = ev[r] * fcur[r];
#pragma unroll
      for (int m = 0; m < MBO; ++m) {
        const int a0 = m * 32 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int x0 = mb * 32 + 8 * q + i + 4 * kh;
            const float av = (x0 < n0 && a0 < k0) ? B0s[x0 * ldb + a0] : 0.f;
            acc[f][m] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, p[4 * q + i], acc[f][m], 0, 0, 0);
          }
      }
      if (f < 3) {
#pragma unroll
        for (int r = 0; r < 16; ++r) fcur[r] = fnext[r];
      }
    }
  }
  // reduce the waves' partial contractions, one product at a time
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MBO; ++m)
#pragma unroll
      for (int r = 0; r < 16; ++r) red[((wave * MBO + m) * 16 + r) * 64 + lane] = acc[f][m][r];
    __syncthreads();
    for (int e = tid; e < MBO * 1024; e += 256) {
      const int ln = e & 63, r = (e >> 6) & 15, m = e >> 10;
      float sum = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) sum += red[((w * MBO + m) * 16 + r) * 64 + ln];
      const int a0 = m * 32 + acc_row(r, ln), cc = c0 + (ln & 31);
      if (a0 < k0 && cc < C) a.out[((int64_t)f * k0 + a0) * C + cc] = sum * a.inv_n0;
    }
  }
}

}  // namespace

bool back_v1_ok(int n0, int k0) { return k0 <= 64 && (size_t)n0 * (k0 + 1) * 4 + 4 * 2 * 1024 * 4 <= 65536; }

void back_v1(const BackV1Args& a, hipStream_t s) {
  const double bytes = 4.0 * ((double)a.k0 * a.C + 4.0 * a.n0 * a.C + 4.0 * a.k0 * a.C);
  const double flops = 2.0 * (double)a.n0 * a.k0 * a.C * 5.0;
  const int mbo = (a.k0 + 31) / 32;
  const uint32_t sm = (uint32_t)((size_t)a.n0 * (a.k0 + 1) + 4 * mbo * 1024) * sizeof(float);
  dim3 g(ceil_div(a.C, 32));
  if (mbo == 1)
    prof::launch("k_back_v1<1>", bytes, flops, k_back_v1<1>, g, dim3(256), sm, s, a);
  else
    prof::launch("k_back_v1<2>", bytes, flops, k_back_v1<2>, g, dim3(256), sm, s, a);
  LDDMM_LAUNCH_CHECK();
}

}  // namespace lddmm
