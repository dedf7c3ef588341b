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
#include "stage.h"

namespace lddmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ void zero16(f32x16& a) {
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = 0.f;
}

constexpr int kMaxN = 192, kMaxK = 64;
constexpr int kRows = 32;  // grid rows of axis 1 per block

// LDS floats of k_iota_ab for an xc-column block, with and without the staged axis-2 matrix
__host__ __device__ inline int iota_lds(int k1, int k2, int xc, bool stage_w2) {
  return k1 * (k2 + 1) + k1 * (xc + 4) + k1 * kRows + (stage_w2 ? k2 * xc : 0);
}
// LDS floats of k_pi_ba: the slab rows (aliased by the wave partials after stage A), U, and the
// staged projection operands (P2 whole, the block's 32 rows of P1) when they fit
__host__ __device__ inline int pi_lds(int k1, int k2, int n2, bool stage_p) {
  const int in_r = kRows * (n2 + 1) > 4096 ? kRows * (n2 + 1) : 4096;
  return in_r + kRows * (k2 + 1) + (stage_p ? n2 * k2 + kRows * k1 : 0);
}

// grid (ceil(n1 / 32) * ceil(n2 / xc), k0, nf): each block expands one (field, a0) slab for 32 rows
// of x1 and xc columns of x2 (xc = all of n2 unless the slabs alone give too few blocks)
template <bool STAGE_W2>
__global__ __launch_bounds__(256) void k_iota_ab(IotaABArgs a, int xc) {
  extern __shared__ float smem[];
  const int f = blockIdx.z, a0 = blockIdx.y;
  const int k0 = a.k0, k1 = a.k1, k2 = a.k2, n1 = a.n1, n2 = a.n2;
  const int nxb = (n1 + kRows - 1) / kRows;
  const int x1b = (blockIdx.x % nxb) * kRows, x2b = (blockIdx.x / nxb) * xc;
  const int ncol = min(xc, n2 - x2b);
  const int lds = k2 + 1, ldt = xc + 4;
  float* S = smem;               // [a1][a2]
  float* T = S + k1 * lds;       // [a1][x2 - x2b]
  float* W1s = T + k1 * ldt;     // [a1][32 rows of x1]
  float* W2s = W1s + k1 * kRows;  // [a2][x2 - x2b] (when staged)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kh = lane >> 5, li = lane & 31;
  const float* __restrict__ W2t = a.w2t[f];  // [k2][n2]
  const float* __restrict__ W1t = a.w1t[f];  // [k1][n1]
  // prologue: slab = x + alpha y, and the matrix operands, loads batched ahead of the stores
  {
    const int64_t off = (int64_t)a0 * k1 * k2;
    const float* x = a.x[f] + off;
    const float* y = a.y[f] ? a.y[f] + off : nullptr;
    const float al = a.alpha[f];
    constexpr int U = 8;
    TileWalk w(256, tid, k2, k2, lds);
    while (w.r < k1) {
      const TileWalk w0 = w;
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = 0.f;
        if (w.r < k1) v[u] = y ? x[w.o1] + al * y[w.o1] : x[w.o1];
        w.next();
      }
      w = w0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (w.r < k1) S[w.o2] = v[u];
        w.next();
      }
    }
    stage_tile<256, 8>(W1s, kRows, W1t + x1b, n1, k1, kRows, k1, n1 - x1b);
    if (STAGE_W2) stage_tile<256, 16>(W2s, xc, W2t + x2b, n2, k2, xc, k2, ncol);
  }
  __syncthreads();
  const float* W2 = STAGE_W2 ? W2s : W2t + x2b;
  const int ld2 = STAGE_W2 ? xc : n2;
  // stage 1: T[a1][x2] = sum_a2 S[a1][a2] W2[x2][a2] over this block's columns
  const int mb1 = (k1 + 31) / 32, nb = (ncol + 31) / 32;
  for (int tile = wave; tile < mb1 * nb; tile += 4) {
    const int mb = tile / nb, cb = tile - mb * nb;
    f32x16 acc;
    zero16(acc);
    const int arow = mb * 32 + li, xl = cb * 32 + li;
    if constexpr (STAGE_W2) {
#pragma unroll 4
      for (int kk = 0; kk < k2; kk += 2) {
        const int l = kk + kh;
        const float av = (arow < k1 && l < k2) ? S[arow * lds + l] : 0.f;
        const float bv = (xl < ncol && l < k2) ? W2[l * ld2 + xl] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
    } else {
      // W2 read from global memory: every k-step's operand requested before the first product
      // (k2 <= 64: at most 32 steps; 32-bit offsets, out-of-range entries read a valid element)
      float bq[kMaxK / 2];
#pragma unroll
      for (int j = 0; j < kMaxK / 2; ++j) {
        const int l = 2 * j + kh;
        const bool ok = xl < ncol && l < k2;
        const float t = W2[ok ? l * ld2 + xl : 0];
        bq[j] = ok ? t : 0.f;
      }
#pragma unroll
      for (int j = 0; j < kMaxK / 2; ++j) {
        if (2 * j >= k2) break;
        const int l = 2 * j + kh;
        const float av = (arow < k1 && l < k2) ? S[arow * lds + l] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bq[j], acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int a1 = mb * 32 + acc_row(r, lane);
      if (a1 < k1 && xl < ncol) T[a1 * ldt + xl] = acc[r];
    }
  }
  __syncthreads();
  // stage 2: out[x1][x2] = sum_a1 W1[x1][a1] T[a1][x2], x1 in [x1b, x1b + 32)
  float* out = a.out + ((int64_t)f * k0 + a0) * n1 * n2;
  for (int cb = wave; cb < nb; cb += 4) {
    const int xl = cb * 32 + li;
    f32x16 acc;
    zero16(acc);
#pragma unroll 4
    for (int kk = 0; kk < k1; kk += 2) {
      const int l = kk + kh;
      const float av = l < k1 ? W1s[l * kRows + li] : 0.f;
      const float bv = (xl < ncol && l < k1) ? T[l * ldt + xl] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
    if (xl < ncol) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int xr = x1b + acc_row(r, lane);
        if (xr < n1) out[(int64_t)xr * n2 + x2b + xl] = acc[r];
      }
    }
  }
}

// grid (nsplit = ceil(n1 / 32), <= k0, nf): each block projects 32 rows of x1 of the (field, a0)
// slabs it walks to partial band blocks in the workspace; k_pi_fin then sums the partials of every slab
// in split order (deterministic) and applies the epilogue.  (A last-block-done reduction inside
// this kernel would need a device-scope release per block, which writes back the XCD's L2.)
template <bool STAGE_P, bool WALK>
__global__ __launch_bounds__(256) void k_pi_ba(PiBAArgs a) {
  extern __shared__ float smem[];
  const int sp = blockIdx.x, f = blockIdx.z, nsplit = gridDim.x;
  const int k0 = a.k0, k1 = a.k1, k2 = a.k2, n1 = a.n1, n2 = a.n2;
  const int x1b = sp * kRows;
  const int ldi = n2 + 1, ldu = k2 + 1;
  const int in_r = kRows * ldi > 4096 ? kRows * ldi : 4096;
  float* In = smem;              // [32][n2 + 1] rows x1b.. of the slab
  float* R = smem;               // [4][1024] partial accumulators of the waves (after stage A reads In)
  float* U = smem + in_r;        // [32][k2 + 1]
  float* P2s = U + kRows * ldu;  // [n2][k2] (staged)
  float* P1s = P2s + n2 * k2;    // [32 rows of x1][k1] (staged)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kh = lane >> 5, li = lane & 31;
  const int vr = n1 - x1b < kRows ? n1 - x1b : kRows;
  const float* P2t = STAGE_P ? P2s : a.p2t;  // [n2][k2]
  const int cb2 = (k2 + 31) / 32, wpt = 4 / cb2;
  const int mb2 = (k1 + 31) / 32;
  // WALK: the block walks the slabs a0 = blockIdx.y + j gridDim.y with the operands staged once;
  // otherwise it takes the one slab a0 = blockIdx.y (a separate instance: the loop costs registers)
  const int nwalk = WALK ? (k0 - (int)blockIdx.y + (int)gridDim.y - 1) / (int)gridDim.y : 1;
  for (int j = 0; j < nwalk; ++j) {
    const int a0 = blockIdx.y + j * gridDim.y;
    const int slab = f * k0 + a0;
    const float* __restrict__ in = a.in + (int64_t)slab * n1 * n2;
    if (WALK && j > 0) __syncthreads();  // the previous slab's reads of U are done
    stage_tile<256, 16>(In, ldi, in + (int64_t)x1b * n2, n2, kRows, n2, vr, n2);
    if (STAGE_P && j == 0) {
      stage_tile<256, 16>(P2s, k2, a.p2t, k2, n2, k2, n2, k2);
      stage_tile<256, 4>(P1s, k1, a.p1t + (int64_t)x1b * k1, k1, kRows, k1, vr, k1);
    }
    __syncthreads();
    // stage A: U[x][a2] = sum_x2 In[x][x2] P2[a2][x2]; cb2 column tiles, 4 / cb2 waves split x2
    {
      const int tile = wave / wpt, part = wave - tile * wpt;
      const int a2 = tile * 32 + li;
      const int seg = ((n2 + 2 * wpt - 1) / (2 * wpt)) * 2;
      const int lb = part * seg, le = min(n2, lb + seg);
      f32x16 acc;
      zero16(acc);
      if constexpr (STAGE_P) {
#pragma unroll 4
        for (int kk = lb; kk < le; kk += 2) {
          const int l = kk + kh;
          const float av = l < le ? In[li * ldi + l] : 0.f;
          const float bv = (a2 < k2 && l < le) ? P2t[l * k2 + a2] : 0.f;
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
      } else {
        // P2 from global memory: the operands of up to kPreP k-steps requested at a time, before
        // their products (32-bit offsets; out-of-range entries read a valid element and are zeroed)
        constexpr int kPreP = 16;
        for (int kb = lb; kb < le; kb += 2 * kPreP) {
          float bq[kPreP];
#pragma unroll
          for (int j = 0; j < kPreP; ++j) {
            const int l = kb + 2 * j + kh;
            const bool ok = a2 < k2 && l < le;
            const float t = P2t[ok ? l * k2 + a2 : 0];
            bq[j] = ok ? t : 0.f;
          }
#pragma unroll
          for (int j = 0; j < kPreP; ++j) {
            const int l = kb + 2 * j + kh;
            if (kb + 2 * j >= le) break;
            const float av = l < le ? In[li * ldi + l] : 0.f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bq[j], acc, 0, 0, 0);
          }
        }
      }
      __syncthreads();  // every wave is done reading In before R overwrites it
#pragma unroll
      for (int r = 0; r < 16; ++r) R[wave * 1024 + r * 64 + lane] = acc[r];
    }
    __syncthreads();
    for (TileWalk e(256, tid, k2, k2, ldu); e.r < kRows; e.next()) {
      const int x = e.r, c = e.c;
      const int t = c >> 5, reg = ((x >> 3) << 2) + (x & 3), lanei = (c & 31) + 32 * ((x >> 2) & 1);
      float sum = 0.f;
      for (int w = 0; w < wpt; ++w) sum += R[(t * wpt + w) * 1024 + reg * 64 + lanei];
      U[e.o2] = sum;
    }
    __syncthreads();
    // stage B: partial r[a1][a2] = sum_{x < 32} P1[a1][x1b + x] U[x][a2], one wave per 32x32 tile
    float* part = a.part + ((int64_t)slab * nsplit + sp) * k1 * k2;
    if (wave < mb2 * cb2) {
      const int mb = wave / cb2, cb = wave - mb * cb2;
      const int a1 = mb * 32 + li, a2 = cb * 32 + li;
      f32x16 acc;
      zero16(acc);
      if constexpr (STAGE_P) {
#pragma unroll 4
        for (int kk = 0; kk < kRows; kk += 2) {
          const int l = kk + kh;
          const float av = a1 < k1 ? P1s[l * k1 + a1] : 0.f;
          const float bv = a2 < k2 ? U[l * ldu + a2] : 0.f;
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
      } else {
        // P1 rows from global memory, all 16 k-steps' operands requested before the first product
        float aq[kRows / 2];
#pragma unroll
        for (int j = 0; j < kRows / 2; ++j) {
          const int l = 2 * j + kh;
          const bool ok = a1 < k1 && x1b + l < n1;
          const float t = a.p1t[ok ? (x1b + l) * k1 + a1 : 0];
          aq[j] = ok ? t : 0.f;
        }
#pragma unroll
        for (int j = 0; j < kRows / 2; ++j) {
          const int l = 2 * j + kh;
          const float bv = a2 < k2 ? U[l * ldu + a2] : 0.f;
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(aq[j], bv, acc, 0, 0, 0);
        }
      }
      if (a2 < k2) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = mb * 32 + acc_row(r, lane);
          if (row < k1) part[row * k2 + a2] = acc[r];
        }
      }
    }
  }  // slabs
}

// out[f][a0][:] = beta out + alpha * sum_q part[f][a0][q][:], one thread per band coefficient
__global__ __launch_bounds__(256) void k_pi_fin(PiBAArgs a, int nsplit) {
  const int kk = a.k1 * a.k2;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kk) return;
  const int a0 = blockIdx.y, f = blockIdx.z;
  const int slab = f * a.k0 + a0;
  const float* p0 = a.part + (int64_t)slab * nsplit * kk + e;
  float sum = 0.f;
  for (int q = 0; q < nsplit; ++q) sum += p0[(int64_t)q * kk];
  float* dst = a.out[f] + (int64_t)a0 * kk + e;
  const float al = a.alpha[f], be = a.beta[f];
  *dst = be == 0.f ? al * sum : be * *dst + al * sum;
}

}  // namespace

bool fused_dft_ok(int n1, int n2, int k1, int k2) {
  return n1 <= kMaxN && n2 <= kMaxN && k1 <= kMaxK && k2 <= kMaxK && k1 >= 2 && k2 >= 2 &&
         (size_t)iota_lds(k1, k2, ceil_div(n2, 32) * 32, false) * sizeof(float) <= 65536 &&
         (size_t)pi_lds(k1, k2, n2, false) * sizeof(float) <= 65536;
}

int pi_ba_splits(int n1) { return ceil_div(n1, kRows); }

void iota_ab(const IotaABArgs& a, int nf, hipStream_t s) {
  const double bytes = 4.0 * nf * ((double)a.k0 * a.k1 * a.k2 + (double)a.k0 * a.n1 * a.n2);
  const double flops = 2.0 * nf * a.k0 * ((double)a.k1 * a.k2 * a.n2 + (double)a.n1 * a.k1 * a.n2);
  // whole rows while the slabs give a block per CU; otherwise 64-column blocks
  const int nxb = ceil_div(a.n1, kRows);
  const int full = ceil_div(a.n2, 32) * 32;
  const int xc = (int64_t)nxb * a.k0 * nf >= 256 || full <= 64 ? full : 64;
  dim3 g(nxb * ceil_div(a.n2, xc), a.k0, nf);
  const bool stage = (size_t)iota_lds(a.k1, a.k2, xc, true) * sizeof(float) <= 65536;
  const uint32_t sm = (uint32_t)iota_lds(a.k1, a.k2, xc, stage) * sizeof(float);
  if (stage)
    prof::launch("k_iota_ab", bytes, flops, k_iota_ab<true>, g, dim3(256), sm, s, a, xc);
  else
    prof::launch("k_iota_ab", bytes, flops, k_iota_ab<false>, g, dim3(256), sm, s, a, xc);
  LDDMM_LAUNCH_CHECK();
}

void pi_ba(const PiBAArgs& a, int nf, hipStream_t s) {
  const double bytes = 4.0 * nf * ((double)a.k0 * a.n1 * a.n2 + (double)a.k0 * a.k1 * a.k2);
  const double flops = 2.0 * nf * a.k0 * ((double)a.k2 * a.n1 * a.n2 + (double)a.k1 * a.n1 * a.k2);
  if (!a.part) throw ArgError("pi_ba needs its partial-sum workspace");
  const int nsplit = pi_ba_splits(a.n1);
  const bool stage = (size_t)pi_lds(a.k1, a.k2, a.n2, true) * sizeof(float) <= 65536;
  const uint32_t sm = (uint32_t)pi_lds(a.k1, a.k2, a.n2, stage) * sizeof(float);
  // staged operands: no more workgroups than the CUs hold at once (160 KB of LDS each; the
  // registers allow 4), every one walking the same number of slabs, since a second, partial
  // round would stage the operands again
  const int per_cu = std::max(1, std::min(4, (int)(163840 / sm)));
  const int slots = std::max(1, 256 * per_cu / (nsplit * nf));
  const int walk = stage ? ceil_div(a.k0, std::min(a.k0, slots)) : 1;
  dim3 g(nsplit, ceil_div(a.k0, walk), nf);
  if (walk > 1)
    prof::launch("k_pi_ba", bytes, flops, k_pi_ba<true, true>, g, dim3(256), sm, s, a);
  else if (stage)
    prof::launch("k_pi_ba", bytes, flops, k_pi_ba<true, false>, g, dim3(256), sm, s, a);
  else
    prof::launch("k_pi_ba", bytes, flops, k_pi_ba<false, false>, g, dim3(256), sm, s, a);
  LDDMM_LAUNCH_CHECK();
  dim3 gf(ceil_div(a.k1 * a.k2, 256), a.k0, nf);
  prof::launch("k_pi_fin", 4.0 * nf * a.k0 * a.k1 * a.k2 * (nsplit + 2.0), 0.0, k_pi_fin, gf, dim3(256), 0, s, a,
               nsplit);
  LDDMM_LAUNCH_CHECK();
}

}  // namespace lddmm
