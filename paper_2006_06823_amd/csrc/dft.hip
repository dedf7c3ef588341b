// Separable truncated DFT contractions (iota / pi of Section 2.2) on gfx950.
//
// A 3D truncated transform is three one-axis contractions with small dense
// per-axis basis matrices (<= 192 x 48).  Two kernel shapes cover all stages:
//   left : out[b][m][c] = sum_l W[m][l] in[b][l][c]   (contract a non-last axis;
//          rows l of the input are contiguous in c, so loads are coalesced)
//   right: out[r][m]    = sum_l in[r][l] W[m][l]      (contract the last axis)
// In float the products run on the matrix cores (v_mfma_f32_32x32x2f32: each
// wave owns a 32 x 32 output block); in double the same tiling runs on the
// vector FMA units.  Tiles of W and of the input are staged through LDS.
#include "kernels.h"
#include "prof.h"
#include "stage.h"
#include "tune.h"

#include <algorithm>
#include <string>
#include <type_traits>

namespace lddmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int LC = 32;  // contraction chunk staged in LDS

// Row (within the wave's 32 x 32 block) held by accumulator register r of a lane,
// for the 32x32 output layout of the matrix-core instruction.
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

template <typename T>
struct Acc16 {
  T v[16];
};

// One LC-deep chunk of a 32x32 block product: acc[i][j] += sum_k A[i][k] B[k][j],
// A read as As[(arow0 + i) * lda + k], B as Bs[k * ldb + bcol0 + j].
__device__ __forceinline__ void chunk_mma(f32x16& acc, const float* As, int lda, const float* Bs, int ldb,
                                          int lane) {
  const int i = lane & 31, kh = lane >> 5;
#pragma unroll
  for (int kk = 0; kk < LC; kk += 2) {
    const float a = As[i * lda + kk + kh];
    const float b = Bs[(kk + kh) * ldb + i];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
}

__device__ __forceinline__ void chunk_mma(Acc16<double>& acc, const double* As, int lda, const double* Bs,
                                          int ldb, int lane) {
  const int j = lane & 31;
#pragma unroll 4
  for (int kk = 0; kk < LC; ++kk) {
    const double b = Bs[kk * ldb + j];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc.v[r] += As[acc_row(r, lane) * lda + kk] * b;
  }
}

template <typename T>
struct AccOf;
template <>
struct AccOf<float> {
  using type = f32x16;
  static __device__ __forceinline__ float get(const f32x16& a, int r) { return a[r]; }
  static __device__ __forceinline__ void zero(f32x16& a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = 0.f;
  }
};
template <>
struct AccOf<double> {
  using type = Acc16<double>;
  static __device__ __forceinline__ double get(const Acc16<double>& a, int r) { return a.v[r]; }
  static __device__ __forceinline__ void zero(Acc16<double>& a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a.v[r] = 0.0;
  }
};

// out[b][m][c] = sum_l W[m][l] in[b][l][c]; block tile (32 WM) x (32 WC), one wave per 32x32 block.
template <typename T, int WM, int WC>
__global__ __launch_bounds__(64 * WM * WC) void dft_left_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                                FieldMats<T> mats, int bpf, int M, int L,
                                                                int C, int64_t sIb, int64_t sOb) {
  constexpr int TM = 32 * WM, TC = 32 * WC, NT = 64 * WM * WC;
  constexpr int LDA = LC + 1;
  __shared__ T Ws[TM * LDA];
  __shared__ T Xs[LC * TC];
  const int b = blockIdx.z;
  const T* __restrict__ W = mats.w[b / bpf];
  const int m0 = blockIdx.y * TM, c0 = blockIdx.x * TC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WC, wc = wave % WC;
  in += b * sIb;
  out += b * sOb;
  typename AccOf<T>::type acc;
  AccOf<T>::zero(acc);
  for (int l0 = 0; l0 < L; l0 += LC) {
    for (int e = tid; e < TM * LC; e += NT) {
      const int mm = e / LC, ll = e - mm * LC;
      const int m = m0 + mm, l = l0 + ll;
      Ws[mm * LDA + ll] = (m < M && l < L) ? W[(int64_t)m * L + l] : T(0);
    }
    for (int e = tid; e < LC * TC; e += NT) {
      const int ll = e / TC, cc = e - ll * TC;
      const int l = l0 + ll, c = c0 + cc;
      Xs[ll * TC + cc] = (l < L && c < C) ? in[(int64_t)l * C + c] : T(0);
    }
    __syncthreads();
    chunk_mma(acc, Ws + wm * 32 * LDA, LDA, Xs + wc * 32, TC, lane);
    __syncthreads();
  }
  const int c = c0 + wc * 32 + (lane & 31);
  if (c < C) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = m0 + wm * 32 + acc_row(r, lane);
      if (m < M) out[(int64_t)m * C + c] = AccOf<T>::get(acc, r);
    }
  }
}

// out[f][r][m] = sum_l in[f][r][l] W_f[m][l]; block tile rows (32 WR) x outputs (32 WM).
template <typename T, int WR, int WM>
__global__ __launch_bounds__(64 * WR * WM) void dft_right_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                                 FieldMats<T> mats, int R, int L, int Mo) {
  constexpr int TR = 32 * WR, TMo = 32 * WM, NT = 64 * WR * WM;
  constexpr int LDA = LC + 1;
  __shared__ T Xs[TR * LDA];
  __shared__ T Ws[LC * TMo];
  const int f = blockIdx.z;
  const T* __restrict__ W = mats.w[f];
  in += (int64_t)f * R * L;
  out += (int64_t)f * R * Mo;
  const int r0 = blockIdx.y * TR, m0 = blockIdx.x * TMo;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WM, wm = wave % WM;
  typename AccOf<T>::type acc;
  AccOf<T>::zero(acc);
  for (int l0 = 0; l0 < L; l0 += LC) {
    for (int e = tid; e < TR * LC; e += NT) {
      const int rr = e / LC, ll = e - rr * LC;
      const int r = r0 + rr, l = l0 + ll;
      Xs[rr * LDA + ll] = (r < R && l < L) ? in[(int64_t)r * L + l] : T(0);
    }
    // W staged transposed, [l][m], so the B operand is read contiguously
    for (int e = tid; e < TMo * LC; e += NT) {
      const int mm = e / LC, ll = e - mm * LC;
      const int m = m0 + mm, l = l0 + ll;
      Ws[ll * TMo + mm] = (m < Mo && l < L) ? W[(int64_t)m * L + l] : T(0);
    }
    __syncthreads();
    chunk_mma(acc, Xs + wr * 32 * LDA, LDA, Ws + wm * 32, TMo, lane);
    __syncthreads();
  }
  const int m = m0 + wm * 32 + (lane & 31);
  if (m < Mo) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = r0 + wr * 32 + acc_row(q, lane);
      if (r < R) out[(int64_t)r * Mo + m] = AccOf<T>::get(acc, q);
    }
  }
}

// ---- streaming float kernels for the large stages ----------------------------------
// The B operand (input rows, contiguous in c) is read straight from global memory
// into the matrix-core operand registers, 32 consecutive floats per half-wave, so
// the input streams through once without LDS staging; only W sits in LDS.
//
// contract mode (M <= 64, L large): the four waves of a block share 32 columns and
// split the contraction range; partial 32x32 blocks are summed through LDS.
// k-steps of a wave's range whose input loads are issued up front (covers N0 <= 128 / 192)
template <int MB>
constexpr int pre_steps() { return MB == 1 ? 16 : 24; }
template <int MB, int NCT>
__global__ __launch_bounds__(256) void dft_left_contract(const float* __restrict__ in, float* __restrict__ out,
                                                         FieldMats<float> mats, int bpf, int M, int L, int C,
                                                         int64_t sIb, int64_t sOb, int separate_red) {
  extern __shared__ float smem[];
  const int ldw = L + 1;
  float* Ws = smem;                                          // [32 MB][L + 1]
  float* red = separate_red ? smem + 32 * MB * ldw : smem;   // [4][16][64]
  const int b = blockIdx.z;
  const float* __restrict__ W = mats.w[b / bpf];
  in += b * sIb;
  out += b * sOb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // this wave's contraction range (even length, so each k-step pairs two rows)
  const int seg = ((L + 7) / 8) * 2;
  const int lb = wave * seg, le = min(L, lb + seg);
  const int kh = lane >> 5;
  const int ncb = (C + 32 * NCT - 1) / (32 * NCT);
  // without a separate reduction buffer the W tile is reloaded per column block
  for (int cb = blockIdx.x; cb < ncb; cb += gridDim.x) {
    const int c0 = cb * 32 * NCT;
    // a wave range of up to 2 kPre rows: all of its input loads are issued before the W tile is
    // staged, so the block waits one memory latency instead of one per unrolled group of steps
    // (one 32-row output tile only: with two the registers would halve the occupancy)
    constexpr int kPre = pre_steps<MB>();
    constexpr bool kPrefetch = true;
    const bool pre = kPrefetch && seg <= 2 * kPre;
    float bq[kPrefetch ? kPre : 1][NCT];
    if constexpr (kPrefetch) {
      if (pre) {
        // 32-bit offsets from the uniform base (one address register per load, not two)
        const int lrow = lb + kh;
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
          const int l = lrow + 2 * i;
#pragma unroll
          for (int t = 0; t < NCT; ++t) {
            const int c = c0 + t * 32 + (lane & 31);
            bq[i][t] = (c < C && l < le) ? in[l * C + c] : 0.f;
          }
        }
      }
    }
    if (cb == blockIdx.x || !separate_red) {
      __syncthreads();
      stage_tile<256, 16>(Ws, ldw, W, L, 32 * MB, L, M, L);
      __syncthreads();
    }
    f32x16 acc[MB][NCT];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int t = 0; t < NCT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[mb][t][r] = 0.f;
    if (pre) {
      if constexpr (kPrefetch) {
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
          const int l = lb + 2 * i + kh;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            const float av = l < le ? Ws[(mb * 32 + (lane & 31)) * ldw + l] : 0.f;
#pragma unroll
            for (int t = 0; t < NCT; ++t)
              acc[mb][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bq[i][t], acc[mb][t], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll 4
      for (int kk = lb; kk < le; kk += 2) {
        const int l = kk + kh;
        float bv[NCT];
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
          const int c = c0 + t * 32 + (lane & 31);
          bv[t] = (c < C && l < le) ? in[(int64_t)l * C + c] : 0.f;
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const float av = l < le ? Ws[(mb * 32 + (lane & 31)) * ldw + l] : 0.f;
#pragma unroll
          for (int t = 0; t < NCT; ++t)
            acc[mb][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[t], acc[mb][t], 0, 0, 0);
        }
      }
    }
    // reduce the waves' partial sums one 32 x 32 tile at a time through a 16 KB buffer
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        __syncthreads();  // W reads done (aliased case) / previous reduction consumed
#pragma unroll
        for (int r = 0; r < 16; ++r) red[(wave * 16 + r) * 64 + lane] = acc[mb][t][r];
        __syncthreads();
        for (int e = tid; e < 16 * 64; e += 256) {
          const int ln = e & 63, r = e >> 6;
          const float sum = red[r * 64 + ln] + red[(16 + r) * 64 + ln] + red[(32 + r) * 64 + ln] +
                            red[(48 + r) * 64 + ln];
          const int m = mb * 32 + acc_row(r, ln), cc = c0 + t * 32 + (ln & 31);
          if (m < M && cc < C) out[(int64_t)m * C + cc] = sum;
        }
      }
  }
}

// expand mode (L <= 64): a block owns a 128-row x 64-column output tile.  The input rows of
// its 64 columns are staged in LDS with one coalesced burst (float4 when aligned), each wave
// owns one 32-row block and both 32-column halves; the W tile stays in LDS while the block
// walks several column tiles.
constexpr int kExpCols = 64, kExpLdb = kExpCols + 4;
__global__ __launch_bounds__(256) void dft_left_expand(const float* __restrict__ in, float* __restrict__ out,
                                                       FieldMats<float> mats, int bpf, int M, int L, int C,
                                                       int64_t sIb, int64_t sOb, int vec) {
  extern __shared__ float smem[];
  const int ldw = L + 1;
  float* Ws = smem;              // [128][L + 1]
  float* Bs = smem + 128 * ldw;  // [L][68]
  const int b = blockIdx.z;
  const float* __restrict__ W = mats.w[b / bpf];
  in += b * sIb;
  out += b * sOb;
  const int m0 = blockIdx.y * 128;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 31;
  stage_tile<256, 16>(Ws, ldw, W + (int64_t)m0 * L, L, 128, L, M - m0, L);
  const int mw = m0 + wave * 32;
  const int kh = lane >> 5;
  const float* Wr = Ws + (wave * 32 + li) * ldw;
  const int ncb = (C + kExpCols - 1) / kExpCols;
  for (int cb = blockIdx.x; cb < ncb; cb += gridDim.x) {
    const int c0 = cb * kExpCols;
    __syncthreads();  // W tile loaded; previous tile's reads of Bs done
    if (vec) {
      for (int e = tid; e < L * (kExpCols / 4); e += 256) {
        const int l = e >> 4, j = (e & 15) * 4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c0 + j < C) v = *reinterpret_cast<const float4*>(in + (int64_t)l * C + c0 + j);
        *reinterpret_cast<float4*>(Bs + l * kExpLdb + j) = v;
      }
    } else {
      for (int e = tid; e < L * kExpCols; e += 256) {
        const int l = e >> 6, j = e & 63;
        Bs[l * kExpLdb + j] = (c0 + j < C) ? in[(int64_t)l * C + c0 + j] : 0.f;
      }
    }
    __syncthreads();
    if (mw < M) {
      f32x16 acc0, acc1;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0.f;
#pragma unroll 4
      for (int kk = 0; kk < L; kk += 2) {
        const int l = kk + kh;
        const bool ok = l < L;
        const float av = ok ? Wr[l] : 0.f;
        const float b0 = ok ? Bs[l * kExpLdb + li] : 0.f;
        const float b1 = ok ? Bs[l * kExpLdb + 32 + li] : 0.f;
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b1, acc1, 0, 0, 0);
      }
      const int c = c0 + li;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mw + acc_row(r, lane);
        if (m < M) {
          if (c < C) out[(int64_t)m * C + c] = acc0[r];
          if (c + 32 < C) out[(int64_t)m * C + c + 32] = acc1[r];
        }
      }
    }
  }
}

// ---- split-bf16 variants (precision LDDMM_BL_BF16_DFT) --------------------------------
// Every float operand x is split into bf16 hi = rn(x) and lo = rn(x - hi); a product
// is formed as hi*hi + hi*lo + lo*hi on the bf16 matrix cores (v_mfma_f32_32x32x16_bf16,
// 16-deep contraction per instruction) with float accumulation, which keeps about 16
// significant bits per operand at a third of the instruction count of the float path.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rn(float x) {
  const unsigned int b = __float_as_uint(x);
  return static_cast<unsigned short>((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ void split8(const float v[8], bf16x8& hi, bf16x8& lo) {
  u16x8 h, l;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const unsigned short hb = bf16_rn(v[j]);
    h[j] = hb;
    l[j] = bf16_rn(v[j] - __uint_as_float(static_cast<unsigned int>(hb) << 16));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

__device__ __forceinline__ f32x16 mma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh, const bf16x8& bl,
                                       f32x16 acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
}

template <int MB>
__global__ __launch_bounds__(256) void dft_left_contract_bf16(const float* __restrict__ in, float* __restrict__ out,
                                                              FieldMats<float> mats, int bpf, int M, int L, int C,
                                                              int64_t sIb, int64_t sOb) {
  extern __shared__ float smem[];
  const int ldw = L + 1;
  float* Ws = smem;
  float* red = smem;
  const int b = blockIdx.z;
  const float* __restrict__ W = mats.w[b / bpf];
  in += b * sIb;
  out += b * sOb;
  const int c0 = blockIdx.x * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int seg = ((L + 63) / 64) * 16;  // per-wave range, a multiple of 16 (at most 48: L <= 192)
  const int lb = wave * seg, le = min(L, lb + seg);
  const int c = c0 + (lane & 31);
  const bool cok = c < C;
  const int kh = lane >> 5;
  // the wave's input rows are all requested before the W tile is staged (32-bit offsets from the
  // uniform base; rows past the range read a valid element and are zeroed)
  float bq[3][8];
#pragma unroll
  for (int it = 0; it < 3; ++it)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int l = lb + 16 * it + 8 * kh + j;
      const bool ok = cok && l < le;
      const float t = in[ok ? l * C + c : 0];
      bq[it][j] = ok ? t : 0.f;
    }
  stage_tile<256, 16>(Ws, ldw, W, L, 32 * MB, L, M, L);
  __syncthreads();
  f32x16 acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[mb][r] = 0.f;
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    const int kk = lb + 16 * it;
    if (kk >= le) break;
    float* bv = bq[it];
    bf16x8 bh, bl;
    split8(bv, bh, bl);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      float av[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int l = kk + 8 * kh + j;
        av[j] = l < le ? Ws[(mb * 32 + (lane & 31)) * ldw + l] : 0.f;
      }
      bf16x8 ah, al;
      split8(av, ah, al);
      acc[mb] = mma3(ah, al, bh, bl, acc[mb]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) red[((wave * MB + mb) * 16 + r) * 64 + lane] = acc[mb][r];
  __syncthreads();
  for (int e = tid; e < MB * 16 * 64; e += 256) {
    const int ln = e & 63, r = (e >> 6) & 15, mb = e >> 10;
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) sum += red[((w * MB + mb) * 16 + r) * 64 + ln];
    const int m = mb * 32 + acc_row(r, ln), cc = c0 + (ln & 31);
    if (m < M && cc < C) out[(int64_t)m * C + cc] = sum;
  }
}

__global__ __launch_bounds__(256) void dft_left_expand_bf16(const float* __restrict__ in, float* __restrict__ out,
                                                            FieldMats<float> mats, int bpf, int M, int L, int C,
                                                            int64_t sIb, int64_t sOb) {
  extern __shared__ float smem[];
  const int ldw = L + 1;
  float* Ws = smem;  // [128][L + 1]
  const int b = blockIdx.z;
  const float* __restrict__ W = mats.w[b / bpf];
  in += b * sIb;
  out += b * sOb;
  const int m0 = blockIdx.y * 128;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kh = lane >> 5;
  const int ncb = (C + 31) / 32;
  // the block walks the 32-column tiles cb = blockIdx.x + j gridDim.x with its W tile staged once;
  // a tile's input rows (L <= 64) are all requested before its products (for the first tile,
  // before the W tile is staged; 32-bit offsets, entries outside the input read a valid element
  // and are zeroed)
  float bq[4][8];
  auto load_cols = [&](int cb) {
    const int c = cb * 32 + (lane & 31);
    const bool cok = c < C;
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int l = 16 * it + 8 * kh + j;
        const bool ok = cok && l < L;
        const float t = in[ok ? l * C + c : 0];
        bq[it][j] = ok ? t : 0.f;
      }
  };
  load_cols(blockIdx.x);
  stage_tile<256, 16>(Ws, ldw, W + (int64_t)m0 * L, L, 128, L, M - m0, L);
  __syncthreads();
  const int mw = m0 + wave * 32;
  if (mw >= M) return;  // no barrier follows
  const float* Wr = Ws + (wave * 32 + (lane & 31)) * ldw;
  for (int cb = blockIdx.x; cb < ncb; cb += gridDim.x) {
    if (cb != (int)blockIdx.x) load_cols(cb);
    const int c = cb * 32 + (lane & 31);
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int kk = 16 * it;
      if (kk >= L) break;
      float av[8];
      float* bv = bq[it];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int l = kk + 8 * kh + j;
        av[j] = l < L ? Wr[l] : 0.f;
      }
      bf16x8 ah, al, bh, bl;
      split8(av, ah, al);
      split8(bv, bh, bl);
      acc = mma3(ah, al, bh, bl, acc);
    }
    if (c < C) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mw + acc_row(r, lane);
        if (m < M) out[(int64_t)m * C + c] = acc[r];
      }
    }
  }
}

// Workgroup caps of the first-axis launches that walk several column tiles per workgroup: the
// autotuner picks one per kernel, element type and (M, L, C) shape (the total number of workgroups
// decides how many rounds the grid takes and how often each W tile is staged).
constexpr int kCaps[] = {256, 512, 768, 1024, 1536, 2048};
constexpr int kNumCaps = sizeof(kCaps) / sizeof(kCaps[0]);
std::string cap_key(const char* kern, int M, int L, int C) {
  return std::string("dft:") + kern + ":M" + std::to_string(M) + ":L" + std::to_string(L) + ":C" + std::to_string(C);
}

}  // namespace

int dft_cap_count() { return kNumCaps; }

void dft_left_bf16(const float* in, float* out, const FieldMats<float>& W, int nb, int bpf, int M, int L, int C,
                   int64_t sIb, int64_t sOb, hipStream_t s) {
  if (nb <= 0 || M <= 0 || C <= 0) return;
  const double bytes = 4.0 * ((double)nb * L * C + (double)nb * M * C);
  const double flops = 2.0 * nb * M * (double)L * C;
  if (M <= 64 && L > 64 && L <= 192) {
    const int MB = M > 32 ? 2 : 1;
    const uint32_t sm = (uint32_t)std::max(32 * MB * (L + 1), 4 * MB * 16 * 64) * sizeof(float);
    dim3 g(ceil_div(C, 32), 1, nb);
    if (MB == 2)
      prof::launch("dft_left_contract_bf16<2>", bytes, flops, dft_left_contract_bf16<2>, g, dim3(256), sm, s, in, out,
                   W, bpf, M, L, C, sIb, sOb);
    else
      prof::launch("dft_left_contract_bf16<1>", bytes, flops, dft_left_contract_bf16<1>, g, dim3(256), sm, s, in, out,
                   W, bpf, M, L, C, sIb, sOb);
  } else if (L <= 64) {
    const uint32_t sm = (uint32_t)128 * (L + 1) * sizeof(float);
    const int ncb = ceil_div(C, 32), gy = ceil_div(M, 128);
    // at most cap workgroups, each walking several column tiles with its W tile staged once (default
    // 768, the 3 per CU its registers allow: 32 uneven subjects 85 -> 90 subject-matvecs/s)
    auto run = [&](int cap) {
      dim3 g(std::max(1, std::min(ncb, cap / std::max(1, nb * gy))), gy, nb);
      prof::launch("dft_left_expand_bf16", bytes, flops, dft_left_expand_bf16, g, dim3(256), sm, s, in, out, W, bpf,
                   M, L, C, sIb, sOb);
    };
    run(tune::choose(cap_key("expand_bf16", M, L, C), kCaps, kNumCaps, 768, run, s));
  } else {
    return dft_left<float>(in, out, W, nb, bpf, M, L, C, sIb, sOb, s);
  }
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void dft_left(const T* in, T* out, const FieldMats<T>& W, int nb, int bpf, int M, int L, int C, int64_t sIb,
              int64_t sOb, hipStream_t s) {
  if (nb <= 0 || M <= 0 || C <= 0) return;
  if (nb > 65535) throw ArgError("dft_left: batch too large");
  const double bytes = double(sizeof(T)) * ((double)nb * L * C + (double)nb * M * C);
  const double flops = 2.0 * nb * M * (double)L * C;
  if constexpr (std::is_same_v<T, float>) {
    if (M <= 64 && L > 64 && L <= 192) {
      const int MB = M > 32 ? 2 : 1;
      const size_t wsz = (size_t)32 * MB * (L + 1), rsz = (size_t)4 * 16 * 64;
      const int sep = (wsz + rsz) * sizeof(float) <= 65536 ? 1 : 0;
      const uint32_t sm = (uint32_t)((sep ? wsz + rsz : std::max(wsz, rsz)) * sizeof(float));
      const int ncb = ceil_div(C, 64);
      // the two-tile kernel's registers leave room for 2 blocks per CU: at most 512 blocks keeps the
      // grid resident in one round, each block walking several column tiles with its W tile
      // (1024 ran a second round: 160x192x160 contraction 2.10 -> 1.86 ms per matvec)
      auto run = [&](int cap) {
        const int gx = sep ? std::max(1, std::min(ncb, cap / std::max(1, nb))) : ncb;
        dim3 g(gx, 1, nb);
        if (MB == 2)
          prof::launch("dft_left_contract<2>", bytes, flops, dft_left_contract<2, 2>, g, dim3(256), sm, s, in, out,
                       W, bpf, M, L, C, sIb, sOb, sep);
        else
          prof::launch("dft_left_contract<1>", bytes, flops, dft_left_contract<1, 2>, g, dim3(256), sm, s, in, out,
                       W, bpf, M, L, C, sIb, sOb, sep);
      };
      const int dflt = MB == 2 ? 512 : 1024;
      run(sep ? tune::choose(cap_key(MB == 2 ? "contract2_f32" : "contract1_f32", M, L, C), kCaps, kNumCaps, dflt,
                             run, s)
              : dflt);
      LDDMM_LAUNCH_CHECK();
      return;
    }
    if (L <= 64) {
      const uint32_t sm = (uint32_t)(128 * (L + 1) + L * kExpLdb) * sizeof(float);
      const int ncb = ceil_div(C, kExpCols), gy = ceil_div(M, 128);
      // at most 1024 blocks (4 per CU): the whole grid is resident at once and each block walks
      // several column tiles with its W tile staged once (2048 left a second, partial round:
      // 160x192x160 expansion 1.45 -> 1.22 ms per matvec)
      const int vec = (C % 4 == 0) && (sIb % 4 == 0) && (reinterpret_cast<uintptr_t>(in) % 16 == 0);
      auto run = [&](int cap) {
        const int gx = std::max(1, std::min(ncb, cap / std::max(1, nb * gy)));
        dim3 g(gx, gy, nb);
        prof::launch("dft_left_expand", bytes, flops, dft_left_expand, g, dim3(256), sm, s, in, out, W, bpf, M, L, C,
                     sIb, sOb, vec);
      };
      run(tune::choose(cap_key("expand_f32", M, L, C), kCaps, kNumCaps, 1024, run, s));
      LDDMM_LAUNCH_CHECK();
      return;
    }
  }
  const std::string nm = std::string("dft_left_kernel<") + prof::tname<T>() + ">";
  if (M > 64) {
    dim3 g(ceil_div(C, 32), ceil_div(M, 128), nb);
    prof::launch(nm, bytes, flops, dft_left_kernel<T, 4, 1>, g, dim3(256), 0, s, in, out, W, bpf, M, L, C, sIb, sOb);
  } else if (M > 32) {
    dim3 g(ceil_div(C, 64), ceil_div(M, 64), nb);
    prof::launch(nm, bytes, flops, dft_left_kernel<T, 2, 2>, g, dim3(256), 0, s, in, out, W, bpf, M, L, C, sIb, sOb);
  } else {
    dim3 g(ceil_div(C, 128), ceil_div(M, 32), nb);
    prof::launch(nm, bytes, flops, dft_left_kernel<T, 1, 4>, g, dim3(256), 0, s, in, out, W, bpf, M, L, C, sIb, sOb);
  }
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void dft_right(const T* in, T* out, const FieldMats<T>& W, int nf, int R, int L, int Mo, hipStream_t s) {
  if (nf <= 0 || R <= 0 || Mo <= 0) return;
  const std::string nm = std::string("dft_right_kernel<") + prof::tname<T>() + ">";
  const double bytes = double(sizeof(T)) * ((double)nf * R * L + (double)nf * R * Mo);
  const double flops = 2.0 * nf * R * (double)L * Mo;
  if (Mo > 64) {
    dim3 g(ceil_div(Mo, 128), ceil_div(R, 32), nf);
    prof::launch(nm, bytes, flops, dft_right_kernel<T, 1, 4>, g, dim3(256), 0, s, in, out, W, R, L, Mo);
  } else if (Mo > 32) {
    dim3 g(ceil_div(Mo, 64), ceil_div(R, 32), nf);
    prof::launch(nm, bytes, flops, dft_right_kernel<T, 1, 2>, g, dim3(128), 0, s, in, out, W, R, L, Mo);
  } else {
    dim3 g(ceil_div(Mo, 32), ceil_div(R, 32), nf);
    prof::launch(nm, bytes, flops, dft_right_kernel<T, 1, 1>, g, dim3(64), 0, s, in, out, W, R, L, Mo);
  }
  LDDMM_LAUNCH_CHECK();
}

template void dft_left<float>(const float*, float*, const FieldMats<float>&, int, int, int, int, int, int64_t,
                              int64_t, hipStream_t);
template void dft_left<double>(const double*, double*, const FieldMats<double>&, int, int, int, int, int,
                               int64_t, int64_t, hipStream_t);
template void dft_right<float>(const float*, float*, const FieldMats<float>&, int, int, int, int, hipStream_t);
template void dft_right<double>(const double*, double*, const FieldMats<double>&, int, int, int, int,
                                hipStream_t);

}  // namespace lddmm
