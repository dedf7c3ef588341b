// Plane-wise truncated DFT (Section 2.2) on the matrix cores, float.
//
// The 3D transforms are split at the first axis into a band-side stage and a
// plane-side stage, joined by "plane-band" arrays [x0][a1][a2] (one K1 x K2
// block per grid plane x0):
//   iota:  T[x0] = sum_a0 W0[x0][a0] c[a0]            (k_axis0, P part)
//          out[x0][x1][x2] = W1 T[x0] W2^T             (k_expand)
//   pi:    R[x0] = P1 f[x0] P2^T                       (k_reduce)
//          c[a0] = sum_x0 P0[a0][x0] R[x0]             (k_axis0, F part)
// k_axis0 does both first-axis stages in one launch: it finishes a projection
// (with an epilogue out = beta out + alpha r + gamma z) and forms from the
// finished coefficients, or from any band arrays, the plane-band inputs of the
// next expansions, so one semi-Lagrangian step costs expand -> interpolate ->
// reduce -> axis0.
//
// Each wave owns 32 x 32 output tiles of v_mfma_f32_32x32x2f32 (lane l holds
// A[l%32][l/32] and B[l/32][l%32] of a k-step; the accumulator register r of
// lane l holds D[acc_row(r, l)][l%32]).  Every operand load of a k-step is one
// coalesced row segment: the matrices are read in the layout whose rows are the
// contraction index, and grid fields and plane-band arrays are read along their
// contiguous axis.  The two contractions of a plane are chained in registers:
// the accumulator of the first, read as the A operand of the second (lane l%32
// its row, register r its k-step), contracts the first product's row index, so
// no LDS transpose or barrier sits between them.  A contraction's k-steps may
// visit the summation index in any order as long as both operands follow it.
#include "kernels.h"
#include "prof.h"

#include <algorithm>
#include <string>
#include <vector>

namespace lddmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

// row of the 32 x 32 accumulator tile held in register r of a lane
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ f32x16 mfma(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void zero16(f32x16& a) {
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = 0.f;
}

constexpr int kMaxKh = 32;  // k-steps of a contraction over a band axis (K <= 64)

// Raw buffer loads: one 32-bit offset register per load (the compiler batches them instead of waiting
// on each 64-bit address), and the hardware range check returns 0 for an offset at or past the end of
// the buffer, so a tile that runs past the last row of an array reads zeros.  kOut is such an offset.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr unsigned kOut = 0xFFFFFFF0u;
__device__ __forceinline__ Rsrc rsrc(const float* p, int64_t n) {
  const int64_t bytes = n * 4 < 0x7FFFFFF0 ? n * 4 : 0x7FFFFFF0;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(Rsrc r, unsigned idx) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(idx * 4u), 0, 0));
}
__device__ __forceinline__ float bload_if(Rsrc r, unsigned idx, bool ok) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(ok ? idx * 4u : kOut), 0, 0));
}

// Values the compiler cannot see are equal across a wave (they derive from the wave index) are moved
// to scalar registers, so pointer tables indexed by them are read with scalar loads.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ------------------------------------------------------------------ expansion
// One workgroup (4 waves) per (field f, plane x0, x1 block b of 32 rows).  Stage 1,
// V[a2][x1] = sum_a1 T[a1][a2] W1t[a1][x1] (T read along a2, W1t along x1), is split over the waves by
// k-steps and summed in LDS in wave order; stage 2, out[x1][x2] = sum_a2 V[a2][x1] W2t[a2][x2] with V's
// registers as the A operand, takes the x2 tiles wave, wave + 4, ...  Ragged lanes need no test: a
// lane past n1 or n2 reads finite neighbouring entries and its results are not stored, and rows
// a2 >= k2 of V meet rows of W2t past its end, which read as zeros (every plane-band entry a tile can
// reach is written or zero-initialised, so finite).
template <int JB, int KT2, bool EXACT>
__global__ __launch_bounds__(256) void k_expand(PlaneExpandArgs a) {
  __shared__ float red[4 * KT2 * 1024];
  constexpr int JW = (JB + 3) / 4;  // stage-1 k-steps per wave
  const int lane = threadIdx.x & 63, i = lane & 31, kh = lane >> 5;
  const int wave = uniform(threadIdx.x >> 6);
  const int n1 = a.n1, n2 = a.n2, k1 = a.k1, k2 = a.k2, J1 = EXACT ? JB : k1 >> 1;
  const int T2 = (n2 + 31) >> 5;
  const int b = blockIdx.x, x0 = blockIdx.y, f = blockIdx.z;
  const Rsrc rT = rsrc(a.T[f] + x0 * (k1 * k2), (int64_t)(a.n0 - x0) * k1 * k2);
  const Rsrc r1 = rsrc(a.w1t[f], (int64_t)k1 * n1);  // [k1][n1]
  const Rsrc r2 = rsrc(a.w2t[f], (int64_t)k2 * n2);  // [k2][n2]
  float* __restrict__ out = a.out + (size_t)(f * a.n0 + x0) * (size_t)(n1 * n2);
  const int x1 = b * 32 + i;
  // stage-2 operands of the wave's first x2 tile, requested first
  float wc[KT2][16];
#pragma unroll
  for (int q = 0; q < KT2; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r)
      wc[q][r] = bload_if(r2, (unsigned)((q * 32 + acc_row(r, lane)) * n2 + wave * 32 + i), wave < T2);
  // stage 1, this wave's k-steps j = wave JW .. wave JW + JW - 1 (a1 = kh J1 + j)
  float wb[JW];
#pragma unroll
  for (int u = 0; u < JW; ++u) {
    const int j = wave * JW + u;
    wb[u] = bload_if(r1, (unsigned)((kh * J1 + j) * n1 + x1), (EXACT && JW * 4 == JB) || j < J1);
  }
  f32x16 V[KT2];
#pragma unroll
  for (int q = 0; q < KT2; ++q) {
    zero16(V[q]);
    const int a2 = q * 32 + i;
    float ta[JW];
#pragma unroll
    for (int u = 0; u < JW; ++u) {
      const int j = wave * JW + u;
      ta[u] = bload_if(rT, (unsigned)((kh * J1 + j) * k2 + a2), (EXACT && JW * 4 == JB) || j < J1);
    }
#pragma unroll
    for (int u = 0; u < JW; ++u) V[q] = mfma(ta[u], wb[u], V[q]);
  }
#pragma unroll
  for (int q = 0; q < KT2; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) red[((wave * KT2 + q) * 16 + r) * 64 + lane] = V[q][r];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < KT2; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = (q * 16 + r) * 64 + lane;
      V[q][r] = red[e] + red[KT2 * 1024 + e] + red[2 * KT2 * 1024 + e] + red[3 * KT2 * 1024 + e];
    }
  // stage 2: k-step r of tile q contracts a2 = q 32 + acc_row(r); output rows x1, columns x2
  const bool fullrows = b * 32 + 32 <= n1;
  for (int t2 = wave; t2 < T2; t2 += 4) {
    const int x2b = t2 * 32, x2 = x2b + i;
    if (t2 != wave) {
#pragma unroll
      for (int q = 0; q < KT2; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) wc[q][r] = bload(r2, (unsigned)((q * 32 + acc_row(r, lane)) * n2 + x2));
    }
    f32x16 acc;
    zero16(acc);
#pragma unroll
    for (int q = 0; q < KT2; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc = mfma(V[q][r], wc[q][r], acc);
    if (fullrows && x2b + 32 <= n2) {
#pragma unroll
      for (int r = 0; r < 16; ++r) out[(unsigned)((b * 32 + acc_row(r, lane)) * n2 + x2)] = acc[r];
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = b * 32 + acc_row(r, lane);
        if (row < n1 && x2 < n2) out[(unsigned)(row * n2 + x2)] = acc[r];
      }
    }
  }
}

// ------------------------------------------------------------------ reduction
// Grid value of field f at node offset p (within the field) for the modes: a plain field, or a
// pointwise product of band-limited fields on the product grid.  Loads past the arrays read 0.
template <int MODE>
struct RedIn {
  Rsrc in, e, divv, G;
  unsigned P, en;
  __device__ __forceinline__ RedIn(const PlaneReduceArgs& a) : P((unsigned)a.P), en((unsigned)a.e_node) {
    if constexpr (MODE == kRedPlain) {
      in = rsrc(a.in, (int64_t)a.nf * a.P);
    } else {
      const int64_t ne = (MODE == kRedV1Products) ? 1 : (MODE == kRedV1Source || MODE == kRedV3Source) && a.e_node
                         ? (int64_t)(MODE == kRedV1Source ? a.nf : a.nf / 3) * 3 : 3;
      const int ng = MODE == kRedV1Products ? 3 : MODE == kRedV3Products ? 9
                   : MODE == kRedV1Source   ? 3 * a.nf : 3 * a.nf;
      e = rsrc(a.e, (int64_t)ne * a.P);
      G = rsrc(a.G, (int64_t)ng * a.P);
      divv = rsrc(a.divv ? a.divv : a.e, a.P);
    }
  }
  __device__ __forceinline__ float operator()(int f, unsigned p) const {
    if constexpr (MODE == kRedPlain) {
      return bload(in, (unsigned)f * P + p);
    } else if constexpr (MODE == kRedV1Products) {  // [e div v, e G0, e G1, e G2]
      const float o = f == 0 ? bload(divv, p) : bload(G, (unsigned)(f - 1) * P + p);
      return bload(e, p) * o;
    } else if constexpr (MODE == kRedV3Products) {  // [e_i div v (3), sum_i e_i d_j u_i (3)]
      if (f < 3) return bload(e, (unsigned)f * P + p) * bload(divv, p);
      const unsigned j = f - 3;
      return bload(e, p) * bload(G, j * P + p) + bload(e, P + p) * bload(G, (3 + j) * P + p) +
             bload(e, 2 * P + p) * bload(G, (6 + j) * P + p);
    } else if constexpr (MODE == kRedV1Source) {  // node f: -G_f . dv_f
      const unsigned g = 3u * f * P, q = f * en + p;
      return -(bload(G, g + p) * bload(e, q) + bload(G, g + P + p) * bload(e, P + q) +
               bload(G, g + 2 * P + p) * bload(e, 2 * P + q));
    } else {  // kRedV3Source, field f = 3 n + c: dv_c - sum_j d_j u_c dv_j at node n (dv of node n)
      const unsigned n = f / 3, c = f - 3 * n, g = (9 * n + 3 * c) * P, q = n * en + p;
      return bload(e, c * P + q) - (bload(G, g + p) * bload(e, q) + bload(G, g + P + p) * bload(e, P + q) +
                                    bload(G, g + 2 * P + p) * bload(e, 2 * P + q));
    }
  }
};

// One workgroup per (field, plane x0); its waves take the tasks (x2 tile t of 32 columns, x1 chunk s of
// 64 rows) of the plane.  Stage A: W[x2][a1] = sum_x1 in[x1][x2] P1t[x1][a1] over the chunk (the field
// read along x2; chunks of JC k-steps alternate between two accumulators, shorter rounding chains);
// stage B: R[a1][a2] += sum_x2 W[x2][a1] P2t[x2][a2], W's registers as the A operand.  Ragged tiles need
// no test: rows x1 >= n1 meet rows of P1t past its end and columns x2 >= n2 rows of P2t past its end,
// which read as zeros, against finite grid entries.  The waves' partial R are summed in LDS in wave
// order (deterministic) and stored.
template <int MODE, int KT1, int KT2, int WAVES, int CH>
__global__ __launch_bounds__(64 * WAVES) void k_reduce(PlaneReduceArgs a) {
  extern __shared__ float red[];  // [WAVES / 2][KT1 KT2][16][64]
  const int lane = threadIdx.x & 63, i = lane & 31, kh = lane >> 5;
  const int wave = uniform(threadIdx.x >> 6);
  const int plane = blockIdx.x;
  const int f = plane / a.n0, x0 = plane - f * a.n0;
  const int n1 = a.n1, n2 = a.n2, k1 = a.k1, k2 = a.k2;
  const int T2 = (n2 + 31) >> 5, S1 = (n1 + CH - 1) / CH;
  const RedIn<MODE> src(a);
  const Rsrc rp1 = rsrc(a.p1t, (int64_t)n1 * k1), rp2 = rsrc(a.p2t, (int64_t)n2 * k2);
  f32x16 R[KT1][KT2];
#pragma unroll
  for (int p = 0; p < KT1; ++p)
#pragma unroll
    for (int q = 0; q < KT2; ++q) zero16(R[p][q]);
  const unsigned pbase = (unsigned)(x0 * n1 * n2);
  constexpr int JA = CH / 2;  // stage-A k-steps of a task
  constexpr int JC = MODE == kRedPlain ? (JA < 16 ? JA : 16) : 8;
  constexpr int NH = JA / JC > 1 ? 2 : 1;  // accumulators (shorter rounding chains)
  for (int task = wave; task < T2 * S1; task += WAVES) {
    const int t = task % T2, s = task / T2;
    const int x2 = t * 32 + i;
    f32x16 W[NH][KT1];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int p = 0; p < KT1; ++p) zero16(W[h][p]);
#pragma unroll
    for (int jc = 0; jc < JA; jc += JC) {
      float xa[JC];
#pragma unroll
      for (int j = 0; j < JC; ++j) {
        const int x1 = s * CH + kh * JA + jc + j;
        xa[j] = src(f, pbase + (unsigned)(x1 * n2 + x2));
      }
#pragma unroll
      for (int p = 0; p < KT1; ++p) {
        const int a1 = p * 32 + i;
        float pb[JC];
#pragma unroll
        for (int j = 0; j < JC; ++j) {
          const int x1 = s * CH + kh * JA + jc + j;
          pb[j] = bload_if(rp1, (unsigned)(x1 * k1 + a1), a1 < k1);
        }
        const int h = (jc / JC) % NH;
#pragma unroll
        for (int j = 0; j < JC; ++j) W[h][p] = mfma(xa[j], pb[j], W[h][p]);
      }
    }
    // stage B: k-step r contracts x2 = t 32 + acc_row(r)
#pragma unroll
    for (int q = 0; q < KT2; ++q) {
      const int a2 = q * 32 + i;
      float pc[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) pc[r] = bload_if(rp2, (unsigned)((t * 32 + acc_row(r, lane)) * k2 + a2), a2 < k2);
#pragma unroll
      for (int p = 0; p < KT1; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) R[p][q] = mfma(NH == 2 ? W[0][p][r] + W[NH - 1][p][r] : W[0][p][r], pc[r], R[p][q]);
    }
  }
  // the waves' partials summed in a fixed order in NS = WAVES / 2 slots of LDS: waves w < NS store theirs
  // in slot w, waves w >= NS add theirs to slot w - NS, then the slots are summed in order
  constexpr int TILES = KT1 * KT2;
  constexpr int NS = (WAVES + 1) / 2;
  for (int half = 0; half < 2; ++half) {
    if (half == 0 ? wave < NS : wave >= NS) {
      const int slot = half == 0 ? wave : wave - NS;
#pragma unroll
      for (int p = 0; p < KT1; ++p)
#pragma unroll
        for (int q = 0; q < KT2; ++q)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            float& d = red[((slot * TILES + p * KT2 + q) * 16 + r) * 64 + lane];
            d = half == 0 ? R[p][q][r] : d + R[p][q][r];
          }
    }
    __syncthreads();
  }
  float* __restrict__ part = a.part + (size_t)plane * (k1 * k2);
  for (int e = threadIdx.x; e < TILES * 16 * 64; e += 64 * WAVES) {
    const int l = e & 63, r = (e >> 6) & 15, tile = e >> 10;
    const int p = tile / KT2, q = tile - p * KT2;
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < NS; ++w) sum += red[(w * TILES * 16) * 64 + e];
    const int a1 = p * 32 + acc_row(r, l), a2 = q * 32 + (l & 31);
    if (a1 < k1 && a2 < k2) part[a1 * k2 + a2] = sum;
  }
}

// ------------------------------------------------------------------ product-grid step
// Expansion and product reduction of one plane in one pass, for the products of a band-limited
// field e~ (1 or 3 components, plane-band inputs T) with node fields on the product grid:
//   part[f][x0] = P1 (prod_f(x0, ., .)) P2^T,  prod_f = e div v, e G_j  (MODE kRedV1Products)
//                                              e_c div v, sum_i e_i G_{3i+j}  (kRedV3Products).
// One workgroup per (output field f, plane x0); wave w owns the grid tile (x1 tile s, x2 tile t) of
// 32 x 32 nodes.  It expands the e components f needs on its tile (V = T W1t, then D = V^T W2t, the
// accumulator of the first read as the A operand of the second), multiplies by the node fields in
// registers, and contracts the tile with P1 over its rows (the product's registers as the A operand)
// and with P2 over its columns; the tiles' partials are summed in LDS in wave order.  The expanded
// field never goes to memory.  Ragged tiles need no test, as in the separate kernels: grid entries past
// n1 / n2 are finite and meet rows of P1t / P2t past their ends, which read as zeros.
template <int MODE, int KT1, int KT2, int JB, bool EXACT>
__global__ __launch_bounds__(512) void k_prod_plane(ProdPlaneArgs a) {
  extern __shared__ float red[];  // [ceil(waves / 2)][KT1 KT2][16][64]
  constexpr int NE = MODE == kRedV1Products ? 1 : 3;
  const int lane = threadIdx.x & 63, i = lane & 31, kh = lane >> 5;
  const int wave = uniform(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int n1 = a.n1, n2 = a.n2, k1 = a.k1, k2 = a.k2, J1 = EXACT ? JB : k1 >> 1;
  const int T2 = (n2 + 31) >> 5;
  const int f = blockIdx.x / a.n0, x0 = blockIdx.x - f * a.n0;
  const int s = wave / T2, t = wave - s * T2;
  const int x1 = s * 32 + i, x2 = t * 32 + i;
  const unsigned P = (unsigned)a.P, pbase = (unsigned)(x0 * n1 * n2);
  const Rsrc r1 = rsrc(a.w1t, (int64_t)k1 * n1), r2 = rsrc(a.w2t, (int64_t)k2 * n2);
  const Rsrc rp1 = rsrc(a.p1t, (int64_t)n1 * k1), rp2 = rsrc(a.p2t, (int64_t)n2 * k2);
  const Rsrc rdiv = rsrc(a.divv, a.P), rG = rsrc(a.G, (int64_t)(MODE == kRedV1Products ? 3 : 9) * a.P);
  // node offsets of this lane's accumulator rows
  unsigned pr[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) pr[r] = pbase + (unsigned)((s * 32 + acc_row(r, lane)) * n2 + x2);
  // the e components this output reads: V1 e; V3 f < 3 e_f, f >= 3 all three
  const int c0 = (MODE == kRedV3Products && f < 3) ? f : 0;
  const int ne = (MODE == kRedV3Products && f >= 3) ? 3 : 1;
  // node-field factors of each e component at this lane's nodes (requested before the expansion)
  float gf[NE][16];
#pragma unroll
  for (int c = 0; c < NE; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      unsigned q;
      if constexpr (MODE == kRedV1Products) q = f == 0 ? kOut : (unsigned)(f - 1) * P + pr[r];
      else q = f < 3 ? kOut : (unsigned)(3 * c + f - 3) * P + pr[r];
      gf[c][r] = c < ne ? (q == kOut ? bload(rdiv, pr[r]) : bload(rG, q)) : 0.f;
    }
  f32x16 Y;
  zero16(Y);
#pragma unroll
  for (int c = 0; c < NE; ++c) {
    if (c >= ne) break;
    const Rsrc rT = rsrc(a.T[c0 + c] + x0 * (k1 * k2), (int64_t)(a.n0 - x0) * k1 * k2);
    // V[a2][x1] = sum_a1 T[a1][a2] W1t[a1][x1]
    f32x16 V[KT2];
#pragma unroll
    for (int q = 0; q < KT2; ++q) {
      zero16(V[q]);
      const int a2 = q * 32 + i;
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        const bool ok = EXACT || j < J1;
        const float ta = bload_if(rT, (unsigned)((kh * J1 + j) * k2 + a2), ok);
        const float wb = bload_if(r1, (unsigned)((kh * J1 + j) * n1 + x1), ok);
        V[q] = mfma(ta, wb, V[q]);
      }
    }
    // D[x1][x2] = sum_a2 V[a2][x1] W2t[a2][x2]
    f32x16 D;
    zero16(D);
#pragma unroll
    for (int q = 0; q < KT2; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) D = mfma(V[q][r], bload(r2, (unsigned)((q * 32 + acc_row(r, lane)) * n2 + x2)), D);
#pragma unroll
    for (int r = 0; r < 16; ++r) Y[r] += D[r] * gf[c][r];
  }
  // W[x2][a1] = sum_x1 Y[x1][x2] P1t[x1][a1] over the tile's rows
  f32x16 W[KT1];
#pragma unroll
  for (int p = 0; p < KT1; ++p) {
    zero16(W[p]);
    const int a1 = p * 32 + i;
#pragma unroll
    for (int r = 0; r < 16; ++r)
      W[p] = mfma(Y[r], bload_if(rp1, (unsigned)((s * 32 + acc_row(r, lane)) * k1 + a1), a1 < k1), W[p]);
  }
  // R[a1][a2] = sum_x2 W[x2][a1] P2t[x2][a2] over the tile's columns
  f32x16 R[KT1][KT2];
#pragma unroll
  for (int q = 0; q < KT2; ++q) {
    const int a2 = q * 32 + i;
    float pc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) pc[r] = bload_if(rp2, (unsigned)((t * 32 + acc_row(r, lane)) * k2 + a2), a2 < k2);
#pragma unroll
    for (int p = 0; p < KT1; ++p) {
      zero16(R[p][q]);
#pragma unroll
      for (int r = 0; r < 16; ++r) R[p][q] = mfma(W[p][r], pc[r], R[p][q]);
    }
  }
  // partials summed in LDS in a fixed order: waves w < ns store theirs in slot w, then waves w >= ns add
  // theirs to slot w - ns, then the slots are summed in order (ns = ceil(nw / 2) slots of LDS)
  constexpr int TILES = KT1 * KT2;
  const int ns = (nw + 1) >> 1;
  for (int half = 0; half < 2; ++half) {
    const bool mine = half == 0 ? wave < ns : wave >= ns;
    if (mine) {
      const int slot = half == 0 ? wave : wave - ns;
#pragma unroll
      for (int p = 0; p < KT1; ++p)
#pragma unroll
        for (int q = 0; q < KT2; ++q)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            float& d = red[((slot * TILES + p * KT2 + q) * 16 + r) * 64 + lane];
            d = half == 0 ? R[p][q][r] : d + R[p][q][r];
          }
    }
    __syncthreads();
  }
  float* __restrict__ part = a.part + (size_t)blockIdx.x * (k1 * k2);
  for (int e = threadIdx.x; e < TILES * 16 * 64; e += blockDim.x) {
    const int l = e & 63, r = (e >> 6) & 15, tile = e >> 10;
    const int p = tile / KT2, q = tile - p * KT2;
    float sum = 0.f;
    for (int w = 0; w < ns; ++w) sum += red[(w * TILES * 16) * 64 + e];
    const int a1 = p * 32 + acc_row(r, l), a2 = q * 32 + (l & 31);
    if (a1 < k1 && a2 < k2) part[a1 * k2 + a2] = sum;
  }
}

// ------------------------------------------------------------------ first axis
// Workgroup (column tile of 32 band columns (a1, a2), row y) with the descriptor row[y] resolved on the
// host: F of field row.f (if any): r[a0][c] = sum_x0 P0t[x0][a0] part[x0][c] (x0 in chunks of 8 dealt
// to the 4 waves, summed in LDS in wave order), out = beta out + alpha r + gamma z; then up to two P
// outputs T[x0'][c] = sum_a0 W0t[a0][x0'] (c1 g1 + c2 g2 + cf fin)[a0][c], fin the field just
// finished.  Every operand that does not depend on F is requested at the start; absent band sources
// point at zeros.  As in the other stages, ragged lanes read finite neighbours and are not stored, and
// rows past the end of an operand read as zeros.
template <int KT0, int JB, bool EXACT, int CPW>
__global__ __launch_bounds__(256) void k_axis0(Axis0Kernel a) {
  __shared__ float red[4 * KT0 * 1024];
  __shared__ float fin[64 * 32];  // the finished field of this workgroup, [a0][32 columns]
  const int lane = threadIdx.x & 63, i = lane & 31, kh = lane >> 5;
  const int wave = uniform(threadIdx.x >> 6);
  const int C = a.C, k0 = a.k0, J0 = EXACT ? JB : (k0 + 1) >> 1;
  const int cb = blockIdx.x * 32;
  const int c = cb + i;
  const Axis0Kernel::Row& row = a.row[blockIdx.y];
  const int np = row.np;
  // P operands that do not depend on F: band-array sources and the first row tile of W0t
  float gsrc[2][JB], wrow[2][JB];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const Axis0Kernel::Out& o = row.p[u < np ? u : 0];
    const Rsrc r1 = rsrc(o.g1, (int64_t)k0 * C), r2 = rsrc(o.g2, (int64_t)k0 * C);
    const Rsrc rw = rsrc(o.w0t, (int64_t)k0 * o.n0t);
    const int x0 = wave * 32 + i;
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const int a0 = kh * J0 + j;
      const bool ok = u < np && (EXACT || j < J0);
      gsrc[u][j] = o.c1 * bload_if(r1, (unsigned)(a0 * C + c), ok) + o.c2 * bload_if(r2, (unsigned)(a0 * C + c), ok);
      wrow[u][j] = bload_if(rw, (unsigned)(a0 * o.n0t + x0), ok);
    }
  }
  if (row.f >= 0) {
    const Axis0Kernel::Field& F = a.fld[row.f];
    const int n0 = a.n0;
    // epilogue operands of this thread's elements
    float prev[4 * KT0];
#pragma unroll
    for (int m = 0; m < 4 * KT0; ++m) {
      const int e = threadIdx.x + 256 * m;
      const int l = e & 63, r = (e >> 6) & 15, p = e >> 10;
      const int a0 = p * 32 + acc_row(r, l), cc = cb + (l & 31);
      const bool ok = a0 < k0 && cc < C;
      const unsigned o = ok ? (unsigned)(a0 * C + cc) : 0u;
      // (in is read only when beta != 0: an output buffer need not hold finite values before)
      float v = F.beta != 0.f ? F.beta * F.in[o] : 0.f;
      v += F.gamma * F.z[o];
      if (F.ysym) v += static_cast<float>(F.ysym[o]) * F.y[o];
      prev[m] = ok ? v : 0.f;
    }
    const Rsrc rpart = rsrc(F.part, (int64_t)n0 * C), rp0 = rsrc(a.p0t, (int64_t)n0 * k0);
    f32x16 acc[KT0];
#pragma unroll
    for (int p = 0; p < KT0; ++p) zero16(acc[p]);
    // x0 in chunks of 8 (4 k-steps, lane halves 4 apart) dealt to the waves in turn; with CPW > 0 the
    // wave's CPW chunks are requested at once (chunks past n0 read zeros)
    const int nch = (n0 + 7) >> 3;
    if constexpr (CPW > 0) {
      float bv[CPW][4], av[CPW][KT0][4];
#pragma unroll
      for (int u = 0; u < CPW; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int x0 = (wave + 4 * u) * 8 + kh * 4 + j;
          bv[u][j] = bload(rpart, (unsigned)(x0 * C + c));
#pragma unroll
          for (int p = 0; p < KT0; ++p) av[u][p][j] = bload(rp0, (unsigned)(x0 * k0 + p * 32 + i));
        }
#pragma unroll
      for (int u = 0; u < CPW; ++u)
#pragma unroll
        for (int p = 0; p < KT0; ++p)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[p] = mfma(av[u][p][j], bv[u][j], acc[p]);
    } else {
      for (int ch = wave; ch < nch; ch += 4) {
        float bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = bload(rpart, (unsigned)((ch * 8 + kh * 4 + j) * C + c));
#pragma unroll
        for (int p = 0; p < KT0; ++p) {
          const int a0 = p * 32 + i;
          float av[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) av[j] = bload(rp0, (unsigned)((ch * 8 + kh * 4 + j) * k0 + a0));
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[p] = mfma(av[j], bv[j], acc[p]);
        }
      }
    }
#pragma unroll
    for (int p = 0; p < KT0; ++p)
#pragma unroll
      for (int r = 0; r < 16; ++r) red[((wave * KT0 + p) * 16 + r) * 64 + lane] = acc[p][r];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4 * KT0; ++m) {
      const int e = threadIdx.x + 256 * m;
      const int l = e & 63, r = (e >> 6) & 15, p = e >> 10;
      const float sum = red[e] + red[KT0 * 1024 + e] + red[2 * KT0 * 1024 + e] + red[3 * KT0 * 1024 + e];
      const int a0 = p * 32 + acc_row(r, l), cc = cb + (l & 31);
      if (a0 < k0 && cc < C) {
        const unsigned o = (unsigned)(a0 * C + cc);
        const float v = F.alpha * sum + prev[m];
        F.out[o] = v;
        if (F.out2) F.out2[o] = F.s2 * v;
        fin[a0 * 32 + (l & 31)] = v;
      }
    }
    __syncthreads();
  }
  // P: row tiles rt = wave, wave + 4, ... (the first one's W0t rows were requested at the start)
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (u >= np) break;
    const Axis0Kernel::Out& o = row.p[u];
    const bool useF = row.f >= 0 && o.cf != 0.f;
    float bv[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const int a0 = kh * J0 + j;
      const bool ok = useF && (EXACT || (j < J0 && a0 < k0));
      const float fv = fin[ok ? a0 * 32 + i : 0];
      bv[j] = gsrc[u][j] + (ok ? o.cf * fv : 0.f);
    }
    const Rsrc rw = rsrc(o.w0t, (int64_t)k0 * o.n0t);
    const int RT = (o.n0t + 31) >> 5;
    for (int rt = wave; rt < RT; rt += 4) {
      const int x0 = rt * 32 + i;
      float av[JB];
      if (rt == wave) {
#pragma unroll
        for (int j = 0; j < JB; ++j) av[j] = wrow[u][j];
      } else {
#pragma unroll
        for (int j = 0; j < JB; ++j) av[j] = bload_if(rw, (unsigned)((kh * J0 + j) * o.n0t + x0), EXACT || j < J0);
      }
      f32x16 acc;
      zero16(acc);
#pragma unroll
      for (int j = 0; j < JB; ++j) acc = mfma(av[j], bv[j], acc);
      if (c < C) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int rr = rt * 32 + acc_row(r, lane);
          if (rr < o.n0t) o.T[(unsigned)(rr * C + c)] = acc[r];
        }
      }
    }
  }
}

}  // namespace

bool planes_ok(const Dims& d) {
  // 32-bit offsets within a field and within a first-axis stage
  return d.k[0] <= 64 && d.k[1] <= 64 && d.k[2] <= 64 && (d.k[0] == 1 || d.k[0] % 2 == 0) && d.k[1] % 2 == 0 &&
         d.k[2] % 2 == 0 && d.P < (int64_t(1) << 31) && (int64_t)d.n[0] * d.k[1] * d.k[2] < (int64_t(1) << 31);
}

static int jb_of(int j) { return j <= 8 ? 8 : j <= 16 ? 16 : j <= 24 ? 24 : 32; }

void plane_expand(const PlaneExpandArgs& a, hipStream_t s) {
  const int B1 = ceil_div(a.n1, 32);
  if (a.n0 > 65535 || a.nf > 65535) throw ArgError("plane_expand: grid too large");
  const double bytes = 4.0 * a.nf * ((double)a.n0 * a.k1 * a.k2 + (double)a.n0 * a.n1 * a.n2);
  const double flops = 2.0 * a.nf * a.n0 * ((double)a.k1 * a.k2 * a.n1 + (double)a.n1 * a.k2 * a.n2);
  dim3 g(B1, a.n0, a.nf);
  const int j1 = a.k1 / 2, jb = jb_of(j1);
  auto go = [&](auto kern) { prof::launch("k_expand", bytes, flops, kern, g, dim3(256), 0, s, a); };
  if (a.k2 <= 32) {
    if (j1 == 16) go(k_expand<16, 1, true>); else if (j1 == 20) go(k_expand<20, 1, true>);
    else if (j1 == 24) go(k_expand<24, 1, true>); else if (j1 == 32) go(k_expand<32, 1, true>);
    else if (jb == 8) go(k_expand<8, 1, false>); else if (jb == 16) go(k_expand<16, 1, false>);
    else if (jb == 24) go(k_expand<24, 1, false>); else go(k_expand<32, 1, false>);
  } else {
    if (j1 == 16) go(k_expand<16, 2, true>); else if (j1 == 20) go(k_expand<20, 2, true>);
    else if (j1 == 24) go(k_expand<24, 2, true>); else if (j1 == 32) go(k_expand<32, 2, true>);
    else if (jb == 8) go(k_expand<8, 2, false>); else if (jb == 16) go(k_expand<16, 2, false>);
    else if (jb == 24) go(k_expand<24, 2, false>); else go(k_expand<32, 2, false>);
  }
  LDDMM_LAUNCH_CHECK();
}

template <int MODE>
static void reduce_mode(const PlaneReduceArgs& a, hipStream_t s, double bytes, double flops) {
  const int kt1 = a.k1 > 32 ? 2 : 1, kt2 = a.k2 > 32 ? 2 : 1;
  dim3 g(static_cast<unsigned>(a.nf * a.n0));
  const char* nm = MODE == kRedPlain ? "k_reduce" : "k_reduce_products";
  // tasks of 64 rows (16-wave workgroups with 32-row tasks measured slower); 8 waves (4 for two band tiles
  // per axis: 8 slowed the product modes of the 40x48x40 band from 29 to 54 us), their partials in half as
  // many slots of LDS (KT1 KT2 x 4 KB each)
  // Small planes (the 48 x 48 product grid of a 32-wide band: two 64-row tasks for eight waves) take
  // 16-row tasks instead, one per wave: each wave's chain of dependent load groups is then one group
  // long instead of four.
  const int t2 = ceil_div(a.n2, 32);
  const bool small = 2 * t2 * ceil_div(a.n1, 64) <= 8 && t2 * ceil_div(a.n1, 16) <= 8;
  if (kt1 == 1 && kt2 == 1 && small)
    prof::launch(nm, bytes, flops, k_reduce<MODE, 1, 1, 8, 16>, g, dim3(512), 4 * 1024 * 4, s, a);
  else if (kt1 == 1 && kt2 == 1)
    prof::launch(nm, bytes, flops, k_reduce<MODE, 1, 1, 8, 64>, g, dim3(512), 4 * 1024 * 4, s, a);
  else if (kt1 == 1)
    prof::launch(nm, bytes, flops, k_reduce<MODE, 1, 2, 8, 64>, g, dim3(512), 4 * 2048 * 4, s, a);
  else if (kt2 == 1)
    prof::launch(nm, bytes, flops, k_reduce<MODE, 2, 1, 8, 64>, g, dim3(512), 4 * 2048 * 4, s, a);
  else
    prof::launch(nm, bytes, flops, k_reduce<MODE, 2, 2, 4, 64>, g, dim3(256), 2 * 4096 * 4, s, a);
  LDDMM_LAUNCH_CHECK();
}

void plane_reduce(const PlaneReduceArgs& a, hipStream_t s) {
  const double flops = 2.0 * a.nf * a.n0 * ((double)a.n1 * a.n2 * a.k1 + (double)a.k1 * a.n2 * a.k2);
  const double bytes = 4.0 * a.nf * a.n0 * ((double)a.n1 * a.n2 + (double)a.k1 * a.k2);
  if (a.P >= (int64_t(1) << 31)) throw ArgError("plane_reduce: field too large");
  switch (a.mode) {
    case kRedPlain: return reduce_mode<kRedPlain>(a, s, bytes, flops);
    case kRedV1Products: return reduce_mode<kRedV1Products>(a, s, bytes, flops);
    case kRedV3Products: return reduce_mode<kRedV3Products>(a, s, bytes, flops);
    case kRedV1Source: return reduce_mode<kRedV1Source>(a, s, bytes, flops);
    case kRedV3Source: return reduce_mode<kRedV3Source>(a, s, bytes, flops);
    default: throw ArgError("plane_reduce: unknown mode");
  }
}

// one wave per 32 x 32 tile of a plane (at most 8), their partials in ceil(tiles / 2) slots of at
// most 64 KB of LDS together.  The fused pass is chosen for inner bands of at most 32 (one band tile
// per axis): with two, every workgroup's repeated expansions (each output field's workgroup expands
// the e components it reads) cost more than the separate kernels save (160x192x160 / 40x48x40
// deformation state: 46 us per fused launch against 30 us for the separate reduction).
static size_t prod_plane_lds(int tiles, int kt) { return (size_t)((tiles + 1) / 2) * kt * 4096; }
bool prod_plane_ok(const Dims& d) {
  const int tiles = ceil_div(d.n[1], 32) * ceil_div(d.n[2], 32);
  const int kt = (d.k[1] > 32 ? 2 : 1) * (d.k[2] > 32 ? 2 : 1);
  return planes_ok(d) && tiles <= 8 && kt == 1 && prod_plane_lds(tiles, kt) <= 64 * 1024;
}

void plane_prod(const ProdPlaneArgs& a, hipStream_t s) {
  const int tiles = ceil_div(a.n1, 32) * ceil_div(a.n2, 32);
  const int kt1 = a.k1 > 32 ? 2 : 1, kt2 = a.k2 > 32 ? 2 : 1;
  if (tiles > 8 || kt1 * kt2 != 1 || prod_plane_lds(tiles, 1) > 64 * 1024)
    throw ArgError("plane_prod: plane or band too large");
  if (a.P >= (int64_t(1) << 31)) throw ArgError("plane_prod: field too large");
  const int nf = a.mode == kRedV1Products ? 4 : 6;
  const int ne = a.mode == kRedV1Products ? 1 : 3;
  const double bytes = 4.0 * a.n0 * (ne * (double)a.k1 * a.k2 + nf * (double)a.k1 * a.k2) +
                       4.0 * a.P * (a.mode == kRedV1Products ? 4 : 10);
  const double flops = 2.0 * nf * a.n0 *
                       ((double)a.k1 * a.k2 * a.n1 + (double)a.n1 * a.k2 * a.n2 + (double)a.n1 * a.n2 * a.k1 +
                        (double)a.k1 * a.n2 * a.k2);
  dim3 g(static_cast<unsigned>(nf * a.n0));
  const dim3 b(64 * tiles);
  const size_t lds = prod_plane_lds(tiles, kt1 * kt2);
  const int j1 = a.k1 / 2;
  const bool ex = j1 == 16 || j1 == 20 || j1 == 24 || j1 == 32;
  const int jb = ex ? j1 : jb_of(j1);
  auto go = [&](auto kern) { prof::launch("k_prod_plane", bytes, flops, kern, g, b, lds, s, a); };
  auto pick = [&](auto mode) {
    constexpr int M = decltype(mode)::value;
    if (ex && jb == 16) go(k_prod_plane<M, 1, 1, 16, true>);
    else go(k_prod_plane<M, 1, 1, 16, false>);
  };
  if (a.mode == kRedV1Products) pick(std::integral_constant<int, kRedV1Products>{});
  else if (a.mode == kRedV3Products) pick(std::integral_constant<int, kRedV3Products>{});
  else throw ArgError("plane_prod: unknown mode");
  LDDMM_LAUNCH_CHECK();
}

void plane_axis0(const Axis0Args& a, hipStream_t s) {
  if (a.nin > kMaxFields || a.nout > kMaxFields) throw ArgError("plane_axis0: too many fields");
  if (a.k0 > 64) throw ArgError("plane_axis0: band above 64");
  if (!a.zeros) throw ArgError("plane_axis0: zero source missing");
  // descriptor rows: one per finished field (with the P outputs that read it), then one per P output
  // that reads band arrays only
  Axis0Kernel k{};
  k.p0t = a.p0t, k.n0 = a.n0, k.k0 = a.k0, k.C = a.C;
  for (int f = 0; f < a.nin; ++f) {
    Axis0Kernel::Field& F = k.fld[f];
    F.part = a.part[f], F.out = a.out[f], F.in = a.in[f] ? a.in[f] : a.out[f], F.out2 = a.out2[f];
    F.z = a.z[f] ? a.z[f] : a.zeros;
    F.y = a.y[f], F.ysym = a.y[f] ? a.ysym[f] : nullptr;
    if (F.y && !F.ysym) throw ArgError("plane_axis0: a symbol-weighted term needs its symbol");
    F.alpha = a.alpha[f], F.beta = a.beta[f], F.gamma = a.z[f] ? a.gamma[f] : 0.f;
    F.s2 = a.s2[f] != 0.f ? a.s2[f] : 1.f;
  }
  int nrow = a.nin;
  for (int f = 0; f < a.nin; ++f) k.row[f].f = f, k.row[f].np = 0;
  double bytes = 4.0 * a.nin * ((double)a.n0 + a.k0) * a.C, flops = 2.0 * a.nin * a.k0 * a.n0 * (double)a.C;
  for (int g = 0; g < a.nout; ++g) {
    const Axis0Out& o = a.o[g];
    const int src = std::max(o.s1, o.s2);
    if (src >= a.nin) throw ArgError("plane_axis0: a P source names an unfinished field");
    if (o.s1 >= 0 && o.s2 >= 0 && o.s1 != o.s2) throw ArgError("plane_axis0: one finished field per P output");
    Axis0Kernel::Row* r;
    if (src >= 0) {
      r = &k.row[src];
      if (r->np >= 2) throw ArgError("plane_axis0: at most two P outputs per finished field");
    } else {
      if (nrow >= Axis0Kernel::kRows) throw ArgError("plane_axis0: too many P outputs");
      r = &k.row[nrow++];
      r->f = -1, r->np = 0;
    }
    Axis0Kernel::Out& p = r->p[r->np++];
    p.w0t = o.w0t, p.T = o.T, p.n0t = o.n0t;
    p.g1 = o.g1 ? o.g1 : a.zeros, p.c1 = o.g1 ? o.c1 : 0.f;
    p.g2 = o.g2 ? o.g2 : a.zeros, p.c2 = o.g2 ? o.c2 : 0.f;
    p.cf = (o.s1 >= 0 ? o.c1 : 0.f) + (o.s2 >= 0 ? o.c2 : 0.f);
    bytes += 4.0 * (double)o.n0t * a.C;
    flops += 2.0 * o.n0t * a.k0 * (double)a.C;
  }
  for (int y = 0; y < nrow; ++y)  // rows without outputs read their first slot's pointers: valid ones
    for (int u = k.row[y].np; u < 2; ++u) {
      Axis0Kernel::Out& p = k.row[y].p[u];
      p.w0t = a.p0t, p.T = nullptr, p.n0t = 0, p.g1 = p.g2 = a.zeros, p.c1 = p.c2 = p.cf = 0.f;
    }
  if (nrow == 0) return;
  dim3 g(ceil_div(a.C, 32), nrow);
  const int j0 = (a.k0 + 1) / 2, jb = jb_of(j0);
  const bool ex = a.k0 % 2 == 0;
  const int cpw = ceil_div(ceil_div(a.n0, 8), 4);  // x0 chunks per wave
  const std::string nm = "k_axis0[" + std::to_string(a.nin) + "F" + std::to_string(a.nout) + "P]";
  auto go = [&](auto kern) { prof::launch(nm, bytes, flops, kern, g, dim3(256), 0, s, k); };
  if (ex && j0 == 16 && cpw <= 2) go(k_axis0<1, 16, true, 2>);
  else if (ex && j0 == 16 && cpw <= 4) go(k_axis0<1, 16, true, 4>);
  else if (ex && j0 == 16) go(k_axis0<1, 16, true, 0>);
  else if (ex && j0 == 20 && cpw <= 2) go(k_axis0<2, 20, true, 2>);
  else if (ex && j0 == 20 && cpw <= 6) go(k_axis0<2, 20, true, 6>);
  else if (ex && j0 == 20) go(k_axis0<2, 20, true, 0>);
  else if (ex && j0 == 24 && cpw <= 2) go(k_axis0<2, 24, true, 2>);
  else if (ex && j0 == 24 && cpw <= 6) go(k_axis0<2, 24, true, 6>);
  else if (ex && j0 == 24) go(k_axis0<2, 24, true, 0>);
  else if (ex && j0 == 32) go(k_axis0<2, 32, true, 0>);
  else if (a.k0 <= 32) {
    if (jb == 8) go(k_axis0<1, 8, false, 0>); else go(k_axis0<1, 16, false, 0>);
  } else {
    if (jb == 24) go(k_axis0<2, 24, false, 0>); else go(k_axis0<2, 32, false, 0>);
  }
  LDDMM_LAUNCH_CHECK();
}

}  // namespace lddmm
