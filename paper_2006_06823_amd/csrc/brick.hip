// Tricubic B-spline interpolation at SL departure points through LDS bricks
// (float, 3D grids).
//
// A workgroup owns a 4 x 8 x 32 tile of output nodes.  Per coefficient field
// it stages the tile plus a 2-node halo on every side (8 x 12 x 36 floats,
// 13.8 KB) into LDS with coalesced, periodically wrapped loads (the wrapped row
// offsets and columns are tabulated once per workgroup), then evaluates
// the 64-tap tensor B-spline for each of its nodes from LDS.  A departure
// point whose 4 x 4 x 4 stencil leaves the brick (displacement of a voxel or
// more) falls back to a gather from global memory, so any displacement is
// handled; at the SL step sizes of the configurations (about 0.8 voxel) every
// stencil lies in the brick.  The epilogue functor consumes the interpolated
// values of a node together with its other pointwise operands, fusing the
// SL-RK2 step update of each equation into the same pass.
#include "kernels.h"

#include <climits>
#include <type_traits>
#include "prof.h"
#include "tune.h"

namespace lddmm {

namespace {

constexpr int HALO = 2;

// Output tile of one workgroup; the autotuner picks one of these per grid shape.
// LD2 >= B2 is the LDS row stride of the brick (B2 plus PAD2 unused columns)
template <int X0, int X1, int X2, int NT, int PAD2 = 0>
struct Tile {
  static constexpr int TX0 = X0, TX1 = X1, TX2 = X2, NTHR = NT;
  static constexpr int B0 = TX0 + 2 * HALO, B1 = TX1 + 2 * HALO, B2 = TX2 + 2 * HALO;
  static constexpr int LD2 = B2 + PAD2;
  static constexpr int NPT = B0 * B1 * B2;   // staged points
  static constexpr int VOL = B0 * B1 * LD2;  // LDS floats per field
  static constexpr int PPT = TX0 * TX1 * TX2 / NTHR;  // nodes per thread
};
using TileA = Tile<4, 8, 32, 256>;
using TileB = Tile<8, 8, 32, 512>;
using TileC = Tile<2, 16, 32, 256>;
using TileD = Tile<4, 4, 64, 256>;
// 1024-thread tiles for the 160 KB LDS of a gfx950 workgroup: a 16 x 8 x 32 tile re-reads 2.1x its
// coefficient volume through the halo instead of 2.5x (8 x 8 x 32), and two workgroups fill a CU
using TileE = Tile<16, 8, 32, 1024>;
using TileF = Tile<8, 16, 32, 1024>;
// row strides a multiple of 32 floats: a departure point's bank depends only on its column, so
// neighbouring lanes in different brick rows no longer collide (3-5x fewer LDS bank conflicts
// than the unpadded stride 36 at sub-voxel displacements)
using TileG = Tile<8, 8, 32, 512, 28>;  // row stride 64
using TileH = Tile<4, 4, 64, 256, 28>;  // row stride 96
constexpr int kTiles = 8;

struct Grid3 {
  int n0, n1, n2;
  int64_t P;
};

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Cubic B-spline weights of a tap offset t in [0, 1): w3 = t^3/6, w0 = (1-t)^3/6, w1 = 2/3 - t^2 (1 - t/2),
// and w2 from the partition of unity (12 operations instead of the polynomial forms' 15).
__device__ __forceinline__ void brick_weights(float t, float w[4]) {
  const float t2 = t * t, u = 1.f - t;
  w[3] = t2 * (t * (1.f / 6.f));
  w[0] = (u * u) * (u * (1.f / 6.f));
  w[1] = fmaf(t2, fmaf(t, 0.5f, -1.f), 2.f / 3.f);
  w[2] = 1.f - w[0] - w[1] - w[3];
}

// LDS views of the brick: with the address space explicit, tap addresses stay 32-bit and the rows of a
// stencil are reached by immediate offsets from one base per node
typedef const __attribute__((address_space(3))) float lds_float;
typedef const __attribute__((address_space(3))) unsigned long long lds_pair;  // two interleaved floats

// p + off as a base the compiler cannot see through: the taps of one slab (row offsets b B2 + c <= 3 B2 + 3)
// are then reached by the LDS reads' immediate offsets from this one register, instead of an address
// add per pair of taps (the slab offset itself exceeds the 8-bit offsets of the paired reads)
template <typename P>
__device__ __forceinline__ P* opaque_base(P* p, int off) {
  unsigned u = static_cast<unsigned>(reinterpret_cast<uintptr_t>(p + off));
  asm volatile("" : "+v"(u));
  return reinterpret_cast<P*>(static_cast<uintptr_t>(u));
}

// 64-tap evaluation from the LDS brick at the brick-relative first tap (s0, s1, s2).  The stencil is read
// in four slabs of 4 x 4 taps (first index a), the next slab's reads issued before the current one is
// summed; empty asm statements (no instruction) keep the compiler from moving a slab's sums below the
// next slab's reads.
template <int B1, int B2>
__device__ __forceinline__ float eval_brick(const float* br, int s0, int s1, int s2, const float w0[4],
                                            const float w1[4], const float w2[4]) {
  lds_float* p = (lds_float*)br + ((s0 * B1 + s1) * B2 + s2);
  float v[2][4][4];
  auto load = [&](int a, float (&d)[4][4]) {
    lds_float* q = opaque_base(p, a * B1 * B2);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) d[b][c] = q[b * B2 + c];
  };
  load(0, v[0]);
  float acc = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (a < 3) load(a + 1, v[(a + 1) & 1]);
    const float(&d)[4][4] = v[a & 1];
    float sa = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) sa += w1[b] * (w2[0] * d[b][0] + w2[1] * d[b][1] + w2[2] * d[b][2] + w2[3] * d[b][3]);
    acc += w0[a] * sa;
    asm volatile("" : "+v"(acc)::"memory");
  }
  return acc;
}

// two fields stored interleaved (float2): one LDS read per tap serves both, and the products
// w1[b] w2[c] are formed once for the two
template <int B1, int B2>
__device__ __forceinline__ float2 eval_brick2(const float2* br, int s0, int s1, int s2, const float w0[4],
                                              const float w1[4], const float w2[4]) {
  lds_pair* p = (lds_pair*)br + ((s0 * B1 + s1) * B2 + s2);
  float w12[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < 4; ++c) w12[b][c] = w1[b] * w2[c];
  float2 v[2][4][4];
  auto load = [&](int a, float2 (&d)[4][4]) {
    lds_pair* q = opaque_base(p, a * B1 * B2);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) d[b][c] = __builtin_bit_cast(float2, q[b * B2 + c]);
  };
  load(0, v[0]);
  float ax = 0.f, ay = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (a < 3) load(a + 1, v[(a + 1) & 1]);
    const float2(&d)[4][4] = v[a & 1];
    float sx = 0.f, sy = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sx = fmaf(w12[b][c], d[b][c].x, sx);
        sy = fmaf(w12[b][c], d[b][c].y, sy);
      }
    ax = fmaf(w0[a], sx, ax);
    ay = fmaf(w0[a], sy, ay);
    asm volatile("" : "+v"(ax), "+v"(ay)::"memory");
  }
  return make_float2(ax, ay);
}

// GS fields stored one after the other (stride VOL): each slab's reads of every field are issued
// together, and the products w1[b] w2[c] are shared by the fields
template <int GS, int B1, int B2, int VOL>
__device__ __forceinline__ void eval_brick_n(const float* br, int s0, int s1, int s2, const float w0[4],
                                             const float w1[4], const float w2[4], float out[GS]) {
  lds_float* p = (lds_float*)br + ((s0 * B1 + s1) * B2 + s2);
  float w12[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < 4; ++c) w12[b][c] = w1[b] * w2[c];
#pragma unroll
  for (int k = 0; k < GS; ++k) out[k] = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    float d[GS][4][4];
#pragma unroll
    for (int k = 0; k < GS; ++k) {
      lds_float* q = opaque_base(p, k * VOL + a * B1 * B2);
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) d[k][b][c] = q[b * B2 + c];
    }
#pragma unroll
    for (int k = 0; k < GS; ++k) {
      float sk = 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) sk = fmaf(w12[b][c], d[k][b][c], sk);
      out[k] = fmaf(w0[a], sk, out[k]);
      asm volatile("" : "+v"(out[k])::"memory");
    }
  }
}

// (the grid sizes go by value: a reference would put the caller's Grid3 on the stack, a 24-byte
// scratch store per lane on every launch whether or not the gather runs)
__device__ __noinline__ float eval_global(const float* __restrict__ c, float x0, float x1, float x2, int n0, int n1,
                                          int n2) {
  const Grid3 g{n0, n1, n2, 0};
  int i0[4], i1[4], i2[4];
  float w0[4], w1[4], w2[4];
  bspline_weights(tap_indices(x0, g.n0, i0), w0);
  bspline_weights(tap_indices(x1, g.n1, i1), w1);
  bspline_weights(tap_indices(x2, g.n2, i2), w2);
  float acc = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    float sa = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float* row = c + (static_cast<int64_t>(i0[a]) * g.n1 + i1[b]) * g.n2;
      sa += w1[b] * (w2[0] * row[i2[0]] + w2[1] * row[i2[1]] + w2[2] * row[i2[2]] + w2[3] * row[i2[3]]);
    }
    acc += w0[a] * sa;
  }
  return acc;
}

// Epilogues that also take the interpolant at the node itself (NODE = true, accum_node).
template <class E, class = void>
struct HasNode : std::false_type {};
template <class E>
struct HasNode<E, std::void_t<decltype(E::NODE)>> : std::bool_constant<E::NODE> {};

// Generic brick kernel.  Epi provides:
//   NF, GROUPS, GSIZE and field(g, k): the NF coefficient fields (stacked with
//       stride P in `coef`) are staged GSIZE at a time, GROUPS times;
//   struct State                 per-node accumulator;
//   pos(p, i0, i1, i2, x[3])     departure point of node p (grid units);
//   init(p, State&)              loads the node's pointwise operands;
//   accum(State&, f, value)      folds the interpolated value of field f in;
//   emit(p, const State&)        writes the node's results.
// The B-spline weights of a node are computed once per group and shared by the
// group's fields.
template <class Epi, class TL>
__global__ __launch_bounds__(TL::NTHR) void k_brick(Epi epi, const float* __restrict__ coef, Grid3 g) {
  constexpr int TX0 = TL::TX0, TX1 = TL::TX1, TX2 = TL::TX2, NTHR = TL::NTHR, PPT = TL::PPT;
  constexpr int B0 = TL::B0, B1 = TL::B1, B2 = TL::B2, LD2 = TL::LD2, VOL = TL::VOL, NPT = TL::NPT;
  constexpr int GS = Epi::GSIZE;
  __shared__ __align__(16) float br[GS * VOL];
  __shared__ int rowoff[B0 * B1];  // wrapped (i0, i1) row offsets of the brick
  __shared__ int colidx[B2];       // wrapped i2 of the brick columns
  // Workgroups are dealt to the 8 XCDs round-robin in launch order, so grid neighbours would sit in
  // different L2s and every halo would be fetched again from the fabric.  When the block count is a
  // multiple of 8 the launch index is remapped so that each XCD owns one contiguous run of tiles
  // (whole rows and slabs of the volume), whose shared halos then hit in its own L2.
  const int gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
  int bid = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
  const int bx = bid % gx, byz = bid / gx, by = byz % gy, bz = byz / gy;
  const int t0 = bz * TX0, t1 = by * TX1, t2 = bx * TX2;
  const int o0 = t0 - HALO, o1 = t1 - HALO, o2 = t2 - HALO;
  const int tid = threadIdx.x;
  for (int e = tid; e < B0 * B1; e += NTHR) {
    const int b0 = e / B1, b1 = e - b0 * B1;
    rowoff[e] = (wrapi(o0 + b0, g.n0) * g.n1 + wrapi(o1 + b1, g.n1)) * g.n2;
  }
  for (int e = tid; e < B2; e += NTHR) colidx[e] = wrapi(o2 + e, g.n2);
  float x[PPT][3];
  int pidx[PPT];  // node index (grids stay below 2^31 nodes)
  bool live[PPT];
  typename Epi::State st[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int q = tid + NTHR * j;
    const int l2 = q % TX2, l1 = (q / TX2) % TX1, l0 = q / (TX1 * TX2);
    const int i0 = t0 + l0, i1 = t1 + l1, i2 = t2 + l2;
    live[j] = (i0 < g.n0) && (i1 < g.n1) && (i2 < g.n2);
    pidx[j] = (i0 * g.n1 + i1) * g.n2 + i2;
    if (live[j]) {
      epi.pos(pidx[j], i0, i1, i2, x[j]);
      epi.init(pidx[j], st[j]);
    } else {
      x[j][0] = x[j][1] = x[j][2] = 0.f;
    }
  }
  // every load of the thread is issued before its first LDS store (one memory latency per brick);
  // with several field groups the next group's loads are issued before the current group's
  // evaluation, so their latency hides behind it
  constexpr int NIT = (NPT + NTHR - 1) / NTHR;
  float v[NIT][GS];
  __syncthreads();  // row offsets and columns tabulated
  // fields below 2^29 nodes are read through raw buffer loads (one resource per field, 32-bit byte
  // offsets: no 64-bit address arithmetic per staged point)
  const bool rawbuf = g.P < (int64_t(1) << 29);
  auto load_group = [&](int grp) {
    if (rawbuf) {
      __amdgpu_buffer_rsrc_t rs[GS];
#pragma unroll
      for (int k = 0; k < GS; ++k)
        rs[k] = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(coef + Epi::field(grp, k) * g.P), (short)0,
                                                  (int)(g.P * 4), 0x00020000);
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int e = tid + it * NTHR;
        if (e < NPT) {
          const int row = e / B2, b2 = e - row * B2;
          const unsigned off = (unsigned)(rowoff[row] + colidx[b2]) * 4u;
#pragma unroll
          for (int k = 0; k < GS; ++k)
            v[it][k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs[k], (int)off, 0, 0));
        }
      }
      return;
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = tid + it * NTHR;
      if (e < NPT) {
        const int row = e / B2, b2 = e - row * B2;
        const int off = rowoff[row] + colidx[b2];
#pragma unroll
        for (int k = 0; k < GS; ++k) v[it][k] = coef[Epi::field(grp, k) * g.P + off];
      }
    }
  };
  load_group(0);
#pragma unroll 1
  for (int grp = 0; grp < Epi::GROUPS; ++grp) {
    __syncthreads();  // the previous group's evaluation is done with the brick
    {
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int e = tid + it * NTHR;
        if (e < NPT) {
          const int row = e / B2, b2 = e - row * B2;
          const int q = row * LD2 + b2;
          if constexpr (GS == 2) {  // interleaved pair
            reinterpret_cast<float2*>(br)[q] = make_float2(v[it][0], v[it][1]);
          } else {
#pragma unroll
            for (int k = 0; k < GS; ++k) br[k * VOL + q] = v[it][k];
          }
        }
      }
    }
    __syncthreads();
    if (grp + 1 < Epi::GROUPS) load_group(grp + 1);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (!live[j]) continue;
      if constexpr (HasNode<Epi>::value) {
        // the interpolant at the node itself: taps node-1 .. node+2, always inside the brick
        const int q = tid + NTHR * j;
        const int l2 = q % TX2, l1 = (q / TX2) % TX1, l0 = q / (TX1 * TX2);
        float wn[4];
        bspline_weights(0.f, wn);
#pragma unroll
        for (int k = 0; k < GS; ++k)
          epi.accum_node(st[j], Epi::field(grp, k),
                         eval_brick<B1, LD2>(br + k * VOL, l0 + HALO - 1, l1 + HALO - 1, l2 + HALO - 1, wn, wn, wn));
      }
      const float f0 = floorf(x[j][0]), f1 = floorf(x[j][1]), f2 = floorf(x[j][2]);
      const int s0 = static_cast<int>(f0) - 1 - o0, s1 = static_cast<int>(f1) - 1 - o1,
                s2 = static_cast<int>(f2) - 1 - o2;
      const bool inb = s0 >= 0 && s0 + 3 < B0 && s1 >= 0 && s1 + 3 < B1 && s2 >= 0 && s2 + 3 < B2;
      if (inb) {
        float w0[4], w1[4], w2[4];
        brick_weights(x[j][0] - f0, w0);
        brick_weights(x[j][1] - f1, w1);
        brick_weights(x[j][2] - f2, w2);
        if constexpr (GS == 2) {
          const float2 v = eval_brick2<B1, LD2>(reinterpret_cast<const float2*>(br), s0, s1, s2, w0, w1, w2);
          epi.accum(st[j], Epi::field(grp, 0), v.x);
          epi.accum(st[j], Epi::field(grp, 1), v.y);
        } else if constexpr (GS >= 3) {
          float o[GS];
          eval_brick_n<GS, B1, LD2, VOL>(br, s0, s1, s2, w0, w1, w2, o);
#pragma unroll
          for (int k = 0; k < GS; ++k) epi.accum(st[j], Epi::field(grp, k), o[k]);
        } else {
#pragma unroll
          for (int k = 0; k < GS; ++k)
            epi.accum(st[j], Epi::field(grp, k), eval_brick<B1, LD2>(br + k * VOL, s0, s1, s2, w0, w1, w2));
        }
      } else {
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          const int f = Epi::field(grp, k);
          epi.accum(st[j], f, eval_global(coef + f * g.P, x[j][0], x[j][1], x[j][2], g.n0, g.n1, g.n2));
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PPT; ++j)
    if (live[j]) epi.emit(pidx[j], st[j]);
}

// default field staging: all fields in one group
template <int NFv>
struct OneGroup {
  static constexpr int NF = NFv, GROUPS = 1, GSIZE = NFv;
  __device__ static int field(int, int k) { return k; }
};

// ---- epilogues ---------------------------------------------------------------------

// nodes displaced by a stored departure displacement field (grid units)
struct DispPos {
  const float* __restrict__ disp;
  int64_t P;
  __device__ __forceinline__ void pos(int64_t p, int i0, int i1, int i2, float x[3]) const {
    x[0] = i0 + disp[p];
    x[1] = i1 + disp[P + p];
    x[2] = i2 + disp[2 * P + p];
  }
};

template <int NFv>
struct EpiInterp : DispPos, OneGroup<NFv> {
  static constexpr int NF = NFv;
  struct State {
    float o[NF];
  };
  float* __restrict__ out;
  __device__ __forceinline__ void init(int64_t, State&) const {}
  __device__ __forceinline__ void accum(State& s, int f, float v) const {
#pragma unroll
    for (int i = 0; i < NF; ++i) s.o[i] = (f == i) ? v : s.o[i];
  }
  __device__ __forceinline__ void emit(int64_t p, const State& s) const {
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f * P + p] = s.o[f];
  }
};

// out_f = P(c_f) o X - P(c_f)(x): the interpolant's change along the characteristic (projected, it is
// the step's increment of a band-limited field, whose own projection the caller adds back exactly)
template <int NFv>
struct EpiInterpDiff : DispPos, OneGroup<NFv> {
  static constexpr int NF = NFv;
  static constexpr bool NODE = true;
  static_assert(NFv != 2, "two fields are staged interleaved");
  struct State {
    float o[NF], n[NF];
  };
  float* __restrict__ out;
  __device__ __forceinline__ void init(int64_t, State&) const {}
  __device__ __forceinline__ void accum(State& s, int f, float v) const {
#pragma unroll
    for (int i = 0; i < NF; ++i) s.o[i] = (f == i) ? v : s.o[i];
  }
  __device__ __forceinline__ void accum_node(State& s, int f, float v) const {
#pragma unroll
    for (int i = 0; i < NF; ++i) s.n[i] = (f == i) ? v : s.n[i];
  }
  __device__ __forceinline__ void emit(int64_t p, const State& s) const {
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f * P + p] = s.o[f] - s.n[f];
  }
};

// band-limited adjoint Heun step: out_f = cA_f o X + dt/2 divv (cB_f o X)
// FS: fields between cA_i and cB_i (NC, or 3 for one component of a three-component pair of stacks)
template <int NC, int FS = NC>
struct EpiBLAdjoint : DispPos {
  // fields [cA_0..cA_{NC-1}, cB_0..cB_{NC-1}], staged as the pairs (cA_i, cB_i)
  static constexpr int NF = 2 * NC, GROUPS = NC, GSIZE = 2;
  __device__ static int field(int g, int k) { return g + k * FS; }
  struct State {
    float hd, o[NC];
  };
  float* __restrict__ out;
  const float* __restrict__ divv;
  float dt;
  __device__ __forceinline__ void init(int64_t p, State& s) const {
    s.hd = 0.5f * dt * divv[p];
#pragma unroll
    for (int i = 0; i < NC; ++i) s.o[i] = 0.f;
  }
  __device__ __forceinline__ void accum(State& s, int f, float v) const {
    const float w = f < NC ? v : s.hd * v;
    const int i0 = f < NC ? f : f - FS;
#pragma unroll
    for (int i = 0; i < NC; ++i) s.o[i] += (i0 == i) ? w : 0.f;
  }
  __device__ __forceinline__ void emit(int64_t p, const State& s) const {
#pragma unroll
    for (int f = 0; f < NC; ++f) out[f * P + p] = s.o[f];
  }
};

// image-transport adjoint on the grid: a = c1 o X, b = c2 o X,
// out = a + dt/2 (b + (a + dt b) divv) = (1 + dt/2 divv) a + dt/2 (1 + dt divv) b
struct EpiAdjointGrid : DispPos, OneGroup<2> {
  static constexpr int NF = 2;
  struct State {
    float ca, cb, o;
  };
  float* __restrict__ out;
  const float* __restrict__ divv;
  float dt;
  __device__ __forceinline__ void init(int64_t p, State& s) const {
    const float dv = divv[p];
    s.ca = 1.f + 0.5f * dt * dv;
    s.cb = 0.5f * dt * (1.f + dt * dv);
    s.o = 0.f;
  }
  __device__ __forceinline__ void accum(State& s, int f, float v) const { s.o += (f == 0 ? s.ca : s.cb) * v; }
  __device__ __forceinline__ void emit(int64_t p, const State& s) const { out[p] = s.o; }
};

// characteristics: X* = x + sdt v, X - x = sdt/2 (v + v o X*) (grid units)
struct EpiCharacteristics : OneGroup<3> {
  static constexpr int NF = 3;
  struct State {
    float o[3];
  };
  const float* __restrict__ v;
  float* __restrict__ disp;
  int64_t P;
  float sdt, s0, s1, s2;  // signed dt and per-axis grid sizes
  __device__ __forceinline__ void pos(int64_t p, int i0, int i1, int i2, float x[3]) const {
    x[0] = i0 + sdt * v[p] * s0;
    x[1] = i1 + sdt * v[P + p] * s1;
    x[2] = i2 + sdt * v[2 * P + p] * s2;
  }
  __device__ __forceinline__ void init(int64_t, State&) const {}
  __device__ __forceinline__ void accum(State& s, int f, float val) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) s.o[i] = (f == i) ? val : s.o[i];
  }
  __device__ __forceinline__ void emit(int64_t p, const State& s) const {
    const float h = 0.5f * sdt;
    disp[p] = h * (v[p] * s0 + s.o[0] * s0);
    disp[P + p] = h * (v[P + p] * s1 + s.o[1] * s1);
    disp[2 * P + p] = h * (v[2 * P + p] * s2 + s.o[2] * s2);
  }
};

template <class Epi, class TL>
void launch_tile(const std::string& name, double bytes, const Epi& epi, const float* coef, const Grid3& g,
                 hipStream_t s) {
  dim3 grid(ceil_div(g.n2, TL::TX2), ceil_div(g.n1, TL::TX1), ceil_div(g.n0, TL::TX0));
  prof::launch(name, bytes, 0.0, k_brick<Epi, TL>, grid, dim3(TL::NTHR), 0, s, epi, coef, g);
}

std::string shape_key(const Dims& d) {
  return "brick:" + std::to_string(d.n[0]) + "x" + std::to_string(d.n[1]) + "x" + std::to_string(d.n[2]);
}

template <class Epi>
void launch(const std::string& name, double bytes, const Epi& epi, const float* coef, const Dims& d,
            hipStream_t s, int tile = -1) {
  const Grid3 g{d.n[0], d.n[1], d.n[2], d.P};
  if (tile < 0) tile = std::max(0, tune::get(shape_key(d) + ":gs" + std::to_string(Epi::GSIZE), 0));
  // epilogues with more than three fields would spill at 1024 threads: they keep the 512-thread tile
  if ((tile == 4 || tile == 5) && Epi::NF > 3) tile = 1;
  switch (tile) {
    case 1:
      launch_tile<Epi, TileB>(name, bytes, epi, coef, g, s);
      break;
    case 2:
      launch_tile<Epi, TileC>(name, bytes, epi, coef, g, s);
      break;
    case 3:
      launch_tile<Epi, TileD>(name, bytes, epi, coef, g, s);
      break;
    case 4:  // (not instantiated for the epilogues that keep the 512-thread tile)
      if constexpr (Epi::NF <= 3) launch_tile<Epi, TileE>(name, bytes, epi, coef, g, s);
      break;
    case 5:
      if constexpr (Epi::NF <= 3) launch_tile<Epi, TileF>(name, bytes, epi, coef, g, s);
      break;
    case 6:
      launch_tile<Epi, TileG>(name, bytes, epi, coef, g, s);
      break;
    case 7:
      launch_tile<Epi, TileH>(name, bytes, epi, coef, g, s);
      break;
    default:
      launch_tile<Epi, TileA>(name, bytes, epi, coef, g, s);
  }
  LDDMM_LAUNCH_CHECK();
}

std::string nm(const char* base) { return std::string("k_brick<") + base + ">"; }

// smooth sub-voxel departure displacements (amplitude 0.8 voxel) for timing the tiles under the
// LDS access pattern of real steps
__global__ void k_tune_disp(float* disp, int n0, int n1, int n2) {
  const int64_t P = (int64_t)n0 * n1 * n2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int i2 = (int)(p % n2), i1 = (int)((p / n2) % n1), i0 = (int)(p / ((int64_t)n1 * n2));
  const float ph = 6.2831853f * ((float)i0 / n0 + 2.f * i1 / n1 + 3.f * i2 / n2);
#pragma unroll
  for (int c = 0; c < 3; ++c) disp[c * P + p] = 0.8f * sinf(ph + 1.7f * c);
}

// ---- transformation through whole-deformation maps ------------------------------------

// 64-tap evaluation from a staged box with runtime strides (rows of e2 floats, planes of e1 rows)
__device__ __forceinline__ float eval_box(const float* __restrict__ br, int s0, int s1, int s2, int e1, int e2,
                                          const float w0[4], const float w1[4], const float w2[4]) {
  float acc = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    float sa = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float* row = br + ((s0 + a) * e1 + (s1 + b)) * e2 + s2;
      sa += w1[b] * (w2[0] * row[0] + w2[1] * row[1] + w2[2] * row[2] + w2[3] * row[3]);
    }
    acc += w0[a] * sa;
  }
  return acc;
}

// out_n(x) = a w_n(x) P(c)(x - u_n(x)) for node n = blockIdx.y (u_n [3][P] in unit-torus units, w_n
// optional).  The departure points lie up to a whole deformation away from their nodes, beyond any
// fixed halo, but they move smoothly: the workgroup takes the bounding box of its tile's 4 x 4 x 4
// stencils (a min / max over the workgroup), stages the box into LDS when it holds at most CAP floats
// and evaluates every node from there; a larger box falls back to gathers from global memory.
template <int TX0, int TX1, int TX2, int NTHR, int CAP>
__global__ __launch_bounds__(NTHR) void k_pull_back_box(float* __restrict__ out, const float* __restrict__ c,
                                                        const float* __restrict__ u, const float* __restrict__ w,
                                                        float a, Grid3 g) {
  constexpr int PPT = TX0 * TX1 * TX2 / NTHR, NW = NTHR / 64;
  __shared__ float br[CAP];
  __shared__ int bmin[3], bmax[3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T2 = (g.n2 + TX2 - 1) / TX2, T1 = (g.n1 + TX1 - 1) / TX1;
  // consecutive tiles of one node on one XCD (its L2 then holds the boxes' overlap)
  const int nb = gridDim.x;
  int bid = blockIdx.x;
  if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
  const int bx = bid % T2, rest = bid / T2, by = rest % T1, bz = rest / T1;
  const int64_t P = g.P, node = blockIdx.y;
  const float* __restrict__ un = u + node * 3 * P;
  if (tid < 3) bmin[tid] = INT_MAX, bmax[tid] = INT_MIN;
  float x[PPT][3];
  int pidx[PPT];
  bool live[PPT];
  int lmin[3] = {INT_MAX, INT_MAX, INT_MAX}, lmax[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int q = tid + NTHR * j;
    const int l2 = q % TX2, l1 = (q / TX2) % TX1, l0 = q / (TX1 * TX2);
    const int i0 = bz * TX0 + l0, i1 = by * TX1 + l1, i2 = bx * TX2 + l2;
    live[j] = i0 < g.n0 && i1 < g.n1 && i2 < g.n2;
    pidx[j] = (i0 * g.n1 + i1) * g.n2 + i2;
    x[j][0] = x[j][1] = x[j][2] = 0.f;
    if (live[j]) {
      const int p = pidx[j];
      x[j][0] = i0 - un[p] * g.n0;
      x[j][1] = i1 - un[P + p] * g.n1;
      x[j][2] = i2 - un[2 * P + p] * g.n2;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int f = static_cast<int>(floorf(x[j][k]));
        lmin[k] = min(lmin[k], f - 1);
        lmax[k] = max(lmax[k], f + 2);
      }
    }
  }
  __syncthreads();  // bounds initialised
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (lmin[k] != INT_MAX) {
      atomicMin(&bmin[k], lmin[k]);
      atomicMax(&bmax[k], lmax[k]);
    }
  }
  __syncthreads();
  const int lo0 = bmin[0], lo1 = bmin[1], lo2 = bmin[2];
  // every tile holds a live node (the grid is ceil-divided), so bmin <= bmax on every axis
  const int64_t w0b = (int64_t)bmax[0] - lo0 + 1, w1b = (int64_t)bmax[1] - lo1 + 1, w2b = (int64_t)bmax[2] - lo2 + 1;
  const bool staged = w0b > 0 && w1b > 0 && w2b > 0 && w0b <= g.n0 && w1b <= g.n1 && w2b <= g.n2 && w2b <= 128 &&
                      w0b * w1b * w2b <= CAP;
  const int e0 = staged ? (int)w0b : 0, e1 = staged ? (int)w1b : 0, e2 = staged ? (int)w2b : 0;
  if (staged) {
    const int m0 = ((lo0 % g.n0) + g.n0) % g.n0, m1 = ((lo1 % g.n1) + g.n1) % g.n1, m2 = ((lo2 % g.n2) + g.n2) % g.n2;
    // a wave stages rows of e2 columns, two rows per 64 lanes when they are at most 32 columns wide,
    // RB (pairs of) rows at a time with all their loads requested before its LDS stores
    constexpr int RB = 4;
    const int rows = e0 * e1;
    const bool half = e2 <= 32;
    const int lrow = half ? (lane >> 5) : 0, lcol = half ? (lane & 31) : lane, rstep = half ? 2 : 1;
    for (int row0 = wave * RB * rstep; row0 < rows; row0 += NW * RB * rstep) {
      float vals[RB][2];
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        const int row = row0 + k * rstep + lrow;
        vals[k][0] = vals[k][1] = 0.f;
        if (row < rows) {
          const int b0 = row / e1, b1 = row - b0 * e1;
          int r0 = m0 + b0, r1 = m1 + b1;
          if (r0 >= g.n0) r0 -= g.n0;
          if (r1 >= g.n1) r1 -= g.n1;
          const float* __restrict__ src = c + ((int64_t)r0 * g.n1 + r1) * g.n2;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int cc = lcol + 64 * h;
            if (cc < e2) {
              int c2 = m2 + cc;
              if (c2 >= g.n2) c2 -= g.n2;
              vals[k][h] = src[c2];
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        const int row = row0 + k * rstep + lrow;
        if (row < rows) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int cc = lcol + 64 * h;
            if (cc < e2) br[row * e2 + cc] = vals[k][h];
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    if (!live[j]) continue;
    float val;
    if (staged) {
      const float f0 = floorf(x[j][0]), f1 = floorf(x[j][1]), f2 = floorf(x[j][2]);
      float w0[4], w1[4], w2[4];
      bspline_weights(x[j][0] - f0, w0);
      bspline_weights(x[j][1] - f1, w1);
      bspline_weights(x[j][2] - f2, w2);
      val = eval_box(br, static_cast<int>(f0) - 1 - lo0, static_cast<int>(f1) - 1 - lo1,
                     static_cast<int>(f2) - 1 - lo2, e1, e2, w0, w1, w2);
    } else {
      val = eval_global(c, x[j][0], x[j][1], x[j][2], g.n0, g.n1, g.n2);
    }
    const int64_t o = node * P + pidx[j];
    out[o] = a * (w ? w[o] * val : val);
  }
}

}  // namespace

bool brick_ok(const Dims& d) { return d.n[0] > 1; }

void brick_pull_back(float* out, const float* c, const float* u, const float* w, float a, int nodes, const Dims& d,
                     hipStream_t s) {
  // 8 x 8 x 16 nodes per workgroup: the boxes of an 8-voxel deformation of 128^3 hold 5 staged values per
  // node on average and all fit in 8192 floats (32 KB, five workgroups per CU)
  constexpr int TX0 = 8, TX1 = 8, TX2 = 16, NTHR = 256, CAP = 8192;
  if (nodes < 1 || nodes > 65535) throw ArgError("brick_pull_back: node count out of range");
  const Grid3 g{d.n[0], d.n[1], d.n[2], d.P};
  const int64_t tiles = (int64_t)ceil_div(d.n[0], TX0) * ceil_div(d.n[1], TX1) * ceil_div(d.n[2], TX2);
  if (tiles > INT_MAX) throw ArgError("brick_pull_back: grid too large");
  prof::launch("k_pull_back_box", double(nodes) * (w ? 5.0 : 4.0) * d.P * 4 + d.P * 4.0, 0.0,
               k_pull_back_box<TX0, TX1, TX2, NTHR, CAP>, dim3(static_cast<unsigned>(tiles), nodes), dim3(NTHR), 0,
               s, out, c, u, w, a, g);
  LDDMM_LAUNCH_CHECK();
}

int brick_tile_count() { return kTiles; }

// One tile per grid shape and staging width (fields staged together: 1, 2 interleaved, or 3), timed
// on the interpolation epilogue of that width; out holds 3 fields, coef 3 fields.
void brick_autotune(float* out, const float* coef, float* disp, const Dims& d, hipStream_t s) {
  const std::string key = shape_key(d) + ":gs";
  if (tune::get(key + "1", -1) >= 0 && tune::get(key + "2", -1) >= 0 && tune::get(key + "3", -1) >= 0) return;
  k_tune_disp<<<ceil_div(d.P, 256), 256, 0, s>>>(disp, d.n[0], d.n[1], d.n[2]);
  LDDMM_LAUNCH_CHECK();
  EpiInterp<1> e1;
  e1.disp = disp, e1.P = d.P, e1.out = out;
  EpiInterp<2> e2;
  e2.disp = disp, e2.P = d.P, e2.out = out;
  EpiInterp<3> e3;
  e3.disp = disp, e3.P = d.P, e3.out = out;
  tune::set(key + "1", tune::pick(kTiles, [&](int c) { launch("tune", 0.0, e1, coef, d, s, c); }, s));
  tune::set(key + "2", tune::pick(kTiles, [&](int c) { launch("tune", 0.0, e2, coef, d, s, c); }, s));
  tune::set(key + "3", tune::pick(kTiles, [&](int c) { launch("tune", 0.0, e3, coef, d, s, c); }, s));
}

void brick_interp(float* out, const float* coef, int nf, const float* disp, const Dims& d, hipStream_t s) {
  const std::string name_ = nm("k_interp") + std::to_string(nf);
  const double bytes_ = (3.0 + 2.0 * nf) * d.P * 4;
  if (nf == 1) {
    EpiInterp<1> e;
    e.disp = disp, e.P = d.P, e.out = out;
    launch(name_, bytes_, e, coef, d, s);
  } else if (nf == 3) {
    EpiInterp<3> e;
    e.disp = disp, e.P = d.P, e.out = out;
    launch(name_, bytes_, e, coef, d, s);
  } else {
    throw ArgError("brick_interp: nf must be 1 or 3");
  }
}

void brick_interp_diff(float* out, const float* coef, int nf, const float* disp, const Dims& d, hipStream_t s) {
  const std::string name_ = nm("k_interp_diff") + std::to_string(nf);
  const double bytes_ = (3.0 + 2.0 * nf) * d.P * 4;
  if (nf == 1) {
    EpiInterpDiff<1> e;
    e.disp = disp, e.P = d.P, e.out = out;
    launch(name_, bytes_, e, coef, d, s);
  } else if (nf == 3) {
    EpiInterpDiff<3> e;
    e.disp = disp, e.P = d.P, e.out = out;
    launch(name_, bytes_, e, coef, d, s);
  } else {
    throw ArgError("brick_interp_diff: nf must be 1 or 3");
  }
}

void brick_bl_adjoint_step(float* out, const float* cAB, int nc, const float* disp, const float* divv,
                           const Dims& d, float dt, hipStream_t s) {
  const std::string name_ = nm("k_bl_adjoint_step") + std::to_string(nc);
  const double bytes_ = (4.0 + 3.0 * nc) * d.P * 4;
  if (nc == 1) {
    EpiBLAdjoint<1> e;
    e.disp = disp, e.P = d.P, e.out = out, e.divv = divv, e.dt = dt;
    launch(name_, bytes_, e, cAB, d, s);
  } else if (nc == 3) {
    // one launch per component on its pair (cA_i, cB_i): a single staged pair per workgroup keeps the
    // registers (and the occupancy) of the one-component kernel
    const double bytes_i = 7.0 * d.P * 4;
    for (int i = 0; i < 3; ++i) {
      EpiBLAdjoint<1, 3> e;
      e.disp = disp, e.P = d.P, e.out = out + i * d.P, e.divv = divv, e.dt = dt;
      launch(name_, bytes_i, e, cAB + i * d.P, d, s);
    }
  } else {
    throw ArgError("brick_bl_adjoint_step: nc must be 1 or 3");
  }
}

void brick_adjoint_grid_step(float* out, const float* c12, const float* disp, const float* divv, const Dims& d,
                             float dt, hipStream_t s) {
  const std::string name_ = nm("k_adjoint_grid_step");
  const double bytes_ = 7.0 * d.P * 4;
  EpiAdjointGrid e;
  e.disp = disp, e.P = d.P, e.out = out, e.divv = divv, e.dt = dt;
  launch(name_, bytes_, e, c12, d, s);
}

void brick_characteristics(float* disp, const float* v, const float* cv, const Dims& d, float dt, int dir,
                           hipStream_t s) {
  const std::string name_ = nm("k_characteristics");
  const double bytes_ = 9.0 * d.P * 4;
  EpiCharacteristics e;
  e.v = v, e.disp = disp, e.P = d.P;
  e.sdt = dir > 0 ? dt : -dt;
  e.s0 = float(d.n[0]), e.s1 = float(d.n[1]), e.s2 = float(d.n[2]);
  launch(name_, bytes_, e, cv, d, s);
}

}  // namespace lddmm
