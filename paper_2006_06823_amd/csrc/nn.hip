// Learned warm start and low-rank PCG preconditioner: a small 3D convolutional
// encoder with hand-written bf16 matrix-core kernels (forward, backward-data,
// backward-weight), float master weights and Adam, all on the device.
//
// Convolutions are implicit GEMMs on v_mfma_f32_32x32x16_bf16 (each wave owns a
// 32 x 32 output block; operands are converted to bf16 as they are gathered, the
// accumulation is float):
//   forward      Y[b][co][o]       = act(bias[co] + sum_{ci,t} W[co][ci][t] X[b][ci][pos(o,t)])
//   backward-data dX[b][ci][i]     = sum_{co,t} W[co][ci][t] G[b][co][o(i,t)]   (o(i,t) when it exists)
//   backward-wt   dW[co][ci][t]   += sum_{b,o} G[b][co][o] X[b][ci][pos(o,t)]  (split over blocks, atomics)
// with G = dY * act'(Y).  Activations are [B][C][D][H][W] float.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "nn.h"
#include "prof.h"

namespace lddmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ unsigned short bf16_rn(float x) {
  const unsigned int b = __float_as_uint(x);
  return static_cast<unsigned short>((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ bf16x8 to_bf16x8(const float v[8]) {
  u16x8 h;
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = bf16_rn(v[j]);
  return __builtin_bit_cast(bf16x8, h);
}

struct ConvArgs {
  const float* x;   // [B][Cin][Di][Hi][Wi]
  const float* w;   // [Cout][Cin][k^3]
  const float* b;   // [Cout] (forward)
  const float* g;   // [B][Cout][Do][Ho][Wo] gradient after the activation derivative (backward)
  float* y;         // forward output / backward-data dX / backward-weight dW
  int B, Cin, Cout, Di, Hi, Wi, Do, Ho, Wo, k, stride, pad, relu;
};

// input position of output voxel o (flattened) and tap t, or -1 when it falls in the zero padding
__device__ __forceinline__ int in_pos(const ConvArgs& a, int o, int t) {
  const int k = a.k, k2 = k * k;
  const int tz = t / k2, ty = (t / k) % k, tx = t % k;
  const int ox = o % a.Wo, oy = (o / a.Wo) % a.Ho, oz = o / (a.Wo * a.Ho);
  const int iz = oz * a.stride - a.pad + tz, iy = oy * a.stride - a.pad + ty, ix = ox * a.stride - a.pad + tx;
  if (iz < 0 || iz >= a.Di || iy < 0 || iy >= a.Hi || ix < 0 || ix >= a.Wi) return -1;
  return (iz * a.Hi + iy) * a.Wi + ix;
}

// output voxel reached from input voxel i through tap t, or -1
__device__ __forceinline__ int out_pos(const ConvArgs& a, int i, int t) {
  const int k = a.k, k2 = k * k;
  const int tz = t / k2, ty = (t / k) % k, tx = t % k;
  const int ix = i % a.Wi, iy = (i / a.Wi) % a.Hi, iz = i / (a.Wi * a.Hi);
  int oz = iz + a.pad - tz, oy = iy + a.pad - ty, ox = ix + a.pad - tx;
  if (oz < 0 || oy < 0 || ox < 0) return -1;
  if (oz % a.stride || oy % a.stride || ox % a.stride) return -1;
  oz /= a.stride, oy /= a.stride, ox /= a.stride;
  if (oz >= a.Do || oy >= a.Ho || ox >= a.Wo) return -1;
  return (oz * a.Ho + oy) * a.Wo + ox;
}

// forward: M = Cout, N = output voxels of one sample, K = Cin k^3; block = 4 waves on 4 voxel blocks
__global__ __launch_bounds__(256) void k_conv_fwd(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 31, kh = lane >> 5;
  const int No = a.Do * a.Ho * a.Wo, Ni = a.Di * a.Hi * a.Wi, k3 = a.k * a.k * a.k, K = a.Cin * k3;
  const int b = blockIdx.z, co0 = blockIdx.y * 32, o0 = (blockIdx.x * 4 + wave) * 32;
  if (o0 >= No) return;
  const int co = co0 + li, o = o0 + li;
  const float* xb = a.x + (int64_t)b * a.Cin * Ni;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int kk = 0; kk < K; kk += 16) {
    float av[8], bv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kj = kk + 8 * kh + j;
      av[j] = (co < a.Cout && kj < K) ? a.w[(int64_t)co * K + kj] : 0.f;
      float xv = 0.f;
      if (o < No && kj < K) {
        const int ci = kj / k3, t = kj - ci * k3;
        const int ip = in_pos(a, o, t);
        if (ip >= 0) xv = xb[(int64_t)ci * Ni + ip];
      }
      bv[j] = xv;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(to_bf16x8(av), to_bf16x8(bv), acc, 0, 0, 0);
  }
  if (o < No) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = co0 + acc_row(r, lane);
      if (c < a.Cout) {
        float v = acc[r] + a.b[c];
        if (a.relu) v = v > 0.f ? v : 0.f;
        a.y[((int64_t)b * a.Cout + c) * No + o] = v;
      }
    }
  }
}

// backward-data: M = Cin, N = input voxels, K = Cout k^3
__global__ __launch_bounds__(256) void k_conv_bwd_data(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 31, kh = lane >> 5;
  const int No = a.Do * a.Ho * a.Wo, Ni = a.Di * a.Hi * a.Wi, k3 = a.k * a.k * a.k, K = a.Cout * k3;
  const int b = blockIdx.z, ci0 = blockIdx.y * 32, i0 = (blockIdx.x * 4 + wave) * 32;
  if (i0 >= Ni) return;
  const int ci = ci0 + li, i = i0 + li;
  const float* gb = a.g + (int64_t)b * a.Cout * No;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int kk = 0; kk < K; kk += 16) {
    float av[8], bv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kj = kk + 8 * kh + j;
      const int co = kj / k3, t = kj - co * k3;
      av[j] = (ci < a.Cin && kj < K) ? a.w[((int64_t)co * a.Cin + ci) * k3 + t] : 0.f;
      float gv = 0.f;
      if (i < Ni && kj < K) {
        const int op = out_pos(a, i, t);
        if (op >= 0) gv = gb[(int64_t)co * No + op];
      }
      bv[j] = gv;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(to_bf16x8(av), to_bf16x8(bv), acc, 0, 0, 0);
  }
  if (i < Ni) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = ci0 + acc_row(r, lane);
      if (c < a.Cin) a.y[((int64_t)b * a.Cin + c) * Ni + i] = acc[r];
    }
  }
}

// backward-weight: M = Cout, N = Cin k^3, K = B x output voxels split into chunks of KC per block
constexpr int KC = 512;
__global__ __launch_bounds__(256) void k_conv_bwd_weight(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 31, kh = lane >> 5;
  const int No = a.Do * a.Ho * a.Wo, Ni = a.Di * a.Hi * a.Wi, k3 = a.k * a.k * a.k, N = a.Cin * k3;
  const int Ktot = a.B * No;
  const int co0 = blockIdx.y * 32, n0 = (blockIdx.x * 4 + wave) * 32, kb = blockIdx.z * KC;
  if (n0 >= N) return;
  const int co = co0 + li, n = n0 + li;
  const int ci = n / k3, t = n - ci * k3;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  const int ke = min(Ktot, kb + KC);
  for (int kk = kb; kk < ke; kk += 16) {
    float av[8], bv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kj = kk + 8 * kh + j;
      float gv = 0.f, xv = 0.f;
      if (kj < ke) {
        const int b = kj / No, o = kj - b * No;
        if (co < a.Cout) gv = a.g[((int64_t)b * a.Cout + co) * No + o];
        if (n < N) {
          const int ip = in_pos(a, o, t);
          if (ip >= 0) xv = a.x[((int64_t)b * a.Cin + ci) * Ni + ip];
        }
      }
      av[j] = gv;
      bv[j] = xv;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(to_bf16x8(av), to_bf16x8(bv), acc, 0, 0, 0);
  }
  if (n < N) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = co0 + acc_row(r, lane);
      if (c < a.Cout) atomicAdd(&a.y[(int64_t)c * N + n], acc[r]);
    }
  }
}

// G = dY * act'(Y) and the bias gradient db[c] += sum over the block's slice of G[b][c][:]
__global__ __launch_bounds__(256) void k_act_bwd(const float* dy, const float* y, float* g, float* db, int C,
                                                 int No, int relu) {
  const int bc = blockIdx.y;  // b * C + c
  const int c = bc % C;
  float s = 0.f;
  for (int o = blockIdx.x * 256 + threadIdx.x; o < No; o += gridDim.x * 256) {
    const int64_t idx = (int64_t)bc * No + o;
    float v = dy[idx];
    if (relu && y[idx] <= 0.f) v = 0.f;
    g[idx] = v;
    s += v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  __shared__ float part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&db[c], part[0] + part[1] + part[2] + part[3]);
}

__global__ void k_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_fill(float* p, int64_t n, float v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// network input from an image pair: box average of each f0 x f1 x f2 voxel cell, out [2][S^3]
__global__ void k_pool_pair(const float* __restrict__ I0, const float* __restrict__ I1, int n1, int n2, int f0, int f1,
                            int f2, int S, float* __restrict__ out) {
  const int64_t S3 = (int64_t)S * S * S;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= 2 * S3) return;
  const int ch = (int)(e / S3);
  const int64_t o = e - ch * S3;
  const int oz = (int)(o / (S * S)), oy = (int)((o / S) % S), ox = (int)(o % S);
  const float* I = ch == 0 ? I0 : I1;
  float sum = 0.f;
  for (int a = 0; a < f0; ++a)
    for (int b = 0; b < f1; ++b) {
      const float* row = I + ((int64_t)(oz * f0 + a) * n1 + (oy * f1 + b)) * n2 + (int64_t)ox * f2;
      for (int c = 0; c < f2; ++c) sum += row[c];
    }
  out[e] = sum / (float)(f0 * f1 * f2);
}

// coarse velocity samples [B][3][s^3] -> band-limited coefficients [B][3][K0][K1][K2]:
// the separable projection P[a][x] onto the s-point band for slots a < s - 1, zero elsewhere
__global__ void k_samples_to_bl(const float* __restrict__ samp, const float* __restrict__ P, int B, int gs, int sz,
                                int k0, int k1, int k2, float* __restrict__ v) {
  const int64_t Q = (int64_t)k0 * k1 * k2;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * 3 * Q) return;
  const int64_t bc = e / Q, q = e - bc * Q;
  const int64_t sc = (bc / 3) * gs * 3 + bc % 3;  // sample channel: group b at stride gs
  const int a0 = (int)(q / ((int64_t)k1 * k2)), a1 = (int)((q / k2) % k1), a2 = (int)(q % k2);
  const int nb = sz - 1;
  float r = 0.f;
  if (a0 < nb && a1 < nb && a2 < nb) {
    const float* sp = samp + sc * sz * sz * sz;
    for (int x0 = 0; x0 < sz; ++x0) {
      float t1 = 0.f;
      for (int x1 = 0; x1 < sz; ++x1) {
        float t2 = 0.f;
        for (int x2 = 0; x2 < sz; ++x2) t2 += P[a2 * sz + x2] * sp[(x0 * sz + x1) * sz + x2];
        t1 += P[a1 * sz + x1] * t2;
      }
      r += P[a0 * sz + x0] * t1;
    }
  }
  v[e] = r;
}

// gradient of the weighted squared coefficient error with respect to the samples:
// ds[b][c][x] = scale * sum_{a in block} P[a0][x0] P[a1][x1] P[a2][x2] w[a] diff[b][c][a]
__global__ void k_block_grad(const float* __restrict__ diff, const double* __restrict__ w, const float* __restrict__ P,
                             int B, int gs, int sz, int k0, int k1, int k2, float scale, float* __restrict__ ds) {
  const int s3 = sz * sz * sz;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * 3 * s3) return;
  const int64_t bc = e / s3;
  const int x = (int)(e - bc * s3);
  const int64_t sc = (bc / 3) * gs * 3 + bc % 3;  // output channel: group b at stride gs
  const int x0 = x / (sz * sz), x1 = (x / sz) % sz, x2 = x % sz;
  const int nb = sz - 1;
  const float* dp = diff + bc * k0 * k1 * k2;
  float r = 0.f;
  for (int a0 = 0; a0 < nb; ++a0) {
    float t1 = 0.f;
    for (int a1 = 0; a1 < nb; ++a1) {
      float t2 = 0.f;
      for (int a2 = 0; a2 < nb; ++a2) {
        const int64_t q = ((int64_t)a0 * k1 + a1) * k2 + a2;
        t2 += P[a2 * sz + x2] * (float)w[q] * dp[q];
      }
      t1 += P[a1 * sz + x1] * t2;
    }
    r += P[a0 * sz + x0] * t1;
  }
  ds[sc * s3 + x] = scale * r;
}

}  // namespace

// ------------------------------------------------------------------------------------------
void conv_forward(const ConvLayer& L, const float* x, float* y, int B, int Di, hipStream_t s) {
  ConvArgs a{};
  a.x = x, a.w = L.w, a.b = L.b, a.y = y;
  a.B = B, a.Cin = L.cin, a.Cout = L.cout, a.k = L.k, a.stride = L.stride, a.pad = L.pad, a.relu = L.relu;
  a.Di = a.Hi = a.Wi = Di;
  a.Do = a.Ho = a.Wo = (Di + 2 * L.pad - L.k) / L.stride + 1;
  const int No = a.Do * a.Ho * a.Wo;
  dim3 g(ceil_div(No, 128), ceil_div(L.cout, 32), B);
  prof::launch("k_conv_fwd", 4.0 * ((double)B * L.cin * Di * Di * Di + (double)B * L.cout * No),
               2.0 * B * (double)No * L.cout * L.cin * L.k * L.k * L.k, k_conv_fwd, g, dim3(256), 0, s, a);
  LDDMM_LAUNCH_CHECK();
}

void conv_backward(const ConvLayer& L, const float* x, const float* y, const float* dy, float* g, float* dx, int B,
                   int Di, hipStream_t s) {
  ConvArgs a{};
  a.x = x, a.w = L.w, a.g = g;
  a.B = B, a.Cin = L.cin, a.Cout = L.cout, a.k = L.k, a.stride = L.stride, a.pad = L.pad, a.relu = L.relu;
  a.Di = a.Hi = a.Wi = Di;
  a.Do = a.Ho = a.Wo = (Di + 2 * L.pad - L.k) / L.stride + 1;
  const int No = a.Do * a.Ho * a.Wo, Ni = Di * Di * Di, k3 = L.k * L.k * L.k;
  // activation derivative and bias gradient
  dim3 ga(std::max(1, std::min(64, ceil_div(No, 256))), B * L.cout);
  k_act_bwd<<<ga, 256, 0, s>>>(dy, y, g, L.db, L.cout, No, L.relu);
  LDDMM_LAUNCH_CHECK();
  // weight gradient (accumulated)
  a.y = L.dw;
  const int N = L.cin * k3;
  dim3 gw(ceil_div(N, 128), ceil_div(L.cout, 32), ceil_div((int64_t)B * No, KC));
  prof::launch("k_conv_bwd_weight", 0.0, 2.0 * B * (double)No * L.cout * N, k_conv_bwd_weight, gw, dim3(256), 0,
               s, a);
  LDDMM_LAUNCH_CHECK();
  if (dx) {
    a.y = dx;
    dim3 gd(ceil_div(Ni, 128), ceil_div(L.cin, 32), B);
    prof::launch("k_conv_bwd_data", 0.0, 2.0 * B * (double)Ni * L.cin * L.cout * k3, k_conv_bwd_data, gd,
                 dim3(256), 0, s, a);
    LDDMM_LAUNCH_CHECK();
  }
}

void adam_step(float* w, float* m, float* v, const float* g, int64_t n, float lr, int t, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
  k_adam<<<ceil_div(n, 256), 256, 0, s>>>(w, m, v, g, n, lr, b1, b2, c1, c2, 1e-8f);
  LDDMM_LAUNCH_CHECK();
}

void fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  k_fill<<<ceil_div(n, 256), 256, 0, s>>>(p, n, v);
  LDDMM_LAUNCH_CHECK();
}

void pool_pair(const float* I0, const float* I1, const int n[3], int S, float* out, hipStream_t s) {
  const int64_t tot = 2LL * S * S * S;
  k_pool_pair<<<ceil_div(tot, 256), 256, 0, s>>>(I0, I1, n[1], n[2], n[0] / S, n[1] / S, n[2] / S, S, out);
  LDDMM_LAUNCH_CHECK();
}

void samples_to_bl(const float* samp, const float* P, int B, int gs, int sz, const int k[3], float* v,
                   hipStream_t s) {
  const int64_t tot = (int64_t)B * 3 * k[0] * k[1] * k[2];
  k_samples_to_bl<<<ceil_div(tot, 256), 256, 0, s>>>(samp, P, B, gs, sz, k[0], k[1], k[2], v);
  LDDMM_LAUNCH_CHECK();
}

void block_grad(const float* diff, const double* w, const float* P, int B, int gs, int sz, const int k[3],
                float scale, float* ds, hipStream_t s) {
  const int64_t tot = (int64_t)B * 3 * sz * sz * sz;
  k_block_grad<<<ceil_div(tot, 256), 256, 0, s>>>(diff, w, P, B, gs, sz, k[0], k[1], k[2], scale, ds);
  LDDMM_LAUNCH_CHECK();
}

}  // namespace lddmm
