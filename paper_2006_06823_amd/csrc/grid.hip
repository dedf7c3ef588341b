// Grid-point and band-coefficient kernels: characteristics, tricubic B-spline
// interpolation fused with the SL-RK2 step updates (Section 3), the periodic
// B-spline prefilter, source terms and products of the variants' equations
// (Sections 2.3.1, 2.3.3, Table 1) and the Jacobian determinant.
//
// Every grid kernel maps one thread to one node; fields are component-major
// [c][n0][n1][n2], n2 contiguous, so neighbouring lanes touch neighbouring nodes.
#include "kernels.h"
#include "prof.h"
#include "stage.h"

#include <type_traits>

namespace lddmm {

namespace {

constexpr int kBlock = 256;

struct GridIdx {
  int i0, i1, i2;
};

__device__ __forceinline__ GridIdx unflatten(int64_t p, int n1, int n2) {
  GridIdx g;
  g.i2 = static_cast<int>(p % n2);
  const int64_t q = p / n2;
  g.i1 = static_cast<int>(q % n1);
  g.i0 = static_cast<int>(q / n1);
  return g;
}

// Tricubic B-spline taps of one point: periodic indices and weights per axis.
template <typename T>
struct Taps {
  int i0[4], i1[4], i2[4];
  T w0[4], w1[4], w2[4];
  __device__ __forceinline__ void set(T x0, T x1, T x2, int n0, int n1, int n2) {
    bspline_weights(tap_indices(x0, n0, i0), w0);
    bspline_weights(tap_indices(x1, n1, i1), w1);
    bspline_weights(tap_indices(x2, n2, i2), w2);
  }
  __device__ __forceinline__ T eval(const T* __restrict__ c, int n1, int n2) const {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      T sa = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const T* row = c + (static_cast<int64_t>(i0[a]) * n1 + i1[b]) * n2;
        const T sb = w2[0] * row[i2[0]] + w2[1] * row[i2[1]] + w2[2] * row[i2[2]] + w2[3] * row[i2[3]];
        sa += w1[b] * sb;
      }
      acc += w0[a] * sa;
    }
    return acc;
  }
};

// ---- band coefficient kernels ----------------------------------------------

template <typename T>
__global__ void k_axpby(T* out, T a, const T* x, T b, const T* y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  T r = a * x[i];
  if (y) r += b * y[i];
  out[i] = r;
}

template <typename T>
__global__ void k_scale_sym(T* out, const T* x, const double* sym, int ncomp, int64_t Q, const T* y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Q * ncomp) return;
  T r = static_cast<T>(sym[i % Q]) * x[i];
  if (y) r += y[i];
  out[i] = r;
}

// derivative along one axis in the real basis: slot 2k-1 (cos) <- 2 pi k * slot 2k (sin),
// slot 2k (sin) <- -2 pi k * slot 2k-1 (cos); slot 0 and the pad slot -> 0.
__device__ __forceinline__ int deriv_src(int a, int K, double& fac) {
  const double two_pi = 6.283185307179586476925286766559;
  if (a == 0 || (K % 2 == 0 && a == K - 1)) {
    fac = 0.0;
    return a;
  }
  const int k = (a + 1) / 2;
  if (a & 1) {
    fac = two_pi * k;
    return a + 1;
  }
  fac = -two_pi * k;
  return a - 1;
}

template <typename T>
__global__ void k_bl_div(T* out, const T* v, int k0, int k1, int k2) {
  const int64_t Q = (int64_t)k0 * k1 * k2;
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= Q) return;
  const int a2 = static_cast<int>(q % k2);
  const int a1 = static_cast<int>((q / k2) % k1);
  const int a0 = static_cast<int>(q / ((int64_t)k1 * k2));
  double acc = 0.0, f;
  int s = deriv_src(a0, k0, f);
  if (k0 > 1 && f != 0.0) acc += f * static_cast<double>(v[0 * Q + ((int64_t)s * k1 + a1) * k2 + a2]);
  s = deriv_src(a1, k1, f);
  if (k1 > 1 && f != 0.0) acc += f * static_cast<double>(v[1 * Q + ((int64_t)a0 * k1 + s) * k2 + a2]);
  s = deriv_src(a2, k2, f);
  if (k2 > 1 && f != 0.0) acc += f * static_cast<double>(v[2 * Q + ((int64_t)a0 * k1 + a1) * k2 + s]);
  out[q] = static_cast<T>(acc);
}

// ---- characteristics (Section 3.1) ----------------------------------------

template <typename T>
__global__ void k_characteristics(T* __restrict__ disp, const T* __restrict__ v, const T* __restrict__ cv,
                                  int n0, int n1, int n2, T dt, int dir) {
  const int64_t P = (int64_t)n0 * n1 * n2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const GridIdx g = unflatten(p, n1, n2);
  const T sdt = dir > 0 ? dt : -dt;
  const T v0 = v[p] * n0, v1 = v[P + p] * n1, v2 = v[2 * P + p] * n2;  // grid units
  Taps<T> t;
  t.set(g.i0 + sdt * v0, g.i1 + sdt * v1, g.i2 + sdt * v2, n0, n1, n2);
  const T s0 = t.eval(cv, n1, n2) * n0;
  const T s1 = t.eval(cv + P, n1, n2) * n1;
  const T s2 = t.eval(cv + 2 * P, n1, n2) * n2;
  const T h = T(0.5) * sdt;
  disp[p] = h * (v0 + s0);
  disp[P + p] = h * (v1 + s1);
  disp[2 * P + p] = h * (v2 + s2);
}

template <typename T, int NF>
__global__ void k_interp(T* __restrict__ out, const T* __restrict__ c, const T* __restrict__ disp, int n0,
                         int n1, int n2) {
  const int64_t P = (int64_t)n0 * n1 * n2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const GridIdx g = unflatten(p, n1, n2);
  Taps<T> t;
  t.set(g.i0 + disp[p], g.i1 + disp[P + p], g.i2 + disp[2 * P + p], n0, n1, n2);
#pragma unroll
  for (int f = 0; f < NF; ++f) out[f * P + p] = t.eval(c + f * P, n1, n2);
}

// variant-1 adjoint (Table 1 row 2, -D_t lambda = lambda div v), one Heun step
template <typename T>
__global__ void k_adjoint_grid_step(T* __restrict__ out, const T* __restrict__ c1, const T* __restrict__ c2,
                                    const T* __restrict__ disp, const T* __restrict__ divv, int n0, int n1, int n2,
                                    T dt) {
  const int64_t P = (int64_t)n0 * n1 * n2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const GridIdx g = unflatten(p, n1, n2);
  Taps<T> t;
  t.set(g.i0 + disp[p], g.i1 + disp[P + p], g.i2 + disp[2 * P + p], n0, n1, n2);
  const T a = t.eval(c1, n1, n2), b = t.eval(c2, n1, n2);
  out[p] = a + T(0.5) * dt * (b + (a + dt * b) * divv[p]);
}

// band-limited adjoint step: out_f = cA_f o X + dt/2 divv (cB_f o X)
template <typename T, int NF>
__global__ void k_bl_adjoint_step(T* __restrict__ out, const T* __restrict__ cA, const T* __restrict__ cB,
                                  const T* __restrict__ disp, const T* __restrict__ divv, int n0, int n1, int n2,
                                  T dt) {
  const int64_t P = (int64_t)n0 * n1 * n2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const GridIdx g = unflatten(p, n1, n2);
  Taps<T> t;
  t.set(g.i0 + disp[p], g.i1 + disp[P + p], g.i2 + disp[2 * P + p], n0, n1, n2);
  const T hd = T(0.5) * dt * divv[p];
#pragma unroll
  for (int f = 0; f < NF; ++f) out[f * P + p] = t.eval(cA + f * P, n1, n2) + hd * t.eval(cB + f * P, n1, n2);
}

template <typename T>
__device__ __forceinline__ void v3_src_point(T o[3], const T* __restrict__ Du, const T* __restrict__ dv,
                                             int64_t p, int64_t P) {
  const T w0 = dv[p], w1 = dv[P + p], w2 = dv[2 * P + p];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T* D = Du + (int64_t)(3 * i) * P;  // d_j u_i at D[j * P]
    o[i] = (i == 0 ? w0 : (i == 1 ? w1 : w2)) - (D[p] * w0 + D[P + p] * w1 + D[2 * P + p] * w2);
  }
}

template <typename T>
__global__ void k_v3_source(T* __restrict__ out, const T* __restrict__ Du, const T* __restrict__ dv, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  T o[3];
  v3_src_point(o, Du, dv, p, P);
  out[p] = o[0];
  out[P + p] = o[1];
  out[2 * P + p] = o[2];
}

template <typename T>
__global__ void k_v1_source(T* __restrict__ out, const T* __restrict__ G, const T* __restrict__ dv, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  out[p] = -(G[p] * dv[p] + G[P + p] * dv[P + p] + G[2 * P + p] * dv[2 * P + p]);
}

template <typename T>
__global__ void k_v1_products(T* __restrict__ out, const T* __restrict__ e, const T* __restrict__ divv,
                              const T* __restrict__ G, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const T x = e[p];
  out[p] = x * divv[p];
  out[P + p] = x * G[p];
  out[2 * P + p] = x * G[P + p];
  out[3 * P + p] = x * G[2 * P + p];
}

template <typename T>
__global__ void k_v3_products(T* __restrict__ out, const T* __restrict__ e, const T* __restrict__ divv,
                              const T* __restrict__ Du, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const T r0 = e[p], r1 = e[P + p], r2 = e[2 * P + p], dv = divv[p];
  out[p] = r0 * dv;
  out[P + p] = r1 * dv;
  out[2 * P + p] = r2 * dv;
  // (Du)^T r: component j = sum_i r_i d_j u_i, Du[(3 i + j) P]
#pragma unroll
  for (int j = 0; j < 3; ++j)
    out[(3 + j) * P + p] = r0 * Du[(0 + j) * P + p] + r1 * Du[(3 + j) * P + p] + r2 * Du[(6 + j) * P + p];
}

// Transformation of a grid field through per-node maps (state-equation variant, Section 2.3.2):
// out_n(x) = a w_n(x) P(c)(x - u_n(x)), n = blockIdx.y, with u_n a displacement in unit-torus units
// ([n][3][P]) and w_n an optional weight field ([n][P]).  One gather of the 64 taps per node: the
// displacements here are whole deformations, not one step's, so no brick around the node holds them.
template <typename T>
__global__ void k_pull_back(T* __restrict__ out, const T* __restrict__ c, const T* __restrict__ u,
                            const T* __restrict__ w, T a, int n0, int n1, int n2) {
  const int64_t P = (int64_t)n0 * n1 * n2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t node = blockIdx.y;
  const T* un = u + node * 3 * P;
  const GridIdx g = unflatten(p, n1, n2);
  Taps<T> t;
  t.set(g.i0 - un[p] * n0, g.i1 - un[P + p] * n1, g.i2 - un[2 * P + p] * n2, n0, n1, n2);
  T r = a * t.eval(c, n1, n2);
  if (w) r *= w[node * P + p];
  out[node * P + p] = r;
}

// out_j = sum_n e_n G_n,j (e [ns][P], G [ns][3][P]): the time integral of the state-equation variant's
// gradient and Hessian terms on the product grid, its weights folded into e_n
template <typename T>
__global__ void k_node_sum(T* __restrict__ out, const T* __restrict__ e, const T* __restrict__ G, int ns, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  T a0 = 0, a1 = 0, a2 = 0;
  for (int n = 0; n < ns; ++n) {
    const T x = e[n * P + p];
    const T* g = G + 3 * n * P;
    a0 += x * g[p];
    a1 += x * g[P + p];
    a2 += x * g[2 * P + p];
  }
  out[p] = a0;
  out[P + p] = a1;
  out[2 * P + p] = a2;
}

// Right-hand sides of the explicit RK comparator (deformation-state equations in Eulerian form) on the
// product grid, where the truncated products are exact:
//   adjoint:            out_i = -(sum_j d_j r_i v_j + r_i div v)   (the product rule of -div(r_i v))
//   incremental state:  out_i = dv_i - sum_j d_j du_i v_j - sum_j (a Du_a + b Du_b)_ij dv_j
// (D fields [i][j] = d_j x_i, 9 per vector)
template <typename T>
__global__ void k_rk_adjoint_rhs(T* __restrict__ out, const T* __restrict__ Dr, const T* __restrict__ r,
                                 const T* __restrict__ v, const T* __restrict__ divv, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const T v0 = v[p], v1 = v[P + p], v2 = v[2 * P + p], dv = divv[p];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T* D = Dr + 3 * i * P;
    out[i * P + p] = -(D[p] * v0 + D[P + p] * v1 + D[2 * P + p] * v2 + r[i * P + p] * dv);
  }
}

template <typename T>
__global__ void k_rk_inc_rhs(T* __restrict__ out, const T* __restrict__ Ddu, const T* __restrict__ Dua,
                             const T* __restrict__ Dub, T a, T b, const T* __restrict__ v, const T* __restrict__ dv,
                             int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const T v0 = v[p], v1 = v[P + p], v2 = v[2 * P + p];
  const T w0 = dv[p], w1 = dv[P + p], w2 = dv[2 * P + p];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T* D = Ddu + 3 * i * P;
    const T* A = Dua + 3 * i * P;
    const T* B = Dub + 3 * i * P;
    const T u0 = a * A[p] + b * B[p], u1 = a * A[P + p] + b * B[P + p], u2 = a * A[2 * P + p] + b * B[2 * P + p];
    out[i * P + p] = dv[i * P + p] - (D[p] * v0 + D[P + p] * v1 + D[2 * P + p] * v2) - (u0 * w0 + u1 * w1 + u2 * w2);
  }
}

template <typename T>
__global__ void k_band_copy(T* __restrict__ out, int o0, int o1, int o2, const T* __restrict__ in, int i0, int i1,
                            int i2, int m0, int m1, int m2, int ncomp, bool keep_rest) {
  const int64_t Qo = (int64_t)o0 * o1 * o2;
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= ncomp * Qo) return;
  const int c = static_cast<int>(q / Qo);
  const int64_t r = q - c * Qo;
  const int a2 = static_cast<int>(r % o2), a1 = static_cast<int>((r / o2) % o1), a0 = static_cast<int>(r / ((int64_t)o1 * o2));
  if (a0 < m0 && a1 < m1 && a2 < m2)
    out[q] = in[(int64_t)c * i0 * i1 * i2 + ((int64_t)a0 * i1 + a1) * i2 + a2];
  else if (!keep_rest)
    out[q] = T(0);
}

template <typename T>
__global__ void k_restrict_grid(T* __restrict__ out, const T* __restrict__ in, int n0, int n1, int n2, int f0,
                                int f1, int f2) {
  const int c0 = n0 / f0, c1 = n1 / f1, c2 = n2 / f2;
  const int64_t Pc = (int64_t)c0 * c1 * c2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= Pc) return;
  const GridIdx g = unflatten(p, c1, c2);
  T acc = 0;
  for (int a = 0; a < f0; ++a)
    for (int b = 0; b < f1; ++b)
      for (int e = 0; e < f2; ++e)
        acc += in[((int64_t)(g.i0 * f0 + a) * n1 + (g.i1 * f1 + b)) * n2 + (g.i2 * f2 + e)];
  out[p] = acc / T(f0 * f1 * f2);
}

template <typename T>
__global__ void k_final_warp(T* __restrict__ m1, T* __restrict__ g1, const T* __restrict__ cI0,
                             const T* __restrict__ u, int n0, int n1, int n2) {
  const int64_t P = (int64_t)n0 * n1 * n2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const GridIdx g = unflatten(p, n1, n2);
  int i0[4], i1[4], i2[4];
  T w0[4], w1[4], w2[4], d0[4], d1[4], d2[4];
  const T t0 = tap_indices(g.i0 - u[p] * n0, n0, i0);
  const T t1 = tap_indices(g.i1 - u[P + p] * n1, n1, i1);
  const T t2 = tap_indices(g.i2 - u[2 * P + p] * n2, n2, i2);
  bspline_weights(t0, w0);
  bspline_weights(t1, w1);
  bspline_weights(t2, w2);
  bspline_dweights(t0, d0);
  bspline_dweights(t1, d1);
  bspline_dweights(t2, d2);
  T val = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T sv = 0, sy = 0, sz = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const T* row = cI0 + (static_cast<int64_t>(i0[a]) * n1 + i1[b]) * n2;
      const T r0 = row[i2[0]], r1 = row[i2[1]], r2 = row[i2[2]], r3 = row[i2[3]];
      const T s = w2[0] * r0 + w2[1] * r1 + w2[2] * r2 + w2[3] * r3;
      const T sd = d2[0] * r0 + d2[1] * r1 + d2[2] * r2 + d2[3] * r3;
      sv += w1[b] * s;
      sy += d1[b] * s;
      sz += w1[b] * sd;
    }
    val += w0[a] * sv;
    gx += d0[a] * sv;
    gy += w0[a] * sy;
    gz += w0[a] * sz;
  }
  m1[p] = val;
  g1[p] = gx * n0;
  g1[P + p] = gy * n1;
  g1[2 * P + p] = gz * n2;
}

template <typename T>
__global__ void k_scaled_diff(T* out, T a, const T* x, const T* y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * (x[i] - y[i]);
}

template <typename T>
__global__ void k_residual_times_grad(T* out, T a, const T* x, const T* y, const T* g1, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const T r = a * (x[p] - y[p]);
  out[p] = r * g1[p];
  out[P + p] = r * g1[P + p];
  out[2 * P + p] = r * g1[2 * P + p];
}

template <typename T>
__global__ void k_coupling_v3(T* out, T a, const T* g1, const T* w, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  const T s = a * (g1[p] * w[p] + g1[P + p] * w[P + p] + g1[2 * P + p] * w[2 * P + p]);
  out[p] = s * g1[p];
  out[P + p] = s * g1[P + p];
  out[2 * P + p] = s * g1[2 * P + p];
}

template <typename T>
__global__ void k_mul(T* out, const T* x, const T* y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i] * y[i];
}

template <typename T>
__global__ void k_copy(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <typename T>
__global__ void k_zero(T* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

template <typename T>
__global__ void k_jacobian(double* out, const T* Du, int64_t P) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - static_cast<double>(Du[(3 * i + j) * P + p]);
  out[p] = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// ---- periodic cubic B-spline prefilter -----------------------------------------
// Interpolating coefficients c of samples f solve (c[i-1] + 4 c[i] + c[i+1]) / 6 = f[i]
// on a periodic line.  The inverse filter factors into a causal and an anti-causal
// first-order recursion with pole z = sqrt(3) - 2 and gain 6; the periodic start
// values are the geometrically weighted wrap-around sums (truncated where z^h is
// below the working precision).
template <typename T>
struct Pole {
  static constexpr double z = -0.26794919243112270647255365849413;  // sqrt(3) - 2
  static constexpr int horizon = sizeof(T) == 4 ? 16 : 32;
};

template <typename T>
__device__ void filter_line(T* f, int64_t stride, int n) {
  const double z = Pole<T>::z;
  const int h = n < Pole<T>::horizon ? n : Pole<T>::horizon;
  double zn = 1.0;
  for (int i = 0; i < n; ++i) zn *= z;
  const double inv = 1.0 / (1.0 - zn);
  // causal start: sum_i z^i x[-i], x = 6 f
  double acc = 0.0, zi = 1.0;
  for (int i = 0; i < h; ++i) {
    const int j = (n - i) % n;
    acc += zi * 6.0 * static_cast<double>(f[j * stride]);
    zi *= z;
  }
  double prev = acc * inv;
  f[0] = static_cast<T>(prev);
  for (int k = 1; k < n; ++k) {
    prev = 6.0 * static_cast<double>(f[k * stride]) + z * prev;
    f[k * stride] = static_cast<T>(prev);
  }
  // anti-causal start: -z/(1-z^n) sum_i z^i y+[n-1+i]
  acc = 0.0;
  zi = 1.0;
  for (int i = 0; i < h; ++i) {
    const int j = (n - 1 + i) % n;
    acc += zi * static_cast<double>(f[j * stride]);
    zi *= z;
  }
  prev = -z * inv * acc;
  f[(n - 1) * stride] = static_cast<T>(prev);
  for (int k = n - 2; k >= 0; --k) {
    prev = z * (prev - static_cast<double>(f[k * stride]));
    f[k * stride] = static_cast<T>(prev);
  }
}

// lines along axis 0 or 1: one thread per line, lanes on consecutive n2 indices (coalesced)
template <typename T>
__global__ void k_prefilter_outer(T* f, int n0, int n1, int n2, int axis, int64_t lines_per_field,
                                  int64_t P, int nf) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= lines_per_field * nf) return;
  const int fld = static_cast<int>(t / lines_per_field);
  const int64_t l = t - fld * lines_per_field;
  T* base = f + fld * P;
  if (axis == 0) {  // lines indexed by (i1, i2)
    filter_line(base + l, (int64_t)n1 * n2, n0);
  } else {  // lines indexed by (i0, i2)
    const int64_t i0 = l / n2, i2 = l % n2;
    filter_line(base + i0 * n1 * n2 + i2, (int64_t)n2, n1);
  }
}

// lines along the contiguous axis: stage up to 64 rows through LDS so global accesses stay coalesced
template <typename T>
__global__ void k_prefilter_inner(T* f, int n2, int64_t rows, int rpb) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int ld = n2 + 1;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int nr = static_cast<int>(rows - r0 < rpb ? rows - r0 : rpb);
  for (int e = threadIdx.x; e < nr * n2; e += blockDim.x) {
    const int r = e / n2, c = e - r * n2;
    sm[r * ld + c] = f[(r0 + r) * n2 + c];
  }
  __syncthreads();
  if (threadIdx.x < nr) filter_line(sm + threadIdx.x * ld, 1, n2);
  __syncthreads();
  for (int e = threadIdx.x; e < nr * n2; e += blockDim.x) {
    const int r = e / n2, c = e - r * n2;
    f[(r0 + r) * n2 + c] = sm[r * ld + c];
  }
}

// chunk-parallel form for lines of at most kChunkMaxN points: a block stages 32 lines in LDS,
// 8 threads per line each own one chunk; a chunk starts its causal (anti-causal) recursion from
// the truncated geometric sum over the horizon points before (after) it, the same truncation
// as the serial start values, so every chunk runs independently.
constexpr int kChunkLines = 32, kChunkGroups = 8, kChunkMaxC = 24, kChunkMaxN = kChunkGroups * kChunkMaxC;

template <typename T>
__global__ __launch_bounds__(256) void k_prefilter_chunked(T* f, int n, int64_t gl, int64_t gi, int nlines_max,
                                                           int64_t tile_stride_a, int tiles_a, int64_t tile_stride_b,
                                                           int64_t P, double inv) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);  // [n][33]: element (line l, point i) at i * 33 + l
  constexpr int ld = kChunkLines + 1;
  // block -> (field, outer index b, tile of 32 lines a)
  const int ta = blockIdx.x % tiles_a;
  const int64_t tb = blockIdx.x / tiles_a;
  T* base = f + blockIdx.y * P + tb * tile_stride_b + (int64_t)ta * kChunkLines * tile_stride_a;
  const int nl = min(kChunkLines, nlines_max - ta * kChunkLines);
  const int tid = threadIdx.x;
  const bool line_major = gi == 1;  // points of a line contiguous in memory
  // the tile is walked line by line (points contiguous) or point by point (lines contiguous), its
  // loads batched ahead of the LDS stores and its indices advanced without integer division; the
  // element offsets stay below 2^31 (a tile spans at most 32 lines of 192 points of one field)
  const int rows = line_major ? kChunkLines : n, cols = line_major ? n : kChunkLines;
  const int gstride = static_cast<int>(line_major ? gl : gi);
  {
    constexpr int U = 8;
    TileWalk w(256, tid, cols, gstride, 0);
    while (w.r < rows) {
      const TileWalk w0 = w;
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int l = line_major ? w.r : w.c;
        const bool ok = w.r < rows && l < nl;
        const T t = base[ok ? w.o1 : 0];
        v[u] = ok ? t : T(0);
        w.next();
      }
      w = w0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int l = line_major ? w.r : w.c, i = line_major ? w.c : w.r;
        if (w.r < rows) sm[i * ld + l] = v[u];
        w.next();
      }
    }
  }
  __syncthreads();
  const double z = Pole<T>::z;  // inv = 1 / (1 - z^n), from the host
  const int h = n < Pole<T>::horizon ? n : Pole<T>::horizon;
  const int l = tid % kChunkLines, g = tid / kChunkLines;
  const int Lc = (n + kChunkGroups - 1) / kChunkGroups;
  const int c0 = g * Lc, c1 = min(n, c0 + Lc);
  double cp[kChunkMaxC];
  // causal: c+[i] = 6 f[i] + z c+[i-1]
  {
    double acc = 0.0, zi = 1.0;
    for (int k = 0; k < h; ++k) {
      int j = c0 - k;  // periodic: k < h <= n, one wrap at most
      if (j < 0) j += n;
      acc += zi * 6.0 * static_cast<double>(sm[j * ld + l]);
      zi *= z;
    }
    double prev = acc * inv;
#pragma unroll
    for (int q = 0; q < kChunkMaxC; ++q) {
      const int i = c0 + q;
      if (i < c1) {
        if (q > 0) prev = 6.0 * static_cast<double>(sm[i * ld + l]) + z * prev;
        cp[q] = prev;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kChunkMaxC; ++q)
    if (c0 + q < c1) sm[(c0 + q) * ld + l] = static_cast<T>(cp[q]);
  __syncthreads();
  // anti-causal: c[i] = z (c[i+1] - c+[i]), started at the chunk's last point
  {
    const int e = c1 - 1;
    double acc = 0.0, zi = 1.0;
    for (int k = 0; k < h; ++k) {
      const int j = e + k < n ? e + k : e + k - n;
      acc += zi * static_cast<double>(sm[j * ld + l]);
      zi *= z;
    }
    double prev = -z * inv * acc;
#pragma unroll
    for (int q = kChunkMaxC - 1; q >= 0; --q) {
      const int i = c0 + q;
      if (i < c1) {
        if (i < e) prev = z * (prev - static_cast<double>(sm[i * ld + l]));
        cp[q] = prev;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kChunkMaxC; ++q)
    if (c0 + q < c1) sm[(c0 + q) * ld + l] = static_cast<T>(cp[q]);
  __syncthreads();
  for (TileWalk w(256, tid, cols, gstride, 0); w.r < rows; w.next()) {
    const int ll = line_major ? w.r : w.c, i = line_major ? w.c : w.r;
    if (ll < nl) base[w.o1] = sm[i * ld + ll];
  }
}

inline dim3 grid_for(int64_t n) { return dim3(ceil_div(n, kBlock)); }

}  // namespace

// ---- launchers -----------------------------------------------------------------

template <typename T>
void bl_axpby(T* out, T a, const T* x, T b, const T* y, int64_t n, hipStream_t s) {
  prof::launch(std::string("k_axpby<") + prof::tname<T>() + ">", (y ? 3.0 : 2.0) * n * sizeof(T), 0.0, k_axpby<T>, grid_for(n), dim3(kBlock), 0, s, out, a, x, b, y, n);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void bl_scale_sym(T* out, const T* x, const double* sym, int ncomp, int64_t Q, const T* y, hipStream_t s) {
  prof::launch(std::string("k_scale_sym<") + prof::tname<T>() + ">", 3.0 * Q * ncomp * sizeof(T), 0.0, k_scale_sym<T>, grid_for(Q * ncomp), dim3(kBlock), 0, s, out, x, sym, ncomp, Q, y);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void bl_div(T* out, const T* v, const Dims& d, hipStream_t s) {
  prof::launch(std::string("k_bl_div<") + prof::tname<T>() + ">", 4.0 * d.Q * sizeof(T), 0.0, k_bl_div<T>, grid_for(d.Q), dim3(kBlock), 0, s, out, v, d.k[0], d.k[1], d.k[2]);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void characteristics(T* disp, const T* v, const T* cv, const Dims& d, T dt, int dir, hipStream_t s) {
  if constexpr (std::is_same_v<T, float>) {
    if (brick_ok(d)) return brick_characteristics(disp, v, cv, d, dt, dir, s);
  }
  prof::launch("k_characteristics<" + std::string(prof::tname<T>()) + ">", 9.0 * d.P * sizeof(T), 0.0, k_characteristics<T>, grid_for(d.P), dim3(kBlock), 0, s, disp, v, cv, d.n[0], d.n[1], d.n[2], dt, dir);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void interp(T* out, const T* coef, int nf, const T* disp, const Dims& d, hipStream_t s) {
  if constexpr (std::is_same_v<T, float>) {
    if (brick_ok(d) && (nf == 1 || nf == 3)) return brick_interp(out, coef, nf, disp, d, s);
  }
  switch (nf) {
    case 1:
      prof::launch("k_interp<" + std::string(prof::tname<T>()) + "," + std::to_string(nf) + ">", (3.0 + 2.0 * nf) * d.P * sizeof(T), 0.0, k_interp<T, 1>, grid_for(d.P), dim3(kBlock), 0, s, out, coef, disp, d.n[0], d.n[1], d.n[2]);
      break;
    case 2:
      prof::launch("k_interp<" + std::string(prof::tname<T>()) + "," + std::to_string(nf) + ">", (3.0 + 2.0 * nf) * d.P * sizeof(T), 0.0, k_interp<T, 2>, grid_for(d.P), dim3(kBlock), 0, s, out, coef, disp, d.n[0], d.n[1], d.n[2]);
      break;
    case 3:
      prof::launch("k_interp<" + std::string(prof::tname<T>()) + "," + std::to_string(nf) + ">", (3.0 + 2.0 * nf) * d.P * sizeof(T), 0.0, k_interp<T, 3>, grid_for(d.P), dim3(kBlock), 0, s, out, coef, disp, d.n[0], d.n[1], d.n[2]);
      break;
    default:
      throw ArgError("interp: nf must be 1..3");
  }
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void prefilter(T* f, int nf, const Dims& d, hipStream_t s) {
  const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
  const std::string nm = std::string("k_prefilter_chunked<") + prof::tname<T>() + ">";
  // lines of `n` points at element stride gi; 32 consecutive lines (stride gl) per tile, tiles
  // along the line index a, outer index b
  auto chunked = [&](int n, int64_t gl, int64_t gi, int nlines_a, int64_t stride_b, int nb) {
    const int tiles_a = ceil_div(nlines_a, kChunkLines);
    const uint32_t sm = (uint32_t)((size_t)n * (kChunkLines + 1) * sizeof(T));
    double zn = 1.0;
    for (int i = 0; i < n; ++i) zn *= Pole<T>::z;
    prof::launch(nm, 2.0 * nf * d.P * sizeof(T), 0.0, k_prefilter_chunked<T>, dim3(tiles_a * nb, nf), dim3(256),
                 sm, s, f, n, gl, gi, nlines_a, gl, tiles_a, stride_b, d.P, 1.0 / (1.0 - zn));
    LDDMM_LAUNCH_CHECK();
  };
  if (n2 > 1) {
    if (n2 <= kChunkMaxN) {
      // lines along axis 2: tiles of 32 consecutive rows x1 at fixed x0
      chunked(n2, (int64_t)n2, 1, n1, (int64_t)n1 * n2, n0);
    } else {
      const int64_t rows = (int64_t)nf * n0 * n1;
      int rpb = static_cast<int>(49152 / ((size_t)(n2 + 1) * sizeof(T)));
      rpb = rpb > 64 ? 64 : rpb;
      if (rpb < 1) throw ArgError("prefilter: grid line too long");
      const size_t sm = (size_t)rpb * (n2 + 1) * sizeof(T);
      prof::launch(std::string("k_prefilter_inner<") + prof::tname<T>() + ">", 2.0 * rows * n2 * sizeof(T), 0.0,
                   k_prefilter_inner<T>, dim3(ceil_div(rows, rpb)), dim3(64), (uint32_t)sm, s, f, n2, rows, rpb);
      LDDMM_LAUNCH_CHECK();
    }
  }
  if (n1 > 1) {
    if (n1 <= kChunkMaxN) {
      // lines along axis 1: tiles of 32 consecutive x2 at fixed x0
      chunked(n1, 1, (int64_t)n2, n2, (int64_t)n1 * n2, n0);
    } else {
      const int64_t lines = (int64_t)n0 * n2;
      prof::launch(std::string("k_prefilter_outer<") + prof::tname<T>() + ">", 2.0 * nf * d.P * sizeof(T), 0.0,
                   k_prefilter_outer<T>, grid_for(lines * nf), dim3(kBlock), 0, s, f, n0, n1, n2, 1, lines, d.P, nf);
      LDDMM_LAUNCH_CHECK();
    }
  }
  if (n0 > 1) {
    if (n0 <= kChunkMaxN) {
      // lines along axis 0: tiles of 32 consecutive x2 at fixed x1
      chunked(n0, 1, (int64_t)n1 * n2, n2, (int64_t)n2, n1);
    } else {
      const int64_t lines = (int64_t)n1 * n2;
      prof::launch(std::string("k_prefilter_outer<") + prof::tname<T>() + ">", 2.0 * nf * d.P * sizeof(T), 0.0,
                   k_prefilter_outer<T>, grid_for(lines * nf), dim3(kBlock), 0, s, f, n0, n1, n2, 0, lines, d.P, nf);
      LDDMM_LAUNCH_CHECK();
    }
  }
}

template <typename T>
void adjoint_grid_step(T* out, const T* c1, const T* c2, const T* disp, const T* divv, const Dims& d, T dt,
                       hipStream_t s) {
  if constexpr (std::is_same_v<T, float>) {
    if (brick_ok(d) && c2 == c1 + d.P) return brick_adjoint_grid_step(out, c1, disp, divv, d, dt, s);
  }
  prof::launch("k_adjoint_grid_step<" + std::string(prof::tname<T>()) + ">", 7.0 * d.P * sizeof(T), 0.0, k_adjoint_grid_step<T>, grid_for(d.P), dim3(kBlock), 0, s, out, c1, c2, disp, divv, d.n[0], d.n[1], d.n[2], dt);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void bl_adjoint_step(T* out, const T* cA, const T* cB, int nf, const T* disp, const T* divv, const Dims& d, T dt,
                     hipStream_t s) {
  if constexpr (std::is_same_v<T, float>) {
    if (brick_ok(d) && cB == cA + nf * d.P) return brick_bl_adjoint_step(out, cA, nf, disp, divv, d, dt, s);
  }
  if (nf == 1)
    prof::launch("k_bl_adjoint_step<" + std::string(prof::tname<T>()) + "," + std::to_string(nf) + ">", (4.0 + 3.0 * nf) * d.P * sizeof(T), 0.0, k_bl_adjoint_step<T, 1>, grid_for(d.P), dim3(kBlock), 0, s, out, cA, cB, disp, divv, d.n[0], d.n[1], d.n[2], dt);
  else if (nf == 3)
    prof::launch("k_bl_adjoint_step<" + std::string(prof::tname<T>()) + "," + std::to_string(nf) + ">", (4.0 + 3.0 * nf) * d.P * sizeof(T), 0.0, k_bl_adjoint_step<T, 3>, grid_for(d.P), dim3(kBlock), 0, s, out, cA, cB, disp, divv, d.n[0], d.n[1], d.n[2], dt);
  else
    throw ArgError("bl_adjoint_step: nf must be 1 or 3");
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void v3_source(T* out, const T* Du, const T* dv, const Dims& d, hipStream_t s) {
  prof::launch("k_v3_source<" + std::string(prof::tname<T>()) + ">", 15.0 * d.P * sizeof(T), 0.0, k_v3_source<T>, grid_for(d.P), dim3(kBlock), 0, s, out, Du, dv, d.P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void v1_source(T* out, const T* G, const T* dv, const Dims& d, hipStream_t s) {
  prof::launch("k_v1_source<" + std::string(prof::tname<T>()) + ">", 7.0 * d.P * sizeof(T), 0.0, k_v1_source<T>, grid_for(d.P), dim3(kBlock), 0, s, out, G, dv, d.P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void v1_products(T* out, const T* e, const T* divv, const T* G, const Dims& d, hipStream_t s) {
  prof::launch("k_v1_products<" + std::string(prof::tname<T>()) + ">", 9.0 * d.P * sizeof(T), 0.0, k_v1_products<T>, grid_for(d.P), dim3(kBlock), 0, s, out, e, divv, G, d.P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void v3_products(T* out, const T* e, const T* divv, const T* Du, const Dims& d, hipStream_t s) {
  prof::launch("k_v3_products<" + std::string(prof::tname<T>()) + ">", 19.0 * d.P * sizeof(T), 0.0, k_v3_products<T>, grid_for(d.P), dim3(kBlock), 0, s, out, e, divv, Du, d.P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void final_warp(T* m1, T* g1, const T* cI0, const T* u, const Dims& d, hipStream_t s) {
  prof::launch("k_final_warp<" + std::string(prof::tname<T>()) + ">", 8.0 * d.P * sizeof(T), 0.0, k_final_warp<T>, grid_for(d.P), dim3(kBlock), 0, s, m1, g1, cI0, u, d.n[0], d.n[1], d.n[2]);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void pull_back(T* out, const T* c, const T* u, const T* w, T a, int nodes, const Dims& d, hipStream_t s) {
  if (nodes < 1 || nodes > 65535) throw ArgError("pull_back: node count out of range");
  const dim3 g(static_cast<unsigned>((d.P + kBlock - 1) / kBlock), static_cast<unsigned>(nodes));
  prof::launch("k_pull_back<" + std::string(prof::tname<T>()) + ">",
               double(nodes) * (w ? 5.0 : 4.0) * d.P * sizeof(T) + d.P * sizeof(T), 0.0, k_pull_back<T>, g,
               dim3(kBlock), 0, s, out, c, u, w, a, d.n[0], d.n[1], d.n[2]);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void node_sum(T* out, const T* e, const T* G, int ns, int64_t P, hipStream_t s) {
  prof::launch("k_node_sum<" + std::string(prof::tname<T>()) + ">", (4.0 * ns + 3.0) * P * sizeof(T), 0.0,
               k_node_sum<T>, grid_for(P), dim3(kBlock), 0, s, out, e, G, ns, P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void rk_adjoint_rhs(T* out, const T* Dr, const T* r, const T* v, const T* divv, int64_t P, hipStream_t s) {
  prof::launch("k_rk_adjoint_rhs<" + std::string(prof::tname<T>()) + ">", 20.0 * P * sizeof(T), 0.0,
               k_rk_adjoint_rhs<T>, grid_for(P), dim3(kBlock), 0, s, out, Dr, r, v, divv, P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void rk_inc_rhs(T* out, const T* Ddu, const T* Dua, const T* Dub, T a, T b, const T* v, const T* dv, int64_t P,
                hipStream_t s) {
  prof::launch("k_rk_inc_rhs<" + std::string(prof::tname<T>()) + ">", 39.0 * P * sizeof(T), 0.0, k_rk_inc_rhs<T>,
               grid_for(P), dim3(kBlock), 0, s, out, Ddu, Dua, Dub, a, b, v, dv, P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void band_copy(T* out, const int ko[3], const T* in, const int ki[3], const int m[3], int ncomp, bool keep_rest,
               hipStream_t s) {
  const int64_t n = (int64_t)ncomp * ko[0] * ko[1] * ko[2];
  for (int j = 0; j < 3; ++j)
    if (m[j] > ko[j] || m[j] > ki[j]) throw ArgError("band_copy: copy extent beyond a band");
  prof::launch("k_band_copy<" + std::string(prof::tname<T>()) + ">", 2.0 * n * sizeof(T), 0.0, k_band_copy<T>,
               grid_for(n), dim3(kBlock), 0, s, out, ko[0], ko[1], ko[2], in, ki[0], ki[1], ki[2], m[0], m[1], m[2],
               ncomp, keep_rest);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void restrict_grid(T* out, const T* in, const Dims& fine, hipStream_t s) {
  int f[3];
  for (int j = 0; j < 3; ++j) {
    f[j] = fine.n[j] > 1 ? 2 : 1;
    if (fine.n[j] % f[j]) throw ArgError("restrict_grid: odd grid size");
  }
  const int64_t Pc = fine.P / (f[0] * f[1] * f[2]);
  prof::launch("k_restrict_grid<" + std::string(prof::tname<T>()) + ">", 1.0 * (fine.P + Pc) * sizeof(T), 0.0,
               k_restrict_grid<T>, grid_for(Pc), dim3(kBlock), 0, s, out, in, fine.n[0], fine.n[1], fine.n[2], f[0],
               f[1], f[2]);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void scaled_diff(T* out, T a, const T* x, const T* y, int64_t n, hipStream_t s) {
  prof::launch(std::string("k_scaled_diff<") + prof::tname<T>() + ">", 3.0 * n * sizeof(T), 0.0, k_scaled_diff<T>, grid_for(n), dim3(kBlock), 0, s, out, a, x, y, n);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void residual_times_grad(T* out, T a, const T* x, const T* y, const T* g1, const Dims& d, hipStream_t s) {
  prof::launch(std::string("k_residual_times_grad<") + prof::tname<T>() + ">", 6.0 * d.P * sizeof(T), 0.0, k_residual_times_grad<T>, grid_for(d.P), dim3(kBlock), 0, s, out, a, x, y, g1, d.P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void coupling_v3(T* out, T a, const T* g1, const T* w, const Dims& d, hipStream_t s) {
  prof::launch(std::string("k_coupling_v3<") + prof::tname<T>() + ">", 9.0 * d.P * sizeof(T), 0.0, k_coupling_v3<T>, grid_for(d.P), dim3(kBlock), 0, s, out, a, g1, w, d.P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void mul(T* out, const T* x, const T* y, int64_t n, hipStream_t s) {
  prof::launch(std::string("k_mul<") + prof::tname<T>() + ">", 3.0 * n * sizeof(T), 0.0, k_mul<T>, grid_for(n), dim3(kBlock), 0, s, out, x, y, n);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void jacobian_det(double* out, const T* Du, int dim, int64_t P, hipStream_t s) {
  (void)dim;
  prof::launch(std::string("k_jacobian<") + prof::tname<T>() + ">", 9.0 * P * sizeof(T) + 8.0 * P, 0.0, k_jacobian<T>, grid_for(P), dim3(kBlock), 0, s, out, Du, P);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void copy_dev(T* dst, const T* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  prof::launch(std::string("k_copy<") + prof::tname<T>() + ">", 2.0 * n * sizeof(T), 0.0, k_copy<T>, grid_for(n), dim3(kBlock), 0, s, dst, src, n);
  LDDMM_LAUNCH_CHECK();
}

template <typename T>
void zero(T* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  prof::launch(std::string("k_zero<") + prof::tname<T>() + ">", 1.0 * n * sizeof(T), 0.0, k_zero<T>, grid_for(n), dim3(kBlock), 0, s, p, n);
  LDDMM_LAUNCH_CHECK();
}

#define LDDMM_INST(T)                                                                                   \
  template void bl_axpby<T>(T*, T, const T*, T, const T*, int64_t, hipStream_t);                        \
  template void bl_scale_sym<T>(T*, const T*, const double*, int, int64_t, const T*, hipStream_t);      \
  template void bl_div<T>(T*, const T*, const Dims&, hipStream_t);                                      \
  template void characteristics<T>(T*, const T*, const T*, const Dims&, T, int, hipStream_t);           \
  template void interp<T>(T*, const T*, int, const T*, const Dims&, hipStream_t);                       \
  template void prefilter<T>(T*, int, const Dims&, hipStream_t);                                        \
  template void adjoint_grid_step<T>(T*, const T*, const T*, const T*, const T*, const Dims&, T,        \
                                     hipStream_t);                                                      \
  template void bl_adjoint_step<T>(T*, const T*, const T*, int, const T*, const T*, const Dims&, T,     \
                                   hipStream_t);                                                        \
  template void v3_source<T>(T*, const T*, const T*, const Dims&, hipStream_t);                         \
  template void v1_source<T>(T*, const T*, const T*, const Dims&, hipStream_t);                         \
  template void v1_products<T>(T*, const T*, const T*, const T*, const Dims&, hipStream_t);             \
  template void v3_products<T>(T*, const T*, const T*, const T*, const Dims&, hipStream_t);             \
  template void final_warp<T>(T*, T*, const T*, const T*, const Dims&, hipStream_t);                    \
  template void pull_back<T>(T*, const T*, const T*, const T*, T, int, const Dims&, hipStream_t);        \
  template void node_sum<T>(T*, const T*, const T*, int, int64_t, hipStream_t);                          \
  template void band_copy<T>(T*, const int*, const T*, const int*, const int*, int, bool, hipStream_t);   \
  template void restrict_grid<T>(T*, const T*, const Dims&, hipStream_t);                                 \
  template void rk_adjoint_rhs<T>(T*, const T*, const T*, const T*, const T*, int64_t, hipStream_t);      \
  template void rk_inc_rhs<T>(T*, const T*, const T*, const T*, T, T, const T*, const T*, int64_t,         \
                              hipStream_t);                                                              \
  template void scaled_diff<T>(T*, T, const T*, const T*, int64_t, hipStream_t);                        \
  template void residual_times_grad<T>(T*, T, const T*, const T*, const T*, const Dims&, hipStream_t);  \
  template void coupling_v3<T>(T*, T, const T*, const T*, const Dims&, hipStream_t);                    \
  template void mul<T>(T*, const T*, const T*, int64_t, hipStream_t);                                   \
  template void jacobian_det<T>(double*, const T*, int, int64_t, hipStream_t);                          \
  template void zero<T>(T*, int64_t, hipStream_t);                                                     \
  template void copy_dev<T>(T*, const T*, int64_t, hipStream_t);

LDDMM_INST(float)
LDDMM_INST(double)

}  // namespace lddmm
