// Launchers of the gfx950 kernels (HIP device code lives in the .hip files).
#pragma once

#include "common.h"

namespace lddmm {

// ---- separable truncated DFT contractions (dft.hip) -------------------------
// left:  out[b][m][c] = sum_l W_f[m][l] in[b][l][c],   f = b / bpf, b < nb
// right: out[f][r][m] = sum_l in[f][r][l] W_f[m][l],   r < R, f < nf
template <typename T>
void dft_left(const T* in, T* out, const FieldMats<T>& W, int nb, int bpf, int M, int L, int C,
              int64_t sIb, int64_t sOb, hipStream_t s);
template <typename T>
void dft_right(const T* in, T* out, const FieldMats<T>& W, int nf, int R, int L, int Mo, hipStream_t s);

// bf16 hi/lo split variants (float in/out, bf16 matrix-core products, float accumulation)
void dft_left_bf16(const float* in, float* out, const FieldMats<float>& W, int nb, int bpf, int M, int L,
                   int C, int64_t sIb, int64_t sOb, hipStream_t s);
void dft_right_bf16(const float* in, float* out, const FieldMats<float>& W, int nf, int R, int L, int Mo,
                    hipStream_t s);

// fused inner-axis stages (dft_fused.hip), float
struct IotaABArgs {
  const float* x[kMaxFields];  // per-field band input [k0][k1][k2]
  const float* y[kMaxFields];  // optional second input (null: none); slab = x + alpha y
  float alpha[kMaxFields];
  const float* w1t[kMaxFields];  // axis-1 matrix transposed, [k1][n1]
  const float* w2t[kMaxFields];  // axis-2 matrix transposed, [k2][n2]
  float* out;                   // [nf][k0][n1][n2]
  int k0, k1, k2, n1, n2;
};
struct PiBAArgs {
  const float* in;  // [nf][k0][n1][n2]
  const float* p1t;  // axis-1 projection transposed, [n1][k1]
  const float* p2t;  // axis-2 projection transposed, [n2][k2]
  float* out[kMaxFields];  // per-field band output [k0][k1][k2]: out = beta out + alpha r
  float alpha[kMaxFields];
  float beta[kMaxFields];
  float* part;  // workspace: [nf][k0][pi_ba_splits(n1)][k1][k2] partial projections
  int k0, k1, k2, n1, n2;
};
bool fused_dft_ok(int n1, int n2, int k1, int k2);
int pi_ba_splits(int n1);
void iota_ab(const IotaABArgs& a, int nf, hipStream_t s);
void pi_ba(const PiBAArgs& a, int nf, hipStream_t s);

// fused image-transport backward grid pass (fused_back.hip), float
struct BackV1Args {
  const float* t2;    // [k0][C] inner-axis slab of iota(dl~), C = n1 n2
  const float* divv;  // [n0][C]
  const float* G;     // [3][n0][C]
  const float* B0;    // [n0][k0] axis-0 basis
  float* out;         // [4][k0][C] axis-0 projections of e divv, e G_0, e G_1, e G_2
  int n0, k0, C;
  float inv_n0;
};
bool back_v1_ok(int n0, int k0);
void back_v1(const BackV1Args& a, hipStream_t s);

// ---- band-limited coefficient kernels (grid.hip) ----------------------------
// out = a x + b y (n elements; y may be null when b == 0)
template <typename T>
void bl_axpby(T* out, T a, const T* x, T b, const T* y, int64_t n, hipStream_t s);
// out = x * sym (+ y), sym a per-coefficient symbol (double), repeated over ncomp components
template <typename T>
void bl_scale_sym(T* out, const T* x, const double* sym, int ncomp, int64_t Q, const T* y_or_null,
                  hipStream_t s);
// out[Q] = sum_j d_j v[j]  (spectral divergence in the real basis)
template <typename T>
void bl_div(T* out, const T* v, const Dims& d, hipStream_t s);

// ---- grid kernels (grid.hip) ------------------------------------------------
// departure displacements (grid units) of the characteristic scheme:
// X = x + dir dt/2 (v + v o (x + dir dt v)), v given in unit-torus units
template <typename T>
void characteristics(T* disp, const T* v, const T* cv, const Dims& d, T dt, int dir, hipStream_t s);
// out_f = P(c_f) o X, X = x + disp, for nf <= 3 coefficient fields
template <typename T>
void interp(T* out, const T* coef, int nf, const T* disp, const Dims& d, hipStream_t s);
// periodic cubic B-spline prefilter of nf fields, in place
template <typename T>
void prefilter(T* f, int nf, const Dims& d, hipStream_t s);
// variant-1 adjoint Heun step on the grid:
//   a = c1 o X, b = c2 o X, out = a + dt/2 (b + (a + dt b) divv)
template <typename T>
void adjoint_grid_step(T* out, const T* c1, const T* c2, const T* disp, const T* divv, const Dims& d, T dt,
                       hipStream_t s);
// band-limited adjoint Heun step for nf components:
//   out_f = cA_f o X + dt/2 divv (cB_f o X), cA = P(x + dt/2 f), cB = P(x + dt f)
template <typename T>
void bl_adjoint_step(T* out, const T* cA, const T* cB, int nf, const T* disp, const T* divv, const Dims& d,
                     T dt, hipStream_t s);
// variant-1 incremental state step: out0 = c o X, out1 = -G . dv
template <typename T>
// out[0] = c o X + hdt s, out[1] = s with s = -G . dv (the step's trapezoid sum and its source)
void inc_state_v1(T* out, const T* c, const T* disp, const T* G, const T* dv, T hdt, const Dims& d, hipStream_t s);
// variant-3 incremental state step: out[0..2] = c_f o X + hdt s_f, out[3..5] = s = dv - Du dv
template <typename T>
void inc_state_v3(T* out, const T* c, const T* disp, const T* Du, const T* dv, T hdt, const Dims& d, hipStream_t s);
// variant-3 state source at node n: out = dv - Du dv  (3 comps)
template <typename T>
void v3_source(T* out, const T* Du, const T* dv, const Dims& d, hipStream_t s);
// variant-1 source at node n: out = -G . dv
template <typename T>
void v1_source(T* out, const T* G, const T* dv, const Dims& d, hipStream_t s);
// products for the variant-1 backward sweeps: out = [e divv, e G0, e G1, e G2]
template <typename T>
void v1_products(T* out, const T* e, const T* divv, const T* G, const Dims& d, hipStream_t s);
// products for the variant-3 backward sweeps: out = [e_i divv (3), (Du)^T e (3)]
template <typename T>
void v3_products(T* out, const T* e, const T* divv, const T* Du, const Dims& d, hipStream_t s);
// variant-3 final warp: m1 = P(I0) o (x - u n), g1 = grad P(I0) o (.) in unit-torus units
template <typename T>
void final_warp(T* m1, T* g1, const T* cI0, const T* u, const Dims& d, hipStream_t s);
// out = a * (x - y)
template <typename T>
void scaled_diff(T* out, T a, const T* x, const T* y, int64_t n, hipStream_t s);
// out_i = a * r * g1_i  (3 comps), r = x - y
template <typename T>
void residual_times_grad(T* out, T a, const T* x, const T* y, const T* g1, const Dims& d, hipStream_t s);
// out_i = a * (g1 . w) * g1_i
template <typename T>
void coupling_v3(T* out, T a, const T* g1, const T* w, const Dims& d, hipStream_t s);
// out = x * y (elementwise, n)
template <typename T>
void mul(T* out, const T* x, const T* y, int64_t n, hipStream_t s);
// det(I - Du) in double from 9 derivative fields (T)
template <typename T>
void jacobian_det(double* out, const T* Du, int dim, int64_t P, hipStream_t s);
// p[0..n) = 0 and dst[0..n) = src[0..n) as kernels (safe inside captured graphs)
template <typename T>
void zero(T* p, int64_t n, hipStream_t s);
template <typename T>
void copy_dev(T* dst, const T* src, int64_t n, hipStream_t s);

// ---- LDS-brick interpolation, float 3D grids (brick.hip) ---------------------
bool brick_ok(const Dims& d);
int brick_tile_count();  // workgroup tile candidates of the brick kernels
// times every brick tile shape on this grid (one- and two-field interpolations into `out` at a smooth
// synthetic sub-voxel displacement written to the scratch `disp`) and caches the fastest
void brick_autotune(float* out, const float* coef, float* disp, const Dims& d, hipStream_t s);
void brick_interp(float* out, const float* coef, int nf, const float* disp, const Dims& d, hipStream_t s);
void brick_bl_adjoint_step(float* out, const float* cAB, int nc, const float* disp, const float* divv,
                           const Dims& d, float dt, hipStream_t s);
void brick_adjoint_grid_step(float* out, const float* c12, const float* disp, const float* divv, const Dims& d,
                             float dt, hipStream_t s);
void brick_inc_state_v1(float* out, const float* c, const float* disp, const float* G, const float* dv, float hdt,
                        const Dims& d, hipStream_t s);
void brick_inc_state_v3(float* out, const float* c, const float* disp, const float* Du, const float* dv, float hdt,
                        const Dims& d, hipStream_t s);
void brick_characteristics(float* disp, const float* v, const float* cv, const Dims& d, float dt, int dir,
                           hipStream_t s);

// ---- FP64 reductions (reduce.hip) -------------------------------------------
// partial results go to `work` (device, >= reduce_work_size doubles); result to host
int64_t reduce_work_size();
template <typename T>
double dot(const T* a, const T* b, int64_t n, double* work, double* host_pinned, hipStream_t s);
template <typename T>
double sqdiff(const T* a, const T* b, int64_t n, double* work, double* host_pinned, hipStream_t s);
template <typename T>
double maxabs(const T* a, int64_t n, double* work, double* host_pinned, hipStream_t s);
// sum_i sym_i x_i y_i over ncomp components of length Q (sym double)
template <typename T>
double sym_dot(const T* x, const T* y, const double* sym, int ncomp, int64_t Q, double* work,
               double* host_pinned, hipStream_t s);
void minmax_f64(const double* a, int64_t n, double* work, double* host_pinned2, hipStream_t s);
// Asynchronous forms: the result stays in result slot `slot` (0..7) of `work` until fetch_async
// copies slots 0 .. count-1 into pinned host memory on the stream; the values are valid once the
// stream has been synchronised.
enum class RedKind { Dot, SqDiff, MaxAbs };
template <typename T>
void reduce_launch(RedKind kind, const T* a, const T* b, int64_t n, double* work, int slot, hipStream_t s);
template <typename T>
void sym_dot_launch(const T* x, const T* y, const double* sym, int ncomp, int64_t Q, double* work, int slot,
                    hipStream_t s);
void fetch_async(double* work, double* host_pinned, int count, hipStream_t s);

}  // namespace lddmm
