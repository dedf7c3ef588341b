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

// plane-wise truncated DFT (dft_planes.hip), float.  Plane-band arrays are [x0][a1][a2] with
// C = K1 K2 columns per grid plane.
// expansion of planes: out[f][x0][x1][x2] = sum_{a1,a2} w1t_f[a1][x1] T_f[x0][a1][a2] w2t_f[a2][x2]
struct PlaneExpandArgs {
  const float* T[kMaxFields];    // [n0][k1][k2] per field
  const float* w1t[kMaxFields];  // [k1][n1]
  const float* w2t[kMaxFields];  // [k2][n2]
  float* out;                    // [nf][n0][n1][n2]
  int nf, n0, n1, n2, k1, k2;
};
// reduction of planes: part[f][x0][a1][a2] = sum_{x1,x2} p1t[x1][a1] v_f(x0, x1, x2) p2t[x2][a2], with the
// grid value v_f of the mode: a plain field, or a pointwise product of fields of the product grid
enum { kRedPlain = 0, kRedV1Products = 1, kRedV3Products = 2, kRedV1Source = 3, kRedV3Source = 4 };
struct PlaneReduceArgs {
  const float* in;    // plain: [nf][P]
  const float* e;     // products: e (1 or 3 fields); sources: dv (3 fields)
  const float* divv;  // products: div v
  const float* G;     // v1 products: G_n [3]; v3 products: D u_n [9]; sources: all nodes [nn][3] / [nn][9]
  const float* p1t;   // [n1][k1]
  const float* p2t;   // [n2][k2]
  float* part;        // [nf][n0][k1][k2]
  int mode, nf, n0, n1, n2, k1, k2;
  int64_t P;          // grid points per field
  int64_t e_node;     // sources: offset of node n's dv (0: one dv for every node; 3 P: a dv per node)
};
// expansion of e~ (T, 1 or 3 components) and reduction of its products with node fields in one pass
// per plane (product grid): part[f][x0] as PlaneReduceArgs in the modes kRedV1Products / kRedV3Products
struct ProdPlaneArgs {
  const float* T[3];  // [n0][k1][k2] per component of e~
  const float* w1t;   // [k1][n1]
  const float* w2t;   // [k2][n2]
  const float* divv;  // div v
  const float* G;     // v1: G_n [3]; v3: D u_n [9]
  const float* p1t;   // [n1][k1]
  const float* p2t;   // [n2][k2]
  float* part;        // [nf][n0][k1][k2]
  int mode, n0, n1, n2, k1, k2;
  int64_t P;
};
// first-axis stages (see dft_planes.hip): F finishes nin projections, P forms nout plane-band arrays
struct Axis0Out {
  const float* w0t;  // [k0][n0t] first-axis expansion matrix of the target grid
  float* T;         // [n0t][C]
  int n0t;
  int s1, s2;       // finished fields of F used as sources (-1: none)
  const float* g1;  // band arrays used as sources (null: none)
  const float* g2;
  float c1, c2;     // source = c1 (s1 + g1) + c2 (s2 + g2)
};
struct Axis0Args {
  const float* part[kMaxFields];  // [n0][C]
  const float* p0t;               // [n0][k0]
  float* out[kMaxFields];         // [k0][C]: out = alpha r + beta in + gamma z + ysym y
  const float* in[kMaxFields];    // optional (default: out)
  float* out2[kMaxFields];        // optional copy of out, scaled by s2 (0: 1)
  const float* z[kMaxFields];     // optional
  const float* y[kMaxFields];     // optional, weighted by the per-coefficient symbol ysym
  const double* ysym[kMaxFields];
  float alpha[kMaxFields], beta[kMaxFields], gamma[kMaxFields], s2[kMaxFields];
  Axis0Out o[kMaxFields];
  int nin, nout, n0, k0, C;
  const float* zeros;  // >= k0 C zeros, read in place of absent sources
};
// kernel view of Axis0Args: one descriptor row per workgroup row (built by plane_axis0)
struct Axis0Kernel {
  static constexpr int kRows = 2 * kMaxFields;
  struct Field {
    const float* part;
    float* out;
    const float* in;
    float* out2;
    const float* z;
    const float* y;
    const double* ysym;
    float alpha, beta, gamma, s2;
  };
  struct Out {
    const float* w0t;
    float* T;
    const float* g1;
    const float* g2;
    float c1, c2, cf;
    int n0t;
  };
  struct Row {
    int f, np;
    Out p[2];
  };
  const float* p0t;
  int n0, k0, C;
  Field fld[kMaxFields];
  Row row[kRows];
};
bool planes_ok(const Dims& d);
void plane_expand(const PlaneExpandArgs& a, hipStream_t s);
void plane_reduce(const PlaneReduceArgs& a, hipStream_t s);
void plane_axis0(const Axis0Args& a, hipStream_t s);
bool prod_plane_ok(const Dims& d);
void plane_prod(const ProdPlaneArgs& a, hipStream_t s);

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
// out_n = a w_n P(c)(x - u_n) for nodes n < nodes: u [nodes][3][P] (unit-torus units), w [nodes][P] or null
template <typename T>
void pull_back(T* out, const T* c, const T* u, const T* w, T a, int nodes, const Dims& d, hipStream_t s);
// explicit RK comparator right-hand sides on the product grid (D fields [i][j] = d_j x_i):
// adjoint out_i = -(sum_j Dr_ij v_j + r_i divv); incremental state
// out_i = dv_i - sum_j Ddu_ij v_j - sum_j (a Dua + b Dub)_ij dv_j
template <typename T>
void rk_adjoint_rhs(T* out, const T* Dr, const T* r, const T* v, const T* divv, int64_t P, hipStream_t s);
template <typename T>
void rk_inc_rhs(T* out, const T* Ddu, const T* Dua, const T* Dub, T a, T b, const T* v, const T* dv, int64_t P,
                hipStream_t s);
// out [3][P] = sum_n e_n G_n (e [ns][P], G [ns][3][P])
template <typename T>
void node_sum(T* out, const T* e, const T* G, int ns, int64_t P, hipStream_t s);
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
int dft_cap_count();     // workgroup-cap candidates of the first-axis DFT launches
// times every brick tile shape on this grid (one- and two-field interpolations into `out` at a smooth
// synthetic sub-voxel displacement written to the scratch `disp`) and caches the fastest
void brick_autotune(float* out, const float* coef, float* disp, const Dims& d, hipStream_t s);
void brick_interp(float* out, const float* coef, int nf, const float* disp, const Dims& d, hipStream_t s);
// out_f = P(c_f) o X - P(c_f) at the nodes (nf 1 or 3)
void brick_interp_diff(float* out, const float* coef, int nf, const float* disp, const Dims& d, hipStream_t s);
// pull_back through LDS-staged bounding boxes of each tile's stencils (float, 3D grids)
void brick_pull_back(float* out, const float* c, const float* u, const float* w, float a, int nodes, const Dims& d,
                     hipStream_t s);
void brick_bl_adjoint_step(float* out, const float* cAB, int nc, const float* disp, const float* divv,
                           const Dims& d, float dt, hipStream_t s);
void brick_adjoint_grid_step(float* out, const float* c12, const float* disp, const float* divv, const Dims& d,
                             float dt, hipStream_t s);
void brick_characteristics(float* disp, const float* v, const float* cv, const Dims& d, float dt, int dir,
                           hipStream_t s);

// ---- FP64 reductions (reduce.hip) -------------------------------------------
// partial results go to `work` (device, >= reduce_work_size doubles); result to host
constexpr int kRedSlots = 32;  // device result slots of the asynchronous forms
int64_t reduce_work_size();
double* reduce_slots(double* work);
// PCG vector updates reading their scalars from the result slots (no host round trip):
// x += a p, r -= a Ap with a = slot[irz] / slot[ipap], skipped unless slot[ipap] > 0
template <typename T>
void pcg_step(T* x, T* r, const T* p, const T* Ap, double* work, int irz, int ipap, int64_t n, hipStream_t s);
// p = z + beta p, skipped unless slot[ipap] > 0: beta = slot[irzn] / slot[irz], or, with ixz >= 0 (flexible
// CG; slot[ixz] = r_new . z_old), beta = (slot[irzn] - slot[ixz]) / slot[irz]
template <typename T>
void pcg_dir(T* p, const T* z, double* work, int irz, int irzn, int ipap, int64_t n, hipStream_t s, int ixz = -1);
// band arrays [c][K0][K1][K2]: out = in on the slots a_j < m_j of every axis; the other slots of out are
// zeroed (keep_rest = false) or kept.  Restriction to a coarse band (out Kc, in K, m = Kc - 1 per axis with
// more than one slot) and its extension or overwrite of the fine band's low slots (out K, in Kc).
template <typename T>
void band_copy(T* out, const int ko[3], const T* in, const int ki[3], const int m[3], int ncomp, bool keep_rest,
               hipStream_t s);
// 2^d block means of a grid field (axes with one node are kept): out on the grid n / f, f_j = 2 or 1
template <typename T>
void restrict_grid(T* out, const T* in, const Dims& fine, hipStream_t s);
// z += sum_i (Minv c)_i Z_i with c_i = slot[ic + i] (device Minv r x r, Z r x n)
template <typename T>
void lowrank_add(T* z, const T* Z, const double* Minv, double* work, int ic, int r, int64_t n, hipStream_t s);
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
// Asynchronous forms: the result stays in result slot `slot` (0..kRedSlots-1) of `work` until fetch_async
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
