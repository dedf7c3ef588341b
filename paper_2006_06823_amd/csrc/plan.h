// Truncated DFT plan of one grid (Section 2.2): the per-axis basis matrices of a
// grid/band pair and the staging buffers of the contractions, with iota (band ->
// grid) and pi (grid -> band) of several fields at once.
//
// The solver holds two plans over the same band: the image grid, where the
// semi-Lagrangian interpolations run, and a coarser product grid with
// N'_j >= 3 (K_j / 2 - 1) + 1 nodes per axis.  The product of two band-limited
// fields holds frequencies up to twice the band edge, so its projection on any
// grid of at least that many nodes is the exact truncated convolution a * b of
// the coefficient arrays (no alias reaches the band); the products of
// band-limited fields the sweeps need are formed there.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"

namespace lddmm {

// per-axis matrices: B, S B, dB as [n][k]; B^T / n as [k][n]; the transposes of the first three
// as [k][n] and B / n as [n][k], so the fused kernels read every operand with coalesced rows
enum MatKind { kPlain = 0, kPref = 1, kDeriv = 2, kProj = 3, kPlainT = 4, kPrefT = 5, kDerivT = 6, kProjT = 7 };
constexpr int kNumMats = 8;

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline int slot_freq(int a, int K) {
  if (a == 0) return 0;
  if (K % 2 == 0 && a == K - 1) return -1;  // pad
  return (a + 1) / 2;
}

// value (or derivative) of the real basis function of slot a at x in [0,1)
inline double basis(int a, int K, double x, bool deriv) {
  const int k = slot_freq(a, K);
  if (k < 0) return 0.0;
  if (k == 0) return deriv ? 0.0 : 1.0;
  const double th = kTwoPi * k * x, r2 = std::sqrt(2.0);
  if (a & 1) return deriv ? -kTwoPi * k * r2 * std::sin(th) : r2 * std::cos(th);
  return deriv ? kTwoPi * k * r2 * std::cos(th) : r2 * std::sin(th);
}

// Smallest product grid on which the truncated product of two band-K fields is exact:
// N' >= 3 (K / 2 - 1) + 1, rounded up to a multiple of 8 and never above the image grid.
inline int product_grid_size(int n, int k) {
  if (n == 1) return 1;
  const int need = 3 * (k / 2 - 1) + 1;
  const int r = ((need + 7) / 8) * 8;
  return r < n ? r : n;
}

// Device allocation owned by the solver.
template <typename T>
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(int64_t n) { alloc(n); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void alloc(int64_t n) {
    release();
    if (n <= 0) return;
    if (hipMalloc(reinterpret_cast<void**>(&p_), static_cast<size_t>(n) * sizeof(T)) != hipSuccess) {
      p_ = nullptr;
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    n_ = n;
  }
  void release() {
    if (p_) (void)hipFree(p_);
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  int64_t size() const { return n_; }

 private:
  T* p_ = nullptr;
  int64_t n_ = 0;
};

template <typename T>
class Plan {
 public:
  // `st` points at the owner's stream, which the batched solver may swap between calls
  void init(const Dims& d, bool bf16, const hipStream_t* st) {
    d_ = d;
    bf16_ = bf16;
    st_ = st;
    build_matrices();
    const int64_t t_sz = (int64_t)kMaxFields * std::max<int64_t>((int64_t)d_.k[0] * d_.n[1] * d_.n[2],
                                                                 (int64_t)d_.k[0] * d_.k[1] * d_.n[2]);
    t1_.alloc(t_sz);
    t2_.alloc(t_sz);
    stk_.alloc(kMaxFields * d_.Q);
    blC_.alloc(kMaxFields * d_.Q);
    if (std::is_same<T, float>::value) {
      // partial projections of the split fused projection
      const int64_t slabs = (int64_t)kMaxFields * d_.k[0];
      pipart_.alloc(slabs * pi_ba_splits(d_.n[1]) * d_.k[1] * d_.k[2]);
      planes_ = !bf16_ && planes_ok(d_) && std::getenv("LDDMM_BL_NO_PLANES") == nullptr;
      prod_fused_ = planes_ && prod_plane_ok(d_) && std::getenv("LDDMM_BL_NO_PROD_FUSE") == nullptr;
      if (planes_) {
        Tp_.alloc(2 * kMaxFields * d_.n[0] * C());
        LDDMM_HIP(hipMemset(Tp_.get(), 0, Tp_.size() * sizeof(float)));
        reserve_parts(kMaxFields);
        zeros_.alloc(std::max<int64_t>(d_.Q, 64 * C()));
        LDDMM_HIP(hipMemset(zeros_.get(), 0, zeros_.size() * sizeof(float)));
      }
    }
  }
  // ---- plane-wise float path (dft_planes.hip)
  bool planes() const { return planes_; }
  int64_t C() const { return (int64_t)d_.k[1] * d_.k[2]; }
  // plane-band arrays [x0][a1][a2] of the expansions (2 kMaxFields slots) and of the reductions
  float* Tbuf(int f) { return Tp_.get() + (int64_t)f * d_.n[0] * C(); }
  float* part(int f) { return part_.get() + (int64_t)f * d_.n[0] * C(); }
  void reserve_parts(int nf) {
    if ((int64_t)nf * d_.n[0] * C() > part_.size()) {
      part_.alloc((int64_t)nf * d_.n[0] * C());
      LDDMM_HIP(hipMemset(part_.get(), 0, part_.size() * sizeof(float)));
    }
  }
  // expansion of nf plane-band arrays (Tbuf(t0 + f)) into out with the axis-1 / axis-2 kinds
  void expand(int nf, const int kinds[][3], float* out, int t0 = 0) {
    PlaneExpandArgs a{};
    for (int f = 0; f < nf; ++f) {
      a.T[f] = Tbuf(t0 + f);
      a.w1t[f] = mat(1, kinds[f][1] + kPlainT);
      a.w2t[f] = mat(2, kinds[f][2] + kPlainT);
    }
    a.out = out;
    a.nf = nf, a.n0 = d_.n[0], a.n1 = d_.n[1], a.n2 = d_.n[2], a.k1 = d_.k[1], a.k2 = d_.k[2];
    plane_expand(a, s());
  }
  void expand_kind(int nf, int kind, float* out, int t0 = 0) {
    int kinds[kMaxFields][3];
    for (int f = 0; f < nf; ++f) kinds[f][0] = kinds[f][1] = kinds[f][2] = kind;
    expand(nf, kinds, out, t0);
  }
  // reduction of nf grid values (plain fields or products, see PlaneReduceArgs) into part(0..nf)
  void reduce(int mode, int nf, const float* in, const float* e = nullptr, const float* divv = nullptr,
              const float* G = nullptr, int64_t e_node = 0) {
    reserve_parts(nf);
    PlaneReduceArgs a{};
    a.in = in, a.e = e, a.divv = divv, a.G = G, a.e_node = e_node;
    a.p1t = mat(1, kProjT), a.p2t = mat(2, kProjT);
    a.part = part_.get();
    a.mode = mode, a.nf = nf, a.n0 = d_.n[0], a.n1 = d_.n[1], a.n2 = d_.n[2], a.k1 = d_.k[1], a.k2 = d_.k[2];
    a.P = d_.P;
    plane_reduce(a, s());
  }
  // expansion of the e~ components in Tbuf(0 ..) fused with the reduction of their products with node
  // fields (kRedV1Products: 4 outputs, kRedV3Products: 6) into part(0 ..), when prod_fused()
  bool prod_fused() const { return prod_fused_; }
  void prod_reduce(int mode, const float* divv, const float* G) {
    const int nf = mode == kRedV1Products ? 4 : 6, ne = mode == kRedV1Products ? 1 : 3;
    reserve_parts(nf);
    ProdPlaneArgs a{};
    for (int c = 0; c < ne; ++c) a.T[c] = Tbuf(c);
    a.w1t = mat(1, kPlainT), a.w2t = mat(2, kPlainT);
    a.divv = divv, a.G = G;
    a.p1t = mat(1, kProjT), a.p2t = mat(2, kProjT);
    a.part = part_.get();
    a.mode = mode, a.n0 = d_.n[0], a.n1 = d_.n[1], a.n2 = d_.n[2], a.k1 = d_.k[1], a.k2 = d_.k[2];
    a.P = d_.P;
    plane_prod(a, s());
  }
  // pi of nf stacked grid fields into bl with the reductions' plane-band partials in a caller-given
  // workspace of cap floats (float plane-wise path only)
  void pi_ws(const float* grid, float* bl, int nf, float* ws, int64_t cap) {
    if (!planes_) throw ArgError("this context's projection does not run the plane-wise FP32 path");
    const int64_t need = (int64_t)nf * d_.n[0] * C();
    if (need > cap)
      throw ArgError("projection workspace of " + std::to_string(need * 4) + " bytes exceeds the " +
                     std::to_string(cap * 4) + "-byte static scratch");
    PlaneReduceArgs r{};
    r.in = grid;
    r.p1t = mat(1, kProjT), r.p2t = mat(2, kProjT);
    r.part = ws;
    r.mode = kRedPlain, r.nf = nf, r.n0 = d_.n[0], r.n1 = d_.n[1], r.n2 = d_.n[2], r.k1 = d_.k[1], r.k2 = d_.k[2];
    r.P = d_.P;
    plane_reduce(r, s());
    for (int f0 = 0; f0 < nf; f0 += kMaxFields) {
      const int m = std::min(kMaxFields, nf - f0);
      Axis0Args a = axis0_args(m);
      for (int f = 0; f < m; ++f) {
        a.part[f] = ws + (int64_t)(f0 + f) * d_.n[0] * C();
        a.out[f] = bl + (int64_t)(f0 + f) * d_.Q;
        a.alpha[f] = 1.f;
      }
      plane_axis0(a, s());
    }
  }
  // first-axis launch with this plan's projection shape (F inputs from part(f0 ..))
  Axis0Args axis0_args(int nin, int f0 = 0) {
    Axis0Args a{};
    a.nin = nin;
    for (int f = 0; f < kMaxFields; ++f) a.s2[f] = 1.f;
    for (int f = 0; f < nin; ++f) a.part[f] = part(f0 + f);
    a.p0t = mat(0, kProjT);
    a.n0 = d_.n[0], a.k0 = d_.k[0], a.C = static_cast<int>(C());
    a.zeros = zeros_.get();
    for (int g = 0; g < kMaxFields; ++g) a.o[g].s1 = a.o[g].s2 = -1;
    return a;
  }
  // P target on this plan: Tbuf(slot) = w0(kind) (c1 (s1 + g1) + c2 (s2 + g2))
  Axis0Out target(int slot, int kind, int s1, const float* g1, float c1, int s2 = -1, const float* g2 = nullptr,
                  float c2 = 0.f) {
    Axis0Out o{};
    o.w0t = mat(0, kind + kPlainT);
    o.T = Tbuf(slot);
    o.n0t = d_.n[0];
    o.s1 = s1, o.s2 = s2, o.g1 = g1, o.g2 = g2, o.c1 = c1, o.c2 = c2;
    return o;
  }
  const Dims& dims() const { return d_; }
  const T* mat(int axis, int kind) const { return mats_.get() + mat_off_[axis][kind]; }

  // iota of nf stacked BL fields; kinds[f][axis] picks plain / prefiltered / derivative matrices
  void iota(const T* bl, T* out, int nf, const int kinds[][3]) {
    const int n0 = d_.n[0], n1 = d_.n[1], n2 = d_.n[2], k0 = d_.k[0], k1 = d_.k[1], k2 = d_.k[2];
    if constexpr (std::is_same_v<T, float>) {
      if (planes_ || fused_dft_ok(n1, n2, k1, k2)) {
        const T* xs[kMaxFields];
        for (int f = 0; f < nf; ++f) xs[f] = bl + f * d_.Q;
        return iota_comb(xs, nullptr, nullptr, out, nf, kinds);
      }
    }
    FieldMats<T> W{};
    for (int f = 0; f < nf; ++f) W.w[f] = mat(2, kinds[f][2]);
    dft_right(bl, t1_.get(), W, nf, k0 * k1, k2, n2, s());
    const bool skip0 = (n0 == 1 && k0 == 1);
    T* dstB = skip0 ? out : t2_.get();
    for (int f = 0; f < nf; ++f) W.w[f] = mat(1, kinds[f][1]);
    left(t1_.get(), dstB, W, nf * k0, k0, n1, k1, n2, (int64_t)k1 * n2, (int64_t)n1 * n2);
    if (!skip0) {
      for (int f = 0; f < nf; ++f) W.w[f] = mat(0, kinds[f][0]);
      left(t2_.get(), out, W, nf, 1, n0, k0, n1 * n2, (int64_t)k0 * n1 * n2, d_.P);
    } else {
      zero_degenerate_derivatives(out, nf, kinds);
    }
  }
  // iota of per-field combinations x_f + alpha_f y_f (y_f may be null)
  void iota_comb(const T* const* xs, const T* const* ys, const T* al, T* out, int nf, const int kinds[][3]) {
    const int n0 = d_.n[0], n1 = d_.n[1], n2 = d_.n[2], k0 = d_.k[0], k1 = d_.k[1], k2 = d_.k[2];
    const bool skip0 = (n0 == 1 && k0 == 1);
    if constexpr (std::is_same_v<T, float>) {
      if (planes_) {
        // P: Tbuf(f) = W0 (x_f + alpha_f y_f), then the plane expansion
        for (int f0 = 0; f0 < nf; f0 += kMaxFields) {
          const int m = std::min(kMaxFields, nf - f0);
          Axis0Args a = axis0_args(0);
          a.nout = m;
          for (int f = 0; f < m; ++f)
            a.o[f] = target(f, kinds[f0 + f][0], -1, xs[f0 + f], 1.f, -1, ys ? ys[f0 + f] : nullptr,
                            (ys && ys[f0 + f]) ? al[f0 + f] : 0.f);
          plane_axis0(a, s());
          expand(m, kinds + f0, out + (int64_t)f0 * d_.P);
        }
        return;
      }
      if (fused_dft_ok(n1, n2, k1, k2)) {
        IotaABArgs a{};
        for (int f = 0; f < nf; ++f) {
          a.x[f] = xs[f];
          a.y[f] = ys ? ys[f] : nullptr;
          a.alpha[f] = al ? al[f] : 0.f;
          a.w1t[f] = mat(1, kinds[f][1] + kPlainT);
          a.w2t[f] = mat(2, kinds[f][2] + kPlainT);
        }
        a.out = skip0 ? out : t2_.get();
        a.k0 = k0, a.k1 = k1, a.k2 = k2, a.n1 = n1, a.n2 = n2;
        iota_ab(a, nf, s());
        if (!skip0) {
          FieldMats<T> W{};
          for (int f = 0; f < nf; ++f) W.w[f] = mat(0, kinds[f][0]);
          left(t2_.get(), out, W, nf, 1, n0, k0, n1 * n2, (int64_t)k0 * n1 * n2, d_.P);
        } else {
          zero_degenerate_derivatives(out, nf, kinds);
        }
        return;
      }
    }
    // generic path: stack the combinations, then the separable stages
    for (int f = 0; f < nf; ++f) {
      if (ys && ys[f])
        bl_axpby<T>(stk_.get() + f * d_.Q, T(1), xs[f], al[f], ys[f], d_.Q, s());
      else
        copy_dev<T>(stk_.get() + f * d_.Q, xs[f], d_.Q, s());
    }
    iota(stk_.get(), out, nf, kinds);
  }
  void iota_comb_kind(const T* const* xs, const T* const* ys, const T* al, T* out, int nf, int kind) {
    int kinds[kMaxFields][3];
    for (int f = 0; f < nf; ++f) kinds[f][0] = kinds[f][1] = kinds[f][2] = kind;
    iota_comb(xs, ys, al, out, nf, kinds);
  }
  void iota_kind(const T* bl, T* out, int nf, int kind) {
    int kinds[kMaxFields][3];
    for (int f = 0; f < nf; ++f) kinds[f][0] = kinds[f][1] = kinds[f][2] = kind;
    iota(bl, out, nf, kinds);
  }
  // gradients of nc band fields: out[3 c + j] = iota(d_j x_c) (x_c stacked with stride Q, nc <= 4)
  void iota_grad(const T* x, T* out, int nc) {
    int kinds[kMaxFields][3] = {};
    const T* xs[kMaxFields];
    for (int c = 0; c < nc; ++c)
      for (int j = 0; j < 3; ++j) {
        xs[3 * c + j] = x + c * d_.Q;
        for (int a = 0; a < 3; ++a) kinds[3 * c + j][a] = (a == j) ? kDeriv : kPlain;
      }
    iota_comb(xs, nullptr, nullptr, out, 3 * nc, kinds);
  }
  // pi of nf stacked grid fields into per-field destinations: dst_f = beta_f dst_f + alpha_f pi(grid_f)
  void pi_acc(const T* grid, int nf, T* const* dst, const T* alpha, const T* beta) {
    const int n0 = d_.n[0], n1 = d_.n[1], n2 = d_.n[2], k0 = d_.k[0], k1 = d_.k[1], k2 = d_.k[2];
    if constexpr (std::is_same_v<T, float>) {
      if (planes_) {
        reduce(kRedPlain, nf, grid);
        for (int f0 = 0; f0 < nf; f0 += kMaxFields) {
          const int m = std::min(kMaxFields, nf - f0);
          Axis0Args a = axis0_args(m, f0);
          for (int f = 0; f < m; ++f) {
            a.out[f] = dst[f0 + f];
            a.alpha[f] = alpha[f0 + f];
            a.beta[f] = beta[f0 + f];
          }
          plane_axis0(a, s());
        }
        return;
      }
      if (fused_dft_ok(n1, n2, k1, k2)) {
        const T* srcB = grid;
        if (!(n0 == 1 && k0 == 1)) {
          FieldMats<T> W{};
          for (int f = 0; f < nf; ++f) W.w[f] = mat(0, kProj);
          left(grid, t1_.get(), W, nf, 1, k0, n0, n1 * n2, d_.P, (int64_t)k0 * n1 * n2);
          srcB = t1_.get();
        }
        PiBAArgs b{};
        b.in = srcB;
        b.p1t = mat(1, kProjT);
        b.part = pipart_.get();
        b.p2t = mat(2, kProjT);
        for (int f = 0; f < nf; ++f) {
          b.out[f] = dst[f];
          b.alpha[f] = alpha[f];
          b.beta[f] = beta[f];
        }
        b.k0 = k0, b.k1 = k1, b.k2 = k2, b.n1 = n1, b.n2 = n2;
        pi_ba(b, nf, s());
        return;
      }
    }
    pi_sep(grid, blC_.get(), nf);
    for (int f = 0; f < nf; ++f) {
      if (beta[f] == T(0))
        bl_axpby<T>(dst[f], alpha[f], blC_.get() + f * d_.Q, T(0), nullptr, d_.Q, s());  // never reads dst
      else
        bl_axpby<T>(dst[f], beta[f], dst[f], alpha[f], blC_.get() + f * d_.Q, d_.Q, s());
    }
  }
  void pi(const T* grid, T* bl, int nf) {
    T* dst[kMaxFields];
    T one[kMaxFields], zer[kMaxFields];
    for (int f = 0; f < nf; ++f) dst[f] = bl + f * d_.Q, one[f] = T(1), zer[f] = T(0);
    pi_acc(grid, nf, dst, one, zer);
  }

 private:
  hipStream_t s() const { return *st_; }
  void build_matrices() {
    int64_t total = 0;
    for (int a = 0; a < 3; ++a) total += (int64_t)kNumMats * d_.n[a] * d_.k[a];
    std::vector<T> h(total);
    int64_t o = 0;
    for (int a = 0; a < 3; ++a) {
      const int n = d_.n[a], k = d_.k[a];
      for (int m = 0; m < kNumMats; ++m) mat_off_[a][m] = o + (int64_t)m * n * k;
      for (int x = 0; x < n; ++x) {
        const double xx = double(x) / n;
        for (int sl = 0; sl < k; ++sl) {
          const double b = basis(sl, k, xx, false);
          const int f = slot_freq(sl, k);
          const double sc = f < 0 ? 0.0 : 3.0 / (2.0 + std::cos(kTwoPi * f / n));
          h[mat_off_[a][kPlain] + (int64_t)x * k + sl] = static_cast<T>(b);
          h[mat_off_[a][kPref] + (int64_t)x * k + sl] = static_cast<T>(b * sc);
          h[mat_off_[a][kDeriv] + (int64_t)x * k + sl] = static_cast<T>(basis(sl, k, xx, true));
          h[mat_off_[a][kProj] + (int64_t)sl * n + x] = static_cast<T>(b / n);
          h[mat_off_[a][kPlainT] + (int64_t)sl * n + x] = static_cast<T>(b);
          h[mat_off_[a][kPrefT] + (int64_t)sl * n + x] = static_cast<T>(b * sc);
          h[mat_off_[a][kDerivT] + (int64_t)sl * n + x] = static_cast<T>(basis(sl, k, xx, true));
          h[mat_off_[a][kProjT] + (int64_t)x * k + sl] = static_cast<T>(b / n);
        }
      }
      o += (int64_t)kNumMats * n * k;
    }
    mats_.alloc(total);
    LDDMM_HIP(hipMemcpy(mats_.get(), h.data(), total * sizeof(T), hipMemcpyHostToDevice));
  }
  // axis contraction for the first-axis stages: float or split-bf16 matrix cores
  void left(const T* in, T* out, const FieldMats<T>& W, int nb, int bpf, int M, int L, int C, int64_t sIb,
            int64_t sOb) {
    if constexpr (std::is_same_v<T, float>) {
      if (bf16_) return dft_left_bf16(in, out, W, nb, bpf, M, L, C, sIb, sOb, s());
    }
    dft_left<T>(in, out, W, nb, bpf, M, L, C, sIb, sOb, s());
  }
  // A 2D problem skips the 1 x 1 stage of its degenerate first axis; that stage is the identity
  // except for a derivative along the axis, which vanishes: such fields are zero.
  void zero_degenerate_derivatives(T* out, int nf, const int kinds[][3]) {
    for (int f = 0; f < nf; ++f)
      if (kinds[f][0] == kDeriv) zero<T>(out + f * d_.P, d_.P, s());
  }
  // pi of nf stacked grid fields (separable stages)
  void pi_sep(const T* grid, T* bl, int nf) {
    const int n0 = d_.n[0], n1 = d_.n[1], n2 = d_.n[2], k0 = d_.k[0], k1 = d_.k[1], k2 = d_.k[2];
    FieldMats<T> W{};
    const T* srcB = grid;
    if (!(n0 == 1 && k0 == 1)) {
      for (int f = 0; f < nf; ++f) W.w[f] = mat(0, kProj);
      left(grid, t1_.get(), W, nf, 1, k0, n0, n1 * n2, d_.P, (int64_t)k0 * n1 * n2);
      srcB = t1_.get();
    }
    for (int f = 0; f < nf; ++f) W.w[f] = mat(1, kProj);
    left(srcB, t2_.get(), W, nf * k0, k0, k1, n1, n2, (int64_t)n1 * n2, (int64_t)k1 * n2);
    for (int f = 0; f < nf; ++f) W.w[f] = mat(2, kProj);
    dft_right(t2_.get(), bl, W, nf, k0 * k1, n2, k2, s());
  }

  Dims d_{};
  bool bf16_ = false, planes_ = false, prod_fused_ = false;
  const hipStream_t* st_ = nullptr;
  int64_t mat_off_[3][kNumMats] = {};
  DevBuf<T> mats_, t1_, t2_, stk_, blC_;
  DevBuf<float> pipart_, Tp_, part_, zeros_;
};

}  // namespace lddmm
