// Band-limited PDE-LDDMM with SL-RK2 integration: the sweeps of Table 1 for the
// image-transport variant (Section 2.3.1), the state-equation variant (Section
// 2.3.2) and the deformation-state variant (Section 2.3.3), their gradient and
// Gauss-Newton Hessian-vector product, and the Gauss-Newton-Krylov driver
// (Section 2.2, eqs. BLNewton / BLKKT).
//
// Readings of the paper used throughout (it leaves them open):
//  - unit periodic torus, grid-mean L^2 product, real orthonormal band basis with
//    a zero pad slot per axis, L~ = (1 + alpha (2 pi)^2 |k|^2)^s;
//  - characteristics X = x -/+ dt/2 (v + v o (x -/+ dt v)) (Section 3.1), one pair
//    per velocity since v is stationary;
//  - RK along the characteristic = Heun; a source that does not depend on the
//    unknown reduces it to the trapezoid rule;
//  - each band-limited unknown is projected once per step: the stage-1 source is
//    the exact truncated product of the band-limited snapshot, the predictor stays
//    a grid field and the stage-2 source is projected with the step result;
//  - the B-spline interpolant of a band-limited field c has coefficients
//    iota(S c) with S(k) = prod_j 3 / (2 + cos(2 pi k_j / N_j)): the prefilter is
//    folded into the inclusion matrices;
//  - time integrals of the gradient and Hessian terms: trapezoid rule;
//  - deformation-state gradient term (Du)^T rho, Gauss-Newton Hessian term
//    (Du)^T drho, final conditions with g1 = (grad P(I0)) o phi(1);
//  - state-equation variant: the nu~ equation's right-hand side is -v~; the
//    Jacobian J~ = 1 - U~ is integrated in the equivalent form -D~_t J~ =
//    J~ star div~ v~ from J~(1) = 1 (the same SL-RK2 arithmetic as the printed U~
//    equation, since the interpolant of a constant is that constant and
//    pi(iota(div~ v~)) = div~ v~); the Gauss-Newton incremental adjoint is
//    dlambda(t) = J(t) dlambda(1) o psi(t), dlambda(1) = -(2/sigma^2) dm(1),
//    dm(1) = -g1 . iota(du~(1)).
//
// Work placement.  Every truncated product of two band-limited fields (the
// sources f = x * div~ v~, the gradient and Hessian terms x * grad~ m~_n and
// (D~u~_n)^T x, the incremental source -grad~ m~_n . dv~ and dv~ - D~u~_n dv~) is
// formed on the product grid of the second plan, where it is exact and costs a
// small fraction of the image grid.  On the image grid remain the semi-Lagrangian
// interpolations, the image-transport state and adjoint, and the final warp.  In
// the incremental state the source does not depend on the unknown, so by
// linearity pi[c o X + dt/2 s_{n+1}] = pi[c o X] + dt/2 f~_{n+1}: every f~_n is
// formed before the sweep and each step projects one interpolated field.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <type_traits>

#include "prof.h"
#include "solver.h"
#include "tune.h"

namespace lddmm {

template <typename T>
class Solver final : public SolverBase {
 public:
  Solver(const lddmm_bl_params& p, hipStream_t s) : st_(s), params_(p) {
    dim_ = p.dim;
    if (dim_ != 2 && dim_ != 3) throw ArgError("dim must be 2 or 3");
    if (p.nt < 1) throw ArgError("nt must be >= 1");
    if (p.variant != LDDMM_BL_IMAGE_TRANSPORT && p.variant != LDDMM_BL_STATE_EQUATION &&
        p.variant != LDDMM_BL_DEFORMATION_STATE)
      throw ArgError("unknown variant");
    if (!(p.alpha > 0) || p.s < 1 || !(p.sigma2 > 0)) throw ArgError("alpha, s, sigma2 must be positive");
    if (p.integrator != LDDMM_BL_SL_RK2 && p.integrator != LDDMM_BL_EULER_RK4) throw ArgError("unknown integrator");
    rk_ = p.integrator == LDDMM_BL_EULER_RK4;
    if (rk_ && p.variant != LDDMM_BL_DEFORMATION_STATE)
      throw ArgError("the explicit RK4 comparator integrates the deformation-state variant only");
    if (p.nonstationary != 0 && p.nonstationary != 1) throw ArgError("nonstationary must be 0 or 1");
    ns_ = p.nonstationary == 1;
    if (ns_ && (rk_ || p.variant == LDDMM_BL_STATE_EQUATION))
      throw ArgError("non-stationary velocities: image-transport and deformation-state variants with SL-RK2 only");
    const int off = 3 - dim_;
    d_.n[0] = d_.n[1] = d_.n[2] = 1;
    d_.k[0] = d_.k[1] = d_.k[2] = 1;
    for (int j = 0; j < dim_; ++j) {
      const int n = p.n[j], k = p.k[j];
      if (k < 2 || (k % 2) || n < 3 * (k / 2 - 1) + 1 || k - 1 > n || n > 4096)
        throw ArgError("band must be even with N >= 3 (K/2 - 1) + 1 on every axis");
      d_.n[off + j] = n;
      d_.k[off + j] = k;
    }
    d_.P = (int64_t)d_.n[0] * d_.n[1] * d_.n[2];
    d_.Q = (int64_t)d_.k[0] * d_.k[1] * d_.k[2];
    ds_ = d_;
    for (int a = 0; a < 3; ++a) ds_.n[a] = product_grid_size(d_.n[a], d_.k[a]);
    ds_.P = (int64_t)ds_.n[0] * ds_.n[1] * ds_.n[2];
    nt_ = p.nt;
    dt_ = T(1.0 / p.nt);
    variant_ = p.variant;
    alpha_ = p.alpha;
    s_ = p.s;
    sigma2_ = p.sigma2;
    bf16_ = std::is_same_v<T, float> && p.precision == LDDMM_BL_BF16_DFT;
    full_.init(d_, bf16_, &st_);
    sm_.init(ds_, bf16_, &st_);
    build_symbols();
    allocate();
    autotune();
  }

  // Pick the brick tile for this grid shape, and the workgroup caps of the first-axis DFT launches of
  // plans that do not run the plane-wise path (split-bf16), once per process (timed on zeroed scratch
  // fields, three components as in the velocity and displacement transforms).
  void autotune() {
    if constexpr (std::is_same_v<T, float>) {
      if (std::getenv("LDDMM_BL_NO_TUNE")) return;
      if (brick_ok(d_)) {
        zero(S(0), 3 * d_.P, st_);
        zero(Xb_.get(), 3 * d_.P, st_);
        brick_autotune(S(3), S(0), Xb_.get(), d_, st_);
      }
      if (!full_.planes() || !sm_.planes()) {
        tune::Collect scope;
        zero(S(0), 3 * d_.P, st_);
        zero(tmpbl_.get(), 3 * d_.Q, st_);
        full_.iota_kind(tmpbl_.get(), S(0), 3, kPlain);
        full_.pi(S(0), tmpbl_.get(), 3);
        zero(Ps(0), 3 * ds_.P, st_);
        sm_.iota_kind(tmpbl_.get(), Ps(0), 3, kPlain);
        sm_.pi(Ps(0), tmpbl_.get(), 3);
      }
      sync();
    }
  }

  // ---------------------------------------------------------------- API ops
  void set_images(const void* I0, const void* I1) override {
    copy(I0_.get(), static_cast<const T*>(I0), d_.P);
    copy(I1_.get(), static_cast<const T*>(I1), d_.P);
    copy(cI0_.get(), I0_.get(), d_.P);
    prefilter(cI0_.get(), 1, d_, st_);
    have_images_ = true;
    state_valid_ = false;
    coarse_.reset();  // the coarse level restricts these images
  }

  void state_solve(const void* v, void* m1, double* E3) override {
    if (!have_images_) throw StateError("set_images must precede state_solve");
    to_internal(vbl_.get(), static_cast<const T*>(v), 3);
    double e[3];
    run_state(e);
    if (m1) copy(static_cast<T*>(m1), m1_ptr(), d_.P);
    if (E3) std::memcpy(E3, e, sizeof(e));
    sync();
  }

  void adjoint_solve(void* grad, double* ginf) override {
    require_state();
    run_adjoint(gbl_.get());
    if (grad) from_internal(static_cast<T*>(grad), gbl_.get(), 3);
    if (ginf) *ginf = grad_inf(gbl_.get());
    sync();
  }

  void hess_matvec(const void* dv, void* hdv) override {
    require_state();
    const T* x = static_cast<const T*>(dv);
    T* y = static_cast<T*>(hdv);
    if (dim_ == 3 && x != y && use_graphs()) {
      // the caller's layout is the internal one: replay a graph captured on the caller's buffers
      LDDMM_HIP(hipGraphLaunch(user_matvec_graph(x, y), st_));
    } else {
      to_internal(dvbl_.get(), x, 3);
      matvec_graph();
      from_internal(y, hbl_.get(), 3);
    }
    // enqueued only: the result is ready when the stream reaches it (no host scalar to return)
  }

  ~Solver() override {
    (void)hipStreamSynchronize(st_);  // replays still queued read the graphs and buffers freed below
    if (mv_exec_) (void)hipGraphExecDestroy(mv_exec_);
    for (auto& u : user_mv_) (void)hipGraphExecDestroy(u.exec);
  }

  int gn_solve(const lddmm_bl_gn_opts& o, void* v, const void* Z, int r, lddmm_bl_gn_report* rep) override;

  void jacobian(double* detmap, double* minmax) override {
    require_state();
    double mm[2];
    jacobian_into(detmap, mm);
    if (minmax) minmax[0] = mm[0], minmax[1] = mm[1];
    sync();
  }
  // det(I - D iota(u~(1))) into `detmap` (or the context's own buffer when null) and its extrema
  void jacobian_into(double* detmap, double mm[2]) {
    // u~(1): the deformation state (variant 3 holds it; variant 1 integrates it here)
    const T* u1;
    if (variant_ != LDDMM_BL_IMAGE_TRANSPORT) {
      u1 = ubl_.get() + (int64_t)nt_ * 3 * d_.Q;
    } else {
      displacement_only(tmpbl_.get());
      u1 = tmpbl_.get();
    }
    full_.iota_grad(u1, S9(), 3);
    double* det = detmap;
    if (!det) {
      if (!det_.get()) det_.alloc(d_.P);
      det = det_.get();
    }
    jacobian_det(det, S9(), dim_, d_.P, st_);
    minmax_f64(det, d_.P, work_.get(), host_.get(), st_);
    mm[0] = host_.get()[0];
    mm[1] = host_.get()[1];
  }

  void project(const void* grid, void* bl, int ncomp) override {
    check_ncomp(ncomp);
    full_.pi(static_cast<const T*>(grid), static_cast<T*>(bl), ncomp);
    sync();
  }

  void project_ws(const void* grid, void* bl, int ncomp, float* ws, int64_t cap) override {
    check_ncomp(ncomp);
    if constexpr (std::is_same_v<T, float>) {
      full_.pi_ws(static_cast<const float*>(grid), static_cast<float*>(bl), ncomp, ws, cap);
    } else {
      (void)grid, (void)bl, (void)ws, (void)cap;
      throw ArgError("the projection without allocation takes FP32 contexts");
    }
  }

  void include(const void* bl, void* grid, int ncomp) override {
    check_ncomp(ncomp);
    int kinds[kMaxFields][3] = {};
    full_.iota(static_cast<const T*>(bl), static_cast<T*>(grid), ncomp, kinds);
    sync();
  }

  int64_t get_field(int which, int index, void* dst) override;

  double dot(const void* a, const void* b, int64_t n) override {
    return lddmm::dot<T>(static_cast<const T*>(a), static_cast<const T*>(b), n, work_.get(), host_.get(), st_);
  }

 private:
  // ------------------------------------------------------------ set-up
  void build_symbols() {
    // L~ symbol and its inverse; zero on pad slots
    std::vector<double> L(d_.Q), Li(d_.Q);
    for (int a0 = 0; a0 < d_.k[0]; ++a0)
      for (int a1 = 0; a1 < d_.k[1]; ++a1)
        for (int a2 = 0; a2 < d_.k[2]; ++a2) {
          const int f0 = slot_freq(a0, d_.k[0]), f1 = slot_freq(a1, d_.k[1]), f2 = slot_freq(a2, d_.k[2]);
          const int64_t q = ((int64_t)a0 * d_.k[1] + a1) * d_.k[2] + a2;
          if (f0 < 0 || f1 < 0 || f2 < 0) {
            L[q] = Li[q] = 0.0;
            continue;
          }
          const double k2 = double(f0) * f0 + double(f1) * f1 + double(f2) * f2;
          L[q] = std::pow(1.0 + alpha_ * kTwoPi * kTwoPi * k2, s_);
          Li[q] = 1.0 / L[q];
        }
    Lsym_.alloc(d_.Q);
    Linv_.alloc(d_.Q);
    LDDMM_HIP(hipMemcpy(Lsym_.get(), L.data(), d_.Q * sizeof(double), hipMemcpyHostToDevice));
    LDDMM_HIP(hipMemcpy(Linv_.get(), Li.data(), d_.Q * sizeof(double), hipMemcpyHostToDevice));
  }

  void allocate() {
    const int64_t P = d_.P, Q = d_.Q, Ps = ds_.P, nn = nt_ + 1;
    I0_.alloc(P);
    I1_.alloc(P);
    cI0_.alloc(P);
    // velocity-like band vectors hold one node (stationary) or nt + 1 nodes (non-stationary); so do the
    // per-node divergence fields, and the departure displacements one per step
    const int64_t VQ = (ns_ ? nn : 1) * 3 * Q, nsteps = ns_ ? nt_ : 1, nnodes = ns_ ? nn : 1;
    vbl_.alloc(VQ);
    dvbl_.alloc(VQ);
    gbl_.alloc(VQ);
    hbl_.alloc(VQ);
    tmpbl_.alloc(3 * Q);
    blA_.alloc(kMaxFields * Q);
    acc_.alloc(VQ);
    vg_.alloc(3 * P);
    divv_.alloc(nnodes * P);
    Xb_.alloc(nsteps * 3 * P);
    Xf_.alloc(nsteps * 3 * P);
    if (ns_) {
      // node weights of the trapezoid rule per element: the node-field inner product and regulariser
      std::vector<double> wv(VQ), wl(VQ), Lh(Q);
      LDDMM_HIP(hipMemcpy(Lh.data(), Lsym_.get(), Q * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < VQ; ++i) {
        const int64_t n = i / (3 * Q);
        const double w = (n == 0 || n == nt_) ? 0.5 / nt_ : 1.0 / nt_;
        wv[i] = w;
        wl[i] = w * Lh[i % Q];
      }
      wvec_.alloc(VQ);
      wLsym_.alloc(VQ);
      LDDMM_HIP(hipMemcpy(wvec_.get(), wv.data(), VQ * sizeof(double), hipMemcpyHostToDevice));
      LDDMM_HIP(hipMemcpy(wLsym_.get(), wl.data(), VQ * sizeof(double), hipMemcpyHostToDevice));
    }
    scratch_.alloc(13 * P);  // 9P-field transforms + 4P staging
    inc_.alloc(nn * 3 * Q);
    incadj_.alloc(nn * 3 * Q);
    // node 0 of the incremental state is 0 in every matvec; the plane-wise sweep never writes it
    LDDMM_HIP(hipMemset(inc_.get(), 0, inc_.size() * sizeof(T)));
    fsrc_.alloc(nn * 3 * Q);
    // product grid: div v, the state's gradient fields, the expanded operand and the products
    divvs_.alloc(nnodes * Ps);
    dvs_.alloc(nnodes * 3 * Ps);
    es_.alloc(std::max<int64_t>(3, variant_ == LDDMM_BL_STATE_EQUATION ? std::min(nn, (int64_t)kMaxFields) : 3) * Ps);
    prods_.alloc(std::max<int64_t>(kMaxFields, 3 * nn) * Ps);
    if (variant_ != LDDMM_BL_DEFORMATION_STATE) {
      m_.alloc(nn * P);
      mt_.alloc(nn * Q);
      Gs_.alloc(nn * 3 * Ps);
    }
    if (variant_ == LDDMM_BL_IMAGE_TRANSPORT) lam0_.alloc(P);
    if (variant_ != LDDMM_BL_IMAGE_TRANSPORT) {
      ubl_.alloc(nn * 3 * Q);
      Dus_.alloc(nn * 9 * Ps);
      m1_.alloc(P);
      g1_.alloc(3 * P);
    }
    if (variant_ == LDDMM_BL_DEFORMATION_STATE) rho_.alloc(nn * 3 * Q);
    if (rk_) {
      // the RK comparator's velocity samples, right-hand side and operand transforms on the product grid
      vs_.alloc(3 * Ps);
      rkw_.alloc(3 * Ps);
      rkD_.alloc(12 * Ps);
    }
    if (variant_ == LDDMM_BL_STATE_EQUATION) {
      // inverse map, its Jacobian, their grid samples at every node, and the pulled-back adjoint
      nubl_.alloc(nn * 3 * Q);
      Jbl_.alloc(nn * Q);
      psi_.alloc(nn * 3 * P);
      Jg_.alloc(nn * P);
      lamg_.alloc(nn * P);
      lamt_.alloc(nn * Q);
      // J~(1) = 1: the constant slot of the band
      std::vector<T> e0(Q, T(0));
      e0[0] = T(1);
      one_.alloc(Q);
      LDDMM_HIP(hipMemcpy(one_.get(), e0.data(), Q * sizeof(T), hipMemcpyHostToDevice));
    }
    work_.alloc(reduce_work_size());
    // the incremental sources of every node are reduced in one launch (no allocation inside a capture)
    if (sm_.planes()) sm_.reserve_parts(std::max<int>(kMaxFields, 3 * (int)nn));
    double* hp = nullptr;
    LDDMM_HIP(hipHostMalloc(reinterpret_cast<void**>(&hp), 8 * sizeof(double), hipHostMallocDefault));
    host_.reset(hp);
  }

  struct PinnedFree {
    void operator()(double* p) const { (void)hipHostFree(p); }
  };

  // ------------------------------------------------------ graph capture
  // The Hessian matvec has no host synchronisation inside: its whole launch
  // sequence (about 130 kernels for Nt = 10) is captured once into a HIP graph
  // over the context's fixed buffers (input dvbl_, output hbl_) and replayed.
  // Needs a non-default stream; not used while per-kernel profiling is on.
  bool use_graphs() const { return st_ != nullptr && graphs_enabled_ && !prof::enabled(); }
  void capture_matvec() {
    hipGraph_t g = nullptr;
    LDDMM_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    try {
      run_matvec(dvbl_.get(), hbl_.get());
    } catch (...) {
      (void)hipStreamEndCapture(st_, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    LDDMM_HIP(hipStreamEndCapture(st_, &g));
    const hipError_t e = hipGraphInstantiate(&mv_exec_, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      mv_exec_ = nullptr;
      throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }
  // Graphs of H x -> y over callers' buffers (the four most recent pointer pairs; the oldest is dropped).
  // A graph holds only the two addresses: replaying it for the same pair reads and writes whatever the
  // caller keeps there at the time.
  struct UserGraph {
    const T* x;
    T* y;
    hipGraphExec_t exec;
  };
  std::vector<UserGraph> user_mv_;
  hipGraphExec_t user_matvec_graph(const T* x, T* y) {
    for (const auto& u : user_mv_)
      if (u.x == x && u.y == y) return u.exec;
    hipGraph_t g = nullptr;
    LDDMM_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    try {
      run_matvec(x, y);
    } catch (...) {
      (void)hipStreamEndCapture(st_, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    LDDMM_HIP(hipStreamEndCapture(st_, &g));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    if (user_mv_.size() == 4) {
      sync();  // the oldest graph may still be queued on the stream
      (void)hipGraphExecDestroy(user_mv_.front().exec);
      user_mv_.erase(user_mv_.begin());
    }
    user_mv_.push_back({x, y, exec});
    return exec;
  }
  // H dvbl_ -> hbl_ (replay of the captured graph, or eager launches)
  void matvec_graph() {
    if (use_graphs()) {
      if (!mv_exec_) capture_matvec();
      LDDMM_HIP(hipGraphLaunch(mv_exec_, st_));
    } else {
      run_matvec(dvbl_.get(), hbl_.get());
    }
  }

  // --------------------------------------------------------- small helpers
  void copy(T* dst, const T* src, int64_t n) { copy_dev<T>(dst, src, n, st_); }
  void sync() { LDDMM_HIP(hipStreamSynchronize(st_)); }
  void check_ncomp(int ncomp) const {
    if (ncomp < 1 || ncomp > kMaxFields) throw ArgError("ncomp must be in 1..12");
  }
  void require_state() const {
    if (!state_valid_) throw StateError("no state solve at the current velocity");
  }
  T* S(int i) { return scratch_.get() + (int64_t)i * d_.P; }
  T* S9() { return scratch_.get(); }
  // per-node / per-step views (the one stationary array when the velocity is stationary)
  int64_t VQ() const { return (ns_ ? nt_ + 1 : 1) * 3 * d_.Q; }
  T* vnode(int n) { return vbl_.get() + (ns_ ? (int64_t)n * 3 * d_.Q : 0); }
  T* XbN(int n) { return Xb_.get() + (ns_ ? (int64_t)n * 3 * d_.P : 0); }
  T* XfN(int n) { return Xf_.get() + (ns_ ? (int64_t)n * 3 * d_.P : 0); }
  T* divvN(int n) { return divv_.get() + (ns_ ? (int64_t)n * d_.P : 0); }
  T* divvsN(int n) { return divvs_.get() + (ns_ ? (int64_t)n * ds_.P : 0); }
  T* dvsN(int n) { return dvs_.get() + (ns_ ? (int64_t)n * 3 * ds_.P : 0); }
  // the dv samples on the product grid (per node when non-stationary)
  void dv_on_product_grid(const T* dv) {
    const int nodes = ns_ ? nt_ + 1 : 1;
    for (int n0 = 0; n0 < nodes; n0 += 4) {
      const int m = std::min(4, nodes - n0);
      sm_.iota_kind(dv + (int64_t)n0 * 3 * d_.Q, dvs_.get() + (int64_t)n0 * 3 * ds_.P, 3 * m, kPlain);
    }
  }
  T* Ps(int i) { return prods_.get() + (int64_t)i * ds_.P; }
  const T* m1_ptr() const {
    return variant_ == LDDMM_BL_IMAGE_TRANSPORT ? m_.get() + (int64_t)nt_ * d_.P : m1_.get();
  }
  // projection / inclusion of any number of stacked fields (kMaxFields per transform)
  void pi_many(const T* grid, T* bl, int nf) {
    for (int f0 = 0; f0 < nf; f0 += kMaxFields)
      full_.pi(grid + (int64_t)f0 * d_.P, bl + (int64_t)f0 * d_.Q, std::min(kMaxFields, nf - f0));
  }
  void iota_many(const T* bl, T* grid, int nf) {
    for (int f0 = 0; f0 < nf; f0 += kMaxFields)
      full_.iota_kind(bl + (int64_t)f0 * d_.Q, grid + (int64_t)f0 * d_.P, std::min(kMaxFields, nf - f0), kPlain);
  }

  // user [dim][..] <-> internal [3][..] for velocity-like arrays of length Q per component ([nt + 1][..] of them
  // when non-stationary)
  void to_internal(T* dst, const T* src, int ncomp) {
    const int64_t Q = d_.Q;
    const int nodes = (ns_ && ncomp == 3) ? nt_ + 1 : 1;
    if (dim_ == 3) {
      copy(dst, src, (int64_t)nodes * ncomp * Q);
      return;
    }
    for (int n = 0; n < nodes; ++n) {
      zero(dst + n * 3 * Q, Q, st_);
      copy(dst + n * 3 * Q + Q, src + n * 2 * Q, 2 * Q);
    }
  }
  void from_internal(T* dst, const T* src, int ncomp) {
    const int64_t Q = d_.Q;
    const int nodes = (ns_ && ncomp == 3) ? nt_ + 1 : 1;
    if (dim_ == 3) {
      copy(dst, src, (int64_t)nodes * ncomp * Q);
      return;
    }
    for (int n = 0; n < nodes; ++n) copy(dst + n * 2 * Q, src + n * 3 * Q + Q, 2 * Q);
  }
  void axpby(T* out, T a, const T* x, T b, const T* y, int64_t n) { bl_axpby<T>(out, a, x, b, y, n, st_); }

  double grad_inf(const T* g) {
    double m = 0.0;
    for (int n = 0; n < (ns_ ? nt_ + 1 : 1); ++n) {
      full_.iota_kind(g + (int64_t)n * 3 * d_.Q, S(0), 3, kPlain);
      m = std::max(m, maxabs<T>(S(0), 3 * d_.P, work_.get(), host_.get(), st_));
    }
    return m;
  }

  // ------------------------------------ truncated products on the product grid
  // x (ncomp band fields) against the state at node n:
  //   image transport (ncomp 1): pi'([e div v, e G_0, e G_1, e G_2]), G = grad~ m~_n
  //   deformation state (ncomp 3): pi'([e_i div v (3), (D~u~_n)^T e (3)])
  // with e = iota'(x), into dst with dst_f = beta_f dst_f + alpha_f (.)
  // (one-component x: the image-transport form, with the state-equation variant's G_n as well)
  void products(const T* x, int nc, int n, T* const* dst, const T* al, const T* be) {
    if constexpr (std::is_same_v<T, float>) {
      if (sm_.planes()) {
        const bool v1 = nc == 1;
        const int nc = v1 ? 1 : 3, np = v1 ? 4 : 6;
        const float* Gn = v1 ? Gs_.get() + (int64_t)n * 3 * ds_.P : Dus_.get() + (int64_t)n * 9 * ds_.P;
        if (sm_.prod_fused()) {  // plane-band inputs of x, then expansion and reduction in one pass
          Axis0Args t = sm_.axis0_args(0);
          t.nout = nc;
          for (int c = 0; c < nc; ++c) t.o[c] = sm_.target(c, kPlain, -1, x + c * d_.Q, 1.f);
          plane_axis0(t, st_);
          sm_.prod_reduce(v1 ? kRedV1Products : kRedV3Products, divvsN(n), Gn);
        } else {
          sm_.iota_kind(x, es_.get(), nc, kPlain);
          sm_.reduce(v1 ? kRedV1Products : kRedV3Products, np, nullptr, es_.get(), divvsN(n), Gn);
        }
        Axis0Args a = sm_.axis0_args(np);
        for (int f = 0; f < np; ++f) a.out[f] = dst[f], a.alpha[f] = al[f], a.beta[f] = be[f];
        plane_axis0(a, st_);
        return;
      }
    }
    if (nc == 1) {
      sm_.iota_kind(x, es_.get(), 1, kPlain);
      v1_products<T>(Ps(0), es_.get(), divvsN(n), Gs_.get() + (int64_t)n * 3 * ds_.P, ds_, st_);
      sm_.pi_acc(Ps(0), 4, dst, al, be);
    } else {
      sm_.iota_kind(x, es_.get(), 3, kPlain);
      v3_products<T>(Ps(0), es_.get(), divvsN(n), Dus_.get() + (int64_t)n * 9 * ds_.P, ds_, st_);
      sm_.pi_acc(Ps(0), 6, dst, al, be);
    }
  }

  // ---------------------------------------------- per-velocity set-up (Section 3.1)
  void setup_velocity() {
    // a non-finite coefficient would turn into non-finite departure points; reject it before any
    // interpolation runs
    if (!std::isfinite(maxabs<T>(vbl_.get(), VQ(), work_.get(), host_.get(), st_)))
      throw NonFiniteError("velocity has non-finite coefficients");
    setup_velocity_body();
  }
  void setup_velocity_body() {
    if (ns_) return setup_velocity_ns();
    const int64_t P = d_.P;
    // velocity samples and the B-spline coefficients of the velocity in one 6-field transform
    const T* xs[6];
    int kinds[kMaxFields][3] = {};
    for (int f = 0; f < 6; ++f) xs[f] = vbl_.get() + (f % 3) * d_.Q;
    for (int f = 3; f < 6; ++f) kinds[f][0] = kinds[f][1] = kinds[f][2] = kPref;
    full_.iota_comb(xs, nullptr, nullptr, S(0), 6, kinds);
    copy(vg_.get(), S(0), 3 * P);
    const T* cv = S(3);
    characteristics<T>(Xb_.get(), vg_.get(), cv, d_, dt_, -1, st_);
    characteristics<T>(Xf_.get(), vg_.get(), cv, d_, dt_, +1, st_);
    bl_div<T>(tmpbl_.get(), vbl_.get(), d_, st_);
    full_.iota_kind(tmpbl_.get(), divv_.get(), 1, kPlain);
    sm_.iota_kind(tmpbl_.get(), divvs_.get(), 1, kPlain);
    if (rk_) sm_.iota_kind(vbl_.get(), vs_.get(), 3, kPlain);
  }

  // per step n -> n + 1: X_b from the arrival velocity v_{n+1} and the departure velocity's interpolant
  // P(v_n); X_f (arrival t_n, departure t_{n+1}) from v_n and P(v_{n+1}); div v at every node
  void setup_velocity_ns() {
    const int64_t Q = d_.Q;
    for (int n = 0; n < nt_; ++n) {
      const T* xs[12];
      int kinds[kMaxFields][3];
      for (int f = 0; f < 12; ++f) {
        const int which = f / 3, c = f % 3;
        xs[f] = vnode(n + (which & 1)) + c * Q;  // v_n, v_{n+1}, P v_n, P v_{n+1}
        kinds[f][0] = kinds[f][1] = kinds[f][2] = which >= 2 ? kPref : kPlain;
      }
      full_.iota_comb(xs, nullptr, nullptr, S(0), 12, kinds);
      characteristics<T>(XbN(n), S(3), S(6), d_, dt_, -1, st_);
      characteristics<T>(XfN(n), S(0), S(9), d_, dt_, +1, st_);
    }
    for (int n = 0; n <= nt_; ++n) {
      bl_div<T>(tmpbl_.get(), vnode(n), d_, st_);
      full_.iota_kind(tmpbl_.get(), divvN(n), 1, kPlain);
      sm_.iota_kind(tmpbl_.get(), divvsN(n), 1, kPlain);
    }
  }

  double regulariser() {
    if (ns_)  // sum_n w_n 1/2 <L~ v_n, v_n>
      return 0.5 * sym_dot<T>(vbl_.get(), vbl_.get(), wLsym_.get(), 1, VQ(), work_.get(), host_.get(), st_);
    return 0.5 * sym_dot<T>(vbl_.get(), vbl_.get(), Lsym_.get(), 3, d_.Q, work_.get(), host_.get(), st_);
  }

  void finish_objective(double e[3]) {
    const double data = sqdiff<T>(m1_ptr(), I1_.get(), d_.P, work_.get(), host_.get(), st_) / d_.P / sigma2_;
    const double reg = regulariser();
    e[0] = reg + data;
    e[1] = reg;
    e[2] = data;
    if (!std::isfinite(e[0])) throw NonFiniteError("objective is not finite");
  }

  void run_state(double e[3]) {
    state_valid_ = false;
    setup_velocity();
    state_body();
    finish_objective(e);
    std::memcpy(last_e_, e, sizeof(last_e_));
    state_valid_ = true;
  }
  // ---- split forms for the batched solver: launched without a host synchronisation and finished
  // once the stream has been synchronised (pinned result slots: 0 velocity check, 1 data term,
  // 2 regulariser, 3 gradient sup-norm, 4 squared gradient norm); the same arithmetic as
  // setup_velocity / finish_objective / grad_inf / dot_internal
  void check_launch(const T* v) {
    reduce_launch<T>(RedKind::MaxAbs, v, nullptr, 3 * d_.Q, work_.get(), 0, st_);
    fetch_async(work_.get(), host_.get(), 1, st_);
  }
  bool check_ok() const { return std::isfinite(host_.get()[0]); }
  void state_launch(const T* v) {  // v has passed check_launch / check_ok
    state_compute(v);
    fetch_async(work_.get(), host_.get(), 3, st_);
  }
  // the state solve's launches with its scalars left in the device slots (capturable: no copy to the host)
  void state_compute(const T* v) {
    state_valid_ = false;
    copy(vbl_.get(), v, 3 * d_.Q);
    setup_velocity_body();
    state_body();
    reduce_launch<T>(RedKind::SqDiff, m1_ptr(), I1_.get(), d_.P, work_.get(), 1, st_);
    sym_dot_launch<T>(vbl_.get(), vbl_.get(), Lsym_.get(), 3, d_.Q, work_.get(), 2, st_);
  }
  void state_finish(double e[3]) {
    const double* h = host_.get();
    const double data = h[1] / d_.P / sigma2_;
    const double reg = 0.5 * h[2];
    e[0] = reg + data;
    e[1] = reg;
    e[2] = data;
    if (!std::isfinite(e[0])) throw NonFiniteError("objective is not finite");
    std::memcpy(last_e_, e, sizeof(last_e_));
    state_valid_ = true;
  }
  void adjoint_launch(T* g) {
    adjoint_compute(g);
    fetch_async(work_.get(), host_.get(), 5, st_);
  }
  void adjoint_compute(T* g) {
    run_adjoint(g);
    full_.iota_kind(g, S(0), 3, kPlain);
    reduce_launch<T>(RedKind::MaxAbs, S(0), nullptr, 3 * d_.P, work_.get(), 3, st_);
    reduce_launch<T>(RedKind::Dot, g, g, 3 * d_.Q, work_.get(), 4, st_);
  }
  void fetch_slots(int count) { fetch_async(work_.get(), host_.get(), count, st_); }
  const double* host_slots() const { return host_.get(); }
  double launched_ginf() const { return host_.get()[3]; }
  double launched_gnorm2() const { return host_.get()[4]; }

  // true when the held state was solved at exactly the internal velocity v (tmp: scratch of v's size)
  bool state_is_at(const T* v, T* tmp) {
    if (!state_valid_) return false;
    axpby(tmp, T(1), v, T(-1), vbl_.get(), VQ());
    return maxabs<T>(tmp, VQ(), work_.get(), host_.get(), st_) == 0.0;
  }

  void state_body() {
    if (variant_ == LDDMM_BL_IMAGE_TRANSPORT)
      state_v1();
    else if (variant_ == LDDMM_BL_STATE_EQUATION)
      state_v2();
    else
      state_v3();
  }

  // ------------------------------------ image transport: state (Table 1 row 1)
  void state_v1() {
    const int64_t P = d_.P, Q = d_.Q;
    copy(m_.get(), I0_.get(), P);
    for (int n = 0; n <= nt_; ++n) {
      T* mn = m_.get() + n * P;
      full_.pi(mn, mt_.get() + n * Q, 1);  // m~_n
      if (n < nt_) {
        copy(S(0), mn, P);
        prefilter(S(0), 1, d_, st_);
        interp<T>(mn + P, S(0), 1, XbN(n), d_, st_);
      }
    }
    // G_n = iota'(grad~ m~_n) on the product grid, four nodes per transform
    for (int n = 0; n <= nt_; n += 4)
      sm_.iota_grad(mt_.get() + n * Q, Gs_.get() + (int64_t)n * 3 * ds_.P, std::min(4, nt_ + 1 - n));
  }

  // ------------------------------ deformation state: state (Table 1 row 3)
  void state_v3() {
    const int64_t Q = d_.Q;
    zero(ubl_.get(), 3 * Q, st_);
    for (int n = 0; n < nt_; ++n) {
      if (rk_)
        rk4_step(ubl_.get() + n * 3 * Q, ubl_.get() + (n + 1) * 3 * Q, dt_,
                 [&](const T* x, int, T* o) { rk_rhs_state(x, o); });
      else
        u_step(ubl_.get() + n * 3 * Q, ubl_.get() + (n + 1) * 3 * Q, n);
    }
    // D u_n = iota'(D~ u~_n) on the product grid
    for (int n = 0; n <= nt_; ++n) sm_.iota_grad(ubl_.get() + n * 3 * Q, Dus_.get() + (int64_t)n * 9 * ds_.P, 3);
    full_.iota_kind(ubl_.get() + (int64_t)nt_ * 3 * Q, S(0), 3, kPlain);
    final_warp<T>(m1_.get(), g1_.get(), cI0_.get(), S(0), d_, st_);
  }
  // ------------------------------- state-equation variant (Section 2.3.2)
  // phi(t) = id - iota(u~(t)), psi(t) = id - iota(nu~(t)), J(t) = 1 - iota(U~(t)) = iota(J~(t));
  // m(t_n) = I0 o phi(t_n); every node's m~_n, G_n (image-transport form), D u_n (incremental sources),
  // and the grid samples of psi_n and J_n are kept for the adjoint and the matvecs.
  void state_v2() {
    const int64_t P = d_.P, Q = d_.Q;
    const int nn = nt_ + 1;
    zero(ubl_.get(), 3 * Q, st_);
    for (int n = 0; n < nt_; ++n) u_step(ubl_.get() + n * 3 * Q, ubl_.get() + (n + 1) * 3 * Q, n);
    for (int n = 0; n <= nt_; ++n) sm_.iota_grad(ubl_.get() + n * 3 * Q, Dus_.get() + (int64_t)n * 9 * ds_.P, 3);
    // m(t_n) at every node (psi_ holds the samples of u~_n until the inverse map replaces them)
    iota_many(ubl_.get(), psi_.get(), 3 * nn);
    pull_back_any(m_.get(), cI0_.get(), psi_.get(), nullptr, T(1), nn);
    final_warp<T>(m1_.get(), g1_.get(), cI0_.get(), psi_.get() + (int64_t)nt_ * 3 * P, d_, st_);
    pi_many(m_.get(), mt_.get(), nn);
    for (int n = 0; n <= nt_; n += 4)
      sm_.iota_grad(mt_.get() + n * Q, Gs_.get() + (int64_t)n * 3 * ds_.P, std::min(4, nt_ + 1 - n));
    // -D~_t nu~ = -v~ from nu~(1) = 0, and -D~_t J~ = J~ star div~ v~ from J~(1) = 1 (the image-transport
    // products the band-limited sweep also forms land in scratch)
    zero(nubl_.get() + (int64_t)nt_ * 3 * Q, 3 * Q, st_);
    for (int n = nt_ - 1; n >= 0; --n)
      map_step(nubl_.get() + (n + 1) * 3 * Q, nubl_.get() + n * 3 * Q, Xf_.get(), -1, vbl_.get(), vbl_.get());
    copy(Jbl_.get() + (int64_t)nt_ * Q, one_.get(), Q);
    bl_backward(Jbl_.get(), 1, tmpbl_.get());
    iota_many(nubl_.get(), psi_.get(), 3 * nn);
    iota_many(Jbl_.get(), Jg_.get(), nn);
  }

  void pull_back_any(T* out, const T* c, const T* u, const T* w, T a, int nodes) {
    if constexpr (std::is_same_v<T, float>) {
      if (brick_ok(d_)) return brick_pull_back(out, c, u, w, a, nodes, d_, st_);
    }
    pull_back<T>(out, c, u, w, a, nodes, d_, st_);
  }

  // acc = sum_n w_n pi(iota(f~_n) G_n) with f_n = a J_n P(c) o psi_n (c: prefiltered grid samples at
  // t = 1) and f~_n = pi(f_n) written to bl [nt+1][Q]: the gradient term (c from lambda(1)) or the
  // Hessian term (c from dlambda(1)) of the state-equation variant
  // With h_out (float plane-wise path): h_out = L~ x_sym + acc, acc left unspecified.
  void pull_back_terms(const T* c, T a, T* bl, T* acc, T* h_out = nullptr, const T* x_sym = nullptr) {
    const int nn = nt_ + 1;
    const int64_t Q = d_.Q;
    pull_back_any(lamg_.get(), c, psi_.get(), Jg_.get(), a, nn);
    if constexpr (std::is_same_v<T, float>) {
      if (full_.planes() && sm_.planes() && h_out) {
        // per chunk of nodes: f~_n and the product-grid plane-band inputs of w_n iota'(f~_n) in one axis-0
        // stage, their expansion, sum_n w_n e_n G_n in one node-sum reduction, and its axis-0 stage
        // (accumulating over chunks; the last one writes h_out = L~ x_sym + acc)
        for (int n0 = 0; n0 < nn; n0 += kMaxFields) {
          const int m = std::min(kMaxFields, nn - n0);
          const bool last = n0 + m == nn;
          full_.reduce(kRedPlain, m, lamg_.get() + (int64_t)n0 * d_.P);
          Axis0Args b = full_.axis0_args(m);
          b.nout = m;
          for (int f = 0; f < m; ++f) {
            b.out[f] = bl + (int64_t)(n0 + f) * Q;
            b.alpha[f] = 1.f;
            b.o[f] = sm_.target(f, kPlain, f, nullptr, trap_w(n0 + f));
          }
          plane_axis0(b, st_);
          sm_.expand_kind(m, kPlain, es_.get());
          node_sum<float>(Ps(0), es_.get(), Gs_.get() + (int64_t)n0 * 3 * ds_.P, m, ds_.P, st_);
          sm_.reduce(kRedPlain, 3, Ps(0));
          Axis0Args r = sm_.axis0_args(3);
          for (int j = 0; j < 3; ++j) {
            r.out[j] = acc + j * Q;
            r.alpha[j] = 1.f;
            r.beta[j] = n0 == 0 ? 0.f : 1.f;
            if (last) {
              r.in[j] = acc + j * Q;
              r.out[j] = h_out + j * Q;
              r.y[j] = x_sym + j * Q;
              r.ysym[j] = Lsym_.get();
            }
          }
          plane_axis0(r, st_);
        }
        return;
      }
    }
    pi_many(lamg_.get(), bl, nn);
    zero(acc, 3 * Q, st_);
    for (int n = 0; n <= nt_; ++n) {
      const T w = trap_w(n);
      T* dst[4] = {blA_.get(), acc, acc + Q, acc + 2 * Q};
      const T al[4] = {T(1), w, w, w}, be[4] = {T(0), T(1), T(1), T(1)};
      products(bl + n * Q, 1, n, dst, al, be);
    }
  }

  // lambda(1) = -(2/sigma^2)(m(1) - I1)
  void adjoint_v2(T* g) {
    scaled_diff<T>(S(0), T(-2.0 / sigma2_), m1_.get(), I1_.get(), d_.P, st_);
    prefilter(S(0), 1, d_, st_);
    pull_back_terms(S(0), T(1), lamt_.get(), acc_.get(), g, vbl_.get());
  }

  // Gauss-Newton incremental adjoint: dlambda(1) = -(2/sigma^2) dm(1), dm(1) = -g1 . iota(du~(1))
  void matvec_tail_v2(const T* du1, T* h, const T* dv) {
    full_.iota_kind(du1, S(0), 3, kPlain);
    v1_source<T>(S(3), g1_.get(), S(0), d_, st_);
    prefilter(S(3), 1, d_, st_);
    pull_back_terms(S(3), T(-2.0 / sigma2_), incadj_.get(), acc_.get(), h, dv);
  }

  // ----------------- explicit RK4 comparator (deformation-state equations in Eulerian form)
  // Band-limited right-hand sides, each formed on the product grid (exact truncated products) and
  // projected: d_t u~ = v~ - D~u~ star v~; d_t r~ = -div~(r~ star v~) for the adjoint and the incremental
  // adjoint; d_t du~ = dv~ - D~du~ star v~ - D~u~ star dv~ with D~u~ at the stage's time (a node, or the
  // mean of the step's two nodes at its half step).
  void rk_rhs_state(const T* u, T* out) {
    sm_.iota_grad(u, rkD_.get(), 3);
    v3_source<T>(rkw_.get(), rkD_.get(), vs_.get(), ds_, st_);
    sm_.pi(rkw_.get(), out, 3);
  }
  void rk_rhs_adjoint(const T* r, T* out) {
    const int64_t Q = d_.Q;
    int kinds[kMaxFields][3] = {};
    const T* xs[kMaxFields];
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) {
        xs[3 * i + j] = r + i * Q;
        for (int a = 0; a < 3; ++a) kinds[3 * i + j][a] = (a == j) ? kDeriv : kPlain;
      }
      xs[9 + i] = r + i * Q;
    }
    sm_.iota_comb(xs, nullptr, nullptr, rkD_.get(), 12, kinds);
    rk_adjoint_rhs<T>(rkw_.get(), rkD_.get(), rkD_.get() + 9 * ds_.P, vs_.get(), divvs_.get(), ds_.P, st_);
    sm_.pi(rkw_.get(), out, 3);
  }
  void rk_rhs_inc(const T* du, int n, T a, T b, T* out) {
    const T* Da = Dus_.get() + (int64_t)n * 9 * ds_.P;
    const T* Db = b != T(0) ? Da + 9 * ds_.P : Da;
    sm_.iota_grad(du, rkD_.get(), 3);
    rk_inc_rhs<T>(rkw_.get(), rkD_.get(), Da, Db, a, b, vs_.get(), dvs_.get(), ds_.P, st_);
    sm_.pi(rkw_.get(), out, 3);
  }
  // one classical four-stage step y_next = y + h/6 (k1 + 2 k2 + 2 k3 + k4) of y' = rhs(y) for a band
  // vector (h < 0 steps backward); rhs(stage input, stage 0..3, out); y_next must not alias y
  template <class F>
  void rk4_step(const T* y, T* ynext, T h, F&& rhs) {
    const int64_t n3 = 3 * d_.Q;
    T* k = blA_.get();
    T* ys = blA_.get() + n3;
    const T c[4] = {T(0), h / 2, h / 2, h}, w[4] = {h / 6, h / 3, h / 3, h / 6};
    copy(ynext, y, n3);
    for (int st = 0; st < 4; ++st) {
      const T* in = y;
      if (st > 0) {
        axpby(ys, T(1), y, c[st], k, n3);
        in = ys;
      }
      rhs(in, st, k);
      axpby(ynext, T(1), ynext, w[st], k, n3);
    }
  }
  // backward RK4 sweep of -d_t r~ = div~(r~ star v~) from traj[nt] to traj[0]
  void rk_backward(T* traj) {
    const int64_t Q = d_.Q;
    for (int n = nt_; n > 0; --n)
      rk4_step(traj + n * 3 * Q, traj + (n - 1) * 3 * Q, -dt_, [&](const T* x, int, T* o) { rk_rhs_adjoint(x, o); });
  }
  // acc = sum_n w_n (x_n - pi((D u_n)^T iota(x_n))): the deformation-state gradient / Hessian term
  void v3_terms(const T* traj, T* acc) {
    const int64_t Q = d_.Q;
    zero(acc, 3 * Q, st_);
    for (int n = 0; n <= nt_; ++n) {
      const T w = trap_w(n);
      const T* xn = traj + n * 3 * Q;
      T* dst[6] = {tmpbl_.get(), tmpbl_.get() + Q, tmpbl_.get() + 2 * Q, acc, acc + Q, acc + 2 * Q};
      const T al[6] = {T(1), T(1), T(1), -w, -w, -w}, be[6] = {T(0), T(0), T(0), T(1), T(1), T(1)};
      products(xn, 3, n, dst, al, be);
      axpby(acc, T(1), acc, w, xn, 3 * Q);
    }
  }
  void run_matvec_rk(const T* dv, T* h) {
    const int64_t Q = d_.Q;
    sm_.iota_kind(dv, dvs_.get(), 3, kPlain);
    T* du = inc_.get();
    zero(du, 3 * Q, st_);
    for (int n = 0; n < nt_; ++n)
      rk4_step(du + n * 3 * Q, du + (n + 1) * 3 * Q, dt_, [&](const T* x, int st, T* o) {
        if (st == 0)
          rk_rhs_inc(x, n, T(1), T(0), o);
        else if (st == 3)
          rk_rhs_inc(x, n + 1, T(1), T(0), o);
        else
          rk_rhs_inc(x, n, T(0.5), T(0.5), o);
      });
    // t = 1 coupling as in the SL form
    full_.iota_kind(du + (int64_t)nt_ * 3 * Q, S(0), 3, kPlain);
    coupling_v3<T>(S(3), T(2.0 / sigma2_), g1_.get(), S(0), d_, st_);
    T* dr = incadj_.get();
    full_.pi(S(3), dr + (int64_t)nt_ * 3 * Q, 3);
    rk_backward(dr);
    v3_terms(dr, acc_.get());
    bl_scale_sym<T>(h, dv, Lsym_.get(), 3, Q, acc_.get(), st_);
  }

  // deformation-state step n -> n + 1: u_next = pi[P(u + dt/2 v_n) o X_b] + dt/2 v_{n+1}
  void u_step(const T* un, T* un1, int n) { map_step(un, un1, XbN(n), 1, vnode(n), vnode(n + 1)); }
  // one step of a displacement map along the departure displacements X, with the velocity vd at the
  // departure time and va at the arrival time: next = pi[P(u + sgn dt/2 vd) o X] + sgn dt/2 va (sgn = +1: u~
  // forward along X_b; sgn = -1: the inverse map nu~ of the state-equation variant, backward along X_f)
  void map_step(const T* un, T* un1, const T* X, int sgn, const T* vd, const T* va) {
    const int64_t Q = d_.Q;
    const T hdt = T(0.5) * dt_ * T(sgn), sdt = dt_ * T(sgn);
    const T* xs[3] = {un, un + Q, un + 2 * Q};
    const T* ys[3] = {vd, vd + Q, vd + 2 * Q};
    const T al[3] = {hdt, hdt, hdt};
    full_.iota_comb_kind(xs, ys, al, S(0), 3, kPref);
    if constexpr (std::is_same_v<T, float>) {
      if (brick_ok(d_)) {
        // increment form: the B-spline interpolant of c = u + dt/2 v equals iota(c) at the nodes and
        // pi iota(c) = c, so u_next = u + dt v + pi[P(c) o X_b - P(c)]; the projection then carries one
        // step's change instead of the whole displacement (an FP32 rounding error that does not grow
        // with the displacement already accumulated)
        brick_interp_diff(S(3), S(0), 3, X, d_, st_);
        if (vd == va) {
          axpby(un1, T(1), un, sdt, vd, 3 * Q);
        } else {
          axpby(un1, T(1), un, hdt, vd, 3 * Q);
          axpby(un1, T(1), un1, hdt, va, 3 * Q);
        }
        T* dst[3] = {un1, un1 + Q, un1 + 2 * Q};
        const T one[3] = {T(1), T(1), T(1)};
        full_.pi_acc(S(3), 3, dst, one, one);
        return;
      }
    }
    interp<T>(S(3), S(0), 3, X, d_, st_);
    copy(un1, va, 3 * Q);
    T* dst[3] = {un1, un1 + Q, un1 + 2 * Q};
    const T one[3] = {T(1), T(1), T(1)}, hd[3] = {hdt, hdt, hdt};
    full_.pi_acc(S(3), 3, dst, one, hd);
  }

  // u~(1) only, for the Jacobian of the image-transport variant
  void displacement_only(T* u) {
    const int64_t Q = d_.Q;
    zero(u, 3 * Q, st_);
    for (int n = 0; n < nt_; ++n) {
      u_step(u, blA_.get(), n);
      copy(u, blA_.get(), 3 * Q);
    }
  }

  T trap_w(int n) const { return (n == 0 || n == nt_) ? T(0.5) * dt_ : dt_; }
  // weight of node n's gradient / Hessian term and its offset in a velocity-like vector: the trapezoid
  // weight into one accumulated field (stationary), or 1 into the node's own field (non-stationary)
  T term_w(int n) const { return ns_ ? T(1) : trap_w(n); }
  int64_t node_off(int n) const { return ns_ ? (int64_t)n * 3 * d_.Q : 0; }

  // ------------------------------------------ adjoint + gradient (rows 2 / 4)
  void run_adjoint(T* g) {
    if (variant_ == LDDMM_BL_IMAGE_TRANSPORT) {
      adjoint_v1();
    } else if (variant_ == LDDMM_BL_STATE_EQUATION) {
      if constexpr (std::is_same_v<T, float>) {
        if (full_.planes() && sm_.planes()) return adjoint_v2(g);  // g = L~ v + acc
      }
      adjoint_v2(nullptr);
    } else if (rk_) {
      residual_times_grad<T>(S(0), T(-2.0 / sigma2_), m1_.get(), I1_.get(), g1_.get(), d_, st_);
      full_.pi(S(0), rho_.get() + (int64_t)nt_ * 3 * d_.Q, 3);
      rk_backward(rho_.get());
      v3_terms(rho_.get(), acc_.get());
    } else {
      if constexpr (std::is_same_v<T, float>) {
        if (full_.planes() && sm_.planes()) {
          residual_times_grad<T>(S(0), T(-2.0 / sigma2_), m1_.get(), I1_.get(), g1_.get(), d_, st_);
          full_.pi(S(0), rho_.get() + (int64_t)nt_ * 3 * d_.Q, 3);
          return bl_backward_planes(rho_.get(), 3, acc_.get(), false, g, vbl_.get());  // g = L~ v + acc
        }
      }
      adjoint_v3();
    }
    bl_scale_sym<T>(g, vbl_.get(), Lsym_.get(), ns_ ? 3 * (nt_ + 1) : 3, d_.Q, acc_.get(), st_);
  }

  void adjoint_v1() {
    const int64_t P = d_.P, Q = d_.Q;
    T* lam = S(9);
    T* lam_next = S(10);
    scaled_diff<T>(lam, T(-2.0 / sigma2_), m1_ptr(), I1_.get(), P, st_);
    zero(acc_.get(), VQ(), st_);
    for (int n = nt_; n >= 0; --n) {
      // gradient term w_n pi(iota(pi lambda_n) G_n), accumulated into acc (the first product, the
      // band-limited source, is not used by the grid adjoint); non-stationary: the node's own term
      full_.pi(lam, tmpbl_.get(), 1);
      {
        const T w = term_w(n);
        T* an = acc_.get() + node_off(n);
        T* dst[4] = {blA_.get(), an, an + Q, an + 2 * Q};
        const T al[4] = {T(1), w, w, w}, be[4] = {T(0), T(1), T(1), T(1)};
        products(tmpbl_.get(), 1, n, dst, al, be);
      }
      if (n == 0) break;
      copy(S(5), lam, P);
      mul<T>(S(6), lam, divvN(n), P, st_);
      prefilter(S(5), 2, d_, st_);
      adjoint_grid_step<T>(lam_next, S(5), S(6), XfN(n - 1), divvN(n - 1), d_, dt_, st_);
      std::swap(lam, lam_next);
    }
    copy(lam0_.get(), lam, P);
  }

  // band-limited backward sweep with source (.) star div~ v~ (rows 4, 6, 8), ncomp 1 or 3,
  // accumulating the Hessian / gradient term: variant 1 pi(e G_n), variant 3 -pi((Du_n)^T e)
  void bl_backward(T* traj, int ncomp, T* acc) {
    if constexpr (std::is_same_v<T, float>) {
      if (full_.planes() && sm_.planes()) return bl_backward_planes(traj, ncomp, acc);
    }
    const int64_t Q = d_.Q;
    const int64_t stride = (int64_t)ncomp * Q;
    const T hdt = T(0.5) * dt_;
    zero(acc, ns_ ? VQ() : 3 * Q, st_);
    for (int n = nt_; n >= 0; --n) {
      T* xn = traj + n * stride;
      const T w = term_w(n);
      T* an = acc + node_off(n);
      if (ncomp == 1) {
        // [fl, e G0, e G1, e G2]: fl to blA, the Hessian / gradient terms accumulated into acc
        T* dst[4] = {blA_.get(), an, an + Q, an + 2 * Q};
        const T al[4] = {T(1), w, w, w}, be[4] = {T(0), T(1), T(1), T(1)};
        products(xn, 1, n, dst, al, be);
      } else {
        // [fl (3), (Du)^T e (3)]
        T* dst[6] = {blA_.get(), blA_.get() + Q, blA_.get() + 2 * Q, an, an + Q, an + 2 * Q};
        const T al[6] = {T(1), T(1), T(1), -w, -w, -w}, be[6] = {T(0), T(0), T(0), T(1), T(1), T(1)};
        products(xn, 3, n, dst, al, be);
        axpby(an, T(1), an, w, xn, 3 * Q);
      }
      if (n == 0) break;
      const T* fl = blA_.get();
      // cA = P(x + dt/2 fl), cB = P(x + dt fl), stacked
      const T* xs[6];
      const T* ys[6];
      T al2[6];
      for (int c = 0; c < ncomp; ++c) {
        xs[c] = xs[ncomp + c] = xn + c * Q;
        ys[c] = ys[ncomp + c] = fl + c * Q;
        al2[c] = hdt;
        al2[ncomp + c] = dt_;
      }
      full_.iota_comb_kind(xs, ys, al2, S(3), 2 * ncomp, kPref);
      bl_adjoint_step<T>(S(9), S(3), S(3 + ncomp), ncomp, XfN(n - 1), divvN(n - 1), d_, dt_, st_);
      full_.pi(S(9), traj + (n - 1) * stride, ncomp);
    }
  }

  void adjoint_v3() {
    const int64_t Q = d_.Q;
    residual_times_grad<T>(S(0), T(-2.0 / sigma2_), m1_.get(), I1_.get(), g1_.get(), d_, st_);
    full_.pi(S(0), rho_.get() + (int64_t)nt_ * 3 * Q, 3);
    bl_backward(rho_.get(), 3, acc_.get());
  }

  // ----------------------------------- Hessian matvec (rows 5-8, Section 2.3)
  void run_matvec(const T* dv, T* h) {
    if (rk_) return run_matvec_rk(dv, h);
    if constexpr (std::is_same_v<T, float>) {
      if (full_.planes() && sm_.planes()) return run_matvec_planes(dv, h);
    }
    const int64_t Q = d_.Q, Psm = ds_.P;
    const T hdt = T(0.5) * dt_;
    const int nc = variant_ == LDDMM_BL_IMAGE_TRANSPORT ? 1 : 3;
    const int nn = nt_ + 1;
    // incremental sources f~_n = pi'(s_n) for every node, scaled by dt/2, on the product grid:
    // image transport s_n = -G_n . dv, deformation state s_n = dv - (D u_n) dv
    dv_on_product_grid(dv);
    for (int n = 0; n < nn; ++n) {
      if (nc == 1)
        v1_source<T>(Ps(n), Gs_.get() + (int64_t)n * 3 * Psm, dvsN(n), ds_, st_);
      else
        v3_source<T>(Ps(3 * n), Dus_.get() + (int64_t)n * 9 * Psm, dvsN(n), ds_, st_);
    }
    for (int f0 = 0; f0 < nn * nc; f0 += kMaxFields) {
      const int nf = std::min<int>(kMaxFields, nn * nc - f0);
      T* dst[kMaxFields];
      T al[kMaxFields], be[kMaxFields];
      for (int f = 0; f < nf; ++f) dst[f] = fsrc_.get() + (int64_t)(f0 + f) * Q, al[f] = hdt, be[f] = T(0);
      sm_.pi_acc(Ps(f0), nf, dst, al, be);
    }
    // incremental state: dm_0 = 0, dm_{n+1} = pi[P(dm_n + dt/2 f_n) o X_b] + dt/2 f_{n+1}
    T* dm = inc_.get();  // [nt+1][nc][Q]
    zero(dm, nc * Q, st_);
    copy(dm + nc * Q, fsrc_.get() + nc * Q, (int64_t)nt_ * nc * Q);
    for (int n = 0; n < nt_; ++n) {
      const T* xs[3];
      const T* ys[3];
      T al[3], one[3];
      T* dst[3];
      for (int c = 0; c < nc; ++c) {
        xs[c] = dm + (n * nc + c) * Q;
        ys[c] = fsrc_.get() + (n * nc + c) * Q;
        dst[c] = dm + ((n + 1) * nc + c) * Q;
        al[c] = one[c] = T(1);
      }
      full_.iota_comb_kind(xs, ys, al, S(0), nc, kPref);
      interp<T>(S(3), S(0), nc, XbN(n), d_, st_);
      full_.pi_acc(S(3), nc, dst, one, one);
    }
    if (nc == 1) {
      T* dl = incadj_.get();
      axpby(dl + (int64_t)nt_ * Q, T(-2.0 / sigma2_), dm + (int64_t)nt_ * Q, T(0), nullptr, Q);
      bl_backward(dl, 1, acc_.get());
    } else if (variant_ == LDDMM_BL_STATE_EQUATION) {
      matvec_tail_v2(dm + (int64_t)nt_ * 3 * Q, nullptr, nullptr);
    } else {
      // t = 1 coupling: drho~(1) = pi((2/sigma^2) (g1 . iota(du~(1))) g1)
      full_.iota_kind(dm + (int64_t)nt_ * 3 * Q, S(0), 3, kPlain);
      coupling_v3<T>(S(3), T(2.0 / sigma2_), g1_.get(), S(0), d_, st_);
      T* dr = incadj_.get();
      full_.pi(S(3), dr + (int64_t)nt_ * 3 * Q, 3);
      bl_backward(dr, 3, acc_.get());
    }
    bl_scale_sym<T>(h, dv, Lsym_.get(), ns_ ? 3 * nn : 3, Q, acc_.get(), st_);
  }

  // ------------------------- plane-wise forms of the sweeps (float; dft_planes.hip)
  // Launch sequence per step: incremental state expand -> interpolate -> reduce -> axis0 (the axis-0
  // stage finishes dm_{n+1} and forms the next step's plane-band input); backward: the product-grid
  // expansion, product reduction and axis0 (source fl, Hessian terms, and the plane-band inputs of
  // P(x + dt/2 fl), P(x + dt fl)), then expand -> interpolate -> reduce -> axis0 (x_{n-1} and its
  // product-grid plane-band input).
  void run_matvec_planes(const float* dv, float* h) {
    const int64_t Q = d_.Q, Psm = ds_.P;
    const float hdt = 0.5f * dt_;
    const int nc = variant_ == LDDMM_BL_IMAGE_TRANSPORT ? 1 : 3;
    const int nn = nt_ + 1;
    int kpref[kMaxFields][3];
    for (int f = 0; f < kMaxFields; ++f) kpref[f][0] = kpref[f][1] = kpref[f][2] = kPref;
    float* dm = inc_.get();  // [nt+1][nc][Q]
    // f~_n dt/2 for every node (into fsrc, and into dm_n for n >= 1), and the plane-band input of
    // the first step's interpolant P(dm_0 + dt/2 f~_0) = P(dt/2 f~_0)
    dv_on_product_grid(dv);
    sm_.reduce(nc == 1 ? kRedV1Source : kRedV3Source, nn * nc, nullptr, dvs_.get(), nullptr,
               nc == 1 ? Gs_.get() : Dus_.get(), ns_ ? 3 * Psm : 0);
    for (int f0 = 0; f0 < nn * nc; f0 += kMaxFields) {
      const int m = std::min(kMaxFields, nn * nc - f0);
      Axis0Args a = sm_.axis0_args(m, f0);
      for (int f = 0; f < m; ++f) {
        a.out[f] = fsrc_.get() + (int64_t)(f0 + f) * Q;
        a.out2[f] = (f0 + f >= nc) ? dm + (int64_t)(f0 + f) * Q : nullptr;
        a.alpha[f] = hdt;
      }
      if (f0 == 0) {
        a.nout = nc;
        for (int c = 0; c < nc; ++c) a.o[c] = full_.target(c, kPref, c, nullptr, 1.f);
      }
      plane_axis0(a, st_);
    }
    // incremental state: dm_{n+1} = pi[P(dm_n + dt/2 f_n) o X_b] + dt/2 f_{n+1} (dm_0 = 0, kept)
    float* dl = incadj_.get();
    const float cpl = -2.0f / float(sigma2_);  // image transport: dl~(1) = -(2/sigma^2) dm~(1)
    for (int n = 0; n < nt_; ++n) {
      full_.expand(nc, kpref, S(0));
      interp<float>(S(3), S(0), nc, XbN(n), d_, st_);
      full_.reduce(kRedPlain, nc, S(3));
      Axis0Args a = full_.axis0_args(nc);
      for (int c = 0; c < nc; ++c) {
        a.out[c] = dm + (int64_t)((n + 1) * nc + c) * Q;
        a.alpha[c] = a.beta[c] = 1.f;
      }
      if (n + 1 < nt_) {
        a.nout = nc;
        for (int c = 0; c < nc; ++c)
          a.o[c] = full_.target(c, kPref, c, nullptr, 1.f, -1, fsrc_.get() + (int64_t)((n + 1) * nc + c) * Q, 1.f);
      } else if (nc == 1) {
        // the t = 1 coupling and the product-grid plane-band input of the backward sweep's first step
        a.out2[0] = dl + (int64_t)nt_ * Q;
        a.s2[0] = cpl;
        a.nout = 1;
        a.o[0] = sm_.target(0, kPlain, 0, nullptr, cpl);
      }
      plane_axis0(a, st_);
    }
    if (nc == 1) {
      bl_backward_planes(dl, 1, acc_.get(), true, h, dv);
    } else if (variant_ == LDDMM_BL_STATE_EQUATION) {
      matvec_tail_v2(dm + (int64_t)nt_ * 3 * Q, h, dv);  // h = L~ dv + acc
    } else {
      // t = 1 coupling: drho~(1) = pi((2/sigma^2) (g1 . iota(du~(1))) g1)
      full_.iota_kind(dm + (int64_t)nt_ * 3 * Q, S(0), 3, kPlain);
      coupling_v3<float>(S(3), 2.0f / float(sigma2_), g1_.get(), S(0), d_, st_);
      float* dr = incadj_.get();
      full_.pi(S(3), dr + (int64_t)nt_ * 3 * Q, 3);
      bl_backward_planes(dr, 3, acc_.get(), false, h, dv);
    }
  }

  // With h_out, the last step writes h_out = L~ x_sym + (the accumulated term) instead of acc; with
  // t_formed, the product-grid plane-band input of the first step was formed by the caller.
  void bl_backward_planes(float* traj, int nc, float* acc, bool t_formed = false, float* h_out = nullptr,
                          const float* x_sym = nullptr) {
    const int64_t Q = d_.Q;
    const int64_t stride = (int64_t)nc * Q;
    const float hdt = 0.5f * dt_;
    const bool v1 = nc == 1;  // image-transport form (also the state-equation variant's J~ sweep)
    const int np = v1 ? 4 : 6;
    int kpref[kMaxFields][3];
    for (int f = 0; f < kMaxFields; ++f) kpref[f][0] = kpref[f][1] = kpref[f][2] = kPref;
    if (!t_formed) {  // product-grid plane-band input of x_Nt
      Axis0Args a = sm_.axis0_args(0);
      a.nout = nc;
      for (int c = 0; c < nc; ++c) a.o[c] = sm_.target(c, kPlain, -1, traj + nt_ * stride + c * Q, 1.f);
      plane_axis0(a, st_);
    }
    for (int n = nt_; n >= 0; --n) {
      float* xn = traj + n * stride;
      const float w = term_w(n);
      const int64_t off = node_off(n);
      // products on the product grid: fl = x * div~ v~ and the Hessian / gradient terms (expansion and
      // reduction fused into one pass per plane where the plane fits)
      const float* Gn = v1 ? Gs_.get() + (int64_t)n * 3 * ds_.P : Dus_.get() + (int64_t)n * 9 * ds_.P;
      if (sm_.prod_fused()) {
        sm_.prod_reduce(v1 ? kRedV1Products : kRedV3Products, divvsN(n), Gn);
      } else {
        sm_.expand_kind(nc, kPlain, es_.get());
        sm_.reduce(v1 ? kRedV1Products : kRedV3Products, np, nullptr, es_.get(), divvsN(n), Gn);
      }
      Axis0Args a = sm_.axis0_args(np);
      for (int c = 0; c < nc; ++c) a.out[c] = blA_.get() + c * Q, a.alpha[c] = 1.f;
      for (int j = 0; j < 3; ++j) {
        a.out[nc + j] = acc + off + j * Q;
        a.alpha[nc + j] = v1 ? w : -w;
        // stationary: the first step starts the accumulation; non-stationary: each node its own term
        a.beta[nc + j] = (ns_ || n == nt_) ? 0.f : 1.f;
        if (!v1) a.z[nc + j] = xn + j * Q, a.gamma[nc + j] = w;  // + w x_n
        if (h_out && (ns_ || n == 0)) {  // h = L~ x_sym + acc (non-stationary: node by node)
          if (!ns_) a.in[nc + j] = acc + j * Q;
          a.out[nc + j] = h_out + off + j * Q;
          a.y[nc + j] = x_sym + off + j * Q;
          a.ysym[nc + j] = Lsym_.get();
        }
      }
      if (n > 0) {  // plane-band inputs of cA = P(x + dt/2 fl), cB = P(x + dt fl)
        a.nout = 2 * nc;
        for (int c = 0; c < nc; ++c) {
          a.o[c] = full_.target(c, kPref, -1, xn + c * Q, 1.f, c, nullptr, hdt);
          a.o[nc + c] = full_.target(nc + c, kPref, -1, xn + c * Q, 1.f, c, nullptr, dt_);
        }
      }
      plane_axis0(a, st_);
      if (n == 0) break;
      full_.expand(2 * nc, kpref, S(3));
      bl_adjoint_step<float>(S(9), S(3), S(3 + nc), nc, XfN(n - 1), divvN(n - 1), d_, dt_, st_);
      full_.reduce(kRedPlain, nc, S(9));
      Axis0Args b = full_.axis0_args(nc);
      b.nout = nc;
      for (int c = 0; c < nc; ++c) {
        b.out[c] = traj + (n - 1) * stride + c * Q;
        b.alpha[c] = 1.f;
        b.o[c] = sm_.target(c, kPlain, c, nullptr, 1.f);
      }
      plane_axis0(b, st_);
    }
  }

  // ------------------------------------------------------------------ state
  hipStream_t st_;
  Dims d_{};   // image grid
  Dims ds_{};  // product grid (same band)
  Plan<T> full_, sm_;
  int dim_ = 3, nt_ = 1, variant_ = 1, s_ = 2;
  T dt_ = T(1);
  double alpha_ = 0, sigma2_ = 1;
  bool have_images_ = false, state_valid_ = false;
  double last_e_[3] = {0, 0, 0};  // objective terms of the held state
  bool graphs_enabled_ = std::getenv("LDDMM_BL_NO_GRAPH") == nullptr;
  bool bf16_ = false;  // split-bf16 contractions for the first-axis DFT stages
  bool rk_ = false;    // explicit RK4 comparator instead of the SL-RK2 sweeps
  bool ns_ = false;    // a velocity per time node
  bool trace_ = std::getenv("LDDMM_BL_TRACE") != nullptr;  // Gauss-Newton scalars to stderr

  template <typename U>
  friend int gn_solve_batched_impl(std::vector<Solver<U>*>& subs, const lddmm_bl_gn_opts& o,
                                   void* const* v_user, lddmm_bl_gn_report* reps, hipStream_t st);
  hipGraphExec_t mv_exec_ = nullptr;
  lddmm_bl_params params_{};
  // two-level preconditioner: the coarse problem and its band vectors (restricted residual and velocity,
  // inner solution and inner PCG scratch)
  std::unique_ptr<Solver<T>> coarse_;
  DevBuf<T> cb_, cx_, cr_, cz_, cv_;
  int kf3_[3] = {1, 1, 1}, kc3_[3] = {1, 1, 1}, m3_[3] = {1, 1, 1};
  DevBuf<double> Lsym_, Linv_, work_;
  std::unique_ptr<double, PinnedFree> host_;
  DevBuf<T> I0_, I1_, cI0_;
  DevBuf<T> vbl_, dvbl_, gbl_, hbl_, tmpbl_, blA_, acc_;
  DevBuf<T> vg_, divv_, Xb_, Xf_, scratch_;
  DevBuf<T> inc_, incadj_, fsrc_;
  DevBuf<T> divvs_, dvs_, es_, prods_;          // product grid
  DevBuf<T> m_, mt_, Gs_, lam0_;                // image transport
  DevBuf<T> ubl_, Dus_, m1_, g1_, rho_;         // deformation state (and the state-equation variant)
  DevBuf<T> nubl_, Jbl_, psi_, Jg_, lamg_, lamt_, one_;  // state-equation variant
  DevBuf<T> vs_, rkw_, rkD_;                    // explicit RK4 comparator (product grid)
  DevBuf<double> wvec_, wLsym_;                 // non-stationary: node weights, node-weighted L~ symbol
  DevBuf<double> det_;  // Jacobian map when the caller keeps none

 public:
  // accessors used by the Gauss-Newton driver
  int64_t vec_len() const { return VQ(); }
  bool nonstationary() const { return ns_; }
  void set_velocity_internal(const T* v) { copy(vbl_.get(), v, VQ()); }
  void state_internal(double e[3]) { run_state(e); }
  void adjoint_internal(T* g) { run_adjoint(g); }
  // H x into y through the captured graph (its fixed buffers dvbl_ -> hbl_)
  void matvec_internal(const T* x, T* y) {
    if (x != dvbl_.get()) copy(dvbl_.get(), x, VQ());
    matvec_graph();
    if (y != hbl_.get()) copy(y, hbl_.get(), VQ());
  }
  void precond_internal(const T* r, T* z) {
    bl_scale_sym<T>(z, r, Linv_.get(), ns_ ? 3 * (nt_ + 1) : 3, d_.Q, nullptr, st_);
  }
  // the PCG / Armijo inner product (non-stationary: sum_n w_n <a_n, b_n>)
  double dot_internal(const T* a, const T* b) {
    if (ns_) return sym_dot<T>(a, b, wvec_.get(), 1, VQ(), work_.get(), host_.get(), st_);
    return lddmm::dot<T>(a, b, 3 * d_.Q, work_.get(), host_.get(), st_);
  }
  void dot_launch(const T* a, const T* b, int slot) {
    if (ns_)
      sym_dot_launch<T>(a, b, wvec_.get(), 1, VQ(), work_.get(), slot, st_);
    else
      reduce_launch<T>(RedKind::Dot, a, b, 3 * d_.Q, work_.get(), slot, st_);
  }
  double grad_inf_internal(const T* g) { return grad_inf(g); }
  void axpby_internal(T* out, T a, const T* x, T b, const T* y) { axpby(out, a, x, b, y, VQ()); }
  void copy_internal(T* dst, const T* src) { copy(dst, src, VQ()); }
  void user_to_internal(T* dst, const T* src) { to_internal(dst, src, 3); }
  void internal_to_user(T* dst, const T* src) { from_internal(dst, src, 3); }
  double mse_rel() {
    const double num = sqdiff<T>(m1_ptr(), I1_.get(), d_.P, work_.get(), host_.get(), st_);
    const double den = sqdiff<T>(I0_.get(), I1_.get(), d_.P, work_.get(), host_.get(), st_);
    return den > 0 ? num / den : 0.0;
  }
  hipStream_t stream() const { return st_; }
  void synchronize() { sync(); }

  // x = PCG from 0 on H x = b with L~^-1 for a fixed number of iterations, every scalar on the device (no
  // host synchronisation); r, z: scratch band vectors.  A direction with p.Hp <= 0 leaves x unchanged.
  void inner_pcg(const T* b, T* x, T* r, T* z, int iters) {
    const int64_t n = vec_len();
    double* wk = work_.get();
    T* const pv = dvbl_.get();
    T* const Apv = hbl_.get();
    zero(x, n, st_);
    copy(r, b, n);
    precond_internal(r, z);
    copy(pv, z, n);
    int irz = 2, irzn = 3;
    reduce_launch<T>(RedKind::Dot, r, z, n, wk, irz, st_);
    for (int it = 0; it < iters; ++it) {
      matvec_graph();
      reduce_launch<T>(RedKind::Dot, pv, Apv, n, wk, 0, st_);
      pcg_step<T>(x, r, pv, Apv, wk, irz, 0, n, st_);
      precond_internal(r, z);
      reduce_launch<T>(RedKind::Dot, r, z, n, wk, irzn, st_);
      pcg_dir<T>(pv, z, wk, irz, irzn, 0, n, st_);
      std::swap(irz, irzn);
    }
  }
  // the coarse level of the two-level preconditioner: grid N / 2, band 2 floor(K / 4), images restricted
  // by 2^d block means
  void ensure_coarse() {
    if (coarse_) return;
    lddmm_bl_params cp = params_;
    for (int j = 0; j < dim_; ++j) {
      if (params_.n[j] % 2) throw ArgError("two-level preconditioner: grid sizes must be even");
      cp.n[j] = params_.n[j] / 2;
      cp.k[j] = 2 * (params_.k[j] / 4);
      if (cp.k[j] < 2) throw ArgError("two-level preconditioner: band too small for a coarse level");
    }
    coarse_ = std::make_unique<Solver<T>>(cp, st_);
    Solver<T>& c = *coarse_;
    DevBuf<T> a(c.d_.P), b(c.d_.P);
    restrict_grid<T>(a.get(), I0_.get(), d_, st_);
    restrict_grid<T>(b.get(), I1_.get(), d_, st_);
    c.set_images(a.get(), b.get());
    const int64_t nc = c.vec_len();
    cb_.alloc(nc), cx_.alloc(nc), cr_.alloc(nc), cz_.alloc(nc), cv_.alloc(nc);
    for (int j = 0; j < 3; ++j) {
      kf3_[j] = d_.k[j];
      kc3_[j] = c.d_.k[j];
      m3_[j] = d_.k[j] > 1 ? c.d_.k[j] - 1 : 1;
    }
    sync();
  }
  // re-linearise the coarse level at the restricted velocity R v
  void coarse_at(const T* v) {
    band_copy<T>(cv_.get(), kc3_, v, kf3_, m3_, 3, false, st_);
    coarse_->set_velocity_internal(cv_.get());
    double e[3];
    coarse_->state_internal(e);
  }
  // M^-1 r = L~^-1 r with the coarse band's slots replaced by the inner solve of C x = R r
  void two_level_precond(const T* r, T* z, int inner) {
    band_copy<T>(cb_.get(), kc3_, r, kf3_, m3_, 3, false, st_);
    coarse_->inner_pcg(cb_.get(), cx_.get(), cr_.get(), cz_.get(), inner);
    precond_internal(r, z);
    band_copy<T>(z, kf3_, cx_.get(), kc3_, m3_, 3, true, st_);
  }
};

// ---------------------------------------------------------------- field access
template <typename T>
int64_t Solver<T>::get_field(int which, int index, void* dst_v) {
  T* dst = static_cast<T*>(dst_v);
  const int64_t P = d_.P, Q = d_.Q;
  const int off = 3 - dim_;
  auto grid_vec = [&](const T* src) -> int64_t {
    if (dst) copy(dst, src + off * P, dim_ * P);
    return dim_ * P;
  };
  auto bl_vec = [&](const T* src) -> int64_t {
    if (dst) copy(dst, src + off * Q, dim_ * Q);
    return dim_ * Q;
  };
  auto check_index = [&]() {
    if (index < 0 || index > nt_) throw ArgError("time index out of range");
  };
  int64_t count = 0;
  const bool v1 = variant_ == LDDMM_BL_IMAGE_TRANSPORT;
  const bool v2 = variant_ == LDDMM_BL_STATE_EQUATION;
  if (which != LDDMM_BL_FIELD_INC_STATE && which != LDDMM_BL_FIELD_INC_ADJOINT) require_state();
  auto grid_node = [&](const T* base) -> int64_t {
    check_index();
    if (dst) copy(dst, base + index * P, P);
    return P;
  };
  switch (which) {
    case LDDMM_BL_FIELD_VELOCITY:
      if (ns_) {  // iota(v~_n) at node index
        check_index();
        full_.iota_kind(vnode(index), S(0), 3, kPlain);
        count = grid_vec(S(0));
      } else {
        count = grid_vec(vg_.get());
      }
      break;
    case LDDMM_BL_FIELD_DEP_BACKWARD:
    case LDDMM_BL_FIELD_DEP_FORWARD:
      if (ns_ && (index < 0 || index >= nt_)) throw ArgError("step index out of range");
      count = grid_vec(which == LDDMM_BL_FIELD_DEP_BACKWARD ? XbN(ns_ ? index : 0) : XfN(ns_ ? index : 0));
      break;
    case LDDMM_BL_FIELD_DIV_V:
      if (ns_) check_index();
      if (dst) copy(dst, divvN(ns_ ? index : 0), P);
      count = P;
      break;
    case LDDMM_BL_FIELD_STATE:
      check_index();
      if (v1) {
        if (dst) copy(dst, m_.get() + index * P, P);
        count = P;
      } else {
        count = bl_vec(ubl_.get() + index * 3 * Q);
      }
      break;
    case LDDMM_BL_FIELD_M1:
      if (dst) copy(dst, m1_ptr(), P);
      count = P;
      break;
    case LDDMM_BL_FIELD_ADJOINT0:
      if (v1) {
        if (dst) copy(dst, lam0_.get(), P);
        count = P;
      } else if (v2) {
        if (dst) copy(dst, lamg_.get(), P);
        count = P;
      } else {
        count = bl_vec(rho_.get());
      }
      break;
    case LDDMM_BL_FIELD_INC_STATE:
    case LDDMM_BL_FIELD_INC_ADJOINT: {
      check_index();
      const T* base = which == LDDMM_BL_FIELD_INC_STATE ? inc_.get() : incadj_.get();
      if (v1 || (v2 && which == LDDMM_BL_FIELD_INC_ADJOINT)) {
        if (dst) copy(dst, base + index * Q, Q);
        count = Q;
      } else {
        count = bl_vec(base + index * 3 * Q);
      }
      break;
    }
    case LDDMM_BL_FIELD_IMAGE:
      if (!v1 && !v2) throw ArgError("the deformation-state variant keeps m(1) only");
      count = grid_node(m_.get());
      break;
    case LDDMM_BL_FIELD_ADJOINT_GRID:
      if (!v2) throw ArgError("grid adjoint at every node: state-equation variant only");
      count = grid_node(lamg_.get());
      break;
    case LDDMM_BL_FIELD_INVERSE_STATE:
      if (!v2) throw ArgError("inverse map: state-equation variant only");
      check_index();
      count = bl_vec(nubl_.get() + index * 3 * Q);
      break;
    case LDDMM_BL_FIELD_JACOBIAN_STATE:
      if (!v2) throw ArgError("Jacobian state: state-equation variant only");
      check_index();
      if (dst) copy(dst, Jbl_.get() + index * Q, Q);
      count = Q;
      break;
    default:
      throw ArgError("unknown field");
  }
  sync();
  return count;
}

// ------------------------------------------------------- Gauss-Newton-Krylov
// PCG on H dv = -g from dv = 0 with L~^{-1} (or the two-level preconditioner),
// stopped at ||r|| <= eta ||g||, eta = min(0.5, sqrt(||g_k|| / ||g_0||)), the cap, or
// non-positive curvature; Armijo backtracking from eps = 1 (<= 10 halvings,
// c = 1e-4); stop at ||g||_inf <= rtol * reference.
template <typename T>
int Solver<T>::gn_solve(const lddmm_bl_gn_opts& o, void* v_user, const void* Zu, int r, lddmm_bl_gn_report* rep) {
  if (!have_images_) throw StateError("set_images must precede gn_solve");
  if (o.max_gn < 0 || o.max_pcg < 1) throw ArgError("max_gn >= 0 and max_pcg >= 1 required");
  if (Zu && (r < 1 || r > 16)) throw ArgError("preconditioner rank must be 1..16");
  const bool ml = o.ml_inner > 0;
  if (ml && Zu) throw ArgError("the low-rank and the two-level preconditioners exclude each other");
  if (ns_ && (ml || Zu)) throw ArgError("non-stationary velocities take the L~^-1 preconditioner only");
  if (o.ml_inner < 0 || o.ml_inner > 1000) throw ArgError("ml_inner must be in 0..1000");
  if (ml) ensure_coarse();
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = vec_len();
  DevBuf<T> v(n), g(n), x(n), rr(n), z(n), vt(n), Z, HZ, zold;
  if (ml) zold.alloc(n);
  std::vector<double> ZHZinv;
  int status = LDDMM_BL_OK;
  lddmm_bl_gn_report R{};
  user_to_internal(v.get(), static_cast<T*>(v_user));
  double e[3];
  if (state_is_at(v.get(), x.get())) {
    std::memcpy(e, last_e_, sizeof(e));  // a state solve at this velocity is already held
  } else {
    set_velocity_internal(v.get());
    state_internal(e);
  }
  double E = e[0];
  R.E0 = E;
  adjoint_internal(g.get());
  double ginf = grad_inf_internal(g.get());
  const double ref = o.grad_ref_inf > 0 ? o.grad_ref_inf : ginf;
  const double gnorm0 = std::sqrt(dot_internal(g.get(), g.get()));
  const bool fixed = o.fixed_iters != 0;
  // two-level preconditioner: M^-1 r = L^-1 r + Z (Z^T H Z)^-1 Z^T r, Z recomputed per GN iteration
  const bool twolevel = Zu != nullptr;
  if (twolevel) {
    Z.alloc(r * n);
    HZ.alloc(r * n);
    for (int i = 0; i < r; ++i)
      user_to_internal(Z.get() + i * n, static_cast<const T*>(Zu) + (int64_t)i * (n / 3) * dim_);
    ZHZinv.assign(r * r, 0.0);
  }
  // device result slots of the PCG: p.Hp, r.r, r.z (ping-pong), r.z_old (flexible CG), Z^T r
  enum { kPAP = 0, kRN2 = 1, kRZ0 = 2, kRZX = 4, kZC = 8 };
  DevBuf<double> Minv;
  if (twolevel) Minv.alloc(r * r);
  double* const wk = work_.get();
  const double* const hs = host_.get();
  // M^-1 r = L~^-1 r (+ Z (Z^T H Z)^-1 Z^T r), every scalar on the device
  auto precond = [&](const T* rin, T* zout) {
    if (ml) return two_level_precond(rin, zout, o.ml_inner);
    precond_internal(rin, zout);
    if (!twolevel) return;
    for (int i = 0; i < r; ++i) reduce_launch<T>(RedKind::Dot, Z.get() + i * n, rin, n, wk, kZC + i, stream());
    lowrank_add<T>(zout, Z.get(), Minv.get(), wk, kZC, r, n, stream());
  };
  auto log_iter = [&](int it, int pcg, int neg, int bt) {
    if (it >= LDDMM_BL_LOG_MAX) return;
    R.log_pcg[it] = pcg;
    R.log_negcurv[it] = neg;
    R.log_backtracks[it] = bt;
    R.log_count = it + 1;
  };
  bool ls_failed = false;
  auto converged = [&] {
    return ginf <= o.grad_rtol * ref || (o.energy_target > 0 && E <= o.energy_target);
  };
  int k = 0;
  for (k = 0; k < o.max_gn; ++k) {
    if (trace_) fprintf(stderr, "[lddmm_bl] gn %d E %.17g ginf_rel %.6g\n", k, E, ginf / ref);
    if (!fixed && converged()) break;
    if (twolevel) {
      // Z^T H Z at the current velocity (r extra matvecs), inverted by Gauss-Jordan in double
      std::vector<double> A(r * r);
      for (int i = 0; i < r; ++i) {
        matvec_internal(Z.get() + i * n, HZ.get() + i * n);
        ++R.hess_matvecs;
      }
      for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) A[i * r + j] = dot_internal(Z.get() + i * n, HZ.get() + j * n);
      for (int i = 0; i < r; ++i)
        for (int j = 0; j < i; ++j) A[i * r + j] = A[j * r + i] = 0.5 * (A[i * r + j] + A[j * r + i]);
      std::vector<double> Inv(r * r, 0.0);
      for (int i = 0; i < r; ++i) Inv[i * r + i] = 1.0;
      bool ok = true;
      for (int c = 0; c < r && ok; ++c) {
        int piv = c;
        for (int i = c + 1; i < r; ++i)
          if (std::fabs(A[i * r + c]) > std::fabs(A[piv * r + c])) piv = i;
        if (!(std::fabs(A[piv * r + c]) > 1e-300)) {
          ok = false;
          break;
        }
        for (int j = 0; j < r; ++j) {
          std::swap(A[c * r + j], A[piv * r + j]);
          std::swap(Inv[c * r + j], Inv[piv * r + j]);
        }
        const double dv = A[c * r + c];
        for (int j = 0; j < r; ++j) {
          A[c * r + j] /= dv;
          Inv[c * r + j] /= dv;
        }
        for (int i = 0; i < r; ++i) {
          if (i == c) continue;
          const double f = A[i * r + c];
          for (int j = 0; j < r; ++j) {
            A[i * r + j] -= f * A[c * r + j];
            Inv[i * r + j] -= f * Inv[c * r + j];
          }
        }
      }
      if (ok)
        ZHZinv = Inv;
      else
        std::fill(ZHZinv.begin(), ZHZinv.end(), 0.0);
      LDDMM_HIP(hipMemcpyAsync(Minv.get(), ZHZinv.data(), r * r * sizeof(double), hipMemcpyHostToDevice, stream()));
      synchronize();
    }
    if (ml) coarse_at(v.get());
    const double gnorm = std::sqrt(dot_internal(g.get(), g.get()));
    const double eta = gnorm0 > 0 ? std::min(0.5, std::sqrt(gnorm / gnorm0)) : 0.5;
    const double tol = eta * gnorm;
    // PCG from x = 0.  p and H p are the matvec graph's own buffers; the step lengths stay on the device
    // and one host round trip per iteration reads p.Hp and r.r
    T* const pv = dvbl_.get();
    T* const Apv = hbl_.get();
    zero(x.get(), n, stream());
    axpby_internal(rr.get(), T(-1), g.get(), T(0), nullptr);
    precond(rr.get(), z.get());
    copy_internal(pv, z.get());
    int irz = kRZ0, irzn = kRZ0 + 1;
    dot_launch(rr.get(), z.get(), irz);
    dot_launch(rr.get(), rr.get(), kRN2);
    fetch_async(wk, host_.get(), 2, stream());
    synchronize();
    double rn = std::sqrt(hs[kRN2]);
    int its = 0, negcurv = 0;
    for (its = 0; its < o.max_pcg; ++its) {
      if (!fixed && rn <= tol) break;
      matvec_graph();  // H p
      ++R.hess_matvecs;
      dot_launch(pv, Apv, kPAP);
      pcg_step<T>(x.get(), rr.get(), pv, Apv, wk, irz, kPAP, n, stream());
      if (ml) copy_internal(zold.get(), z.get());
      precond(rr.get(), z.get());
      dot_launch(rr.get(), z.get(), irzn);
      if (ml) dot_launch(rr.get(), zold.get(), kRZX);
      dot_launch(rr.get(), rr.get(), kRN2);
      pcg_dir<T>(pv, z.get(), wk, irz, irzn, kPAP, n, stream(), ml ? kRZX : -1);
      fetch_async(wk, host_.get(), trace_ ? 4 : 2, stream());
      synchronize();
      const double pAp = hs[kPAP];
      if (!std::isfinite(pAp)) throw NonFiniteError("non-finite curvature in PCG");
      if (pAp <= 0.0) {
        negcurv = 1;  // truncated CG: the direction so far (or the first search direction, p unchanged)
        if (its == 0) copy_internal(x.get(), pv);
        break;
      }
      if (trace_) fprintf(stderr, "[lddmm_bl] gn %d pcg %d rz %.17g pAp %.17g a %.17g\n", k, its, hs[irz], pAp, hs[irz] / pAp);
      rn = std::sqrt(hs[kRN2]);
      std::swap(irz, irzn);
    }
    R.pcg_iters_total += its;
    // Armijo line search on the objective
    const double gd = dot_internal(g.get(), x.get());
    double eps = 1.0;
    bool accepted = false;
    const int bt_before = R.backtracks;
    double Et = E;
    for (int bt = 0; bt <= 10; ++bt) {
      axpby_internal(vt.get(), T(1), v.get(), T(eps), x.get());
      set_velocity_internal(vt.get());
      state_internal(e);
      Et = e[0];
      if (trace_) fprintf(stderr, "[lddmm_bl] gn %d ls eps %.17g E %.17g Et %.17g gd %.17g\n", k, eps, E, Et, gd);
      if (Et <= E + 1e-4 * eps * gd) {
        accepted = true;
        break;
      }
      ++R.backtracks;
      eps *= 0.5;
    }
    log_iter(k, its, negcurv, accepted ? R.backtracks - bt_before : -1);
    if (!accepted) {
      set_velocity_internal(v.get());
      state_internal(e);
      ls_failed = true;
      break;
    }
    copy_internal(v.get(), vt.get());
    E = Et;
    adjoint_internal(g.get());
    ginf = grad_inf_internal(g.get());
    R.gn_iters = k + 1;
  }
  // final status from the line search, convergence and the cap (truncated PCG solves are
  // recorded per iteration in the log, not in the status)
  if (ls_failed)
    status = LDDMM_BL_W_LINESEARCH;
  else if (!fixed && !converged())
    status = LDDMM_BL_W_MAXITER;
  internal_to_user(static_cast<T*>(v_user), v.get());
  R.E = E;
  R.grad_inf_rel = ref > 0 ? ginf / ref : 0.0;
  R.mse_rel = mse_rel();
  {
    double mm[2];
    jacobian_into(nullptr, mm);
    R.det_min = mm[0];
    R.det_max = mm[1];
  }
  synchronize();
  R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = R;
  return status;
}

// ---------------------------------------------------- batched Gauss-Newton-Krylov
// Several subjects (each with its own grid and band) registered in lockstep on one
// stream.  The Hessian matvecs of the subjects still iterating in a PCG iteration run as
// one HIP graph launch (one graph per set of active subjects, captured on first use);
// the PCG scalars live on the device and come back once per iteration for all
// subjects together; line searches and stopping tests stay per subject.  A subject
// that has converged (or whose PCG has stopped) keeps its results and drops out of
// the launched work.
template <typename T>
int gn_solve_batched_impl(std::vector<Solver<T>*>& subs, const lddmm_bl_gn_opts& o, void* const* v_user,
                          lddmm_bl_gn_report* reps, hipStream_t st) {
  const int B = static_cast<int>(subs.size());
  const auto t0 = std::chrono::steady_clock::now();
  struct Sub {
    DevBuf<T> v, g, x, r, z, vt;
    double E = 0, ginf = 0, ref = 0, gnorm0 = 0, tol = 0;
    bool converged = false, failed = false, pcg_done = false;
    int its = 0, negcurv = 0, bt = 0;  // this GN iteration's PCG iterations, truncation, backtracks
    lddmm_bl_gn_report R{};
    void log(int k, int backtracks) {
      if (k >= LDDMM_BL_LOG_MAX) return;
      R.log_pcg[k] = its;
      R.log_negcurv[k] = negcurv;
      R.log_backtracks[k] = backtracks;
      R.log_count = k + 1;
    }
  };
  std::vector<Sub> S(B);
  const bool fixed = o.fixed_iters != 0;
  const bool trace = std::getenv("LDDMM_BL_TRACE") != nullptr;
  auto mark = [&](const char* what) {  // phase timings to stderr with LDDMM_BL_TRACE
    if (trace)
      fprintf(stderr, "[lddmm_bl] batched %s at %.3f s\n", what,
              std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  };
  for (int i = 0; i < B; ++i) {
    Solver<T>& sv = *subs[i];
    if (!sv.have_images_) throw StateError("set_images must precede the batched solve");
    if (sv.st_ != st) throw ArgError("the batched subjects must share the batch's stream");
    const int64_t n = sv.vec_len();
    S[i].v.alloc(n), S[i].g.alloc(n), S[i].x.alloc(n), S[i].r.alloc(n), S[i].z.alloc(n), S[i].vt.alloc(n);
    sv.user_to_internal(S[i].v.get(), static_cast<const T*>(v_user[i]));
  }
  // The subjects are independent, so their solves and matvecs run as parallel branches: subject i
  // on branch stream i mod nb, forked from and joined back into st; the GPU then overlaps the
  // short, latency-bound kernels of different subjects instead of running B chains back to back.
  // Scalars (objectives, gradient norms) come back through pinned memory after one synchronisation
  // per phase instead of one per subject and reduction.
  const int nb = std::min(B, 8);
  struct Branches {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> ev;  // [0] fork, [1 + j] join of branch j
    ~Branches() {
      for (hipStream_t x : s) (void)hipStreamDestroy(x);
      for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    }
  } br;
  for (int j = 0; j < nb; ++j) {
    hipStream_t x;
    LDDMM_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    br.s.push_back(x);
  }
  for (int j = 0; j <= nb; ++j) {
    hipEvent_t x;
    LDDMM_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    br.ev.push_back(x);
  }
  std::vector<hipStream_t> own(B);
  for (int i = 0; i < B; ++i) own[i] = subs[i]->st_;
  auto restore = [&] {
    for (int i = 0; i < B; ++i) subs[i]->st_ = own[i];
  };
  // runs fn(i) for the listed subjects on the branches
  auto on_branches = [&](const std::vector<int>& who, const std::function<void(int)>& fn) {
    try {
      LDDMM_HIP(hipEventRecord(br.ev[0], st));
      for (int j = 0; j < nb; ++j) LDDMM_HIP(hipStreamWaitEvent(br.s[j], br.ev[0], 0));
      int k = 0;
      for (int i : who) {
        subs[i]->st_ = br.s[k++ % nb];
        fn(i);
      }
      restore();
      for (int j = 0; j < nb; ++j) {
        LDDMM_HIP(hipEventRecord(br.ev[1 + j], br.s[j]));
        LDDMM_HIP(hipStreamWaitEvent(st, br.ev[1 + j], 0));
      }
    } catch (...) {
      restore();
      throw;
    }
  };
  auto sync_st = [&] { LDDMM_HIP(hipStreamSynchronize(st)); };
  std::vector<int> all(B);
  for (int i = 0; i < B; ++i) all[i] = i;
  // Every phase that runs the same launches for the same subjects again (the Hessian matvecs of a PCG
  // iteration; the state solves of a line-search round; the adjoint solves of new gradients) is captured
  // once per (phase, subject set) into a HIP graph over fixed buffers and replayed; a subject that has
  // converged or stopped drops out of the set, so its work is not computed.  Graphs are not used while
  // profiling or with LDDMM_BL_NO_GRAPH set (the same launches then run eagerly).
  const bool use_graph = !prof::enabled() && std::getenv("LDDMM_BL_NO_GRAPH") == nullptr;
  std::map<std::pair<int, std::vector<int>>, hipGraphExec_t> graphs;
  struct GraphsGuard {
    std::map<std::pair<int, std::vector<int>>, hipGraphExec_t>& g;
    ~GraphsGuard() {
      for (auto& kv : g) (void)hipGraphExecDestroy(kv.second);
    }
  } graphs_guard{graphs};
  auto run_phase = [&](int phase, const std::vector<int>& who, const std::function<void(int)>& fn) {
    if (who.empty()) return;
    if (!use_graph) return on_branches(who, fn);
    auto key = std::make_pair(phase, who);
    auto it = graphs.find(key);
    if (it == graphs.end()) {
      hipGraph_t graph = nullptr;
      LDDMM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        on_branches(who, fn);
      } catch (...) {
        (void)hipStreamEndCapture(st, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      LDDMM_HIP(hipStreamEndCapture(st, &graph));
      hipGraphExec_t exec = nullptr;
      const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      it = graphs.emplace(key, exec).first;
    }
    LDDMM_HIP(hipGraphLaunch(it->second, st));
  };
  enum { kPhaseMatvec = 0, kPhaseTrial = 1, kPhaseAdjoint = 2 };
  // velocity checks (a non-finite velocity never reaches an interpolation), then every subject's
  // state and adjoint solve
  for (int i = 0; i < B; ++i) subs[i]->check_launch(S[i].v.get());
  sync_st();
  for (int i = 0; i < B; ++i)
    if (!subs[i]->check_ok()) throw NonFiniteError("velocity has non-finite coefficients");
  on_branches(all, [&](int i) {
    subs[i]->state_compute(S[i].v.get());
    subs[i]->adjoint_compute(S[i].g.get());
  });
  for (int i = 0; i < B; ++i) subs[i]->fetch_slots(5);
  sync_st();
  for (int i = 0; i < B; ++i) {
    double e[3];
    subs[i]->state_finish(e);
    S[i].E = S[i].R.E0 = e[0];
    S[i].ginf = subs[i]->launched_ginf();
    S[i].ref = o.grad_ref_inf > 0 ? o.grad_ref_inf : S[i].ginf;
    S[i].gnorm0 = std::sqrt(subs[i]->launched_gnorm2());
  }
  mark("initial solves done");
  // PCG scalars stay on the device (slots: 0 p.Hp, 1 r.r, 2 / 3 r.z ping-pong); one host round trip per
  // PCG iteration brings every subject's p.Hp and r.r back together
  enum { kPAP = 0, kRN2 = 1, kRZ0 = 2 };
  std::vector<int> irz(B, kRZ0), irzn(B, kRZ0 + 1);
  std::vector<double> rn(B, 0.0);
  for (int k = 0; k < o.max_gn; ++k) {
    bool any = false;
    for (int i = 0; i < B; ++i) {
      Sub& u = S[i];
      if (u.failed || u.converged) continue;
      if (!fixed && (u.ginf <= o.grad_rtol * u.ref || (o.energy_target > 0 && u.E <= o.energy_target))) {
        u.converged = true;
        continue;
      }
      any = true;
    }
    if (!any) break;
    // PCG in lockstep
    for (int i = 0; i < B; ++i) {
      Sub& u = S[i];
      Solver<T>& sv = *subs[i];
      u.pcg_done = u.failed || u.converged;
      if (u.pcg_done) continue;
      u.its = u.negcurv = u.bt = 0;
      const double gnorm = std::sqrt(sv.dot_internal(u.g.get(), u.g.get()));
      const double eta = u.gnorm0 > 0 ? std::min(0.5, std::sqrt(gnorm / u.gnorm0)) : 0.5;
      u.tol = eta * gnorm;
      zero(u.x.get(), sv.vec_len(), st);
      sv.axpby_internal(u.r.get(), T(-1), u.g.get(), T(0), nullptr);
      sv.precond_internal(u.r.get(), u.z.get());
      sv.copy_internal(sv.dvbl_.get(), u.z.get());
      irz[i] = kRZ0, irzn[i] = kRZ0 + 1;
      sv.dot_launch(u.r.get(), u.z.get(), irz[i]);
      sv.dot_launch(u.r.get(), u.r.get(), kRN2);
      sv.fetch_slots(2);
    }
    sync_st();
    for (int i = 0; i < B; ++i)
      if (!S[i].pcg_done) rn[i] = std::sqrt(subs[i]->host_slots()[kRN2]);
    for (int it = 0; it < o.max_pcg; ++it) {
      std::vector<int> active;
      for (int i = 0; i < B; ++i) {
        Sub& u = S[i];
        if (u.pcg_done) continue;
        if (!fixed && rn[i] <= u.tol) {
          u.pcg_done = true;
          continue;
        }
        active.push_back(i);
      }
      if (active.empty()) break;
      run_phase(kPhaseMatvec, active,
                [&](int i) { subs[i]->run_matvec(subs[i]->dvbl_.get(), subs[i]->hbl_.get()); });
      for (int i : active) {
        Sub& u = S[i];
        Solver<T>& sv = *subs[i];
        ++u.R.hess_matvecs;
        T* p = sv.dvbl_.get();
        const T* Ap = sv.hbl_.get();
        const int64_t n = sv.vec_len();
        double* wk = sv.work_.get();
        sv.dot_launch(p, Ap, kPAP);
        pcg_step<T>(u.x.get(), u.r.get(), p, Ap, wk, irz[i], kPAP, n, st);
        sv.precond_internal(u.r.get(), u.z.get());
        sv.dot_launch(u.r.get(), u.z.get(), irzn[i]);
        sv.dot_launch(u.r.get(), u.r.get(), kRN2);
        pcg_dir<T>(p, u.z.get(), wk, irz[i], irzn[i], kPAP, n, st);
        sv.fetch_slots(2);
      }
      sync_st();
      for (int i : active) {
        Sub& u = S[i];
        const double pAp = subs[i]->host_slots()[kPAP];
        if (!std::isfinite(pAp)) throw NonFiniteError("non-finite curvature in batched PCG");
        if (pAp <= 0.0) {  // the device updates were skipped; p is unchanged
          if (it == 0) subs[i]->copy_internal(u.x.get(), subs[i]->dvbl_.get());
          u.negcurv = 1;
          u.pcg_done = true;
          continue;
        }
        ++u.R.pcg_iters_total;
        ++u.its;
        rn[i] = std::sqrt(subs[i]->host_slots()[kRN2]);
        std::swap(irz[i], irzn[i]);
      }
    }
    mark("PCG done");
    // Armijo line search, every subject's trial state of a backtracking round in parallel
    std::vector<int> pending, accepted;
    std::vector<double> gd(B, 0.0), eps(B, 1.0);
    for (int i = 0; i < B; ++i) {
      if (S[i].failed || S[i].converged) continue;
      gd[i] = subs[i]->dot_internal(S[i].g.get(), S[i].x.get());
      pending.push_back(i);
    }
    for (int bt = 0; bt <= 10 && !pending.empty(); ++bt) {
      for (int i : pending) {
        subs[i]->axpby_internal(S[i].vt.get(), T(1), S[i].v.get(), T(eps[i]), S[i].x.get());
        subs[i]->check_launch(S[i].vt.get());
      }
      sync_st();
      for (int i : pending)
        if (!subs[i]->check_ok()) throw NonFiniteError("velocity has non-finite coefficients");
      run_phase(kPhaseTrial, pending, [&](int i) { subs[i]->state_compute(S[i].vt.get()); });
      for (int i : pending) subs[i]->fetch_slots(3);
      sync_st();
      std::vector<int> next;
      for (int i : pending) {
        double e[3];
        subs[i]->state_finish(e);
        if (e[0] <= S[i].E + 1e-4 * eps[i] * gd[i]) {
          subs[i]->copy_internal(S[i].v.get(), S[i].vt.get());
          S[i].E = e[0];
          S[i].log(k, S[i].bt);
          accepted.push_back(i);
        } else {
          ++S[i].R.backtracks;
          ++S[i].bt;
          eps[i] *= 0.5;
          next.push_back(i);
        }
      }
      pending.swap(next);
    }
    // no acceptable step: back to the last velocity's state
    for (int i : pending) {
      double e[3];
      subs[i]->set_velocity_internal(S[i].v.get());
      subs[i]->state_internal(e);
      S[i].failed = true;
      S[i].log(k, -1);
    }
    // new gradients of the subjects that moved
    run_phase(kPhaseAdjoint, accepted, [&](int i) { subs[i]->adjoint_compute(S[i].g.get()); });
    for (int i : accepted) subs[i]->fetch_slots(5);
    sync_st();
    for (int i : accepted) {
      S[i].ginf = subs[i]->launched_ginf();
      S[i].R.gn_iters = k + 1;
    }
    mark("line search and gradients done");
  }
  // per-subject status as in gn_solve; the batch returns the worst (line search, then cap)
  int status = LDDMM_BL_OK;
  for (int i = 0; i < B; ++i) {
    Sub& u = S[i];
    Solver<T>& sv = *subs[i];
    sv.internal_to_user(static_cast<T*>(v_user[i]), u.v.get());
    u.R.E = u.E;
    u.R.grad_inf_rel = u.ref > 0 ? u.ginf / u.ref : 0.0;
    u.R.mse_rel = sv.mse_rel();
    double mm[2];
    sv.jacobian_into(nullptr, mm);
    u.R.det_min = mm[0];
    u.R.det_max = mm[1];
    const bool conv = u.ginf <= o.grad_rtol * u.ref || (o.energy_target > 0 && u.E <= o.energy_target);
    if (u.failed)
      status = LDDMM_BL_W_LINESEARCH;
    else if (!fixed && !conv && status == LDDMM_BL_OK)
      status = LDDMM_BL_W_MAXITER;
  }
  LDDMM_HIP(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < B; ++i) {
    S[i].R.seconds = secs;
    if (reps) reps[i] = S[i].R;
  }
  return status;
}

int gn_solve_batched(std::vector<SolverBase*>& subs, const lddmm_bl_gn_opts& o, void* const* v_user,
                     lddmm_bl_gn_report* reps, hipStream_t st) {
  std::vector<Solver<float>*> f;
  for (auto* b : subs) {
    auto* s = dynamic_cast<Solver<float>*>(b);
    if (!s) throw ArgError("batched solves take float (FP32 or BF16_DFT) subjects");
    f.push_back(s);
  }
  return gn_solve_batched_impl<float>(f, o, v_user, reps, st);
}

std::unique_ptr<SolverBase> make_solver(const lddmm_bl_params& p, hipStream_t s) {
  if (p.precision == LDDMM_BL_FP64) return std::make_unique<Solver<double>>(p, s);
  if (p.precision == LDDMM_BL_FP32 || p.precision == LDDMM_BL_BF16_DFT) return std::make_unique<Solver<float>>(p, s);
  throw ArgError("unsupported precision");
}

}  // namespace lddmm
