// C ABI of the learned warm-start network (declared in include/lddmm_bl.h).
//
// Architecture: `levels` convolutions with 3^3 kernels, padding 1 and ReLU, stride 2
// except the last (stride 1), channels[0..levels-1], on a 2-channel input of
// in_size^3 voxels (the image pair); then a 1^3 head to out_channels without
// activation.  The head's output, of (in_size / 2^(levels-1))^3 voxels per channel,
// holds grid samples whose band-limited projection gives velocity coefficients in the
// real-basis layout.  With a requested output grid, the levels take stride 2 while the
// grid is larger than it and stride 1 afterwards.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/lddmm_bl.h"
#include "kernels.h"
#include "nn.h"
#include "solver.h"

namespace lddmm {

class Net {
 public:
  // out_size 0: the default schedule (stride 2 on every level but the last)
  Net(int levels, const int* channels, int in_size, int rank_r, uint64_t seed, hipStream_t s, int out_size = 0)
      : st_(s) {
    if (levels < 1 || levels > 6 || in_size < 4 || rank_r < 0 || rank_r > 16 || out_size < 0 || out_size > in_size)
      throw ArgError("bad network shape");
    const int out_channels = 3 * (1 + rank_r);
    rank_ = rank_r;
    for (int l = 0; l < levels; ++l) channels_.push_back(channels[l]);
    in_size_ = in_size;
    req_out_ = out_size;
    int cin = 2, size = in_size;
    for (int l = 0; l < levels; ++l) {
      ConvLayer L;
      L.cin = cin;
      L.cout = channels[l];
      L.k = 3;
      L.pad = 1;
      L.stride = out_size > 0 ? (size > out_size ? 2 : 1) : (l < levels - 1) ? 2 : 1;
      L.relu = 1;
      if (L.cout < 1 || L.cout > 1024) throw ArgError("bad channel count");
      layers_.push_back(L);
      sizes_.push_back(size);
      size = (size + 2 - 3) / L.stride + 1;
      cin = L.cout;
    }
    if (out_size > 0 && size != out_size) throw ArgError("output grid not reachable by halving the input grid");
    ConvLayer H;
    H.cin = cin, H.cout = out_channels, H.k = 1, H.pad = 0, H.stride = 1, H.relu = 0;
    layers_.push_back(H);
    sizes_.push_back(size);
    out_size_ = size;
    // parameters: one arena of masters, gradients and moments
    int64_t total = 0;
    for (auto& L : layers_) total += L.nw() + L.cout;
    nparam_ = total;
    if (hipMalloc(&arena_, sizeof(float) * total * 5) != hipSuccess) throw std::bad_alloc();
    float* p = arena_;
    std::vector<float> host(total);
    std::mt19937_64 rng(seed);
    int64_t o = 0;
    for (auto& L : layers_) {
      const int fan_in = L.cin * L.k * L.k * L.k;
      std::normal_distribution<float> nd(0.f, std::sqrt(2.f / fan_in) * (L.relu ? 1.f : 0.1f));
      for (int64_t i = 0; i < L.nw(); ++i) host[o + i] = nd(rng);
      for (int i = 0; i < L.cout; ++i) host[o + L.nw() + i] = 0.f;
      L.w = p + o;
      L.b = p + o + L.nw();
      L.dw = L.w + total;
      L.db = L.b + total;
      L.mw = L.w + 2 * total;
      L.mb = L.b + 2 * total;
      L.vw = L.w + 3 * total;
      L.vb = L.b + 3 * total;
      o += L.nw() + L.cout;
    }
    LDDMM_HIP(hipMemcpy(arena_, host.data(), sizeof(float) * total, hipMemcpyHostToDevice));
    fill(arena_ + total, 4 * total, 0.f, st_);
    LDDMM_HIP(hipStreamSynchronize(st_));
  }
  ~Net() {
    if (arena_) (void)hipFree(arena_);
    for (auto* a : acts_) (void)hipFree(a);
    if (gbuf_) (void)hipFree(gbuf_);
    if (dbuf_[0]) (void)hipFree(dbuf_[0]);
    if (dbuf_[1]) (void)hipFree(dbuf_[1]);
    if (P_) (void)hipFree(P_);
    if (diff_) (void)hipFree(diff_);
    if (Lw_) (void)hipFree(Lw_);
    if (work_) (void)hipFree(work_);
    if (host_) (void)hipHostFree(host_);
  }

  int out_size() const { return out_size_; }
  int out_channels() const { return layers_.back().cout; }
  int64_t nparam() const { return nparam_; }

  // Parameter file: the 8-byte tag, levels, channels[levels], in_size, rank_r (int32 each), the
  // parameter count (int64) and the float master parameters in layer order (weights, then biases).
  // A network with a requested output grid writes the second tag and out_size (int32) after rank_r;
  // files with the first tag hold networks of the default schedule.
  static constexpr char kTag[8] = {'L', 'D', 'D', 'M', 'M', 'N', 'N', '1'};
  static constexpr char kTag2[8] = {'L', 'D', 'D', 'M', 'M', 'N', 'N', '2'};
  void save(const char* path) {
    std::vector<float> h(nparam_);
    get(h.data(), 0);
    std::FILE* f = std::fopen(path, "wb");
    if (!f) throw ArgError(std::string("cannot open for writing: ") + path);
    std::vector<int32_t> hdr{(int32_t)channels_.size()};
    for (int c : channels_) hdr.push_back(c);
    hdr.push_back(in_size_);
    hdr.push_back(rank_);
    if (req_out_ > 0) hdr.push_back(req_out_);
    const int64_t n = nparam_;
    bool ok = std::fwrite(req_out_ > 0 ? kTag2 : kTag, 1, 8, f) == 8 &&
              std::fwrite(hdr.data(), 4, hdr.size(), f) == hdr.size() &&
              std::fwrite(&n, 8, 1, f) == 1 && std::fwrite(h.data(), 4, h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw ArgError(std::string("cannot write ") + path);
  }
  void load(const char* path) {
    std::FILE* f = std::fopen(path, "rb");
    if (!f) throw ArgError(std::string("cannot open: ") + path);
    char tag[8];
    int32_t levels = 0;
    bool ok = std::fread(tag, 1, 8, f) == 8;
    const bool v2 = ok && std::memcmp(tag, kTag2, 8) == 0;
    ok = ok && (v2 || std::memcmp(tag, kTag, 8) == 0) && std::fread(&levels, 4, 1, f) == 1 &&
         levels == (int32_t)channels_.size();
    std::vector<int32_t> hdr(ok ? levels + (v2 ? 3 : 2) : 0);
    int64_t n = -1;
    ok = ok && std::fread(hdr.data(), 4, hdr.size(), f) == hdr.size() && std::fread(&n, 8, 1, f) == 1;
    for (int l = 0; ok && l < levels; ++l) ok = hdr[l] == channels_[l];
    // the file's output grid (the default schedule's for the first tag) must be this network's
    ok = ok && hdr[levels] == in_size_ && hdr[levels + 1] == rank_ && n == nparam_ &&
         (v2 ? hdr[levels + 2] : (in_size_ >> (levels - 1))) == out_size_;
    std::vector<float> h(ok ? nparam_ : 0);
    ok = ok && std::fread(h.data(), 4, h.size(), f) == h.size();
    std::fclose(f);
    if (!ok) throw ArgError(std::string("parameter file does not match this network: ") + path);
    set(h.data());
  }

  void forward(const float* in, int B, float* out) {
    ensure(B);
    const float* x = in;
    in_ = in;
    for (size_t l = 0; l < layers_.size(); ++l) {
      float* y = (l + 1 == layers_.size()) ? out : acts_[l];
      conv_forward(layers_[l], x, y, B, sizes_[l], st_);
      x = y;
    }
    out_ = out;
    lastB_ = B;
    LDDMM_HIP(hipStreamSynchronize(st_));
  }

  // accumulates parameter gradients for the last forward pass
  void backward(const float* dout, int B) {
    if (B != lastB_ || !out_) throw StateError("backward needs a forward pass with the same batch");
    const float* dy = dout;
    for (int l = static_cast<int>(layers_.size()) - 1; l >= 0; --l) {
      const float* x = l == 0 ? in_ : acts_[l - 1];
      const float* y = (l + 1 == (int)layers_.size()) ? out_ : acts_[l];
      float* dx = l == 0 ? nullptr : dbuf_[l & 1];
      conv_backward(layers_[l], x, y, dy, gbuf_, dx, B, sizes_[l], st_);
      dy = dx;
    }
    LDDMM_HIP(hipStreamSynchronize(st_));
  }

  void zero_grad() {
    fill(arena_ + nparam_, nparam_, 0.f, st_);
    LDDMM_HIP(hipStreamSynchronize(st_));
  }

  void step(float lr) {
    ++t_;
    adam_step(arena_, arena_ + 2 * nparam_, arena_ + 3 * nparam_, arena_ + nparam_, nparam_, lr, t_, st_);
    LDDMM_HIP(hipStreamSynchronize(st_));
  }

  void get(float* host, int which) {
    LDDMM_HIP(hipMemcpy(host, arena_ + which * nparam_, sizeof(float) * nparam_, hipMemcpyDeviceToHost));
  }
  void set(const float* host) {
    LDDMM_HIP(hipMemcpy(arena_, host, sizeof(float) * nparam_, hipMemcpyHostToDevice));
  }

  // image pair (n[0] x n[1] x n[2], each a multiple of the input size) -> one [2][S^3] input slot
  void pool(const float* I0, const float* I1, const int n[3], float* slot) {
    const int S = sizes_[0];
    for (int j = 0; j < 3; ++j)
      if (n[j] < S || n[j] % S) throw ArgError("image size must be a multiple of the network input size");
    pool_pair(I0, I1, n, S, slot, st_);
    LDDMM_HIP(hipStreamSynchronize(st_));
  }

  // network output [B][3(1+r)][s^3] -> coefficients [B][1+r][3][k0][k1][k2] (velocity, then directions)
  void velocity(const float* out, int B, const int k[3], float* v) {
    check_velocity_args(B, k);
    samples_to_bl(out, proj(), B * (1 + rank_), 1, out_size_, k, v, st_);
    LDDMM_HIP(hipStreamSynchronize(st_));
  }

  // mean squared V-norm error of the predicted velocities against v_target [B][3][K] and its
  // gradient with respect to the network output
  double loss(const float* out, const float* vt, int B, const int k[3], double alpha, int s_exp, float* dout) {
    check_velocity_args(B, k);
    if (alpha < 0 || s_exp < 0) throw ArgError("bad regularisation parameters");
    const int64_t Q = (int64_t)k[0] * k[1] * k[2], n = (int64_t)B * 3 * Q;
    if (n > diff_cap_) {
      if (diff_) (void)hipFree(diff_);
      diff_ = nullptr;
      if (hipMalloc(&diff_, sizeof(float) * n) != hipSuccess) throw std::bad_alloc();
      diff_cap_ = n;
    }
    weights(k, alpha, s_exp);
    const int gs = 1 + rank_;  // the velocity channels are the first 3 of each sample's 3 (1 + r)
    samples_to_bl(out, proj(), B, gs, out_size_, k, diff_, st_);
    bl_axpby<float>(diff_, 1.f, diff_, -1.f, vt, n, st_);
    if (!work_) {
      if (hipMalloc(&work_, sizeof(double) * reduce_work_size()) != hipSuccess) throw std::bad_alloc();
      if (hipHostMalloc(reinterpret_cast<void**>(&host_), 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
        throw std::bad_alloc();
    }
    const double l = sym_dot<float>(diff_, diff_, Lw_, 3 * B, Q, work_, host_, st_) / B;
    if (dout) {
      // the loss does not depend on the direction channels
      if (rank_ > 0) fill(dout, (int64_t)B * out_channels() * out_size_ * out_size_ * out_size_, 0.f, st_);
      block_grad(diff_, Lw_, proj(), B, gs, out_size_, k, 2.f / B, dout, st_);
    }
    LDDMM_HIP(hipStreamSynchronize(st_));
    return l;
  }

 private:
  void check_velocity_args(int B, const int k[3]) const {
    if (B < 1) throw ArgError("batch must be >= 1");
    for (int j = 0; j < 3; ++j)
      if (k[j] < out_size_ - 1 || k[j] < 2 || k[j] % 2) throw ArgError("band too small for the network output");
  }
  // projection onto the out_size-point band: P[a][x] = b_a(x / s) / s in the real basis
  // (slot 0 the constant, 2m-1 / 2m sqrt2 cos / sqrt2 sin of frequency m, last slot zero)
  const float* proj() {
    if (P_) return P_;
    const int sz = out_size_;
    std::vector<float> h((size_t)sz * sz, 0.f);
    const double r2 = std::sqrt(2.0), tp = 2.0 * M_PI;
    for (int x = 0; x < sz; ++x) {
      const double xx = (double)x / sz;
      h[x] = (float)(1.0 / sz);
      for (int m = 1; 2 * m < sz; ++m) {
        h[(2 * m - 1) * sz + x] = (float)(r2 * std::cos(tp * m * xx) / sz);
        h[(2 * m) * sz + x] = (float)(r2 * std::sin(tp * m * xx) / sz);
      }
    }
    if (hipMalloc(&P_, sizeof(float) * h.size()) != hipSuccess) throw std::bad_alloc();
    LDDMM_HIP(hipMemcpy(P_, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice));
    return P_;
  }
  // diagonal of L~ = (1 + alpha (2 pi)^2 |m|^2)^s on the real slots (zero on the pad slots)
  void weights(const int k[3], double alpha, int s_exp) {
    if (Lw_ && k[0] == wk_[0] && k[1] == wk_[1] && k[2] == wk_[2] && alpha == walpha_ && s_exp == ws_) return;
    const int64_t Q = (int64_t)k[0] * k[1] * k[2];
    std::vector<double> h(Q);
    auto fr = [](int a, int K) { return a == K - 1 ? -1 : (a + 1) / 2; };
    const double c = alpha * 4.0 * M_PI * M_PI;
    for (int a0 = 0; a0 < k[0]; ++a0)
      for (int a1 = 0; a1 < k[1]; ++a1)
        for (int a2 = 0; a2 < k[2]; ++a2) {
          const int f0 = fr(a0, k[0]), f1 = fr(a1, k[1]), f2 = fr(a2, k[2]);
          double w = 0.0;
          if (f0 >= 0 && f1 >= 0 && f2 >= 0) w = std::pow(1.0 + c * (f0 * f0 + f1 * f1 + f2 * f2), s_exp);
          h[((int64_t)a0 * k[1] + a1) * k[2] + a2] = w;
        }
    if (Lw_) (void)hipFree(Lw_);
    Lw_ = nullptr;
    if (hipMalloc(&Lw_, sizeof(double) * Q) != hipSuccess) throw std::bad_alloc();
    LDDMM_HIP(hipMemcpy(Lw_, h.data(), sizeof(double) * Q, hipMemcpyHostToDevice));
    wk_[0] = k[0], wk_[1] = k[1], wk_[2] = k[2], walpha_ = alpha, ws_ = s_exp;
  }

  int64_t act_elems(int l, int B) const {
    const int so = (l + 1 < (int)sizes_.size()) ? sizes_[l + 1] : out_size_;
    return (int64_t)B * layers_[l].cout * so * so * so;
  }
  void ensure(int B) {
    if (B <= capB_) return;
    for (auto* a : acts_) (void)hipFree(a);
    acts_.clear();
    int64_t maxe = 0;
    for (size_t l = 0; l < layers_.size(); ++l) {
      const int64_t e = act_elems(static_cast<int>(l), B);
      maxe = std::max(maxe, e);
      float* a = nullptr;
      if (l + 1 < layers_.size()) {
        if (hipMalloc(&a, sizeof(float) * e) != hipSuccess) throw std::bad_alloc();
        acts_.push_back(a);
      }
    }
    const int64_t in_e = (int64_t)B * 2 * sizes_[0] * sizes_[0] * sizes_[0];
    maxe = std::max(maxe, in_e);
    if (gbuf_) (void)hipFree(gbuf_);
    if (dbuf_[0]) (void)hipFree(dbuf_[0]);
    if (dbuf_[1]) (void)hipFree(dbuf_[1]);
    if (hipMalloc(&gbuf_, sizeof(float) * maxe) != hipSuccess || hipMalloc(&dbuf_[0], sizeof(float) * maxe) != hipSuccess ||
        hipMalloc(&dbuf_[1], sizeof(float) * maxe) != hipSuccess)
      throw std::bad_alloc();
    capB_ = B;
  }

  hipStream_t st_;
  int rank_ = 0, in_size_ = 0;
  std::vector<int> channels_;
  std::vector<ConvLayer> layers_;
  std::vector<int> sizes_;  // input size of each layer
  int out_size_ = 0, req_out_ = 0, capB_ = 0, lastB_ = 0, t_ = 0;
  int64_t nparam_ = 0;
  float* arena_ = nullptr;
  std::vector<float*> acts_;
  float* gbuf_ = nullptr;
  float* dbuf_[2] = {nullptr, nullptr};
  const float* in_ = nullptr;
  const float* out_ = nullptr;
  float* P_ = nullptr;
  float* diff_ = nullptr;
  int64_t diff_cap_ = 0;
  double* Lw_ = nullptr;
  int wk_[3] = {0, 0, 0}, ws_ = -1;
  double walpha_ = -1.0;
  double* work_ = nullptr;
  double* host_ = nullptr;
};

}  // namespace lddmm

struct lddmm_nn_ctx {
  std::unique_ptr<lddmm::Net> net;
};

namespace {
template <typename F>
lddmm_bl_status nn_guard(lddmm_nn_ctx* c, F&& f) {
  if (!c || !c->net) {
    lddmm::set_global_error("null network context");
    return LDDMM_BL_E_ARG;
  }
  try {
    f();
    return LDDMM_BL_OK;
  } catch (const lddmm::ArgError& e) {
    lddmm::set_global_error(e.what());
    return LDDMM_BL_E_ARG;
  } catch (const lddmm::StateError& e) {
    lddmm::set_global_error(e.what());
    return LDDMM_BL_E_STATE;
  } catch (const std::bad_alloc&) {
    lddmm::set_global_error("device allocation failed");
    return LDDMM_BL_E_OOM;
  } catch (const std::exception& e) {
    lddmm::set_global_error(e.what());
    return LDDMM_BL_E_HIP;
  } catch (...) {
    lddmm::set_global_error("unknown error");
    return LDDMM_BL_E_HIP;
  }
}
}  // namespace

extern "C" {

lddmm_bl_status lddmm_nn_create(int32_t levels, const int32_t* channels, int32_t in_size, int32_t rank_r,
                                uint64_t seed, void* hip_stream, lddmm_nn_ctx** out) {
  return lddmm_nn_create_out(levels, channels, in_size, 0, rank_r, seed, hip_stream, out);
}

lddmm_bl_status lddmm_nn_create_out(int32_t levels, const int32_t* channels, int32_t in_size, int32_t out_size,
                                    int32_t rank_r, uint64_t seed, void* hip_stream, lddmm_nn_ctx** out) {
  if (!channels || !out) return LDDMM_BL_E_ARG;
  *out = nullptr;
  auto* c = new (std::nothrow) lddmm_nn_ctx();
  if (!c) return LDDMM_BL_E_OOM;
  try {
    c->net = std::make_unique<lddmm::Net>(levels, channels, in_size, rank_r, seed,
                                          static_cast<hipStream_t>(hip_stream), out_size);
  } catch (const lddmm::ArgError& e) {
    lddmm::set_global_error(e.what());
    delete c;
    return LDDMM_BL_E_ARG;
  } catch (const std::exception& e) {
    lddmm::set_global_error(e.what());
    delete c;
    return LDDMM_BL_E_OOM;
  } catch (...) {
    lddmm::set_global_error("unknown error");
    delete c;
    return LDDMM_BL_E_OOM;
  }
  *out = c;
  return LDDMM_BL_OK;
}

lddmm_bl_status lddmm_nn_save(const lddmm_nn_ctx* c, const char* path) {
  return nn_guard(const_cast<lddmm_nn_ctx*>(c), [&] {
    if (!path) throw lddmm::ArgError("null path");
    c->net->save(path);
  });
}

lddmm_bl_status lddmm_nn_load(lddmm_nn_ctx* c, const char* path) {
  return nn_guard(c, [&] {
    if (!path) throw lddmm::ArgError("null path");
    c->net->load(path);
  });
}

lddmm_bl_status lddmm_nn_destroy(lddmm_nn_ctx* c) {
  if (!c) return LDDMM_BL_E_ARG;
  delete c;
  return LDDMM_BL_OK;
}

lddmm_bl_status lddmm_nn_info(lddmm_nn_ctx* c, int32_t* out_size, int32_t* out_channels, int64_t* nparam) {
  return nn_guard(c, [&] {
    if (out_size) *out_size = c->net->out_size();
    if (out_channels) *out_channels = c->net->out_channels();
    if (nparam) *nparam = c->net->nparam();
  });
}

lddmm_bl_status lddmm_nn_forward(lddmm_nn_ctx* c, const void* in, int32_t B, void* out) {
  return nn_guard(c, [&] {
    if (!in || !out || B < 1) throw lddmm::ArgError("bad forward arguments");
    c->net->forward(static_cast<const float*>(in), B, static_cast<float*>(out));
  });
}

lddmm_bl_status lddmm_nn_backward(lddmm_nn_ctx* c, const void* dout, int32_t B) {
  return nn_guard(c, [&] {
    if (!dout) throw lddmm::ArgError("null gradient");
    c->net->backward(static_cast<const float*>(dout), B);
  });
}

lddmm_bl_status lddmm_nn_zero_grad(lddmm_nn_ctx* c) {
  return nn_guard(c, [&] { c->net->zero_grad(); });
}

lddmm_bl_status lddmm_nn_step(lddmm_nn_ctx* c, double lr) {
  return nn_guard(c, [&] { c->net->step(static_cast<float>(lr)); });
}

lddmm_bl_status lddmm_nn_get(lddmm_nn_ctx* c, int32_t which, void* host_dst) {
  return nn_guard(c, [&] {
    if (!host_dst || which < 0 || which > 1) throw lddmm::ArgError("bad get arguments");
    c->net->get(static_cast<float*>(host_dst), which);
  });
}

lddmm_bl_status lddmm_nn_set(lddmm_nn_ctx* c, const void* host_src) {
  return nn_guard(c, [&] {
    if (!host_src) throw lddmm::ArgError("null parameters");
    c->net->set(static_cast<const float*>(host_src));
  });
}

lddmm_bl_status lddmm_nn_pool_pair(lddmm_nn_ctx* c, const void* I0, const void* I1, const int32_t* n,
                                   void* in_slot) {
  return nn_guard(c, [&] {
    if (!I0 || !I1 || !n || !in_slot) throw lddmm::ArgError("null pool arguments");
    const int nn[3] = {n[0], n[1], n[2]};
    c->net->pool(static_cast<const float*>(I0), static_cast<const float*>(I1), nn, static_cast<float*>(in_slot));
  });
}

lddmm_bl_status lddmm_nn_velocity(lddmm_nn_ctx* c, const void* out, int32_t B, const int32_t* k, void* v_bl) {
  return nn_guard(c, [&] {
    if (!out || !k || !v_bl) throw lddmm::ArgError("null velocity arguments");
    const int kk[3] = {k[0], k[1], k[2]};
    c->net->velocity(static_cast<const float*>(out), B, kk, static_cast<float*>(v_bl));
  });
}

lddmm_bl_status lddmm_nn_loss(lddmm_nn_ctx* c, const void* out, const void* v_target, int32_t B, const int32_t* k,
                              double alpha, int32_t s, void* dout_or_null, double* loss) {
  return nn_guard(c, [&] {
    if (!out || !v_target || !k || !loss) throw lddmm::ArgError("null loss arguments");
    const int kk[3] = {k[0], k[1], k[2]};
    *loss = c->net->loss(static_cast<const float*>(out), static_cast<const float*>(v_target), B, kk, alpha, s,
                         static_cast<float*>(dout_or_null));
  });
}

}  // extern "C"
