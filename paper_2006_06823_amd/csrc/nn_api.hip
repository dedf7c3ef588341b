// C ABI of the learned warm-start network (declared in include/lddmm_bl.h).
//
// Architecture: `levels` convolutions with 3^3 kernels, padding 1 and ReLU, stride 2
// except the last (stride 1), channels[0..levels-1], on a 2-channel input of
// in_size^3 voxels (the image pair); then a 1^3 head to out_channels without
// activation.  The head's output, of (in_size / 2^(levels-1))^3 voxels per channel,
// is read as band-limited velocity coefficients in the real-basis layout.
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/lddmm_bl.h"
#include "nn.h"
#include "solver.h"

namespace lddmm {

class Net {
 public:
  Net(int levels, const int* channels, int in_size, int out_channels, uint64_t seed, hipStream_t s) : st_(s) {
    if (levels < 1 || levels > 6 || in_size < 4 || out_channels < 1) throw ArgError("bad network shape");
    int cin = 2, size = in_size;
    for (int l = 0; l < levels; ++l) {
      ConvLayer L;
      L.cin = cin;
      L.cout = channels[l];
      L.k = 3;
      L.pad = 1;
      L.stride = (l < levels - 1) ? 2 : 1;
      L.relu = 1;
      if (L.cout < 1 || L.cout > 1024) throw ArgError("bad channel count");
      layers_.push_back(L);
      sizes_.push_back(size);
      size = (size + 2 - 3) / L.stride + 1;
      cin = L.cout;
    }
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
  }

  int out_size() const { return out_size_; }
  int out_channels() const { return layers_.back().cout; }
  int64_t nparam() const { return nparam_; }

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

 private:
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
  std::vector<ConvLayer> layers_;
  std::vector<int> sizes_;  // input size of each layer
  int out_size_ = 0, capB_ = 0, lastB_ = 0, t_ = 0;
  int64_t nparam_ = 0;
  float* arena_ = nullptr;
  std::vector<float*> acts_;
  float* gbuf_ = nullptr;
  float* dbuf_[2] = {nullptr, nullptr};
  const float* in_ = nullptr;
  const float* out_ = nullptr;
};

}  // namespace lddmm

struct lddmm_nn_ctx {
  std::unique_ptr<lddmm::Net> net;
};

namespace {
template <typename F>
lddmm_bl_status nn_guard(lddmm_nn_ctx* c, F&& f) {
  if (!c || !c->net) return LDDMM_BL_E_ARG;
  try {
    f();
    return LDDMM_BL_OK;
  } catch (const lddmm::ArgError&) {
    return LDDMM_BL_E_ARG;
  } catch (const lddmm::StateError&) {
    return LDDMM_BL_E_STATE;
  } catch (const std::bad_alloc&) {
    return LDDMM_BL_E_OOM;
  } catch (...) {
    return LDDMM_BL_E_HIP;
  }
}
}  // namespace

extern "C" {

lddmm_bl_status lddmm_nn_create(int32_t levels, const int32_t* channels, int32_t in_size, int32_t out_channels,
                                uint64_t seed, void* hip_stream, lddmm_nn_ctx** out) {
  if (!channels || !out) return LDDMM_BL_E_ARG;
  *out = nullptr;
  auto* c = new (std::nothrow) lddmm_nn_ctx();
  if (!c) return LDDMM_BL_E_OOM;
  try {
    c->net = std::make_unique<lddmm::Net>(levels, channels, in_size, out_channels, seed,
                                          static_cast<hipStream_t>(hip_stream));
  } catch (const lddmm::ArgError&) {
    delete c;
    return LDDMM_BL_E_ARG;
  } catch (...) {
    delete c;
    return LDDMM_BL_E_OOM;
  }
  *out = c;
  return LDDMM_BL_OK;
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

}  // extern "C"
