// extern "C" entry points of the library (declared in include/lddmm_bl.h).
// Every call catches its own exceptions and turns them into status codes; the
// text of the last error is kept per context.
#include <algorithm>
#include <array>
#include <mutex>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "prof.h"
#include "solver.h"
#include "tune.h"

struct lddmm_bl_ctx {
  std::unique_ptr<lddmm::SolverBase> solver;
  std::string err;
};

namespace lddmm {
// text of the last error of a call without a context, per thread (lddmm_bl_last_error(NULL))
thread_local std::string g_last_error;
void set_global_error(const char* what) { g_last_error = what ? what : ""; }
}  // namespace lddmm

// Workspace of lddmm_bl_project_noalloc: the plane-band partial projections of its reduction (16 MiB).
// Each GPU the library runs on holds its own copy until the process ends; host code uses the device
// address hipGetSymbolAddress returns for the current device, never the array's name.
constexpr int64_t kNoAllocFloats = int64_t(4) << 20;
static __device__ __align__(256) float scratch[kNoAllocFloats];

namespace {

std::mutex g_scratch_mu;
std::array<float*, 64> g_scratch_ptr{};  // per device, set on the first call with that device current

float* scratch_for_current_device() {
  int dev = 0;
  LDDMM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= static_cast<int>(g_scratch_ptr.size())) throw lddmm::ArgError("device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw lddmm::HipError(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  return g_scratch_ptr[dev];
}

template <typename F>
lddmm_bl_status guarded(lddmm_bl_ctx* ctx, F&& f) {
  if (!ctx || !ctx->solver) return LDDMM_BL_E_ARG;
  try {
    return static_cast<lddmm_bl_status>(f());
  } catch (const lddmm::ArgError& e) {
    ctx->err = e.what();
    return LDDMM_BL_E_ARG;
  } catch (const lddmm::StateError& e) {
    ctx->err = e.what();
    return LDDMM_BL_E_STATE;
  } catch (const lddmm::NonFiniteError& e) {
    ctx->err = e.what();
    return LDDMM_BL_E_NONFINITE;
  } catch (const lddmm::HipError& e) {
    ctx->err = e.what();
    return LDDMM_BL_E_HIP;
  } catch (const std::bad_alloc&) {
    ctx->err = "device allocation failed";
    return LDDMM_BL_E_OOM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return LDDMM_BL_E_HIP;
  }
}

}  // namespace

extern "C" {

lddmm_bl_status lddmm_bl_create(const lddmm_bl_params* params, void* hip_stream, lddmm_bl_ctx** out) {
  if (!params || !out) return LDDMM_BL_E_ARG;
  *out = nullptr;
  auto* ctx = new (std::nothrow) lddmm_bl_ctx();
  if (!ctx) return LDDMM_BL_E_OOM;
  try {
    ctx->solver = lddmm::make_solver(*params, static_cast<hipStream_t>(hip_stream));
  } catch (const lddmm::ArgError& e) {
    lddmm::set_global_error(e.what());
    delete ctx;
    return LDDMM_BL_E_ARG;
  } catch (const std::bad_alloc&) {
    lddmm::set_global_error("device allocation failed");
    delete ctx;
    return LDDMM_BL_E_OOM;
  } catch (const std::exception& e) {
    lddmm::set_global_error(e.what());
    delete ctx;
    return LDDMM_BL_E_HIP;
  } catch (...) {
    lddmm::set_global_error("unknown error");
    delete ctx;
    return LDDMM_BL_E_HIP;
  }
  *out = ctx;
  return LDDMM_BL_OK;
}

lddmm_bl_status lddmm_bl_destroy(lddmm_bl_ctx* ctx) {
  if (!ctx) return LDDMM_BL_E_ARG;
  try {
    delete ctx;
  } catch (...) {
    return LDDMM_BL_E_HIP;
  }
  return LDDMM_BL_OK;
}

const char* lddmm_bl_last_error(const lddmm_bl_ctx* ctx) {
  if (!ctx) return lddmm::g_last_error.c_str();
  return ctx->err.c_str();
}

lddmm_bl_status lddmm_bl_set_images(lddmm_bl_ctx* ctx, const void* I0, const void* I1) {
  return guarded(ctx, [&] {
    if (!I0 || !I1) throw lddmm::ArgError("null image");
    ctx->solver->set_images(I0, I1);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_state_solve(lddmm_bl_ctx* ctx, const void* v_bl, void* m1_or_null, double* E) {
  return guarded(ctx, [&] {
    if (!v_bl) throw lddmm::ArgError("null velocity");
    ctx->solver->state_solve(v_bl, m1_or_null, E);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_adjoint_solve(lddmm_bl_ctx* ctx, void* grad_bl, double* grad_inf) {
  return guarded(ctx, [&] {
    ctx->solver->adjoint_solve(grad_bl, grad_inf);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_hess_matvec(lddmm_bl_ctx* ctx, const void* dv_bl, void* hdv_bl) {
  return guarded(ctx, [&] {
    if (!dv_bl || !hdv_bl) throw lddmm::ArgError("null vector");
    if (dv_bl == hdv_bl) throw lddmm::ArgError("dv and hdv may not alias");
    ctx->solver->hess_matvec(dv_bl, hdv_bl);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_gn_solve(lddmm_bl_ctx* ctx, const lddmm_bl_gn_opts* opts, void* v_bl_inout,
                                  const void* precond_Z_or_null, int32_t r, lddmm_bl_gn_report* report) {
  return guarded(ctx, [&] {
    if (!opts || !v_bl_inout) throw lddmm::ArgError("null options or velocity");
    return ctx->solver->gn_solve(*opts, v_bl_inout, precond_Z_or_null, r, report);
  });
}

lddmm_bl_status lddmm_bl_gn_solve_batched(const lddmm_bl_params* per_subject, int32_t count, const void* const* I0,
                                          const void* const* I1, void* const* v_bl_inout,
                                          const lddmm_bl_gn_opts* opts, void* hip_stream,
                                          lddmm_bl_gn_report* reports) {
  if (!per_subject || count < 1 || count > 4096 || !I0 || !I1 || !v_bl_inout || !opts) {
    lddmm::set_global_error("batched solve: null argument or count outside 1..4096");
    return LDDMM_BL_E_ARG;
  }
  if (!hip_stream) {  // graphs need a non-default stream
    lddmm::set_global_error("batched solve: the stream must not be NULL");
    return LDDMM_BL_E_ARG;
  }
  try {
    std::vector<std::unique_ptr<lddmm::SolverBase>> owned;
    std::vector<lddmm::SolverBase*> subs;
    for (int i = 0; i < count; ++i) {
      if (per_subject[i].precision == LDDMM_BL_FP64) throw lddmm::ArgError("batched subjects must be float");
      if (per_subject[i].nonstationary) throw lddmm::ArgError("batched subjects must have stationary velocities");
      owned.push_back(lddmm::make_solver(per_subject[i], static_cast<hipStream_t>(hip_stream)));
      owned.back()->set_images(I0[i], I1[i]);
      subs.push_back(owned.back().get());
    }
    return static_cast<lddmm_bl_status>(
        lddmm::gn_solve_batched(subs, *opts, v_bl_inout, reports, static_cast<hipStream_t>(hip_stream)));
  } catch (const lddmm::ArgError& e) {
    lddmm::set_global_error(e.what());
    return LDDMM_BL_E_ARG;
  } catch (const lddmm::StateError& e) {
    lddmm::set_global_error(e.what());
    return LDDMM_BL_E_STATE;
  } catch (const lddmm::NonFiniteError& e) {
    lddmm::set_global_error(e.what());
    return LDDMM_BL_E_NONFINITE;
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

lddmm_bl_status lddmm_bl_jacobian(lddmm_bl_ctx* ctx, void* detmap_or_null, double* minmax) {
  return guarded(ctx, [&] {
    ctx->solver->jacobian(static_cast<double*>(detmap_or_null), minmax);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_project(lddmm_bl_ctx* ctx, const void* grid, void* bl, int32_t ncomp) {
  return guarded(ctx, [&] {
    if (!grid || !bl) throw lddmm::ArgError("null buffer");
    ctx->solver->project(grid, bl, ncomp);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_project_noalloc(lddmm_bl_ctx* ctx, const void* grid, void* bl, int32_t ncomp) {
  return guarded(ctx, [&] {
    if (!grid || !bl) throw lddmm::ArgError("null buffer");
    float* ws = scratch_for_current_device();
    ctx->solver->project_ws(grid, bl, ncomp, ws, kNoAllocFloats);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_include(lddmm_bl_ctx* ctx, const void* bl, void* grid, int32_t ncomp) {
  return guarded(ctx, [&] {
    if (!grid || !bl) throw lddmm::ArgError("null buffer");
    ctx->solver->include(bl, grid, ncomp);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_get_field(lddmm_bl_ctx* ctx, int32_t which, int32_t index, void* dst, int64_t* count) {
  return guarded(ctx, [&] {
    const int64_t c = ctx->solver->get_field(which, index, dst);
    if (count) *count = c;
    return 0;
  });
}

lddmm_bl_status lddmm_bl_dot(lddmm_bl_ctx* ctx, const void* a, const void* b, int64_t n, double* dot) {
  return guarded(ctx, [&] {
    if (!a || !b || !dot || n < 0) throw lddmm::ArgError("bad dot arguments");
    *dot = ctx->solver->dot(a, b, n);
    return 0;
  });
}

lddmm_bl_status lddmm_bl_profile_enable(int32_t on) {
  try {
    if (on) lddmm::prof::collect();  // drop stale records
    lddmm::prof::set_enabled(on != 0);
  } catch (...) {
    return LDDMM_BL_E_HIP;
  }
  return LDDMM_BL_OK;
}

int32_t lddmm_bl_tune_candidates(const char* family) {
  if (family && std::strcmp(family, "brick") == 0) return lddmm::brick_tile_count();
  if (family && std::strcmp(family, "dft") == 0) return lddmm::dft_cap_count();
  return 0;
}

int32_t lddmm_bl_tune_get(const char* key) {
  if (!key) return -1;
  try {
    return lddmm::tune::get(key, -1);
  } catch (...) {
    return -1;
  }
}

lddmm_bl_status lddmm_bl_tune_set(const char* key, int32_t choice) {
  if (!key) return LDDMM_BL_E_ARG;
  int ncand = 0;
  if (std::strncmp(key, "brick:", 6) == 0) ncand = lddmm::brick_tile_count();
  else if (std::strncmp(key, "dft:", 4) == 0) ncand = lddmm::dft_cap_count();
  else return LDDMM_BL_E_ARG;
  if (choice < -1 || choice >= ncand) return LDDMM_BL_E_ARG;
  try {
    lddmm::tune::set(key, choice);
  } catch (...) {
    return LDDMM_BL_E_HIP;
  }
  return LDDMM_BL_OK;
}

int64_t lddmm_bl_tune_table(char* buf, int64_t len) {
  static std::string last;
  if (buf == nullptr || len <= 0) {
    try {
      last.clear();
      for (const auto& kv : lddmm::tune::table()) last += kv.first + "=" + std::to_string(kv.second) + "\n";
    } catch (...) {
      return -1;
    }
    return static_cast<int64_t>(last.size()) + 1;
  }
  const int64_t n = std::min<int64_t>(len - 1, static_cast<int64_t>(last.size()));
  std::memcpy(buf, last.data(), static_cast<size_t>(n));
  buf[n] = 0;
  return n;
}

int64_t lddmm_bl_profile_read(char* buf, int64_t len) {
  static std::string last;
  if (buf == nullptr || len <= 0) {
    last = lddmm::prof::collect();
    return static_cast<int64_t>(last.size()) + 1;
  }
  const int64_t n = std::min<int64_t>(len - 1, static_cast<int64_t>(last.size()));
  std::memcpy(buf, last.data(), n);
  buf[n] = 0;
  return n + 1;
}

}  // extern "C"
