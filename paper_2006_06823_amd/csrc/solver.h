// Host runtime of the band-limited PDE-LDDMM solver: device workspaces, the
// SL-RK2 sweeps of both variants, the Hessian matvec and Gauss-Newton-Krylov.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "../../include/lddmm_bl.h"
#include "kernels.h"
#include "plan.h"

namespace lddmm {

// Type-erased interface used by the C ABI.
class SolverBase {
 public:
  virtual ~SolverBase() = default;
  virtual void set_images(const void* I0, const void* I1) = 0;
  virtual void state_solve(const void* v, void* m1, double* E3) = 0;
  virtual void adjoint_solve(void* grad, double* ginf) = 0;
  virtual void hess_matvec(const void* dv, void* hdv) = 0;
  virtual int gn_solve(const lddmm_bl_gn_opts& o, void* v, const void* Z, int r, lddmm_bl_gn_report* rep) = 0;
  virtual void jacobian(double* detmap, double* minmax) = 0;
  virtual void project(const void* grid, void* bl, int ncomp) = 0;
  virtual void include(const void* bl, void* grid, int ncomp) = 0;
  // project with the reduction workspace in ws (cap floats of device memory); enqueued, no host wait
  virtual void project_ws(const void* grid, void* bl, int ncomp, float* ws, int64_t cap) = 0;
  virtual int64_t get_field(int which, int index, void* dst) = 0;
  virtual double dot(const void* a, const void* b, int64_t n) = 0;
  std::string err;
};

std::unique_ptr<SolverBase> make_solver(const lddmm_bl_params& p, hipStream_t s);
int gn_solve_batched(std::vector<SolverBase*>& subs, const lddmm_bl_gn_opts& o, void* const* v_user,
                     lddmm_bl_gn_report* reps, hipStream_t st);

// Records the text of the last error of a call without a context (this thread).
void set_global_error(const char* what);

// Thrown when a call needs a state solve at the current velocity first.
class StateError : public std::runtime_error {
 public:
  explicit StateError(const std::string& s) : std::runtime_error(s) {}
};
class NonFiniteError : public std::runtime_error {
 public:
  explicit NonFiniteError(const std::string& s) : std::runtime_error(s) {}
};

}  // namespace lddmm
