// Library context shared by the host drivers (internal header).
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/mfgmg.h"
#include "mesh.h"
#include "ops.h"

namespace mfgmg {

struct LevelDev {
  DevLevel v;
  double* mu_d = nullptr;
  float* mu_f = nullptr;
  double* minv_d = nullptr;
  float* minv_f = nullptr;
  const int64_t* P_ptr = nullptr;
  const int32_t* P_col = nullptr;
  const float* P_w = nullptr;
  const int64_t* R_ptr = nullptr;
  const int32_t* R_col = nullptr;
  const float* R_w = nullptr;
  const int32_t* mu_src = nullptr;
  double lambda = 0.0;               // plain smoother: minv = 1/diag, Chebyshev bound
  void* work[2][5] = {{nullptr}};   // [prec][b, x, r, d, t]
  // learned scaling (installed by mfgmg_set_scaling): minv_s = s / diag
  double* minv_s_d = nullptr;
  float* minv_s_f = nullptr;
  double lambda_s = 0.0;
  bool scaled = false;
  double* node_count = nullptr;     // cells per free node (lazily built)
  double* lz_p = nullptr;           // eigenvalue-estimate search direction
};


// One level of the local-smoothing hierarchy above its uniform base.
struct LocalDev {
  LevelDev a;                       // refinement edge fixed: smoother operator, transfers from below, work
  LevelDev k;                       // refinement edge free: interface terms (shares a's viscosity)
  const uint8_t* kind = nullptr;    // per node: 0 inner, 1 domain boundary, 2 refinement edge
  const int32_t* gc_cell = nullptr; // per cell: its cell in the global-coarsening level
  const int32_t* copy_leaf = nullptr;
  const int32_t* copy_node = nullptr;
  int64_t ncopy = 0;
  void* ext[2][2] = {{nullptr}};    // [prec][coarse correction z, K y_E]
};

}  // namespace mfgmg

struct mfgmg_ctx {
  std::unique_ptr<mfgmg::Mesh> mesh;
  std::string err;
  bool dev_ready = false;
  bool mu_ready = false;
  int device = -1;
  std::vector<void*> allocs;
  std::vector<mfgmg::LevelDev> lv;
  mfgmg::DevPressure pres;
  double* khat_d = nullptr;
  double* Ainv_d = nullptr;
  float* Ainv_f = nullptr;
  int32_t* coarse_free = nullptr;
  int ncfree = 0;
  double* red_part = nullptr;   // reduction partials
  double* red_res = nullptr;    // device results (up to 128)
  double* host_res = nullptr;   // pinned host copy
  double* pmass_minv = nullptr; // Jacobi preconditioner of M_p
  double* pmean_w = nullptr;    // int psi_j (constrained) for the zero-mean pressure
  double pmean_total = 0.0;
  std::vector<double> mu_host_leaf;
  bool use_scaling = false;     // V-cycles use the installed scalings
  std::vector<void*> scratch;   // learned-part work buffers (released with the context)
  hipStream_t capture_stream = nullptr;   // V-cycle graph capture (default priority)
  // local-smoothing hierarchy (built on first use)
  std::vector<mfgmg::LocalDev> ls;
  bool ls_ready = false;                  // device data of the local levels
  bool ls_mu_ready = false;               // their viscosity, diagonals, bounds
  const int32_t* ls_base_leaf = nullptr;  // leaf free nodes whose finest level is the base
  const int32_t* ls_base_node = nullptr;
  int64_t ls_base_ncopy = 0;

  int set(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  template <typename T>
  T* dalloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    allocs.push_back(p);
    return static_cast<T*>(p);
  }
  template <typename T>
  T* upload(const std::vector<T>& h) {
    T* p = dalloc<T>(h.size());
    if (p && !h.empty()) (void)hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return p;
  }
};


#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return ctx->set(MFGMG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace mfgmg {
namespace detail {

int upload_mesh(mfgmg_ctx* ctx);
int upload_level(mfgmg_ctx* ctx, const Level& h, LevelDev& d, bool leaf, bool top, bool transfers, bool work);
double dot_sync(mfgmg_ctx* ctx, int64_t n, const double* a, const double* b, hipStream_t s);
template <typename T>
void smooth(mfgmg_ctx* ctx, int ell, const T* b, T* x, bool x_zero, hipStream_t s);
template <typename T>
void smooth_on(mfgmg_ctx* ctx, LevelDev& d, const T* b, T* x, bool x_zero, hipStream_t s);
template <typename T>
void vcycle(mfgmg_ctx* ctx, int ell, const T* b, T* x, hipStream_t s);
int estimate_lambda(mfgmg_ctx* ctx, int ell, hipStream_t s);
// largest eigenvalue estimate (x 1.2) of diag(minv) A on a level (FP64 CG-Lanczos);
// with basis (12 n doubles) and ritz (n) non-null, ritz receives the Ritz vector of
// that eigenvalue (M-orthonormal Lanczos basis (-1)^k z_k / sqrt(r_k . z_k))
int lanczos_lambda(mfgmg_ctx* ctx, int ell, const double* minv, double* lam, hipStream_t s,
                   double* basis = nullptr, double* ritz = nullptr);
int lanczos_on(mfgmg_ctx* ctx, LevelDev& d, const Level& h, const double* minv, double* lam, hipStream_t s,
               double* basis = nullptr, double* ritz = nullptr);
// local smoothing: device set-up (idempotent) and one V-cycle on leaf vectors
int local_setup(mfgmg_ctx* ctx, hipStream_t s);
template <typename T>
void local_vcycle(mfgmg_ctx* ctx, const T* b, T* x, hipStream_t s);
constexpr int kLanczosSteps = 12;
double splitmix_pm1(uint64_t seed, uint64_t counter);
int check_level(const mfgmg_ctx* ctx, int32_t level);

}  // namespace detail
}  // namespace mfgmg
