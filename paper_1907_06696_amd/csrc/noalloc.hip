// The Q2 strain-rate operator on a uniform mesh without any allocation:
// mfgmg_vmult_uniform_noalloc (declared in include/mfgmg.h).
//
// The brick operator of a uniform level needs, besides x, y and the cell
// viscosity, its halo slots: per brick the contributions to the nodes of its
// upper neighbours, written by the brick kernel and added by the halo kernel,
// plus a zero pad that the halo kernel reads in place of slots that do not
// apply.  Here those slots live in one file-scope device array, `scratch`,
// sized for the largest mesh this entry point takes (64^3 cells, FP64:
// 1024 bricks of 8x8x4 cells), instead of a buffer the library
// allocates per context.  Each GPU the library runs on holds its own copy of
// the array until the process ends; its device address is looked up once
// per device (hipGetSymbolAddress) and only that address is passed to kernels.
// Calls on one GPU share the array: work enqueued by overlapping calls (other
// streams, other threads) races on it.  Only the zero pad must hold zeros; it
// is cleared by a fill kernel at every call (a previous call on a larger mesh
// may have written slots there).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/mfgmg.h"
#include "brick_kernel.h"
#include "ops.h"

namespace mfgmg {
namespace detail {
extern thread_local std::string g_last_error;
}
}

namespace {

using namespace mfgmg;
using detail::g_last_error;

constexpr int kMaxEdge = 64;   // largest mesh: 64^3 cells
// halo words of the brick shapes the operator uses on the supported edges
constexpr int64_t kMaxWords = brick::halo_buffer_words(32) > brick::halo_buffer_words(kMaxEdge)
                                  ? brick::halo_buffer_words(32)
                                  : brick::halo_buffer_words(kMaxEdge);
constexpr int64_t kScratchBytes = kMaxWords * 8;   // FP64 words

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).  Returns nullptr and sets the message on failure.
void* scratch_address(std::string& err) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    err = "no current HIP device";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(rc);
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

bool edge_supported(int64_t n) {
  return n == 32 || n == 64;
}

}  // namespace

extern "C" int mfgmg_vmult_uniform_noalloc(int32_t n_edge, mfgmg_prec prec, const void* mu, const void* src,
                                           void* dst, void* stream) {
  if (n_edge > kMaxEdge) {
    g_last_error = "n_edge " + std::to_string(n_edge) + " exceeds the scratch limit of " + std::to_string(kMaxEdge) +
                   " cells per edge";
    return MFGMG_ERR_INVALID;
  }
  if (!edge_supported(n_edge)) {
    g_last_error = "n_edge must be 32 or 64";
    return MFGMG_ERR_INVALID;
  }
  if (!mu || !src || !dst || src == dst || (prec != MFGMG_FP32 && prec != MFGMG_FP64)) {
    g_last_error = "null or aliased pointer, or bad precision";
    return MFGMG_ERR_INVALID;
  }
  std::string err;
  void* base = scratch_address(err);
  if (!base) {
    g_last_error = err;
    return MFGMG_ERR_HIP;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = n_edge;
  DevLevel v;
  v.uniform = true;
  v.n_edge = n;
  v.ncell = n * n * n;
  v.nnode = (2 * n + 1) * (2 * n + 1) * (2 * n + 1);
  if (prec == MFGMG_FP64) {
    const int64_t words = brick_halo_words<double>(n);
    if (words <= 64 || words * int64_t(sizeof(double)) > kScratchBytes) {
      g_last_error = "halo slots exceed the scratch array";
      return MFGMG_ERR_INVALID;
    }
    v.mu_d = static_cast<const double*>(mu);
    v.halo_d = static_cast<double*>(base);
    launch_fill(64, 0.0, v.halo_d + (words - 64), s);
    launch_vmult<double>(v, static_cast<const double*>(src), static_cast<double*>(dst), s, true);
  } else {
    const int64_t words = brick_halo_words<float>(n);
    if (words <= 64 || words * int64_t(sizeof(float)) > kScratchBytes) {
      g_last_error = "halo slots exceed the scratch array";
      return MFGMG_ERR_INVALID;
    }
    v.mu_f = static_cast<const float*>(mu);
    v.halo_f = static_cast<float*>(base);
    launch_fill_f(64, 0.0f, v.halo_f + (words - 64), s);
    launch_vmult<float>(v, static_cast<const float*>(src), static_cast<float*>(dst), s, true);
  }
  const hipError_t rc = hipGetLastError();
  if (rc != hipSuccess) {
    g_last_error = std::string("launch failed: ") + hipGetErrorString(rc);
    return MFGMG_ERR_HIP;
  }
  return MFGMG_OK;
}
