// Learned smoother scaling: device kernels and launchers (internal header).
//
// Not part of the paper, whose Chebyshev smoother is preconditioned by the
// inverse diagonal (Sec. 2.2.1).  The extension replaces diag(1/d) on a level
// by diag(s/d); s_(node, c) = exp(mean of y_{K,c} over the cells K holding the
// node), y_K = MLP(27 relative log10 viscosities of K's 3x3x3 neighbourhood),
// MLP 27 -> 64 -> 64 -> 3 with GELU (erf form) and the output clamped to
// [-2, 2].  Parameters (6147 floats) are stored as W1[64][27], b1[64],
// W2[64][64], b2[64], W3[3][64], b3[3], row-major [out][in].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ops.h"

namespace mfgmg {
namespace learned {

constexpr int kIn = 27, kH = 64, kOut = 3;
constexpr int kParams = kIn * kH + kH + kH * kH + kH + kH * kOut + kOut;   // 6147
constexpr int kCache = kH + kH + kOut;                                       // z1, z2, z3 per sample
constexpr int kOffB1 = kIn * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH,
              kOffB3 = kOffW3 + kH * kOut;
constexpr float kClamp = 2.0f;

// per-dof scaling on a level: acc/cnt (zeroed by the caller) accumulate y
// over the cells holding each free node; finish writes s (per dof, 1 on
// constrained dofs) and minv_s = s * minv
void launch_scaling_accum(const DevLevel& L, const double* y, double* acc, double* cnt, hipStream_t s);
void launch_scaling_finish(int64_t nnode, const double* acc, const double* cnt, const double* minv, double* sdof,
                           double* minv_s_d, float* minv_s_f, hipStream_t s);
// ybar_{K,c} = sum over the free nodes a of K of sbar_(a,c) s_(a,c) / cnt_a
void launch_scaling_grad(const DevLevel& L, const double* sbar, const double* sdof, const double* cnt, double* ybar,
                         hipStream_t s);
// adjoint Chebyshev step pieces:
//   a: dbar += xbar; rbar += beta minv dbar; sbar += sgn beta dbar r_k minv_plain
//   b: dbar = alpha dbar - t
void launch_chebrev_a(int64_t n, const double* xbar, const double* minv, const double* minv_plain, const double* rk,
                      double* dbar, double* rbar, double* sbar, double beta, double sgn, hipStream_t s);
void launch_chebrev_b(int64_t n, double* dbar, const double* t, double alpha, hipStream_t s);
// out = v / minv (the Ritz vector weighted by M = diag(1 / minv))
void launch_ritz_mass(int64_t n, const double* v, const double* minv, double* out, hipStream_t s);
// sbar -= coef v^2 / (minv sdof): the part of dJ/ds that goes through lambda(s)
void launch_lambda_term(int64_t n, const double* v, const double* minv, const double* sdof, double coef, double* sbar,
                        hipStream_t s);
// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// w -= lr (m / bc1) / (sqrt(v / bc2) + eps), bc = 1 - b^t; clamp > 0 clips w
template <typename T>
void launch_adam(int64_t n, T* w, const T* g, T* m, T* v, double lr, double b1, double b2, double eps, int64_t t,
                 double clamp, hipStream_t s);
// features: feat[c][j] = log10 mu_all[nbr[c][j]] - log10 mu_all[self[c]]
void launch_features(int64_t ncell, const int32_t* nbr, const int32_t* self, const double* mu_all, float* feat,
                     hipStream_t s);
// MLP over n samples (x: [n][27], y: [n][3], cache: [n][131])
void launch_mlp_forward(const float* w, const float* x, int64_t n, float* y, float* cache, hipStream_t s);
// gradient of sum(dy * y) w.r.t. the parameters; work >= n * 260 floats,
// part >= ceil(n / 64) * 6147 floats
void launch_mlp_backward(const float* w, const float* x, const float* cache, const float* dy, int64_t n, float* dw,
                         float* work, float* part, hipStream_t s);
// dy = scale (y - t) over n3 entries; loss[0] += sum (y - t)^2 (double)
void launch_mse(int64_t n3, const float* y, const float* t, float* dy, float scale, double* loss, hipStream_t s);
// dst[i][:] = src[idx[i]][:] (cols floats per row)
void launch_gather_rows(const float* src, int cols, const int64_t* idx, int64_t n, float* dst, hipStream_t s);
void launch_d2f(int64_t n, const double* a, float* b, hipStream_t s);
void launch_f2d(int64_t n, const float* a, double* b, hipStream_t s);

}  // namespace learned
}  // namespace mfgmg
