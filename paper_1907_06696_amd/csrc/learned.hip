// Device kernels of the learned smoother scaling (see learned.h).
#include "learned.h"

#include <cmath>

namespace mfgmg {
namespace learned {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block = kBlock, int64_t cap = 1 << 20) {
  int64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return unsigned(g);
}

// velocity slot of local node a of cell c: node >= 0 when free, < 0 otherwise
// (on general levels a free slot also marks the components fixed by the
// no-normal-flux condition: slot_node / slot_fixed)
__device__ __forceinline__ int32_t lslot(const DevLevel& L, int64_t c, int a) {
  if (!L.uniform) return L.slots[27 * c + a];
  const int64_t n = L.n_edge, m = 2 * n + 1;
  const int64_t i = c % n, j = (c / n) % n, k = c / (n * n);
  const int64_t X = 2 * i + a % 3, Y = 2 * j + (a / 3) % 3, Z = 2 * k + a / 9;
  if (X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1) return -1;
  return int32_t(X + m * (Y + m * Z));
}

__global__ void k_scal_accum(DevLevel L, const double* __restrict__ y, double* __restrict__ acc,
                             double* __restrict__ cnt) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < L.ncell; c += int64_t(gridDim.x) * blockDim.x) {
    const double y0 = y[3 * c], y1 = y[3 * c + 1], y2 = y[3 * c + 2];
    for (int a = 0; a < 27; ++a) {
      const int32_t s = lslot(L, c, a);
      if (s < 0) continue;
      // a fixed component keeps s = 1 (its acc stays 0)
      const int64_t b = 3 * int64_t(slot_node(s));
      if (!slot_fixed(s, 0)) atomicAdd(&acc[b], y0);
      if (!slot_fixed(s, 1)) atomicAdd(&acc[b + 1], y1);
      if (!slot_fixed(s, 2)) atomicAdd(&acc[b + 2], y2);
      if (cnt) atomicAdd(&cnt[slot_node(s)], 1.0);
    }
  }
}

__global__ void k_scal_finish(int64_t nn, const double* __restrict__ acc, const double* __restrict__ cnt,
                              const double* __restrict__ minv, double* __restrict__ sdof, double* __restrict__ md,
                              float* __restrict__ mf) {
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < nn; v += int64_t(gridDim.x) * blockDim.x) {
    const double k = cnt[v];
    for (int q = 0; q < 3; ++q) {
      const double sv = k > 0 ? exp(acc[3 * v + q] / k) : 1.0;
      const double ms = k > 0 ? sv * minv[3 * v + q] : minv[3 * v + q];
      if (sdof) sdof[3 * v + q] = sv;
      if (md) md[3 * v + q] = ms;
      if (mf) mf[3 * v + q] = float(ms);
    }
  }
}

__global__ void k_scal_grad(DevLevel L, const double* __restrict__ sbar, const double* __restrict__ sdof,
                            const double* __restrict__ cnt, double* __restrict__ ybar) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < L.ncell; c += int64_t(gridDim.x) * blockDim.x) {
    double g0 = 0, g1 = 0, g2 = 0;
    for (int a = 0; a < 27; ++a) {
      const int32_t s = lslot(L, c, a);
      if (s < 0) continue;
      const int64_t b = 3 * int64_t(slot_node(s));
      const double ic = 1.0 / cnt[slot_node(s)];
      if (!slot_fixed(s, 0)) g0 += sbar[b] * sdof[b] * ic;
      if (!slot_fixed(s, 1)) g1 += sbar[b + 1] * sdof[b + 1] * ic;
      if (!slot_fixed(s, 2)) g2 += sbar[b + 2] * sdof[b + 2] * ic;
    }
    ybar[3 * c] = g0, ybar[3 * c + 1] = g1, ybar[3 * c + 2] = g2;
  }
}

__global__ void k_chebrev_a(int64_t n, const double* __restrict__ xbar, const double* __restrict__ minv,
                            const double* __restrict__ mp, const double* __restrict__ rk, double* __restrict__ dbar,
                            double* __restrict__ rbar, double* __restrict__ sbar, double beta, double sgn) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double d = dbar[i] + xbar[i];
    dbar[i] = d;
    rbar[i] += beta * minv[i] * d;
    sbar[i] += sgn * beta * d * rk[i] * mp[i];
  }
}

// M-weight of the Ritz vector: out_i = v_i M_ii = v_i / minv_i
__global__ void k_ritz_mass(int64_t n, const double* __restrict__ v, const double* __restrict__ minv,
                            double* __restrict__ out) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = v[i] / minv[i];
}

// term of dJ/ds through lambda(s): sbar_i -= coef v_i^2 M_ii / s_i
__global__ void k_lambda_term(int64_t n, const double* __restrict__ v, const double* __restrict__ minv,
                              const double* __restrict__ sdof, double coef, double* __restrict__ sbar) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    sbar[i] -= coef * v[i] * v[i] / (minv[i] * sdof[i]);
}

__global__ void k_chebrev_b(int64_t n, double* __restrict__ dbar, const double* __restrict__ t, double alpha) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    dbar[i] = alpha * dbar[i] - t[i];
}

template <typename T>
__global__ void k_adam(int64_t n, T* __restrict__ w, const T* __restrict__ g, T* __restrict__ m, T* __restrict__ v,
                       T lr, T b1, T b2, T eps, T bc1, T bc2, T clamp) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const T gi = g[i];
    const T mi = b1 * m[i] + (T(1) - b1) * gi;
    const T vi = b2 * v[i] + (T(1) - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    T wi = w[i] - lr * (mi / bc1) / (sqrt(vi / bc2) + eps);
    if (clamp > T(0)) wi = wi > clamp ? clamp : (wi < -clamp ? -clamp : wi);
    w[i] = wi;
  }
}

__global__ void k_features(int64_t ncell, const int32_t* __restrict__ nbr, const int32_t* __restrict__ self,
                           const double* __restrict__ mu, float* __restrict__ feat) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < 27 * ncell;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = e / 27;
    feat[e] = float(log10(mu[nbr[e]]) - log10(mu[self[c]]));
  }
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ __launch_bounds__(128) void k_mlp_forward(const float* __restrict__ w, const float* __restrict__ x,
                                                     int64_t n, float* __restrict__ y, float* __restrict__ cache) {
  __shared__ float sw[kParams];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) sw[i] = w[i];
  __syncthreads();
  const int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (s >= n) return;
  float xi[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) xi[i] = x[s * kIn + i];
  float h1[kH];
#pragma unroll
  for (int o = 0; o < kH; ++o) {
    float z = sw[kOffB1 + o];
#pragma unroll
    for (int i = 0; i < kIn; ++i) z += sw[o * kIn + i] * xi[i];
    cache[s * kCache + o] = z;
    h1[o] = gelu(z);
  }
  float h2[kH];
#pragma unroll
  for (int o = 0; o < kH; ++o) {
    float z = sw[kOffB2 + o];
#pragma unroll
    for (int j = 0; j < kH; ++j) z += sw[kOffW2 + o * kH + j] * h1[j];
    cache[s * kCache + kH + o] = z;
    h2[o] = gelu(z);
  }
#pragma unroll
  for (int c = 0; c < kOut; ++c) {
    float z = sw[kOffB3 + c];
#pragma unroll
    for (int j = 0; j < kH; ++j) z += sw[kOffW3 + c * kH + j] * h2[j];
    cache[s * kCache + 2 * kH + c] = z;
    y[s * kOut + c] = z > kClamp ? kClamp : (z < -kClamp ? -kClamp : z);
  }
}

// per sample: deltas and activations (work: D1 | D2 | H1 | H2 | D3[4])
__global__ __launch_bounds__(128) void k_mlp_deltas(const float* __restrict__ w, const float* __restrict__ cache,
                                                    const float* __restrict__ dy, int64_t n,
                                                    float* __restrict__ work) {
  __shared__ float sw[kParams];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) sw[i] = w[i];
  __syncthreads();
  const int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (s >= n) return;
  float* D1 = work;
  float* D2 = work + n * kH;
  float* H1 = work + 2 * n * kH;
  float* H2 = work + 3 * n * kH;
  float* D3 = work + 4 * n * kH;
  const float* cz = cache + s * kCache;
  float d3[kOut];
#pragma unroll
  for (int c = 0; c < kOut; ++c) {
    const float z = cz[2 * kH + c];
    d3[c] = (z > -kClamp && z < kClamp) ? dy[s * kOut + c] : 0.0f;
    D3[s * 4 + c] = d3[c];
  }
  D3[s * 4 + 3] = 0.0f;
  float d2[kH];
#pragma unroll
  for (int o = 0; o < kH; ++o) {
    const float z = cz[kH + o];
    float a = 0.0f;
#pragma unroll
    for (int c = 0; c < kOut; ++c) a += sw[kOffW3 + c * kH + o] * d3[c];
    d2[o] = a * gelu_d(z);
    D2[s * kH + o] = d2[o];
    H2[s * kH + o] = gelu(z);
  }
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    const float z = cz[j];
    float a = 0.0f;
#pragma unroll
    for (int o = 0; o < kH; ++o) a += sw[kOffW2 + o * kH + j] * d2[o];
    D1[s * kH + j] = a * gelu_d(z);
    H1[s * kH + j] = gelu(z);
  }
}

// partial sums over a chunk of samples of the weight gradients
// grid (nsplit, 3): layer 0: D1 x X -> W1, b1; layer 1: D2 x H1 -> W2, b2; layer 2: D3 x H2 -> W3, b3
__global__ __launch_bounds__(256) void k_mlp_wgrad_partial(const float* __restrict__ x, const float* __restrict__ work,
                                                           int64_t n, int chunk, float* __restrict__ part) {
  const int layer = blockIdx.y;
  const float* A;
  const float* B;
  int P, Q, lda, ldb, offW, offB;
  if (layer == 0) {
    A = work, lda = kH, P = kH, B = x, ldb = kIn, Q = kIn, offW = 0, offB = kOffB1;
  } else if (layer == 1) {
    A = work + n * kH, lda = kH, P = kH, B = work + 2 * n * kH, ldb = kH, Q = kH, offW = kOffW2, offB = kOffB2;
  } else {
    A = work + 4 * n * kH, lda = 4, P = kOut, B = work + 3 * n * kH, ldb = kH, Q = kH, offW = kOffW3, offB = kOffB3;
  }
  const int64_t s0 = int64_t(blockIdx.x) * chunk;
  const int64_t s1 = s0 + chunk < n ? s0 + chunk : n;
  float* out = part + int64_t(blockIdx.x) * kParams;
  for (int idx = threadIdx.x; idx < P * (Q + 1); idx += blockDim.x) {
    const int p = idx / (Q + 1), q = idx % (Q + 1);
    float acc = 0.0f;
    for (int64_t i = s0; i < s1; ++i) acc += A[i * lda + p] * (q < Q ? B[i * ldb + q] : 1.0f);
    out[q < Q ? offW + p * Q + q : offB + p] = acc;
  }
}

__global__ void k_sum_parts(int nsplit, const float* __restrict__ part, float* __restrict__ dw) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kParams; i += gridDim.x * blockDim.x) {
    float a = 0.0f;
    for (int k = 0; k < nsplit; ++k) a += part[int64_t(k) * kParams + i];
    dw[i] = a;
  }
}

__global__ __launch_bounds__(kBlock) void k_mse(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                                                float* __restrict__ dy, float scale, double* __restrict__ loss) {
  __shared__ double sm[kBlock / 64];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = scale * d;
    acc += double(d) * double(d);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) {
    double b = 0.0;
    for (int i = 0; i < int(blockDim.x >> 6); ++i) b += sm[i];
    atomicAdd(loss, b);
  }
}

__global__ void k_gather_rows(const float* __restrict__ src, int cols, const int64_t* __restrict__ idx, int64_t n,
                              float* __restrict__ dst) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n * cols; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / cols, j = e % cols;
    dst[e] = src[idx[i] * cols + j];
  }
}

__global__ void k_d2f(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = float(a[i]);
}
__global__ void k_f2d(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = double(a[i]);
}

}  // namespace

void launch_scaling_accum(const DevLevel& L, const double* y, double* acc, double* cnt, hipStream_t s) {
  k_scal_accum<<<grid_for(L.ncell), kBlock, 0, s>>>(L, y, acc, cnt);
}
void launch_scaling_finish(int64_t nn, const double* acc, const double* cnt, const double* minv, double* sdof,
                           double* md, float* mf, hipStream_t s) {
  k_scal_finish<<<grid_for(nn), kBlock, 0, s>>>(nn, acc, cnt, minv, sdof, md, mf);
}
void launch_scaling_grad(const DevLevel& L, const double* sbar, const double* sdof, const double* cnt, double* ybar,
                         hipStream_t s) {
  k_scal_grad<<<grid_for(L.ncell), kBlock, 0, s>>>(L, sbar, sdof, cnt, ybar);
}
void launch_chebrev_a(int64_t n, const double* xbar, const double* minv, const double* mp, const double* rk,
                      double* dbar, double* rbar, double* sbar, double beta, double sgn, hipStream_t s) {
  k_chebrev_a<<<grid_for(n), kBlock, 0, s>>>(n, xbar, minv, mp, rk, dbar, rbar, sbar, beta, sgn);
}
void launch_ritz_mass(int64_t n, const double* v, const double* minv, double* out, hipStream_t s) {
  k_ritz_mass<<<grid_for(n), kBlock, 0, s>>>(n, v, minv, out);
}
void launch_lambda_term(int64_t n, const double* v, const double* minv, const double* sdof, double coef, double* sbar,
                        hipStream_t s) {
  k_lambda_term<<<grid_for(n), kBlock, 0, s>>>(n, v, minv, sdof, coef, sbar);
}
void launch_chebrev_b(int64_t n, double* dbar, const double* t, double alpha, hipStream_t s) {
  k_chebrev_b<<<grid_for(n), kBlock, 0, s>>>(n, dbar, t, alpha);
}
template <typename T>
void launch_adam(int64_t n, T* w, const T* g, T* m, T* v, double lr, double b1, double b2, double eps, int64_t t,
                 double clamp, hipStream_t s) {
  const double bc1 = 1.0 - std::pow(b1, double(t)), bc2 = 1.0 - std::pow(b2, double(t));
  k_adam<T><<<grid_for(n), kBlock, 0, s>>>(n, w, g, m, v, T(lr), T(b1), T(b2), T(eps), T(bc1), T(bc2), T(clamp));
}
template void launch_adam<float>(int64_t, float*, const float*, float*, float*, double, double, double, double,
                                 int64_t, double, hipStream_t);
template void launch_adam<double>(int64_t, double*, const double*, double*, double*, double, double, double, double,
                                  int64_t, double, hipStream_t);
void launch_features(int64_t ncell, const int32_t* nbr, const int32_t* self, const double* mu, float* feat,
                     hipStream_t s) {
  k_features<<<grid_for(27 * ncell), kBlock, 0, s>>>(ncell, nbr, self, mu, feat);
}
void launch_mlp_forward(const float* w, const float* x, int64_t n, float* y, float* cache, hipStream_t s) {
  if (n <= 0) return;
  k_mlp_forward<<<unsigned((n + 127) / 128), 128, 0, s>>>(w, x, n, y, cache);
}
void launch_mlp_backward(const float* w, const float* x, const float* cache, const float* dy, int64_t n, float* dw,
                         float* work, float* part, hipStream_t s) {
  if (n <= 0) return;
  k_mlp_deltas<<<unsigned((n + 127) / 128), 128, 0, s>>>(w, cache, dy, n, work);
  const int chunk = 64;
  const int nsplit = int((n + chunk - 1) / chunk);
  k_mlp_wgrad_partial<<<dim3(unsigned(nsplit), 3), 256, 0, s>>>(x, work, n, chunk, part);
  k_sum_parts<<<grid_for(kParams), kBlock, 0, s>>>(nsplit, part, dw);
}
void launch_mse(int64_t n3, const float* y, const float* t, float* dy, float scale, double* loss, hipStream_t s) {
  k_mse<<<grid_for(n3, kBlock, 1024), kBlock, 0, s>>>(n3, y, t, dy, scale, loss);
}
void launch_gather_rows(const float* src, int cols, const int64_t* idx, int64_t n, float* dst, hipStream_t s) {
  k_gather_rows<<<grid_for(n * cols), kBlock, 0, s>>>(src, cols, idx, n, dst);
}
void launch_d2f(int64_t n, const double* a, float* b, hipStream_t s) { k_d2f<<<grid_for(n), kBlock, 0, s>>>(n, a, b); }
void launch_f2d(int64_t n, const float* a, double* b, hipStream_t s) { k_f2d<<<grid_for(n), kBlock, 0, s>>>(n, a, b); }

}  // namespace learned
}  // namespace mfgmg
