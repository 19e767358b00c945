// Per-cell Q2 strain-rate operator by sum factorisation (device code).
//
// Paper: A_ij = int 2 mu eps(phi_i) : eps(phi_j) (Sec. 2.1), evaluated
// matrix-free "at the quadrature level" (Sec. 2.2.1).  On an axis-aligned cube
// of side h with cell-constant mu the cell contribution is
//   y_(a,c) = sum_q sum_d F_cd(q) dphi_a/dxi_d(xi_q),
//   F(q) = 2 mu h w_q sym(grad_xi u(xi_q)),
// with 3x3x3 Gauss points (exact here).  Values are first interpolated to the
// Gauss points (collocation basis), differentiated there with the collocation
// derivative matrix, and the transposed steps run backwards; every index is a
// compile-time constant so the 81 inputs and 81 outputs live in registers.
#pragma once

#include <hip/hip_runtime.h>

namespace mfgmg {
namespace cellop {

// 1D Gauss points xi = 1/2 -+ g, 1/2 with g = sqrt(15)/10.
// Interpolation from the Q2 nodes {0, 1/2, 1} to the Gauss points:
//   N = [[0.3+g, 0.4, 0.3-g], [0, 1, 0], [0.3-g, 0.4, 0.3+g]].
// Collocation derivative on the Gauss points, scaled by g:
//   g*D = [[-1.5, 2, -0.5], [-0.5, 0, 0.5], [0.5, -2, 1.5]];
// the factor 1/g^2 of the two derivatives goes into the cell coefficient.
constexpr double kG = 0.38729833462074168852;
constexpr double kNa = 0.3 + kG;
constexpr double kNb = 0.3 - kG;
constexpr double kInvG2 = 1.0 / (kG * kG);   // = 20/3
constexpr double kW0 = 5.0 / 18.0;
constexpr double kW1 = 8.0 / 18.0;

template <typename T>
__device__ __forceinline__ void interp3(T& v0, T& v1, T& v2) {
  const T a = T(kNa), b = T(kNb), f = T(0.4);
  const T o0 = a * v0 + f * v1 + b * v2;
  const T o2 = b * v0 + f * v1 + a * v2;
  v0 = o0;
  v2 = o2;
}

template <typename T>
__device__ __forceinline__ void interp3_t(T& v0, T& v1, T& v2) {
  const T a = T(kNa), b = T(kNb), f = T(0.4);
  const T o0 = a * v0 + b * v2;
  const T o1 = v1 + f * (v0 + v2);
  const T o2 = b * v0 + a * v2;
  v0 = o0;
  v1 = o1;
  v2 = o2;
}

// derivative (scaled by g) at Gauss point q of the collocation values v0..v2
template <int q, typename T>
__device__ __forceinline__ T deriv(T v0, T v1, T v2) {
  if constexpr (q == 0) return T(-1.5) * v0 + T(2.0) * v1 - T(0.5) * v2;
  else if constexpr (q == 1) return T(0.5) * (v2 - v0);
  else return T(0.5) * v0 - T(2.0) * v1 + T(1.5) * v2;
}

// transposed derivative: add f * gD[q][p] to o_p
template <int q, typename T>
__device__ __forceinline__ void deriv_t(T f, T& o0, T& o1, T& o2) {
  if constexpr (q == 0) {
    o0 += T(-1.5) * f;
    o1 += T(2.0) * f;
    o2 += T(-0.5) * f;
  } else if constexpr (q == 1) {
    const T h = T(0.5) * f;
    o0 -= h;
    o2 += h;
  } else {
    o0 += T(0.5) * f;
    o1 += T(-2.0) * f;
    o2 += T(1.5) * f;
  }
}

// Apply (N x N x N) (forward) or its transpose to a 27-value tensor, x fastest.
template <typename T>
__device__ __forceinline__ void interp_all(T* v) {
#pragma unroll
  for (int l = 0; l < 9; ++l) interp3(v[3 * l], v[3 * l + 1], v[3 * l + 2]);            // x lines
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int x = 0; x < 3; ++x) interp3(v[x + 9 * z], v[x + 3 + 9 * z], v[x + 6 + 9 * z]);  // y lines
#pragma unroll
  for (int l = 0; l < 9; ++l) interp3(v[l], v[l + 9], v[l + 18]);                      // z lines
}

template <typename T>
__device__ __forceinline__ void interp_all_t(T* v) {
#pragma unroll
  for (int l = 0; l < 9; ++l) interp3_t(v[l], v[l + 9], v[l + 18]);
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int x = 0; x < 3; ++x) interp3_t(v[x + 9 * z], v[x + 3 + 9 * z], v[x + 6 + 9 * z]);
#pragma unroll
  for (int l = 0; l < 9; ++l) interp3_t(v[3 * l], v[3 * l + 1], v[3 * l + 2]);
}

template <int qx, int qy, int qz, typename T>
__device__ __forceinline__ void quad_point(const T (&W)[3][27], T (&Y)[3][27], T coef) {
  constexpr double wx = qx == 1 ? kW1 : kW0;
  constexpr double wy = qy == 1 ? kW1 : kW0;
  constexpr double wz = qz == 1 ? kW1 : kW0;
  constexpr int q = qx + 3 * qy + 9 * qz;
  T gx[3], gy[3], gz[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gx[c] = deriv<qx>(W[c][q - qx], W[c][q - qx + 1], W[c][q - qx + 2]);
    gy[c] = deriv<qy>(W[c][q - 3 * qy], W[c][q - 3 * qy + 3], W[c][q - 3 * qy + 6]);
    gz[c] = deriv<qz>(W[c][q - 9 * qz], W[c][q - 9 * qz + 9], W[c][q - 9 * qz + 18]);
  }
  const T cq = coef * T(wx * wy * wz);
  const T c2 = cq + cq;
  // F = 2 mu h w_q sym(grad u) (with the derivative scaling folded into coef)
  const T f00 = c2 * gx[0], f11 = c2 * gy[1], f22 = c2 * gz[2];
  const T f01 = cq * (gy[0] + gx[1]);
  const T f02 = cq * (gz[0] + gx[2]);
  const T f12 = cq * (gz[1] + gy[2]);
  // row c of F is contracted with the derivative in direction d
  deriv_t<qx>(f00, Y[0][q - qx], Y[0][q - qx + 1], Y[0][q - qx + 2]);
  deriv_t<qy>(f01, Y[0][q - 3 * qy], Y[0][q - 3 * qy + 3], Y[0][q - 3 * qy + 6]);
  deriv_t<qz>(f02, Y[0][q - 9 * qz], Y[0][q - 9 * qz + 9], Y[0][q - 9 * qz + 18]);
  deriv_t<qx>(f01, Y[1][q - qx], Y[1][q - qx + 1], Y[1][q - qx + 2]);
  deriv_t<qy>(f11, Y[1][q - 3 * qy], Y[1][q - 3 * qy + 3], Y[1][q - 3 * qy + 6]);
  deriv_t<qz>(f12, Y[1][q - 9 * qz], Y[1][q - 9 * qz + 9], Y[1][q - 9 * qz + 18]);
  deriv_t<qx>(f02, Y[2][q - qx], Y[2][q - qx + 1], Y[2][q - qx + 2]);
  deriv_t<qy>(f12, Y[2][q - 3 * qy], Y[2][q - 3 * qy + 3], Y[2][q - 3 * qy + 6]);
  deriv_t<qz>(f22, Y[2][q - 9 * qz], Y[2][q - 9 * qz + 9], Y[2][q - 9 * qz + 18]);
}

// derivative (scaled by g) along direction D at Gauss point (qx, qy, qz) of the
// collocation values v [27]
template <int D, int qx, int qy, int qz, typename T>
__device__ __forceinline__ T line_deriv(const T* v) {
  constexpr int q = qx + 3 * qy + 9 * qz;
  if constexpr (D == 0) return deriv<qx>(v[q - qx], v[q - qx + 1], v[q - qx + 2]);
  else if constexpr (D == 1) return deriv<qy>(v[q - 3 * qy], v[q - 3 * qy + 3], v[q - 3 * qy + 6]);
  else return deriv<qz>(v[q - 9 * qz], v[q - 9 * qz + 9], v[q - 9 * qz + 18]);
}

// One Gauss point's contribution to output component C only: row C of F,
// F_Cd = cq (d_d u_C + d_C u_d) (2 cq d_C u_C on the diagonal), contracted
// with the derivative in direction d: the operations of row C of quad_point,
// in the same order (so the results agree bit for bit).
template <int C, int qx, int qy, int qz, typename T>
__device__ __forceinline__ void quad_point_row(const T (&W)[3][27], T (&Y)[27], T coef) {
  constexpr double wx = qx == 1 ? kW1 : kW0;
  constexpr double wy = qy == 1 ? kW1 : kW0;
  constexpr double wz = qz == 1 ? kW1 : kW0;
  constexpr int q = qx + 3 * qy + 9 * qz;
  const T cq = coef * T(wx * wy * wz);
  T f[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T gcd;   // d_d u_C
    if (d == 0) gcd = line_deriv<0, qx, qy, qz>(W[C]);
    else if (d == 1) gcd = line_deriv<1, qx, qy, qz>(W[C]);
    else gcd = line_deriv<2, qx, qy, qz>(W[C]);
    if (d == C) {
      f[d] = (cq + cq) * gcd;
    } else {
      const T gdc = line_deriv<C, qx, qy, qz>(W[d]);   // d_C u_d
      f[d] = cq * (gcd + gdc);
    }
  }
  deriv_t<qx>(f[0], Y[q - qx], Y[q - qx + 1], Y[q - qx + 2]);
  deriv_t<qy>(f[1], Y[q - 3 * qy], Y[q - 3 * qy + 3], Y[q - 3 * qy + 6]);
  deriv_t<qz>(f[2], Y[q - 9 * qz], Y[q - 9 * qz + 9], Y[q - 9 * qz + 18]);
}

// Output component C of the cell operator from the Gauss-point values W
// (interp_all already applied to every component); Y: collocation-basis
// result (interp_all_t still to be applied).  coef = mu * h.
template <int C, typename T>
__device__ __forceinline__ void apply_cell_row(const T (&W)[3][27], T (&Y)[27], T mu_h) {
#pragma unroll
  for (int a = 0; a < 27; ++a) Y[a] = T(0);
  const T coef = mu_h * T(kInvG2);
#define MFGMG_QPR(x, y, z) quad_point_row<C, x, y, z>(W, Y, coef);
  MFGMG_QPR(0, 0, 0) MFGMG_QPR(1, 0, 0) MFGMG_QPR(2, 0, 0)
  MFGMG_QPR(0, 1, 0) MFGMG_QPR(1, 1, 0) MFGMG_QPR(2, 1, 0)
  MFGMG_QPR(0, 2, 0) MFGMG_QPR(1, 2, 0) MFGMG_QPR(2, 2, 0)
  MFGMG_QPR(0, 0, 1) MFGMG_QPR(1, 0, 1) MFGMG_QPR(2, 0, 1)
  MFGMG_QPR(0, 1, 1) MFGMG_QPR(1, 1, 1) MFGMG_QPR(2, 1, 1)
  MFGMG_QPR(0, 2, 1) MFGMG_QPR(1, 2, 1) MFGMG_QPR(2, 2, 1)
  MFGMG_QPR(0, 0, 2) MFGMG_QPR(1, 0, 2) MFGMG_QPR(2, 0, 2)
  MFGMG_QPR(0, 1, 2) MFGMG_QPR(1, 1, 2) MFGMG_QPR(2, 1, 2)
  MFGMG_QPR(0, 2, 2) MFGMG_QPR(1, 2, 2) MFGMG_QPR(2, 2, 2)
#undef MFGMG_QPR
}

// transposed derivative along direction D at Gauss point (qx, qy, qz): adds
// f * gD[q_D][p] to the collocation values y of the line through the point
template <int D, int qx, int qy, int qz, typename T>
__device__ __forceinline__ void line_deriv_t(T f, T* y) {
  constexpr int q = qx + 3 * qy + 9 * qz;
  if constexpr (D == 0) deriv_t<qx>(f, y[q - qx], y[q - qx + 1], y[q - qx + 2]);
  else if constexpr (D == 1) deriv_t<qy>(f, y[q - 3 * qy], y[q - 3 * qy + 3], y[q - 3 * qy + 6]);
  else deriv_t<qz>(f, y[q - 9 * qz], y[q - 9 * qz + 9], y[q - 9 * qz + 18]);
}

// The terms of one Gauss point that involve input component D only.  With
// g_e = d_e u_D, u_D enters F_DD as 2 cq g_D and F_De = F_eD (e != D) as
// cq g_e; row D of F is contracted with the derivative in every direction,
// row e != D only in direction D.  Summed over D these are the terms of
// quad_point, added in another order.
template <int D, int qx, int qy, int qz, typename T>
__device__ __forceinline__ void quad_point_input(const T (&V)[27], T (&Y)[3][27]) {
  constexpr double w = (qx == 1 ? kW1 : kW0) * (qy == 1 ? kW1 : kW0) * (qz == 1 ? kW1 : kW0);
  const T g0 = line_deriv<0, qx, qy, qz>(V);
  const T g1 = line_deriv<1, qx, qy, qz>(V);
  const T g2 = line_deriv<2, qx, qy, qz>(V);
  const T f0 = T(D == 0 ? 2.0 * w : w) * g0;
  const T f1 = T(D == 1 ? 2.0 * w : w) * g1;
  const T f2 = T(D == 2 ? 2.0 * w : w) * g2;
  line_deriv_t<0, qx, qy, qz>(f0, Y[D]);
  line_deriv_t<1, qx, qy, qz>(f1, Y[D]);
  line_deriv_t<2, qx, qy, qz>(f2, Y[D]);
  if constexpr (D != 0) line_deriv_t<D, qx, qy, qz>(f0, Y[0]);
  if constexpr (D != 1) line_deriv_t<D, qx, qy, qz>(f1, Y[1]);
  if constexpr (D != 2) line_deriv_t<D, qx, qy, qz>(f2, Y[2]);
}

template <typename T, int N>
__device__ __forceinline__ void pin_all(T (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]));
}
template <typename T, int N, int M>
__device__ __forceinline__ void pin_all(T (&v)[N][M]) {
#pragma unroll
  for (int i = 0; i < N; ++i) pin_all(v[i]);
}

template <int D, typename T>
__device__ __forceinline__ void input_pass(const T (&V)[27], T (&Y)[3][27]) {
#define MFGMG_QPI(x, y, z) quad_point_input<D, x, y, z>(V, Y);
  MFGMG_QPI(0, 0, 0) MFGMG_QPI(1, 0, 0) MFGMG_QPI(2, 0, 0)
  MFGMG_QPI(0, 1, 0) MFGMG_QPI(1, 1, 0) MFGMG_QPI(2, 1, 0)
  MFGMG_QPI(0, 2, 0) MFGMG_QPI(1, 2, 0) MFGMG_QPI(2, 2, 0)
  MFGMG_QPI(0, 0, 1) MFGMG_QPI(1, 0, 1) MFGMG_QPI(2, 0, 1)
  MFGMG_QPI(0, 1, 1) MFGMG_QPI(1, 1, 1) MFGMG_QPI(2, 1, 1)
  MFGMG_QPI(0, 2, 1) MFGMG_QPI(1, 2, 1) MFGMG_QPI(2, 2, 1)
  MFGMG_QPI(0, 0, 2) MFGMG_QPI(1, 0, 2) MFGMG_QPI(2, 0, 2)
  MFGMG_QPI(0, 1, 2) MFGMG_QPI(1, 1, 2) MFGMG_QPI(2, 1, 2)
  MFGMG_QPI(0, 2, 2) MFGMG_QPI(1, 2, 2) MFGMG_QPI(2, 2, 2)
#undef MFGMG_QPI
}

// The cell operator one input component at a time: get(D, V) fetches the 27
// nodal values of component D, which are interpolated and whose terms are
// added into all three result components before the next component is
// fetched, so only 27 inputs live beside the 81 results.  Y: the cell's
// output contributions y_(a,c) on return.  coef = mu * h.
template <typename T, typename Get>
__device__ __forceinline__ void apply_cell_by_input(const Get& get, T (&Y)[3][27], T mu_h) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 27; ++a) Y[c][a] = T(0);
  const T coef = mu_h * T(kInvG2);
  {
    T V[27];
    get(0, V);
    interp_all(V);
#pragma unroll
    for (int a = 0; a < 27; ++a) V[a] *= coef;
    pin_all(V);
    input_pass<0>(V, Y);
  }
  asm volatile("" ::: "memory");   // the next component's loads stay below
  {
    T V[27];
    pin_all(Y);
    get(1, V);
    interp_all(V);
#pragma unroll
    for (int a = 0; a < 27; ++a) V[a] *= coef;
    pin_all(V);
    input_pass<1>(V, Y);
  }
  asm volatile("" ::: "memory");
  {
    T V[27];
    pin_all(Y);
    get(2, V);
    interp_all(V);
#pragma unroll
    for (int a = 0; a < 27; ++a) V[a] *= coef;
    pin_all(V);
    input_pass<2>(V, Y);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) interp_all_t(Y[c]);
}

// U[c][a]: nodal values of component c at local node a (x fastest) on input,
// the cell's output contributions y_(a,c) on return.  coef = mu * h.
template <typename T>
__device__ __forceinline__ void apply_cell(T (&U)[3][27], T mu_h) {
  T Y[3][27];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    interp_all(U[c]);
#pragma unroll
    for (int a = 0; a < 27; ++a) Y[c][a] = T(0);
  }
  const T coef = mu_h * T(kInvG2);
#define MFGMG_QP(x, y, z) quad_point<x, y, z>(U, Y, coef);
  MFGMG_QP(0, 0, 0) MFGMG_QP(1, 0, 0) MFGMG_QP(2, 0, 0)
  MFGMG_QP(0, 1, 0) MFGMG_QP(1, 1, 0) MFGMG_QP(2, 1, 0)
  MFGMG_QP(0, 2, 0) MFGMG_QP(1, 2, 0) MFGMG_QP(2, 2, 0)
  MFGMG_QP(0, 0, 1) MFGMG_QP(1, 0, 1) MFGMG_QP(2, 0, 1)
  MFGMG_QP(0, 1, 1) MFGMG_QP(1, 1, 1) MFGMG_QP(2, 1, 1)
  MFGMG_QP(0, 2, 1) MFGMG_QP(1, 2, 1) MFGMG_QP(2, 2, 1)
  MFGMG_QP(0, 0, 2) MFGMG_QP(1, 0, 2) MFGMG_QP(2, 0, 2)
  MFGMG_QP(0, 1, 2) MFGMG_QP(1, 1, 2) MFGMG_QP(2, 1, 2)
  MFGMG_QP(0, 2, 2) MFGMG_QP(1, 2, 2) MFGMG_QP(2, 2, 2)
#undef MFGMG_QP
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    interp_all_t(Y[c]);
#pragma unroll
    for (int a = 0; a < 27; ++a) U[c][a] = Y[c][a];
  }
}

}  // namespace cellop
}  // namespace mfgmg
