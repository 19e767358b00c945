// Device kernels of the Q3-Q2 pair (k = 2 of Sec. 2.1) on uniform lattice
// levels (see q3.h for the numbering).
//
// One wavefront per cell: lane l = x + 4 y + 16 z stands for the tensor
// point (x, y, z) of the cell's 4 x 4 x 4 nodes and, after interpolation, of
// its 4 x 4 x 4 Gauss points.  A one-dimensional 4 x 4 contraction along an
// axis is four reads of other lanes and four multiply-adds per lane, so the
// sum-factorised operator keeps one value per lane and component:
//   interpolate u to the Gauss points (3 axes x 3 components),
//   differentiate there with the Gauss-collocation derivative (9 sweeps),
//   F_cd = mu h w_q (d_d u_c + d_c u_d),
//   y_c = N^T N^T N^T sum_d D_d^T F_cd (9 + 9 transposed sweeps).
// In the operator the x and y contractions read the other lanes through DPP
// (quad broadcast along x, row rotation by 4, 8, 12 lanes along y: VALU
// operand modifiers, no LDS traffic) and the z contraction, across rows,
// through __shfl (ds_bpermute); the other kernels use __shfl throughout.
// The operator's results are summed over a 2 x 2 x 2 block of cells (one
// workgroup, a wavefront per cell): each wavefront stores its 3 x 64 results
// in its own LDS slot, and each thread of the write-back sums the (up to 8)
// slot entries of one block lattice point and component.  Owner computes, as
// in the Q2 brick kernel: a lattice point belongs to the block whose
// half-open box [6b, 6b + 6) holds it (the last block along an axis also owns
// the closing plane); the block writes the points it owns (y = its sum, or
// y = x on constrained points: identity rows; accumulating, y += its sum on
// free points) and stores the sums of the 127 points of its high faces, owned
// by upper neighbours, in its halo slot; a second kernel adds, for every
// point on a block's low face, the neighbours' slot values.  No atomics and
// no separate initialisation of y.  Constrained (boundary) nodes are read as
// zero.
#include <hip/hip_runtime.h>

#include "ops.h"

namespace mfgmg {

namespace {

__constant__ double c_q3N[16];    // N[q][a] = L_a(xg_q)
__constant__ double c_q3D[16];    // D[q][r] = l_r'(xg_q)
__constant__ double c_q3W[4];     // Gauss weights on [0, 1]
__constant__ double c_q3P[12];    // P2[q][i]: Q2 pressure basis at the Gauss points
__constant__ double c_q3M2[9];    // 1D Q2 mass

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block = kBlock, int64_t cap = 1 << 20) {
  int64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return unsigned(g);
}

// out(.., q, ..) = sum_a c[a] v(.., a, ..) along axis AX, c the lane's row
template <int AX, typename T>
__device__ __forceinline__ T sweep(T v, int lane, const T (&c)[4]) {
  constexpr int S = 1 << (2 * AX);
  const int base = lane - ((lane >> (2 * AX)) & 3) * S;
  T out = c[0] * __shfl(v, base);
  out += c[1] * __shfl(v, base + S);
  out += c[2] * __shfl(v, base + 2 * S);
  out += c[3] * __shfl(v, base + 3 * S);
  return out;
}

// the lane's row of a 4 x 4 matrix along axis AX (row = lane coordinate), and
// its column (transposed sweep)
template <int AX, typename T>
__device__ __forceinline__ void row_of(const double* M, int lane, T (&c)[4]) {
  const int q = (lane >> (2 * AX)) & 3;
#pragma unroll
  for (int a = 0; a < 4; ++a) c[a] = T(M[4 * q + a]);
}
template <int AX, typename T>
__device__ __forceinline__ void col_of(const double* M, int lane, T (&c)[4]) {
  const int a = (lane >> (2 * AX)) & 3;
#pragma unroll
  for (int q = 0; q < 4; ++q) c[q] = T(M[4 * q + a]);
}

// DPP move of a 32-bit value (CTRL: quad_perm / row_ror encodings of GFX9)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i<CTRL>(int(b & 0xffffffffLL)), hi = dpp_i<CTRL>(int(b >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
constexpr int kQuadBcast[4] = {0x00, 0x55, 0xAA, 0xFF};   // quad_perm: every lane of a quad reads lane a
constexpr int kRowRor[4] = {0, 0x124, 0x128, 0x12C};      // row_ror by 0, 4, 8, 12 lanes

// x contraction: c[a] the lane's coefficient of quad lane a (row_of / col_of)
template <typename T>
__device__ __forceinline__ T sweep_x(T v, const T (&c)[4]) {
  return c[0] * dpp<kQuadBcast[0]>(v) + c[1] * dpp<kQuadBcast[1]>(v) + c[2] * dpp<kQuadBcast[2]>(v) +
         c[3] * dpp<kQuadBcast[3]>(v);
}
// y contraction: r[k] the lane's coefficient of the value that the rotation by
// 4k lanes brings (the coefficient of that value's y coordinate)
template <typename T>
__device__ __forceinline__ T sweep_y(T v, const T (&r)[4]) {
  return r[0] * v + r[1] * dpp<kRowRor[1]>(v) + r[2] * dpp<kRowRor[2]>(v) + r[3] * dpp<kRowRor[3]>(v);
}
// y coordinate (lane bits 2-3) of the lane each rotation reads
__device__ __forceinline__ void rot_sources(int lane, int (&src)[4]) {
  const int yv = (lane >> 2) & 3;
  src[0] = yv;
  src[1] = dpp_i<kRowRor[1]>(yv);
  src[2] = dpp_i<kRowRor[2]>(yv);
  src[3] = dpp_i<kRowRor[3]>(yv);
}
// coefficients of a y contraction in rotation order: row (out(q) = sum_a M[q][a] v(a))
// or column (out(a) = sum_q M[q][a] v(q)) of M for the lane's y coordinate
template <typename T>
__device__ __forceinline__ void rot_row(const double* M, int lane, const int (&src)[4], T (&r)[4]) {
  const int q = (lane >> 2) & 3;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = T(M[4 * q + src[k]]);
}
template <typename T>
__device__ __forceinline__ void rot_col(const double* M, int lane, const int (&src)[4], T (&r)[4]) {
  const int a = (lane >> 2) & 3;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = T(M[4 * src[k] + a]);
}

struct Q3Cell {
  int64_t node;
  bool bnd;
  __device__ Q3Cell(int64_t n, int64_t c, int lane) {
    const int64_t m = 3 * n + 1;
    const int64_t i = c % n, j = (c / n) % n, k = c / (n * n);
    const int64_t X = 3 * i + (lane & 3), Y = 3 * j + ((lane >> 2) & 3), Z = 3 * k + (lane >> 4);
    node = X + m * (Y + m * Z);
    bnd = X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1;
  }
};

constexpr int kQ3B = 2;                         // cells per block edge
constexpr int kQ3E = 3 * kQ3B + 1;              // lattice points per block edge
constexpr int kQ3P = kQ3E * kQ3E * kQ3E;        // lattice points per block
constexpr int kQ3H = kQ3P - (kQ3E - 1) * (kQ3E - 1) * (kQ3E - 1);   // high-face points per block (127)

// index of a high-face point of the block lattice in the block's halo slot
// (p_x = 6: the 7 x 7 plane; else p_y = 6: 6 x 7; else p_z = 6: 6 x 6)
__device__ __forceinline__ int q3_halo_index(int px, int py, int pz) {
  constexpr int L = kQ3E - 1;
  if (px == L) return py + kQ3E * pz;
  if (py == L) return kQ3E * kQ3E + px + L * pz;
  return kQ3E * kQ3E + L * kQ3E + px + L * py;
}

template <typename T, bool ACC>
__global__ __launch_bounds__(64 * kQ3B * kQ3B * kQ3B) void k_vmult_q3(int64_t n, const T* __restrict__ mu,
                                                                     const T* __restrict__ x, T* __restrict__ y,
                                                                     T* __restrict__ halo) {
  constexpr int NW = kQ3B * kQ3B * kQ3B;
  __shared__ T slot[NW][3][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nb = n / kQ3B;
  const int64_t bx = blockIdx.x % nb, by = (blockIdx.x / nb) % nb, bz = blockIdx.x / (nb * nb);
  const int cx = w % kQ3B, cy = (w / kQ3B) % kQ3B, cz = w / (kQ3B * kQ3B);
  const int64_t c = (bx * kQ3B + cx) + n * ((by * kQ3B + cy) + n * (bz * kQ3B + cz));
  const Q3Cell qc(n, c, lane);
  T u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = qc.bnd ? T(0) : x[3 * qc.node + k];
  int src[4];
  rot_sources(lane, src);
  T Nx[4], Ny[4], Nz[4];
  row_of<0>(c_q3N, lane, Nx), rot_row(c_q3N, lane, src, Ny), row_of<2>(c_q3N, lane, Nz);
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = sweep<2>(sweep_y(sweep_x(u[k], Nx), Ny), lane, Nz);
  T Dx[4], Dy[4], Dz[4];
  row_of<0>(c_q3D, lane, Dx), rot_row(c_q3D, lane, src, Dy), row_of<2>(c_q3D, lane, Dz);
  T g[3][3];   // g[c][d] = d_d u_c at the lane's Gauss point
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g[k][0] = sweep_x(u[k], Dx);
    g[k][1] = sweep_y(u[k], Dy);
    g[k][2] = sweep<2>(u[k], lane, Dz);
  }
  const T wq = T(c_q3W[lane & 3] * c_q3W[(lane >> 2) & 3] * c_q3W[lane >> 4]);
  const T coef = mu[c] / T(n) * wq;
  T F[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) F[a][b] = coef * (g[a][b] + g[b][a]);
  col_of<0>(c_q3D, lane, Dx), rot_col(c_q3D, lane, src, Dy), col_of<2>(c_q3D, lane, Dz);
  col_of<0>(c_q3N, lane, Nx), rot_col(c_q3N, lane, src, Ny), col_of<2>(c_q3N, lane, Nz);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    // every lane takes part in the cross-lane reads; boundary lanes drop the result after
    const T t = sweep_x(F[k][0], Dx) + sweep_y(F[k][1], Dy) + sweep<2>(F[k][2], lane, Dz);
    const T o = sweep<2>(sweep_y(sweep_x(t, Nx), Ny), lane, Nz);
    slot[w][k][lane] = qc.bnd ? T(0) : o;
  }
  __syncthreads();
  // write-back: point p of the block lattice gathers, per axis, the cells
  // (0 or 1) whose local coordinate p - 3 cell lies in 0..3
  const int64_t m = 3 * n + 1;
  for (int e = threadIdx.x; e < 3 * kQ3P; e += blockDim.x) {
    const int p = e / 3, k = e - 3 * p;
    const int px = p % kQ3E, py = (p / kQ3E) % kQ3E, pz = p / (kQ3E * kQ3E);
    const int64_t X = 3 * kQ3B * bx + px, Y = 3 * kQ3B * by + py, Z = 3 * kQ3B * bz + pz;
    const bool own = (px < kQ3E - 1 || bx == nb - 1) && (py < kQ3E - 1 || by == nb - 1) &&
                     (pz < kQ3E - 1 || bz == nb - 1);
    const int64_t d = 3 * (X + m * (Y + m * Z)) + k;
    if (X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1) {
      if (!ACC && own) y[d] = x[d];   // identity row (every constrained point has one owner)
      continue;
    }
    T v = T(0);
    for (int ccz = 0; ccz < kQ3B; ++ccz) {
      const int lz = pz - 3 * ccz;
      if (lz < 0 || lz > 3) continue;
      for (int ccy = 0; ccy < kQ3B; ++ccy) {
        const int ly = py - 3 * ccy;
        if (ly < 0 || ly > 3) continue;
        for (int ccx = 0; ccx < kQ3B; ++ccx) {
          const int lx = px - 3 * ccx;
          if (lx < 0 || lx > 3) continue;
          v += slot[ccx + kQ3B * (ccy + kQ3B * ccz)][k][lx + 4 * ly + 16 * lz];
        }
      }
    }
    if (own) y[d] = ACC ? y[d] + v : v;
    else halo[(int64_t(blockIdx.x) * kQ3H + q3_halo_index(px, py, pz)) * 3 + k] = v;
  }
}

// Adds the halo values of its lower neighbour blocks into every free lattice
// point that lies on a block's low face (one thread per point, 3 components).
template <typename T>
__global__ __launch_bounds__(256) void k_q3_halo_add(int64_t n, const T* __restrict__ halo, T* __restrict__ y) {
  const int64_t nb = n / kQ3B, m = 3 * n + 1, L = 3 * kQ3B;
  // points with a coordinate on an inner block plane (a multiple of 6 in 6 .. m - 7)
  const int64_t node = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (node >= m * m * m) return;
  const int64_t X = node % m, Y = (node / m) % m, Z = node / (m * m);
  if (X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1) return;
  const bool fx = X % L == 0, fy = Y % L == 0, fz = Z % L == 0;
  if (!fx && !fy && !fz) return;
  const int64_t ox = X / L < nb ? X / L : nb - 1, oy = Y / L < nb ? Y / L : nb - 1, oz = Z / L < nb ? Z / L : nb - 1;
  const int px = int(X - L * ox), py = int(Y - L * oy), pz = int(Z - L * oz);
  T a0 = T(0), a1 = T(0), a2 = T(0);
  for (int sv = 1; sv < 8; ++sv) {
    const int sx = sv & 1, sy = (sv >> 1) & 1, sz = sv >> 2;
    if ((sx && !fx) || (sy && !fy) || (sz && !fz)) continue;
    const int64_t nbk = (ox - sx) + nb * ((oy - sy) + nb * (oz - sz));
    const T* h = halo + (nbk * kQ3H + q3_halo_index(px + int(L) * sx, py + int(L) * sy, pz + int(L) * sz)) * 3;
    a0 += h[0], a1 += h[1], a2 += h[2];
  }
  T* yp = y + 3 * node;
  yp[0] += a0, yp[1] += a1, yp[2] += a2;
}

// ---------------------------------------------------------- transfers
// Between two Q3 lattice levels the prolongation is the tensor product of one
// 1D matrix P1 [m_f x m_c] (coarse Q3 functions at the fine lattice points,
// at most 4 entries per row), with the boundary nodes of both levels masked:
// P = D_f (P1 x P1 x P1) D_c, R = P^T.  Each runs as three one-axis passes
// (one thread per output node, 3 components) through two scratch vectors.
// dims: the output's extent along x, y, z; the input has `nin` points along
// axis AX and the output's extents elsewhere.
template <int AX>
__device__ __forceinline__ void pass_coords(int64_t e, int64_t d0, int64_t d1, int64_t (&i)[3]) {
  i[0] = e % d0;
  i[1] = (e / d0) % d1;
  i[2] = e / (d0 * d1);
}
template <int AX>
__device__ __forceinline__ int64_t pass_index(const int64_t (&i)[3], int64_t a, int64_t d0, int64_t d1, int64_t nin) {
  // node index in the input array (extent nin along AX) with coordinate a along AX
  const int64_t e0 = AX == 0 ? nin : d0, e1 = AX == 1 ? nin : d1;
  const int64_t c0 = AX == 0 ? a : i[0], c1 = AX == 1 ? a : i[1], c2 = AX == 2 ? a : i[2];
  return c0 + e0 * (c1 + e1 * c2);
}

// prolongation pass: out(.., X, ..) = sum_j w[4X + j] in(.., c0[X] + j, ..).
// FIRST: the input is the coarse vector, read as 0 on coarse boundary nodes;
// LAST: the output is the fine vector, 0 (or untouched when adding) on fine
// boundary nodes
template <typename T, int AX, bool FIRST, bool LAST>
__global__ __launch_bounds__(256) void k_q3_prolong_pass(int64_t d0, int64_t d1, int64_t d2, int64_t nin,
                                                         const int32_t* __restrict__ c0, const double* __restrict__ w,
                                                         const T* __restrict__ in, T* __restrict__ out, bool add) {
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= d0 * d1 * d2) return;
  int64_t i[3];
  pass_coords<AX>(e, d0, d1, i);
  if (LAST) {
    const int64_t mf = d0;
    const bool bnd = i[0] == 0 || i[1] == 0 || i[2] == 0 || i[0] == mf - 1 || i[1] == mf - 1 || i[2] == mf - 1;
    if (bnd) {
      if (!add) out[3 * e] = out[3 * e + 1] = out[3 * e + 2] = T(0);
      return;
    }
  }
  const int64_t X = i[AX];
  T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t a = c0[X] + j;
    const T wj = T(w[4 * X + j]);
    if (FIRST) {   // coarse boundary: the other two coordinates are coarse as well here
      const int64_t o1 = AX == 0 ? i[1] : i[0], o2 = AX == 2 ? i[1] : i[2];
      if (a == 0 || a == nin - 1 || o1 == 0 || o1 == nin - 1 || o2 == 0 || o2 == nin - 1) continue;
    }
    const T* v = in + 3 * pass_index<AX>(i, a, d0, d1, nin);
    a0 += wj * v[0], a1 += wj * v[1], a2 += wj * v[2];
  }
  T* o = out + 3 * e;
  if (LAST && add) {
    o[0] += a0, o[1] += a1, o[2] += a2;
  } else {
    o[0] = a0, o[1] = a1, o[2] = a2;
  }
}

// restriction pass: out(.., C, ..) = sum over the fine points X of column C of
// P1 (CSR rptr/rcol/rw) of w in(.., X, ..).  FIRST: in = b - t (t may be
// null), read as 0 on fine boundary nodes; LAST: 0 on coarse boundary nodes
template <typename T, int AX, bool FIRST, bool LAST>
__global__ __launch_bounds__(256) void k_q3_restrict_pass(int64_t d0, int64_t d1, int64_t d2, int64_t nin,
                                                          const int32_t* __restrict__ rptr,
                                                          const int32_t* __restrict__ rcol,
                                                          const double* __restrict__ rw, const T* __restrict__ in,
                                                          const T* __restrict__ t, T* __restrict__ out) {
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= d0 * d1 * d2) return;
  int64_t i[3];
  pass_coords<AX>(e, d0, d1, i);
  T* o = out + 3 * e;
  if (LAST) {
    const int64_t mc = d0;
    if (i[0] == 0 || i[1] == 0 || i[2] == 0 || i[0] == mc - 1 || i[1] == mc - 1 || i[2] == mc - 1) {
      o[0] = o[1] = o[2] = T(0);
      return;
    }
  }
  const int64_t C = i[AX];
  T a0 = T(0), a1 = T(0), a2 = T(0);
  for (int32_t q = rptr[C]; q < rptr[C + 1]; ++q) {
    const int64_t a = rcol[q];
    if (FIRST) {   // fine boundary: the other two coordinates are fine as well here
      const int64_t o1 = AX == 0 ? i[1] : i[0], o2 = AX == 2 ? i[1] : i[2];
      if (a == 0 || a == nin - 1 || o1 == 0 || o1 == nin - 1 || o2 == 0 || o2 == nin - 1) continue;
    }
    const int64_t idx = 3 * pass_index<AX>(i, a, d0, d1, nin);
    const T wq = T(rw[q]);
    if (FIRST && t) {
      a0 += wq * (in[idx] - t[idx]), a1 += wq * (in[idx + 1] - t[idx + 1]), a2 += wq * (in[idx + 2] - t[idx + 2]);
    } else {
      a0 += wq * in[idx], a1 += wq * in[idx + 1], a2 += wq * in[idx + 2];
    }
  }
  o[0] = a0, o[1] = a1, o[2] = a2;
}

// diagonal: d[3 node + c] += mu h K_hat[(a, c), (a, c)] over the cells (one thread per cell)
__global__ __launch_bounds__(kBlock) void k_diag_q3(int64_t n, const double* __restrict__ mu,
                                                    const double* __restrict__ kdiag, double* __restrict__ d) {
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= n * n * n) return;
  const double s = mu[c] / double(n);
  for (int a = 0; a < 64; ++a) {
    const Q3Cell qc(n, c, a);
    if (qc.bnd) continue;
    for (int k = 0; k < 3; ++k) atomicAdd(&d[3 * qc.node + k], s * kdiag[3 * a + k]);
  }
}

// mu_K = sum w_q / sum (w_q / mu_q) over the 4^3 Gauss points
__global__ void k_harmonic64(int64_t ncell, const double* __restrict__ mq, double* __restrict__ mu) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < ncell; c += int64_t(gridDim.x) * blockDim.x) {
    double sw = 0.0, s = 0.0;
    for (int q = 0; q < 64; ++q) {
      const double w = c_q3W[q & 3] * c_q3W[(q >> 2) & 3] * c_q3W[q >> 4];
      sw += w;
      s += w / mq[64 * c + q];
    }
    mu[c] = sw / s;
  }
}

// b += D F, F_e[(a, c)] = h^3 sum_q w_q phi_a(xi_q) f_c(x_q); f [ncell][64][3]
__global__ __launch_bounds__(256) void k_rhs_q3(int64_t n, const double* __restrict__ f, double* __restrict__ b) {
  const int lane = threadIdx.x & 63;
  const int64_t cell = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const bool live = cell < n * n * n;
  const int64_t c = live ? cell : 0;
  const Q3Cell qc(n, c, lane);
  const double h = 1.0 / double(n);
  const double wq = c_q3W[lane & 3] * c_q3W[(lane >> 2) & 3] * c_q3W[lane >> 4] * h * h * h;
  double Nx[4], Ny[4], Nz[4];
  col_of<0>(c_q3N, lane, Nx), col_of<1>(c_q3N, lane, Ny), col_of<2>(c_q3N, lane, Nz);
  double out[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double v = wq * f[(64 * c + lane) * 3 + k];
    out[k] = sweep<2>(sweep<1>(sweep<0>(v, lane, Nx), lane, Ny), lane, Nz);
  }
  if (!live || qc.bnd) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) atomicAdd(&b[3 * qc.node + k], out[k]);
}

// ---------------------------------------------------------- Q2 pressure
// The pressure side of the pair on the leaf: B u (-int psi_i div u), B^T p
// and the mu^{-1}-weighted Q2 mass matrix, with psi on the (2n + 1)^3 lattice.
// Lanes hold Gauss points as above; a pressure node (i, j, k) of the cell
// (3 x 3 x 3) is taken by lane i + 4 j + 16 k (lanes with a coordinate 3 idle
// in the contraction to and from the Q2 basis, whose matrix P2 is 4 x 3).

// out(.., q, ..) = sum_i P2[q][i] v(.., i, ..) (i < 3)
template <int AX>
__device__ __forceinline__ double sweep_p(double v, int lane) {
  constexpr int S = 1 << (2 * AX);
  const int q = (lane >> (2 * AX)) & 3;
  const int base = lane - q * S;
  return c_q3P[3 * q] * __shfl(v, base) + c_q3P[3 * q + 1] * __shfl(v, base + S) +
         c_q3P[3 * q + 2] * __shfl(v, base + 2 * S);
}
// out(.., i, ..) = sum_q P2[q][i] v(.., q, ..) (i < 3; lanes with i = 3 get 0)
template <int AX>
__device__ __forceinline__ double sweep_pt(double v, int lane) {
  constexpr int S = 1 << (2 * AX);
  const int i = (lane >> (2 * AX)) & 3;
  const int base = lane - i * S;
  const int ii = i < 3 ? i : 0;
  double o = c_q3P[ii] * __shfl(v, base) + c_q3P[3 + ii] * __shfl(v, base + S) +
             c_q3P[6 + ii] * __shfl(v, base + 2 * S) + c_q3P[9 + ii] * __shfl(v, base + 3 * S);
  return i < 3 ? o : 0.0;
}

struct Q2PCell {
  int64_t pnode;
  bool used;   // lane is a pressure node of the cell (coordinates < 3)
  __device__ Q2PCell(int64_t n, int64_t c, int lane) {
    const int64_t mp = 2 * n + 1;
    const int64_t i = c % n, j = (c / n) % n, k = c / (n * n);
    const int a = lane & 3, b = (lane >> 2) & 3, cc = lane >> 4;
    used = a < 3 && b < 3 && cc < 3;
    pnode = used ? (2 * i + a) + mp * ((2 * j + b) + mp * (2 * k + cc)) : 0;
  }
};

// p_out += B u (accumulated with atomics; p_out zeroed by the caller)
__global__ __launch_bounds__(256) void k_div_q3(int64_t n, const double* __restrict__ u, double* __restrict__ po) {
  const int lane = threadIdx.x & 63;
  const int64_t cell = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const bool live = cell < n * n * n;
  const int64_t c = live ? cell : 0;
  const Q3Cell qc(n, c, lane);
  double Nx[4], Ny[4], Nz[4], Dx[4], Dy[4], Dz[4];
  row_of<0>(c_q3N, lane, Nx), row_of<1>(c_q3N, lane, Ny), row_of<2>(c_q3N, lane, Nz);
  row_of<0>(c_q3D, lane, Dx), row_of<1>(c_q3D, lane, Dy), row_of<2>(c_q3D, lane, Dz);
  double div = 0.0;
  {
    double v = qc.bnd ? 0.0 : u[3 * qc.node];
    div += sweep<0>(sweep<2>(sweep<1>(sweep<0>(v, lane, Nx), lane, Ny), lane, Nz), lane, Dx);
    v = qc.bnd ? 0.0 : u[3 * qc.node + 1];
    div += sweep<1>(sweep<2>(sweep<1>(sweep<0>(v, lane, Nx), lane, Ny), lane, Nz), lane, Dy);
    v = qc.bnd ? 0.0 : u[3 * qc.node + 2];
    div += sweep<2>(sweep<2>(sweep<1>(sweep<0>(v, lane, Nx), lane, Ny), lane, Nz), lane, Dz);
  }
  const double h = 1.0 / double(n);
  const double wq = c_q3W[lane & 3] * c_q3W[(lane >> 2) & 3] * c_q3W[lane >> 4];
  // -int psi_i div u dx = -h^2 sum_q w_q psi_i(xi_q) (div_xi u)(xi_q)
  const double r = sweep_pt<2>(sweep_pt<1>(sweep_pt<0>(-h * h * wq * div, lane), lane), lane);
  const Q2PCell pc(n, c, lane);
  if (live && pc.used) atomicAdd(&po[pc.pnode], r);
}

// u_out += B^T p on the free velocity dofs (-h^2 sum_q w_q p(xi_q) d_c phi_a(xi_q))
__global__ __launch_bounds__(256) void k_grad_q3(int64_t n, const double* __restrict__ p, double* __restrict__ uo) {
  const int lane = threadIdx.x & 63;
  const int64_t cell = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const bool live = cell < n * n * n;
  const int64_t c = live ? cell : 0;
  const Q2PCell pc(n, c, lane);
  double pv = pc.used ? p[pc.pnode] : 0.0;
  pv = sweep_p<2>(sweep_p<1>(sweep_p<0>(pv, lane), lane), lane);
  const double h = 1.0 / double(n);
  const double wq = c_q3W[lane & 3] * c_q3W[(lane >> 2) & 3] * c_q3W[lane >> 4];
  const double f = -h * h * wq * pv;
  double Nx[4], Ny[4], Nz[4], Dx[4], Dy[4], Dz[4];
  col_of<0>(c_q3N, lane, Nx), col_of<1>(c_q3N, lane, Ny), col_of<2>(c_q3N, lane, Nz);
  col_of<0>(c_q3D, lane, Dx), col_of<1>(c_q3D, lane, Dy), col_of<2>(c_q3D, lane, Dz);
  double out[3];
  out[0] = sweep<2>(sweep<1>(sweep<0>(sweep<0>(f, lane, Dx), lane, Nx), lane, Ny), lane, Nz);
  out[1] = sweep<2>(sweep<1>(sweep<0>(sweep<1>(f, lane, Dy), lane, Nx), lane, Ny), lane, Nz);
  out[2] = sweep<2>(sweep<1>(sweep<0>(sweep<2>(f, lane, Dz), lane, Nx), lane, Ny), lane, Nz);
  const Q3Cell qc(n, c, lane);
  if (!live || qc.bnd) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) atomicAdd(&uo[3 * qc.node + k], out[k]);
}

// p_out += M_p p (mu^{-1}-weighted Q2 mass, h^3 / mu_K M2 x M2 x M2), one
// thread per cell; skipped when *gate != 0 (the CG's convergence flag)
__global__ __launch_bounds__(kBlock) void k_pmass_q2(int64_t n, const double* __restrict__ mu,
                                                     const double* __restrict__ p, double* __restrict__ po,
                                                     const double* __restrict__ gate) {
  if (gate && *gate != 0.0) return;
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= n * n * n) return;
  const int64_t mp = 2 * n + 1;
  const int64_t i = c % n, j = (c / n) % n, k = c / (n * n);
  const int64_t base = 2 * i + mp * (2 * j + mp * 2 * k);
  double v[27];
  for (int a = 0; a < 27; ++a) v[a] = p[base + (a % 3) + mp * ((a / 3) % 3 + mp * (a / 9))];
  // contraction with M2 along x, then y, then z
  double t[27];
  for (int a = 0; a < 27; ++a) {
    const int x = a % 3, r = a - x;
    t[a] = c_q3M2[3 * x] * v[r] + c_q3M2[3 * x + 1] * v[r + 1] + c_q3M2[3 * x + 2] * v[r + 2];
  }
  for (int a = 0; a < 27; ++a) {
    const int y = (a / 3) % 3, r = a - 3 * y;
    v[a] = c_q3M2[3 * y] * t[r] + c_q3M2[3 * y + 1] * t[r + 3] + c_q3M2[3 * y + 2] * t[r + 6];
  }
  const double s = 1.0 / (double(n) * double(n) * double(n) * mu[c]);
  for (int a = 0; a < 27; ++a) {
    const int z = a / 9, r = a - 9 * z;
    const double o = c_q3M2[3 * z] * v[r] + c_q3M2[3 * z + 1] * v[r + 9] + c_q3M2[3 * z + 2] * v[r + 18];
    atomicAdd(&po[base + (a % 3) + mp * ((a / 3) % 3 + mp * (a / 9))], s * o);
  }
}

// diag(M_p) by the same cell sums (one thread per cell)
__global__ __launch_bounds__(kBlock) void k_pmass_diag_q2(int64_t n, const double* __restrict__ mu,
                                                          double* __restrict__ dg) {
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= n * n * n) return;
  const int64_t mp = 2 * n + 1;
  const int64_t i = c % n, j = (c / n) % n, k = c / (n * n);
  const int64_t base = 2 * i + mp * (2 * j + mp * 2 * k);
  const double s = 1.0 / (double(n) * double(n) * double(n) * mu[c]);
  for (int a = 0; a < 27; ++a) {
    const int x = a % 3, y = (a / 3) % 3, z = a / 9;
    atomicAdd(&dg[base + x + mp * (y + mp * z)], s * c_q3M2[4 * x] * c_q3M2[4 * y] * c_q3M2[4 * z]);
  }
}

}  // namespace

void set_q3_constants(const double* N, const double* D, const double* w, const double* P2, const double* M2) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_q3N), N, 16 * sizeof(double));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_q3D), D, 16 * sizeof(double));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_q3W), w, 4 * sizeof(double));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_q3P), P2, 12 * sizeof(double));
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_q3M2), M2, 9 * sizeof(double));
}

template <typename T>
T* q3_halo(const DevLevel& L);
template <>
float* q3_halo<float>(const DevLevel& L) {
  return L.q3_halo_f;
}
template <>
double* q3_halo<double>(const DevLevel& L) {
  return L.q3_halo_d;
}

int64_t q3_halo_words(int64_t n) {
  const int64_t nb = n / kQ3B;
  return nb * nb * nb * kQ3H * 3;
}

template <typename T>
void launch_vmult_q3(const DevLevel& L, const T* x, T* y, bool accumulate, hipStream_t s) {
  // uniform levels have n = 2^l >= 2 cells per edge: whole 2 x 2 x 2 blocks
  const int64_t n = L.n_edge, nb = n / kQ3B, m = 3 * n + 1;
  T* halo = q3_halo<T>(L);
  if (accumulate)
    k_vmult_q3<T, true><<<unsigned(nb * nb * nb), 64 * kQ3B * kQ3B * kQ3B, 0, s>>>(n, mu_of<T>(L), x, y, halo);
  else
    k_vmult_q3<T, false><<<unsigned(nb * nb * nb), 64 * kQ3B * kQ3B * kQ3B, 0, s>>>(n, mu_of<T>(L), x, y, halo);
  if (nb > 1) k_q3_halo_add<T><<<grid_for(m * m * m, 256, int64_t(1) << 30), 256, 0, s>>>(n, halo, y);
}
template void launch_vmult_q3<float>(const DevLevel&, const float*, float*, bool, hipStream_t);
template void launch_vmult_q3<double>(const DevLevel&, const double*, double*, bool, hipStream_t);

// fine level F (m_f = 3n + 1), coarse m_c = 3 n / 2 + 1: x, then y, then z
template <typename T>
void launch_prolong_q3(const DevLevel& F, const T* xc, T* xf, bool add, hipStream_t s) {
  const int64_t mf = 3 * F.n_edge + 1, mc = 3 * (F.n_edge / 2) + 1;
  T* t1 = tr_scratch<T>(F, 0);
  T* t2 = tr_scratch<T>(F, 1);
  k_q3_prolong_pass<T, 0, true, false><<<grid_for(mf * mc * mc, 256, int64_t(1) << 30), 256, 0, s>>>(
      mf, mc, mc, mc, F.q3_pc0, F.q3_pw, xc, t1, false);
  k_q3_prolong_pass<T, 1, false, false><<<grid_for(mf * mf * mc, 256, int64_t(1) << 30), 256, 0, s>>>(
      mf, mf, mc, mc, F.q3_pc0, F.q3_pw, t1, t2, false);
  k_q3_prolong_pass<T, 2, false, true><<<grid_for(mf * mf * mf, 256, int64_t(1) << 30), 256, 0, s>>>(
      mf, mf, mf, mc, F.q3_pc0, F.q3_pw, t2, xf, add);
}
template <typename T>
void launch_restrict_q3(const DevLevel& F, const T* b, const T* t, T* xc, hipStream_t s) {
  const int64_t mf = 3 * F.n_edge + 1, mc = 3 * (F.n_edge / 2) + 1;
  T* s1 = tr_scratch<T>(F, 0);
  T* s2 = tr_scratch<T>(F, 1);
  k_q3_restrict_pass<T, 0, true, false><<<grid_for(mc * mf * mf, 256, int64_t(1) << 30), 256, 0, s>>>(
      mc, mf, mf, mf, F.q3_rptr, F.q3_rcol, F.q3_rw, b, t, s1);
  k_q3_restrict_pass<T, 1, false, false><<<grid_for(mc * mc * mf, 256, int64_t(1) << 30), 256, 0, s>>>(
      mc, mc, mf, mf, F.q3_rptr, F.q3_rcol, F.q3_rw, s1, nullptr, s2);
  k_q3_restrict_pass<T, 2, false, true><<<grid_for(mc * mc * mc, 256, int64_t(1) << 30), 256, 0, s>>>(
      mc, mc, mc, mf, F.q3_rptr, F.q3_rcol, F.q3_rw, s2, nullptr, xc);
}
template void launch_prolong_q3<float>(const DevLevel&, const float*, float*, bool, hipStream_t);
template void launch_prolong_q3<double>(const DevLevel&, const double*, double*, bool, hipStream_t);
template void launch_restrict_q3<float>(const DevLevel&, const float*, const float*, float*, hipStream_t);
template void launch_restrict_q3<double>(const DevLevel&, const double*, const double*, double*, hipStream_t);

void launch_diag_q3(const DevLevel& L, const double* kdiag, double* d, hipStream_t s) {
  k_diag_q3<<<grid_for(L.ncell), kBlock, 0, s>>>(L.n_edge, L.mu_d, kdiag, d);
}

void launch_harmonic_mu64(int64_t ncell, const double* mu_qp, double* mu, hipStream_t s) {
  k_harmonic64<<<grid_for(ncell), kBlock, 0, s>>>(ncell, mu_qp, mu);
}

void launch_rhs_q3(const DevLevel& L, const double* f, double* b, hipStream_t s) {
  k_rhs_q3<<<unsigned((L.ncell + 3) / 4), 256, 0, s>>>(L.n_edge, f, b);
}

void launch_div_q3(const DevLevel& L, const double* u, double* po, hipStream_t s) {
  k_div_q3<<<unsigned((L.ncell + 3) / 4), 256, 0, s>>>(L.n_edge, u, po);
}

void launch_grad_q3(const DevLevel& L, const double* p, double* uo, hipStream_t s) {
  k_grad_q3<<<unsigned((L.ncell + 3) / 4), 256, 0, s>>>(L.n_edge, p, uo);
}

void launch_pmass_q2(const DevLevel& L, const double* p, double* po, hipStream_t s, const double* gate) {
  k_pmass_q2<<<grid_for(L.ncell), kBlock, 0, s>>>(L.n_edge, L.mu_d, p, po, gate);
}

void launch_pmass_diag_q2(const DevLevel& L, double* dg, hipStream_t s) {
  k_pmass_diag_q2<<<grid_for(L.ncell), kBlock, 0, s>>>(L.n_edge, L.mu_d, dg);
}

}  // namespace mfgmg
