// Device kernels for the matrix-free GMG Stokes path (gfx950, wave64).
#include "ops.h"

#include <algorithm>
#include <utility>

#include "brick_kernel.h"
#include "cell_kernel.h"

namespace mfgmg {

namespace {

constexpr int kBlock = 256;
constexpr int kCellBlock = 64;     // cells per workgroup for the cell kernels
constexpr int kRedBlocks = 1024;   // partial sums of the reductions
#ifndef MFGMG_RESTRICT_LANES
#define MFGMG_RESTRICT_LANES 16
#endif
#ifndef MFGMG_PROLONG_LANES
#define MFGMG_PROLONG_LANES 4
#endif
constexpr int kRestrictLanes = MFGMG_RESTRICT_LANES;   // lanes per row of the CSR transfers
constexpr int kProlongLanes = MFGMG_PROLONG_LANES;
#ifndef MFGMG_BRICK_MIN_EDGE
#define MFGMG_BRICK_MIN_EDGE 32
#endif
constexpr int64_t kBrickMinEdge = MFGMG_BRICK_MIN_EDGE;   // smallest uniform level using the brick kernel

__constant__ double c_khat_diag[81];
__constant__ double c_bhat[8 * 81];
__constant__ double c_mhat[64];

inline unsigned grid_for(int64_t n, int block = kBlock, int64_t cap = 1 << 20) {
  int64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return unsigned(g);
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  atomicAdd(p, v);   // hardware float/double add (built with -munsafe-fp-atomics)
}

// ----------------------------------------------------------- slot access
// Velocity slot of local node a (x fastest) of cell c: node index >= 0 for a
// free node, -1 for a Dirichlet node, -(2+h) for hanging row h.
struct UniformCell {
  int64_t n, m, base;
  bool lo[3], hi[3];
  __device__ UniformCell(int64_t n_, int64_t c) : n(n_), m(2 * n_ + 1) {
    const int64_t i = c % n, j = (c / n) % n, k = c / (n * n);
    base = 2 * i + m * (2 * j + m * 2 * k);
    lo[0] = i == 0, lo[1] = j == 0, lo[2] = k == 0;
    hi[0] = i == n - 1, hi[1] = j == n - 1, hi[2] = k == n - 1;
  }
  __device__ __forceinline__ int32_t slot(int x, int y, int z) const {
    const bool dir = (x == 0 && lo[0]) || (x == 2 && hi[0]) || (y == 0 && lo[1]) || (y == 2 && hi[1]) ||
                     (z == 0 && lo[2]) || (z == 2 && hi[2]);
    return dir ? -1 : int32_t(base + x + m * (y + m * z));
  }
};

// The value of lane - 1 within the lane's row of 16 lanes (DPP row shift
// right by one; 0 at a row's first lane)
__device__ __forceinline__ int dpp_from_left(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);
}
__device__ __forceinline__ float from_left_lane(float v) {
  return __int_as_float(dpp_from_left(__float_as_int(v)));
}
__device__ __forceinline__ double from_left_lane(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(dpp_from_left(int(b))), hi = unsigned(dpp_from_left(int(b >> 32)));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// ------------------------------------------------------------- vmult
template <typename T>
__global__ __launch_bounds__(256) void k_init_out_uniform(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t m = 2 * n + 1, nn = m * m * m;
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < nn; v += int64_t(gridDim.x) * blockDim.x) {
    const int64_t X = v % m, Y = (v / m) % m, Z = v / (m * m);
    const bool b = X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1;
    y[3 * v] = b ? x[3 * v] : T(0);
    y[3 * v + 1] = b ? x[3 * v + 1] : T(0);
    y[3 * v + 2] = b ? x[3 * v + 2] : T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_init_out_general(int64_t nn, const uint8_t* __restrict__ cmask,
                                                          const T* __restrict__ x, T* __restrict__ y) {
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < nn; v += int64_t(gridDim.x) * blockDim.x) {
    const unsigned b = cmask[v];
    y[3 * v] = (b & 1) ? x[3 * v] : T(0);
    y[3 * v + 1] = (b & 2) ? x[3 * v + 1] : T(0);
    y[3 * v + 2] = (b & 4) ? x[3 * v + 2] : T(0);
  }
}

// The operator on a uniform level below the brick kernel's sizes, three
// threads per cell, one per output component: there the grid is a few waves
// and the time is the per-thread chain of the cell operator, about 2.5x
// shorter than with one thread per cell.
// Block: 64 cells x 3 components (wave c holds component c); each thread
// interpolates its component to the Gauss points, the 81 values are shared
// through LDS, and each thread produces its component's 27 outputs.
template <typename T>
__global__ __launch_bounds__(192) void k_vmult_uniform3(int64_t n, const T* __restrict__ mu, const T* __restrict__ x,
                                                        T* __restrict__ y) {
  __shared__ T wsh[3][27][64];
  const int lane = threadIdx.x & 63;
  const int c = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int64_t cell = blockIdx.x * int64_t(64) + lane;
  const bool live = cell < n * n * n;
  const UniformCell uc(n, live ? cell : 0);
  T w[27];
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int yy = 0; yy < 3; ++yy)
#pragma unroll
      for (int xx = 0; xx < 3; ++xx) {
        const int32_t sl = uc.slot(xx, yy, z);
        w[xx + 3 * yy + 9 * z] = sl >= 0 ? x[3 * int64_t(sl) + c] : T(0);
      }
  cellop::interp_all(w);
#pragma unroll
  for (int a = 0; a < 27; ++a) wsh[c][a][lane] = w[a];
  __syncthreads();
  T W[3][27];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int a = 0; a < 27; ++a) W[cc][a] = wsh[cc][a][lane];
  const T mu_h = mu[live ? cell : 0] / T(n);
  if (c == 0) cellop::apply_cell_row<0>(W, w, mu_h);
  else if (c == 1) cellop::apply_cell_row<1>(W, w, mu_h);
  else cellop::apply_cell_row<2>(W, w, mu_h);
  cellop::interp_all_t(w);
  // A cell's xx = 2 nodes are the next cell's xx = 0 nodes.  Within a row of
  // 16 lanes the next cell along x is the next lane, which adds the values
  // passed on (DPP row shift) into its own: those nodes take one atomic
  // instead of two (device-scope atomics, served beyond the XCD's L2, are most
  // of this kernel's time on a 16^3 level).
  // The same along y: the next cell along y is lane + n (when still in the
  // block), which takes the yy = 2 row of values (those not already passed on
  // along x) into its yy = 0 row.
  const int64_t cc0 = live ? cell : 0;
  const int ix = int(cc0 % n), iy = int((cc0 / n) % n);
  const bool send_x = ix < n - 1 && (lane & 15) != 15, recv_x = ix > 0 && (lane & 15) != 0;
  const bool send_y = iy < n - 1 && lane + n < 64, recv_y = iy > 0 && lane >= n;
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int yy = 0; yy < 3; ++yy) {
      const T r = from_left_lane(w[2 + 3 * yy + 9 * z]);
      if (recv_x) w[3 * yy + 9 * z] += r;
      if (send_x) w[2 + 3 * yy + 9 * z] = T(0);   // handed over
    }
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int xx = 0; xx < 3; ++xx) {
      const T r = __shfl_up(w[xx + 6 + 9 * z], unsigned(n));
      if (recv_y) w[xx + 9 * z] += r;
    }
  if (!live) return;
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int yy = 0; yy < 3; ++yy)
#pragma unroll
      for (int xx = 0; xx < 3; ++xx) {
        const int32_t sl = uc.slot(xx, yy, z);
        if (sl >= 0 && !(xx == 2 && send_x) && !(yy == 2 && send_y))
          atomic_add(&y[3 * int64_t(sl) + c], w[xx + 3 * yy + 9 * z]);
      }
}

// y(node) += the face slots of the node (one thread per node, 2-8 slots)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_face_gather(int64_t nf, const int32_t* __restrict__ node,
                                                        const int32_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ ent,
                                                        const T* __restrict__ fslot, T* __restrict__ y) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nf; i += int64_t(gridDim.x) * blockDim.x) {
    T a0 = T(0), a1 = T(0), a2 = T(0);
    for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      const T* fs = fslot + 3 * int64_t(ent[e]);
      a0 += fs[0], a1 += fs[1], a2 += fs[2];
    }
    T* yp = y + 3 * int64_t(node[i]);
    yp[0] += a0, yp[1] += a1, yp[2] += a2;
  }
}

// pressure version (one value per slot); returns when the gate is set, as the
// mass kernels do
__global__ __launch_bounds__(kBlock) void k_pface_gather(int64_t nf, const int32_t* __restrict__ node,
                                                         const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ ent,
                                                         const double* __restrict__ fslot, double* __restrict__ po,
                                                         const double* __restrict__ gate) {
  if (gate && *gate != 0.0) return;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nf; i += int64_t(gridDim.x) * blockDim.x) {
    double a = 0.0;
    for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) a += fslot[ent[e]];
    po[node[i]] += a;
  }
}

template <typename T>
T* face_slots(const DevLevel& L);
template <>
float* face_slots<float>(const DevLevel& L) {
  return L.fslot_f;
}
template <>
double* face_slots<double>(const DevLevel& L) {
  return L.fslot_d;
}

// The single cells of a non-uniform level (those in no block): the cell
// operator with three threads per cell, one velocity component each (a wave
// per component, as k_vmult_uniform3), hanging nodes resolved through the
// level's constraint rows (HANG).  A thread gathers,
// interpolates and scatters its component's 27 values and computes its
// component's row of the cell operator from all three interpolated
// components, exchanged through LDS.  The single cells are few, so the kernel
// is latency-bound; this cuts each thread's chain of dependent loads,
// arithmetic and atomics to about a third.
// (cm: the level's constrained-component masks on no-normal-flux levels,
// where a master's fixed component carries zero; null otherwise)
template <typename T>
__device__ __forceinline__ T gather1(int32_t s, int comp, const T* __restrict__ x, const int64_t* __restrict__ hptr,
                                     const int32_t* __restrict__ hm, const T* __restrict__ hw,
                                     const uint8_t* __restrict__ cm) {
  if (s >= 0) return slot_fixed(s, comp) ? T(0) : x[3 * int64_t(slot_node(s)) + comp];
  if (s == -1) return T(0);
  const int64_t h = -int64_t(s) - 2;
  T v = T(0);
  for (int64_t q = hptr[h]; q < hptr[h + 1]; ++q)
    if (!cm || !((cm[hm[q]] >> comp) & 1)) v += hw[q] * x[3 * int64_t(hm[q]) + comp];
  return v;
}
template <typename T>
__device__ __forceinline__ void scatter1(int32_t s, int comp, T v, T* __restrict__ y, const int64_t* __restrict__ hptr,
                                         const int32_t* __restrict__ hm, const T* __restrict__ hw,
                                         const uint8_t* __restrict__ cm) {
  if (s >= 0) {
    if (!slot_fixed(s, comp)) atomic_add(&y[3 * int64_t(slot_node(s)) + comp], v);
  } else if (s < -1) {
    const int64_t h = -int64_t(s) - 2;
    for (int64_t q = hptr[h]; q < hptr[h + 1]; ++q)
      if (!cm || !((cm[hm[q]] >> comp) & 1)) atomic_add(&y[3 * int64_t(hm[q]) + comp], hw[q] * v);
  }
}
template <typename T, bool HANG>
__global__ __launch_bounds__(192) void k_vmult_general3(const int32_t* __restrict__ cells, int64_t ncells,
                                                        const int32_t* __restrict__ slots,
                                                        const int8_t* __restrict__ clev, const T* __restrict__ mu,
                                                        const int64_t* __restrict__ hptr,
                                                        const int32_t* __restrict__ hm, const T* __restrict__ hw,
                                                        const uint8_t* __restrict__ cm, const T* __restrict__ x,
                                                        T* __restrict__ y) {
  __shared__ T wsh[3][27][64];
  const int lane = threadIdx.x & 63;
  const int comp = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int64_t t = blockIdx.x * int64_t(64) + lane;
  const bool live = t < ncells;
  const int64_t c = live ? cells[t] : 0;   // a dead lane works on cell 0 and writes nothing
  int32_t sl[27];
  T w[27];
#pragma unroll
  for (int a = 0; a < 27; ++a) {
    sl[a] = slots[27 * c + a];
    if constexpr (HANG)
      w[a] = gather1<T>(sl[a], comp, x, hptr, hm, hw, cm);
    else
      w[a] = sl[a] >= 0 && !slot_fixed(sl[a], comp) ? x[3 * int64_t(slot_node(sl[a])) + comp] : T(0);
  }
  cellop::interp_all(w);
#pragma unroll
  for (int a = 0; a < 27; ++a) wsh[comp][a][lane] = w[a];
  __syncthreads();
  T W[3][27];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int a = 0; a < 27; ++a) W[cc][a] = wsh[cc][a][lane];
  const T mu_h = mu[c] * T(ldexp(1.0, -int(clev[c])));
  if (comp == 0) cellop::apply_cell_row<0>(W, w, mu_h);
  else if (comp == 1) cellop::apply_cell_row<1>(W, w, mu_h);
  else cellop::apply_cell_row<2>(W, w, mu_h);
  cellop::interp_all_t(w);
  if (!live) return;
#pragma unroll
  for (int a = 0; a < 27; ++a) {
    if constexpr (HANG)
      scatter1<T>(sl[a], comp, w[a], y, hptr, hm, hw, cm);
    else if (sl[a] >= 0 && !slot_fixed(sl[a], comp))
      atomic_add(&y[3 * int64_t(slot_node(sl[a])) + comp], w[a]);
  }
}

// Blocks of B x B x B same-level cells on a non-uniform level (complete
// sibling groups of the level mesh: the 8 children, or the 64 grandchildren,
// of one cell).  One wave per workgroup treats 64 / B^3 blocks, one lane per
// cell.  As in the brick kernel, each block's (2B+1)^3 node box is staged in
// LDS, the cells gather from LDS, and their results are accumulated in LDS
// class by class (local node a in {0,1} | {2} per axis: within a class no
// two cells of a block share a node).  Hanging points are resolved inside
// the box: their masters are lattice points of the same block, so the
// gather interpolates them from the staged masters and the write-back first
// distributes their accumulated values onto the masters (FP64: LDS atomics;
// FP32: one lane per hanging point, then one per master).  Nodes strictly inside a block belong to its cells alone and are
// stored; the values of its free face nodes go to the block's face slots
// and k_face_gather adds each node's slots into y.  LDS layout per block and
// component: every axis split into even then odd lattice points.
template <int B>
__device__ __forceinline__ int bsplit(int l) {
  return (l & 1) ? (B + 1) + (l >> 1) : (l >> 1);
}

template <typename T>
__device__ __forceinline__ const T* blk_hw(const DevBlocks& b);
template <>
__device__ __forceinline__ const float* blk_hw<float>(const DevBlocks& b) {
  return b.hw_f;
}
template <>
__device__ __forceinline__ const double* blk_hw<double>(const DevBlocks& b) {
  return b.hw_d;
}
template <typename T>
__device__ __forceinline__ const T* blk_hw2(const DevBlocks& b);
template <>
__device__ __forceinline__ const float* blk_hw2<float>(const DevBlocks& b) {
  return b.hw2_f;
}
template <>
__device__ __forceinline__ const double* blk_hw2<double>(const DevBlocks& b) {
  return b.hw2_d;
}

// ACC: inner points are added to y (y += A x); otherwise stored (y was initialised to zero there)
template <typename T, int B, bool ACC>
__global__ __launch_bounds__(64) void k_vmult_blocks(DevBlocks blk, const int8_t* __restrict__ clev,
                                                     const T* __restrict__ mu, const T* __restrict__ x,
                                                     T* __restrict__ y, T* __restrict__ fslot) {
  constexpr int NC = B * B * B, NB = 64 / NC;   // cells per block, blocks per wave
  constexpr int E = 2 * B + 1, P = E * E * E, W = 3 * P;
  constexpr int KP = (NB * P + 63) / 64;        // lattice points per lane
  __shared__ T buf[NB * W];
  const int lane = threadIdx.x;
  const int64_t blk0 = int64_t(blockIdx.x) * NB;
  const int nb = int(std::min<int64_t>(NB, blk.n - blk0));   // blocks of this wave
  const int np = nb * P;
  const T* __restrict__ hw = blk_hw<T>(blk);
  // lattice point p of the wave (block p / P) -> LDS offset of its component 0
  auto lds_of = [&](int bl, int p) {
    const int px = p % E, py = (p / E) % E, pz = p / (E * E);
    return bl * W + bsplit<B>(px) + E * bsplit<B>(py) + E * E * bsplit<B>(pz);
  };
  // staging: every slot load, then every value load, issued before use;
  // points of missing blocks, Dirichlet and hanging points (and components
  // fixed by the no-normal-flux condition) store zero.  The slots stay in
  // registers for the write-back.
  int32_t sl[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int pa = lane + 64 * k;
    sl[k] = pa < np ? blk.slots[blk0 * P + pa] : -1;
  }
  {
    T v[KP][3];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int64_t i = 3 * int64_t(sl[k] >= 0 ? slot_node(sl[k]) : 0);
      v[k][0] = x[i], v[k][1] = x[i + 1], v[k][2] = x[i + 2];
    }
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int pa = lane + 64 * k;
      if (pa < NB * P) {
        const int o = lds_of(pa / P, pa % P);
        const bool f = sl[k] >= 0;
        buf[o] = f && !slot_fixed(sl[k], 0) ? v[k][0] : T(0);
        buf[o + P] = f && !slot_fixed(sl[k], 1) ? v[k][1] : T(0);
        buf[o + 2 * P] = f && !slot_fixed(sl[k], 2) ? v[k][2] : T(0);
      }
    }
  }
  __syncthreads();
  // hanging points: interpolate from their masters in the box.  FP32: one
  // lane per hanging point (its entries are consecutive), no LDS atomics,
  // whose FP32 form is slow here (leaf of the adaptive 32^3 + 2 workload: 144
  // -> 125 us per call); FP64: one lane per entry with LDS atomics (the
  // grouped form: 198 -> 225 us)
  if constexpr (sizeof(T) == 8) {
    const int h0 = blk.hoff[blk0], h1 = blk.hoff[blk0 + nb];
    for (int e = h0 + lane; e < h1; e += 64) {
      const int32_t en = blk.hent[e];
      const int p = en & 1023, pm = (en >> 10) & 1023, bl = en >> 20;
      const T w = hw[e];
      const int o = lds_of(bl, p), om = lds_of(bl, pm);
#pragma unroll
      for (int q = 0; q < 3; ++q) atomicAdd(&buf[o + q * P], w * buf[om + q * P]);
    }
  } else {
    const int k0 = blk.g1off[blockIdx.x], k1 = blk.g1off[blockIdx.x + 1] - 1;
    for (int k = k0 + lane; k < k1; k += 64) {
      const int e0 = blk.g1[k], e1 = blk.g1[k + 1];
      T a0 = T(0), a1 = T(0), a2 = T(0);
      int o = 0;
      for (int e = e0; e < e1; ++e) {
        const int32_t en = blk.hent[e];
        const int p = en & 1023, pm = (en >> 10) & 1023, bl = en >> 20;
        const T w = hw[e];
        const int om = lds_of(bl, pm);
        o = lds_of(bl, p);
        a0 += w * buf[om], a1 += w * buf[om + P], a2 += w * buf[om + 2 * P];
      }
      buf[o] = a0, buf[o + P] = a1, buf[o + 2 * P] = a2;
    }
  }
  __syncthreads();
  const int bl = lane / NC, lc = lane - bl * NC;
  const int ca = lc % B, cb = (lc / B) % B, cc = lc / (B * B);
  const int base = bl * W;
  T U[3][27];
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int yy = 0; yy < 3; ++yy)
#pragma unroll
      for (int xx = 0; xx < 3; ++xx) {
        const int off = base + bsplit<B>(2 * ca + xx) + E * bsplit<B>(2 * cb + yy) + E * E * bsplit<B>(2 * cc + z);
#pragma unroll
        for (int q = 0; q < 3; ++q) U[q][xx + 3 * yy + 9 * z] = buf[off + q * P];
      }
  __syncthreads();
  for (int e = lane; e < NB * W; e += 64) buf[e] = T(0);
  T coef = T(0);
  if (bl < nb) {
    const int32_t c = blk.cells[(blk0 + bl) * NC + lc];
    coef = mu[c] * T(ldexp(1.0, -int(clev[c])));
  }
  cellop::apply_cell<T>(U, coef);
  __syncthreads();
#pragma unroll
  for (int cls = 0; cls < 8; ++cls) {
    const int ac = cls & 1, bc = (cls >> 1) & 1, zc = cls >> 2;
#pragma unroll
    for (int z = zc ? 2 : 0; z < (zc ? 3 : 2); ++z)
#pragma unroll
      for (int yy = bc ? 2 : 0; yy < (bc ? 3 : 2); ++yy)
#pragma unroll
        for (int xx = ac ? 2 : 0; xx < (ac ? 3 : 2); ++xx) {
          const int off = base + bsplit<B>(2 * ca + xx) + E * bsplit<B>(2 * cb + yy) + E * E * bsplit<B>(2 * cc + z);
#pragma unroll
          for (int q = 0; q < 3; ++q) buf[off + q * P] += U[q][xx + 3 * yy + 9 * z];
        }
    __syncthreads();
  }
  // hanging points pass their accumulated values on to their masters (the
  // hanging entries themselves are not read again): FP64 one lane per entry
  // with LDS atomics, FP32 one lane per master over the entries sorted by
  // master
  if constexpr (sizeof(T) == 8) {
    const int h0 = blk.hoff[blk0], h1 = blk.hoff[blk0 + nb];
    for (int e = h0 + lane; e < h1; e += 64) {
      const int32_t en = blk.hent[e];
      const int p = en & 1023, pm = (en >> 10) & 1023, bl2 = en >> 20;
      const T w = hw[e];
      const int o = lds_of(bl2, p), om = lds_of(bl2, pm);
#pragma unroll
      for (int q = 0; q < 3; ++q) atomicAdd(&buf[om + q * P], w * buf[o + q * P]);
    }
  } else {
    const T* __restrict__ hw2 = blk_hw2<T>(blk);
    const int k0 = blk.g2off[blockIdx.x], k1 = blk.g2off[blockIdx.x + 1] - 1;
    for (int k = k0 + lane; k < k1; k += 64) {
      const int e0 = blk.g2[k], e1 = blk.g2[k + 1];
      T a0 = T(0), a1 = T(0), a2 = T(0);
      int om = 0;
      for (int e = e0; e < e1; ++e) {
        const int32_t en = blk.hent2[e];
        const int p = en & 1023, pm = (en >> 10) & 1023, bl2 = en >> 20;
        const T w = hw2[e];
        const int o = lds_of(bl2, p);
        om = lds_of(bl2, pm);
        a0 += w * buf[o], a1 += w * buf[o + P], a2 += w * buf[o + 2 * P];
      }
      buf[om] += a0, buf[om + P] += a1, buf[om + 2 * P] += a2;
    }
  }
  __syncthreads();
  // write-back of the free points: inside the block stored (added when
  // accumulating); on its faces, where other cells contribute too, to the
  // block's slots, summed into y by the face gather (no atomics).  Fixed
  // components (on the domain boundary, so never inside a block) send zero.
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (sl[k] < 0) continue;
    const int pa = lane + 64 * k, p = pa % P;
    const int o = lds_of(pa / P, p);
    const T v0 = slot_fixed(sl[k], 0) ? T(0) : buf[o];
    const T v1 = slot_fixed(sl[k], 1) ? T(0) : buf[o + P];
    const T v2 = slot_fixed(sl[k], 2) ? T(0) : buf[o + 2 * P];
    const int px = p % E, py = (p / E) % E, pz = p / (E * E);
    const bool inner = px > 0 && px < E - 1 && py > 0 && py < E - 1 && pz > 0 && pz < E - 1;
    T* yp = y + 3 * int64_t(slot_node(sl[k]));
    if (inner && ACC) {
      yp[0] += v0, yp[1] += v1, yp[2] += v2;
    } else if (inner) {
      yp[0] = v0, yp[1] = v1, yp[2] = v2;
    } else {
      T* fs = fslot + 3 * ((blk0 + pa / P) * P + p);
      fs[0] = v0, fs[1] = v1, fs[2] = v2;
    }
  }
}

template <typename T>
const T* hw_of(const DevLevel& L);
template <>
const float* hw_of<float>(const DevLevel& L) {
  return L.hw_f;
}
template <>
const double* hw_of<double>(const DevLevel& L) {
  return L.hw_d;
}

// ------------------------------------------------------------- diagonal
__global__ __launch_bounds__(kCellBlock) void k_diag_uniform(int64_t n, const double* __restrict__ mu,
                                                             double* __restrict__ d) {
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= n * n * n) return;
  const UniformCell cell(n, c);
  const double s = mu[c] / double(n);
  for (int z = 0; z < 3; ++z)
    for (int y = 0; y < 3; ++y)
      for (int x = 0; x < 3; ++x) {
        const int32_t sl = cell.slot(x, y, z);
        if (sl < 0) continue;
        const int a = x + 3 * y + 9 * z;
        for (int cc = 0; cc < 3; ++cc) atomicAdd(&d[3 * int64_t(sl) + cc], s * c_khat_diag[3 * a + cc]);
      }
}

__global__ __launch_bounds__(kCellBlock) void k_diag_regular(const int32_t* __restrict__ cells, int64_t ncells,
                                                             const int32_t* __restrict__ slots,
                                                             const int8_t* __restrict__ clev,
                                                             const double* __restrict__ mu, double* __restrict__ d) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= ncells) return;
  const int64_t c = cells[t];
  const double s = mu[c] * ldexp(1.0, -int(clev[c]));
  for (int a = 0; a < 27; ++a) {
    const int32_t sl = slots[27 * c + a];
    if (sl < 0) continue;
    for (int cc = 0; cc < 3; ++cc) atomicAdd(&d[3 * int64_t(slot_node(sl)) + cc], s * c_khat_diag[3 * a + cc]);
  }
}

// Cells with hanging nodes: diagonal of the resolved local matrix C_l^T K_e C_l.
// One workgroup per cell; entry (M, c) gets sum_{p,q} w_p w_q K[(a_p,c),(a_q,c)]
// over the local nodes a_p, a_q whose expansions contain master M.
__global__ __launch_bounds__(64) void k_diag_hanging(const int32_t* __restrict__ cells,
                                                     const int32_t* __restrict__ slots,
                                                     const int8_t* __restrict__ clev, const double* __restrict__ mu,
                                                     const int64_t* __restrict__ hptr,
                                                     const int32_t* __restrict__ hm, const double* __restrict__ hw,
                                                     const double* __restrict__ khat, double* __restrict__ d) {
  __shared__ int32_t t_a[256];
  __shared__ int32_t t_m[256];
  __shared__ double t_w[256];
  __shared__ int32_t dm[256];
  __shared__ int nt, nd;
  const int64_t c = cells[blockIdx.x];
  if (threadIdx.x == 0) {
    int k = 0;
    for (int a = 0; a < 27; ++a) {
      const int32_t s = slots[27 * c + a];
      if (s >= 0) {
        t_a[k] = a, t_m[k] = slot_node(s), t_w[k] = 1.0, ++k;
      } else if (s < -1) {
        const int64_t h = -int64_t(s) - 2;
        for (int64_t q = hptr[h]; q < hptr[h + 1] && k < 256; ++q) t_a[k] = a, t_m[k] = hm[q], t_w[k] = hw[q], ++k;
      }
    }
    nt = k;
    int u = 0;
    for (int p = 0; p < k; ++p) {
      bool found = false;
      for (int q = 0; q < u; ++q)
        if (dm[q] == t_m[p]) {
          found = true;
          break;
        }
      if (!found) dm[u++] = t_m[p];
    }
    nd = u;
  }
  __syncthreads();
  const double s = mu[c] * ldexp(1.0, -int(clev[c]));
  for (int r = threadIdx.x; r < nd; r += blockDim.x) {
    const int32_t M = dm[r];
    for (int cc = 0; cc < 3; ++cc) {
      double acc = 0.0;
      for (int p = 0; p < nt; ++p) {
        if (t_m[p] != M) continue;
        for (int q = 0; q < nt; ++q) {
          if (t_m[q] != M) continue;
          acc += t_w[p] * t_w[q] * khat[(3 * t_a[p] + cc) * 81 + 3 * t_a[q] + cc];
        }
      }
      atomicAdd(&d[3 * int64_t(M) + cc], s * acc);
    }
  }
}

__global__ void k_invert_diag_uniform(int64_t n, const double* __restrict__ d, double* __restrict__ md,
                                      float* __restrict__ mf) {
  const int64_t m = 2 * n + 1, nn = m * m * m;
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < nn; v += int64_t(gridDim.x) * blockDim.x) {
    const int64_t X = v % m, Y = (v / m) % m, Z = v / (m * m);
    const bool b = X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1;
    for (int c = 0; c < 3; ++c) {
      const double r = b ? 1.0 : 1.0 / d[3 * v + c];
      md[3 * v + c] = r;
      mf[3 * v + c] = float(r);
    }
  }
}

__global__ void k_invert_diag_general(int64_t nn, const uint8_t* __restrict__ cmask, const double* __restrict__ d,
                                      double* __restrict__ md, float* __restrict__ mf) {
  for (int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; v < nn; v += int64_t(gridDim.x) * blockDim.x) {
    const unsigned b = cmask[v];
    for (int c = 0; c < 3; ++c) {
      const double r = ((b >> c) & 1) ? 1.0 : 1.0 / d[3 * v + c];
      md[3 * v + c] = r;
      mf[3 * v + c] = float(r);
    }
  }
}

// ------------------------------------------------------------- Chebyshev
// The smoother's Chebyshev updates (k_chebx_*) can also prepare the output of
// the next operator call on levels whose operator otherwise starts with an
// initialisation kernel (k_init_out_*): tn = (constrained dof ? src : 0), src
// being the new d, or the new x when from_x.  Constrained: the dof's bit of
// cmask on general levels (cmask given), a boundary node of the m^3 lattice on
// uniform ones.  tn may be t itself (each entry is read before it is written, by the
// same thread; t and tn are therefore not restrict).
template <typename T>
struct OutPrep {
  T* tn;
  const uint8_t* cmask;
  int64_t m;
  int from_x;
};
__device__ __forceinline__ bool constrained_dof(int64_t i, const uint8_t* cmask, int64_t m) {
  const int64_t v = i / 3;
  if (cmask) return (cmask[v] >> (i - 3 * v)) & 1;
  const int64_t X = v % m, Y = (v / m) % m, Z = v / (m * m);
  return X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1;
}
template <typename T>
__device__ __forceinline__ void out_prep(const OutPrep<T>& o, int64_t i, T di, T xi) {
  if (o.tn) o.tn[i] = constrained_dof(i, o.cmask, o.m) ? (o.from_x ? xi : di) : T(0);
}

template <typename T>
__global__ void k_cheb_init0(int64_t n, const T* __restrict__ b, const T* __restrict__ minv, T* __restrict__ r,
                             T* __restrict__ d, T* __restrict__ x, T it) {
  // XCD-contiguous ranges: t was just written by the operator in the same order
  for (int64_t i = brick::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const T bi = b[i];
    const T di = minv[i] * bi * it;
    r[i] = bi;
    d[i] = di;
    x[i] = di;
  }
}

template <typename T>
__global__ void k_cheb_init(int64_t n, const T* __restrict__ b, const T* __restrict__ t, const T* __restrict__ minv,
                            T* __restrict__ r, T* __restrict__ d, T* __restrict__ x, T it) {
  // XCD-contiguous ranges: t was just written by the operator in the same order
  for (int64_t i = brick::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const T ri = b[i] - t[i];
    const T di = minv[i] * ri * it;
    const T xi = x[i] + di;
    r[i] = ri;
    d[i] = di;
    x[i] = xi;
  }
}

template <typename T>
__global__ void k_cheb_step(int64_t n, const T* __restrict__ t, const T* __restrict__ minv, T* __restrict__ r,
                            T* __restrict__ d, T* __restrict__ x, T alpha, T beta) {
  // XCD-contiguous ranges: t was just written by the operator in the same order
  for (int64_t i = brick::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const T ri = r[i] - t[i];
    const T di = alpha * d[i] + beta * minv[i] * ri;
    const T xi = x[i] + di;
    r[i] = ri;
    d[i] = di;
    x[i] = xi;
  }
}

// The smoother's own form of the same iteration: the residual is formed as
// b - A x_k instead of by the recurrence r_k = r_{k-1} - A d_{k-1} (equal in
// exact arithmetic), so r is never stored and the operator is applied to x.
// x0 = 0: d = (1/theta) M b, x = d; first step from a given x: t = A x,
// d = (1/theta) M (b - t), x += d; later steps: d = alpha d + beta M (b - t),
// x += d.  Each prepares t for the next operator call on x (out_prep).
template <typename T>
__global__ void k_chebx_init0(int64_t n, const T* __restrict__ b, const T* __restrict__ minv, T* __restrict__ d,
                              T* __restrict__ x, T it, OutPrep<T> o) {
  for (int64_t i = brick::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const T di = minv[i] * b[i] * it;
    d[i] = di;
    x[i] = di;
    out_prep(o, i, di, di);
  }
}
template <typename T>
__global__ void k_chebx_step(int64_t n, const T* __restrict__ b, const T* t, const T* __restrict__ minv,
                             T* __restrict__ d, T* __restrict__ x, T alpha, T beta, OutPrep<T> o) {
  // alpha = 0: the first step from a given x (d is not read)
  for (int64_t i = brick::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const T ri = b[i] - t[i];
    const T di = (alpha != T(0) ? alpha * d[i] : T(0)) + beta * minv[i] * ri;
    const T xi = x[i] + di;
    d[i] = di;
    x[i] = xi;
    out_prep(o, i, di, xi);
  }
}

// ------------------------------------------------------------- transfers
// CSR transfers, G lanes per row (rows of R hold up to 125 fine nodes, rows
// of P up to 27 coarse ones): the lanes of a group read consecutive entries
// (coalesced column and weight loads, G gathers in flight per row) and
// reduce with shuffles inside the group.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// (cmf, cmc: constrained-component masks of the fine and coarse level, or
// null: a masked coarse component carries nothing, a masked fine component
// receives nothing)
template <typename T, int G, typename W = float>
__global__ __launch_bounds__(kBlock) void k_prolong(int64_t nf, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col, const W* __restrict__ w,
                                                    const T* __restrict__ xc, T* __restrict__ xf, bool add,
                                                    const uint8_t* __restrict__ cmf, const uint8_t* __restrict__ cmc) {
  const int sub = int(threadIdx.x) % G;
  for (int64_t f = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) / G; f < nf;
       f += int64_t(gridDim.x) * (blockDim.x / G)) {
    T a0 = T(0), a1 = T(0), a2 = T(0);
    for (int64_t q = ptr[f] + sub; q < ptr[f + 1]; q += G) {
      const int64_t cc = 3 * int64_t(col[q]);
      const T ww = T(w[q]);
      if (cmc) {
        const unsigned m = cmc[col[q]];
        a0 += (m & 1) ? T(0) : ww * xc[cc];
        a1 += (m & 2) ? T(0) : ww * xc[cc + 1];
        a2 += (m & 4) ? T(0) : ww * xc[cc + 2];
      } else {
        a0 += ww * xc[cc];
        a1 += ww * xc[cc + 1];
        a2 += ww * xc[cc + 2];
      }
    }
    a0 = group_sum<G>(a0), a1 = group_sum<G>(a1), a2 = group_sum<G>(a2);
    if (cmf) {
      const unsigned m = cmf[f];
      if (m & 1) a0 = T(0);
      if (m & 2) a1 = T(0);
      if (m & 4) a2 = T(0);
    }
    if (sub == 0) {
      if (add) {
        xf[3 * f] += a0;
        xf[3 * f + 1] += a1;
        xf[3 * f + 2] += a2;
      } else {
        xf[3 * f] = a0;
        xf[3 * f + 1] = a1;
        xf[3 * f + 2] = a2;
      }
    }
  }
}

template <typename T, int G, typename W = float>
__global__ __launch_bounds__(kBlock) void k_restrict(int64_t nc, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col, const W* __restrict__ w,
                                                     const T* __restrict__ b, const T* __restrict__ t,
                                                     T* __restrict__ xc, const uint8_t* __restrict__ cmf,
                                                     const uint8_t* __restrict__ cmc) {
  const int sub = int(threadIdx.x) % G;
  for (int64_t c = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) / G; c < nc;
       c += int64_t(gridDim.x) * (blockDim.x / G)) {
    T a0 = T(0), a1 = T(0), a2 = T(0);
    for (int64_t q = ptr[c] + sub; q < ptr[c + 1]; q += G) {
      const int64_t ff = 3 * int64_t(col[q]);
      const T ww = T(w[q]);
      T r0, r1, r2;
      if (t) {
        r0 = b[ff] - t[ff], r1 = b[ff + 1] - t[ff + 1], r2 = b[ff + 2] - t[ff + 2];
      } else {
        r0 = b[ff], r1 = b[ff + 1], r2 = b[ff + 2];
      }
      if (cmf) {
        const unsigned m = cmf[col[q]];
        if (m & 1) r0 = T(0);
        if (m & 2) r1 = T(0);
        if (m & 4) r2 = T(0);
      }
      a0 += ww * r0;
      a1 += ww * r1;
      a2 += ww * r2;
    }
    a0 = group_sum<G>(a0), a1 = group_sum<G>(a1), a2 = group_sum<G>(a2);
    if (cmc) {
      const unsigned m = cmc[c];
      if (m & 1) a0 = T(0);
      if (m & 2) a1 = T(0);
      if (m & 4) a2 = T(0);
    }
    if (sub == 0) {
      xc[3 * c] = a0;
      xc[3 * c + 1] = a1;
      xc[3 * c + 2] = a2;
    }
  }
}

// Transfers between two uniform levels (nc coarse cells per edge, 2nc fine).
// Prolongation: a fine lattice coordinate X (0..4nc) that is even sits on
// coarse node X/2; an odd X lies at a quarter point of coarse cell k = X/4,
// where the coarse Q2 basis takes the values (3/8, 3/4, -1/8) (X = 4k+1) or
// (-1/8, 3/4, 3/8) (X = 4k+3) on coarse nodes 2k, 2k+1, 2k+2.  Restriction is
// the exact transpose: coarse node C collects fine X = 2C (weight 1) and, for
// even C, 2C+-1 (3/8) and 2C+-3 (-1/8); for odd C, 2C+-1 (3/4).  Boundary
// (Dirichlet) nodes of either level carry and receive nothing.
template <typename T>
__device__ __forceinline__ int prolong_axis(int X, int mc, int (&idx)[3], T (&w)[3]) {
  if (!(X & 1)) {
    const int c = X >> 1;
    idx[0] = c, w[0] = T(1);
    return (c == 0 || c == mc - 1) ? 0 : 1;
  }
  const int base = 2 * (X >> 2);
  const bool q1 = (X & 3) == 1;
  idx[0] = base, idx[1] = base + 1, idx[2] = base + 2;
  w[0] = q1 ? T(0.375) : T(-0.125);
  w[1] = T(0.75);
  w[2] = q1 ? T(-0.125) : T(0.375);
  if (base == 0) w[0] = T(0);
  if (base + 2 == mc - 1) w[2] = T(0);
  return 3;
}

template <typename T>
__global__ void k_prolong_uniform(int nc, const T* __restrict__ xc, T* __restrict__ xf, bool add) {
  const int mc = 2 * nc + 1, mf = 4 * nc + 1;
  const int64_t nn = int64_t(mf) * mf * mf;
  // XCD-contiguous node ranges: neighbouring fine nodes read the same coarse ones
  for (int64_t v = brick::xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; v < nn;
       v += int64_t(gridDim.x) * blockDim.x) {
    const int X = int(v % mf), Y = int((v / mf) % mf), Z = int(v / (int64_t(mf) * mf));
    T a0 = T(0), a1 = T(0), a2 = T(0);
    const bool dir = X == 0 || Y == 0 || Z == 0 || X == mf - 1 || Y == mf - 1 || Z == mf - 1;
    if (!dir) {
      int ix[3], iy[3], iz[3];
      T wx[3], wy[3], wz[3];
      const int nx = prolong_axis<T>(X, mc, ix, wx), ny = prolong_axis<T>(Y, mc, iy, wy),
                nz = prolong_axis<T>(Z, mc, iz, wz);
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
          const T wzy = wz[k] * wy[j];
          const int64_t rowc = int64_t(mc) * (iy[j] + int64_t(mc) * iz[k]);
          for (int i = 0; i < nx; ++i) {
            const T ww = wzy * wx[i];
            const T* p = xc + 3 * (rowc + ix[i]);
            a0 += ww * p[0], a1 += ww * p[1], a2 += ww * p[2];
          }
        }
    }
    T* q = xf + 3 * v;
    if (add) {
      q[0] += a0, q[1] += a1, q[2] += a2;
    } else {
      q[0] = a0, q[1] = a1, q[2] = a2;
    }
  }
}

// The same prolongation, one wave per fine lattice row (Y, Z), four rows per
// workgroup, for coarse levels up to kRowMaxCoarse cells per edge: the wave
// first combines the up to 3 x 3 coarse rows its (Y, Z) touches into one
// coarse row (weights wy wz, coalesced reads along the rows) in its part of
// LDS, then forms every fine node of the row from up to 3 of its values.  The
// gather kernel above reads up to 27 coarse nodes per fine node with lanes two
// nodes apart; this one reads each coarse row once per fine row it serves.
// A wave's LDS writes and later reads are ordered by an LDS wait (its LDS
// operations complete in order), so the rows need no workgroup barrier.
constexpr int kRowMaxCoarse = 64;
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
  asm volatile("" ::: "memory");
}
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_rows(int nc, const T* __restrict__ xc, T* __restrict__ xf,
                                                      bool add) {
  __shared__ T rcs[4][3 * (2 * kRowMaxCoarse + 1)];
  const int mc = 2 * nc + 1, mf = 4 * nc + 1;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = threadIdx.x & 63;
  // XCD-contiguous row ranges: neighbouring fine rows read the same coarse rows
  const int row = 4 * int(brick::xcd_order(blockIdx.x, gridDim.x)) + w;
  if (row >= mf * mf) return;
  T* rc = rcs[w];
  const int Y = row % mf, Z = row / mf;
  T* q = xf + 3 * int64_t(mf) * row;
  if (Y == 0 || Z == 0 || Y == mf - 1 || Z == mf - 1) {   // boundary row: receives nothing
    if (!add)
      for (int i = lane; i < 3 * mf; i += 64) q[i] = T(0);
    return;
  }
  int iy[3], iz[3];
  T wy[3], wz[3];
  const int ny = prolong_axis<T>(Y, mc, iy, wy), nz = prolong_axis<T>(Z, mc, iz, wz);
  // ny, nz (1 or 3) are the wave's: each case is unrolled, so that all loads of
  // four row chunks are issued before the first is used
  auto combine = [&](auto kny, auto knz) {
    constexpr int NY = decltype(kny)::value, NZ = decltype(knz)::value;
    const T* src[NY * NZ];
    T ww[NY * NZ];
#pragma unroll
    for (int k = 0; k < NZ; ++k)
#pragma unroll
      for (int j = 0; j < NY; ++j) {
        src[j + NY * k] = xc + 3 * int64_t(mc) * (iy[j] + int64_t(mc) * iz[k]);
        ww[j + NY * k] = wz[k] * wy[j];
      }
    for (int i0 = 0; i0 < 3 * mc; i0 += 256) {
      T v[4][NY * NZ];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = min(i0 + 64 * u + lane, 3 * mc - 1);
#pragma unroll
        for (int e = 0; e < NY * NZ; ++e) v[u][e] = src[e][i];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u + lane;
        T a = T(0);
#pragma unroll
        for (int e = 0; e < NY * NZ; ++e) a += ww[e] * v[u][e];
        if (i < 3 * mc) rc[i] = a;
      }
    }
  };
  using one = std::integral_constant<int, 1>;
  using three = std::integral_constant<int, 3>;
  if (ny == 1 && nz == 1) combine(one(), one());
  else if (ny == 1) combine(one(), three());
  else if (nz == 1) combine(three(), one());
  else combine(three(), three());
  wave_lds_sync();
  for (int i0 = 0; i0 < 3 * mf; i0 += 256) {
    T old[4];
    if (add) {
#pragma unroll
      for (int u = 0; u < 4; ++u) old[u] = q[min(i0 + 64 * u + lane, 3 * mf - 1)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u + lane, X = i / 3, comp = i - 3 * X;
      T a = T(0);
      if (X > 0 && X < mf - 1) {
        int ix[3];
        T wx[3];
        const int nx = prolong_axis<T>(X, mc, ix, wx);
        for (int l = 0; l < nx; ++l) a += wx[l] * rc[3 * ix[l] + comp];
      }
      if (i < 3 * mf) q[i] = add ? old[u] + a : a;
    }
  }
}

// Restriction between uniform levels, R = P^T, as three one-axis passes
// (each a bandwidth-bound stream with coalesced neighbours) with the 1D
// weights of R: offsets -3, -1, 0, 1, 3 from the fine node 2C, weights
// (-1/8, 3/8, 1, 3/8, -1/8) for even C and (0, 3/4, 1, 3/4, 0) for odd C.
// x over the residual b - t (fine boundary nodes count 0) into s1, laid out
// [fz][fy][cx][3]; y into s2 [fz][cy][cx][3]; z into the coarse vector
// (coarse boundary nodes 0).  s1 and s2 are scratch of 3 mc mf^2 and
// 3 mc^2 mf values (mc = 2 nc + 1, mf = 4 nc + 1).
template <typename T>
__device__ __forceinline__ T restrict_w(int C, int q) {
  if (C & 1) return q == 0 || q == 4 ? T(0) : (q == 2 ? T(1) : T(0.75));
  return q == 2 ? T(1) : ((q == 1 || q == 3) ? T(0.375) : T(-0.125));
}
__device__ __forceinline__ constexpr int restrict_off(int q) { return q == 0 ? -3 : q == 1 ? -1 : q == 2 ? 0 : q == 3 ? 1 : 3; }
// one thread per output node (its 3 components)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_x(int nc, const T* __restrict__ b, const T* __restrict__ t,
                                                      T* __restrict__ s1) {
  const int mc = 2 * nc + 1, mf = 4 * nc + 1;
  const int n = mc * mf * mf;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int cx = v % mc, fy = (v / mc) % mf, fz = v / (mc * mf);
    T a0 = T(0), a1 = T(0), a2 = T(0);
    if (fy > 0 && fy < mf - 1 && fz > 0 && fz < mf - 1) {
      const int64_t row = 3 * int64_t(mf) * (fy + int64_t(mf) * fz);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const int fx = 2 * cx + restrict_off(q);
        if (fx > 0 && fx < mf - 1) {
          const int64_t f = row + 3 * fx;
          const T w = restrict_w<T>(cx, q);
          if (t) {
            a0 += w * (b[f] - t[f]), a1 += w * (b[f + 1] - t[f + 1]), a2 += w * (b[f + 2] - t[f + 2]);
          } else {
            a0 += w * b[f], a1 += w * b[f + 1], a2 += w * b[f + 2];
          }
        }
      }
    }
    T* o = s1 + 3 * int64_t(v);
    o[0] = a0, o[1] = a1, o[2] = a2;
  }
}
// The x pass, one wave per fine row (fy, fz), four rows per workgroup, for
// coarse levels up to kRowMaxCoarse cells per edge: the row's residual is
// read once, coalesced, into the wave's part of LDS, and each output
// (cx, component) sums its five values there (the one-thread-per-output form
// reads them from memory with lanes two nodes apart).  Same terms in the
// same order as k_restrict_x.
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_x_rows(int nc, const T* __restrict__ b, const T* __restrict__ t,
                                                         T* __restrict__ s1) {
  __shared__ T rs[4][3 * (4 * kRowMaxCoarse + 1)];
  const int mc = 2 * nc + 1, mf = 4 * nc + 1;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), lane = threadIdx.x & 63;
  const int row = 4 * int(brick::xcd_order(blockIdx.x, gridDim.x)) + w;   // fy + mf fz
  if (row >= mf * mf) return;
  T* r = rs[w];
  const int fy = row % mf, fz = row / mf;
  T* o = s1 + 3 * int64_t(mc) * row;
  if (fy == 0 || fz == 0 || fy == mf - 1 || fz == mf - 1) {   // boundary rows count 0
    for (int i = lane; i < 3 * mc; i += 64) o[i] = T(0);
    return;
  }
  const int64_t f0 = 3 * int64_t(mf) * row;
  // four row chunks per round, every load issued before the first is used
  for (int i0 = 0; i0 < 3 * mf; i0 += 256) {
    T vb[4], vt[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t f = f0 + min(i0 + 64 * u + lane, 3 * mf - 1);
      vb[u] = b[f];
      vt[u] = t ? t[f] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u + lane, fx = i / 3;
      if (i < 3 * mf) r[i] = (fx > 0 && fx < mf - 1) ? (t ? vb[u] - vt[u] : vb[u]) : T(0);
    }
  }
  wave_lds_sync();
  for (int i = lane; i < 3 * mc; i += 64) {
    const int cx = i / 3, comp = i - 3 * cx;
    T a = T(0);
#pragma unroll
    for (int qq = 0; qq < 5; ++qq) {
      const int fx = 2 * cx + restrict_off(qq);
      if (fx > 0 && fx < mf - 1) a += restrict_w<T>(cx, qq) * r[3 * fx + comp];
    }
    o[i] = a;
  }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_y(int nc, const T* __restrict__ s1, T* __restrict__ s2) {
  const int mc = 2 * nc + 1, mf = 4 * nc + 1;
  const int n = mc * mc * mf;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int cx = v % mc, cy = (v / mc) % mc, fz = v / (mc * mc);
    T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int fy = 2 * cy + restrict_off(q);
      if (fy >= 0 && fy < mf) {
        const T* p = s1 + 3 * (cx + int64_t(mc) * (fy + int64_t(mf) * fz));
        const T w = restrict_w<T>(cy, q);
        a0 += w * p[0], a1 += w * p[1], a2 += w * p[2];
      }
    }
    T* o = s2 + 3 * int64_t(v);
    o[0] = a0, o[1] = a1, o[2] = a2;
  }
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_z(int nc, const T* __restrict__ s2, T* __restrict__ xc) {
  const int mc = 2 * nc + 1, mf = 4 * nc + 1;
  const int n = mc * mc * mc;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int cx = v % mc, cy = (v / mc) % mc, cz = v / (mc * mc);
    T a0 = T(0), a1 = T(0), a2 = T(0);
    if (cx > 0 && cx < mc - 1 && cy > 0 && cy < mc - 1 && cz > 0 && cz < mc - 1) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const int fz = 2 * cz + restrict_off(q);
        if (fz >= 0 && fz < mf) {
          const T* p = s2 + 3 * (cx + int64_t(mc) * (cy + int64_t(mc) * fz));
          const T w = restrict_w<T>(cz, q);
          a0 += w * p[0], a1 += w * p[1], a2 += w * p[2];
        }
      }
    }
    T* o = xc + 3 * int64_t(v);
    o[0] = a0, o[1] = a1, o[2] = a2;
  }
}

// ------------------------------------------------------------- coarse
// the level-1 mesh (2^3 cells) has 125 Q2 nodes: at most 375 free dofs (81
// under u = 0, 225 under u . n = 0)
constexpr int kCoarseMaxFree = 375;
template <typename T>
__global__ __launch_bounds__(128) void k_coarse(const T* __restrict__ Ainv, const int32_t* __restrict__ fd,
                                                int nfree, int n, const T* __restrict__ b, T* __restrict__ x) {
  __shared__ T bs[kCoarseMaxFree];
  for (int i = threadIdx.x; i < nfree; i += blockDim.x) bs[i] = b[fd[i]];
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = b[i];
  __syncthreads();
  for (int r = threadIdx.x; r < nfree; r += blockDim.x) {
    T acc = T(0);
    for (int j = 0; j < nfree; ++j) acc += Ainv[r * nfree + j] * bs[j];
    x[fd[r]] = acc;
  }
}

// ------------------------------------------------------------- the 4^3 level
// One V-cycle on the uniform 4^3 level (9^3 nodes, 64 cells) together with the
// coarse solve of the 2^3 level below it, in one workgroup.  The level's
// vectors (x, A x, b, the Chebyshev direction d, the inverse diagonal) live
// in LDS, and the steps of the cycle are separated by workgroup barriers
// instead of the ~22 kernel boundaries the level takes otherwise, each of
// which costs more than the level's arithmetic.  Every step computes what its
// kernel computes (some sums in another order): the Chebyshev
// updates of k_chebx_init0 / k_chebx_step, the operator of k_vmult_uniform3
// (three threads per cell; its sums go into LDS), the passes of
// k_restrict_x_rows / k_restrict_y / k_restrict_z, k_coarse (a row's sum in
// three parts) and the prolongation (here by axes, z, y, x).  Pre-smoothing
// starts from x = 0; post-smoothing's first step has alpha = 0; steps 1-3 of
// both take (alpha_k, beta_k).
template <typename T>
struct TailCoef {
  T it0, alpha[4], beta[4];
};
constexpr int kTailN = 4, kTailFree = 81;   // free dofs of the 2^3 level under u = 0
template <typename T>
__global__ __launch_bounds__(256) void k_vcycle_tail(const T* __restrict__ mu, const T* __restrict__ minv,
                                                     const T* __restrict__ Ainv, const int32_t* __restrict__ fd,
                                                     TailCoef<T> cf, const T* __restrict__ b, T* __restrict__ x) {
  constexpr int n = kTailN, m = 2 * n + 1, NV = 3 * m * m * m, KV = (NV + 255) / 256;
  constexpr int mc = n + 1, mf = m, NC = 3 * mc * mc * mc;
  __shared__ T xs[NV], ts[NV], bs[NV], ds[NV], ms[NV];
  __shared__ T wsh[3][27][64];
  __shared__ T s1[3 * mc * mf * mf], s2[3 * mc * mc * mf], bc[NC], xc[NC], bf[kTailFree], part[3 * kTailFree];
  const int tid = threadIdx.x;
  // this thread's entries tid + 256 k: in range (bit k of `live`) and on a
  // boundary node (`fixed`).  Wherever x changes, ts is set to x on the
  // fixed entries and 0 elsewhere, the output the operator then adds to
  // (identity rows), as the smoother's kernels prepare it.
  unsigned live = 0, fixed = 0;
#pragma unroll
  for (int k = 0; k < KV; ++k) {
    const int i = tid + 256 * k, v = i / 3, X = v % m, Y = (v / m) % m, Z = v / (m * m);
    if (i < NV) live |= 1u << k;
    if (i < NV && (X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1)) fixed |= 1u << k;
  }
  auto each = [&](auto f) {
#pragma unroll
    for (int k = 0; k < KV; ++k)
      if ((live >> k) & 1) f(tid + 256 * k, ((fixed >> k) & 1) != 0);
  };
  each([&](int i, bool) { bs[i] = b[i], ms[i] = minv[i]; });
  // the operator's thread: cell `cell`, output component c (waves 0-2)
  const bool opt = tid < 192;
  const int c = tid >> 6, cell = tid & 63;
  const UniformCell uc(n, cell);
  const T mu_h = opt ? mu[cell] / T(n) : T(0);
  __syncthreads();
  auto apply = [&]() {   // ts += the cells' sums: ts = A xs
    T w[27];
    if (opt) {
#pragma unroll
      for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int yy = 0; yy < 3; ++yy)
#pragma unroll
          for (int xx = 0; xx < 3; ++xx) {
            const int32_t sl = uc.slot(xx, yy, z);
            const T v = xs[3 * max(sl, 0) + c];   // every read issued, the Dirichlet ones dropped
            w[xx + 3 * yy + 9 * z] = sl >= 0 ? v : T(0);
          }
      cellop::interp_all(w);
#pragma unroll
      for (int a = 0; a < 27; ++a) wsh[c][a][cell] = w[a];
    }
    __syncthreads();
    if (opt) {
      T W[3][27];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int a = 0; a < 27; ++a) W[cc][a] = wsh[cc][a][cell];
      if (c == 0) cellop::apply_cell_row<0>(W, w, mu_h);
      else if (c == 1) cellop::apply_cell_row<1>(W, w, mu_h);
      else cellop::apply_cell_row<2>(W, w, mu_h);
      cellop::interp_all_t(w);
      if constexpr (sizeof(T) == 8) {   // FP64: LDS atomics (the ordered form below spills here)
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
          for (int yy = 0; yy < 3; ++yy)
#pragma unroll
            for (int xx = 0; xx < 3; ++xx) {
              const int32_t sl = uc.slot(xx, yy, z);
              if (sl >= 0) atomicAdd(&ts[3 * sl + c], w[xx + 3 * yy + 9 * z]);
            }
      } else {
        // FP32: the 64 cells of a wave add into ts without atomics (LDS float
        // atomics made the whole cycle 73 instead of 56 us): local nodes in
        // classes (0-1 | 2 per axis), within which no two (cell, local node)
        // pairs share a node, one class after the other (a wave's LDS
        // operations complete in order)
#pragma unroll
        for (int cls = 0; cls < 8; ++cls) {
          const int a0 = (cls & 1) ? 2 : 0, a1 = (cls & 1) ? 3 : 2;
          const int b0 = (cls & 2) ? 2 : 0, b1 = (cls & 2) ? 3 : 2;
          const int z0 = (cls & 4) ? 2 : 0, z1 = (cls & 4) ? 3 : 2;
          T old[8];
#pragma unroll
          for (int z = z0; z < z1; ++z)
#pragma unroll
            for (int yy = b0; yy < b1; ++yy)
#pragma unroll
              for (int xx = a0; xx < a1; ++xx)
                old[(xx - a0) + 2 * (yy - b0) + 4 * (z - z0)] = ts[3 * max(uc.slot(xx, yy, z), 0) + c];
#pragma unroll
          for (int z = z0; z < z1; ++z)
#pragma unroll
            for (int yy = b0; yy < b1; ++yy)
#pragma unroll
              for (int xx = a0; xx < a1; ++xx) {
                const int32_t sl = uc.slot(xx, yy, z);
                if (sl >= 0) ts[3 * sl + c] = old[(xx - a0) + 2 * (yy - b0) + 4 * (z - z0)] + w[xx + 3 * yy + 9 * z];
              }
          wave_lds_sync();
        }
      }
    }
    __syncthreads();
  };
  auto step = [&](T alpha, T beta) {
    each([&](int i, bool fx) {
      const T ri = bs[i] - ts[i];
      const T di = (alpha != T(0) ? alpha * ds[i] : T(0)) + beta * ms[i] * ri;
      const T xi = xs[i] + di;
      ds[i] = di;
      xs[i] = xi;
      ts[i] = fx ? xi : T(0);
    });
    __syncthreads();
  };
  // the coarse correction: residual restricted, coarse solve, prolongation
  auto correct = [&]() {
    // R (b - A x): x, y and z passes
    for (int v = tid; v < 3 * mc * mf * mf; v += 256) {
      const int comp = v % 3, o = v / 3, cx = o % mc, fy = (o / mc) % mf, fz = o / (mc * mf);
      T a = T(0);
      if (fy > 0 && fy < mf - 1 && fz > 0 && fz < mf - 1) {
#pragma unroll
        for (int qq = 0; qq < 5; ++qq) {
          const int fx = 2 * cx + restrict_off(qq);
          if (fx > 0 && fx < mf - 1) {
            const int f = 3 * (fx + mf * (fy + mf * fz)) + comp;
            a += restrict_w<T>(cx, qq) * (bs[f] - ts[f]);
          }
        }
      }
      s1[v] = a;
    }
    __syncthreads();
    for (int v = tid; v < 3 * mc * mc * mf; v += 256) {
      const int comp = v % 3, o = v / 3, cx = o % mc, cy = (o / mc) % mc, fz = o / (mc * mc);
      T a = T(0);
#pragma unroll
      for (int qq = 0; qq < 5; ++qq) {
        const int fy = 2 * cy + restrict_off(qq);
        if (fy >= 0 && fy < mf) a += restrict_w<T>(cy, qq) * s1[3 * (cx + mc * (fy + mf * fz)) + comp];
      }
      s2[v] = a;
    }
    __syncthreads();
    for (int v = tid; v < NC; v += 256) {
      const int comp = v % 3, o = v / 3, cx = o % mc, cy = (o / mc) % mc, cz = o / (mc * mc);
      T a = T(0);
      if (cx > 0 && cx < mc - 1 && cy > 0 && cy < mc - 1 && cz > 0 && cz < mc - 1) {
#pragma unroll
        for (int qq = 0; qq < 5; ++qq) {
          const int fz = 2 * cz + restrict_off(qq);
          if (fz >= 0 && fz < mf) a += restrict_w<T>(cz, qq) * s2[3 * (cx + mc * (cy + mc * fz)) + comp];
        }
      }
      bc[v] = a;
    }
    __syncthreads();
    // coarse solve on the free dofs (the others keep b): three threads per
    // row of Ainv, each summing a third of its columns (all loads issued
    // first), then the row's first thread adds the three sums
    for (int i = tid; i < kTailFree; i += 256) bf[i] = bc[fd[i]];
    for (int i = tid; i < NC; i += 256) xc[i] = bc[i];
    __syncthreads();
    {
      constexpr int JC = kTailFree / 3;
      const int r = tid % kTailFree, q = tid / kTailFree;
      if (tid < 3 * kTailFree) {
        T v[JC];
#pragma unroll
        for (int j = 0; j < JC; ++j) v[j] = Ainv[r * kTailFree + q * JC + j];
        T a = T(0);
#pragma unroll
        for (int j = 0; j < JC; ++j) a += v[j] * bf[q * JC + j];
        part[q * kTailFree + r] = a;
      }
      __syncthreads();
      if (tid < kTailFree) xc[fd[tid]] = (part[tid] + part[kTailFree + tid]) + part[2 * kTailFree + tid];
    }
    __syncthreads();
    // x += P xc by axes: z (into s2 [Z][cy][cx]), y (into s1 [Z][Y][cx]), then
    // x into the fine entries (1D weights of prolong_axis; the fine boundary
    // receives nothing)
    for (int v = tid; v < 3 * mc * mc * mf; v += 256) {
      const int comp = v % 3, o = v / 3, cx = o % mc, cy = (o / mc) % mc, Z = o / (mc * mc);
      int id[3];
      T wt[3];
      const int nz = prolong_axis<T>(Z, mc, id, wt);
      T a = T(0);
      for (int k = 0; k < nz; ++k) a += wt[k] * xc[3 * (cx + mc * (cy + mc * id[k])) + comp];
      s2[v] = a;
    }
    __syncthreads();
    for (int v = tid; v < 3 * mc * mf * mf; v += 256) {
      const int comp = v % 3, o = v / 3, cx = o % mc, Y = (o / mc) % mf, Z = o / (mc * mf);
      int id[3];
      T wt[3];
      const int ny = prolong_axis<T>(Y, mc, id, wt);
      T a = T(0);
      for (int j = 0; j < ny; ++j) a += wt[j] * s2[3 * (cx + mc * (id[j] + mc * Z)) + comp];
      s1[v] = a;
    }
    __syncthreads();
    each([&](int i, bool fx) {
      if (!fx) {
        const int comp = i % 3, v = i / 3, X = v % m, YZ = v / m;
        int id[3];
        T wt[3];
        const int nx = prolong_axis<T>(X, mc, id, wt);
        T a = T(0);
        for (int l = 0; l < nx; ++l) a += wt[l] * s1[3 * (id[l] + mc * YZ) + comp];
        xs[i] = xs[i] + a;
      }
      ts[i] = fx ? xs[i] : T(0);
    });
    __syncthreads();
  };
  // pre-smoothing from zero
  each([&](int i, bool fx) {
    const T di = ms[i] * bs[i] * cf.it0;
    ds[i] = di;
    xs[i] = di;
    ts[i] = fx ? di : T(0);
  });
  __syncthreads();
  // the cycle's eight operator applications, one copy of their code (the
  // unrolled cycle overflows the instruction cache): p = 0-2 pre-smoothing
  // steps 1-3, p = 3 the residual and the coarse correction, p = 4-7
  // post-smoothing steps 0-3
#pragma nounroll
  for (int p = 0; p < 8; ++p) {
    apply();
    if (p == 3) {
      correct();
    } else if (p == 4) {
      step(T(0), cf.it0);
    } else {
      const int k = p < 3 ? p + 1 : p - 4;
      step(k == 1 ? cf.alpha[1] : k == 2 ? cf.alpha[2] : cf.alpha[3],
           k == 1 ? cf.beta[1] : k == 2 ? cf.beta[2] : cf.beta[3]);
    }
  }
  each([&](int i, bool) { x[i] = xs[i]; });
}

// ------------------------------------------------------------- viscosity
__global__ void k_harmonic(int64_t ncell, const double* __restrict__ mq, double* __restrict__ mu) {
  const double w1[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < ncell;
       c += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < 3; ++z)
      for (int y = 0; y < 3; ++y)
        for (int x = 0; x < 3; ++x) s += w1[x] * w1[y] * w1[z] / mq[27 * c + x + 3 * y + 9 * z];
    mu[c] = 1.0 / s;
  }
}

__global__ void k_restrict_mu(int64_t ncell, const int32_t* __restrict__ src, const double* __restrict__ mf,
                              double* __restrict__ mc) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < ncell;
       c += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    int k = 0;
    for (int q = 0; q < 8; ++q) {
      const int32_t f = src[8 * c + q];
      if (f >= 0) s += mf[f], ++k;
    }
    mc[c] = s / double(k);
  }
}

__global__ void k_to_float(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = float(a[i]);
}
__global__ void k_to_double(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = double(a[i]);
}

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sm[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) r += sm[i];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kBlock) void k_dot_partial(int64_t n, const double* __restrict__ a,
                                                        const double* __restrict__ b, double* __restrict__ part) {
  double v = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    v += a[i] * b[i];
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(int np, const double* __restrict__ part,
                                                         double* __restrict__ out) {
  // block j sums part[j*np .. j*np + np)
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[int64_t(blockIdx.x) * np + i];
  v = block_sum(v);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

__global__ void k_mupdate(int64_t n, int nv, const double* __restrict__ V, int64_t ldv, const double* __restrict__ h,
                          double* __restrict__ w) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    double acc = w[i];
    for (int j = 0; j < nv; ++j) acc -= h[j] * V[int64_t(j) * ldv + i];
    w[i] = acc;
  }
}

// w <- w - sum_{j < nv} h_j V_j, fused with the block partials that the next
// Gram-Schmidt step needs of the new w: part[j * gridDim.x + b] = V_j . w for
// j < nv (DOTS) and, in the last row (j = nv, or 0 without DOTS), w . w.  V is
// read once: the nv values of an element stay in registers (nv <= NV).
template <int NV, bool DOTS>
__global__ __launch_bounds__(kBlock) void k_mupdate_dots(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                         const double* __restrict__ h, double* __restrict__ w,
                                                         double* __restrict__ part) {
  constexpr int NA = DOTS ? NV + 1 : 1;
  double acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    double v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = j < nv ? V[int64_t(j) * ldv + i] : 0.0;
    double wi = w[i];
#pragma unroll
    for (int j = 0; j < NV; ++j)
      if (j < nv) wi -= h[j] * v[j];
    w[i] = wi;
    if constexpr (DOTS) {
#pragma unroll
      for (int j = 0; j < NV; ++j)
        if (j < nv) acc[j] += v[j] * wi;
    }
    acc[NA - 1] += wi * wi;
  }
  // one wave reduction per row, one barrier, then thread r sums row r
  __shared__ double sm[kBlock / 64][NA];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    if (a < nv || a == NA - 1) {
      double val = acc[a];
      for (int o = 32; o > 0; o >>= 1) val += __shfl_down(val, o, 64);
      if (lane == 0) sm[wid][a] = val;
    }
  }
  __syncthreads();
  const int rows = DOTS ? nv + 1 : 1;
  const int r = threadIdx.x;
  if (r < rows) {
    const int a = r < rows - 1 ? r : NA - 1;
    double sum = 0.0;
    for (int k = 0; k < int(blockDim.x >> 6); ++k) sum += sm[k][a];
    part[int64_t(r) * gridDim.x + blockIdx.x] = sum;
  }
}

// Gram-Schmidt over tiles of 64 entries: wave v of a block takes the basis
// vectors j = j0 + v + 4k (k < JPW), lane l the entry i0 + l of each tile,
// so that every V_j is read once and the tile of w once per block (its four
// waves share it in L1); the per-vector partial sums stay in registers until
// the end.  (One block per (vector, block) pair read w once per vector; one
// thread per entry holding all nv values ran at one wave per SIMD.)
template <int JPW>
__device__ __forceinline__ void tile_rows_out(double (&acc)[JPW + 1], int j0, int nv, bool norm_row, int norm_at,
                                              double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= JPW; ++k) {
    double val = acc[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) val += __shfl_down(val, o, 64);
    if (lane == 0) {
      if (k < JPW) {
        const int j = j0 + wv + 4 * k;
        if (j < nv) part[int64_t(j) * gridDim.x + blockIdx.x] = val;
      } else if (norm_row && wv == 0) {
        part[int64_t(norm_at) * gridDim.x + blockIdx.x] = val;
      }
    }
  }
}

// part[j nb + b] = partial of V_j . w for j0 <= j < min(nv, j0 + 4 JPW); with
// norm, row nv holds the partials of w . w
template <int JPW>
__global__ __launch_bounds__(256) void k_mdot_tiles(int64_t n, int j0, int nv, const double* __restrict__ V,
                                                    int64_t ldv, const double* __restrict__ w, bool norm,
                                                    double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[JPW + 1];
#pragma unroll
  for (int k = 0; k <= JPW; ++k) acc[k] = 0.0;
  for (int64_t t0 = int64_t(blockIdx.x) * 64; t0 < n; t0 += int64_t(gridDim.x) * 64) {
    const int64_t i = t0 + lane;
    const bool ok = i < n;
    double v[JPW];
#pragma unroll
    for (int k = 0; k < JPW; ++k) {
      const int j = j0 + wv + 4 * k;
      v[k] = ok && j < nv ? V[int64_t(j) * ldv + i] : 0.0;
    }
    const double wi = ok ? w[i] : 0.0;
#pragma unroll
    for (int k = 0; k < JPW; ++k) acc[k] += v[k] * wi;
    acc[JPW] += wi * wi;
  }
  tile_rows_out<JPW>(acc, j0, nv, norm, nv, part);
}

// w <- w - sum_{j < nv} h_j V_j (nv <= 4 JPW), V read once: the waves' partial
// sums meet in LDS; then, with DOTS, the partials of V_j . w (rows j < nv) and
// of w . w (row nv; row 0 without DOTS) of the new w
template <int JPW, bool DOTS>
__global__ __launch_bounds__(256) void k_mupdate_tiles(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                       const double* __restrict__ h, double* __restrict__ w,
                                                       double* __restrict__ part) {
  __shared__ double ps[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double hk[JPW], acc[JPW + 1];
#pragma unroll
  for (int k = 0; k < JPW; ++k) {
    const int j = wv + 4 * k;
    hk[k] = j < nv ? h[j] : 0.0;
  }
#pragma unroll
  for (int k = 0; k <= JPW; ++k) acc[k] = 0.0;
  for (int64_t t0 = int64_t(blockIdx.x) * 64; t0 < n; t0 += int64_t(gridDim.x) * 64) {
    const int64_t i = t0 + lane;
    const bool ok = i < n;
    double v[JPW];
#pragma unroll
    for (int k = 0; k < JPW; ++k) {
      const int j = wv + 4 * k;
      v[k] = ok && j < nv ? V[int64_t(j) * ldv + i] : 0.0;
    }
    const double wi = ok ? w[i] : 0.0;
    double pv = 0.0;
#pragma unroll
    for (int k = 0; k < JPW; ++k) pv += hk[k] * v[k];
    ps[wv][lane] = pv;
    __syncthreads();
    const double wn = wi - (((ps[0][lane] + ps[1][lane]) + ps[2][lane]) + ps[3][lane]);
    if (wv == 0 && ok) w[i] = wn;
    if constexpr (DOTS) {
#pragma unroll
      for (int k = 0; k < JPW; ++k) acc[k] += v[k] * wn;
    }
    acc[JPW] += wn * wn;
    __syncthreads();   // ps is refilled by the next tile
  }
  if constexpr (DOTS) {
    tile_rows_out<JPW>(acc, 0, nv, true, nv, part);
  } else {
#pragma unroll
    for (int k = 0; k < JPW; ++k) acc[k] = 0.0;
    tile_rows_out<JPW>(acc, 0, 0, true, 0, part);
  }
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];   // b = 0: y is not read (may be uninitialised)
}
__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = a * x[i];
}
__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = v;
}
__global__ void k_fill_f(int64_t n, float v, float* __restrict__ y) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = v;
}
__global__ void k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = a[i] * b[i];
}

// ------------------------------------------------------------- pressure
__device__ __forceinline__ int32_t vslot(const DevLevel& L, int64_t c, int a) {
  if (L.uniform) {
    const UniformCell cell(L.n_edge, c);
    return cell.slot(a % 3, (a / 3) % 3, a / 9);
  }
  return L.slots[27 * c + a];
}

__device__ __forceinline__ double cell_h(const DevLevel& L, int64_t c) {
  return L.uniform ? 1.0 / double(L.n_edge) : ldexp(1.0, -int(L.clev[c]));
}

__device__ __forceinline__ double pgather(const DevPressure& P, int32_t s, const double* p) {
  if (s >= 0) return p[s];
  const int64_t h = -int64_t(s) - 2;
  double v = 0.0;
  for (int64_t q = P.hptr[h]; q < P.hptr[h + 1]; ++q) v += P.hw[q] * p[P.hmaster[q]];
  return v;
}

__device__ __forceinline__ void pscatter(const DevPressure& P, int32_t s, double v, double* p) {
  if (s >= 0) {
    atomicAdd(&p[s], v);
    return;
  }
  const int64_t h = -int64_t(s) - 2;
  for (int64_t q = P.hptr[h]; q < P.hptr[h + 1]; ++q) atomicAdd(&p[P.hmaster[q]], P.hw[q] * v);
}

// a hanging node's master component that the no-normal-flux condition fixes
__device__ __forceinline__ bool master_fixed(const DevLevel& L, int32_t m, int comp) {
  return L.noflux && ((L.cmask[m] >> comp) & 1);
}

__device__ __forceinline__ double vgather1(const DevLevel& L, int32_t s, int comp, const double* u) {
  if (s >= 0) return slot_fixed(s, comp) ? 0.0 : u[3 * int64_t(slot_node(s)) + comp];
  if (s == -1) return 0.0;
  const int64_t h = -int64_t(s) - 2;
  double v = 0.0;
  for (int64_t q = L.hptr[h]; q < L.hptr[h + 1]; ++q)
    if (!master_fixed(L, L.hmaster[q], comp)) v += L.hw_d[q] * u[3 * int64_t(L.hmaster[q]) + comp];
  return v;
}

__device__ __forceinline__ void vscatter1(const DevLevel& L, int32_t s, int comp, double v, double* u) {
  if (s >= 0) {
    if (!slot_fixed(s, comp)) atomicAdd(&u[3 * int64_t(slot_node(s)) + comp], v);
  } else if (s < -1) {
    const int64_t h = -int64_t(s) - 2;
    for (int64_t q = L.hptr[h]; q < L.hptr[h + 1]; ++q)
      if (!master_fixed(L, L.hmaster[q], comp)) atomicAdd(&u[3 * int64_t(L.hmaster[q]) + comp], L.hw_d[q] * v);
  }
}

__global__ __launch_bounds__(kCellBlock) void k_div(DevLevel L, DevPressure P, const int32_t* __restrict__ cells,
                                                    int64_t ncells, const double* __restrict__ u,
                                                    double* __restrict__ po) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= ncells) return;
  const int64_t c = cells ? cells[t] : t;
  const double h = cell_h(L, c);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 27; ++a) {
    const int32_t s = vslot(L, c, a);
    for (int comp = 0; comp < 3; ++comp) {
      const double v = vgather1(L, s, comp, u);
      if (v == 0.0) continue;
      for (int i = 0; i < 8; ++i) acc[i] += c_bhat[i * 81 + 3 * a + comp] * v;
    }
  }
  for (int i = 0; i < 8; ++i) pscatter(P, P.pslots[8 * c + i], h * h * acc[i], po);
}

__global__ __launch_bounds__(kCellBlock) void k_grad_add(DevLevel L, DevPressure P,
                                                         const int32_t* __restrict__ cells, int64_t ncells,
                                                         const double* __restrict__ p, double* __restrict__ uo) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= ncells) return;
  const int64_t c = cells ? cells[t] : t;
  const double h = cell_h(L, c);
  double pl[8];
  for (int i = 0; i < 8; ++i) pl[i] = h * h * pgather(P, P.pslots[8 * c + i], p);
  for (int a = 0; a < 27; ++a) {
    const int32_t s = vslot(L, c, a);
    if (s == -1) continue;
    for (int comp = 0; comp < 3; ++comp) {
      double v = 0.0;
      for (int i = 0; i < 8; ++i) v += c_bhat[i * 81 + 3 * a + comp] * pl[i];
      vscatter1(L, s, comp, v, uo);
    }
  }
}

__global__ __launch_bounds__(kCellBlock) void k_pmass(DevLevel L, DevPressure P, const int32_t* __restrict__ cells,
                                                      int64_t ncells, const double* __restrict__ p,
                                                      double* __restrict__ po, const double* __restrict__ gate) {
  if (gate && *gate != 0.0) return;
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= ncells) return;
  const int64_t c = cells ? cells[t] : t;
  const double h = cell_h(L, c);
  const double s = h * h * h / L.mu_d[c];
  double pl[8];
  for (int i = 0; i < 8; ++i) pl[i] = pgather(P, P.pslots[8 * c + i], p);
  for (int i = 0; i < 8; ++i) {
    double v = 0.0;
    for (int j = 0; j < 8; ++j) v += c_mhat[i * 8 + j] * pl[j];
    pscatter(P, P.pslots[8 * c + i], s * v, po);
  }
}

// B^T p (added into uo) and B u on the blocks of the leaf (FP64): the
// velocity side goes through the block's LDS node box exactly as in the
// operator kernel (hanging points resolved in the box, class-ordered
// accumulation, atomics only on block faces); the 8 pressure values of a
// cell are gathered (or scattered) directly.
template <int B>
__global__ __launch_bounds__(64) void k_grad_blocks(DevBlocks blk, DevLevel L, DevPressure P,
                                                    const double* __restrict__ p, double* __restrict__ uo,
                                                    double* __restrict__ fslot) {
  constexpr int NC = B * B * B, NB = 64 / NC;
  constexpr int E = 2 * B + 1, PP = E * E * E, W = 3 * PP;
  constexpr int KP = (NB * PP + 63) / 64;
  __shared__ double buf[NB * W];
  const int lane = threadIdx.x;
  const int64_t blk0 = int64_t(blockIdx.x) * NB;
  const int nb = int(std::min<int64_t>(NB, blk.n - blk0));
  const int np = nb * PP;
  auto lds_of = [&](int bl, int q) {
    const int px = q % E, py = (q / E) % E, pz = q / (E * E);
    return bl * W + bsplit<B>(px) + E * bsplit<B>(py) + E * E * bsplit<B>(pz);
  };
  for (int e = lane; e < NB * W; e += 64) buf[e] = 0.0;
  const int bl = lane / NC, lc = lane - bl * NC;
  const int ca = lc % B, cb = (lc / B) % B, cc = lc / (B * B);
  double pl[8];
  if (bl < nb) {
    const int64_t c = blk.cells[(blk0 + bl) * NC + lc];
    const double h = cell_h(L, c);
#pragma unroll
    for (int i = 0; i < 8; ++i) pl[i] = h * h * pgather(P, P.pslots[8 * c + i], p);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) pl[i] = 0.0;
  }
  __syncthreads();
  const int base = bl * W;
#pragma unroll
  for (int cls = 0; cls < 8; ++cls) {
    const int ac = cls & 1, bc = (cls >> 1) & 1, zc = cls >> 2;
#pragma unroll
    for (int z = zc ? 2 : 0; z < (zc ? 3 : 2); ++z)
#pragma unroll
      for (int yy = bc ? 2 : 0; yy < (bc ? 3 : 2); ++yy)
#pragma unroll
        for (int xx = ac ? 2 : 0; xx < (ac ? 3 : 2); ++xx) {
          const int a = xx + 3 * yy + 9 * z;
          const int off = base + bsplit<B>(2 * ca + xx) + E * bsplit<B>(2 * cb + yy) + E * E * bsplit<B>(2 * cc + z);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            double v = 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) v += c_bhat[i * 81 + 3 * a + q] * pl[i];
            buf[off + q * PP] += v;
          }
        }
    __syncthreads();
  }
  const int h0 = blk.hoff[blk0], h1 = blk.hoff[blk0 + nb];
  for (int e = h0 + lane; e < h1; e += 64) {
    const int32_t en = blk.hent[e];
    const int q = en & 1023, qm = (en >> 10) & 1023, b2 = en >> 20;
    const double w = blk.hw_d[e];
    const int o = lds_of(b2, q), om = lds_of(b2, qm);
#pragma unroll
    for (int k = 0; k < 3; ++k) atomicAdd(&buf[om + k * PP], w * buf[o + k * PP]);
  }
  __syncthreads();
  int32_t sl[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int pa = lane + 64 * k;
    sl[k] = pa < np ? blk.slots[blk0 * PP + pa] : -1;
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (sl[k] < 0) continue;
    const int pa = lane + 64 * k, q = pa % PP;
    const int o = lds_of(pa / PP, q);
    // components fixed by the no-normal-flux condition receive nothing
    const double v0 = slot_fixed(sl[k], 0) ? 0.0 : buf[o];
    const double v1 = slot_fixed(sl[k], 1) ? 0.0 : buf[o + PP];
    const double v2 = slot_fixed(sl[k], 2) ? 0.0 : buf[o + 2 * PP];
    const int px = q % E, py = (q / E) % E, pz = q / (E * E);
    const bool inner = px > 0 && px < E - 1 && py > 0 && py < E - 1 && pz > 0 && pz < E - 1;
    double* yp = uo + 3 * int64_t(slot_node(sl[k]));
    if (inner) {
      yp[0] += v0, yp[1] += v1, yp[2] += v2;
    } else {   // shared face point: the block's slot, added by the face gather
      double* fs = fslot + 3 * ((blk0 + pa / PP) * PP + q);
      fs[0] = v0, fs[1] = v1, fs[2] = v2;
    }
  }
}

// B^T p added into uo on a uniform leaf, gathered per velocity node (no
// atomics), by sum factorisation: with B_qj = -int psi_q div phi_j and both
// bases tensor products, the coupling of Q2 node X and Q1 node P is, per
// axis, the 1D mass int psi phi (M1 = [[1/6, 1/3, 0], [0, 1/3, 1/6]]) or,
// along the velocity component, the 1D derivative coupling int psi phi'
// (G1 = [[-5/6, 2/3, 1/6], [-1/6, -2/3, 5/6]]).  Assembled over the cells
// around a node, an odd coordinate X = 2i+1 couples to P = i, i+1 with mass
// (1/3, 1/3) and derivative (2/3, -2/3); an even X = 2i to P = i-1, i, i+1
// with mass (0, 1/3, 0) and derivative (1/6, 0, -1/6).  The node reads the
// <= 27 pressure values of its 3x3x3 lattice window and contracts them axis
// by axis; the cell size enters as h^2.
// A workgroup takes a 16 x 4 x 4 tile of velocity nodes and first stages the
// pressure values of the lattice window its nodes read (11 x 5 x 5 points,
// 0 off the lattice) in LDS.
// FROM: uo = src + B^T p (every node written; src may not alias uo),
// otherwise uo += B^T p.
constexpr int kGradTX = 16, kGradTY = 4, kGradTZ = 4;
template <bool FROM>
__global__ __launch_bounds__(kGradTX * kGradTY * kGradTZ) void k_grad_uniform(int64_t n, DevPressure P,
                                                                            const double* __restrict__ p,
                                                                            const double* __restrict__ src,
                                                                            double* __restrict__ uo) {
  constexpr int NT = kGradTX * kGradTY * kGradTZ;
  constexpr int WX = kGradTX / 2 + 3, WY = kGradTY / 2 + 3, WZ = kGradTZ / 2 + 3;
  __shared__ double sp[WZ * WY * WX];
  const int64_t m = 2 * n + 1, np1 = n + 1;
  const int64_t ntx = (m + kGradTX - 1) / kGradTX, nty = (m + kGradTY - 1) / kGradTY;
  const int64_t tile = blockIdx.x;
  const int64_t X0 = (tile % ntx) * kGradTX, Y0 = ((tile / ntx) % nty) * kGradTY, Z0 = (tile / (ntx * nty)) * kGradTZ;
  // the first window point of each axis: the lowest P0 = (X - 1) / 2 of the
  // tile's interior nodes
  const int64_t q0[3] = {X0 > 0 ? (X0 - 1) / 2 : 0, Y0 > 0 ? (Y0 - 1) / 2 : 0, Z0 > 0 ? (Z0 - 1) / 2 : 0};
  for (int e = threadIdx.x; e < WX * WY * WZ; e += NT) {
    const int64_t px = q0[0] + e % WX, py = q0[1] + (e / WX) % WY, pz = q0[2] + e / (WX * WY);
    sp[e] = px < np1 && py < np1 && pz < np1 ? p[P.plat[px + np1 * (py + np1 * pz)]] : 0.0;
  }
  __syncthreads();
  const double h2 = 1.0 / double(n * n);
  const int64_t X[3] = {X0 + int(threadIdx.x) % kGradTX, Y0 + (int(threadIdx.x) / kGradTX) % kGradTY,
                        Z0 + int(threadIdx.x) / (kGradTX * kGradTY)};
  if (X[0] >= m || X[1] >= m || X[2] >= m) return;
  const int64_t v = X[0] + m * (X[1] + m * X[2]);
  if (X[0] == 0 || X[1] == 0 || X[2] == 0 || X[0] == m - 1 || X[1] == m - 1 || X[2] == m - 1) {
    if (FROM) uo[3 * v] = src[3 * v], uo[3 * v + 1] = src[3 * v + 1], uo[3 * v + 2] = src[3 * v + 2];
    return;
  }
  int o[3];   // window offset of the node's first pressure point per axis
  double wm[3][3], wg[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    o[d] = int((X[d] - 1) / 2 - q0[d]);
    if (X[d] & 1) {
      wm[d][0] = 1.0 / 3.0, wm[d][1] = 1.0 / 3.0, wm[d][2] = 0.0;
      wg[d][0] = 2.0 / 3.0, wg[d][1] = -2.0 / 3.0, wg[d][2] = 0.0;
    } else {
      wm[d][0] = 0.0, wm[d][1] = 1.0 / 3.0, wm[d][2] = 0.0;
      wg[d][0] = 1.0 / 6.0, wg[d][1] = 0.0, wg[d][2] = -1.0 / 6.0;
    }
  }
  double zm[3][3], zg[3][3];   // contracted along z with mass / derivative weights
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) zm[b][a] = zg[b][a] = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double val = sp[(o[2] + c) * (WY * WX) + (o[1] + b) * WX + o[0] + a];
        zm[b][a] += wm[2][c] * val;
        zg[b][a] += wg[2][c] * val;
      }
  double ymm[3], ygm[3], ymg[3];   // then along y: (y, z) weights mass/mass, deriv/mass, mass/deriv
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ymm[a] = wm[1][0] * zm[0][a] + wm[1][1] * zm[1][a] + wm[1][2] * zm[2][a];
    ygm[a] = wg[1][0] * zm[0][a] + wg[1][1] * zm[1][a] + wg[1][2] * zm[2][a];
    ymg[a] = wm[1][0] * zg[0][a] + wm[1][1] * zg[1][a] + wm[1][2] * zg[2][a];
  }
  const double g0 = wg[0][0] * ymm[0] + wg[0][1] * ymm[1] + wg[0][2] * ymm[2];
  const double g1 = wm[0][0] * ygm[0] + wm[0][1] * ygm[1] + wm[0][2] * ygm[2];
  const double g2 = wm[0][0] * ymg[0] + wm[0][1] * ymg[1] + wm[0][2] * ymg[2];
  if (FROM) {
    uo[3 * v] = src[3 * v] - h2 * g0, uo[3 * v + 1] = src[3 * v + 1] - h2 * g1;
    uo[3 * v + 2] = src[3 * v + 2] - h2 * g2;
  } else {
    uo[3 * v] -= h2 * g0, uo[3 * v + 1] -= h2 * g1, uo[3 * v + 2] -= h2 * g2;
  }
}
unsigned grad_uniform_tiles(int64_t n) {
  const int64_t m = 2 * n + 1;
  return unsigned(((m + kGradTX - 1) / kGradTX) * ((m + kGradTY - 1) / kGradTY) * ((m + kGradTZ - 1) / kGradTZ));
}

// M_p p on a uniform leaf of n^3 cells, one thread per Q1 lattice point (no
// atomics).  A workgroup takes an 8 x 8 x 4 tile of points: it stages the
// tile's window of values and pressure node indices (10 x 10 x 6 points,
// through the lattice -> pressure node map; points off the lattice are 0) and
// the scales h^3 / mu of the 9 x 9 x 5 cells around it (0 off the mesh) in
// LDS.  Each point then
// contracts its 3 x 3 x 3 window with the 1D linear-element mass (1/3 on the
// point itself, 1/6 on its neighbour; h^3 comes with the cell scale) cell by
// cell, axis by axis, and each of the 8 cells around it adds its contraction
// times its scale.  Every point is written (stored: po is zero on entry and
// no other kernel adds to it on a uniform leaf).
constexpr int kPmTX = 8, kPmTY = 8, kPmTZ = 4;
// One tile of the uniform-leaf M_p p for the calling workgroup (all its
// threads must call it): value(id) gives the input at pressure node id (it
// may compute it, e.g. a CG direction update).  Returns, for the thread's
// point, whether it lies on the lattice, its node (id), its input value (pv)
// and its output (the return value).
struct PmassPoint {
  bool valid;
  int32_t id;
  double pv;
  double out;
};
template <typename F>
__device__ __forceinline__ PmassPoint pmass_tile(int64_t n, const DevPressure& P, const double* __restrict__ mu,
                                                 F value) {
  constexpr int WX = kPmTX + 2, WY = kPmTY + 2, WZ = kPmTZ + 2;
  constexpr int CX = kPmTX + 1, CY = kPmTY + 1, CZ = kPmTZ + 1;
  constexpr int NT = kPmTX * kPmTY * kPmTZ;
  __shared__ double sp[WZ * WY * WX];
  __shared__ int32_t si[WZ * WY * WX];
  __shared__ double ss[CZ * CY * CX];
  const int64_t np1 = n + 1;
  const int64_t ntx = (np1 + kPmTX - 1) / kPmTX, nty = (np1 + kPmTY - 1) / kPmTY;
  const int64_t tile = blockIdx.x;
  const int64_t X0 = (tile % ntx) * kPmTX, Y0 = ((tile / ntx) % nty) * kPmTY, Z0 = (tile / (ntx * nty)) * kPmTZ;
  const double h3 = 1.0 / double(n * n * n);
  for (int e = threadIdx.x; e < WX * WY * WZ; e += NT) {
    const int64_t px = X0 - 1 + e % WX, py = Y0 - 1 + (e / WX) % WY, pz = Z0 - 1 + e / (WX * WY);
    const bool in = px >= 0 && px < np1 && py >= 0 && py < np1 && pz >= 0 && pz < np1;
    const int32_t id = in ? P.plat[px + np1 * (py + np1 * pz)] : -1;
    si[e] = id;
    sp[e] = in ? value(id) : 0.0;
  }
  for (int e = threadIdx.x; e < CX * CY * CZ; e += NT) {
    const int64_t cx = X0 - 1 + e % CX, cy = Y0 - 1 + (e / CX) % CY, cz = Z0 - 1 + e / (CX * CY);
    const bool in = cx >= 0 && cx < n && cy >= 0 && cy < n && cz >= 0 && cz < n;
    ss[e] = in ? h3 / mu[cx + n * (cy + n * cz)] : 0.0;
  }
  __syncthreads();
  const int lx = threadIdx.x % kPmTX, ly = (threadIdx.x / kPmTX) % kPmTY, lz = threadIdx.x / (kPmTX * kPmTY);
  PmassPoint r{false, -1, 0.0, 0.0};
  if (X0 + lx >= np1 || Y0 + ly >= np1 || Z0 + lz >= np1) return r;
  // along x: the cell on side ax in {0, 1} covers window points ax, ax + 1,
  // the point itself being window point 1
  double wx[3][3][2];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double* w = sp + (lz + c) * (WY * WX) + (ly + b) * WX + lx;
      wx[c][b][0] = w[0] * (1.0 / 6.0) + w[1] * (1.0 / 3.0);
      wx[c][b][1] = w[1] * (1.0 / 3.0) + w[2] * (1.0 / 6.0);
    }
  double wy[3][2][2];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
      wy[c][0][ax] = wx[c][0][ax] * (1.0 / 6.0) + wx[c][1][ax] * (1.0 / 3.0);
      wy[c][1][ax] = wx[c][1][ax] * (1.0 / 3.0) + wx[c][2][ax] * (1.0 / 6.0);
    }
  double out = 0.0;
#pragma unroll
  for (int az = 0; az < 2; ++az)
#pragma unroll
    for (int ay = 0; ay < 2; ++ay)
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) {
        const double t = az ? wy[1][ay][ax] * (1.0 / 3.0) + wy[2][ay][ax] * (1.0 / 6.0)
                            : wy[0][ay][ax] * (1.0 / 6.0) + wy[1][ay][ax] * (1.0 / 3.0);
        out += ss[(lz + az) * (CY * CX) + (ly + ay) * CX + lx + ax] * t;
      }
  const int c = (lz + 1) * (WY * WX) + (ly + 1) * WX + lx + 1;
  r.valid = true, r.id = si[c], r.pv = sp[c], r.out = out;
  return r;
}
__global__ __launch_bounds__(kPmTX * kPmTY * kPmTZ) void k_pmass_uniform(int64_t n, DevPressure P,
                                                                         const double* __restrict__ mu,
                                                                         const double* __restrict__ p,
                                                                         double* __restrict__ po,
                                                                         const double* __restrict__ gate) {
  if (gate && *gate != 0.0) return;
  const PmassPoint r = pmass_tile(n, P, mu, [&](int32_t id) { return p[id]; });
  if (r.valid) po[r.id] = r.out;
}
unsigned pmass_uniform_tiles(int64_t n) {
  const int64_t np1 = n + 1;
  return unsigned(((np1 + kPmTX - 1) / kPmTX) * ((np1 + kPmTY - 1) / kPmTY) * ((np1 + kPmTZ - 1) / kPmTZ));
}

template <int B>
__global__ __launch_bounds__(64) void k_div_blocks(DevBlocks blk, DevLevel L, DevPressure P,
                                                   const double* __restrict__ u, double* __restrict__ po) {
  constexpr int NC = B * B * B, NB = 64 / NC;
  constexpr int E = 2 * B + 1, PP = E * E * E, W = 3 * PP;
  constexpr int KP = (NB * PP + 63) / 64;
  __shared__ double buf[NB * W];
  const int lane = threadIdx.x;
  const int64_t blk0 = int64_t(blockIdx.x) * NB;
  const int nb = int(std::min<int64_t>(NB, blk.n - blk0));
  const int np = nb * PP;
  auto lds_of = [&](int bl, int q) {
    const int px = q % E, py = (q / E) % E, pz = q / (E * E);
    return bl * W + bsplit<B>(px) + E * bsplit<B>(py) + E * E * bsplit<B>(pz);
  };
  {
    int32_t sl[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int pa = lane + 64 * k;
      sl[k] = pa < np ? blk.slots[blk0 * PP + pa] : -1;
    }
    double v[KP][3];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int64_t i = 3 * int64_t(sl[k] >= 0 ? slot_node(sl[k]) : 0);
      v[k][0] = u[i], v[k][1] = u[i + 1], v[k][2] = u[i + 2];
    }
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int pa = lane + 64 * k;
      if (pa < NB * PP) {
        const int o = lds_of(pa / PP, pa % PP);
        const bool f = sl[k] >= 0;
        buf[o] = f && !slot_fixed(sl[k], 0) ? v[k][0] : 0.0;
        buf[o + PP] = f && !slot_fixed(sl[k], 1) ? v[k][1] : 0.0;
        buf[o + 2 * PP] = f && !slot_fixed(sl[k], 2) ? v[k][2] : 0.0;
      }
    }
  }
  __syncthreads();
  const int h0 = blk.hoff[blk0], h1 = blk.hoff[blk0 + nb];
  for (int e = h0 + lane; e < h1; e += 64) {
    const int32_t en = blk.hent[e];
    const int q = en & 1023, qm = (en >> 10) & 1023, b2 = en >> 20;
    const double w = blk.hw_d[e];
    const int o = lds_of(b2, q), om = lds_of(b2, qm);
#pragma unroll
    for (int k = 0; k < 3; ++k) atomicAdd(&buf[o + k * PP], w * buf[om + k * PP]);
  }
  __syncthreads();
  const int bl = lane / NC, lc = lane - bl * NC;
  if (bl >= nb) return;
  const int ca = lc % B, cb = (lc / B) % B, cc = lc / (B * B);
  const int base = bl * W;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int yy = 0; yy < 3; ++yy)
#pragma unroll
      for (int xx = 0; xx < 3; ++xx) {
        const int a = xx + 3 * yy + 9 * z;
        const int off = base + bsplit<B>(2 * ca + xx) + E * bsplit<B>(2 * cb + yy) + E * E * bsplit<B>(2 * cc + z);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double v = buf[off + q * PP];
#pragma unroll
          for (int i = 0; i < 8; ++i) acc[i] += c_bhat[i * 81 + 3 * a + q] * v;
        }
      }
  const int64_t c = blk.cells[(blk0 + bl) * NC + lc];
  const double h = cell_h(L, c);
#pragma unroll
  for (int i = 0; i < 8; ++i) pscatter(P, P.pslots[8 * c + i], h * h * acc[i], po);
}

// M_p p on the blocks of the leaf: the block's Q1 lattice ((B+1)^3 points)
// is staged in LDS with hanging points interpolated from their masters (on
// the lattice), each cell adds its 8 outputs in LDS (cells of equal index
// parity share no vertex: 8 classes), hanging outputs are passed on to the
// masters, and the write-back stores the points inside the block and writes
// those on its faces to the block's face slots (fslot, PP per block), which
// k_pface_gather adds into po.
template <int B>
__global__ __launch_bounds__(64) void k_pmass_blocks(DevBlocks blk, DevLevel L, const double* __restrict__ p,
                                                     double* __restrict__ po, const double* __restrict__ gate,
                                                     double* __restrict__ fslot) {
  if (gate && *gate != 0.0) return;
  constexpr int NC = B * B * B, NB = 64 / NC;
  constexpr int E = B + 1, PP = E * E * E;
  constexpr int KP = (NB * PP + 63) / 64;
  __shared__ double buf[NB * PP];
  const int lane = threadIdx.x;
  const int64_t blk0 = int64_t(blockIdx.x) * NB;
  const int nb = int(std::min<int64_t>(NB, blk.n - blk0));
  const int np = nb * PP;
  {
    int32_t sl[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int pa = lane + 64 * k;
      sl[k] = pa < np ? blk.pslots[blk0 * PP + pa] : -1;
    }
    double v[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) v[k] = p[sl[k] >= 0 ? sl[k] : 0];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int pa = lane + 64 * k;
      if (pa < NB * PP) buf[pa] = sl[k] >= 0 ? v[k] : 0.0;
    }
  }
  __syncthreads();
  const int h0 = blk.phoff[blk0], h1 = blk.phoff[blk0 + nb];
  for (int e = h0 + lane; e < h1; e += 64) {
    const int32_t en = blk.phent[e];
    const int q = en & 1023, qm = (en >> 10) & 1023, b2 = en >> 20;
    atomicAdd(&buf[b2 * PP + q], blk.phw[e] * buf[b2 * PP + qm]);
  }
  __syncthreads();
  const int bl = lane / NC, lc = lane - bl * NC;
  const int ca = lc % B, cb = (lc / B) % B, cc = lc / (B * B);
  const int base = bl * PP + ca + E * (cb + E * cc);
  double pl[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) pl[a] = buf[base + (a & 1) + E * (((a >> 1) & 1) + E * (a >> 2))];
  double sc = 0.0;
  if (bl < nb) {
    const int64_t c = blk.cells[(blk0 + bl) * NC + lc];
    const double h = cell_h(L, c);
    sc = h * h * h / L.mu_d[c];
  }
  double out[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) v += c_mhat[i * 8 + j] * pl[j];
    out[i] = sc * v;
  }
  __syncthreads();
  for (int e = lane; e < NB * PP; e += 64) buf[e] = 0.0;
  __syncthreads();
  const int par = (ca & 1) | ((cb & 1) << 1) | ((cc & 1) << 2);
#pragma unroll
  for (int cls = 0; cls < 8; ++cls) {
    if (par == cls) {
#pragma unroll
      for (int a = 0; a < 8; ++a) buf[base + (a & 1) + E * (((a >> 1) & 1) + E * (a >> 2))] += out[a];
    }
    __syncthreads();
  }
  for (int e = h0 + lane; e < h1; e += 64) {
    const int32_t en = blk.phent[e];
    const int q = en & 1023, qm = (en >> 10) & 1023, b2 = en >> 20;
    atomicAdd(&buf[b2 * PP + qm], blk.phw[e] * buf[b2 * PP + q]);
  }
  __syncthreads();
  int32_t sl[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int pa = lane + 64 * k;
    sl[k] = pa < np ? blk.pslots[blk0 * PP + pa] : -1;
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (sl[k] < 0) continue;
    const int pa = lane + 64 * k, q = pa % PP;
    const int px = q % E, py = (q / E) % E, pz = q / (E * E);
    const bool inner = px > 0 && px < E - 1 && py > 0 && py < E - 1 && pz > 0 && pz < E - 1;
    if (inner) po[sl[k]] = buf[pa];
    else fslot[blk0 * PP + pa] = buf[pa];
  }
}

__global__ void k_p_identity(int64_t nh, const int64_t* __restrict__ nodes, const double* __restrict__ pin,
                             double* __restrict__ pout) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nh; i += int64_t(gridDim.x) * blockDim.x)
    pout[nodes[i]] = pin[nodes[i]];
}

// (cm: constrained-component masks on no-normal-flux levels, else null: a
// master's fixed component carries zero)
__global__ void k_distribute_u(int64_t nh, const int64_t* __restrict__ nodes, const int64_t* __restrict__ hptr,
                               const int32_t* __restrict__ hm, const double* __restrict__ hw,
                               const uint8_t* __restrict__ cm, double* __restrict__ u) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nh; i += int64_t(gridDim.x) * blockDim.x) {
    double v0 = 0, v1 = 0, v2 = 0;
    for (int64_t q = hptr[i]; q < hptr[i + 1]; ++q) {
      const int64_t m = 3 * int64_t(hm[q]);
      const unsigned f = cm ? cm[hm[q]] : 0u;
      v0 += (f & 1) ? 0.0 : hw[q] * u[m];
      v1 += (f & 2) ? 0.0 : hw[q] * u[m + 1];
      v2 += (f & 4) ? 0.0 : hw[q] * u[m + 2];
    }
    const int64_t n = 3 * nodes[i];
    u[n] = v0, u[n + 1] = v1, u[n + 2] = v2;
  }
}

__global__ void k_distribute_p(int64_t nh, const int64_t* __restrict__ nodes, const int64_t* __restrict__ hptr,
                               const int32_t* __restrict__ hm, const double* __restrict__ hw, double* __restrict__ p) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nh; i += int64_t(gridDim.x) * blockDim.x) {
    double v = 0;
    for (int64_t q = hptr[i]; q < hptr[i + 1]; ++q) v += hw[q] * p[hm[q]];
    p[nodes[i]] = v;
  }
}

__global__ void k_zero_dofs(int64_t n, const int64_t* __restrict__ dofs, double* __restrict__ u) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    u[dofs[i]] = 0;
}

__global__ __launch_bounds__(kCellBlock) void k_rhs(DevLevel L, const double* __restrict__ f,
                                                    double* __restrict__ b) {
  const int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (c >= L.ncell) return;
  const double h = cell_h(L, c);
  const double h3 = h * h * h;
  const double w1[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  double U[3][27];
  for (int z = 0; z < 3; ++z)
    for (int y = 0; y < 3; ++y)
      for (int x = 0; x < 3; ++x) {
        const int q = x + 3 * y + 9 * z;
        const double w = w1[x] * w1[y] * w1[z] * h3;
        for (int comp = 0; comp < 3; ++comp) U[comp][q] = w * f[(27 * c + q) * 3 + comp];
      }
  for (int comp = 0; comp < 3; ++comp) cellop::interp_all_t<double>(U[comp]);
  for (int a = 0; a < 27; ++a) {
    const int32_t s = vslot(L, c, a);
    if (s == -1) continue;
    for (int comp = 0; comp < 3; ++comp) vscatter1(L, s, comp, U[comp][a], b);
  }
}

}  // namespace

// =================================================================== launchers
template <>
const float* mu_of<float>(const DevLevel& L) {
  return L.mu_f;
}
template <>
const double* mu_of<double>(const DevLevel& L) {
  return L.mu_d;
}

template <typename T>
T* brick_halo(const DevLevel& L);
template <>
float* brick_halo<float>(const DevLevel& L) {
  return L.halo_f;
}
template <>
double* brick_halo<double>(const DevLevel& L) {
  return L.halo_d;
}

template <typename T>
bool brick_fits(int64_t n) {
  // below 32 cells per edge there are too few bricks to fill the chip and a
  // brick's latency dominates: the cell-parallel kernel is faster there
  return n % 8 == 0 && n <= 256 && n >= kBrickMinEdge;
}

template <typename T>
int64_t brick_halo_words(int64_t n) {
  if (!brick_fits<T>(n)) return 0;
  return brick::halo_buffer_words(n);   // slots + zero pad
}
template int64_t brick_halo_words<float>(int64_t);
template int64_t brick_halo_words<double>(int64_t);

namespace {
// owner computes: no output initialisation, no atomics
template <typename T, int BX, int BY, int BZ>
void launch_brick(const DevLevel& L, const T* x, T* y, T* halo, bool init, hipStream_t s) {
  const int64_t n = L.n_edge;
  const int64_t nb = (n / BX) * (n / BY) * (n / BZ);
  if (init)
    brick::k_vmult_brick<T, BX, BY, BZ, false><<<unsigned(nb), BX * BY * BZ, 0, s>>>(
        int(n), mu_of<T>(L), x, y, halo);
  else
    brick::k_vmult_brick<T, BX, BY, BZ, true><<<unsigned(nb), BX * BY * BZ, 0, s>>>(
        int(n), mu_of<T>(L), x, y, halo);
  brick::k_brick_halo_add<T, BX, BY, BZ>
      <<<unsigned(nb * brick::HaloClasses<BX, BY, BZ>::groups), 256, 0, s>>>(int(n), !init, halo, y);
}

template <typename T>
void vmult_impl(const DevLevel& L, const T* x, T* y, hipStream_t s, bool init, bool prepared) {
  if (L.uniform) {
    const int64_t n = L.n_edge;
    T* halo = brick_halo<T>(L);
    if (halo && brick_fits<T>(n)) {
      if (brick::brick_by(n) == 8) launch_brick<T, 8, 8, 4>(L, x, y, halo, init, s);
      else launch_brick<T, 8, 4, 4>(L, x, y, halo, init, s);
    } else {
      if (init && !prepared) k_init_out_uniform<T><<<grid_for(L.nnode), kBlock, 0, s>>>(L.n_edge, x, y);
      k_vmult_uniform3<T><<<unsigned((L.ncell + 63) / 64), 192, 0, s>>>(n, mu_of<T>(L), x, y);
    }
    return;
  }
  if (L.q3) {   // owner-computes: no initialisation kernel (vmult_has_init is false)
    launch_vmult_q3<T>(L, x, y, !init, s);
    return;
  }
  if (init && !prepared) k_init_out_general<T><<<grid_for(L.nnode), kBlock, 0, s>>>(L.nnode, L.cmask, x, y);
  T* fs = face_slots<T>(L);
  if (L.blk4.n) {
    if (init) k_vmult_blocks<T, 4, false><<<unsigned(L.blk4.n), 64, 0, s>>>(L.blk4, L.clev, mu_of<T>(L), x, y, fs);
    else k_vmult_blocks<T, 4, true><<<unsigned(L.blk4.n), 64, 0, s>>>(L.blk4, L.clev, mu_of<T>(L), x, y, fs);
  }
  if (L.blk2.n) {
    const unsigned g = unsigned((L.blk2.n + 7) / 8);
    T* fs2 = fs + 3 * L.fslot_blk2;
    if (init) k_vmult_blocks<T, 2, false><<<g, 64, 0, s>>>(L.blk2, L.clev, mu_of<T>(L), x, y, fs2);
    else k_vmult_blocks<T, 2, true><<<g, 64, 0, s>>>(L.blk2, L.clev, mu_of<T>(L), x, y, fs2);
  }
  if (L.n_single_reg)
    k_vmult_general3<T, false><<<unsigned((L.n_single_reg + 63) / 64), 192, 0, s>>>(
        L.single_reg, L.n_single_reg, L.slots, L.clev, mu_of<T>(L), nullptr, nullptr, nullptr, nullptr, x, y);
  if (L.n_single_hang)
    k_vmult_general3<T, true><<<unsigned((L.n_single_hang + 63) / 64), 192, 0, s>>>(
        L.single_hang, L.n_single_hang, L.slots, L.clev, mu_of<T>(L), L.hptr, L.hmaster, hw_of<T>(L),
        L.noflux ? L.cmask : nullptr, x, y);
  if (L.n_face)
    k_face_gather<T><<<grid_for(L.n_face), kBlock, 0, s>>>(L.n_face, L.face_node, L.face_ptr, L.face_ent, fs, y);
}
}  // namespace
template <typename T>
void launch_vmult(const DevLevel& L, const T* x, T* y, hipStream_t s, bool init) {
  vmult_impl<T>(L, x, y, s, init, false);
}
template <typename T>
void launch_vmult_prepared(const DevLevel& L, const T* x, T* y, hipStream_t s) {
  vmult_impl<T>(L, x, y, s, true, true);
}
template <typename T>
bool vmult_has_init(const DevLevel& L) {
  return !L.q3 && !(L.uniform && brick_halo<T>(L) && brick_fits<T>(L.n_edge));
}
template void launch_vmult_prepared<float>(const DevLevel&, const float*, float*, hipStream_t);
template void launch_vmult_prepared<double>(const DevLevel&, const double*, double*, hipStream_t);
template bool vmult_has_init<float>(const DevLevel&);
template bool vmult_has_init<double>(const DevLevel&);
template void launch_vmult<float>(const DevLevel&, const float*, float*, hipStream_t, bool);
template void launch_vmult<double>(const DevLevel&, const double*, double*, hipStream_t, bool);

void launch_diag(const DevLevel& L, const double* khat, double* d, hipStream_t s) {
  if (L.q3) {
    launch_diag_q3(L, L.q3_kdiag, d, s);
    return;
  }
  if (L.uniform) {
    k_diag_uniform<<<unsigned((L.ncell + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(L.n_edge, L.mu_d, d);
    return;
  }
  if (L.n_reg_cells)
    k_diag_regular<<<unsigned((L.n_reg_cells + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(
        L.reg_cells, L.n_reg_cells, L.slots, L.clev, L.mu_d, d);
  if (L.n_hang_cells)
    k_diag_hanging<<<unsigned(L.n_hang_cells), 64, 0, s>>>(L.hang_cells, L.slots, L.clev, L.mu_d, L.hptr, L.hmaster,
                                                          L.hw_d, khat, d);
}

void launch_invert_diag(const DevLevel& L, const double* d, double* md, float* mf, hipStream_t s) {
  if (L.uniform)
    k_invert_diag_uniform<<<grid_for(L.nnode), kBlock, 0, s>>>(L.n_edge, d, md, mf);
  else
    k_invert_diag_general<<<grid_for(L.nnode), kBlock, 0, s>>>(L.nnode, L.cmask, d, md, mf);
}

template <typename T>
OutPrep<T> out_prep_of(const ChebPrep& p) {
  OutPrep<T> o{static_cast<T*>(p.tn), p.cmask, p.m, p.from_x ? 1 : 0};
  return o;
}
template <typename T>
void launch_cheb_init0(int64_t n, const T* b, const T* minv, T* r, T* d, T* x, double it, hipStream_t s) {
  k_cheb_init0<T><<<grid_for(n), kBlock, 0, s>>>(n, b, minv, r, d, x, T(it));
}
template <typename T>
void launch_cheb_init(int64_t n, const T* b, const T* t, const T* minv, T* r, T* d, T* x, double it, hipStream_t s) {
  k_cheb_init<T><<<grid_for(n), kBlock, 0, s>>>(n, b, t, minv, r, d, x, T(it));
}
template <typename T>
void launch_cheb_step(int64_t n, const T* t, const T* minv, T* r, T* d, T* x, double alpha, double beta,
                      hipStream_t s) {
  k_cheb_step<T><<<grid_for(n), kBlock, 0, s>>>(n, t, minv, r, d, x, T(alpha), T(beta));
}
template <typename T>
void launch_chebx_init0(int64_t n, const T* b, const T* minv, T* d, T* x, double it, hipStream_t s,
                        const ChebPrep& p) {
  k_chebx_init0<T><<<grid_for(n), kBlock, 0, s>>>(n, b, minv, d, x, T(it), out_prep_of<T>(p));
}
template <typename T>
void launch_chebx_step(int64_t n, const T* b, const T* t, const T* minv, T* d, T* x, double alpha, double beta,
                       hipStream_t s, const ChebPrep& p) {
  k_chebx_step<T><<<grid_for(n), kBlock, 0, s>>>(n, b, t, minv, d, x, T(alpha), T(beta), out_prep_of<T>(p));
}
template void launch_chebx_init0<float>(int64_t, const float*, const float*, float*, float*, double, hipStream_t,
                                        const ChebPrep&);
template void launch_chebx_init0<double>(int64_t, const double*, const double*, double*, double*, double, hipStream_t,
                                         const ChebPrep&);
template void launch_chebx_step<float>(int64_t, const float*, const float*, const float*, float*, float*, double,
                                       double, hipStream_t, const ChebPrep&);
template void launch_chebx_step<double>(int64_t, const double*, const double*, const double*, double*, double*,
                                        double, double, hipStream_t, const ChebPrep&);
#define MFGMG_INST_CHEB(T)                                                                                   \
  template void launch_cheb_init0<T>(int64_t, const T*, const T*, T*, T*, T*, double, hipStream_t);          \
  template void launch_cheb_init<T>(int64_t, const T*, const T*, const T*, T*, T*, T*, double, hipStream_t); \
  template void launch_cheb_step<T>(int64_t, const T*, const T*, T*, T*, T*, double, double, hipStream_t);
MFGMG_INST_CHEB(float)
MFGMG_INST_CHEB(double)

template <typename T>
void launch_prolong(int64_t nf, const int64_t* ptr, const int32_t* col, const float* w, const T* xc, T* xf, bool add,
                    hipStream_t s, const uint8_t* cmf, const uint8_t* cmc) {
  k_prolong<T, kProlongLanes><<<grid_for(nf * kProlongLanes), kBlock, 0, s>>>(nf, ptr, col, w, xc, xf, add, cmf, cmc);
}
template <typename T>
void launch_restrict(int64_t nc, const int64_t* ptr, const int32_t* col, const float* w, const T* b, const T* t,
                     T* xc, hipStream_t s, const uint8_t* cmf, const uint8_t* cmc) {
  k_restrict<T, kRestrictLanes><<<grid_for(nc * kRestrictLanes), kBlock, 0, s>>>(nc, ptr, col, w, b, t, xc, cmf,
                                                                                  cmc);
}
template void launch_prolong<float>(int64_t, const int64_t*, const int32_t*, const float*, const float*, float*, bool,
                                    hipStream_t, const uint8_t*, const uint8_t*);
template void launch_prolong<double>(int64_t, const int64_t*, const int32_t*, const float*, const double*, double*,
                                     bool, hipStream_t, const uint8_t*, const uint8_t*);
template void launch_restrict<float>(int64_t, const int64_t*, const int32_t*, const float*, const float*,
                                     const float*, float*, hipStream_t, const uint8_t*, const uint8_t*);
template void launch_restrict<double>(int64_t, const int64_t*, const int32_t*, const float*, const double*,
                                      const double*, double*, hipStream_t, const uint8_t*, const uint8_t*);

template <typename T>
void launch_coarse(const T* Ainv, const int32_t* fd, int nfree, int n, const T* b, T* x, hipStream_t s) {
  if (nfree > kCoarseMaxFree) return;   // cannot happen: the caller checks the coarse mesh
  k_coarse<T><<<1, 128, 0, s>>>(Ainv, fd, nfree, n, b, x);
}
template void launch_coarse<float>(const float*, const int32_t*, int, int, const float*, float*, hipStream_t);
template <typename T>
bool launch_vcycle_tail(const DevLevel& L, const DevLevel& Lc, const T* minv, const T* Ainv, const int32_t* fd,
                        int nfree, double lam, const T* b, T* x, hipStream_t s) {
  if (!(L.uniform && !L.q3 && !L.noflux && L.n_edge == kTailN && Lc.uniform && Lc.n_edge == kTailN / 2 &&
        nfree == kTailFree))
    return false;
  // the smoother's coefficients (Saad, Alg. 12.1 on [lam / 15, lam]) as the separate kernels take them
  const double lo = lam / 15.0, theta = 0.5 * (lam + lo), delta = 0.5 * (lam - lo), sigma = theta / delta;
  TailCoef<T> cf{};
  cf.it0 = T(1.0 / theta);
  double rho = 1.0 / sigma;
  for (int k = 1; k < 4; ++k) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    cf.alpha[k] = T(rho_new * rho);
    cf.beta[k] = T(2.0 * rho_new / delta);
    rho = rho_new;
  }
  k_vcycle_tail<T><<<1, 256, 0, s>>>(mu_of<T>(L), minv, Ainv, fd, cf, b, x);
  return true;
}
template bool launch_vcycle_tail<float>(const DevLevel&, const DevLevel&, const float*, const float*, const int32_t*,
                                        int, double, const float*, float*, hipStream_t);
template bool launch_vcycle_tail<double>(const DevLevel&, const DevLevel&, const double*, const double*,
                                         const int32_t*, int, double, const double*, double*, hipStream_t);

template void launch_coarse<double>(const double*, const int32_t*, int, int, const double*, double*, hipStream_t);

void launch_harmonic_mu(int64_t ncell, const double* mq, double* mu, hipStream_t s) {
  k_harmonic<<<grid_for(ncell), kBlock, 0, s>>>(ncell, mq, mu);
}
void launch_restrict_mu(int64_t ncell, const int32_t* src, const double* mf, double* mc, hipStream_t s) {
  k_restrict_mu<<<grid_for(ncell), kBlock, 0, s>>>(ncell, src, mf, mc);
}
void launch_to_float(int64_t n, const double* a, float* b, hipStream_t s) {
  k_to_float<<<grid_for(n), kBlock, 0, s>>>(n, a, b);
}
void launch_to_double(int64_t n, const float* a, double* b, hipStream_t s) {
  k_to_double<<<grid_for(n), kBlock, 0, s>>>(n, a, b);
}

void launch_dot(int64_t n, const double* a, const double* b, double* part, double* result, hipStream_t s) {
  k_dot_partial<<<kRedBlocks, kBlock, 0, s>>>(n, a, b, part);
  k_sum_partials<<<1, kBlock, 0, s>>>(kRedBlocks, part, result);
}

void launch_mdot(int64_t n, int nv, const double* V, int64_t ldv, const double* w, double* part, double* result,
                 hipStream_t s, bool with_norm) {
  // part holds rows x nb partials (65536 from the caller: rows <= 256)
  const unsigned rows = unsigned(nv + (with_norm ? 1 : 0));
  if (nv <= 32) {   // up to 8 vectors per wave, more blocks
    const int nb = 1024;   // rows <= 33: 33 x 1024 partials
    if (nv <= 8) k_mdot_tiles<2><<<nb, 256, 0, s>>>(n, 0, nv, V, ldv, w, with_norm, part);
    else if (nv <= 16) k_mdot_tiles<4><<<nb, 256, 0, s>>>(n, 0, nv, V, ldv, w, with_norm, part);
    else k_mdot_tiles<8><<<nb, 256, 0, s>>>(n, 0, nv, V, ldv, w, with_norm, part);
    k_sum_partials<<<rows, kBlock, 0, s>>>(nb, part, result);
    return;
  }
  const int nb = rows <= 128 ? 512 : 256;
  // up to 64 vectors per launch (16 per wave); w . w with the first
  for (int j0 = 0; j0 < nv; j0 += 64)
    k_mdot_tiles<16><<<nb, 256, 0, s>>>(n, j0, nv, V, ldv, w, with_norm && j0 == 0, part);
  k_sum_partials<<<rows, kBlock, 0, s>>>(nb, part, result);
}

bool launch_mupdate_dots(int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w, double* part,
                         double* result, bool dots, hipStream_t s) {
  // one wave per SIMD for NV = 64 (about 270 registers): 256 blocks; part
  // holds at most 65 x 512 partials (65536 from the caller)
  if (nv < 1 || nv > kMupdateDotsMax) return false;
  const unsigned rows = dots ? unsigned(nv + 1) : 1u;
  const int nb = nv <= 64 ? 512 : 256;   // rows x nb <= 65 x 512 or 129 x 256 partials
  // up to 32 vectors: one thread per entry holding its nv values; beyond,
  // where that form runs at one wave per SIMD, the tiles (64 vectors: 697 ->
  // 438 us per call on the 64^3 workload)
#define MFGMG_MUD(NVT)                                                                  \
  if (dots) k_mupdate_dots<NVT, true><<<nb, kBlock, 0, s>>>(n, nv, V, ldv, h, w, part); \
  else k_mupdate_dots<NVT, false><<<nb, kBlock, 0, s>>>(n, nv, V, ldv, h, w, part);
  if (nv <= 16) {
    MFGMG_MUD(16)
  } else if (nv <= 32) {
    MFGMG_MUD(32)
  } else if (nv <= 64) {
    if (dots) k_mupdate_tiles<16, true><<<nb, 256, 0, s>>>(n, nv, V, ldv, h, w, part);
    else k_mupdate_tiles<16, false><<<nb, 256, 0, s>>>(n, nv, V, ldv, h, w, part);
  } else {
    if (dots) k_mupdate_tiles<32, true><<<nb, 256, 0, s>>>(n, nv, V, ldv, h, w, part);
    else k_mupdate_tiles<32, false><<<nb, 256, 0, s>>>(n, nv, V, ldv, h, w, part);
  }
#undef MFGMG_MUD
  k_sum_partials<<<rows, kBlock, 0, s>>>(nb, part, result);
  return true;
}

void launch_mupdate(int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w, hipStream_t s) {
  k_mupdate<<<grid_for(n), kBlock, 0, s>>>(n, nv, V, ldv, h, w);
}
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  k_axpby<<<grid_for(n), kBlock, 0, s>>>(n, a, x, b, y);
}
void launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  k_scale_copy<<<grid_for(n), kBlock, 0, s>>>(n, a, x, y);
}
void launch_fill(int64_t n, double v, double* y, hipStream_t s) { k_fill<<<grid_for(n), kBlock, 0, s>>>(n, v, y); }
void launch_fill_f(int64_t n, float v, float* y, hipStream_t s) {
  k_fill_f<<<grid_for(n), kBlock, 0, s>>>(n, v, y);
}
void launch_mul(int64_t n, const double* a, const double* b, double* y, hipStream_t s) {
  k_mul<<<grid_for(n), kBlock, 0, s>>>(n, a, b, y);
}

void launch_div(const DevLevel& L, const DevPressure& P, const double* u, double* po, hipStream_t s) {
  k_fill<<<grid_for(P.np), kBlock, 0, s>>>(P.np, 0.0, po);
  if (L.q3) {
    launch_div_q3(L, u, po, s);
  } else if (L.blk4.n || L.blk2.n) {
    if (L.blk4.n) k_div_blocks<4><<<unsigned(L.blk4.n), 64, 0, s>>>(L.blk4, L, P, u, po);
    if (L.blk2.n) k_div_blocks<2><<<unsigned((L.blk2.n + 7) / 8), 64, 0, s>>>(L.blk2, L, P, u, po);
    for (auto lst : {std::make_pair(L.single_reg, L.n_single_reg), std::make_pair(L.single_hang, L.n_single_hang)})
      if (lst.second)
        k_div<<<unsigned((lst.second + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(L, P, lst.first, lst.second,
                                                                                          u, po);
  } else {
    k_div<<<unsigned((L.ncell + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(L, P, nullptr, L.ncell, u, po);
  }
}
void launch_grad_from(const DevLevel& L, const DevPressure& P, const double* p, const double* src, double* uo,
                      hipStream_t s) {
  if (L.uniform) {
    k_grad_uniform<true><<<grad_uniform_tiles(L.n_edge), kGradTX * kGradTY * kGradTZ, 0, s>>>(L.n_edge, P, p, src,
                                                                                              uo);
    return;
  }
  (void)hipMemcpyAsync(uo, src, size_t(3 * L.nnode) * sizeof(double), hipMemcpyDeviceToDevice, s);
  launch_grad_add(L, P, p, uo, s);
}
void launch_grad_add(const DevLevel& L, const DevPressure& P, const double* p, double* uo, hipStream_t s) {
  if (L.q3) {
    launch_grad_q3(L, p, uo, s);
  } else if (L.uniform) {
    k_grad_uniform<false><<<grad_uniform_tiles(L.n_edge), kGradTX * kGradTY * kGradTZ, 0, s>>>(L.n_edge, P, p,
                                                                                               nullptr, uo);
  } else if (L.blk4.n || L.blk2.n) {
    double* fs = L.fslot_d;
    if (L.blk4.n) k_grad_blocks<4><<<unsigned(L.blk4.n), 64, 0, s>>>(L.blk4, L, P, p, uo, fs);
    if (L.blk2.n)
      k_grad_blocks<2><<<unsigned((L.blk2.n + 7) / 8), 64, 0, s>>>(L.blk2, L, P, p, uo, fs + 3 * L.fslot_blk2);
    for (auto lst : {std::make_pair(L.single_reg, L.n_single_reg), std::make_pair(L.single_hang, L.n_single_hang)})
      if (lst.second)
        k_grad_add<<<unsigned((lst.second + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(
            L, P, lst.first, lst.second, p, uo);
    if (L.n_face)
      k_face_gather<double><<<grid_for(L.n_face), kBlock, 0, s>>>(L.n_face, L.face_node, L.face_ptr, L.face_ent, fs,
                                                                   uo);
  } else {
    k_grad_add<<<unsigned((L.ncell + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(L, P, nullptr, L.ncell, p,
                                                                                         uo);
  }
}
void launch_pmass(const DevLevel& L, const DevPressure& P, const double* p, double* po, hipStream_t s,
                  const double* gate) {
  // the uniform-leaf kernel writes every entry
  if (!(L.uniform && P.plat)) k_fill<<<grid_for(P.np), kBlock, 0, s>>>(P.np, 0.0, po);
  launch_pmass_add(L, P, p, po, s, gate);
}
void launch_pmass_add(const DevLevel& L, const DevPressure& P, const double* p, double* po, hipStream_t s,
                      const double* gate) {
  if (L.q3) {
    launch_pmass_q2(L, p, po, s, gate);
  } else if (L.uniform && P.plat) {
    k_pmass_uniform<<<pmass_uniform_tiles(L.n_edge), kPmTX * kPmTY * kPmTZ, 0, s>>>(L.n_edge, P, L.mu_d, p, po, gate);
  } else if ((L.blk4.n && L.blk4.pslots) || (L.blk2.n && L.blk2.pslots)) {
    double* fs = L.pfslot;
    if (L.blk4.n) k_pmass_blocks<4><<<unsigned(L.blk4.n), 64, 0, s>>>(L.blk4, L, p, po, gate, fs);
    if (L.blk2.n)
      k_pmass_blocks<2><<<unsigned((L.blk2.n + 7) / 8), 64, 0, s>>>(L.blk2, L, p, po, gate, fs + L.pfslot_blk2);
    for (auto lst : {std::make_pair(L.single_reg, L.n_single_reg), std::make_pair(L.single_hang, L.n_single_hang)})
      if (lst.second)
        k_pmass<<<unsigned((lst.second + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(L, P, lst.first,
                                                                                            lst.second, p, po, gate);
    if (L.n_pface)
      k_pface_gather<<<grid_for(L.n_pface), kBlock, 0, s>>>(L.n_pface, L.pface_node, L.pface_ptr, L.pface_ent, fs, po,
                                                            gate);
  } else {
    k_pmass<<<unsigned((L.ncell + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(L, P, nullptr, L.ncell, p, po,
                                                                                        gate);
  }
  if (P.nh) k_p_identity<<<grid_for(P.nh), kBlock, 0, s>>>(P.nh, P.hang_nodes, p, po);
}

// ------------------------------------------------------- device-resident CG
// Scalars of the Jacobi-CG on M_p live in sc[]: 0, 1 r.z of even and odd
// iterations (iteration k reads slot k mod 2 and writes the other), 4
// stopping threshold on r.r, 5 done flag, 6 iterations.  Once done is set
// every kernel of a further iteration returns at once, so the host may queue
// several iterations between checks without changing the result.  The two
// scalar steps (alpha and the test / beta) are taken by every block of the
// vector kernels from the previous kernel's block partials (same sums, same
// order in every block), so an iteration is M_p p, p.q, and two vector
// kernels; the second also clears q for the next M_p p.
namespace {
// sc[7] holds r.r of the start residual (the right-hand side): the stopping
// threshold is rtol2 r.r, and a zero right-hand side is done at once (x = 0)
__global__ __launch_bounds__(kBlock) void k_cg_setup(double* sc, double rtol2) {
  if (threadIdx.x == 0) {
    const double rr = sc[7];
    sc[1] = 0.0, sc[4] = rtol2 * rr, sc[5] = rr == 0.0 ? 1.0 : 0.0, sc[6] = 0.0;
  }
}
// r = rhs, z = p = minv rhs, x = q = 0
__global__ __launch_bounds__(kBlock) void k_cg_start(int64_t n, const double* __restrict__ rhs,
                                                    const double* __restrict__ minv, double* __restrict__ r,
                                                    double* __restrict__ z, double* __restrict__ p,
                                                    double* __restrict__ x, double* __restrict__ q) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double ri = rhs[i], zi = minv[i] * ri;
    r[i] = ri, z[i] = zi, p[i] = zi, x[i] = 0.0, q[i] = 0.0;
  }
}
// sum of part[0, np) in every thread of the block
__device__ __forceinline__ double block_sum_all(int np, const double* __restrict__ part) {
  __shared__ double bc;
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
  v = block_sum(v);
  if (threadIdx.x == 0) bc = v;
  __syncthreads();
  v = bc;
  __syncthreads();
  return v;
}
// count: this kernel counts the iteration in sc[6] (the uniform-leaf path;
// elsewhere k_cg_pupdate does)
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, int npq, const double* __restrict__ part_pq,
                                                     double* sc, int par, bool count,
                                                     const double* __restrict__ p, const double* __restrict__ q,
                                                     const double* __restrict__ minv, double* __restrict__ x,
                                                     double* __restrict__ r, double* __restrict__ z,
                                                     double* __restrict__ part) {
  if (sc[5] != 0.0) return;
  const double alpha = sc[par] / block_sum_all(npq, part_pq);
  if (count && blockIdx.x == 0 && threadIdx.x == 0) sc[6] += 1.0;
  double rr = 0.0, rz = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    const double zi = minv[i] * ri;
    r[i] = ri, z[i] = zi;
    rr += ri * ri, rz += ri * zi;
  }
  rr = block_sum(rr);
  rz = block_sum(rz);
  if (threadIdx.x == 0) part[blockIdx.x] = rr, part[gridDim.x + blockIdx.x] = rz;
}
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(int64_t n, int np, const double* __restrict__ part, double* sc,
                                                      int par, const double* __restrict__ z, double* __restrict__ p,
                                                      double* __restrict__ q) {
  if (sc[5] != 0.0) return;
  const double rr = block_sum_all(np, part);
  const double rz = block_sum_all(np, part + np);
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (rr <= sc[4]) {
    if (lead) sc[6] += 1.0, sc[5] = 1.0;
    return;
  }
  const double beta = rz / sc[par];
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    p[i] = z[i] + beta * p[i];
    q[i] = 0.0;
  }
  if (lead) sc[6] += 1.0, sc[par ^ 1] = rz;
}
// Uniform leaf: an iteration in two kernels.  This one takes the previous
// iteration's test and direction update (from k_cg_update's partials, as
// k_cg_pupdate does; k_cg_update counts the iterations) into the staging of
// the tiled M_p p: every tile forms
// p_k = z + beta p_{k-1} on its window (a point staged by several tiles gets
// the same value in each), stores p_k on its own points into the other
// direction buffer (p_{k-1} is only read), q = M_p p_k, and its partial of
// p_k . q.  Iteration 0 takes p_0 from pcur as it is.
__global__ __launch_bounds__(kPmTX * kPmTY * kPmTZ) void k_cg_pmass_uniform(
    int64_t n, DevPressure P, const double* __restrict__ mu, const double* __restrict__ z,
    const double* __restrict__ pprev, double* __restrict__ pcur, double* __restrict__ q, int np_part,
    const double* __restrict__ part, double* sc, int k, double* __restrict__ part_pq) {
  if (sc[5] != 0.0) return;
  double beta = 0.0;
  if (k > 0) {
    const double rr = block_sum_all(np_part, part);
    const double rz = block_sum_all(np_part, part + np_part);
    const int pp = (k - 1) & 1;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (rr <= sc[4]) {
      if (lead) sc[5] = 1.0;
      return;
    }
    beta = rz / sc[pp];
    if (lead) sc[pp ^ 1] = rz;
  }
  const PmassPoint r =
      pmass_tile(n, P, mu, [&](int32_t id) { return k > 0 ? z[id] + beta * pprev[id] : pcur[id]; });
  if (r.valid) {
    if (k > 0) pcur[r.id] = r.pv;
    q[r.id] = r.out;
  }
  const double v = block_sum(r.valid ? r.pv * r.out : 0.0);
  if (threadIdx.x == 0) part_pq[blockIdx.x] = v;
}
}  // namespace

void launch_cg_start(int64_t n, const double* rhs, const double* minv, double* r, double* z, double* p, double* x,
                     double* q, hipStream_t s) {
  k_cg_start<<<grid_for(n), kBlock, 0, s>>>(n, rhs, minv, r, z, p, x, q);
}
void launch_cg_setup(double* sc, double rtol2, hipStream_t s) { k_cg_setup<<<1, kBlock, 0, s>>>(sc, rtol2); }

// workgroups of the CG vector kernels: every workgroup of the next kernel
// sums all their partials, so few partials keep that read small (the vectors
// are short: a pressure field)
constexpr int kCgBlocks = 256;

void launch_cg_pmass_iteration(const DevLevel& L, const DevPressure& P, const double* minv, double* x, double* r,
                               double* z, double* p, double* p_alt, double* q, double* part, double* sc, int k,
                               hipStream_t s) {
  const int64_t n = P.np;
  if (L.uniform && P.plat && int64_t(pmass_uniform_tiles(L.n_edge)) + 2 * kRedBlocks <= kRedPartWords) {
    // p_k lives in p for even k, in p_alt for odd k; k_cg_update's partials
    // at part[0, 2g), the tiles' p.q partials after 2 kRedBlocks
    const unsigned g = grid_for(n, kBlock, kCgBlocks), nt = pmass_uniform_tiles(L.n_edge);
    const int par = k & 1;
    double* pk = par ? p_alt : p;
    const double* pprev = par ? p : p_alt;
    double* ppq = part + 2 * kRedBlocks;
    k_cg_pmass_uniform<<<nt, kPmTX * kPmTY * kPmTZ, 0, s>>>(L.n_edge, P, L.mu_d, z, pprev, pk, q, int(g), part, sc,
                                                           k, ppq);
    k_cg_update<<<g, kBlock, 0, s>>>(n, int(nt), ppq, sc, par, true, pk, q, minv, x, r, z, part);
    return;
  }
  // q is zero here: cleared by the setup, then by the previous iteration
  launch_pmass_add(L, P, p, q, s, sc + 5);
  k_dot_partial<<<kCgBlocks, kBlock, 0, s>>>(n, p, q, part);
  const unsigned g = grid_for(n, kBlock, kCgBlocks);
  const int par = k & 1;
  k_cg_update<<<g, kBlock, 0, s>>>(n, kCgBlocks, part, sc, par, false, p, q, minv, x, r, z, part + kRedBlocks);
  k_cg_pupdate<<<g, kBlock, 0, s>>>(n, int(g), part + kRedBlocks, sc, par, z, p, q);
}
void launch_p_identity(const DevPressure& P, const double* pin, double* pout, hipStream_t s) {
  if (P.nh) k_p_identity<<<grid_for(P.nh), kBlock, 0, s>>>(P.nh, P.hang_nodes, pin, pout);
}
void launch_distribute_u(const DevLevel& L, double* u, hipStream_t s) {
  if (L.nhang)
    k_distribute_u<<<grid_for(L.nhang), kBlock, 0, s>>>(L.nhang, L.hnode, L.hptr, L.hmaster, L.hw_d,
                                                        L.noflux ? L.cmask : nullptr, u);
}
void launch_distribute_p(const DevPressure& P, double* p, hipStream_t s) {
  if (P.nh) k_distribute_p<<<grid_for(P.nh), kBlock, 0, s>>>(P.nh, P.hang_nodes, P.hptr, P.hmaster, P.hw, p);
}
void launch_zero_constrained(const DevLevel& L, double* u, hipStream_t s) {
  if (L.n_cons) k_zero_dofs<<<grid_for(L.n_cons), kBlock, 0, s>>>(L.n_cons, L.cons_dofs, u);
}
void launch_rhs(const DevLevel& L, const double* f, double* b, hipStream_t s) {
  k_fill<<<grid_for(3 * L.nnode), kBlock, 0, s>>>(3 * L.nnode, 0.0, b);
  if (L.q3) {
    launch_rhs_q3(L, f, b, s);
    return;
  }
  k_rhs<<<unsigned((L.ncell + kCellBlock - 1) / kCellBlock), kCellBlock, 0, s>>>(L, f, b);
}

void set_element_constants(const double* kd, const double* bh, const double* mh) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_khat_diag), kd, sizeof(double) * 81);
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_bhat), bh, sizeof(double) * 8 * 81);
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_mhat), mh, sizeof(double) * 64);
}

}  // namespace mfgmg

namespace mfgmg {

template <typename T>
bool tr_has_scratch(const DevLevel& F);
template <>
bool tr_has_scratch<float>(const DevLevel& F) {
  return F.tr_s1_f && F.tr_s2_f;
}
template <>
bool tr_has_scratch<double>(const DevLevel& F) {
  return F.tr_s1_d && F.tr_s2_d;
}

template <typename T>
void launch_prolong_level(const DevLevel& F, const DevLevel& Cc, const int64_t* ptr, const int32_t* col,
                          const float* w, const T* xc, T* xf, bool add, hipStream_t s) {
  if (F.uniform && Cc.uniform && F.n_edge == 2 * Cc.n_edge) {
    const int64_t mf = 4 * Cc.n_edge + 1;
    if (Cc.n_edge <= kRowMaxCoarse)
      k_prolong_rows<T><<<unsigned((mf * mf + 3) / 4), 256, 0, s>>>(int(Cc.n_edge), xc, xf, add);
    else
      k_prolong_uniform<T><<<grid_for(F.nnode), kBlock, 0, s>>>(int(Cc.n_edge), xc, xf, add);
    return;
  }
  if (F.q3 && F.q3_pc0 && tr_has_scratch<T>(F)) {
    launch_prolong_q3<T>(F, xc, xf, add, s);
    return;
  }
  if (F.q3) {   // Q3 lattice levels without scratch: the CSR with its FP64 weights (not dyadic)
    k_prolong<T, kProlongLanes, double><<<grid_for(F.nnode * kProlongLanes), kBlock, 0, s>>>(
        F.nnode, ptr, col, F.q3_Pw, xc, xf, add, nullptr, nullptr);
    return;
  }
  // no-normal-flux levels: the fixed components are masked on both sides
  const uint8_t* cmf = F.noflux ? F.cmask : nullptr;
  const uint8_t* cmc = F.noflux ? Cc.cmask : nullptr;
  k_prolong<T, kProlongLanes><<<grid_for(F.nnode * kProlongLanes), kBlock, 0, s>>>(F.nnode, ptr, col, w, xc, xf,
                                                                                    add, cmf, cmc);
}

template <typename T>
void launch_restrict_level(const DevLevel& F, const DevLevel& Cc, const int64_t* ptr, const int32_t* col,
                           const float* w, const T* b, const T* t, T* xc, T* s1, T* s2, hipStream_t s) {
  // (the passes index nodes with 32-bit integers: levels up to 512^3 cells)
  const int64_t mc = 2 * Cc.n_edge + 1, mf = 4 * Cc.n_edge + 1;
  if (F.q3 && F.q3_pc0 && tr_has_scratch<T>(F)) {
    launch_restrict_q3<T>(F, b, t, xc, s);
    return;
  }
  if (F.q3) {
    k_restrict<T, kRestrictLanes, double><<<grid_for(Cc.nnode * kRestrictLanes), kBlock, 0, s>>>(
        Cc.nnode, ptr, col, F.q3_Rw, b, t, xc, nullptr, nullptr);
    return;
  }
  if (F.uniform && Cc.uniform && F.n_edge == 2 * Cc.n_edge && mc * mf * mf < (int64_t(1) << 31)) {
    const int nc = int(Cc.n_edge);
    if (nc <= kRowMaxCoarse) k_restrict_x_rows<T><<<unsigned((mf * mf + 3) / 4), 256, 0, s>>>(nc, b, t, s1);
    else k_restrict_x<T><<<grid_for(mc * mf * mf), kBlock, 0, s>>>(nc, b, t, s1);
    k_restrict_y<T><<<grid_for(mc * mc * mf), kBlock, 0, s>>>(nc, s1, s2);
    k_restrict_z<T><<<grid_for(mc * mc * mc), kBlock, 0, s>>>(nc, s2, xc);
    return;
  }
  const uint8_t* cmf = F.noflux ? F.cmask : nullptr;
  const uint8_t* cmc = F.noflux ? Cc.cmask : nullptr;
  k_restrict<T, kRestrictLanes><<<grid_for(Cc.nnode * kRestrictLanes), kBlock, 0, s>>>(Cc.nnode, ptr, col, w, b,
                                                                                        t, xc, cmf, cmc);
}

#define MFGMG_INST_TRANSFER(T)                                                                                \
  template void launch_prolong_level<T>(const DevLevel&, const DevLevel&, const int64_t*, const int32_t*,    \
                                        const float*, const T*, T*, bool, hipStream_t);                       \
  template void launch_restrict_level<T>(const DevLevel&, const DevLevel&, const int64_t*, const int32_t*,   \
                                         const float*, const T*, const T*, T*, T*, T*, hipStream_t);
MFGMG_INST_TRANSFER(float)
MFGMG_INST_TRANSFER(double)

}  // namespace mfgmg
