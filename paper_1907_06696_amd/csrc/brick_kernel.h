// Brick kernel for the Q2 strain-rate operator on uniform levels (device code).
//
// One workgroup per brick of BX x BY x BZ cells, one thread per cell; n <= 256
// cells per edge.  Node-major vectors (3 values per node), lattice numbering
// node = X + (2n+1)(Y + (2n+1)Z).
//  1. Stage the brick's node box ((2B+1) nodes per axis) in LDS.  One wave per
//     node row: lane j holds word j of the row (3 components x (2BX+1) nodes),
//     so the per-element index work is a few scalar operations; every global
//     load of a thread is issued before its LDS stores.  Dirichlet nodes are
//     staged as zero.  LDS layout per component: z-planes of rows of length
//     24, every axis split into its even then odd local nodes, so that for a
//     fixed local node the cells of a row read consecutive words (the padded
//     row keeps a wavefront's 8x4 cells on distinct banks).
//  2. Each thread gathers its 81 values and applies the cell operator.
//  3. Accumulate the 81 results into the zeroed LDS box without atomics: the
//     local nodes are split into classes a in {0,1} | {2} per axis.  Within a
//     class two (cell, local node) pairs never map to the same node, so a
//     read-add-write over the class is race free.  Classes along z couple
//     different waves and are separated by block barriers; classes along x
//     and y couple lanes of one wave, whose LDS operations complete in
//     order, and are separated by an LDS wait and a compiler barrier.
//  4. Write back row by row, owner computes: a node belongs to the brick whose
//     half-open box holds it (the last brick along an axis also owns the
//     closing plane).  Owned nodes are stored (added when accumulating), the
//     brick's contributions to nodes on its high faces, owned by its upper
//     neighbours, go to the brick's slot of a halo buffer, and the second
//     kernel adds every neighbour's halo values into the low-face nodes of
//     their owner.  No atomics, and no separate initialisation of the output:
//     owned Dirichlet nodes receive y = x (identity rows) unless accumulating.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "cell_kernel.h"

namespace mfgmg {
namespace brick {

// f(std::integral_constant<int, w>) for the (wave-uniform) index w < NW
template <int NW, int W = 0, typename F>
__device__ __forceinline__ void with_wave(int w, const F& f) {
  if constexpr (W < NW) {
    if (w == W) f(std::integral_constant<int, W>());
    else with_wave<NW, W + 1>(w, f);
  }
}

// Position of workgroup g of G in XCD-contiguous order.  The hardware deals
// consecutive workgroups to the 8 XCDs in turn (g mod 8); numbering the work
// by this position gives each XCD one contiguous range of it, so neighbouring
// bricks or blocks, which read the same boundary nodes, share that XCD's L2
// (64^3 FP32 operator 54.5 -> 49.2 us).  A bijection of [0, G) for any G.
__device__ __forceinline__ int64_t xcd_order(int64_t g, int64_t G) {
  const int64_t q = G / 8, r = G % 8, x = g % 8, k = g / 8;
  return x * q + (x < r ? x : r) + k;
}

template <int B>
__device__ __forceinline__ int split_index(int l) {
  return (l & 1) ? (B + 1) + (l >> 1) : (l >> 1);
}

// ACC: nodes inside the brick are added to y (y += A x); otherwise stored
// (the caller initialised y to zero on free nodes)
// Halo slot of brick b: the box [NZ][NY][3 NX] (x fastest, node-major; only
// the rows of the high y and z faces are used), then the low and the high x
// planes packed [NZ][NY][3].  The x planes hold one node per box row, so in
// the box layout every value would sit on a cache line of its own.  The
// buffer holds one slot per brick followed by a pad of 64 zeros.
template <int BX, int BY, int BZ>
constexpr int64_t halo_box_words() {
  return int64_t(2 * BZ + 1) * (2 * BY + 1) * 3 * (2 * BX + 1);
}
template <int BX, int BY, int BZ>
constexpr int64_t halo_plane_words() {
  return int64_t(2 * BZ + 1) * (2 * BY + 1) * 3;
}
template <int BX, int BY, int BZ>
constexpr int64_t halo_words() {
  return halo_box_words<BX, BY, BZ>() + 2 * halo_plane_words<BX, BY, BZ>();
}

// Brick shape of a uniform level with n cells per edge (n a multiple of 8):
// 8 x BY x 4 cells with BY = 8 from 64 cells per edge up and 4 below, so that
// a 32^3 level still has 256 bricks for the 256 CUs
constexpr int brick_by(int64_t n) {
  return n >= 64 ? 8 : 4;
}
// entries of the halo buffer of that level: one slot per brick plus a pad of 64 zeros
constexpr int64_t halo_buffer_words(int64_t n) {
  return brick_by(n) == 8 ? (n / 8) * (n / 8) * (n / 4) * halo_words<8, 8, 4>() + 64
                          : (n / 8) * (n / 4) * (n / 4) * halo_words<8, 4, 4>() + 64;
}

// A thread forms its cell's 81 results one input component at a time
// (cellop::apply_cell_by_input): 27 inputs live beside the 81 results, 128
// VGPRs in FP32 (four waves per SIMD; three when accumulating, whose old
// values need more) and 254 in FP64 (two waves per SIMD).
template <typename T, bool ACC>
constexpr int brick_waves_per_simd() {
  return sizeof(T) == 4 ? (ACC ? 3 : 4) : 2;
}
// LDS row pitch of the node box (doubles or floats per row of 2 BX + 1
// nodes): 20 lets two FP64 workgroups of 8x8x4 cells, or four FP32 ones,
// share a CU's LDS, with half a row's accesses on shared banks
constexpr int kBrickRowPitch = 20;

template <typename T, int BX, int BY, int BZ, bool ACC>
__global__ __launch_bounds__(BX * BY * BZ, (brick_waves_per_simd<T, ACC>())) void k_vmult_brick(
    int n, const T* __restrict__ mu, const T* __restrict__ x, T* __restrict__ y, T* __restrict__ halo) {
  constexpr int NT = BX * BY * BZ, NW = NT / 64;
  constexpr int NX = 2 * BX + 1, NY = 2 * BY + 1, NZ = 2 * BZ + 1;
  constexpr int RX = kBrickRowPitch, PL = RX * NY, CS = PL * NZ;
  constexpr int ROW = 3 * NX;
  static_assert(ROW <= 64, "row");
  constexpr int NR = NY * NZ, RPW = (NR + NW - 1) / NW;
  __shared__ __attribute__((aligned(16))) T buf[3 * CS];
  const int nbx = n / BX, nby = n / BY, nbz = n / BZ;
  const int b = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int m = 2 * n + 1;
  const int X0 = 2 * BX * bx, Y0 = 2 * BY * by, Z0 = 2 * BZ * bz;
  const int t = threadIdx.x, lane = t & 63;
  const int lx = lane / 3, comp = lane - 3 * (lane / 3);
  const bool lane_ok = lane < ROW;
  const int X = X0 + (lane_ok ? lx : 0);
  const bool xdir = X == 0 || X == m - 1;
  const bool first_y = by == 0, first_z = bz == 0, last_y = by == nby - 1, last_z = bz == nbz - 1;
  // byte offsets: 3 m^3 sizeof(T) < 2^32 for n <= 256
  const uint32_t lane_off = uint32_t(3 * X + comp) * uint32_t(sizeof(T));
  const uint32_t row_stride = uint32_t(3 * m) * uint32_t(sizeof(T));
  const uint32_t box_off = row_stride * uint32_t(Y0 + m * Z0);
  const uint32_t plane_stride = row_stride * uint32_t(m);
  const int lds_lane = comp * CS + split_index<BX>(lane_ok ? lx : 0);
  // Rows of the node box go to the waves round robin (row r = ly + NY lz to
  // wave r mod NW).  The row loops are specialised on the wave index, so every
  // row's local indices, LDS offset and boundary tests are compile-time
  // constants or single scalar operations.
  with_wave<NW>(__builtin_amdgcn_readfirstlane(t >> 6), [&](auto wc) {
    constexpr int W = decltype(wc)::value;
    T v[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = W + NW * k, ly = r % NY, lz = r / NY;
      v[k] = T(0);
      if (r < NR) {
        const uint32_t off = box_off + uint32_t(ly) * row_stride + uint32_t(lz) * plane_stride + lane_off;
        v[k] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(x) + off);
      }
    }
    if (lane_ok) {
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int r = W + NW * k, ly = r % NY, lz = r / NY;
        if (r < NR) {
          const bool rdir = (ly == 0 && first_y) || (ly == NY - 1 && last_y) || (lz == 0 && first_z) ||
                            (lz == NZ - 1 && last_z);
          buf[lds_lane + split_index<BZ>(lz) * PL + split_index<BY>(ly) * RX] = (rdir || xdir) ? T(0) : v[k];
        }
      }
    }
  });
  __syncthreads();
  const int cx = t % BX, cy = (t / BX) % BY, cz = t / (BX * BY);
  const int64_t cell = (int64_t(bx) * BX + cx) + int64_t(n) * ((int64_t(by) * BY + cy) + int64_t(n) * (int64_t(bz) * BZ + cz));
  auto zero_box = [&]() {
    constexpr int NV = (3 * CS * int(sizeof(T))) / 16;
    float4* b4 = reinterpret_cast<float4*>(buf);
    for (int e = t; e < NV; e += NT) b4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int e = NV * 16 / int(sizeof(T)) + t; e < 3 * CS; e += NT) buf[e] = T(0);
  };
  // the cell's results, one input component at a time from the box; then
  // the box is zeroed and takes the sums
  T U[3][27];
  const T mu_h = mu[cell] / T(n);
  cellop::apply_cell_by_input<T>(
      [&](int q, T(&V)[27]) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int off = split_index<BZ>(2 * cz + c) * PL + split_index<BY>(2 * cy + bb) * RX +
                              split_index<BX>(2 * cx + a);
              V[a + 3 * bb + 9 * c] = buf[q * CS + off];
            }
      },
      U, mu_h);
  __syncthreads();
  zero_box();
  __syncthreads();
  // phases: local nodes grouped by class (a in {0,1} | {2}) x (b ...) x (c ...); within a
  // class the map (cell, local node) -> node is injective, so read-add-write is race free;
  // c classes are separated by a block barrier (they couple waves), a/b classes by an
  // in-order LDS wait (they couple lanes of one wave).
#pragma unroll
  for (int cc = 0; cc < 2; ++cc) {
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) {
      const int ac = ab & 1, bc = ab >> 1;
      T tmp[3][2][2][2];
#pragma unroll
      for (int c = cc ? 2 : 0; c < (cc ? 3 : 2); ++c)
#pragma unroll
        for (int bb = bc ? 2 : 0; bb < (bc ? 3 : 2); ++bb)
#pragma unroll
          for (int a = ac ? 2 : 0; a < (ac ? 3 : 2); ++a) {
            const int off = split_index<BZ>(2 * cz + c) * PL + split_index<BY>(2 * cy + bb) * RX + split_index<BX>(2 * cx + a);
#pragma unroll
            for (int q = 0; q < 3; ++q) tmp[q][c & 1][bb & 1][a & 1] = buf[q * CS + off];
          }
#pragma unroll
      for (int c = cc ? 2 : 0; c < (cc ? 3 : 2); ++c)
#pragma unroll
        for (int bb = bc ? 2 : 0; bb < (bc ? 3 : 2); ++bb)
#pragma unroll
          for (int a = ac ? 2 : 0; a < (ac ? 3 : 2); ++a) {
            const int off = split_index<BZ>(2 * cz + c) * PL + split_index<BY>(2 * cy + bb) * RX + split_index<BX>(2 * cx + a);
#pragma unroll
            for (int q = 0; q < 3; ++q) buf[q * CS + off] = tmp[q][c & 1][bb & 1][a & 1] + U[q][a + 3 * bb + 9 * c];
          }
      __builtin_amdgcn_s_waitcnt(0xc07f);
      asm volatile("" ::: "memory");
    }
    __syncthreads();
  }
  const bool x_own = lx < NX - 1 || bx == nbx - 1;
  // Lanes of the x planes shared with a neighbour brick.  In the box layout of
  // the halo slot every such value would sit on a cache line of its own, so
  // they go to two packed planes ([NZ][NY][3]): the high plane's
  // contributions for the right neighbour, and the low plane's own (owned)
  // values, which the halo kernel completes and stores (accumulating, it
  // adds y).  The choice is a per-lane store address in the row loop below.
  const bool x_low = lx == 0 && bx > 0, x_high = lx == NX - 1 && bx < nbx - 1;
  T* slot = halo + int64_t(b) * halo_words<BX, BY, BZ>();
  T* plane = slot + halo_box_words<BX, BY, BZ>() + (x_high ? halo_plane_words<BX, BY, BZ>() : 0) + comp;
  T* hslot = slot + lane;
  // Owned nodes are stored (added to the old value when accumulating; x on
  // Dirichlet nodes, identity rows, otherwise), the high-face nodes of the
  // upper neighbours go to the halo slot, the shared x planes of owned rows
  // to the packed planes (Dirichlet rows of the low plane: identity rows,
  // stored).  Accumulating, every old value is read before the first store,
  // so their latency is paid once.
  with_wave<NW>(__builtin_amdgcn_readfirstlane(t >> 6), [&](auto wc) {
    constexpr int W = decltype(wc)::value;
    T old[ACC ? RPW : 1];
    if constexpr (ACC) {
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int r = W + NW * k, ly = r % NY, lz = r / NY;
        old[k] = T(0);
        if (r < NR) {
          const uint32_t off = box_off + uint32_t(ly) * row_stride + uint32_t(lz) * plane_stride + lane_off;
          old[k] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(y) + off);
        }
      }
    }
    if (lane_ok) {
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int r = W + NW * k, ly = r % NY, lz = r / NY;
        if (r < NR) {
          const bool rdir = (ly == 0 && first_y) || (ly == NY - 1 && last_y) || (lz == 0 && first_z) ||
                            (lz == NZ - 1 && last_z);
          const bool row_own = (ly < NY - 1 || last_y) && (lz < NZ - 1 || last_z);
          const uint32_t off = box_off + uint32_t(ly) * row_stride + uint32_t(lz) * plane_stride + lane_off;
          const T val = buf[lds_lane + split_index<BZ>(lz) * PL + split_index<BY>(ly) * RX];
          if (row_own && (x_high || (x_low && !rdir))) {
            plane[(lz * NY + ly) * 3] = val;
          } else if (row_own && x_own) {
            T out;
            if constexpr (ACC) {
              out = (rdir || xdir) ? old[k] : old[k] + val;
            } else {
              out = val;
              if (rdir || xdir) out = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(x) + off);
            }
            *reinterpret_cast<T*>(reinterpret_cast<char*>(y) + off) = out;
          } else {
            hslot[(lz * NY + ly) * ROW] = val;
          }
        }
      }
    }
  });
}

// Adds the halo values of a node's lower neighbour bricks into the node, for
// every free node on a low face of its owner brick.  One workgroup per
// brick; its low-face nodes are enumerated as the z-face (lz = 0), then the
// y-face without it, then the x-face without both, thread t taking
// component t mod 3 of node t / 3 (consecutive threads, consecutive words).
// A low x-plane node of a brick that is not the first along x holds its
// own value in the brick's packed low plane (y is then written without being
// read, unless accumulating), and its x neighbour's contribution in that
// neighbour's packed high plane.
template <typename T, int BX, int BY, int BZ>
__global__ __launch_bounds__(256) void k_brick_halo_add(int n, bool accumulate, const T* __restrict__ halo,
                                                        T* __restrict__ y) {
  constexpr int NX = 2 * BX + 1, NY = 2 * BY + 1, NZ = 2 * BZ + 1, ROW = 3 * NX;
  constexpr int MAXN = NX * NY + NX * (NZ - 1) + (NY - 1) * (NZ - 1);   // low-face nodes, at most
  constexpr int KT = (3 * MAXN + 255) / 256;                             // items per thread
  const int nbx = n / BX, nby = n / BY, nbz = n / BZ;
  const int b = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int m = 2 * n + 1;
  const int X0 = 2 * BX * bx, Y0 = 2 * BY * by, Z0 = 2 * BZ * bz;
  // owned local extents: [0, e) along each axis
  const int ex = bx == nbx - 1 ? NX : NX - 1, ey = by == nby - 1 ? NY : NY - 1, ez = bz == nbz - 1 ? NZ : NZ - 1;
  const int y1 = bz > 0 ? 1 : 0, x1 = by > 0 ? 1 : 0;
  const int fz = bz > 0 ? ex * ey : 0;
  const int fy = by > 0 ? ex * (ez - y1) : 0;
  const int fx = bx > 0 ? (ey - x1) * (ez - y1) : 0;
  const int total = 3 * (fz + fy + fx);
  // every load of a thread's items is issued before its first store, without
  // branches: reads that do not apply go to the zero pad after the last slot
  const T* zero = halo + int64_t(nbx) * nby * nbz * halo_words<BX, BY, BZ>();
  T acc[KT], cur[KT];
  int64_t dst[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int t = threadIdx.x + 256 * k;
    acc[k] = T(0), cur[k] = T(0), dst[k] = -1;
    const int tt = t < total ? t : 0;   // items past the end are dead (read the pad, store nothing)
    const int i = tt / 3, comp = tt - 3 * i;
    int lx, ly, lz;
    if (i < fz) {
      lz = 0, ly = i / ex, lx = i - ly * ex;
    } else if (i < fz + fy) {
      const int j = i - fz;
      ly = 0, lz = y1 + j / ex, lx = j % ex;
    } else {
      const int j = i - fz - fy, wd = ey - x1;
      lx = 0, lz = y1 + j / wd, ly = x1 + j % wd;
    }
    const int X = X0 + lx, Y = Y0 + ly, Z = Z0 + lz;
    const bool live = t < total && !(X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1);
    const bool lowx = live && lx == 0 && bx > 0, lowy = live && ly == 0 && by > 0, lowz = live && lz == 0 && bz > 0;
    constexpr int64_t HB = halo_box_words<BX, BY, BZ>(), HP = halo_plane_words<BX, BY, BZ>();
#pragma unroll
    for (int s = 1; s < 8; ++s) {
      const int sx = s & 1, sy = (s >> 1) & 1, sz = s >> 2;
      const bool use = !((sx && !lowx) || (sy && !lowy) || (sz && !lowz));
      const int64_t nb = (bx - sx) + int64_t(nbx) * ((by - sy) + int64_t(nby) * (bz - sz));
      const int qx = sx ? 2 * BX : lx, qy = sy ? 2 * BY : ly, qz = sz ? 2 * BZ : lz;
      const T* src = s == 1 ? halo + nb * halo_words<BX, BY, BZ>() + HB + HP + (int64_t(lz) * NY + ly) * 3 + comp
                            : halo + nb * halo_words<BX, BY, BZ>() + (int64_t(qz) * NY + qy) * ROW + 3 * qx + comp;
      acc[k] += *(use ? src : zero);
    }
    const bool packed = lx == 0 && bx > 0;
    const T* own = halo + int64_t(b) * halo_words<BX, BY, BZ>() + HB + (int64_t(lz) * NY + ly) * 3 + comp;
    acc[k] += *(live && packed ? own : zero);
    const int64_t d = 3 * (X + int64_t(m) * (Y + int64_t(m) * Z)) + comp;
    dst[k] = live ? d : -1;
    cur[k] = *(live && (!packed || accumulate) ? y + d : zero);
  }
#pragma unroll
  for (int k = 0; k < KT; ++k)
    if (dst[k] >= 0) y[dst[k]] = cur[k] + acc[k];
}

}  // namespace brick
}  // namespace mfgmg
