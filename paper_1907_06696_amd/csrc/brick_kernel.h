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
  // Cell rows are dealt to the 8-lane groups of a z-plane two apart (8 x 8
  // cells: lanes 0-31 take rows 0, 2, 4, 6 and lanes 32-63 rows 1, 3, 5, 7;
  // 8 x 4: rows 0, 2, 1, 3): with the row pitch of 20 the LDS rows that one
  // pass of a gather serves (16 lanes of 8-byte or 32 lanes of 4-byte words)
  // then start 8 doubles or 8 floats apart, on disjoint banks, where
  // consecutive rows (20 words apart) shared half their banks.
  const int grp = (t / BX) % BY;
  const int cx = t % BX, cy = 2 * (grp % (BY / 2)) + grp / (BY / 2), cz = t / (BX * BY);
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
// every free node on a low face of its owner brick.  A brick's low-face
// nodes fall into classes by which local indices are 0: the interiors of
// its z, y and x faces (local indices 1 .. 2B - 1 along the other two axes;
// the closing planes of the last bricks are Dirichlet), whose nodes have one
// lower neighbour each, and the three edges with the corner.  Items are
// (node, component) pairs, component fastest; each wave takes 64 items of
// one class, so a face wave issues only the loads its class needs (the
// neighbour's value and y; on the x face the two packed planes), and only
// the edge waves read all seven neighbours, branch free (reads that do not
// apply go to the zero pad after the last slot).  A low x-plane node of a
// brick that is not the first along x holds its own value in the brick's
// packed low plane (y is written without being read, unless accumulating),
// and its x neighbour's contribution in that neighbour's packed high plane.
// Sums are formed in the order neighbours s = 1 .. 7 (bit x, y, z of s:
// shifted by one brick along that axis), own plane, then y.
template <int BX, int BY, int BZ>
struct HaloClasses {
  static constexpr int IX = 2 * BX - 1, IY = 2 * BY - 1, IZ = 2 * BZ - 1;
  static constexpr int NE = IZ + IX + IY + 1;                       // edge and corner nodes
  static constexpr int CZ = (3 * IX * IY + 63) / 64, CY = (3 * IX * IZ + 63) / 64;
  static constexpr int CX = (3 * IY * IZ + 63) / 64, CE = (3 * NE + 63) / 64;
  static constexpr int waves = CZ + CY + CX + CE;                    // per brick
  static constexpr int groups = (waves + 3) / 4;                     // workgroups of 4 waves per brick
};

template <typename T, int BX, int BY, int BZ>
__global__ __launch_bounds__(256) void k_brick_halo_add(int n, bool accumulate, const T* __restrict__ halo,
                                                        T* __restrict__ y) {
  using HC = HaloClasses<BX, BY, BZ>;
  constexpr int NY = 2 * BY + 1, ROW = 3 * (2 * BX + 1);
  constexpr int64_t HW = halo_words<BX, BY, BZ>(), HB = halo_box_words<BX, BY, BZ>();
  constexpr int64_t HP = halo_plane_words<BX, BY, BZ>();
  const int nbx = n / BX, nby = n / BY;
  const int64_t g = xcd_order(blockIdx.x, gridDim.x);
  const int b = int(g / HC::groups);
  const int wave = int(g % HC::groups) * 4 + __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int m = 2 * n + 1;
  const int X0 = 2 * BX * bx, Y0 = 2 * BY * by, Z0 = 2 * BZ * bz;
  auto dst = [&](int lx, int ly, int lz, int comp) {
    return 3 * (int64_t(X0 + lx) + int64_t(m) * (int64_t(Y0 + ly) + int64_t(m) * (Z0 + lz))) + comp;
  };
  if (wave < HC::CZ) {   // z face: lower neighbour along z, its high z rows
    const int item = wave * 64 + lane;
    if (bz == 0 || item >= 3 * HC::IX * HC::IY) return;
    const int k = item / 3, comp = item - 3 * k;
    const int lx = 1 + k % HC::IX, ly = 1 + k / HC::IX;
    const int64_t nb = b - int64_t(nbx) * nby, d = dst(lx, ly, 0, comp);
    const T h = halo[nb * HW + (int64_t(2 * BZ) * NY + ly) * ROW + 3 * lx + comp];
    y[d] = y[d] + h;
  } else if (wave < HC::CZ + HC::CY) {   // y face: lower neighbour along y, its high y rows
    const int item = (wave - HC::CZ) * 64 + lane;
    if (by == 0 || item >= 3 * HC::IX * HC::IZ) return;
    const int k = item / 3, comp = item - 3 * k;
    const int lx = 1 + k % HC::IX, lz = 1 + k / HC::IX;
    const int64_t nb = b - nbx, d = dst(lx, 0, lz, comp);
    const T h = halo[nb * HW + (int64_t(lz) * NY + 2 * BY) * ROW + 3 * lx + comp];
    y[d] = y[d] + h;
  } else if (wave < HC::CZ + HC::CY + HC::CX) {   // x face: the packed planes
    const int item = (wave - HC::CZ - HC::CY) * 64 + lane;
    if (bx == 0 || item >= 3 * HC::IY * HC::IZ) return;
    const int k = item / 3, comp = item - 3 * k;
    const int ly = 1 + k % HC::IY, lz = 1 + k / HC::IY;
    const int64_t pl = (int64_t(lz) * NY + ly) * 3 + comp, d = dst(0, ly, lz, comp);
    const T acc = halo[(b - 1) * HW + HB + HP + pl] + halo[b * HW + HB + pl];
    const T cur = accumulate ? y[d] : T(0);
    y[d] = cur + acc;
  } else {   // edges (lx = ly = 0; ly = lz = 0; lx = lz = 0) and the corner
    const int item = (wave - HC::CZ - HC::CY - HC::CX) * 64 + lane;
    if (item >= 3 * HC::NE) return;
    const int k = item / 3, comp = item - 3 * k;
    int lx = 0, ly = 0, lz = 0;
    if (k < HC::IZ) lz = 1 + k;
    else if (k < HC::IZ + HC::IX) lx = 1 + (k - HC::IZ);
    else if (k < HC::IZ + HC::IX + HC::IY) ly = 1 + (k - HC::IZ - HC::IX);
    // a local index 0 of the first brick along that axis is a Dirichlet node
    if ((lx == 0 && bx == 0) || (ly == 0 && by == 0) || (lz == 0 && bz == 0)) return;
    const bool lowx = lx == 0, lowy = ly == 0, lowz = lz == 0;
    const T* zero = halo + int64_t(nbx) * nby * (n / BZ) * HW;
    T acc = T(0);
#pragma unroll
    for (int s = 1; s < 8; ++s) {
      const int sx = s & 1, sy = (s >> 1) & 1, sz = s >> 2;
      const bool use = !((sx && !lowx) || (sy && !lowy) || (sz && !lowz));
      const int64_t nb = (bx - sx) + int64_t(nbx) * ((by - sy) + int64_t(nby) * (bz - sz));
      const int qx = sx ? 2 * BX : lx, qy = sy ? 2 * BY : ly, qz = sz ? 2 * BZ : lz;
      const T* src = s == 1 ? halo + nb * HW + HB + HP + (int64_t(lz) * NY + ly) * 3 + comp
                            : halo + nb * HW + (int64_t(qz) * NY + qy) * ROW + 3 * qx + comp;
      acc += *(use ? src : zero);
    }
    acc += *(lowx ? halo + int64_t(b) * HW + HB + (int64_t(lz) * NY + ly) * 3 + comp : zero);
    const int64_t d = dst(lx, ly, lz, comp);
    const T cur = (!lowx || accumulate) ? y[d] : T(0);
    y[d] = cur + acc;
  }
}

}  // namespace brick
}  // namespace mfgmg
