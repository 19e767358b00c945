// C-ABI entry points and host drivers (V-cycle, eigenvalue estimate, FGMRES).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <unordered_map>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "q3.h"

#include "../../include/mfgmg.h"
#include "ctx.h"
#include "mesh.h"
#include "ops.h"

using namespace mfgmg;

namespace {

// ------------------------------------------------------------ element data
// Reference element on the unit cube (mu = 1), 3x3x3 Gauss quadrature:
//   K[(a,c),(b,d)] = int delta_cd grad phi_a . grad phi_b + d_d phi_a d_c phi_b
//   B[i,(b,d)]     = -int psi_i d_d phi_b,     M[i,j] = int psi_i psi_j
struct Element {
  double K[81 * 81];
  double B[8 * 81];
  double M[64];
  Element() {
    const double g = 0.5 * std::sqrt(3.0 / 5.0);
    const double xi[3] = {0.5 - g, 0.5, 0.5 + g};
    const double w1[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    std::memset(K, 0, sizeof K);
    std::memset(B, 0, sizeof B);
    std::memset(M, 0, sizeof M);
    double v[3][3], dv[3][3];   // [point][basis]
    for (int q = 0; q < 3; ++q) q2_basis_1d(xi[q], v[q]), q2_deriv_1d(xi[q], dv[q]);
    for (int qz = 0; qz < 3; ++qz)
      for (int qy = 0; qy < 3; ++qy)
        for (int qx = 0; qx < 3; ++qx) {
          const double w = w1[qx] * w1[qy] * w1[qz];
          double phi[27], gr[27][3], psi[8];
          for (int a = 0; a < 27; ++a) {
            const int i = a % 3, j = (a / 3) % 3, k = a / 9;
            phi[a] = v[qx][i] * v[qy][j] * v[qz][k];
            gr[a][0] = dv[qx][i] * v[qy][j] * v[qz][k];
            gr[a][1] = v[qx][i] * dv[qy][j] * v[qz][k];
            gr[a][2] = v[qx][i] * v[qy][j] * dv[qz][k];
          }
          for (int p = 0; p < 8; ++p) {
            const double tx = (p & 1) ? xi[qx] : 1 - xi[qx], ty = (p & 2) ? xi[qy] : 1 - xi[qy],
                         tz = (p & 4) ? xi[qz] : 1 - xi[qz];
            psi[p] = tx * ty * tz;
          }
          for (int a = 0; a < 27; ++a)
            for (int b = 0; b < 27; ++b) {
              const double lap = gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2];
              for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d)
                  K[(3 * a + c) * 81 + 3 * b + d] += w * ((c == d ? lap : 0.0) + gr[a][d] * gr[b][c]);
            }
          for (int p = 0; p < 8; ++p) {
            for (int b = 0; b < 27; ++b)
              for (int d = 0; d < 3; ++d) B[p * 81 + 3 * b + d] -= w * psi[p] * gr[b][d];
            for (int r = 0; r < 8; ++r) M[p * 8 + r] += w * psi[p] * psi[r];
          }
        }
  }
};

const Element& element() {
  static const Element e;
  return e;
}

// ------------------------------------------------------------ SplitMix64
// Steele, Lea & Flood (2014): state += 0x9E3779B97F4A7C15, then the mixing
// function; counter-based use: value(c) = mix(c + seed * 0xD1B54A32D192ED03 + gamma)
double splitmix_value(uint64_t seed, uint64_t counter) {
  uint64_t z = counter + seed * 0xD1B54A32D192ED03ULL + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return 2.0 * (double(z >> 11) * 0x1.0p-53) - 1.0;
}

// largest eigenvalue of a symmetric tridiagonal matrix by Sturm bisection
double tridiag_max_eig(const std::vector<double>& d, const std::vector<double>& e) {
  const int n = int(d.size());
  double lo = d[0], hi = d[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {   // number of eigenvalues < x
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
      if (q == 0.0) q = 1e-300;
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) >= n) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// eigenvector of the largest eigenvalue of a symmetric tridiagonal matrix (cyclic
// Jacobi rotations on the dense matrix; sizes up to the Lanczos step count)
std::vector<double> tridiag_top_eigvec(const std::vector<double>& d, const std::vector<double>& e) {
  const int n = int(d.size());
  std::vector<double> a(size_t(n) * n, 0.0), v(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    a[size_t(i) * n + i] = d[size_t(i)];
    v[size_t(i) * n + i] = 1.0;
    if (i + 1 < n) a[size_t(i) * n + i + 1] = a[size_t(i + 1) * n + i] = e[size_t(i)];
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? tot : off) += a[size_t(i) * n + j] * a[size_t(i) * n + j];
    if (off <= 1e-30 * (tot + off)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[size_t(p) * n + q];
        if (apq == 0.0) continue;
        // rotation that zeroes a_pq: t = tan(phi) from cot(2 phi) = (a_qq - a_pp) / (2 a_pq)
        const double th = (a[size_t(q) * n + q] - a[size_t(p) * n + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = a[size_t(k) * n + p], akq = a[size_t(k) * n + q];
          a[size_t(k) * n + p] = c * akp - sn * akq;
          a[size_t(k) * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = a[size_t(p) * n + k], aqk = a[size_t(q) * n + k];
          a[size_t(p) * n + k] = c * apk - sn * aqk;
          a[size_t(q) * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[size_t(k) * n + p], vkq = v[size_t(k) * n + q];
          v[size_t(k) * n + p] = c * vkp - sn * vkq;
          v[size_t(k) * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  int best = 0;
  for (int i = 1; i < n; ++i)
    if (a[size_t(i) * n + i] > a[size_t(best) * n + best]) best = i;
  std::vector<double> out(static_cast<size_t>(n));
  for (int k = 0; k < n; ++k) out[size_t(k)] = v[size_t(k) * n + best];
  return out;
}

// Cholesky factorisation and inverse of a dense SPD matrix (row major)
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> Lm(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) s -= Lm[size_t(j) * n + k] * Lm[size_t(j) * n + k];
    if (!(s > 0)) return false;
    Lm[size_t(j) * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) t -= Lm[size_t(i) * n + k] * Lm[size_t(j) * n + k];
      Lm[size_t(i) * n + j] = t / Lm[size_t(j) * n + j];
    }
  }
  // columns of the inverse: solve L L^T x = e_c
  std::vector<double> inv(size_t(n) * n), y(static_cast<size_t>(n));
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= Lm[size_t(i) * n + k] * y[size_t(k)];
      y[size_t(i)] = t / Lm[size_t(i) * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = y[size_t(i)];
      for (int k = i + 1; k < n; ++k) t -= Lm[size_t(k) * n + i] * inv[size_t(k) * n + c];
      inv[size_t(i) * n + c] = t / Lm[size_t(i) * n + i];
    }
  }
  A.swap(inv);
  return true;
}

}  // namespace

namespace mfgmg {
namespace detail {

thread_local std::string g_last_error;

double splitmix_pm1(uint64_t seed, uint64_t counter) { return splitmix_value(seed, counter); }


// Device data of one level from its host mesh: node lists, cell tables and
// the operator's block partition (non-uniform levels; the leaf also keeps
// its cell tables and pressure blocks), transfers from the level below,
// brick halo slots (uniform levels), viscosity, inverse diagonal and work
// vectors (work = false: the operator data only).
int upload_level(mfgmg_ctx* ctx, const Level& h, LevelDev& d, bool leaf, bool top, bool transfers, bool work) {
  DevLevel& v = d.v;
  v.ell = h.ell;
  v.ncell = h.ncell;
  v.nnode = h.nnode;
  v.uniform = h.uniform;
  v.n_edge = h.n_edge;
  // constrained velocity dofs
  std::vector<int64_t> cons;
  for (int64_t i = 0; i < h.nnode; ++i)
    for (int c = 0; c < 3; ++c)
      if (!h.dof_free(i, c)) cons.push_back(3 * i + c);
  v.cons_dofs = ctx->upload(cons);
  v.n_cons = int64_t(cons.size());
  v.noflux = !h.fixmask.empty();
  if (v.noflux && h.nnode > int64_t(kSlotNodeMask))
    return ctx->set(MFGMG_ERR_MESH, "no-normal-flux levels are limited to 2^28 nodes");
  // a free slot with the node's fixed components in its top bits (no-normal-
  // flux levels; the slot itself otherwise)
  auto encode = [&](std::vector<int32_t> sl) {
    if (v.noflux)
      for (int32_t& x : sl)
        if (x >= 0) x |= int32_t(h.fixmask[size_t(x)]) << kSlotFixShift;
    return sl;
  };
  if (!h.uniform || leaf) {   // the leaf keeps cell tables for the pressure operators
    std::vector<int32_t> slots(static_cast<size_t>(27 * h.ncell));
    std::vector<int8_t> clev(static_cast<size_t>(h.ncell));
    std::vector<int32_t> reg, hang;
    for (int64_t c = 0; c < h.ncell; ++c) {
      bool hh = false;
      for (int a = 0; a < 27; ++a) {
        const int32_t n = h.cell_nodes[size_t(27 * c + a)];
        int32_t s = n;
        if (h.ntype[size_t(n)] == NODE_DIRICHLET) s = -1;
        else if (h.ntype[size_t(n)] == NODE_HANGING) s = -(2 + h.hang_index[size_t(n)]), hh = true;
        slots[size_t(27 * c + a)] = s;
      }
      clev[size_t(c)] = int8_t(h.clev[size_t(c)]);
      (hh ? hang : reg).push_back(int32_t(c));
    }
    v.slots = ctx->upload(encode(slots));
    v.clev = ctx->upload(clev);
    {
      std::vector<uint8_t> cm(static_cast<size_t>(h.nnode));
      for (int64_t i = 0; i < h.nnode; ++i) cm[size_t(i)] = h.cmask(i);
      v.cmask = ctx->upload(cm);
    }
    v.reg_cells = ctx->upload(reg);
    v.n_reg_cells = int64_t(reg.size());
    v.hang_cells = ctx->upload(hang);
    v.n_hang_cells = int64_t(hang.size());
    // operator partition into 4^3 blocks, then 2^3 blocks, then single cells
    {
      std::unordered_map<uint64_t, int32_t> at;
      at.reserve(size_t(h.ncell));
      auto code = [](int l, int64_t i, int64_t j, int64_t k) {
        return (uint64_t(l) << 58) | (uint64_t(i) << 38) | (uint64_t(j) << 19) | uint64_t(k);
      };
      for (int64_t c = 0; c < h.ncell; ++c)
        at.emplace(code(h.clev[size_t(c)], h.cijk[size_t(3 * c)], h.cijk[size_t(3 * c + 1)],
                        h.cijk[size_t(3 * c + 2)]),
                   int32_t(c));
      std::vector<char> used(static_cast<size_t>(h.ncell), 0);
      // A block keeps, per hanging lattice point, its masters as lattice
      // points of the same block (a hanging node lies on the face shared with
      // a coarser cell, whose face nodes are all on the block's lattice);
      // blocks where that fails are left to the single-cell kernel.
      struct Blocks {
        std::vector<int32_t> slots, cells, hoff{0}, hent;
        std::vector<double> hw;
        std::vector<int32_t> pslots, phoff{0}, phent;   // leaf: Q1 pressure lattice
        std::vector<double> phw;
      };
      auto make_blocks = [&](int B, Blocks& out) {
        const int E = 2 * B + 1, NC = B * B * B, P = E * E * E, NB = 64 / NC;
        std::vector<int32_t> cs(static_cast<size_t>(NC)), bs(static_cast<size_t>(P));
        std::unordered_map<int32_t, int32_t> at_node;
        std::vector<int32_t> ent;
        std::vector<double> wt;
        for (int64_t c = 0; c < h.ncell; ++c) {
          const int l = h.clev[size_t(c)];
          const int64_t i = h.cijk[size_t(3 * c)], j = h.cijk[size_t(3 * c + 1)], k = h.cijk[size_t(3 * c + 2)];
          if (used[size_t(c)] || i % B || j % B || k % B || (int64_t(1) << l) < B) continue;
          bool ok = true;
          for (int q = 0; q < NC && ok; ++q) {
            auto it = at.find(code(l, i + q % B, j + (q / B) % B, k + q / (B * B)));
            ok = it != at.end() && !used[size_t(it->second)];
            if (ok) cs[size_t(q)] = it->second;
          }
          if (!ok) continue;
          for (int q = 0; q < NC; ++q) {
            const int qa = q % B, qb = (q / B) % B, qc = q / (B * B);
            for (int a = 0; a < 27; ++a) {
              const int p = (2 * qa + a % 3) + E * ((2 * qb + (a / 3) % 3) + E * (2 * qc + a / 9));
              bs[size_t(p)] = slots[size_t(27 * int64_t(cs[size_t(q)]) + a)];
            }
          }
          at_node.clear();
          for (int p = 0; p < P; ++p)
            if (bs[size_t(p)] >= 0) at_node[bs[size_t(p)]] = p;
          ent.clear();
          wt.clear();
          const int32_t bl = int32_t((out.cells.size() / size_t(NC)) % size_t(NB));
          for (int p = 0; p < P && ok; ++p) {
            if (bs[size_t(p)] >= -1) continue;
            const int64_t hr = -int64_t(bs[size_t(p)]) - 2;
            for (int64_t q = h.hang.ptr[size_t(hr)]; q < h.hang.ptr[size_t(hr + 1)] && ok; ++q) {
              auto it = at_node.find(h.hang.master[size_t(q)]);
              ok = it != at_node.end();
              if (ok) {
                ent.push_back(p | (it->second << 10) | (bl << 20));
                wt.push_back(h.hang.weight[size_t(q)]);
              }
            }
          }
          if (!ok) continue;
          // leaf: the pressure lattice of the block, hanging masters on it as well
          std::vector<int32_t> pb;
          std::vector<int32_t> pent;
          std::vector<double> pwt;
          if (leaf) {
            const int EP = B + 1, PP = EP * EP * EP;
            pb.assign(size_t(PP), -1);
            for (int q = 0; q < NC; ++q) {
              const int qa = q % B, qb = (q / B) % B, qc = q / (B * B);
              for (int a = 0; a < 8; ++a) {
                const int pp = (qa + a % 2) + EP * ((qb + (a / 2) % 2) + EP * (qc + a / 4));
                pb[size_t(pp)] = h.cell_pnodes[size_t(8 * int64_t(cs[size_t(q)]) + a)];
              }
            }
            std::unordered_map<int32_t, int32_t> pat;
            for (int pp = 0; pp < PP; ++pp)
              if (h.ptype[size_t(pb[size_t(pp)])] != NODE_HANGING) pat[pb[size_t(pp)]] = pp;
            for (int pp = 0; pp < PP && ok; ++pp) {
              const int32_t nd = pb[size_t(pp)];
              if (h.ptype[size_t(nd)] != NODE_HANGING) continue;
              const int32_t hr = h.phang_index[size_t(nd)];
              for (int64_t q = h.phang.ptr[size_t(hr)]; q < h.phang.ptr[size_t(hr) + 1] && ok; ++q) {
                auto it = pat.find(h.phang.master[size_t(q)]);
                ok = it != pat.end();
                if (ok) {
                  pent.push_back(pp | (it->second << 10) | (bl << 20));
                  pwt.push_back(h.phang.weight[size_t(q)]);
                }
              }
              pb[size_t(pp)] = -2;
            }
            if (!ok) continue;
          }
          for (int q = 0; q < NC; ++q) {
            used[size_t(cs[size_t(q)])] = 1;
            out.cells.push_back(cs[size_t(q)]);
          }
          if (leaf) {
            out.pslots.insert(out.pslots.end(), pb.begin(), pb.end());
            out.phent.insert(out.phent.end(), pent.begin(), pent.end());
            out.phw.insert(out.phw.end(), pwt.begin(), pwt.end());
            out.phoff.push_back(int32_t(out.phent.size()));
          }
          for (int p = 0; p < P; ++p) out.slots.push_back(bs[size_t(p)] < -1 ? -2 : bs[size_t(p)]);
          out.hent.insert(out.hent.end(), ent.begin(), ent.end());
          out.hw.insert(out.hw.end(), wt.begin(), wt.end());
          out.hoff.push_back(int32_t(out.hent.size()));
        }
      };
      Blocks b4, b2;
      std::vector<int32_t> sreg, shang;
      make_blocks(4, b4);
      make_blocks(2, b2);
      for (int64_t c = 0; c < h.ncell; ++c) {
        if (used[size_t(c)]) continue;
        bool hh = false;
        for (int a = 0; a < 27; ++a) hh = hh || slots[size_t(27 * c + a)] < -1;
        (hh ? shang : sreg).push_back(int32_t(c));
      }
      auto upload_blocks = [&](const Blocks& b, DevBlocks& d, int NC) {
        d.slots = ctx->upload(encode(b.slots));
        d.cells = ctx->upload(b.cells);
        d.n = int64_t(b.cells.size() / size_t(NC));
        d.hoff = ctx->upload(b.hoff);
        d.hent = ctx->upload(b.hent);
        d.hw_d = ctx->upload(b.hw);
        d.hw_f = ctx->upload(std::vector<float>(b.hw.begin(), b.hw.end()));
        // per workgroup (64 / NC blocks): the hanging entries grouped by
        // hanging point (consecutive already) and, reordered, by master, so
        // that one lane sums each group (no LDS atomics)
        {
          const int64_t NBW = 64 / NC, nwg = (d.n + NBW - 1) / NBW;
          std::vector<int32_t> g1off{0}, g1, g2off{0}, g2, hent2(b.hent.size()), idx;
          std::vector<double> hw2(b.hw.size());
          for (int64_t g = 0; g < nwg; ++g) {
            const int32_t h0 = b.hoff[size_t(g * NBW)], h1 = b.hoff[size_t(std::min(d.n, (g + 1) * NBW))];
            constexpr int32_t kMasterBits = 1023 << 10;   // entry = p | pm << 10 | block << 20
            for (int32_t e = h0; e < h1; ++e)
              if (e == h0 || (b.hent[size_t(e)] & ~kMasterBits) != (b.hent[size_t(e - 1)] & ~kMasterBits))
                g1.push_back(e);
            g1.push_back(h1);
            g1off.push_back(int32_t(g1.size()));
            idx.resize(size_t(h1 - h0));
            for (int32_t e = h0; e < h1; ++e) idx[size_t(e - h0)] = e;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int32_t u, int32_t v) { return (b.hent[size_t(u)] >> 10) < (b.hent[size_t(v)] >> 10); });
            for (int32_t e = h0; e < h1; ++e) {
              hent2[size_t(e)] = b.hent[size_t(idx[size_t(e - h0)])];
              hw2[size_t(e)] = b.hw[size_t(idx[size_t(e - h0)])];
            }
            for (int32_t e = h0; e < h1; ++e)
              if (e == h0 || (hent2[size_t(e)] >> 10) != (hent2[size_t(e - 1)] >> 10)) g2.push_back(e);
            g2.push_back(h1);
            g2off.push_back(int32_t(g2.size()));
          }
          d.g1off = ctx->upload(g1off);
          d.g1 = ctx->upload(g1);
          d.g2off = ctx->upload(g2off);
          d.g2 = ctx->upload(g2);
          d.hent2 = ctx->upload(hent2);
          d.hw2_d = ctx->upload(hw2);
          d.hw2_f = ctx->upload(std::vector<float>(hw2.begin(), hw2.end()));
        }
        if (leaf) {
          d.pslots = ctx->upload(b.pslots);
          d.phoff = ctx->upload(b.phoff);
          d.phent = ctx->upload(b.phent);
          d.phw = ctx->upload(b.phw);
        }
      };
      upload_blocks(b4, v.blk4, 64);
      upload_blocks(b2, v.blk2, 8);
      // face gather: every free face point of a block -> its slot, grouped by node
      {
        std::vector<std::pair<int32_t, int32_t>> nf;   // (node, slot)
        auto faces = [&](const Blocks& b, int B, int64_t slot0) {
          const int E = 2 * B + 1, P = E * E * E, NC = B * B * B;
          const int64_t nb = int64_t(b.cells.size() / size_t(NC));
          for (int64_t k = 0; k < nb; ++k)
            for (int p = 0; p < P; ++p) {
              const int px = p % E, py = (p / E) % E, pz = p / (E * E);
              const bool inner = px > 0 && px < E - 1 && py > 0 && py < E - 1 && pz > 0 && pz < E - 1;
              const int32_t nd = b.slots[size_t(k * P + p)];
              if (!inner && nd >= 0) nf.emplace_back(nd, int32_t(slot0 + k * P + p));
            }
          return slot0 + nb * P;
        };
        const int64_t s2 = faces(b4, 4, 0);
        const int64_t ns = faces(b2, 2, s2);
        std::sort(nf.begin(), nf.end());
        std::vector<int32_t> fnode, fptr{0}, fent;
        for (size_t i = 0; i < nf.size(); ++i) {
          if (i == 0 || nf[i].first != nf[i - 1].first) {
            if (i) fptr.push_back(int32_t(fent.size()));
            fnode.push_back(nf[i].first);
          }
          fent.push_back(nf[i].second);
        }
        if (!nf.empty()) fptr.push_back(int32_t(fent.size()));
        v.fslot_blk2 = s2;
        v.n_face = int64_t(fnode.size());
        if (v.n_face) {
          v.face_node = ctx->upload(fnode);
          v.face_ptr = ctx->upload(fptr);
          v.face_ent = ctx->upload(fent);
          v.fslot_f = ctx->dalloc<float>(size_t(3 * ns));
          v.fslot_d = ctx->dalloc<double>(size_t(3 * ns));
          if (!v.fslot_f || !v.fslot_d) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
        }
      }
      // the same for the pressure mass blocks of the leaf ((B+1)^3 Q1 lattices)
      if (leaf) {
        std::vector<std::pair<int32_t, int32_t>> nf;
        auto faces = [&](const Blocks& b, int B, int64_t slot0) {
          const int E = B + 1, P = E * E * E, NC = B * B * B;
          const int64_t nb = int64_t(b.cells.size() / size_t(NC));
          for (int64_t k = 0; k < nb; ++k)
            for (int p = 0; p < P; ++p) {
              const int px = p % E, py = (p / E) % E, pz = p / (E * E);
              const bool inner = px > 0 && px < E - 1 && py > 0 && py < E - 1 && pz > 0 && pz < E - 1;
              const int32_t nd = b.pslots[size_t(k * P + p)];
              if (!inner && nd >= 0) nf.emplace_back(nd, int32_t(slot0 + k * P + p));
            }
          return slot0 + nb * P;
        };
        const int64_t s2 = faces(b4, 4, 0);
        const int64_t ns = faces(b2, 2, s2);
        std::sort(nf.begin(), nf.end());
        std::vector<int32_t> fnode, fptr{0}, fent;
        for (size_t i = 0; i < nf.size(); ++i) {
          if (i && nf[i].first != nf[i - 1].first) fptr.push_back(int32_t(fent.size()));
          if (i == 0 || nf[i].first != nf[i - 1].first) fnode.push_back(nf[i].first);
          fent.push_back(nf[i].second);
        }
        if (!nf.empty()) fptr.push_back(int32_t(fent.size()));
        v.pfslot_blk2 = s2;
        v.n_pface = int64_t(fnode.size());
        if (v.n_pface) {
          v.pface_node = ctx->upload(fnode);
          v.pface_ptr = ctx->upload(fptr);
          v.pface_ent = ctx->upload(fent);
          v.pfslot = ctx->dalloc<double>(size_t(ns));
          if (!v.pfslot) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
        }
      }
      v.single_reg = ctx->upload(sreg);
      v.n_single_reg = int64_t(sreg.size());
      v.single_hang = ctx->upload(shang);
      v.n_single_hang = int64_t(shang.size());
    }
    v.hptr = ctx->upload(h.hang.ptr);
    v.hmaster = ctx->upload(h.hang.master);
    v.hw_d = ctx->upload(h.hang.weight);
    std::vector<float> wf(h.hang.weight.begin(), h.hang.weight.end());
    v.hw_f = ctx->upload(wf);
    v.hnode = ctx->upload(h.hang.node);
    v.nhang = int64_t(h.hang.count());
  }
  if (transfers) {
    d.P_ptr = ctx->upload(h.P_ptr);
    d.P_col = ctx->upload(h.P_col);
    d.P_w = ctx->upload(std::vector<float>(h.P_w.begin(), h.P_w.end()));
    d.R_ptr = ctx->upload(h.R_ptr);
    d.R_col = ctx->upload(h.R_col);
    d.R_w = ctx->upload(std::vector<float>(h.R_w.begin(), h.R_w.end()));
  }
  if (h.uniform) {
    const int64_t wf = brick_halo_words<float>(h.n_edge), wd = brick_halo_words<double>(h.n_edge);
    if (wf) v.halo_f = ctx->dalloc<float>(size_t(wf));
    if (wd) v.halo_d = ctx->dalloc<double>(size_t(wd));
    if ((wf && !v.halo_f) || (wd && !v.halo_d)) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
    // the zero pad after the slots is read by the halo kernel and never written
    if (wf) HIPCHK(hipMemset(v.halo_f + (wf - 64), 0, 64 * sizeof(float)));
    if (wd) HIPCHK(hipMemset(v.halo_d + (wd - 64), 0, 64 * sizeof(double)));
  }
  if (!h.mu_src.empty()) d.mu_src = ctx->upload(h.mu_src);
  if (!work) return MFGMG_OK;   // an operator only (it shares the viscosity of another level)
  d.mu_d = ctx->dalloc<double>(size_t(h.ncell));
  d.mu_f = ctx->dalloc<float>(size_t(h.ncell));
  v.mu_d = d.mu_d;
  v.mu_f = d.mu_f;
  d.minv_d = ctx->dalloc<double>(size_t(3 * h.nnode));
  d.minv_f = ctx->dalloc<float>(size_t(3 * h.nnode));
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 5; ++k) {
      if (top && k < 2) continue;   // top-level b, x come from the caller
      d.work[p][k] = p == 0 ? static_cast<void*>(ctx->dalloc<float>(size_t(3 * h.nnode)))
                            : static_cast<void*>(ctx->dalloc<double>(size_t(3 * h.nnode)));
    }
  // the separable transfers' scratch: the smoother's r and d
  v.tr_s1_f = static_cast<float*>(d.work[0][2]);
  v.tr_s2_f = static_cast<float*>(d.work[0][3]);
  v.tr_s1_d = static_cast<double*>(d.work[1][2]);
  v.tr_s2_d = static_cast<double*>(d.work[1][3]);
  return MFGMG_OK;
}

// Device data of a Q3-Q2 lattice level: constrained-component masks and
// list, transfers (node-level CSR with FP64 weights), viscosity, inverse
// diagonal and work vectors; the Q3 kernels compute node indices from the
// lattice, so no cell tables are needed.
int upload_q3_level(mfgmg_ctx* ctx, const Level& h, LevelDev& d, bool top, const double* kdiag) {
  DevLevel& v = d.v;
  v.ell = h.ell;
  v.ncell = h.ncell;
  v.nnode = h.nnode;
  v.uniform = false;
  v.q3 = true;
  v.n_edge = h.n_edge;
  v.q3_kdiag = kdiag;
  std::vector<int64_t> cons;
  std::vector<uint8_t> cm(static_cast<size_t>(h.nnode));
  for (int64_t i = 0; i < h.nnode; ++i) {
    cm[size_t(i)] = h.cmask(i);
    for (int c = 0; c < 3; ++c)
      if (!h.dof_free(i, c)) cons.push_back(3 * i + c);
  }
  v.cmask = ctx->upload(cm);
  v.cons_dofs = ctx->upload(cons);
  v.n_cons = int64_t(cons.size());
  v.q3_halo_f = ctx->dalloc<float>(size_t(q3_halo_words(h.n_edge)));
  v.q3_halo_d = ctx->dalloc<double>(size_t(q3_halo_words(h.n_edge)));
  if (h.ell >= 2) {
    d.P_ptr = ctx->upload(h.P_ptr);
    d.P_col = ctx->upload(h.P_col);
    d.P_w = ctx->upload(std::vector<float>(h.P_w.begin(), h.P_w.end()));
    d.R_ptr = ctx->upload(h.R_ptr);
    d.R_col = ctx->upload(h.R_col);
    d.R_w = ctx->upload(std::vector<float>(h.R_w.begin(), h.R_w.end()));
    v.q3_Pw = ctx->upload(h.P_w);
    v.q3_Rw = ctx->upload(h.R_w);
    // the 1D factor and its transpose (CSR over coarse coordinates)
    const int64_t mf = 3 * h.n_edge + 1, mc = 3 * (h.n_edge / 2) + 1;
    std::vector<int32_t> rptr(size_t(mc + 1), 0), rcol;
    std::vector<double> rw;
    std::vector<std::vector<std::pair<int32_t, double>>> cols(static_cast<size_t>(mc));
    for (int64_t X = 0; X < mf; ++X)
      for (int j = 0; j < 4; ++j) {
        const double w = h.p1_w[size_t(4 * X + j)];
        if (w != 0.0) cols[size_t(h.p1_c0[size_t(X)] + j)].emplace_back(int32_t(X), w);
      }
    for (int64_t C = 0; C < mc; ++C) {
      for (const auto& e : cols[size_t(C)]) rcol.push_back(e.first), rw.push_back(e.second);
      rptr[size_t(C + 1)] = int32_t(rcol.size());
    }
    v.q3_pc0 = ctx->upload(h.p1_c0);
    v.q3_pw = ctx->upload(h.p1_w);
    v.q3_rptr = ctx->upload(rptr);
    v.q3_rcol = ctx->upload(rcol);
    v.q3_rw = ctx->upload(rw);
  }
  if (!h.mu_src.empty()) d.mu_src = ctx->upload(h.mu_src);
  d.mu_d = ctx->dalloc<double>(size_t(h.ncell));
  d.mu_f = ctx->dalloc<float>(size_t(h.ncell));
  v.mu_d = d.mu_d;
  v.mu_f = d.mu_f;
  d.minv_d = ctx->dalloc<double>(size_t(3 * h.nnode));
  d.minv_f = ctx->dalloc<float>(size_t(3 * h.nnode));
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 5; ++k) {
      if (top && k < 2) continue;
      d.work[p][k] = p == 0 ? static_cast<void*>(ctx->dalloc<float>(size_t(3 * h.nnode)))
                            : static_cast<void*>(ctx->dalloc<double>(size_t(3 * h.nnode)));
    }
  // the transfers' scratch: the smoother's r and d, dead while a transfer runs
  v.tr_s1_f = static_cast<float*>(d.work[0][2]);
  v.tr_s2_f = static_cast<float*>(d.work[0][3]);
  v.tr_s1_d = static_cast<double*>(d.work[1][2]);
  v.tr_s2_d = static_cast<double*>(d.work[1][3]);
  return MFGMG_OK;
}

int upload_mesh(mfgmg_ctx* ctx) {
  if (ctx->dev_ready) return MFGMG_OK;
  HIPCHK(hipGetDevice(&ctx->device));
  const Mesh& m = *ctx->mesh;
  const int L = m.L();
  ctx->lv.assign(size_t(L + 1), LevelDev{});
  const Element& E = element();
  double kd[81];
  for (int i = 0; i < 81; ++i) kd[i] = E.K[i * 81 + i];
  set_element_constants(kd, E.B, E.M);
  ctx->khat_d = ctx->upload(std::vector<double>(E.K, E.K + 81 * 81));
  if (m.velocity_degree() == 3) {
    // Q3-Q2: lattice levels, the pressure on the leaf's Q2 lattice (no constraints)
    const Q3Element& Q = q3_element();
    double N[16], D[16], P2[12], M2[9], kd[192];
    for (int q = 0; q < 4; ++q)
      for (int a = 0; a < 4; ++a) N[4 * q + a] = Q.N[q][a], D[4 * q + a] = Q.D[q][a];
    for (int q = 0; q < 4; ++q)
      for (int i = 0; i < 3; ++i) P2[3 * q + i] = Q.P2[q][i];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M2[3 * i + j] = Q.M2[i][j];
    for (int i = 0; i < 192; ++i) kd[i] = Q.K[size_t(i) * 192 + i];
    set_q3_constants(N, D, Q.wg, P2, M2);
    const double* kdiag = ctx->upload(std::vector<double>(kd, kd + 192));
    for (int ell = 1; ell <= L; ++ell) {
      const int st = upload_q3_level(ctx, m.vlevel(ell), ctx->lv[size_t(ell)], ell == L, kdiag);
      if (st) return st;
    }
    ctx->pres.np = m.vleaf().npnode;
  } else {
    for (int ell = 1; ell <= L; ++ell) {
      // between two uniform lattice levels the transfers run from the
      // lattice alone (k_prolong_uniform, k_restrict_x/y/z) unless the
      // restriction passes' 32-bit node indices overflow: no tables there
      bool csr = ell >= 2;
      if (csr && m.transfer_deferred(ell)) {
        const int64_t nc = m.level(ell - 1).n_edge, mc = 2 * nc + 1, mf = 4 * nc + 1;
        csr = mc * mf * mf >= (int64_t(1) << 31);
      }
      const Level& h = csr ? m.level_transfer(ell) : m.level(ell);
      const int st = upload_level(ctx, h, ctx->lv[size_t(ell)], ell == L, ell == L, csr, true);
      if (st) return st;
    }
  }
  // pressure on the leaf
  const Level& lf = m.vleaf();
  if (m.velocity_degree() == 2) {
    std::vector<int32_t> ps(static_cast<size_t>(8 * lf.ncell));
    for (int64_t c = 0; c < lf.ncell; ++c)
      for (int i = 0; i < 8; ++i) {
        const int32_t n = lf.cell_pnodes[size_t(8 * c + i)];
        ps[size_t(8 * c + i)] = lf.ptype[size_t(n)] == NODE_HANGING ? -(2 + lf.phang_index[size_t(n)]) : n;
      }
    ctx->pres.np = lf.npnode;
    ctx->pres.pslots = ctx->upload(ps);
    ctx->pres.hptr = ctx->upload(lf.phang.ptr);
    ctx->pres.hmaster = ctx->upload(lf.phang.master);
    ctx->pres.hw = ctx->upload(lf.phang.weight);
    ctx->pres.hang_nodes = ctx->upload(lf.phang.node);
    ctx->pres.nh = int64_t(lf.phang.count());
    if (lf.uniform) {
      // lattice -> pressure node, from the canonical keys (X + m (Y + m Z) on
      // the (2n+1)^3 Q2 lattice; Q1 nodes sit at even X, Y, Z)
      const int64_t n = lf.n_edge, mq = 2 * n + 1, np1 = n + 1;
      std::vector<int32_t> plat(static_cast<size_t>(np1 * np1 * np1), -1);
      for (int64_t i = 0; i < lf.npnode; ++i) {
        const int64_t k = lf.pkey[size_t(i)];
        const int64_t X = k % mq, Y = (k / mq) % mq, Z = k / (mq * mq);
        plat[size_t(X / 2 + np1 * (Y / 2 + np1 * (Z / 2)))] = int32_t(i);
      }
      for (const int32_t q : plat)
        if (q < 0) return ctx->set(MFGMG_ERR_MESH, "uniform leaf: a Q1 lattice point has no pressure node");
      ctx->pres.plat = ctx->upload(plat);
    }
  }
  // coarse level: free dofs of level 1
  {
    const Level& c1 = m.vlevel(1);
    std::vector<int32_t> fd;
    for (int64_t i = 0; i < c1.nnode; ++i)
      for (int c = 0; c < 3; ++c)
        if (c1.dof_free(i, c)) fd.push_back(int32_t(3 * i + c));
    ctx->ncfree = int(fd.size());
    if (ctx->ncfree > 375 || c1.ncell != 8) return ctx->set(MFGMG_ERR_MESH, "level 1 is not the 2x2x2 mesh");
    ctx->coarse_free = ctx->upload(fd);
    ctx->Ainv_d = ctx->dalloc<double>(size_t(ctx->ncfree) * ctx->ncfree);
    ctx->Ainv_f = ctx->dalloc<float>(size_t(ctx->ncfree) * ctx->ncfree);
  }
  ctx->red_part = ctx->dalloc<double>(size_t(kRedPartWords));
  ctx->red_res = ctx->dalloc<double>(512);
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&ctx->host_res), 512 * sizeof(double), hipHostMallocDefault));
  ctx->pmass_minv = ctx->dalloc<double>(size_t(lf.npnode));
  ctx->pmean_w = ctx->dalloc<double>(size_t(lf.npnode));
  for (void* p : ctx->allocs)
    if (!p) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
  HIPCHK(hipDeviceSynchronize());
  ctx->dev_ready = true;
  return MFGMG_OK;
}

double dot_sync(mfgmg_ctx* ctx, int64_t n, const double* a, const double* b, hipStream_t s) {
  // result slot 511: slots [0, 511) hold batched Gram-Schmidt coefficients
  launch_dot(n, a, b, ctx->red_part, ctx->red_res + 511, s);
  (void)hipMemcpyAsync(ctx->host_res + 511, ctx->red_res + 511, sizeof(double), hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
  return ctx->host_res[511];
}

template <typename T>
constexpr int prec_index() {
  return std::is_same<T, float>::value ? 0 : 1;
}

template <typename T>
const T* minv_of(const LevelDev& d);
template <>
const float* minv_of<float>(const LevelDev& d) {
  return d.minv_f;
}
template <>
const double* minv_of<double>(const LevelDev& d) {
  return d.minv_d;
}
template <typename T>
const T* minv_s_of(const LevelDev& d);
template <>
const float* minv_s_of<float>(const LevelDev& d) {
  return d.minv_s_f;
}
template <>
const double* minv_s_of<double>(const LevelDev& d) {
  return d.minv_s_d;
}

// Chebyshev smoothing (Saad, Alg. 12.1) on [lambda/15, lambda], M^{-1} = minv
template <typename T>
void smooth(mfgmg_ctx* ctx, int ell, const T* b, T* x, bool x_zero, hipStream_t s) {
  smooth_on<T>(ctx, ctx->lv[size_t(ell)], b, x, x_zero, s);
}

template <typename T>
void smooth_on(mfgmg_ctx* ctx, LevelDev& d, const T* b, T* x, bool x_zero, hipStream_t s) {
  // Chebyshev iteration (Saad, Alg. 12.1) with the residual formed as b - A x
  // at each step (the same iterates as the residual recurrence in exact
  // arithmetic; r is never stored)
  const int64_t n = 3 * d.v.nnode;
  T* dd = static_cast<T*>(d.work[prec_index<T>()][3]);
  T* t = static_cast<T*>(d.work[prec_index<T>()][4]);
  const bool sc = ctx->use_scaling && d.scaled;
  const T* minv = sc ? minv_s_of<T>(d) : minv_of<T>(d);
  const double lam = sc ? d.lambda_s : d.lambda, lo = lam / 15.0;
  const double theta = 0.5 * (lam + lo), delta = 0.5 * (lam - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  // where the operator starts with an output initialisation kernel, each
  // update prepares t for the next operator call on x instead (after the last
  // update of a pre-smoothing, for the V-cycle's residual)
  const bool prep = vmult_has_init<T>(d.v);
  ChebPrep cp;
  if (prep) {
    cp.tn = t;
    cp.cmask = d.v.uniform ? nullptr : d.v.cmask;
    cp.m = d.v.uniform ? 2 * d.v.n_edge + 1 : 0;
    cp.from_x = true;
  }
  if (x_zero) {
    launch_chebx_init0<T>(n, b, minv, dd, x, 1.0 / theta, s, cp);
  } else {
    launch_vmult<T>(d.v, x, t, s);
    launch_chebx_step<T>(n, b, t, minv, dd, x, 0.0, 1.0 / theta, s, cp);
  }
  for (int k = 1; k < 4; ++k) {
    if (prep) launch_vmult_prepared<T>(d.v, x, t, s);
    else launch_vmult<T>(d.v, x, t, s);
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    launch_chebx_step<T>(n, b, t, minv, dd, x, rho_new * rho, 2.0 * rho_new / delta, s,
                         k < 3 || x_zero ? cp : ChebPrep());
    rho = rho_new;
  }
}

template <typename T>
const T* ainv_of(mfgmg_ctx* ctx);
template <>
const float* ainv_of<float>(mfgmg_ctx* ctx) {
  return ctx->Ainv_f;
}
template <>
const double* ainv_of<double>(mfgmg_ctx* ctx) {
  return ctx->Ainv_d;
}

template <typename T>
void vcycle(mfgmg_ctx* ctx, int ell, const T* b, T* x, hipStream_t s) {
  if (ell == 1) {
    launch_coarse<T>(ainv_of<T>(ctx), ctx->coarse_free, ctx->ncfree, int(3 * ctx->lv[1].v.nnode), b, x, s);
    return;
  }
  LevelDev& d = ctx->lv[size_t(ell)];
  LevelDev& c = ctx->lv[size_t(ell - 1)];
  if (ell == 2) {   // the 4^3 level and the coarse solve in one workgroup, where it applies
    const bool sc = ctx->use_scaling && d.scaled;
    if (launch_vcycle_tail<T>(d.v, c.v, sc ? minv_s_of<T>(d) : minv_of<T>(d), ainv_of<T>(ctx), ctx->coarse_free,
                              ctx->ncfree, sc ? d.lambda_s : d.lambda, b, x, s))
      return;
  }
  const int pi = prec_index<T>();
  T* t = static_cast<T*>(d.work[pi][4]);
  T* bc = static_cast<T*>(c.work[pi][0]);
  T* xc = static_cast<T*>(c.work[pi][1]);
  smooth<T>(ctx, ell, b, x, true, s);
  // the pre-smoothing left t prepared for A x where the operator needs it
  if (vmult_has_init<T>(d.v)) launch_vmult_prepared<T>(d.v, x, t, s);
  else launch_vmult<T>(d.v, x, t, s);
  // the smoother's r and d are free here: scratch of the restriction passes
  launch_restrict_level<T>(d.v, c.v, d.R_ptr, d.R_col, d.R_w, b, t, bc, static_cast<T*>(d.work[pi][2]),
                           static_cast<T*>(d.work[pi][3]), s);
  vcycle<T>(ctx, ell - 1, bc, xc, s);
  launch_prolong_level<T>(d.v, c.v, d.P_ptr, d.P_col, d.P_w, xc, x, true, s);
  smooth<T>(ctx, ell, b, x, false, s);
}

// lambda_max of M^{-1} A by 12 steps of preconditioned CG-Lanczos (FP64)
int estimate_lambda(mfgmg_ctx* ctx, int ell, hipStream_t s) {
  LevelDev& d = ctx->lv[size_t(ell)];
  return lanczos_lambda(ctx, ell, d.minv_d, &d.lambda, s);
}

int lanczos_lambda(mfgmg_ctx* ctx, int ell, const double* minv, double* lam_out, hipStream_t s, double* basis,
                   double* ritz) {
  return lanczos_on(ctx, ctx->lv[size_t(ell)], ctx->mesh->vlevel(ell), minv, lam_out, s, basis, ritz);
}

// the same on any level: d its device data, h its host mesh (start vector over
// the free nodes of h by canonical key)
int lanczos_on(mfgmg_ctx* ctx, LevelDev& d, const Level& h, const double* minv, double* lam_out, hipStream_t s,
               double* basis, double* ritz) {
  const int64_t n = 3 * h.nnode;
  std::vector<double> r0(static_cast<size_t>(n));
  for (int64_t i = 0; i < h.nnode; ++i)
    for (int c = 0; c < 3; ++c)
      r0[size_t(3 * i + c)] = h.dof_free(i, c) ? splitmix_pm1(12345, uint64_t(3 * h.key[size_t(i)] + c)) : 0.0;
  double* r = static_cast<double*>(d.work[1][2]);
  double* z = static_cast<double*>(d.work[1][3]);
  double* q = static_cast<double*>(d.work[1][4]);
  if (!d.lz_p) d.lz_p = ctx->dalloc<double>(size_t(n));
  double* p = d.lz_p;
  if (!p) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
  HIPCHK(hipMemcpyAsync(r, r0.data(), size_t(n) * sizeof(double), hipMemcpyHostToDevice, s));
  launch_mul(n, minv, r, z, s);
  HIPCHK(hipMemcpyAsync(p, z, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  double rz = dot_sync(ctx, n, r, z, s);
  const double rz0 = rz;
  std::vector<double> alphas, betas;
  for (int it = 0; it < kLanczosSteps; ++it) {
    launch_vmult<double>(d.v, p, q, s);
    const double pq = dot_sync(ctx, n, p, q, s);
    if (!(pq > 0)) break;
    if (ritz) launch_scale_copy(n, (it % 2 ? -1.0 : 1.0) / std::sqrt(rz), z, basis + size_t(it) * size_t(n), s);
    const double alpha = rz / pq;
    alphas.push_back(alpha);
    launch_axpby(n, -alpha, q, 1.0, r, s);
    launch_mul(n, minv, r, z, s);
    const double rz_new = dot_sync(ctx, n, r, z, s);
    const double beta = rz_new / rz;
    if (rz_new <= 1e-30 * rz0) break;
    betas.push_back(beta);
    launch_axpby(n, 1.0, z, beta, p, s);
    rz = rz_new;
  }
  const int k = int(alphas.size());
  if (k == 0) return ctx->set(MFGMG_ERR_NOCONV, "eigenvalue estimate failed");
  std::vector<double> dg(static_cast<size_t>(k)), e(size_t(std::max(k - 1, 0)));
  for (int i = 0; i < k; ++i) {
    dg[size_t(i)] = 1.0 / alphas[size_t(i)] + (i > 0 ? betas[size_t(i - 1)] / alphas[size_t(i - 1)] : 0.0);
    if (i + 1 < k) e[size_t(i)] = std::sqrt(betas[size_t(i)]) / alphas[size_t(i)];
  }
  *lam_out = 1.2 * tridiag_max_eig(dg, e);
  if (ritz) {
    const std::vector<double> c = tridiag_top_eigvec(dg, e);
    launch_fill(n, 0.0, ritz, s);
    for (int i = 0; i < k; ++i) launch_axpby(n, c[size_t(i)], basis + size_t(i) * size_t(n), 1.0, ritz, s);
  }
  HIPCHK(hipStreamSynchronize(s));
  return MFGMG_OK;
}

int factor_coarse(mfgmg_ctx* ctx, hipStream_t s) {
  const Level& c1 = ctx->mesh->vlevel(1);
  std::vector<double> mu(static_cast<size_t>(c1.ncell));
  HIPCHK(hipMemcpyAsync(mu.data(), ctx->lv[1].mu_d, mu.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const Element& E = element();
  const int64_t n = 3 * c1.nnode;
  std::vector<double> A(size_t(n * n), 0.0);
  if (ctx->mesh->velocity_degree() == 3) {
    // Q3 level 1 (2 x 2 x 2 cells, 7^3 lattice nodes): mu_K h K_hat per cell
    const Q3Element& Q = q3_element();
    const int64_t m = 3 * c1.n_edge + 1;
    for (int64_t c = 0; c < c1.ncell; ++c) {
      const double sc = mu[size_t(c)] / double(c1.n_edge);
      const int64_t ci = c % c1.n_edge, cj = (c / c1.n_edge) % c1.n_edge, ck = c / (c1.n_edge * c1.n_edge);
      int64_t nd[64];
      for (int a = 0; a < 64; ++a)
        nd[a] = (3 * ci + a % 4) + m * ((3 * cj + (a / 4) % 4) + m * (3 * ck + a / 16));
      for (int a = 0; a < 192; ++a)
        for (int b = 0; b < 192; ++b)
          A[size_t((3 * nd[a / 3] + a % 3) * n + 3 * nd[b / 3] + b % 3)] += sc * Q.K[size_t(a) * 192 + b];
    }
  }
  for (int64_t c = 0; c < (ctx->mesh->velocity_degree() == 3 ? 0 : c1.ncell); ++c) {
    const double sc = mu[size_t(c)] * std::ldexp(1.0, -c1.clev[size_t(c)]);
    for (int a = 0; a < 27; ++a)
      for (int b = 0; b < 27; ++b)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            const int64_t ra = 3 * c1.cell_nodes[size_t(27 * c + a)] + i;
            const int64_t cb = 3 * c1.cell_nodes[size_t(27 * c + b)] + j;
            A[size_t(ra * n + cb)] += sc * E.K[(3 * a + i) * 81 + 3 * b + j];
          }
  }
  std::vector<int32_t> fd;
  for (int64_t i = 0; i < c1.nnode; ++i)
    for (int c = 0; c < 3; ++c)
      if (c1.dof_free(i, c)) fd.push_back(int32_t(3 * i + c));
  const int nf = int(fd.size());
  std::vector<double> Af(size_t(nf) * nf);
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < nf; ++j) Af[size_t(i) * nf + j] = A[size_t(fd[size_t(i)]) * n + fd[size_t(j)]];
  if (!spd_inverse(Af, nf)) return ctx->set(MFGMG_ERR_NOCONV, "coarse matrix is not positive definite");
  std::vector<float> Aff(Af.begin(), Af.end());
  HIPCHK(hipMemcpyAsync(ctx->Ainv_d, Af.data(), Af.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->Ainv_f, Aff.data(), Aff.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return MFGMG_OK;
}

// Jacobi preconditioner of M_p and the zero-mean weights (host, from leaf mu)
int pressure_setup(mfgmg_ctx* ctx, hipStream_t s) {
  if (ctx->mesh->velocity_degree() == 3) {
    // Q2 pressure on the (2n+1)^3 lattice: Jacobi from diag(M_p) (device),
    // mean weights int psi_j = h^3 (row sums of the 1D Q2 mass: 1/6, 2/3, 1/6)
    const Level& lf = ctx->mesh->vleaf();
    const DevLevel& v = ctx->lv[size_t(ctx->mesh->L())].v;
    const int64_t n = lf.n_edge, mp = 2 * n + 1;
    launch_fill(lf.npnode, 0.0, ctx->pmass_minv, s);
    launch_pmass_diag_q2(v, ctx->pmass_minv, s);
    std::vector<double> dg(static_cast<size_t>(lf.npnode));
    HIPCHK(hipMemcpyAsync(dg.data(), ctx->pmass_minv, dg.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (double& x : dg) x = 1.0 / x;
    const double h3 = 1.0 / double(n * n * n), rs[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    std::vector<double> mw(static_cast<size_t>(lf.npnode), 0.0);
    for (int64_t c = 0; c < lf.ncell; ++c) {
      const int64_t i = c % n, j = (c / n) % n, k = c / (n * n);
      for (int a = 0; a < 27; ++a)
        mw[size_t((2 * i + a % 3) + mp * ((2 * j + (a / 3) % 3) + mp * (2 * k + a / 9)))] +=
            h3 * rs[a % 3] * rs[(a / 3) % 3] * rs[a / 9];
    }
    double tot = 0.0;
    for (double x : mw) tot += x;
    ctx->pmean_total = tot;
    HIPCHK(hipMemcpyAsync(ctx->pmass_minv, dg.data(), dg.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->pmean_w, mw.data(), mw.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return MFGMG_OK;
  }
  const Level& lf = ctx->mesh->leaf();
  const Element& E = element();
  std::vector<double> mu(static_cast<size_t>(lf.ncell));
  HIPCHK(hipMemcpyAsync(mu.data(), ctx->lv[size_t(ctx->mesh->L())].mu_d, mu.size() * sizeof(double),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> dg(size_t(lf.npnode), 0.0), mw(size_t(lf.npnode), 0.0);
  for (int64_t c = 0; c < lf.ncell; ++c) {
    const double h = std::ldexp(1.0, -lf.clev[size_t(c)]);
    const double sm = h * h * h / mu[size_t(c)], sv = h * h * h;
    // expansion of each local Q1 node into free masters
    int ml[8][4];
    double wl[8][4];
    int nl[8];
    for (int i = 0; i < 8; ++i) {
      const int32_t n = lf.cell_pnodes[size_t(8 * c + i)];
      if (lf.ptype[size_t(n)] == NODE_HANGING) {
        const int32_t hh = lf.phang_index[size_t(n)];
        nl[i] = 0;
        for (int64_t q = lf.phang.ptr[size_t(hh)]; q < lf.phang.ptr[size_t(hh) + 1]; ++q)
          ml[i][nl[i]] = lf.phang.master[size_t(q)], wl[i][nl[i]] = lf.phang.weight[size_t(q)], ++nl[i];
      } else {
        ml[i][0] = n, wl[i][0] = 1.0, nl[i] = 1;
      }
    }
    for (int i = 0; i < 8; ++i) {
      double rs = 0.0;
      for (int j = 0; j < 8; ++j) rs += E.M[i * 8 + j];
      for (int a = 0; a < nl[i]; ++a) {
        mw[size_t(ml[i][a])] += sv * wl[i][a] * rs;
        // diagonal: pairs (i, j) sharing the master
        for (int j = 0; j < 8; ++j)
          for (int b = 0; b < nl[j]; ++b)
            if (ml[j][b] == ml[i][a]) dg[size_t(ml[i][a])] += sm * wl[i][a] * wl[j][b] * E.M[i * 8 + j];
      }
    }
  }
  double tot = 0.0;
  for (int64_t i = 0; i < lf.npnode; ++i) {
    if (lf.ptype[size_t(i)] == NODE_HANGING) dg[size_t(i)] = 1.0, mw[size_t(i)] = 0.0;
    dg[size_t(i)] = 1.0 / dg[size_t(i)];
    tot += mw[size_t(i)];
  }
  ctx->pmean_total = tot;
  HIPCHK(hipMemcpyAsync(ctx->pmass_minv, dg.data(), dg.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->pmean_w, mw.data(), mw.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return MFGMG_OK;
}

int check_level(const mfgmg_ctx* ctx, int32_t level) {
  if (!ctx || !ctx->mesh || !ctx->mesh->finalized()) return MFGMG_ERR_STATE;
  if (level < 1 || level > ctx->mesh->L()) return MFGMG_ERR_INVALID;
  return MFGMG_OK;
}

template void smooth<float>(mfgmg_ctx*, int, const float*, float*, bool, hipStream_t);
template void smooth<double>(mfgmg_ctx*, int, const double*, double*, bool, hipStream_t);
template void vcycle<float>(mfgmg_ctx*, int, const float*, float*, hipStream_t);
template void vcycle<double>(mfgmg_ctx*, int, const double*, double*, hipStream_t);
template void smooth_on<float>(mfgmg_ctx*, LevelDev&, const float*, float*, bool, hipStream_t);
template void smooth_on<double>(mfgmg_ctx*, LevelDev&, const double*, double*, bool, hipStream_t);

// the preconditioner's V-cycle: local smoothing or global coarsening
template <typename T>
void vcycle_of(mfgmg_ctx* ctx, bool local, int L, const T* b, T* x, hipStream_t s) {
  if (local) local_vcycle<T>(ctx, b, x, s);
  else vcycle<T>(ctx, L, b, x, s);
}

}  // namespace detail
}  // namespace mfgmg

using namespace mfgmg::detail;

// =================================================================== C ABI
extern "C" {

int mfgmg_create(int32_t base_level, mfgmg_ctx** out) {
  if (!out) return MFGMG_ERR_INVALID;
  *out = nullptr;
  if (base_level < 1 || base_level > MFGMG_MAX_LEVELS - 2) {
    g_last_error = "base_level out of range";
    return MFGMG_ERR_INVALID;
  }
  try {
    auto* c = new mfgmg_ctx;
    c->mesh = std::make_unique<Mesh>(base_level);
    *out = c;
  } catch (...) {
    g_last_error = "out of host memory";
    return MFGMG_ERR_NOMEM;
  }
  return MFGMG_OK;
}

int mfgmg_set_element(mfgmg_ctx* ctx, int32_t k) {
  if (!ctx) return MFGMG_ERR_INVALID;
  if (k != 1 && k != 2) return ctx->set(MFGMG_ERR_INVALID, "element: k = 1 (Q2-Q1) or k = 2 (Q3-Q2)");
  if (ctx->mesh->finalized()) return ctx->set(MFGMG_ERR_STATE, "mesh already finalized");
  ctx->mesh->set_velocity_degree(k + 1);
  return MFGMG_OK;
}

int mfgmg_set_boundary(mfgmg_ctx* ctx, int32_t bc) {
  if (!ctx) return MFGMG_ERR_INVALID;
  if (bc != MFGMG_BC_DIRICHLET && bc != MFGMG_BC_NOFLUX) return ctx->set(MFGMG_ERR_INVALID, "unknown boundary condition");
  if (ctx->mesh->finalized()) return ctx->set(MFGMG_ERR_STATE, "mesh already finalized");
  ctx->mesh->set_noflux(bc == MFGMG_BC_NOFLUX);
  return MFGMG_OK;
}

int mfgmg_refine(mfgmg_ctx* ctx, const int32_t* cells, int64_t n, int32_t levels_up) {
  if (!ctx || (!cells && n > 0) || n < 0) return MFGMG_ERR_INVALID;
  if (ctx->mesh->finalized()) return ctx->set(MFGMG_ERR_STATE, "mesh already finalized");
  try {
    const std::string e = ctx->mesh->refine(cells, n, levels_up);
    if (!e.empty()) return ctx->set(MFGMG_ERR_INVALID, e);
  } catch (...) {
    return ctx->set(MFGMG_ERR_NOMEM, "out of host memory");
  }
  return MFGMG_OK;
}

int mfgmg_finalize_mesh(mfgmg_ctx* ctx) {
  if (!ctx) return MFGMG_ERR_INVALID;
  try {
    const std::string e = ctx->mesh->finalize();
    if (!e.empty()) return ctx->set(MFGMG_ERR_MESH, e);
  } catch (...) {
    return ctx->set(MFGMG_ERR_NOMEM, "out of host memory");
  }
  return MFGMG_OK;
}

int mfgmg_info(const mfgmg_ctx* ctx, mfgmg_info_t* out) {
  if (!ctx || !out) return MFGMG_ERR_INVALID;
  if (!ctx->mesh->finalized()) return MFGMG_ERR_STATE;
  std::memset(out, 0, sizeof(*out));
  const Mesh& m = *ctx->mesh;
  out->n_levels = m.L();
  out->unit_exponent = m.U();
  for (int l = 1; l <= m.L(); ++l) {
    const Level& h = m.vlevel(l);
    out->n_cells[l] = h.ncell;
    out->n_nodes[l] = h.nnode;
    out->n_u[l] = 3 * h.nnode;
    int64_t nf = 0;
    for (int64_t i = 0; i < h.nnode; ++i) {
      const unsigned cm = h.cmask(i);
      nf += 3 - int64_t((cm & 1) + ((cm >> 1) & 1) + ((cm >> 2) & 1));
    }
    out->n_free[l] = nf;
    out->n_hanging[l] = int64_t(h.hang.count());
    out->uniform[l] = h.uniform ? 1 : 0;
  }
  out->n_p = m.vleaf().npnode;
  out->n_p_hanging = int64_t(m.vleaf().phang.count());
  out->element_k = m.velocity_degree() - 1;
  out->boundary = m.noflux() ? MFGMG_BC_NOFLUX : MFGMG_BC_DIRICHLET;
  return MFGMG_OK;
}

int mfgmg_cells(const mfgmg_ctx* ctx, int32_t level, int32_t* cells) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!cells) return MFGMG_ERR_INVALID;
  const Level& h = ctx->mesh->level(level);
  for (int64_t c = 0; c < h.ncell; ++c) {
    cells[4 * c] = h.clev[size_t(c)];
    cells[4 * c + 1] = h.cijk[size_t(3 * c)];
    cells[4 * c + 2] = h.cijk[size_t(3 * c + 1)];
    cells[4 * c + 3] = h.cijk[size_t(3 * c + 2)];
  }
  return MFGMG_OK;
}

int mfgmg_support_points(const mfgmg_ctx* ctx, int32_t level, int32_t field, int64_t* keys) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!keys || field < 0 || field > 1 || (field == 1 && level != ctx->mesh->L())) return MFGMG_ERR_INVALID;
  const Level& h = ctx->mesh->vlevel(level);
  const auto& src = field == 0 ? h.key : h.pkey;
  std::memcpy(keys, src.data(), src.size() * sizeof(int64_t));
  return MFGMG_OK;
}

int mfgmg_node_types(const mfgmg_ctx* ctx, int32_t level, int32_t field, uint8_t* types) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!types || field < 0 || field > 2 || (field == 1 && level != ctx->mesh->L())) return MFGMG_ERR_INVALID;
  const Level& h = ctx->mesh->vlevel(level);
  if (field == 2) {
    for (int64_t i = 0; i < h.nnode; ++i) types[i] = h.cmask(i);
    return MFGMG_OK;
  }
  const auto& src = field == 0 ? h.ntype : h.ptype;
  std::memcpy(types, src.data(), src.size());
  return MFGMG_OK;
}

int mfgmg_constraints(const mfgmg_ctx* ctx, int32_t level, int32_t field, int64_t* nh, int64_t* nnz, int64_t* node,
                      int64_t* ptr, int64_t* master, double* weight) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!nh || !nnz || field < 0 || field > 1 || (field == 1 && level != ctx->mesh->L())) return MFGMG_ERR_INVALID;
  const Level& h = ctx->mesh->vlevel(level);
  const Constraints& cs = field == 0 ? h.hang : h.phang;
  *nh = int64_t(cs.count());
  *nnz = int64_t(cs.master.size());
  if (node && ptr && master && weight) {
    for (size_t i = 0; i < cs.count(); ++i) node[i] = cs.node[i];
    for (size_t i = 0; i <= cs.count(); ++i) ptr[i] = cs.ptr[i];
    for (size_t i = 0; i < cs.master.size(); ++i) master[i] = cs.master[i], weight[i] = cs.weight[i];
  }
  return MFGMG_OK;
}

int mfgmg_transfer(const mfgmg_ctx* ctx, int32_t level, int64_t* nnz, int64_t* ptr, int64_t* col, double* w) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (level < 2 || !nnz) return MFGMG_ERR_INVALID;
  const Level& h = ctx->mesh->velocity_degree() == 3 ? ctx->mesh->vlevel(level) : ctx->mesh->level_transfer(level);
  *nnz = int64_t(h.P_col.size());
  if (ptr && col && w) {
    for (size_t i = 0; i < h.P_ptr.size(); ++i) ptr[i] = h.P_ptr[i];
    for (size_t i = 0; i < h.P_col.size(); ++i) col[i] = h.P_col[i], w[i] = h.P_w[i];
  }
  return MFGMG_OK;
}

int mfgmg_leaf_quadrature_points(const mfgmg_ctx* ctx, double* xyz) {
  if (!ctx || !xyz) return MFGMG_ERR_INVALID;
  if (!ctx->mesh->finalized()) return MFGMG_ERR_STATE;
  ctx->mesh->leaf_quadrature_points(xyz);
  return MFGMG_OK;
}

int mfgmg_set_viscosity(mfgmg_ctx* ctx, const double* mu_qp, void* stream) {
  if (!ctx || !mu_qp) return MFGMG_ERR_INVALID;
  if (!ctx->mesh->finalized()) return ctx->set(MFGMG_ERR_STATE, "finalize the mesh first");
  const Mesh& m = *ctx->mesh;
  const int L = m.L();
  const int64_t nl = m.leaf().ncell;
  const int nq = m.quad_points(), nq3 = nq * nq * nq;
  for (int64_t i = 0; i < nq3 * nl; ++i)
    if (!(mu_qp[i] > 0) || !std::isfinite(mu_qp[i]))
      return ctx->set(MFGMG_ERR_INVALID, "viscosity must be positive and finite");
  int st = upload_mesh(ctx);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* mq = nullptr;
  HIPCHK(hipMalloc(&mq, size_t(nq3 * nl) * sizeof(double)));
  HIPCHK(hipMemcpyAsync(mq, mu_qp, size_t(nq3 * nl) * sizeof(double), hipMemcpyHostToDevice, s));
  if (nq == 4) launch_harmonic_mu64(nl, mq, ctx->lv[size_t(L)].mu_d, s);
  else launch_harmonic_mu(nl, mq, ctx->lv[size_t(L)].mu_d, s);
  for (int ell = L - 1; ell >= 1; --ell)
    launch_restrict_mu(ctx->lv[size_t(ell)].v.ncell, ctx->lv[size_t(ell)].mu_src, ctx->lv[size_t(ell + 1)].mu_d,
                       ctx->lv[size_t(ell)].mu_d, s);
  double* dtmp = nullptr;
  HIPCHK(hipMalloc(&dtmp, size_t(3 * m.vleaf().nnode) * sizeof(double) + 64));
  for (int ell = 1; ell <= L; ++ell) {
    LevelDev& d = ctx->lv[size_t(ell)];
    launch_to_float(d.v.ncell, d.mu_d, d.mu_f, s);
    const int64_t n = 3 * d.v.nnode;
    launch_fill(n, 0.0, dtmp, s);
    launch_diag(d.v, ctx->khat_d, dtmp, s);
    launch_invert_diag(d.v, dtmp, d.minv_d, d.minv_f, s);
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipFree(dtmp));
  HIPCHK(hipFree(mq));
  for (int ell = 2; ell <= L; ++ell) {
    st = estimate_lambda(ctx, ell, s);
    if (st) return st;
  }
  st = factor_coarse(ctx, s);
  if (st) return st;
  st = pressure_setup(ctx, s);
  if (st) return st;
  ctx->ls_mu_ready = false;   // the local levels take their viscosity on first use
  ctx->mu_ready = true;
  return MFGMG_OK;
}

int mfgmg_cell_viscosity(const mfgmg_ctx* ctx, int32_t level, double* mu) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!mu) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return MFGMG_ERR_STATE;
  const LevelDev& d = ctx->lv[size_t(level)];
  if (hipMemcpy(mu, d.mu_d, size_t(d.v.ncell) * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return MFGMG_ERR_HIP;
  return MFGMG_OK;
}

int mfgmg_smoother_lambda(const mfgmg_ctx* ctx, int32_t level, double* out) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!out) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return MFGMG_ERR_STATE;
  *out = ctx->lv[size_t(level)].lambda;
  return MFGMG_OK;
}

int mfgmg_inverse_diagonal(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, void* dst, void* stream) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!dst) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  const LevelDev& d = ctx->lv[size_t(level)];
  const size_t n = size_t(3 * d.v.nnode);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (prec == MFGMG_FP64)
    HIPCHK(hipMemcpyAsync(dst, d.minv_d, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  else
    HIPCHK(hipMemcpyAsync(dst, d.minv_f, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  return MFGMG_OK;
}

int mfgmg_vmult(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* src, void* dst, void* stream) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!src || !dst || src == dst || (prec != MFGMG_FP32 && prec != MFGMG_FP64)) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevLevel& v = ctx->lv[size_t(level)].v;
  if (prec == MFGMG_FP64)
    launch_vmult<double>(v, static_cast<const double*>(src), static_cast<double*>(dst), s);
  else
    launch_vmult<float>(v, static_cast<const float*>(src), static_cast<float*>(dst), s);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_vmult_add(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* src, void* dst, void* stream) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!src || !dst || src == dst || (prec != MFGMG_FP32 && prec != MFGMG_FP64)) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevLevel& v = ctx->lv[size_t(level)].v;
  if (prec == MFGMG_FP64)
    launch_vmult<double>(v, static_cast<const double*>(src), static_cast<double*>(dst), s, false);
  else
    launch_vmult<float>(v, static_cast<const float*>(src), static_cast<float*>(dst), s, false);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_vcycle(mfgmg_ctx* ctx, mfgmg_prec prec, const void* rhs, void* x, void* stream) {
  if (!ctx || !rhs || !x || rhs == x) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int L = ctx->mesh->L();
  if (prec == MFGMG_FP64)
    vcycle<double>(ctx, L, static_cast<const double*>(rhs), static_cast<double*>(x), s);
  else if (prec == MFGMG_FP32)
    vcycle<float>(ctx, L, static_cast<const float*>(rhs), static_cast<float*>(x), s);
  else
    return MFGMG_ERR_INVALID;
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_prolongate(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* coarse, void* fine, void* stream) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (level < 2 || !coarse || !fine) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LevelDev& d = ctx->lv[size_t(level)];
  const DevLevel& cv = ctx->lv[size_t(level - 1)].v;
  if (prec == MFGMG_FP64)
    launch_prolong_level<double>(d.v, cv, d.P_ptr, d.P_col, d.P_w, static_cast<const double*>(coarse),
                                 static_cast<double*>(fine), false, s);
  else
    launch_prolong_level<float>(d.v, cv, d.P_ptr, d.P_col, d.P_w, static_cast<const float*>(coarse),
                                static_cast<float*>(fine), false, s);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_restrict(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* fine, void* coarse, void* stream) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (level < 2 || !coarse || !fine) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const LevelDev& d = ctx->lv[size_t(level)];
  const DevLevel& cv = ctx->lv[size_t(level - 1)].v;
  // scratch: the level's smoother work vectors
  if (prec == MFGMG_FP64)
    launch_restrict_level<double>(d.v, cv, d.R_ptr, d.R_col, d.R_w, static_cast<const double*>(fine), nullptr,
                                  static_cast<double*>(coarse), static_cast<double*>(d.work[1][2]),
                                  static_cast<double*>(d.work[1][3]), s);
  else
    launch_restrict_level<float>(d.v, cv, d.R_ptr, d.R_col, d.R_w, static_cast<const float*>(fine), nullptr,
                                 static_cast<float*>(coarse), static_cast<float*>(d.work[0][2]),
                                 static_cast<float*>(d.work[0][3]), s);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_smooth(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* b, void* x, int32_t x_is_zero,
                 void* stream) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (level < 2 || !b || !x || b == x) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (prec == MFGMG_FP64)
    smooth<double>(ctx, level, static_cast<const double*>(b), static_cast<double*>(x), x_is_zero != 0, s);
  else
    smooth<float>(ctx, level, static_cast<const float*>(b), static_cast<float*>(x), x_is_zero != 0, s);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_coarse_solve(mfgmg_ctx* ctx, mfgmg_prec prec, const void* b, void* x, void* stream) {
  if (!ctx || !b || !x || b == x) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (prec == MFGMG_FP64)
    vcycle<double>(ctx, 1, static_cast<const double*>(b), static_cast<double*>(x), s);
  else
    vcycle<float>(ctx, 1, static_cast<const float*>(b), static_cast<float*>(x), s);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_assemble_rhs(mfgmg_ctx* ctx, const double* f_qp, double* rhs_u, void* stream) {
  if (!ctx || !f_qp || !rhs_u) return MFGMG_ERR_INVALID;
  if (!ctx->mesh->finalized()) return ctx->set(MFGMG_ERR_STATE, "finalize the mesh first");
  int st = upload_mesh(ctx);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevLevel& v = ctx->lv[size_t(ctx->mesh->L())].v;
  const int nq = ctx->mesh->quad_points();
  const size_t nf = size_t(3 * nq * nq * nq) * size_t(v.ncell);
  double* fd = nullptr;
  HIPCHK(hipMalloc(&fd, nf * sizeof(double)));
  HIPCHK(hipMemcpyAsync(fd, f_qp, nf * sizeof(double), hipMemcpyHostToDevice, s));
  launch_rhs(v, fd, rhs_u, s);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipFree(fd));
  return MFGMG_OK;
}

int mfgmg_apply_div(mfgmg_ctx* ctx, const double* u, double* p_out, void* stream) {
  if (!ctx || !u || !p_out) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  launch_div(ctx->lv[size_t(ctx->mesh->L())].v, ctx->pres, u, p_out, static_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_apply_grad(mfgmg_ctx* ctx, const double* p, double* u_out, void* stream) {
  if (!ctx || !p || !u_out) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  const DevLevel& v = ctx->lv[size_t(ctx->mesh->L())].v;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_fill(3 * v.nnode, 0.0, u_out, s);
  launch_grad_add(v, ctx->pres, p, u_out, s);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_apply_pmass(mfgmg_ctx* ctx, const double* p, double* p_out, void* stream) {
  if (!ctx || !p || !p_out || p == p_out) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  launch_pmass(ctx->lv[size_t(ctx->mesh->L())].v, ctx->pres, p, p_out, static_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

int mfgmg_default_opts(mfgmg_solve_opts* o) {
  if (!o) return MFGMG_ERR_INVALID;
  o->rtol = 1e-8;
  o->restart = 50;
  o->max_iter = 1000;
  o->vcycle_prec = MFGMG_FP32;
  o->schur_rtol = 1e-2;   // Sec. 2.2.2: the inner CG converges in 1-5 iterations
  o->schur_max_iter = 200;
  o->use_scaling = 0;
  o->verbose = 0;
  o->use_graph = 1;
  o->krylov = MFGMG_FGMRES;
  o->idr_s = 2;
  o->block = MFGMG_BLOCK_TRIANGULAR;
  o->schur = MFGMG_SCHUR_CG;
  o->schur_degree = 8;
  o->hierarchy = MFGMG_GLOBAL_COARSENING;
  o->idr_fp64_from = 0;
  return MFGMG_OK;
}

int mfgmg_solve_stokes(mfgmg_ctx* ctx, const double* rhs_u, const double* rhs_p, double* u_out, double* p_out,
                       const mfgmg_solve_opts* opts, mfgmg_solve_stats* stats, void* stream) {
  if (!ctx || !rhs_u || !u_out || !p_out) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  mfgmg_solve_opts o;
  mfgmg_default_opts(&o);
  if (opts) o = *opts;
  if (o.restart < 1 || o.restart > 120 || !(o.rtol > 0) || o.max_iter < 1 ||
      (o.vcycle_prec != MFGMG_FP32 && o.vcycle_prec != MFGMG_FP64) || o.krylov < MFGMG_FGMRES ||
      o.krylov > MFGMG_IDR || o.idr_s < 1 || o.idr_s > 8 || (o.block != MFGMG_BLOCK_TRIANGULAR &&
      o.block != MFGMG_BLOCK_DIAGONAL) || (o.schur != MFGMG_SCHUR_CG && o.schur != MFGMG_SCHUR_CHEB) ||
      o.schur_degree < 1 || o.schur_degree > 64 ||
      (o.hierarchy != MFGMG_GLOBAL_COARSENING && o.hierarchy != MFGMG_LOCAL_SMOOTHING) || o.idr_fp64_from < 0)
    return ctx->set(MFGMG_ERR_INVALID, "bad solver options");
  if (o.krylov != MFGMG_FGMRES && o.schur != MFGMG_SCHUR_CHEB)
    return ctx->set(MFGMG_ERR_INVALID, "GMRES and IDR need the linear (Chebyshev) Schur approximation");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool local = o.hierarchy == MFGMG_LOCAL_SMOOTHING;
  if (o.use_scaling && ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "the learned scaling is built for Q2-Q1");
  if (o.schur == MFGMG_SCHUR_CHEB && ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "the Chebyshev Schur map takes the Q1 pressure interval");
  if (local) {
    if (o.use_scaling) return ctx->set(MFGMG_ERR_INVALID, "the learned scaling applies to the global-coarsening levels");
    if (ctx->mesh->noflux() || ctx->mesh->velocity_degree() != 2)
      return ctx->set(MFGMG_ERR_INVALID, "local smoothing is built for Q2-Q1 with the Dirichlet condition");
    const int st = local_setup(ctx, s);
    if (st) return st;
  }
  const auto t0 = std::chrono::steady_clock::now();
  struct ScalingGuard {   // V-cycles of this solve use the installed scalings iff requested
    mfgmg_ctx* c;
    bool saved;
    ~ScalingGuard() { c->use_scaling = saved; }
  } scaling_guard{ctx, ctx->use_scaling};
  ctx->use_scaling = o.use_scaling != 0;
  const int L = ctx->mesh->L();
  LevelDev& top = ctx->lv[size_t(L)];
  const DevLevel& lv = top.v;
  const DevPressure& P = ctx->pres;
  const int64_t nu = 3 * lv.nnode, np = P.np, n = nu + np;
  const int m = o.restart;
  const bool idr = o.krylov == MFGMG_IDR, flex = o.krylov == MFGMG_FGMRES;
  const int sdim = o.idr_s;
  // Krylov storage, FGMRES: V (m+1 vectors), Z (m); GMRES: V (m+1), one z;
  // IDR(s): Q, G, U (s each) in V, v and t in Z.  Then b, x, r, w; FP32
  // staging; CG vectors
  double* V = ctx->dalloc<double>(size_t(idr ? 3 * sdim : m + 1) * n);
  double* Z = ctx->dalloc<double>(size_t(idr ? 2 : flex ? m : 1) * n);
  double* b = ctx->dalloc<double>(size_t(n));
  double* x = ctx->dalloc<double>(size_t(n));
  double* r = ctx->dalloc<double>(size_t(n));
  double* w = ctx->dalloc<double>(size_t(n));
  double* tu = ctx->dalloc<double>(size_t(nu));
  float* bf = ctx->dalloc<float>(size_t(nu));
  float* xf = ctx->dalloc<float>(size_t(nu));
  double* cg = ctx->dalloc<double>(size_t(6 * np));   // r, z (contiguous), p, q, x, p'
  double* yv = ctx->dalloc<double>(size_t(std::max(m + 1, 16)));
  const bool fp64 = o.vcycle_prec == MFGMG_FP64;
  double* zfix = (o.use_graph && fp64) ? ctx->dalloc<double>(size_t(nu)) : nullptr;   // graph's fixed output
  // IDR(s) with the FP32 V-cycle restarts from its best iterate (below)
  const bool idr_restarts = idr && !fp64;
  double* xbest = idr_restarts ? ctx->dalloc<double>(size_t(n)) : nullptr;
  std::vector<void*> mine = {V, Z, b, x, r, w, tu, bf, xf, cg, yv};
  if (o.use_graph && fp64) mine.push_back(zfix);
  if (idr_restarts) mine.push_back(xbest);
  auto release = [&]() {
    for (void* p : mine) {
      auto it = std::find(ctx->allocs.begin(), ctx->allocs.end(), p);
      if (it != ctx->allocs.end()) ctx->allocs.erase(it);
      if (p) (void)hipFree(p);
    }
  };
  for (void* p : mine)
    if (!p) {
      release();
      return ctx->set(MFGMG_ERR_NOMEM, "device allocation for the Krylov space failed");
    }
  double* cr = cg;
  double* cz = cg + np;
  double* cp = cg + 2 * np;
  double* cq = cg + 3 * np;
  double* cx = cg + 4 * np;
  double* cp2 = cg + 5 * np;
  int64_t inner_total = 0;
  int vcycles = 0;
  int fp64_from = -1;

  auto apply_K = [&](const double* in, double* out) {
    launch_vmult<double>(lv, in, out, s);
    launch_grad_add(lv, P, in + nu, out, s);
    launch_div(lv, P, in, out + nu, s);
    launch_p_identity(P, in + nu, out + nu, s);
  };
  // the fixed Chebyshev map: interval [b/27, b], b = max_i (M_p 1)_i minv_i
  double cheb_hi = 0.0;
  if (o.schur == MFGMG_SCHUR_CHEB) {
    launch_fill(np, 1.0, cp, s);
    launch_pmass(lv, P, cp, cq, s);
    launch_mul(np, ctx->pmass_minv, cq, cz, s);
    std::vector<double> h(static_cast<size_t>(np));
    HIPCHK(hipMemcpyAsync(h.data(), cz, size_t(np) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (double v : h) cheb_hi = std::max(cheb_hi, v);
  }
  // Chebyshev iteration (Saad, Alg. 12.1) from 0 on M_p: cx = p(M_p) rhs
  auto schur_cheb = [&](const double* rhs) {
    const double hi = cheb_hi, lo = hi / 27.0;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    launch_cheb_init0<double>(np, rhs, ctx->pmass_minv, cr, cz, cx, 1.0 / theta, s);
    for (int k = 1; k < o.schur_degree; ++k) {
      launch_pmass(lv, P, cz, cq, s);
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      launch_cheb_step<double>(np, cq, ctx->pmass_minv, cr, cz, cx, rho_new * rho, 2.0 * rho_new / delta, s);
      rho = rho_new;
    }
  };
  // Jacobi-preconditioned CG on M_p: cx = M_p^{-1} rhs
  auto schur = [&](const double* rhs) {
    if (o.schur == MFGMG_SCHUR_CHEB) {
      schur_cheb(rhs);
      return;
    }
    // the iterations run with their scalars on the device (no host
    // synchronisation before the first check); the host looks at the
    // stopping flag every kCgBatch iterations
    launch_cg_start(np, rhs, ctx->pmass_minv, cr, cz, cp, cx, cq, s);
    double* sc = ctx->red_res + 480;
    launch_dot(np, cr, cz, ctx->red_part, sc, s);       // sc[0] = r.z
    launch_dot(np, cr, cr, ctx->red_part, sc + 7, s);   // sc[7] = r.r
    launch_cg_setup(sc, o.schur_rtol * o.schur_rtol, s);
    constexpr int kCgBatch = 8;
    for (int base = 0; base < o.schur_max_iter; base += kCgBatch) {
      const int kk = std::min(kCgBatch, o.schur_max_iter - base);
      for (int k = 0; k < kk; ++k)
        launch_cg_pmass_iteration(lv, P, ctx->pmass_minv, cx, cr, cz, cp, cp2, cq, ctx->red_part, sc, base + k, s);
      (void)hipMemcpyAsync(ctx->host_res + 480, sc, 8 * sizeof(double), hipMemcpyDeviceToHost, s);
      (void)hipStreamSynchronize(s);
      if (ctx->host_res[485] != 0.0) break;
    }
    inner_total += int64_t(ctx->host_res[486]);
  };
  // the V-cycle as one HIP graph: captured once per solve (nothing it depends
  // on changes during a solve) and replayed on `s` at every preconditioning
  hipGraphExec_t vexec = nullptr;
  if (o.use_graph) {
    hipError_t e = hipSuccess;
    if (!ctx->capture_stream) e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    hipStream_t cs = ctx->capture_stream;
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      if (fp64) vcycle_of<double>(ctx, local, L, tu, zfix, cs);
      else vcycle_of<float>(ctx, local, L, bf, xf, cs);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);
      if (e == hipSuccess) e = hipGraphInstantiate(&vexec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
    }
    if (e != hipSuccess) {
      release();
      return ctx->set(MFGMG_ERR_HIP, std::string("V-cycle graph capture: ") + hipGetErrorString(e));
    }
  }
  // z = P^{-1} v: z_p = -S^{-1} v_p, z_u = V(v_u - B^T z_p) (block
  // triangular) or V(v_u) (block diagonal)
  // (IDR switches an FP32 V-cycle to FP64 where it stalls, below)
  bool pre64 = fp64;
  auto precondition = [&](const double* v, double* z) {
    schur(v + nu);
    if (o.block == MFGMG_BLOCK_TRIANGULAR) launch_grad_from(lv, P, cx, v, tu, s);
    else (void)hipMemcpyAsync(tu, v, size_t(nu) * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (pre64) {
      if (vexec && fp64) {
        (void)hipGraphLaunch(vexec, s);
        launch_scale_copy(nu, 1.0, zfix, z, s);
      } else {
        vcycle_of<double>(ctx, local, L, tu, z, s);
      }
    } else {
      launch_to_float(nu, tu, bf, s);
      if (vexec) (void)hipGraphLaunch(vexec, s);
      else vcycle_of<float>(ctx, local, L, bf, xf, s);
      launch_to_double(nu, xf, z, s);
    }
    ++vcycles;
    launch_scale_copy(np, -1.0, cx, z + nu, s);
  };

  HIPCHK(hipMemcpyAsync(b, rhs_u, size_t(nu) * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (rhs_p)
    HIPCHK(hipMemcpyAsync(b + nu, rhs_p, size_t(np) * sizeof(double), hipMemcpyDeviceToDevice, s));
  else
    launch_fill(np, 0.0, b + nu, s);
  launch_fill(n, 0.0, x, s);
  const double bn = std::sqrt(dot_sync(ctx, n, b, b, s));
  HIPCHK(hipMemcpyAsync(r, b, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  double beta = bn;
  int its = 0;
  bool bad = !std::isfinite(bn);
  std::vector<double> H(static_cast<size_t>((m + 1) * m)), cs(static_cast<size_t>(m)),
      sn(static_cast<size_t>(m)), g(static_cast<size_t>(m + 1)), y(static_cast<size_t>(m));
  auto Hij = [&](int i, int j) -> double& { return H[size_t(i) * m + j]; };
  if (idr && !bad && bn > 0) {
    // IDR(s) with biorthogonal basis vectors (van Gijzen and Sonneveld, ACM
    // TOMS 38:5, 2011), right preconditioned, x0 = 0: per cycle s steps that
    // keep r orthogonal to Q(:, 0..k), then a dimension-reduction step with
    // the minimal-residual omega, enlarged when cos(t, r) < 0.7
    const int ss = sdim;
    double* Q = V;
    double* G = V + size_t(ss) * n;
    double* U = V + size_t(2 * ss) * n;
    double* vv = Z;
    double* tt = Z + n;
    auto col = [&](double* base, int i) { return base + size_t(i) * n; };
    double* res = ctx->red_res;
    double* hres = ctx->host_res;
    {
      // shadow space: keyed SplitMix64 columns, then Gram-Schmidt
      const Level& h = ctx->mesh->vlevel(L);
      std::vector<double> q(static_cast<size_t>(n));
      for (int i = 0; i < ss; ++i) {
        const uint64_t seed = uint64_t(4711 + i);
        for (int64_t k = 0; k < h.nnode; ++k)
          for (int c = 0; c < 3; ++c) q[size_t(3 * k + c)] = splitmix_pm1(seed, uint64_t(3 * h.key[size_t(k)] + c));
        for (int64_t k = 0; k < np; ++k)
          q[size_t(nu + k)] = splitmix_pm1(seed, (uint64_t(1) << 40) + uint64_t(h.pkey[size_t(k)]));
        HIPCHK(hipMemcpyAsync(col(Q, i), q.data(), size_t(n) * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int j = 0; j < i; ++j) {
          const double a = dot_sync(ctx, n, col(Q, j), col(Q, i), s);
          launch_axpby(n, -a, col(Q, j), 1.0, col(Q, i), s);
        }
        const double nq = std::sqrt(dot_sync(ctx, n, col(Q, i), col(Q, i), s));
        launch_scale_copy(n, 1.0 / nq, col(Q, i), col(Q, i), s);
      }
    }
    launch_fill(2 * int64_t(ss) * n, 0.0, G, s);   // G and U
    std::vector<double> M(static_cast<size_t>(ss * ss), 0.0), f(static_cast<size_t>(ss)), cpos(8), cneg(8);
    auto Mij = [&](int i, int j) -> double& { return M[size_t(i) * ss + j]; };
    for (int i = 0; i < ss; ++i) Mij(i, i) = 1.0;
    double om = 1.0, rn = bn;
    constexpr double kKappa = 0.7;
    bool done = rn <= o.rtol * bn;
    int printed = 0;
    // With the FP32 V-cycle the preconditioner is linear only up to FP32
    // rounding, which IDR's short recurrences (unlike flexible GMRES) do not
    // tolerate at high viscosity contrast: at 128^3+1 cells and contrast 1e6
    // the true residual levels off near 1e-5, and restarting IDR from its
    // best iterate does not move that floor.  So where an FP32 run stalls --
    // while its best residual is still above 100x the tolerance, 200
    // iterations fail to halve that best, or the recursive residual exceeds
    // 100x it (not in the first 50 iterations, whose residual may grow
    // before it falls); or it meets the tolerance but the true residual does
    // not -- the solve restarts from its best iterate with the true residual
    // (fresh G, U and M, the same shadow space) and the FP64 V-cycle; after
    // that it restarts (twice at most) only where the recursion meets the
    // tolerance and the true residual does not.  Runs that start with the
    // FP64 V-cycle never restart.
    constexpr int kMaxRestarts = 3, kWindow = 200, kGrace = 50;
    constexpr double kGrowth = 100.0;
    int restarts = 0, start_it = 0, win_it = 0;
    double best = rn, win_best = rn;
    bool restart_now = false;
    if (idr_restarts) HIPCHK(hipMemcpyAsync(xbest, x, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    auto track = [&]() {
      if (!idr_restarts || pre64) return;
      if (rn < best) {
        best = rn;
        (void)hipMemcpyAsync(xbest, x, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s);
      }
      if (o.idr_fp64_from > 0 && its >= o.idr_fp64_from) {
        restart_now = true;
        return;
      }
      if (best <= 100.0 * o.rtol * bn) return;
      if (rn > kGrowth * best && its - start_it >= kGrace) {
        restart_now = true;
      } else if (its - win_it >= kWindow) {
        if (best > 0.5 * win_best) restart_now = true;
        win_it = its;
        win_best = best;
      }
    };
    auto progress = [&]() {
      if (o.verbose > 0 && its / o.verbose > printed) {
        printed = its / o.verbose;
        std::fprintf(stderr, "[mfgmg] idr(%d) it %d  residual %.3e  %.1f s\n", ss, its, rn / bn,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        std::fflush(stderr);
      }
    };
    for (;;) {
    while (!done && !bad && its < o.max_iter) {
      launch_mdot(n, ss, Q, n, r, ctx->red_part, res, s);   // f = Q^T r
      (void)hipMemcpyAsync(hres, res, size_t(ss) * sizeof(double), hipMemcpyDeviceToHost, s);
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < ss; ++i) f[size_t(i)] = hres[i];
      for (int k = 0; k < ss; ++k) {
        const int q = ss - k;
        // M(k:, k:) c = f(k:), lower triangular
        for (int i = 0; i < q; ++i) {
          double t = f[size_t(k + i)];
          for (int j = 0; j < i; ++j) t -= Mij(k + i, k + j) * cpos[size_t(j)];
          cpos[size_t(i)] = t / Mij(k + i, k + i);
          cneg[size_t(i)] = -cpos[size_t(i)];
        }
        HIPCHK(hipMemcpyAsync(yv, cpos.data(), size_t(q) * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(yv + 8, cneg.data(), size_t(q) * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(vv, r, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_mupdate(n, q, col(G, k), n, yv, vv, s);       // v = r - G(:, k:) c
        precondition(vv, tt);                               // t = P^{-1} v
        launch_scale_copy(n, om, tt, vv, s);
        launch_mupdate(n, q, col(U, k), n, yv + 8, vv, s);   // om t + U(:, k:) c
        HIPCHK(hipMemcpyAsync(col(U, k), vv, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
        apply_K(col(U, k), col(G, k));
        ++its;
        for (int i = 0; i < k; ++i) {   // biorthogonalise against the earlier columns
          const double a = dot_sync(ctx, n, col(Q, i), col(G, k), s) / Mij(i, i);
          launch_axpby(n, -a, col(G, i), 1.0, col(G, k), s);
          launch_axpby(n, -a, col(U, i), 1.0, col(U, k), s);
        }
        launch_mdot(n, q, col(Q, k), n, col(G, k), ctx->red_part, res, s);   // M(k:, k)
        (void)hipMemcpyAsync(hres, res, size_t(q) * sizeof(double), hipMemcpyDeviceToHost, s);
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < q; ++i) Mij(k + i, k) = hres[i];
        if (!(Mij(k, k) != 0.0) || !std::isfinite(Mij(k, k))) {
          bad = true;
          break;
        }
        const double be = f[size_t(k)] / Mij(k, k);
        launch_axpby(n, -be, col(G, k), 1.0, r, s);
        launch_axpby(n, be, col(U, k), 1.0, x, s);
        rn = std::sqrt(dot_sync(ctx, n, r, r, s));
        progress();
        if (!std::isfinite(rn)) bad = true;
        if (!bad) track();
        if (bad || rn <= o.rtol * bn || its >= o.max_iter || restart_now) {
          done = true;
          break;
        }
        for (int i = k + 1; i < ss; ++i) f[size_t(i)] -= be * Mij(i, k);
      }
      if (done || bad) break;
      precondition(r, vv);   // dimension reduction
      apply_K(vv, tt);
      ++its;
      const double t2 = dot_sync(ctx, n, tt, tt, s), tr = dot_sync(ctx, n, tt, r, s);
      om = tr / t2;
      const double rho = std::fabs(tr) / (std::sqrt(t2) * rn);
      if (rho < kKappa) om *= kKappa / rho;
      if (!std::isfinite(om)) {
        bad = true;
        break;
      }
      launch_axpby(n, -om, tt, 1.0, r, s);
      launch_axpby(n, om, vv, 1.0, x, s);
      rn = std::sqrt(dot_sync(ctx, n, r, r, s));
      progress();
      if (!std::isfinite(rn)) bad = true;
      if (!bad) track();
      done = rn <= o.rtol * bn || restart_now;
    }
    if (!idr_restarts || bad || its >= o.max_iter || restarts >= kMaxRestarts) break;
    if (!restart_now) {   // met the tolerance by the recursion: the true residual decides
      apply_K(x, w);
      launch_axpby(n, 1.0, b, -1.0, w, s);
      if (std::sqrt(dot_sync(ctx, n, w, w, s)) <= o.rtol * bn) break;
    }
    // restart with the FP64 V-cycle: a stall from the best iterate, a
    // tolerance gap from the current one
    if (!pre64) fp64_from = its;
    pre64 = true;
    if (restart_now) HIPCHK(hipMemcpyAsync(x, xbest, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    apply_K(x, r);
    launch_axpby(n, 1.0, b, -1.0, r, s);
    rn = std::sqrt(dot_sync(ctx, n, r, r, s));
    if (!std::isfinite(rn)) {
      bad = true;
      break;
    }
    launch_fill(2 * int64_t(ss) * n, 0.0, G, s);
    std::fill(M.begin(), M.end(), 0.0);
    for (int i = 0; i < ss; ++i) Mij(i, i) = 1.0;
    om = 1.0;
    best = rn;
    win_best = rn;
    win_it = its;
    start_it = its;
    restart_now = false;
    ++restarts;
    done = rn <= o.rtol * bn;
    if (o.verbose > 0) {
      std::fprintf(stderr, "[mfgmg] idr(%d) restart at it %d from residual %.3e, FP64 V-cycle\n", ss, its, rn / bn);
      std::fflush(stderr);
    }
    }
    apply_K(x, r);   // the true residual decides
    launch_axpby(n, 1.0, b, -1.0, r, s);
    beta = std::sqrt(dot_sync(ctx, n, r, r, s));
    if (!std::isfinite(beta)) bad = true;
  }
  while (!idr && !bad && bn > 0 && its < o.max_iter && beta > o.rtol * bn) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    launch_scale_copy(n, 1.0 / beta, r, V, s);
    int jd = 0;
    for (int j = 0; j < m; ++j) {
      double* zj = flex ? Z + size_t(j) * n : Z;
      precondition(V + size_t(j) * n, zj);
      apply_K(zj, w);
      // classical Gram-Schmidt, repeated only when the first pass cancelled
      // much of w (||w'|| < ||w|| / sqrt(2), the criterion of Daniel, Gragg,
      // Kaufman and Stewart, 1976).  Coefficients in red_res [0, nv] (h1 and
      // w.w), [256, 256 + nv] (h2 and w'.w') and 400 (w''.w'').  Up to
      // kMupdateDotsMax basis vectors the update of w and the products of
      // the second pass share one read of the basis (three basis reads per
      // step with the repetition instead of four).
      const int nv = j + 1;
      double* res = ctx->red_res;
      double* hres = ctx->host_res;
      launch_mdot(n, nv, V, n, w, ctx->red_part, res, s, /*with_norm=*/true);
      const bool fused = launch_mupdate_dots(n, nv, V, n, res, w, ctx->red_part, res + 256, true, s);
      if (!fused) {
        launch_mupdate(n, nv, V, n, res, w, s);
        launch_dot(n, w, w, ctx->red_part, res + 256 + nv, s);
      }
      (void)hipMemcpyAsync(hres, res, size_t(nv + 1) * sizeof(double), hipMemcpyDeviceToHost, s);
      (void)hipMemcpyAsync(hres + 256, res + 256, size_t(nv + 1) * sizeof(double), hipMemcpyDeviceToHost, s);
      HIPCHK(hipStreamSynchronize(s));
      const double wn0 = std::sqrt(hres[nv]);
      double hn = std::sqrt(hres[256 + nv]);
      for (int i = 0; i < nv; ++i) Hij(i, j) = hres[i];
      if (!(hn >= wn0 * 0.70710678118654752)) {
        if (fused) {
          launch_mupdate_dots(n, nv, V, n, res + 256, w, ctx->red_part, res + 400, false, s);
        } else {
          launch_mdot(n, nv, V, n, w, ctx->red_part, res + 256, s);
          (void)hipMemcpyAsync(hres + 256, res + 256, size_t(nv) * sizeof(double), hipMemcpyDeviceToHost, s);
          launch_mupdate(n, nv, V, n, res + 256, w, s);
          launch_dot(n, w, w, ctx->red_part, res + 400, s);
        }
        (void)hipMemcpyAsync(hres + 400, res + 400, sizeof(double), hipMemcpyDeviceToHost, s);
        HIPCHK(hipStreamSynchronize(s));
        hn = std::sqrt(hres[400]);
        for (int i = 0; i < nv; ++i) Hij(i, j) += hres[256 + i];
      }
      Hij(j + 1, j) = hn;
      if (!std::isfinite(hn)) {
        bad = true;
        break;
      }
      if (hn > 0) launch_scale_copy(n, 1.0 / hn, w, V + size_t(j + 1) * n, s);
      for (int i = 0; i < j; ++i) {
        const double t = cs[size_t(i)] * Hij(i, j) + sn[size_t(i)] * Hij(i + 1, j);
        Hij(i + 1, j) = -sn[size_t(i)] * Hij(i, j) + cs[size_t(i)] * Hij(i + 1, j);
        Hij(i, j) = t;
      }
      const double den = std::hypot(Hij(j, j), Hij(j + 1, j));
      cs[size_t(j)] = Hij(j, j) / den;
      sn[size_t(j)] = Hij(j + 1, j) / den;
      Hij(j, j) = den;
      Hij(j + 1, j) = 0.0;
      g[size_t(j + 1)] = -sn[size_t(j)] * g[size_t(j)];
      g[size_t(j)] = cs[size_t(j)] * g[size_t(j)];
      ++its;
      jd = j + 1;
      if (o.verbose > 0 && its % o.verbose == 0) {
        std::fprintf(stderr, "[mfgmg] fgmres it %d  residual estimate %.3e  %.1f s\n", its,
                     std::fabs(g[size_t(j + 1)]) / bn,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        std::fflush(stderr);
      }
      if (std::fabs(g[size_t(j + 1)]) <= o.rtol * bn || its >= o.max_iter) break;
    }
    if (bad || jd == 0) break;
    for (int i = jd - 1; i >= 0; --i) {
      double t = g[size_t(i)];
      for (int k = i + 1; k < jd; ++k) t -= Hij(i, k) * y[size_t(k)];
      y[size_t(i)] = t / Hij(i, i);
    }
    std::vector<double> ny(static_cast<size_t>(jd));
    for (int i = 0; i < jd; ++i) ny[size_t(i)] = -y[size_t(i)];
    HIPCHK(hipMemcpyAsync(yv, ny.data(), size_t(jd) * sizeof(double), hipMemcpyHostToDevice, s));
    if (flex) {
      launch_mupdate(n, jd, Z, n, yv, x, s);   // x += Z y
    } else {
      launch_fill(n, 0.0, w, s);
      launch_mupdate(n, jd, V, n, yv, w, s);   // w = V y
      precondition(w, Z);
      launch_axpby(n, 1.0, Z, 1.0, x, s);      // x += P^{-1} V y
    }
    apply_K(x, r);
    launch_axpby(n, 1.0, b, -1.0, r, s);     // r = b - K x
    beta = std::sqrt(dot_sync(ctx, n, r, r, s));
    if (!std::isfinite(beta)) bad = true;
  }
  // outputs: zero-mean pressure, hanging values interpolated
  HIPCHK(hipMemcpyAsync(u_out, x, size_t(nu) * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(p_out, x + nu, size_t(np) * sizeof(double), hipMemcpyDeviceToDevice, s));
  const double mean = dot_sync(ctx, np, ctx->pmean_w, p_out, s) / ctx->pmean_total;
  launch_fill(np, 1.0, cr, s);
  launch_axpby(np, -mean, cr, 1.0, p_out, s);
  launch_distribute_u(lv, u_out, s);
  launch_distribute_p(P, p_out, s);
  HIPCHK(hipStreamSynchronize(s));
  if (vexec) (void)hipGraphExecDestroy(vexec);
  release();
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  const bool conv = !bad && (bn == 0 || beta <= o.rtol * bn);
  if (stats) {
    stats->iterations = its;
    stats->vcycles = vcycles;
    stats->inner_cg_iterations = inner_total;
    stats->rel_residual = bn > 0 ? beta / bn : 0.0;
    stats->seconds = secs;
    stats->converged = conv ? 1 : 0;
    stats->fp64_from = fp64_from;
  }
  if (!conv) return ctx->set(MFGMG_ERR_NOCONV, bad ? "NaN or Inf in the solve" : "tolerance not reached");
  return MFGMG_OK;
}

const char* mfgmg_last_error(const mfgmg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

void mfgmg_destroy(mfgmg_ctx* ctx) {
  if (!ctx) return;
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  for (void* p : ctx->allocs)
    if (p) (void)hipFree(p);
  if (ctx->host_res) (void)hipHostFree(ctx->host_res);
  delete ctx;
}

}  // extern "C"
