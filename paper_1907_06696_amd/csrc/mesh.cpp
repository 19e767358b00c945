// Host-side mesh layer (see mesh.h).
//
// Readings of the paper (arXiv 1907.06696), which leaves these open:
//  * meshes are 2:1 balanced across faces, edges and vertices, so a hanging
//    node's masters are never constrained themselves;
//  * the multigrid hierarchy is global coarsening: level l holds every leaf
//    cell of level <= l and the level-l ancestors of finer leaves;
//  * Q2/Q1 Lagrange support points on {0, 1/2, 1} / {0, 1}: a node on the
//    closed box of a cell that is not one of that cell's own nodes hangs, with
//    the cell's interpolation weights (1D: 3/8, 3/4, -1/8 at the quarter
//    points for Q2; 1/2 at the mid point for Q1);
//  * every velocity node on the boundary is Dirichlet (u = 0, Sec. 2 eq.
//    stokes), and Dirichlet wins over hanging.
#include "mesh.h"

#include "q3.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <utility>

namespace mfgmg {

namespace {

constexpr int kOff26 = 26;

inline uint64_t cell_code(int l, int64_t i, int64_t j, int64_t k) {
  const uint64_t off = ((uint64_t(1) << (3 * l)) - 1) / 7;
  const uint64_t n = uint64_t(1) << l;
  return off + uint64_t(i) + n * (uint64_t(j) + n * uint64_t(k));
}

inline uint64_t spread3(uint64_t v) {
  // spread the low 21 bits of v to every third bit
  v &= 0x1fffff;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Open-addressing hash map int64 key -> int32 value (keys are >= 0).
class KeyMap {
 public:
  explicit KeyMap(size_t expected = 16) {
    size_t cap = 16;
    while (cap < 2 * expected + 16) cap <<= 1;
    keys_.assign(cap, -1);
    vals_.assign(cap, -1);
    mask_ = cap - 1;
  }
  int32_t find(int64_t k) const {
    size_t h = hash(uint64_t(k)) & mask_;
    while (true) {
      const int64_t kk = keys_[h];
      if (kk == k) return vals_[h];
      if (kk < 0) return -1;
      h = (h + 1) & mask_;
    }
  }
  // inserts (k, v) if absent; returns the stored value
  int32_t insert(int64_t k, int32_t v) {
    if (2 * (size_ + 1) > keys_.size()) grow();
    size_t h = hash(uint64_t(k)) & mask_;
    while (true) {
      const int64_t kk = keys_[h];
      if (kk == k) return vals_[h];
      if (kk < 0) {
        keys_[h] = k;
        vals_[h] = v;
        ++size_;
        return v;
      }
      h = (h + 1) & mask_;
    }
  }
  size_t size() const { return size_; }

 private:
  static uint64_t hash(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
  }
  void grow() {
    std::vector<int64_t> ok;
    std::vector<int32_t> ov;
    ok.swap(keys_);
    ov.swap(vals_);
    const size_t cap = ok.size() * 2;
    keys_.assign(cap, -1);
    vals_.assign(cap, -1);
    mask_ = cap - 1;
    size_ = 0;
    for (size_t i = 0; i < ok.size(); ++i)
      if (ok[i] >= 0) insert(ok[i], ov[i]);
  }
  std::vector<int64_t> keys_;
  std::vector<int32_t> vals_;
  size_t mask_ = 0;
  size_t size_ = 0;
};

const std::array<std::array<int, 3>, kOff26>& offsets26() {
  static const auto offs = [] {
    std::array<std::array<int, 3>, kOff26> o{};
    int n = 0;
    for (int c = -1; c <= 1; ++c)
      for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a)
          if (a || b || c) o[n++] = {a, b, c};
    return o;
  }();
  return offs;
}

// 1D Q2 basis at the quarter points t = 0, 1/4, 1/2, 3/4, 1 (rows) -- the
// values of L_0, L_1, L_2 there (exact dyadic numbers)
double q2_at_quarter(int a, int i) {
  double v[3];
  q2_basis_1d(0.25 * a, v);
  return v[i];
}
double q1_at_half(int a, int i) {
  const double t = 0.5 * a;
  return i == 0 ? 1.0 - t : t;
}

struct Scratch {
  std::vector<KeyMap> node_map;   // per level: key -> node (non-uniform levels)
  std::vector<KeyMap> cell_map;   // per level: cell code -> cell index
};

thread_local Scratch* g_scratch = nullptr;

inline int64_t lattice_index(const Level& lv, int64_t X, int64_t Y, int64_t Z) {
  const int64_t m = 2 * lv.n_edge + 1;
  return X + m * (Y + m * Z);
}

}  // namespace

void q2_basis_1d(double t, double v[3]) {
  v[0] = 2.0 * (t - 0.5) * (t - 1.0);
  v[1] = -4.0 * t * (t - 1.0);
  v[2] = 2.0 * t * (t - 0.5);
}

void q2_deriv_1d(double t, double v[3]) {
  v[0] = 4.0 * t - 3.0;
  v[1] = 4.0 - 8.0 * t;
  v[2] = 4.0 * t - 1.0;
}

Mesh::Mesh(int base_level) {
  const int64_t n = int64_t(1) << base_level;
  lev_.assign(size_t(n * n * n), base_level);
  ijk_.resize(size_t(3 * n * n * n));
  int64_t c = 0;
  for (int64_t k = 0; k < n; ++k)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i, ++c) {
        ijk_[3 * c] = int32_t(i);
        ijk_[3 * c + 1] = int32_t(j);
        ijk_[3 * c + 2] = int32_t(k);
      }
}

static void refine_marked(std::vector<int32_t>& lev, std::vector<int32_t>& ijk, const std::vector<uint8_t>& mark,
                          int times) {
  std::vector<int32_t> nl, nc;
  nl.reserve(lev.size());
  nc.reserve(ijk.size());
  std::vector<int32_t> wl, wc;
  for (size_t c = 0; c < lev.size(); ++c) {
    if (!mark[c]) {
      nl.push_back(lev[c]);
      nc.insert(nc.end(), {ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]});
      continue;
    }
    wl.assign(1, lev[c]);
    wc.assign({ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]});
    for (int t = 0; t < times; ++t) {
      std::vector<int32_t> l2, c2;
      for (size_t q = 0; q < wl.size(); ++q)
        for (int cz = 0; cz < 2; ++cz)
          for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
              l2.push_back(wl[q] + 1);
              c2.insert(c2.end(), {2 * wc[3 * q] + cx, 2 * wc[3 * q + 1] + cy, 2 * wc[3 * q + 2] + cz});
            }
      wl.swap(l2);
      wc.swap(c2);
    }
    nl.insert(nl.end(), wl.begin(), wl.end());
    nc.insert(nc.end(), wc.begin(), wc.end());
  }
  lev.swap(nl);
  ijk.swap(nc);
}

std::string Mesh::refine(const int32_t* cells, int64_t n, int times) {
  if (finalized_) return "mesh already finalized";
  if (times < 0 || times > 4) return "levels_up must be in [0, 4]";
  KeyMap map(lev_.size());
  int maxl = 0;
  for (size_t c = 0; c < lev_.size(); ++c) {
    map.insert(int64_t(cell_code(lev_[c], ijk_[3 * c], ijk_[3 * c + 1], ijk_[3 * c + 2])), int32_t(c));
    maxl = std::max(maxl, lev_[c]);
  }
  std::vector<uint8_t> mark(lev_.size(), 0);
  for (int64_t q = 0; q < n; ++q) {
    const int32_t l = cells[4 * q], i = cells[4 * q + 1], j = cells[4 * q + 2], k = cells[4 * q + 3];
    if (l < 0 || l > 20 || i < 0 || j < 0 || k < 0 || i >= (1 << l) || j >= (1 << l) || k >= (1 << l))
      return "refine: cell index out of range";
    const int32_t c = map.find(int64_t(cell_code(l, i, j, k)));
    if (c < 0) return "refine: listed cell is not active";
    if (l + times > 13) return "refine: mesh would exceed the maximum depth";
    mark[size_t(c)] = 1;
  }
  refine_marked(lev_, ijk_, mark, times);
  balance();
  return "";
}

void Mesh::balance() {
  const auto& offs = offsets26();
  while (true) {
    int minl = 1 << 30, maxl = 0;
    for (int32_t l : lev_) minl = std::min(minl, l), maxl = std::max(maxl, l);
    if (maxl - minl < 2) return;
    KeyMap map(lev_.size());
    for (size_t c = 0; c < lev_.size(); ++c)
      map.insert(int64_t(cell_code(lev_[c], ijk_[3 * c], ijk_[3 * c + 1], ijk_[3 * c + 2])), int32_t(c));
    std::vector<uint8_t> mark(lev_.size(), 0);
    bool any = false;
    for (size_t c = 0; c < lev_.size(); ++c) {
      const int l = lev_[c];
      if (l < minl + 2) continue;
      const int64_t nl = int64_t(1) << l;
      for (const auto& o : offs) {
        const int64_t x = ijk_[3 * c] + o[0], y = ijk_[3 * c + 1] + o[1], z = ijk_[3 * c + 2] + o[2];
        if (x < 0 || y < 0 || z < 0 || x >= nl || y >= nl || z >= nl) continue;
        // a leaf covering the neighbour at level <= l-2 violates the balance
        for (int m = l - 2; m >= minl; --m) {
          const int s = l - m;
          const int32_t hit = map.find(int64_t(cell_code(m, x >> s, y >> s, z >> s)));
          if (hit >= 0) {
            mark[size_t(hit)] = 1;
            any = true;
            break;
          }
        }
      }
    }
    if (!any) return;
    refine_marked(lev_, ijk_, mark, 1);
  }
}

std::string Mesh::finalize() {
  if (finalized_) return "";
  L_ = 0;
  int minl = 1 << 30;
  for (int32_t l : lev_) L_ = std::max(L_, l), minl = std::min(minl, l);
  if (minl < 1) return "the leaf mesh must have every cell at level >= 1";
  if (L_ > 13) return "mesh too deep";
  levels_.assign(size_t(L_ + 1), Level{});
  Scratch scratch;
  scratch.node_map.resize(size_t(L_ + 1));
  scratch.cell_map.resize(size_t(L_ + 1));
  g_scratch = &scratch;
  for (int ell = 1; ell <= L_; ++ell) build_level(ell);
  transfer_built_.assign(size_t(L_ + 1), 0);
  for (int ell = 2; ell <= L_; ++ell)
    if (!transfer_deferred(ell)) {
      build_transfer(ell);
      transfer_built_[size_t(ell)] = 1;
    }
  for (int ell = 1; ell < L_; ++ell) build_mu_restriction(ell);
  g_scratch = nullptr;
  if (vdeg_ == 3) {
    if (noflux_) return "the Q3-Q2 pair is built for u = 0 on the boundary";
    for (int ell = 1; ell <= L_; ++ell)
      if (!levels_[ell].uniform) return "the Q3-Q2 pair is built for uniform meshes";
    q3_.assign(size_t(L_ + 1), Level{});
    for (int ell = 1; ell <= L_; ++ell) build_q3_level(levels_[ell], ell == L_, q3_[size_t(ell)]);
  }
  // masters of hanging nodes must be free
  for (int ell = 1; ell <= L_; ++ell) {
    const Level& lv = levels_[ell];
    for (int32_t m : lv.hang.master)
      if (lv.ntype[size_t(m)] != NODE_FREE) return "hanging node constrained against a constrained node";
    if (ell == L_)
      for (int32_t m : lv.phang.master)
        if (lv.ptype[size_t(m)] != NODE_FREE) return "pressure hanging node against a constrained node";
  }
  finalized_ = true;
  return "";
}

void Mesh::build_level(int ell) {
  Level& lv = levels_[ell];
  lv.ell = ell;
  const int U = L_ + 1;
  bool all_fine = true;
  for (int32_t l : lev_)
    if (l < ell) {
      all_fine = false;
      break;
    }
  if (all_fine && !noflux_) {
    // uniform level mesh: every 8^ell cell of level ell, lexicographic
    const int64_t n = int64_t(1) << ell;
    lv.uniform = true;
    lv.n_edge = n;
    lv.ncell = n * n * n;
    lv.clev.assign(size_t(lv.ncell), ell);
    lv.cijk.resize(size_t(3 * lv.ncell));
    int64_t c = 0;
    for (int64_t k = 0; k < n; ++k)
      for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i, ++c) {
          lv.cijk[3 * c] = int32_t(i);
          lv.cijk[3 * c + 1] = int32_t(j);
          lv.cijk[3 * c + 2] = int32_t(k);
        }
  } else {
    struct C {
      uint64_t code;
      uint64_t mort;
      int32_t l, i, j, k;
    };
    std::vector<C> cs;
    cs.reserve(lev_.size());
    for (size_t c = 0; c < lev_.size(); ++c) {
      int l = lev_[c];
      int64_t i = ijk_[3 * c], j = ijk_[3 * c + 1], k = ijk_[3 * c + 2];
      if (l > ell) {
        const int s = l - ell;
        i >>= s, j >>= s, k >>= s, l = ell;
      }
      const int sh = U - l;
      cs.push_back({cell_code(l, i, j, k), morton(uint64_t(i) << sh, uint64_t(j) << sh, uint64_t(k) << sh),
                    l, int32_t(i), int32_t(j), int32_t(k)});
    }
    std::sort(cs.begin(), cs.end(), [](const C& a, const C& b) { return a.code < b.code; });
    cs.erase(std::unique(cs.begin(), cs.end(), [](const C& a, const C& b) { return a.code == b.code; }),
             cs.end());
    std::sort(cs.begin(), cs.end(), [](const C& a, const C& b) { return a.mort < b.mort; });
    lv.uniform = false;
    lv.ncell = int64_t(cs.size());
    lv.clev.resize(cs.size());
    lv.cijk.resize(3 * cs.size());
    for (size_t c = 0; c < cs.size(); ++c) {
      lv.clev[c] = cs[c].l;
      lv.cijk[3 * c] = cs[c].i;
      lv.cijk[3 * c + 1] = cs[c].j;
      lv.cijk[3 * c + 2] = cs[c].k;
    }
  }
  lv.min_cell_level = *std::min_element(lv.clev.begin(), lv.clev.end());
  KeyMap& cmap = g_scratch->cell_map[size_t(ell)];
  cmap = KeyMap(size_t(lv.ncell));
  for (int64_t c = 0; c < lv.ncell; ++c)
    cmap.insert(int64_t(cell_code(lv.clev[c], lv.cijk[3 * c], lv.cijk[3 * c + 1], lv.cijk[3 * c + 2])),
                int32_t(c));
  build_nodes(lv, false);
  if (ell == L_) build_nodes(lv, true);
}

void Mesh::build_nodes(Level& lv, bool q1) const {
  const int U = L_ + 1;
  const int64_t S = int64_t(1) << U;
  const int64_t S1 = S + 1;
  auto key_of = [&](int64_t X, int64_t Y, int64_t Z) { return X + S1 * (Y + S1 * Z); };
  const int npc = q1 ? 8 : 27;            // nodes per cell
  const int per = q1 ? 2 : 3;             // nodes per edge of a cell
  std::vector<int32_t>& cn = q1 ? lv.cell_pnodes : lv.cell_nodes;
  std::vector<int64_t>& keys = q1 ? lv.pkey : lv.key;
  std::vector<uint8_t>& types = q1 ? lv.ptype : lv.ntype;
  std::vector<int32_t>& hidx = q1 ? lv.phang_index : lv.hang_index;
  Constraints& cons = q1 ? lv.phang : lv.hang;
  cn.resize(size_t(npc * lv.ncell));

  if (lv.uniform && !q1) {
    const int64_t n = lv.n_edge, m = 2 * n + 1;
    const int sh = U - lv.ell - 1;   // lattice step in key units
    lv.nnode = m * m * m;
    keys.resize(size_t(lv.nnode));
    types.assign(size_t(lv.nnode), NODE_FREE);
    for (int64_t Z = 0; Z < m; ++Z)
      for (int64_t Y = 0; Y < m; ++Y)
        for (int64_t X = 0; X < m; ++X) {
          const int64_t id = X + m * (Y + m * Z);
          keys[size_t(id)] = key_of(X << sh, Y << sh, Z << sh);
          if (X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1)
            types[size_t(id)] = NODE_DIRICHLET;
        }
    for (int64_t c = 0; c < lv.ncell; ++c) {
      const int64_t i = lv.cijk[3 * c], j = lv.cijk[3 * c + 1], k = lv.cijk[3 * c + 2];
      for (int z = 0; z < 3; ++z)
        for (int y = 0; y < 3; ++y)
          for (int x = 0; x < 3; ++x)
            cn[size_t(27 * c + x + 3 * y + 9 * z)] = int32_t(lattice_index(lv, 2 * i + x, 2 * j + y, 2 * k + z));
    }
    hidx.assign(size_t(lv.nnode), -1);
    lv.nfree_nodes = (m - 2) * (m - 2) * (m - 2);
    return;
  }

  // general: first-touch numbering over the cell order
  KeyMap local_map(size_t(lv.ncell) * (q1 ? 2 : 9));
  KeyMap& nmap = q1 ? local_map : g_scratch->node_map[size_t(lv.ell)];
  if (!q1) nmap = KeyMap(size_t(lv.ncell) * 9);
  keys.clear();
  for (int64_t c = 0; c < lv.ncell; ++c) {
    const int l = lv.clev[c];
    const int64_t size = int64_t(1) << (U - l);
    const int64_t step = q1 ? size : size / 2;
    const int64_t ox = int64_t(lv.cijk[3 * c]) * size, oy = int64_t(lv.cijk[3 * c + 1]) * size,
                  oz = int64_t(lv.cijk[3 * c + 2]) * size;
    for (int z = 0; z < per; ++z)
      for (int y = 0; y < per; ++y)
        for (int x = 0; x < per; ++x) {
          const int64_t k = key_of(ox + x * step, oy + y * step, oz + z * step);
          const int32_t id = nmap.insert(k, int32_t(keys.size()));
          if (id == int32_t(keys.size())) keys.push_back(k);
          cn[size_t(npc * c + x + per * (y + per * z))] = id;
        }
  }
  const int64_t nn = int64_t(keys.size());
  if (q1)
    lv.npnode = nn;
  else
    lv.nnode = nn;
  types.assign(size_t(nn), NODE_FREE);
  if (!q1) {
    // u = 0: boundary nodes are Dirichlet nodes; u . n = 0: component c of a
    // node on a face normal to axis c is fixed, the node stays free (or
    // hanging, below)
    if (noflux_) lv.fixmask.assign(size_t(nn), 0);
    else lv.fixmask.clear();
    for (int64_t id = 0; id < nn; ++id) {
      const int64_t k = keys[size_t(id)];
      const int64_t X = k % S1, Y = (k / S1) % S1, Z = k / (S1 * S1);
      const bool bx = X == 0 || X == S, by = Y == 0 || Y == S, bz = Z == 0 || Z == S;
      if (noflux_) lv.fixmask[size_t(id)] = uint8_t((bx ? 1 : 0) | (by ? 2 : 0) | (bz ? 4 : 0));
      else if (bx || by || bz) types[size_t(id)] = NODE_DIRICHLET;
    }
  }

  // cells adjacent to finer cells: the parents of finer cells touch them
  std::vector<uint8_t> coarse_adj(size_t(lv.ncell), 0);
  const KeyMap& cmap = g_scratch->cell_map[size_t(lv.ell)];
  const auto& offs = offsets26();
  for (int64_t c = 0; c < lv.ncell; ++c) {
    const int l = lv.clev[c];
    if (l <= lv.min_cell_level) continue;
    const int64_t np = int64_t(1) << (l - 1);
    const int64_t px = lv.cijk[3 * c] >> 1, py = lv.cijk[3 * c + 1] >> 1, pz = lv.cijk[3 * c + 2] >> 1;
    for (const auto& o : offs) {
      const int64_t x = px + o[0], y = py + o[1], z = pz + o[2];
      if (x < 0 || y < 0 || z < 0 || x >= np || y >= np || z >= np) continue;
      const int32_t hit = cmap.find(int64_t(cell_code(l - 1, x, y, z)));
      if (hit >= 0) coarse_adj[size_t(hit)] = 1;
    }
  }
  // hanging nodes: lattice points on the closed box of such a cell that are
  // nodes of the mesh but not nodes of the cell
  struct Rec {
    int32_t node;
    int32_t nm;
    int32_t m[9];
    double w[9];
  };
  std::vector<Rec> recs;
  hidx.assign(size_t(nn), -1);
  const int lat = q1 ? 3 : 5;   // candidate lattice per direction
  for (int64_t c = 0; c < lv.ncell; ++c) {
    if (!coarse_adj[size_t(c)]) continue;
    const int l = lv.clev[c];
    const int64_t size = int64_t(1) << (U - l);
    const int64_t step = q1 ? size / 2 : size / 4;
    if (step == 0) continue;
    const int64_t ox = int64_t(lv.cijk[3 * c]) * size, oy = int64_t(lv.cijk[3 * c + 1]) * size,
                  oz = int64_t(lv.cijk[3 * c + 2]) * size;
    for (int z = 0; z < lat; ++z)
      for (int y = 0; y < lat; ++y)
        for (int x = 0; x < lat; ++x) {
          const bool bnd = x == 0 || y == 0 || z == 0 || x == lat - 1 || y == lat - 1 || z == lat - 1;
          const bool natural = (x % 2 == 0) && (y % 2 == 0) && (z % 2 == 0);
          if (!bnd || natural) continue;
          const int32_t id = nmap.find(key_of(ox + x * step, oy + y * step, oz + z * step));
          if (id < 0 || hidx[size_t(id)] >= 0 || types[size_t(id)] == NODE_DIRICHLET) continue;
          Rec r{};
          r.node = id;
          r.nm = 0;
          for (int k = 0; k < per; ++k)
            for (int j = 0; j < per; ++j)
              for (int i = 0; i < per; ++i) {
                double w;
                if (q1)
                  w = q1_at_half(x, i) * q1_at_half(y, j) * q1_at_half(z, k);
                else
                  w = q2_at_quarter(x, i) * q2_at_quarter(y, j) * q2_at_quarter(z, k);
                if (w == 0.0) continue;
                const int32_t mnode = cn[size_t(npc * c + i + per * (j + per * k))];
                if (types[size_t(mnode)] == NODE_DIRICHLET) continue;
                r.m[r.nm] = mnode;
                r.w[r.nm] = w;
                ++r.nm;
              }
          hidx[size_t(id)] = 0;   // placeholder until sorted
          recs.push_back(r);
        }
  }
  std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) { return a.node < b.node; });
  cons = Constraints{};
  for (size_t h = 0; h < recs.size(); ++h) {
    const Rec& r = recs[h];
    types[size_t(r.node)] = NODE_HANGING;
    hidx[size_t(r.node)] = int32_t(h);
    cons.node.push_back(r.node);
    for (int q = 0; q < r.nm; ++q) {
      cons.master.push_back(r.m[q]);
      cons.weight.push_back(r.w[q]);
    }
    cons.ptr.push_back(int64_t(cons.master.size()));
  }
  if (!q1) {
    int64_t nf = 0;
    for (uint8_t t : types) nf += (t == NODE_FREE);
    lv.nfree_nodes = nf;
  }
}

static int32_t find_node(const Level& lv, const KeyMap* map, int64_t key, int U) {
  if (lv.uniform) {
    const int64_t S1 = (int64_t(1) << U) + 1;
    const int64_t X = key % S1, Y = (key / S1) % S1, Z = key / (S1 * S1);
    const int sh = U - lv.ell - 1;
    const int64_t msk = (int64_t(1) << sh) - 1;
    if ((X & msk) || (Y & msk) || (Z & msk)) return -1;
    return int32_t(lattice_index(lv, X >> sh, Y >> sh, Z >> sh));
  }
  return map->find(key);
}

bool Mesh::transfer_deferred(int ell) const {
  return ell >= 2 && ell <= L_ && levels_[size_t(ell)].uniform && levels_[size_t(ell - 1)].uniform;
}

const Level& Mesh::level_transfer(int ell) const {
  if (finalized_ && ell >= 2 && ell <= L_ && !transfer_built_[size_t(ell)]) {
    // uniform pair: build_transfer needs no set-up maps
    const_cast<Mesh*>(this)->build_transfer(ell);
    transfer_built_[size_t(ell)] = 1;
  }
  return levels_[size_t(ell)];
}

// Uniform fine levels (uniform coarse level too) use neither set-up map, so
// this also runs after finalize.
void Mesh::build_transfer(int ell) {
  Level& fine = levels_[ell];
  const Level& coarse = levels_[ell - 1];
  const int U = L_ + 1;
  const int64_t S1 = (int64_t(1) << U) + 1;
  auto key_of = [&](int64_t X, int64_t Y, int64_t Z) { return X + S1 * (Y + S1 * Z); };
  const KeyMap* fmap = fine.uniform ? nullptr : &g_scratch->node_map[size_t(ell)];
  const KeyMap* fcells = fine.uniform ? nullptr : &g_scratch->cell_map[size_t(ell)];
  double P1[5][3];
  for (int a = 0; a < 5; ++a)
    for (int i = 0; i < 3; ++i) P1[a][i] = q2_at_quarter(a, i);

  // rows in production order, then compacted by fine node index
  std::vector<int64_t> row_start(size_t(fine.nnode), -1);
  std::vector<int32_t> row_len(size_t(fine.nnode), 0);
  std::vector<int32_t> cols;
  std::vector<double> vals;
  cols.reserve(size_t(fine.nnode) * 8);
  vals.reserve(size_t(fine.nnode) * 8);
  int32_t rc[96];
  double rw[96];
  auto emit = [&](int32_t f, const int32_t* cn27, const double* w27, bool cell_hangs) {
    // w27: weights of the 27 coarse local nodes at fine node f
    int nr = 0;
    if (!cell_hangs) {
      // the 27 nodes of a cell are distinct, so without hanging nodes no
      // column repeats: the entries in local-node order, as the search below
      // would give them
      row_start[size_t(f)] = int64_t(cols.size());
      int len = 0;
      for (int s = 0; s < 27; ++s) {
        const double w = w27[s];
        if (w == 0.0 || coarse.ntype[size_t(cn27[s])] != NODE_FREE) continue;
        cols.push_back(cn27[s]);
        vals.push_back(w);
        ++len;
      }
      row_len[size_t(f)] = len;
      return;
    }
    auto add = [&](int32_t col, double w) {
      for (int q = 0; q < nr; ++q)
        if (rc[q] == col) {
          rw[q] += w;
          return;
        }
      rc[nr] = col;
      rw[nr] = w;
      ++nr;
    };
    for (int s = 0; s < 27; ++s) {
      const double w = w27[s];
      if (w == 0.0) continue;
      const int32_t cnode = cn27[s];
      const uint8_t t = coarse.ntype[size_t(cnode)];
      if (t == NODE_FREE) {
        add(cnode, w);
      } else if (t == NODE_HANGING) {
        const int32_t h = coarse.hang_index[size_t(cnode)];
        for (int64_t q = coarse.hang.ptr[size_t(h)]; q < coarse.hang.ptr[size_t(h) + 1]; ++q)
          add(coarse.hang.master[size_t(q)], w * coarse.hang.weight[size_t(q)]);
      }
    }
    row_start[size_t(f)] = int64_t(cols.size());
    int len = 0;
    for (int q = 0; q < nr; ++q)
      if (rw[q] != 0.0) {
        cols.push_back(rc[q]);
        vals.push_back(rw[q]);
        ++len;
      }
    row_len[size_t(f)] = len;
  };
  std::vector<uint8_t> seen(size_t(fine.nnode), 0);
  double w27[27];
  for (int64_t c = 0; c < coarse.ncell; ++c) {
    const int l = coarse.clev[c];
    const int64_t size = int64_t(1) << (U - l);
    const int64_t ox = int64_t(coarse.cijk[3 * c]) * size, oy = int64_t(coarse.cijk[3 * c + 1]) * size,
                  oz = int64_t(coarse.cijk[3 * c + 2]) * size;
    const int32_t* cn27 = &coarse.cell_nodes[size_t(27 * c)];
    // (every cell of a uniform fine level is a child of a coarse cell)
    const bool refined = (l == ell - 1) &&
                         (fine.uniform || fcells->find(int64_t(cell_code(ell, 2 * int64_t(coarse.cijk[3 * c]),
                                                                         2 * int64_t(coarse.cijk[3 * c + 1]),
                                                                         2 * int64_t(coarse.cijk[3 * c + 2])))) >= 0);
    const int lat = refined ? 5 : 3;
    const int64_t step = refined ? size / 4 : size / 2;
    bool cell_hangs = false;
    for (int q = 0; q < 27; ++q) cell_hangs = cell_hangs || coarse.ntype[size_t(cn27[q])] == NODE_HANGING;
    // fine nodes of the cell's lattice: from the fine cells that cover it (the
    // cell itself, or its 8 children), one cell lookup instead of a node
    // lookup per lattice point on non-uniform fine levels
    int32_t fl[125];
    if (!fine.uniform) {
      const int64_t ci = coarse.cijk[3 * c], cj = coarse.cijk[3 * c + 1], ck = coarse.cijk[3 * c + 2];
      for (int q = 0; q < lat * lat * lat; ++q) fl[q] = -1;
      const int nch = refined ? 2 : 1;
      for (int hz = 0; hz < nch; ++hz)
        for (int hy = 0; hy < nch; ++hy)
          for (int hx = 0; hx < nch; ++hx) {
            const int32_t fc = refined ? fcells->find(int64_t(cell_code(ell, 2 * ci + hx, 2 * cj + hy, 2 * ck + hz)))
                                       : fcells->find(int64_t(cell_code(l, ci, cj, ck)));
            if (fc < 0) continue;   // cannot happen for a valid hierarchy
            const int32_t* fn27 = &fine.cell_nodes[size_t(27 * int64_t(fc))];
            for (int k = 0; k < 3; ++k)
              for (int j = 0; j < 3; ++j)
                for (int i = 0; i < 3; ++i)
                  fl[(2 * hx + i) + lat * ((2 * hy + j) + lat * (2 * hz + k))] = fn27[i + 3 * j + 9 * k];
          }
    }
    for (int z = 0; z < lat; ++z)
      for (int y = 0; y < lat; ++y)
        for (int x = 0; x < lat; ++x) {
          const int32_t f = fine.uniform ? find_node(fine, fmap, key_of(ox + x * step, oy + y * step, oz + z * step), U)
                                         : fl[x + lat * (y + lat * z)];
          if (f < 0) continue;   // cannot happen for a valid hierarchy
          if (seen[size_t(f)]) continue;
          seen[size_t(f)] = 1;
          if (fine.ntype[size_t(f)] != NODE_FREE) {
            row_start[size_t(f)] = int64_t(cols.size());
            row_len[size_t(f)] = 0;
            continue;
          }
          for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j)
              for (int i = 0; i < 3; ++i) {
                double w;
                if (refined)
                  w = P1[x][i] * P1[y][j] * P1[z][k];
                else
                  w = (x == i && y == j && z == k) ? 1.0 : 0.0;
                w27[i + 3 * j + 9 * k] = w;
              }
          emit(f, cn27, w27, cell_hangs);
        }
  }
  fine.P_ptr.assign(size_t(fine.nnode) + 1, 0);
  for (int64_t f = 0; f < fine.nnode; ++f) fine.P_ptr[size_t(f) + 1] = fine.P_ptr[size_t(f)] + row_len[size_t(f)];
  fine.P_col.resize(size_t(fine.P_ptr.back()));
  fine.P_w.resize(size_t(fine.P_ptr.back()));
  for (int64_t f = 0; f < fine.nnode; ++f) {
    const int64_t s = row_start[size_t(f)], d = fine.P_ptr[size_t(f)];
    for (int q = 0; q < row_len[size_t(f)]; ++q) {
      fine.P_col[size_t(d + q)] = cols[size_t(s + q)];
      fine.P_w[size_t(d + q)] = vals[size_t(s + q)];
    }
  }
  // transpose
  fine.R_ptr.assign(size_t(coarse.nnode) + 1, 0);
  for (int32_t c : fine.P_col) ++fine.R_ptr[size_t(c) + 1];
  for (int64_t c = 0; c < coarse.nnode; ++c) fine.R_ptr[size_t(c) + 1] += fine.R_ptr[size_t(c)];
  fine.R_col.resize(fine.P_col.size());
  fine.R_w.resize(fine.P_col.size());
  std::vector<int64_t> pos(fine.R_ptr.begin(), fine.R_ptr.end() - 1);
  for (int64_t f = 0; f < fine.nnode; ++f)
    for (int64_t q = fine.P_ptr[size_t(f)]; q < fine.P_ptr[size_t(f) + 1]; ++q) {
      const int32_t c = fine.P_col[size_t(q)];
      const int64_t d = pos[size_t(c)]++;
      fine.R_col[size_t(d)] = int32_t(f);
      fine.R_w[size_t(d)] = fine.P_w[size_t(q)];
    }
}

// Local-smoothing levels: for every level finer than the finest uniform one,
// the cells of exactly that level (taken from the global-coarsening mesh of
// the level, in its Morton order), their Q2 nodes, the node kinds and the
// refinement edge; the transfers from the level below; and, for every free
// leaf node, the finest level whose cells hold it.
void Mesh::ensure_local() const {
  if (ls_built_ || !finalized_) return;
  build_local_smoothing();
  ls_built_ = true;
}

void Mesh::build_local_smoothing() const {
  const int U = L_ + 1;
  const int64_t S1 = (int64_t(1) << U) + 1;
  int base = 0;
  for (int ell = 1; ell <= L_; ++ell)
    if (levels_[ell].uniform) base = ell;
  ls_base_ = base;
  ls_.assign(size_t(L_ + 1), LocalLevel{});
  ls_base_leaf_.clear();
  ls_base_node_.clear();
  Scratch scratch;
  scratch.node_map.resize(size_t(L_ + 1));
  scratch.cell_map.resize(size_t(L_ + 1));
  Scratch* saved = g_scratch;
  g_scratch = &scratch;
  for (int ell = base + 1; ell <= L_; ++ell) {
    const Level& g = levels_[ell];
    LocalLevel& t = ls_[size_t(ell)];
    Level& m = t.mesh;
    m.ell = ell;
    m.uniform = false;
    for (int64_t c = 0; c < g.ncell; ++c)
      if (g.clev[size_t(c)] == ell) {
        m.clev.push_back(ell);
        for (int d = 0; d < 3; ++d) m.cijk.push_back(g.cijk[size_t(3 * c + d)]);
        t.gc_cell.push_back(int32_t(c));
      }
    m.ncell = int64_t(m.clev.size());
    m.min_cell_level = ell;
    KeyMap& cmap = scratch.cell_map[size_t(ell)];
    cmap = KeyMap(size_t(m.ncell));
    for (int64_t c = 0; c < m.ncell; ++c)
      cmap.insert(int64_t(cell_code(ell, m.cijk[3 * c], m.cijk[3 * c + 1], m.cijk[3 * c + 2])), int32_t(c));
    build_nodes(m, false);   // same-level cells: no hanging nodes
    // kinds; a node is on the refinement edge when a level-ell cell position
    // touching it, inside the domain, holds no cell of the level
    const int64_t size = int64_t(1) << (U - ell), n = int64_t(1) << ell;
    t.kind.assign(size_t(m.nnode), 0);
    for (int64_t id = 0; id < m.nnode; ++id) {
      if (m.ntype[size_t(id)] == NODE_DIRICHLET) {
        t.kind[size_t(id)] = 1;
        continue;
      }
      const int64_t k = m.key[size_t(id)];
      const int64_t P[3] = {k % S1, (k / S1) % S1, k / (S1 * S1)};
      int64_t lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        const bool on = P[d] % size == 0;
        hi[d] = P[d] / size;
        lo[d] = on ? hi[d] - 1 : hi[d];
      }
      bool edge = false;
      for (int64_t z = lo[2]; z <= hi[2] && !edge; ++z)
        for (int64_t y = lo[1]; y <= hi[1] && !edge; ++y)
          for (int64_t x = lo[0]; x <= hi[0] && !edge; ++x) {
            if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) continue;
            edge = cmap.find(int64_t(cell_code(ell, x, y, z))) < 0;
          }
      if (edge) {
        t.kind[size_t(id)] = 2;
        m.ntype[size_t(id)] = NODE_DIRICHLET;
      }
    }
    int64_t nf = 0;
    for (uint8_t ty : m.ntype) nf += ty == NODE_FREE;
    m.nfree_nodes = nf;
  }
  for (int ell = base + 1; ell <= L_; ++ell) build_local_transfer(ell);
  if (base < L_) {
    const Level& leaf = levels_[L_];
    for (int64_t i = 0; i < leaf.nnode; ++i) {
      if (leaf.ntype[size_t(i)] != NODE_FREE) continue;
      const int64_t k = leaf.key[size_t(i)];
      bool done = false;
      for (int ell = L_; ell > base && !done; --ell) {
        const int32_t id = scratch.node_map[size_t(ell)].find(k);
        if (id >= 0) {
          ls_[size_t(ell)].copy_leaf.push_back(int32_t(i));
          ls_[size_t(ell)].copy_node.push_back(id);
          done = true;
        }
      }
      if (!done) {
        const int32_t id = find_node(levels_[base], nullptr, k, U);
        if (id >= 0) {
          ls_base_leaf_.push_back(int32_t(i));
          ls_base_node_.push_back(id);
        }
      }
    }
  }
  g_scratch = saved;
}

// P of local level ell from level ell - 1 (the uniform base level or the
// local level below): the Q2 function of each refined level-(ell-1) cell at
// its children's nodes; boundary rows empty, boundary columns dropped;
// refinement-edge rows and columns kept.
void Mesh::build_local_transfer(int ell) const {
  Level& fine = ls_[size_t(ell)].mesh;
  const std::vector<uint8_t>& fkind = ls_[size_t(ell)].kind;
  const bool cbase = ell - 1 == ls_base_;
  const Level& coarse = cbase ? levels_[ell - 1] : ls_[size_t(ell - 1)].mesh;
  auto coarse_boundary = [&](int32_t cn) {
    return cbase ? coarse.ntype[size_t(cn)] == NODE_DIRICHLET : ls_[size_t(ell - 1)].kind[size_t(cn)] == 1;
  };
  const int U = L_ + 1;
  const int64_t S1 = (int64_t(1) << U) + 1;
  auto key_of = [&](int64_t X, int64_t Y, int64_t Z) { return X + S1 * (Y + S1 * Z); };
  const KeyMap& fmap = g_scratch->node_map[size_t(ell)];
  const KeyMap& fcells = g_scratch->cell_map[size_t(ell)];
  double P1[5][3];
  for (int a = 0; a < 5; ++a)
    for (int i = 0; i < 3; ++i) P1[a][i] = q2_at_quarter(a, i);
  std::vector<std::vector<std::pair<int32_t, double>>> rows(static_cast<size_t>(fine.nnode));
  std::vector<uint8_t> seen(static_cast<size_t>(fine.nnode), 0);
  for (int64_t c = 0; c < coarse.ncell; ++c) {
    if (coarse.clev[size_t(c)] != ell - 1) continue;
    const int64_t ci = coarse.cijk[size_t(3 * c)], cj = coarse.cijk[size_t(3 * c + 1)],
                  ck = coarse.cijk[size_t(3 * c + 2)];
    if (fcells.find(int64_t(cell_code(ell, 2 * ci, 2 * cj, 2 * ck))) < 0) continue;   // not refined
    const int64_t size = int64_t(1) << (U - (ell - 1)), step = size / 4;
    const int32_t* cn27 = &coarse.cell_nodes[size_t(27 * c)];
    for (int z = 0; z < 5; ++z)
      for (int y = 0; y < 5; ++y)
        for (int x = 0; x < 5; ++x) {
          const int32_t f = fmap.find(key_of(ci * size + x * step, cj * size + y * step, ck * size + z * step));
          if (f < 0 || seen[size_t(f)]) continue;
          seen[size_t(f)] = 1;
          if (fkind[size_t(f)] == 1) continue;   // domain boundary: empty row
          for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j)
              for (int i = 0; i < 3; ++i) {
                const double w = P1[x][i] * P1[y][j] * P1[z][k];
                const int32_t cn = cn27[i + 3 * j + 9 * k];
                if (w != 0.0 && !coarse_boundary(cn)) rows[size_t(f)].emplace_back(cn, w);
              }
        }
  }
  fine.P_ptr.assign(size_t(fine.nnode) + 1, 0);
  fine.P_col.clear();
  fine.P_w.clear();
  for (int64_t f = 0; f < fine.nnode; ++f) {
    for (const auto& e : rows[size_t(f)]) {
      fine.P_col.push_back(e.first);
      fine.P_w.push_back(e.second);
    }
    fine.P_ptr[size_t(f) + 1] = int64_t(fine.P_col.size());
  }
  fine.R_ptr.assign(size_t(coarse.nnode) + 1, 0);
  for (int32_t c : fine.P_col) ++fine.R_ptr[size_t(c) + 1];
  for (int64_t c = 0; c < coarse.nnode; ++c) fine.R_ptr[size_t(c) + 1] += fine.R_ptr[size_t(c)];
  fine.R_col.resize(fine.P_col.size());
  fine.R_w.resize(fine.P_col.size());
  std::vector<int64_t> pos(fine.R_ptr.begin(), fine.R_ptr.end() - 1);
  for (int64_t f = 0; f < fine.nnode; ++f)
    for (int64_t q = fine.P_ptr[size_t(f)]; q < fine.P_ptr[size_t(f) + 1]; ++q) {
      const int32_t c = fine.P_col[size_t(q)];
      const int64_t d = pos[size_t(c)]++;
      fine.R_col[size_t(d)] = int32_t(f);
      fine.R_w[size_t(d)] = fine.P_w[size_t(q)];
    }
}

void Mesh::build_mu_restriction(int ell) {
  Level& coarse = levels_[ell];
  const KeyMap& fcells = g_scratch->cell_map[size_t(ell + 1)];
  coarse.mu_src.assign(size_t(8 * coarse.ncell), -1);
  for (int64_t c = 0; c < coarse.ncell; ++c) {
    const int l = coarse.clev[c];
    const int64_t i = coarse.cijk[3 * c], j = coarse.cijk[3 * c + 1], k = coarse.cijk[3 * c + 2];
    const int32_t self = fcells.find(int64_t(cell_code(l, i, j, k)));
    if (self >= 0) {
      coarse.mu_src[size_t(8 * c)] = self;
      continue;
    }
    int q = 0;
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx)
          coarse.mu_src[size_t(8 * c + q++)] = fcells.find(int64_t(cell_code(l + 1, 2 * i + cx, 2 * j + cy, 2 * k + cz)));
  }
}

void Mesh::leaf_quadrature_points(double* out) const {
  const Level& lv = leaf();
  const int nq = quad_points(), nq3 = nq * nq * nq;
  double xi[4];
  if (nq == 3) {
    const double g = 0.5 * std::sqrt(3.0 / 5.0);
    xi[0] = 0.5 - g, xi[1] = 0.5, xi[2] = 0.5 + g;
  } else {
    for (int q = 0; q < 4; ++q) xi[q] = q3_element().xg[q];
  }
  for (int64_t c = 0; c < lv.ncell; ++c) {
    const double h = std::ldexp(1.0, -lv.clev[c]);
    const double ox = lv.cijk[3 * c] * h, oy = lv.cijk[3 * c + 1] * h, oz = lv.cijk[3 * c + 2] * h;
    for (int z = 0; z < nq; ++z)
      for (int y = 0; y < nq; ++y)
        for (int x = 0; x < nq; ++x) {
          double* p = out + 3 * (nq3 * c + x + nq * y + nq * nq * z);
          p[0] = ox + xi[x] * h;
          p[1] = oy + xi[y] * h;
          p[2] = oz + xi[z] * h;
        }
  }
}

}  // namespace mfgmg
