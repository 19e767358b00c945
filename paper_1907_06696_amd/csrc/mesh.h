// Host-side mesh layer: unit-cube octree, 2:1 balance, global-coarsening level
// meshes, Q2/Q1 node numbering, Dirichlet and hanging-node constraints, level
// transfers.  Pure C++ (no GPU); the device layer uploads what it needs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mfgmg {

enum NodeType : uint8_t { NODE_FREE = 0, NODE_DIRICHLET = 1, NODE_HANGING = 2 };

// Hanging-node constraints over the nodes of one level mesh (CSR over the
// hanging nodes, ordered by node index).  Masters are free nodes only:
// Dirichlet masters carry zero and are dropped.
struct Constraints {
  std::vector<int64_t> node;
  std::vector<int64_t> ptr{0};
  std::vector<int32_t> master;
  std::vector<double> weight;
  size_t count() const { return node.size(); }
};

struct Level {
  int ell = 0;
  int64_t ncell = 0;
  std::vector<int32_t> clev;   // [ncell] cell level
  std::vector<int32_t> cijk;   // [3*ncell] integer position at that level
  bool uniform = false;        // all 8^ell cells of level ell, lexicographic order
  int64_t n_edge = 0;          // cells per edge when uniform
  int min_cell_level = 0;

  int64_t nnode = 0;
  std::vector<int64_t> key;         // canonical key per node
  std::vector<int32_t> cell_nodes;  // [27*ncell]
  std::vector<uint8_t> ntype;       // NodeType per node
  // no-normal-flux meshes only (empty otherwise): per node, bit c set when
  // component c is fixed by u . n = 0 (the node lies on a face normal to
  // axis c); such boundary nodes are NODE_FREE or NODE_HANGING
  std::vector<uint8_t> fixmask;
  std::vector<int32_t> hang_index;  // per node: row in `hang` or -1
  Constraints hang;
  int64_t nfree_nodes = 0;
  // per node: bit c set when velocity dof (node, c) is constrained (all three
  // for Dirichlet and hanging nodes, the fixed ones of a free boundary node)
  uint8_t cmask(int64_t i) const {
    return ntype[size_t(i)] != NODE_FREE ? uint8_t(7) : (fixmask.empty() ? uint8_t(0) : fixmask[size_t(i)]);
  }
  bool dof_free(int64_t i, int c) const { return !((cmask(i) >> c) & 1); }

  // prolongation from level ell-1 (node level, applied per component);
  // rows = nodes of this level (constrained rows empty)
  std::vector<int64_t> P_ptr;
  std::vector<int32_t> P_col;
  std::vector<double> P_w;
  // Q3 lattice levels (ell >= 2): the 1D factor of the prolongation, fine
  // lattice coordinate X -> coarse coordinates p1_c0[X] + j, weights p1_w[4X + j]
  std::vector<int32_t> p1_c0;
  std::vector<double> p1_w;
  // transpose (rows = nodes of level ell-1)
  std::vector<int64_t> R_ptr;
  std::vector<int32_t> R_col;
  std::vector<double> R_w;

  // viscosity restriction onto this level from level ell+1:
  // [8*ncell] cell indices in level ell+1 (-1 padded)
  std::vector<int32_t> mu_src;

  // leaf only: Q1 pressure nodes
  int64_t npnode = 0;
  std::vector<int64_t> pkey;
  std::vector<int32_t> cell_pnodes;  // [8*ncell]
  std::vector<uint8_t> ptype;
  std::vector<int32_t> phang_index;
  Constraints phang;
};

// One level of the local-smoothing hierarchy: the cells of refinement level
// exactly `ell` (a part of the domain once the leaf mesh is adaptive), no
// hanging nodes.  In `mesh` the nodes on the refinement edge (on the boundary
// of the part, inside the domain) are typed NODE_DIRICHLET: the level
// operator of the smoother keeps them fixed.  P/R in `mesh` transfer from
// the level below, with the refinement-edge rows kept.
struct LocalLevel {
  Level mesh;
  std::vector<uint8_t> kind;        // per node: 0 inner, 1 domain boundary, 2 refinement edge
  std::vector<int32_t> gc_cell;     // per cell: its index in the global-coarsening mesh of the level
  std::vector<int32_t> copy_leaf;   // leaf free nodes whose finest level is this one ...
  std::vector<int32_t> copy_node;   // ... and their node on this level
};

class Mesh {
 public:
  explicit Mesh(int base_level);
  // velocity boundary condition (before finalize): u = 0 (default) or the
  // no-normal-flux condition u . n = 0.  Under the latter every level mesh
  // is built by the general path (no uniform lattice levels).
  void set_noflux(bool on) { noflux_ = on; }
  bool noflux() const { return noflux_; }
  // velocity element (before finalize): 2 for Q2-Q1 (default), 3 for Q3-Q2
  // (k = 2 of Sec. 2.1; uniform meshes with u = 0 only).  The cell meshes
  // (level(ell)) are the same; vlevel(ell) holds the velocity nodes, the
  // transfers and, on the leaf, the pressure nodes of the chosen pair.
  void set_velocity_degree(int p) { vdeg_ = p; }
  int velocity_degree() const { return vdeg_; }
  const Level& vlevel(int ell) const { return vdeg_ == 3 ? q3_[size_t(ell)] : levels_[size_t(ell)]; }
  const Level& vleaf() const { return vlevel(L_); }
  // Gauss points per direction of the velocity element
  int quad_points() const { return vdeg_ == 3 ? 4 : 3; }
  // refine the listed active cells `times` levels, then 2:1 balance
  // returns "" on success or an error message
  std::string refine(const int32_t* cells, int64_t n, int times);
  std::string finalize();

  bool finalized() const { return finalized_; }
  int L() const { return L_; }
  int U() const { return L_ + 1; }
  int64_t S() const { return int64_t(1) << (L_ + 1); }
  const Level& level(int ell) const { return levels_[ell]; }
  Level& level(int ell) { return levels_[ell]; }
  // Transfers between two uniform lattice levels are applied on the device
  // from their lattice structure alone, so their node-level tables (P_*,
  // R_* of level ell) are built on first use: transfer_deferred(ell) tells
  // whether level ell's tables are such, level_transfer(ell) builds them if
  // needed and returns level(ell).
  bool transfer_deferred(int ell) const;
  const Level& level_transfer(int ell) const;
  const Level& leaf() const { return levels_[L_]; }
  int64_t n_active() const { return int64_t(lev_.size()); }

  // physical Gauss points of the leaf cells [ncell][q^3][3], q = quad_points()
  void leaf_quadrature_points(double* out) const;

  // local-smoothing hierarchy: levels 1 .. local_base() are the uniform
  // global-coarsening levels (every cell of the level exists), the finer
  // ones local_level(ell); local_base() == L() for a uniform leaf mesh.
  // local_base_copy_*: leaf free nodes whose finest level is local_base().
  // (built on first use)
  int local_base() const {
    ensure_local();
    return ls_base_;
  }
  const LocalLevel& local_level(int ell) const {
    ensure_local();
    return ls_[size_t(ell)];
  }
  const std::vector<int32_t>& local_base_copy_leaf() const {
    ensure_local();
    return ls_base_leaf_;
  }
  const std::vector<int32_t>& local_base_copy_node() const {
    ensure_local();
    return ls_base_node_;
  }

 private:
  void balance();
  void build_level(int ell);
  void build_nodes(Level& lv, bool q1) const;
  void build_transfer(int ell);
  void build_mu_restriction(int ell);
  void ensure_local() const;
  void build_local_smoothing() const;
  void build_local_transfer(int ell) const;

  std::vector<int32_t> lev_;   // active cells
  std::vector<int32_t> ijk_;
  bool finalized_ = false;
  bool noflux_ = false;
  int vdeg_ = 2;
  std::vector<Level> q3_;   // Q3-Q2 lattice levels (velocity degree 3)
  int L_ = 0;
  std::vector<Level> levels_;
  // local-smoothing levels, built from the finished global-coarsening levels
  mutable bool ls_built_ = false;
  mutable std::vector<uint8_t> transfer_built_;
  mutable int ls_base_ = 0;
  mutable std::vector<LocalLevel> ls_;
  mutable std::vector<int32_t> ls_base_leaf_, ls_base_node_;
};

// 1D Q2 Lagrange basis on {0, 1/2, 1} evaluated at t
void q2_basis_1d(double t, double v[3]);
void q2_deriv_1d(double t, double v[3]);

}  // namespace mfgmg
