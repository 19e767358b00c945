// The Taylor-Hood Q3-Q2 pair (k = 2 of Sec. 2.1, [Q_{k+1}]^3 x Q_k) on
// uniform meshes of the unit cube: reference element data and the lattice
// level meshes.  Host only.
//
// Support points are the Gauss-Lobatto points of each direction ({0,
// (1 -+ 1/sqrt 5)/2, 1} for Q3, {0, 1/2, 1} for the Q2 pressure); every form
// of Sec. 2.1 is integrated exactly by 4 Gauss points per direction on an
// axis-aligned cube with cell-constant viscosity.  A level of n = 2^l cells
// per edge numbers its Q3 nodes X + m (Y + m Z) on the lattice of m = 3n + 1
// points per axis (cell (i, j, k), local node (a, b, c): X = 3i + a, ...);
// the leaf's Q2 pressure nodes likewise on the (2n + 1)^3 lattice.
#pragma once

#include <cstdint>
#include <vector>

#include "mesh.h"

namespace mfgmg {

struct Q3Element {
  double gll[4];     // Q3 support points on [0, 1]
  double xg[4], wg[4];   // 4-point Gauss rule on [0, 1]
  double N[4][4];    // N[q][a] = L_a(xg_q): nodal values -> Gauss points
  double D[4][4];    // D[q][r] = l_r'(xg_q), l_r the Lagrange basis on the Gauss points
  double P2[4][3];   // Q2 pressure basis at the Gauss points
  double M2[3][3];   // 1D Q2 mass matrix
  std::vector<double> K;   // [192 x 192] int 2 eps(phi_(a,c)) : eps(phi_(b,d)), mu = 1, dof 3a + c
};
const Q3Element& q3_element();

// Level ell (n = 2^ell cells per edge) of the uniform Q3-Q2 hierarchy with
// u = 0 on the boundary: cells from `cells` (the mesh's level ell, uniform),
// lattice nodes and their types, and for ell >= 2 the node-level
// prolongation from level ell - 1 (coarse Q3 functions at the fine lattice
// points; rows of boundary nodes empty, boundary columns dropped) and its
// transpose; on the leaf the Q2 pressure lattice (no constraints).
void build_q3_level(const Level& cells, bool leaf, Level& out);

}  // namespace mfgmg
