"""Local-smoothing V-cycle: the multigrid hierarchy of level meshes only.

Test infrastructure (see ``oracle/__init__``).

Paper, Sec. 2.2.1: the velocity block is preconditioned by the matrix-free
GMG V-cycle of Clevenger et al. (cited there; the cell viscosity of the
levels is restricted as in Sec. 2.3).  That method smooths locally: level l
holds only the cells of refinement level l (the level mesh T_l, which covers
the part Omega_l of the domain refined at least to level l), its smoother
acts on the level-l functions that vanish on the refinement edge (the part of
the boundary of Omega_l inside the domain), and the coupling of interior and
edge degrees of freedom is carried between the levels.  The paper gives no
more detail; the reading here, written out as a subspace correction:

* level space V_l = continuous Q2 functions on T_l that vanish on the
  refinement edge and on the boundary of the domain, extended by zero: a
  subspace of the adaptive (leaf) space with its hanging-node constraints;
* one V-cycle = the symmetric multiplicative correction over V_L, ..., V_2,
  V_1, V_2, ..., V_L: x += E_l S_l E_l^T (b - A x) on each level, where E_l
  maps level coefficients to leaf coefficients, S_l is the degree-4
  Chebyshev smoother of the level operator A_l = E_l^T A E_l (Jacobi, the
  interval rule of ``multigrid``), and V_1 (the 2x2x2 mesh) is solved
  exactly;
* computed level by level, as the method does it: every free leaf node is
  copied to the finest level whose cells hold it; on level l the defect is
  kept on all level nodes including the refinement edge E; after the
  pre-smoothing y (zero on E) the residual t = d - K_l y over all level
  nodes (K_l: the level operator with the edge nodes free, so its edge rows
  give the interface coupling K_EI y) is restricted to level l - 1; the
  coarse correction z = P_l y_{l-1} is kept on E too, and the post-smoothing
  solves A_II y_I = d_I - K_IE z_E from y; finally every free leaf node
  takes the value of the finest level that holds it.

``subspace_correction`` evaluates the first form with explicit matrices (for
the pins); ``LocalSmoothingGMG.vcycle`` the second.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fe
from . import multigrid as mg
from . import operators as ops
from . import rng
from .mesh import LevelMesh, Q2_OFF, cell_code


def level_cells_exact(hier, ell):
    """Cells of refinement level exactly ell (T_ell): the level-ell cells of
    the global-coarsening level mesh G_ell, with their viscosity index."""
    g = hier.levels[ell]
    sel = np.nonzero(g.lev == ell)[0]
    return g.lev[sel], g.ijk[sel], sel


def refinement_edge_mask(mesh):
    """[nnode] True for nodes of T_l on the boundary of Omega_l inside the
    domain: some level-l cell position touching the node (inside the unit
    cube) holds no cell of T_l."""
    ell = int(mesh.lev[0])
    s = np.int64(1) << (mesh.U - ell)           # cell size in lattice units
    n = np.int64(1) << ell
    codes = np.sort(cell_code(mesh.lev, mesh.ijk))
    xyz = mesh.xyz
    edge = np.zeros(mesh.nnode, dtype=bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                d = np.array([dx, dy, dz])
                # candidate cell index along each axis: on a cell boundary the
                # node touches cells c-1 and c, inside a cell only c = floor
                on = (xyz % s) == 0
                base = xyz // s
                c = np.where(on, base - 1 + d[None, :], base)
                # skip duplicate candidates off the boundary (d = 1 where not on)
                dup = np.any((~on) & (d[None, :] == 1), axis=1)
                inside = np.all((c >= 0) & (c < n), axis=1)
                q = cell_code(np.full(len(c), ell), c)
                pos = np.minimum(np.searchsorted(codes, q), len(codes) - 1)
                missing = codes[pos] != q
                edge |= inside & ~dup & missing
    return edge & ~mesh.dirichlet


def prolongation_children(fine, coarse):
    """P: T_{l-1} -> T_l, node level: the resolved Q2 function of each refined
    level-(l-1) cell interpolated at its children's nodes (every T_l cell is
    such a child).  Rows of Dirichlet fine nodes are zero; refinement-edge
    rows are kept."""
    corg = coarse.cell_origin()
    csize = coarse.cell_size_units()
    pcodes = np.unique(cell_code(fine.lev - 1, fine.ijk >> 1))
    r_idx = np.nonzero(np.isin(cell_code(coarse.lev, coarse.ijk), pcodes))[0]
    L5 = np.array([(a, b, c) for c in range(5) for b in range(5) for a in range(5)])
    pts = corg[r_idx][:, None, :] + L5[None] * (csize[r_idx] // 4)[:, None, None]
    fk = fine.key(pts).ravel()
    fi = np.searchsorted(fine.keys, fk)
    ok = (fi < len(fine.keys))
    ok[ok] = fine.keys[fi[ok]] == fk[ok]
    W = np.tile(ops._W125, (len(r_idx), 1))
    cnod = np.repeat(coarse.cell_nodes[r_idx], 125, axis=0)
    fi, W, cnod = fi[ok], W[ok], cnod[ok]
    _, first = np.unique(fi, return_index=True)
    assert len(first) == fine.nnode
    rows = np.repeat(fi[first], 27)
    cols = cnod[first].ravel()
    vals = W[first].ravel()
    nz = vals != 0
    I = sp.csr_matrix((vals[nz], (rows[nz], cols[nz])), shape=(fine.nnode, coarse.nnode))
    Pn = sp.diags((~fine.dirichlet).astype(np.float64)) @ I @ sp.diags((~coarse.dirichlet).astype(np.float64))
    return sp.kron(Pn.tocsr(), sp.identity(3), format='csr')


class LocalSmoothingGMG:
    """Local-smoothing V-cycle on the hierarchy T_1 .. T_L of a leaf mesh.

    hier: ``mesh.Hierarchy`` (its global-coarsening meshes G_l give the
    level-l cells and, through ``mus``, their viscosity: children averaged
    onto parents, Sec. 2.3)."""

    def __init__(self, hier, mus, seed=mg.LAMBDA_SEED):
        assert hier.bc == "dirichlet", "local smoothing is built for the Dirichlet condition"
        self.hier = hier
        self.L = hier.L
        self.T, self.K, self.A, self.P, self.minv, self.lam = {}, {}, {}, {}, {}, {}
        self.edge, self.inner = {}, {}
        for ell in range(1, self.L + 1):
            lev, ijk, sel = level_cells_exact(hier, ell)
            m = LevelMesh(lev, ijk, hier.U)
            assert not m.hanging.any()
            self.T[ell] = m
            mu = mus[ell][sel]
            K = ops.assemble_A(m, mu)                  # Dirichlet on the domain boundary only
            edge = refinement_edge_mask(m)
            self.edge[ell] = np.repeat(edge, 3)
            inner = np.repeat(~(edge | m.dirichlet), 3)
            self.inner[ell] = inner
            keep = sp.diags(inner.astype(np.float64))
            self.K[ell] = K
            self.A[ell] = (keep @ K @ keep + sp.diags((~inner).astype(np.float64))).tocsr()
            self.minv[ell] = np.where(inner, 1.0 / self.A[ell].diagonal(), 1.0)
            if ell >= 2:
                self.P[ell] = prolongation_children(m, self.T[ell - 1])
                r0 = rng.dof_vector(m, seed) * inner
                self.lam[ell] = mg.LAMBDA_SAFETY * mg.cg_lanczos_lambda_max(
                    lambda v: self.A[ell] @ v, self.minv[ell], r0)
        assert not self.edge[1].any()
        A1 = self.A[1].toarray()
        self.coarse_free = np.nonzero(self.inner[1])[0]
        self.coarse_chol = sla.cho_factor(A1[np.ix_(self.coarse_free, self.coarse_free)])
        # leaf free node -> finest level holding it
        leaf = hier.leaf
        self.leaf_free = np.nonzero(leaf.free)[0]
        keys = leaf.keys[self.leaf_free]
        self.copy = {}
        taken = np.zeros(len(keys), dtype=bool)
        for ell in range(self.L, 0, -1):
            tk = self.T[ell].keys
            pos = np.minimum(np.searchsorted(tk, keys), len(tk) - 1)
            hit = (tk[pos] == keys) & ~taken
            self.copy[ell] = (self.leaf_free[hit], pos[hit])    # (leaf node, level node)
            taken |= hit
        assert taken.all()

    def _dofs(self, nodes):
        return (3 * np.asarray(nodes)[:, None] + np.arange(3)[None, :]).ravel()

    def coarse_solve(self, b):
        x = np.zeros_like(b)
        x[self.coarse_free] = sla.cho_solve(self.coarse_chol, b[self.coarse_free])
        return x

    def smooth(self, ell, b, x=None):
        return mg.chebyshev(lambda v: self.A[ell] @ v, self.minv[ell], b, x, self.lam[ell], x_is_zero=x is None)

    def vcycle(self, b):
        """x = V(b) for a leaf vector b (zero on constrained leaf dofs)."""
        d = {ell: np.zeros(self.T[ell].n_u) for ell in range(1, self.L + 1)}
        for ell, (lf, lv) in self.copy.items():
            d[ell][self._dofs(lv)] = b[self._dofs(lf)]
        ys = self._vc(self.L, d)
        x = np.zeros_like(b)
        for ell, (lf, lv) in self.copy.items():
            x[self._dofs(lf)] = ys[ell][self._dofs(lv)]
        return x

    def _vc(self, ell, d):
        if ell == 1:
            return {1: self.coarse_solve(d[1])}
        inner, edge = self.inner[ell], self.edge[ell]
        y = self.smooth(ell, np.where(inner, d[ell], 0.0))
        t = d[ell] - self.K[ell] @ y
        d[ell - 1] = d[ell - 1] + self.P[ell].T @ t
        ys = self._vc(ell - 1, d)
        z = self.P[ell] @ ys[ell - 1]
        y = y + np.where(inner | edge, z, 0.0)
        yE = np.where(edge, y, 0.0)
        rhs = np.where(inner, d[ell] - self.K[ell] @ yE, 0.0) + yE
        ys[ell] = self.smooth(ell, rhs, y)
        return ys


def level_basis(ls, ell):
    """E_l: leaf coefficients (columns) of the level-l basis functions of the
    interior level dofs, by evaluating each level-l Lagrange basis function at
    the leaf free nodes (a leaf node in the closed box of a T_l cell takes that
    cell's interpolant, the same from every such cell as the function is
    continuous; outside Omega_l the function is zero).  Built without the
    transfer matrices.  Returns (E [n_u leaf, 3 n_inner], level dofs of the
    columns)."""
    T = ls.T[ell]
    leaf = ls.hier.leaf
    fx = leaf.xyz[ls.leaf_free].astype(np.float64)        # leaf free node coordinates (lattice units)
    org = T.cell_origin().astype(np.float64)
    size = float(T.cell_size_units()[0])
    inner_nodes = np.nonzero(ls.inner[ell][::3])[0]
    col_of = -np.ones(T.nnode, dtype=np.int64)
    col_of[inner_nodes] = np.arange(len(inner_nodes))
    vals = {}
    for c in range(T.ncell):
        loc = (fx - org[c]) / size
        idx = np.nonzero(np.all((loc >= 0) & (loc <= 1), axis=1))[0]
        if len(idx) == 0:
            continue
        w, _ = fe.q2_basis(loc[idx])                     # [27, npts]
        for a in range(27):
            j = col_of[T.cell_nodes[c, a]]
            if j < 0:
                continue
            for p, val in zip(idx, w[a]):
                if val != 0.0:
                    vals.setdefault((int(p), int(j)), float(val))
    rc = np.array(list(vals.keys()), dtype=np.int64).reshape(-1, 2)
    En = sp.csr_matrix((np.array(list(vals.values())), (rc[:, 0], rc[:, 1])),
                       shape=(len(ls.leaf_free), len(inner_nodes)))
    E = sp.kron(En, sp.identity(3), format='csr')          # rows 3 p + c, columns 3 j + c
    leaf_dofs = ls._dofs(ls.leaf_free)
    S = sp.csr_matrix((np.ones(len(leaf_dofs)), (leaf_dofs, np.arange(len(leaf_dofs)))),
                      shape=(leaf.n_u, len(leaf_dofs)))
    return (S @ E).tocsr(), ls._dofs(inner_nodes)


def subspace_correction(ls, A_leaf, b, E):
    """The symmetric multiplicative correction over V_L..V_2, V_1, V_2..V_L
    with explicit level bases E[l] = (leaf coefficients, level dofs) and the
    Galerkin level operators E_l^T A E_l."""
    x = np.zeros_like(b)
    gal = {}
    for ell in range(1, ls.L + 1):
        El, _ = E[ell]
        gal[ell] = (El.T @ A_leaf @ El).toarray()

    def correct(ell, r):
        El, _ = E[ell]
        rl = El.T @ r
        G = gal[ell]
        if ell == 1:
            return El @ np.linalg.solve(G, rl)
        minv = 1.0 / np.diag(G)
        return El @ mg.chebyshev(lambda v: G @ v, minv, rl, None, ls.lam[ell], x_is_zero=True)

    order = list(range(ls.L, 1, -1)) + [1] + list(range(2, ls.L + 1))
    for ell in order:
        x = x + correct(ell, b - A_leaf @ x)
    return x, gal
