"""Unit-cube octree meshes, global-coarsening level meshes, nodes and constraints.

Test infrastructure (see ``oracle/__init__``).

Paper: the solver works on adaptively refined meshes of the unit cube
(abstract; Sec. 3.2 defines the domain) with a geometric level hierarchy
(Sec. 2.2.1) and homogeneous Dirichlet velocity data on the whole boundary
(Sec. 2, eq. stokes).  The paper does not say how meshes are balanced, which
hierarchy is used, or how hanging nodes are treated.  Readings:

* 2:1 balance across faces, edges and vertices, so that no hanging node is
  constrained against another hanging node;
* global coarsening: level mesh G_l is the leaf mesh with every cell finer
  than l replaced by its level-l ancestor, for l = 1 .. L (L = finest level),
  so G_L is the leaf mesh and G_1 the 2x2x2 coarse mesh;
* Lagrange support points on {0, 1/2, 1} (Q2) and {0, 1} (Q1); a node that
  lies on the closed box of a cell without being one of that cell's own nodes
  is hanging, and its value is that cell's interpolant at the node;
* Dirichlet wins over hanging; constrained (Dirichlet or hanging) rows become
  identity rows.

Integer geometry: with U = L + 1 (L the finest cell level of the leaf mesh),
every Q2 node of every level mesh has integer coordinates in units of 2^-U,
in [0, S] with S = 2^U.  Its canonical key is X + (S+1) (Y + (S+1) Z).
"""
import numpy as np
import scipy.sparse as sp

from . import fe


# --------------------------------------------------------------------- octree
def cell_code(lev, ijk):
    """Unique integer per octree node (level, i, j, k)."""
    lev = np.asarray(lev, dtype=np.int64)
    ijk = np.asarray(ijk, dtype=np.int64)
    off = ((np.int64(1) << (3 * lev)) - 1) // 7
    n = np.int64(1) << lev
    return off + ijk[..., 0] + n * (ijk[..., 1] + n * ijk[..., 2])


def uniform_leaves(L):
    """All 8^L cells of level L, x index fastest."""
    n = 1 << L
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing='ij')
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.int64)
    return np.full(len(ijk), L, dtype=np.int64), ijk


def children(lev, ijk):
    """The 8 children of each cell, child c = (cx + 2 cy + 4 cz)."""
    off = np.array([(a, b, c) for c in range(2) for b in range(2) for a in range(2)], dtype=np.int64)
    cij = (2 * ijk[:, None, :] + off[None, :, :]).reshape(-1, 3)
    return np.repeat(lev + 1, 8), cij


def refine(lev, ijk, mask, times=1):
    """Replace every masked cell by its descendants ``times`` levels down."""
    mask = np.asarray(mask, dtype=bool)
    keep_l, keep_c = lev[~mask], ijk[~mask]
    rl, rc = lev[mask], ijk[mask]
    for _ in range(times):
        rl, rc = children(rl, rc)
    return np.concatenate([keep_l, rl]), np.concatenate([keep_c, rc])


def _neighbour_offsets():
    return np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)
                     if (a, b, c) != (0, 0, 0)], dtype=np.int64)


def covering_leaf(lev_q, ijk_q, leaf_codes_sorted, max_level):
    """For query cells (level, ijk), the level of the leaf that contains them
    (the query itself or an ancestor), or -1 if the region is covered by finer
    leaves."""
    found = np.full(len(lev_q), -1, dtype=np.int64)
    for m in range(max_level, -1, -1):
        cand = (found < 0) & (lev_q >= m)
        if not cand.any():
            continue
        shift = (lev_q[cand] - m)
        anc = ijk_q[cand] >> shift[:, None]
        code = cell_code(np.full(cand.sum(), m), anc)
        pos = np.searchsorted(leaf_codes_sorted, code)
        pos = np.minimum(pos, len(leaf_codes_sorted) - 1)
        hit = leaf_codes_sorted[pos] == code
        idx = np.nonzero(cand)[0][hit]
        found[idx] = m
    return found


def balance(lev, ijk):
    """2:1 balance across faces, edges and vertices: refine any leaf that
    touches a leaf more than one level finer, until none is left."""
    offs = _neighbour_offsets()
    while True:
        codes = np.sort(cell_code(lev, ijk))
        max_level = int(lev.max())
        nq = ijk[:, None, :] + offs[None, :, :]               # [n, 26, 3]
        lq = np.repeat(lev[:, None], 26, axis=1)
        n_at = (np.int64(1) << lq)[..., None]
        inside = np.all((nq >= 0) & (nq < n_at), axis=2)
        lq, nq = lq[inside], nq[inside]
        cov = covering_leaf(lq, nq, codes, max_level)
        bad = (cov >= 0) & (cov < lq - 1)
        if not bad.any():
            return lev, ijk
        anc = nq[bad] >> (lq[bad] - cov[bad])[:, None]
        bad_codes = np.unique(cell_code(cov[bad], anc))
        mask = np.isin(cell_code(lev, ijk), bad_codes)
        lev, ijk = refine(lev, ijk, mask, 1)


def morton_code(xyz, bits):
    """Interleave the bits of integer coordinates [n, 3] (x lowest)."""
    xyz = np.asarray(xyz, dtype=np.uint64)
    code = np.zeros(len(xyz), dtype=np.uint64)
    for b in range(bits):
        for d in range(3):
            code |= ((xyz[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return code


def morton_sort(lev, ijk):
    """Sort cells by the Morton code of their origin at the finest level."""
    U = int(lev.max())
    org = ijk << (U - lev)[:, None]
    order = np.argsort(morton_code(org, U + 1), kind='stable')
    return lev[order], ijk[order]


def level_cells(lev, ijk, ell):
    """Cells of the global-coarsening level mesh G_ell (leaf cells finer than
    ell replaced by their level-ell ancestor), Morton sorted."""
    fine = lev > ell
    anc = ijk[fine] >> (lev[fine] - ell)[:, None]
    l2 = np.concatenate([lev[~fine], np.full(len(anc), ell)])
    c2 = np.concatenate([ijk[~fine], anc])
    codes, first = np.unique(cell_code(l2, c2), return_index=True)
    l2, c2 = l2[first], c2[first]
    U = int(lev.max())
    org = c2 << (U - l2)[:, None]
    order = np.argsort(morton_code(org, U + 1), kind='stable')
    return l2[order], c2[order]


# ---------------------------------------------------------------- level mesh
Q2_OFF = np.array([(a, b, c) for c in range(3) for b in range(3) for a in range(3)], dtype=np.int64)
Q1_OFF = np.array([(a, b, c) for c in range(2) for b in range(2) for a in range(2)], dtype=np.int64)
_L5 = np.array([(a, b, c) for c in range(5) for b in range(5) for a in range(5)], dtype=np.int64)
# boundary points of the 5^3 quarter lattice that are not Q2 nodes of the cell
Q2_HANG_CAND = _L5[np.any((_L5 == 0) | (_L5 == 4), axis=1) & np.any(_L5 % 2 == 1, axis=1)]
# boundary points of the 3^3 half lattice that are not Q1 nodes of the cell
_L3 = Q2_OFF
Q1_HANG_CAND = _L3[np.any((_L3 == 0) | (_L3 == 2), axis=1) & np.any(_L3 == 1, axis=1)]


class LevelMesh:
    """One mesh of the hierarchy with its Q2 (and optionally Q1) node sets.

    Attributes (n = number of cells, nn = number of Q2 nodes):
      lev, ijk   [n], [n, 3]  cell level and integer position at that level
      U, S       unit exponent and lattice size (coordinates in units 2^-U)
      h          [n]          cell edge length 2^-lev
      keys       [nn]         sorted canonical Q2 node keys
      xyz        [nn, 3]      integer node coordinates
      cell_nodes [n, 27]      node index of each local Q2 node
      dirichlet, hanging, free [nn] bool
      C          csr [nn, nn] node-level constraint matrix: x_full = C x;
                 identity on free nodes, interpolation weights on hanging
                 nodes (free masters only), zero rows on Dirichlet nodes.
      bc         boundary condition of the velocity (Sec. 2, eq. stokes):
                 "dirichlet": u = 0 on the boundary (every component of a
                 boundary node is fixed; Dirichlet wins over hanging);
                 "noflux": u . n = 0, read on the axis-aligned unit cube as
                 "component c vanishes on the two faces normal to axis c"
                 (edge and corner nodes fix two or three components); the
                 tangential components stay free, their condition (zero
                 tangential stress) is the natural one of the weak form.
                 Boundary nodes are then free or hanging at node level, and
                 the fixed components are removed per dof in ``Cu``.
      fixed      [nn, 3] bool  components fixed by the boundary condition
    """

    def __init__(self, lev, ijk, U, with_pressure=False, bc="dirichlet"):
        assert bc in ("dirichlet", "noflux"), bc
        self.bc = bc
        self.lev = np.asarray(lev, dtype=np.int64)
        self.ijk = np.asarray(ijk, dtype=np.int64)
        self.U = int(U)
        self.S = 1 << self.U
        self.h = 2.0 ** (-self.lev.astype(np.float64))
        self.ncell = len(self.lev)
        self._build_q2()
        if with_pressure:
            self._build_q1()

    # -- keys
    def key(self, xyz):
        S1 = self.S + 1
        xyz = np.asarray(xyz, dtype=np.int64)
        return xyz[..., 0] + S1 * (xyz[..., 1] + S1 * xyz[..., 2])

    def unkey(self, key):
        S1 = self.S + 1
        key = np.asarray(key, dtype=np.int64)
        return np.stack([key % S1, (key // S1) % S1, key // (S1 * S1)], axis=-1)

    def cell_origin(self):
        return self.ijk << (self.U - self.lev)[:, None]

    def cell_size_units(self):
        return np.int64(1) << (self.U - self.lev)

    def _lookup(self, keys_sorted, q):
        pos = np.searchsorted(keys_sorted, q)
        pos = np.minimum(pos, len(keys_sorted) - 1)
        return pos, keys_sorted[pos] == q

    def _hanging(self, keys_sorted, natural_off, cand_off, denom, basis):
        """Find hanging nodes: lattice points on a cell's closed box that are
        nodes of the mesh but not nodes of that cell.  Returns dict
        key -> (master keys, weights) from the cell's interpolant."""
        org = self.cell_origin()
        size = self.cell_size_units()
        # cells of the finest level cannot have finer neighbours
        ok = (size % (2 * denom)) == 0
        cons = {}
        if not ok.any() or len(cand_off) == 0:
            return cons
        o, s = org[ok], size[ok]
        step = s // (2 * denom)                                   # quarter / half
        pts = o[:, None, :] + cand_off[None, :, :] * step[:, None, None]
        q = self.key(pts)
        pos, hit = self._lookup(keys_sorted, q)
        ci, pi = np.nonzero(hit)
        if len(ci) == 0:
            return cons
        local = cand_off[pi] / (2.0 * denom)                      # local position in [0,1]^3
        w, _ = basis(local)                                       # [nb, nh]
        w = w.T
        nat = o[ci][:, None, :] + natural_off[None, :, :] * (s[ci] // denom)[:, None, None]
        mkeys = self.key(nat)
        for r in range(len(ci)):
            k = int(q[ci[r], pi[r]])
            if k in cons:
                continue
            nz = np.abs(w[r]) > 1e-14
            cons[k] = (mkeys[r][nz], w[r][nz])
        return cons

    def _constraint_matrix(self, keys, hanging_map, dirichlet):
        nn = len(keys)
        hanging = np.zeros(nn, dtype=bool)
        rows, cols, vals = [], [], []
        for k, (mk, w) in hanging_map.items():
            i = int(np.searchsorted(keys, k))
            if dirichlet[i]:
                continue
            hanging[i] = True
            mi = np.searchsorted(keys, mk)
            assert np.all(keys[mi] == mk)
            for m, ww in zip(mi, w):
                if dirichlet[m]:
                    continue
                rows.append(i), cols.append(int(m)), vals.append(float(ww))
        free = ~(hanging | dirichlet)
        # masters of a hanging node must be free (balance guarantees it)
        if len(cols):
            assert np.all(free[np.array(cols)]), "hanging node constrained against a constrained node"
        fi = np.nonzero(free)[0]
        rows = np.concatenate([fi, np.array(rows, dtype=np.int64)])
        cols = np.concatenate([fi, np.array(cols, dtype=np.int64)])
        vals = np.concatenate([np.ones(len(fi)), np.array(vals)])
        C = sp.csr_matrix((vals, (rows, cols)), shape=(nn, nn))
        return hanging, free, C

    def _build_q2(self):
        org = self.cell_origin()
        half = self.cell_size_units() // 2
        pts = org[:, None, :] + Q2_OFF[None, :, :] * half[:, None, None]
        allk = self.key(pts)
        self.keys = np.unique(allk)
        self.cell_nodes = np.searchsorted(self.keys, allk)
        self.xyz = self.unkey(self.keys)
        on_bnd = (self.xyz == 0) | (self.xyz == self.S)            # [nn, 3] per axis
        if self.bc == "dirichlet":
            self.dirichlet = np.any(on_bnd, axis=1)
            self.fixed = np.repeat(self.dirichlet[:, None], 3, axis=1)
        else:
            self.dirichlet = np.zeros(len(self.keys), dtype=bool)
            self.fixed = on_bnd
        hmap = self._hanging(self.keys, Q2_OFF, Q2_HANG_CAND, 2,
                             lambda loc: fe.q2_basis(loc))
        self._hmap = hmap
        self.hanging, self.free, self.C = self._constraint_matrix(self.keys, hmap, self.dirichlet)
        self.nnode = len(self.keys)

    def _build_q1(self):
        org = self.cell_origin()
        size = self.cell_size_units()
        pts = org[:, None, :] + Q1_OFF[None, :, :] * size[:, None, None]
        allk = self.key(pts)
        self.pkeys = np.unique(allk)
        self.cell_pnodes = np.searchsorted(self.pkeys, allk)
        nodir = np.zeros(len(self.pkeys), dtype=bool)
        hmap = self._hanging(self.pkeys, Q1_OFF, Q1_HANG_CAND, 1,
                             lambda loc: fe.q1_basis(loc))
        self.phanging, self.pfree, self.Cp = self._constraint_matrix(self.pkeys, hmap, nodir)
        self.npnode = len(self.pkeys)

    def C_no_dirichlet(self):
        """Constraint matrix with hanging constraints only (no boundary
        condition): used to check the operator's null space."""
        nodir = np.zeros(self.nnode, dtype=bool)
        hanging, free, C = self._constraint_matrix(self.keys, self._hmap, nodir)
        return hanging, free, C

    # -- dof helpers (velocity dof = 3 node + component)
    @property
    def n_u(self):
        return 3 * self.nnode

    def cell_dofs(self):
        return (3 * self.cell_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(self.ncell, 81)

    def free_dofs_mask(self):
        return np.repeat(self.free, 3) & ~self.fixed.ravel()

    def Cu(self):
        """Dof-level constraint matrix: kron(C, I_3), and for "noflux" the rows
        and columns of the components fixed by u . n = 0 zeroed (a hanging
        node's component interpolates the same component of its masters, and
        a master's fixed component carries zero)."""
        Cu = sp.kron(self.C, sp.identity(3), format='csr')
        if self.bc == "noflux":
            D = sp.diags((~self.fixed.ravel()).astype(np.float64))
            Cu = (D @ Cu @ D).tocsr()
        return Cu

    def node_positions(self):
        return self.xyz.astype(np.float64) / self.S

    def cell_centres(self):
        return (self.cell_origin() + self.cell_size_units()[:, None] / 2.0) / self.S


class Hierarchy:
    """Leaf mesh plus its global-coarsening level meshes G_1 .. G_L."""

    def __init__(self, lev, ijk, bc="dirichlet"):
        lev, ijk = morton_sort(np.asarray(lev, dtype=np.int64), np.asarray(ijk, dtype=np.int64))
        self.L = int(lev.max())
        assert int(lev.min()) >= 1, "the coarsest level mesh is the 2x2x2 mesh"
        self.U = self.L + 1
        self.bc = bc
        self.levels = {}
        for ell in range(1, self.L + 1):
            l2, c2 = level_cells(lev, ijk, ell)
            self.levels[ell] = LevelMesh(l2, c2, self.U, with_pressure=(ell == self.L), bc=bc)
        self.leaf = self.levels[self.L]

    @staticmethod
    def uniform(L, bc="dirichlet"):
        return Hierarchy(*uniform_leaves(L), bc=bc)

    def parent_map(self, ell):
        """For each cell of G_ell (ell >= 2): index in G_{ell-1} of the cell that
        contains it (itself if it is also a cell of G_{ell-1})."""
        fine, coarse = self.levels[ell], self.levels[ell - 1]
        pl = np.minimum(fine.lev, ell - 1)
        pc = fine.ijk >> (fine.lev - pl)[:, None]
        ccode = cell_code(coarse.lev, coarse.ijk)
        order = np.argsort(ccode)
        q = cell_code(pl, pc)
        pos = np.searchsorted(ccode[order], q)
        assert np.all(ccode[order][pos] == q)
        return order[pos]
