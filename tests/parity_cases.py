"""Shared set-up for the device parity tests: the same mesh, viscosity and
seeded vectors on the library and on the oracle, with maps between the two
node numberings by canonical key."""
import numpy as np

from oracle import mesh as omesh, operators as ops
from paper_1907_06696_amd import inputs, mfgmg


class Case:
    """Library solver + oracle hierarchy for one mesh and one sinker field."""

    def __init__(self, base, corners=(), times=1, sinkers=4, dr=1e3, seed=1, refine_cells=None,
                 build_oracle=True, bc="dirichlet"):
        self.s = mfgmg.Solver(base)
        self.bc = bc
        if bc != "dirichlet":
            self.s.set_boundary(bc)
        lev, ijk = omesh.uniform_leaves(base)
        cells = None
        if refine_cells is not None:
            cells = np.asarray(refine_cells, dtype=np.int32).reshape(-1, 4)
        elif corners:
            cells = np.array([[base, *c] for c in corners], dtype=np.int32)
        if cells is not None and len(cells):
            self.s.refine(cells, times)
            code = omesh.cell_code(cells[:, 0], cells[:, 1:])
            mask = np.isin(omesh.cell_code(lev, ijk), code)
            lev, ijk = omesh.refine(lev, ijk, mask, times)
            lev, ijk = omesh.balance(lev, ijk)
        self.s.finalize_mesh()
        self.info = self.s.info()
        self.L = self.info["L"]
        self.centres = inputs.sinker_centres(sinkers, seed)
        self.dr = dr
        qp = self.s.leaf_quadrature_points()
        self.mu_qp_lib = inputs.sinker_mu(qp.reshape(-1, 3), self.centres, dr).reshape(-1, 27)
        self.f_qp_lib = inputs.sinker_force(qp.reshape(-1, 3), self.centres).reshape(-1, 27, 3)
        self.H = None
        if build_oracle:
            self.H = omesh.Hierarchy(lev, ijk, bc=bc)
            lf = self.H.leaf
            X = ops.gauss_points_of_cells(lf).reshape(-1, 3)
            self.mu_qp_or = inputs.sinker_mu(X, self.centres, dr).reshape(-1, 27)
            self.f_qp_or = inputs.sinker_force(X, self.centres).reshape(-1, 27, 3)
            self.mus = ops.level_viscosities(self.H, ops.harmonic_cell_viscosity(self.mu_qp_or))

    # ---- numbering maps (library index -> oracle index)
    def node_perm(self, level):
        keys = self.s.support_points(level)
        return np.searchsorted(self.H.levels[level].keys, keys)

    def dof_perm(self, level):
        p = self.node_perm(level)
        return (3 * p[:, None] + np.arange(3)[None, :]).ravel()

    def pnode_perm(self):
        return np.searchsorted(self.H.leaf.pkeys, self.s.support_points(self.L, 1))

    def cell_perm(self, level):
        cl = self.s.cells(level)
        om = self.H.levels[level]
        oc = omesh.cell_code(om.lev, om.ijk)
        order = np.argsort(oc)
        return order[np.searchsorted(oc[order], omesh.cell_code(cl[:, 0], cl[:, 1:]))]

    def close(self):
        self.s.close()


def rel_err(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def abs_bound(mesh, mu, x, chunk=65536):
    """(|C|^T |K| |C| + Pi_c) |x| with |K| = sum over cells of mu_K h |K_hat|:
    an entrywise upper bound of |A| |x| for A = C^T K C + Pi_c.  Rounding in
    any evaluation order of A x is bounded row by row by a multiple of this
    (the terms a computation gathers through the constraints and the cell
    matrices), however small the row's viscosity is against the largest."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    Cu = abs(mesh.Cu())
    kabs = np.abs(ops.khat())
    dofs = mesh.cell_dofs()
    scale = np.asarray(mu) * mesh.h
    xf = Cu @ x
    y = np.zeros(mesh.n_u)
    for s in range(0, len(dofs), chunk):
        d = dofs[s:s + chunk]
        loc = xf[d] @ kabs.T * scale[s:s + chunk, None]
        y += np.bincount(d.ravel(), weights=loc.ravel(), minlength=mesh.n_u)
    return Cu.T @ y + np.where(mesh.free_dofs_mask(), 0.0, x)


def row_err(a, b, bound):
    """max_i |a_i - b_i| / bound_i over the rows with bound_i > 0 (rows whose
    bound is 0 must match exactly)."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    pos = bound > 0
    assert np.all(d[~pos] == 0)
    return float((d[pos] / bound[pos]).max()) if pos.any() else 0.0
