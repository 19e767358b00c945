"""Shared set-up for the device parity tests: the same mesh, viscosity and
seeded vectors on the library and on the oracle, with maps between the two
node numberings by canonical key."""
import numpy as np

from oracle import mesh as omesh, operators as ops
from paper_1907_06696_amd import inputs, mfgmg


class Case:
    """Library solver + oracle hierarchy for one mesh and one sinker field."""

    def __init__(self, base, corners=(), times=1, sinkers=4, dr=1e3, seed=1, refine_cells=None,
                 build_oracle=True):
        self.s = mfgmg.Solver(base)
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
            self.H = omesh.Hierarchy(lev, ijk)
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
