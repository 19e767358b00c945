"""Operators of the Stokes system on a level mesh: A, B, M_p, F, transfers.

Test infrastructure (see ``oracle/__init__``).

Paper: the block system of Sec. 2.1 (eq. stokes_linear_system),
    [A  B^T] [U]   [F]
    [B  0  ] [P] = [0],
    A_ij = int 2 mu eps(phi_i) : eps(phi_j),  B_ij = -int (div phi_j) psi_i,
    F_j  = int phi_j . f,
the mu^{-1}-weighted pressure mass matrix of Sec. 2.2.2, and the cellwise
viscosity of Sec. 2.3 (harmonic mean over the quadrature points of a leaf cell;
parent = mean of its children on every coarser level).

Readings: constrained rows (Dirichlet, hanging) are identity rows, so with the
node-level constraint matrix C (x_full = C x) the level operator is
    A = C_u^T K C_u + Pi_c,
K the unconstrained sum of the element matrices mu_K h K_hat; likewise
B = C_p^T B_full C_u and M_p = C_p^T M_full C_p + Pi_cp.  Cell matrices follow
from the unit-cube ones by affine scaling (cell side h, constant mu_K):
K_e = mu_K h K_hat, B_e = h^2 B_hat, M_e = h^3 / mu_K M_hat.
Transfers: P_l = Pi_f^(l) I_l C^(l-1) (interpolate the resolved coarse Q2
function at the fine nodes, then zero constrained fine rows), R_l = P_l^T.
"""
import numpy as np
import scipy.sparse as sp

from . import fe
from .mesh import Q2_OFF

_KHAT, _BHAT, _MHAT = fe.element_matrices(3)


def khat():
    return _KHAT.copy()


# ----------------------------------------------------------------- viscosity
def harmonic_cell_viscosity(mu_qp):
    """Weighted harmonic mean over the 27 Gauss points of each cell:
    mu_K = sum_q w_q / sum_q (w_q / mu_q) (Sec. 2.3, harmonic averaging)."""
    _, w = fe.gauss_points_3d(3)
    mu_qp = np.asarray(mu_qp, dtype=np.float64)
    return w.sum() / (w[None, :] / mu_qp).sum(axis=1)


def level_viscosities(hier, mu_leaf):
    """Cell viscosity on every level mesh: leaf cells keep their value, a
    level-l octree node gets the arithmetic mean of its 8 children (Sec. 2.3)."""
    mus = {hier.L: np.asarray(mu_leaf, dtype=np.float64)}
    for ell in range(hier.L, 1, -1):
        pmap = hier.parent_map(ell)
        nc = hier.levels[ell - 1].ncell
        s = np.bincount(pmap, weights=mus[ell], minlength=nc)
        cnt = np.bincount(pmap, minlength=nc)
        mus[ell - 1] = s / cnt
    return mus


# ------------------------------------------------------------- assembly
def assemble_K(mesh, mu):
    """Unconstrained sum of mu_K h K_hat over the cells, as CSR [n_u, n_u]."""
    dofs = mesh.cell_dofs()
    scale = (np.asarray(mu) * mesh.h)
    rows = np.repeat(dofs, 81, axis=1).ravel()
    cols = np.tile(dofs, (1, 81)).ravel()
    vals = (scale[:, None, None] * _KHAT[None, :, :]).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n_u, mesh.n_u))


def constrained(Cu, Kfull, free_mask):
    """C^T K C + Pi_c: identity rows/cols on constrained dofs."""
    A = (Cu.T @ Kfull @ Cu).tocsr()
    diag_c = sp.diags((~free_mask).astype(np.float64))
    return (A + diag_c).tocsr()


def assemble_A(mesh, mu):
    return constrained(mesh.Cu(), assemble_K(mesh, mu), mesh.free_dofs_mask())


def assemble_B(mesh):
    """B = C_p^T B_full C_u, rows of hanging pressure nodes zero.  [n_p, n_u]"""
    dofs = mesh.cell_dofs()
    pn = mesh.cell_pnodes
    rows = np.repeat(pn, 81, axis=1).ravel()
    cols = np.tile(dofs, (1, 8)).ravel()
    vals = ((mesh.h ** 2)[:, None, None] * _BHAT[None, :, :]).ravel()
    Bf = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.npnode, mesh.n_u))
    return (mesh.Cp.T @ Bf @ mesh.Cu()).tocsr()


def assemble_Mp(mesh, mu):
    """mu^{-1}-weighted Q1 mass matrix with constraints (Sec. 2.2.2)."""
    pn = mesh.cell_pnodes
    rows = np.repeat(pn, 8, axis=1).ravel()
    cols = np.tile(pn, (1, 8)).ravel()
    vals = ((mesh.h ** 3 / np.asarray(mu))[:, None, None] * _MHAT[None, :, :]).ravel()
    Mf = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.npnode, mesh.npnode))
    return constrained(mesh.Cp, Mf, mesh.pfree)


def pressure_mean_weights(mesh):
    """m_j = int psi_j over the domain (for the zero-mean pressure reading)."""
    pn = mesh.cell_pnodes
    w1 = _MHAT.sum(axis=1)                      # int psi_i over the unit cube
    vals = ((mesh.h ** 3)[:, None] * w1[None, :]).ravel()
    mfull = np.bincount(pn.ravel(), weights=vals, minlength=mesh.npnode)
    return mesh.Cp.T @ mfull


def assemble_F_full(mesh, f_qp):
    """Unconstrained F with F_e[(a,c)] = h^3 sum_q w_q phi_a(x_q) f_c(x_q).
    f_qp: [ncell, 27, 3] body force at the Gauss points (x fastest)."""
    Fhat = fe.element_rhs_weights(3)                     # [27 nodes, 27 qp]
    Fe = np.einsum('aq,nqc->nac', Fhat, np.asarray(f_qp)) * (mesh.h ** 3)[:, None, None]
    return np.bincount(mesh.cell_dofs().ravel(), weights=Fe.reshape(-1), minlength=mesh.n_u)


def assemble_rhs(mesh, f_qp):
    """b_u = C_u^T F (constrained rows zero)."""
    return mesh.Cu().T @ assemble_F_full(mesh, f_qp)


def gauss_points_of_cells(mesh):
    """Physical Gauss points [ncell, 27, 3] of the cells of a level mesh."""
    pts, _ = fe.gauss_points_3d(3)
    org = mesh.cell_origin() / mesh.S
    return org[:, None, :] + pts[None, :, :] * mesh.h[:, None, None]


# --------------------------------------------------- cellwise (large meshes)
class CellwiseA:
    """A = C_u^T K C_u + Pi_c applied cell by cell with the 81x81 K_hat; used
    where the assembled matrix would not fit in memory.  Same operator as
    ``assemble_A``."""

    def __init__(self, mesh, mu):
        self.mesh = mesh
        self.scale = np.asarray(mu) * mesh.h
        self.dofs = mesh.cell_dofs()
        self.Cu = mesh.Cu()
        self.CuT = self.Cu.T.tocsr()
        self.free = mesh.free_dofs_mask()
        self.n = mesh.n_u

    def matvec(self, x, chunk=65536):
        x = np.asarray(x, dtype=np.float64)
        xf = self.Cu @ x
        y = np.zeros(self.n)
        for s in range(0, len(self.dofs), chunk):
            d = self.dofs[s:s + chunk]
            loc = xf[d] @ _KHAT.T * self.scale[s:s + chunk, None]
            y += np.bincount(d.ravel(), weights=loc.ravel(), minlength=self.n)
        return self.CuT @ y + np.where(self.free, 0.0, x)

    __matmul__ = matvec

    def diagonal(self):
        """diag(C_u^T K C_u) on free dofs, 1 on constrained dofs.  Cells without
        hanging nodes add mu_K h K_hat_jj; cells with hanging nodes add the
        diagonal of their resolved local matrix C_l^T K_e C_l."""
        mesh = self.mesh
        d = np.zeros(self.n)
        kd = np.diag(_KHAT)
        hang_node = mesh.hanging[mesh.cell_nodes]
        has_hang = np.any(hang_node, axis=1)
        reg = ~has_hang
        d += np.bincount(self.dofs[reg].ravel(),
                         weights=(self.scale[reg, None] * kd[None, :]).ravel(), minlength=self.n)
        # the same per-cell sum diag(C_l^T K_e C_l), taken for a batch of cells
        # at once: stacked resolved rows G = [C_l1; C_l2; ...] and the block
        # diagonal of their K_e give sum_cells diag(C_l^T K_e C_l) as the
        # column sums of G .* (blockdiag(K_e) G)
        hc = np.nonzero(has_hang)[0]
        kh = sp.csr_matrix(_KHAT)
        for s in range(0, len(hc), 2048):
            cs = hc[s:s + 2048]
            G = self.Cu[self.dofs[cs].ravel()]             # [81 nc, n] resolved local rows
            KG = sp.kron(sp.diags(self.scale[cs]), kh, format='csr') @ G
            d += np.asarray(G.multiply(KG).sum(axis=0)).ravel()
        return np.where(self.free, d, 1.0)


class CellwiseB:
    """B = C_p^T B_full C_u (rows of hanging pressure nodes zero) and its
    transpose applied cell by cell with the 8x81 B_hat scaled by h^2; the same
    operator as ``assemble_B`` for meshes where the assembled matrix (8 x 81
    entries per cell) would not fit in memory."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.dofs = mesh.cell_dofs()
        self.pn = mesh.cell_pnodes
        self.h2 = mesh.h ** 2
        self.Cu = mesh.Cu()
        self.CuT = self.Cu.T.tocsr()
        self.Cp = mesh.Cp
        self.CpT = mesh.Cp.T.tocsr()

    def matvec(self, u, chunk=65536):
        """B u -> [n_p]"""
        uf = self.Cu @ np.asarray(u, dtype=np.float64)
        out = np.zeros(self.mesh.npnode)
        for s in range(0, len(self.dofs), chunk):
            loc = uf[self.dofs[s:s + chunk]] @ _BHAT.T * self.h2[s:s + chunk, None]
            out += np.bincount(self.pn[s:s + chunk].ravel(), weights=loc.ravel(), minlength=self.mesh.npnode)
        return self.CpT @ out

    def rmatvec(self, p, chunk=65536):
        """B^T p -> [n_u]"""
        pf = self.Cp @ np.asarray(p, dtype=np.float64)
        out = np.zeros(self.mesh.n_u)
        for s in range(0, len(self.dofs), chunk):
            loc = pf[self.pn[s:s + chunk]] @ _BHAT * self.h2[s:s + chunk, None]
            out += np.bincount(self.dofs[s:s + chunk].ravel(), weights=loc.ravel(), minlength=self.mesh.n_u)
        return self.CuT @ out


def stokes_residual(mesh, mu, rhs_u, u, p, rhs_p=None, ops_AB=None):
    """Relative residual ||b - K x||_2 / ||b||_2 of the block system of
    Sec. 2.1 (constrained rows identity, R4) for velocity u and pressure p
    given on the mesh's dofs (constrained entries are taken as zero), by the
    cellwise operators (ops_AB: a prebuilt (CellwiseA, CellwiseB) pair)."""
    A, B = ops_AB if ops_AB is not None else (CellwiseA(mesh, mu), CellwiseB(mesh))
    u = np.where(mesh.free_dofs_mask(), u, 0.0)
    p = np.where(mesh.pfree, p, 0.0)
    ru = rhs_u - A.matvec(u) - B.rmatvec(p)
    bp = np.zeros(mesh.npnode) if rhs_p is None else rhs_p
    rp = bp - B.matvec(u)
    nb = np.sqrt(np.dot(rhs_u, rhs_u) + np.dot(bp, bp))
    return float(np.sqrt(np.dot(ru, ru) + np.dot(rp, rp)) / nb)


# ---------------------------------------------------------------- transfers
_P1D = np.array([[1, 0, 0], [3 / 8, 3 / 4, -1 / 8], [0, 1, 0], [-1 / 8, 3 / 4, 3 / 8], [0, 0, 1]])


_L5 = np.array([(a, b, c) for c in range(5) for b in range(5) for a in range(5)])
# W125[r, s]: weight of coarse local node s (3^3, x fastest) at fine point r (5^3)
_W125 = np.einsum('ia,jb,kc->kjicba', _P1D, _P1D, _P1D).reshape(125, 27)


def prolongation(hier, ell, dirichlet=True):
    """P_l = Pi_f^(l) I_l C^(l-1) as CSR [n_u(l), n_u(l-1)] (velocity dofs).

    For a cell of G_{l-1} refined in G_l its resolved Q2 function is evaluated
    at the 5^3 child nodes (1D matrix _P1D: rows are the fine positions 0, 1/4,
    1/2, 3/4, 1, columns the coarse nodes 0, 1/2, 1); for a cell present on
    both levels the nodes coincide.  A fine node shared by several coarse cells
    gets the same value from each (the coarse function is continuous), so the
    first one is kept.  Fine constrained rows are zeroed; under the
    no-normal-flux condition the fixed components of either level carry and
    receive nothing (rows and columns of kron(., I_3) zeroed per dof)."""
    fine, coarse = hier.levels[ell], hier.levels[ell - 1]
    corg = coarse.cell_origin()
    csize = coarse.cell_size_units()
    refined = np.isin(cell_code_of(coarse), cell_code_parents(fine))
    r_idx = np.nonzero(refined)[0]
    k_idx = np.nonzero(~refined)[0]
    pts_r = corg[r_idx][:, None, :] + _L5[None] * (csize[r_idx] // 4)[:, None, None]
    pts_k = corg[k_idx][:, None, :] + Q2_OFF[None] * (csize[k_idx] // 2)[:, None, None]
    fk = np.concatenate([fine.key(pts_r).ravel(), fine.key(pts_k).ravel()])
    fi = np.searchsorted(fine.keys, fk)
    assert np.all(fine.keys[fi] == fk)
    # weight rows [npts, 27] and the coarse nodes they refer to
    wrow = np.concatenate([np.tile(_W125, (len(r_idx), 1)), np.tile(np.eye(27), (len(k_idx), 1))])
    cnod = np.concatenate([np.repeat(coarse.cell_nodes[r_idx], 125, axis=0),
                           np.repeat(coarse.cell_nodes[k_idx], 27, axis=0)])
    _, first = np.unique(fi, return_index=True)
    assert len(first) == fine.nnode
    rows = np.repeat(fi[first], 27)
    cols = cnod[first].ravel()
    vals = wrow[first].ravel()
    nz = vals != 0
    I = sp.csr_matrix((vals[nz], (rows[nz], cols[nz])), shape=(fine.nnode, coarse.nnode))
    if dirichlet:
        Cc, ffree = coarse.C, fine.free
    else:
        _, ffree, _ = fine.C_no_dirichlet()
        _, _, Cc = coarse.C_no_dirichlet()
    Pn = sp.diags(ffree.astype(np.float64)) @ I @ Cc
    P = sp.kron(Pn.tocsr(), sp.identity(3), format='csr')
    if dirichlet and fine.bc == "noflux":
        # the components fixed by u . n = 0 carry and receive nothing
        Df = sp.diags((~fine.fixed.ravel()).astype(np.float64))
        Dc = sp.diags((~coarse.fixed.ravel()).astype(np.float64))
        P = (Df @ P @ Dc).tocsr()
    return P


def cell_code_of(mesh):
    from .mesh import cell_code
    return cell_code(mesh.lev, mesh.ijk)


def cell_code_parents(mesh):
    """Codes of the parents of the cells of ``mesh`` (level >= 1)."""
    from .mesh import cell_code
    return np.unique(cell_code(mesh.lev - 1, mesh.ijk >> 1))
