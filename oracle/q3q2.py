"""Taylor-Hood Q3-Q2 (k = 2) on uniform meshes of the unit cube.

Test infrastructure (see ``oracle/__init__``).

Paper, Sec. 2.1: the velocity-pressure pair is [Q_{k+1}]^3 x Q_k, k >= 1; the
runs of Sec. 3 use k = 1 (``fe``, ``mesh``, ``operators``), this module is
k = 2, with the same forms a(v, u) = int 2 mu eps(v) : eps(u),
b(v, p) = -int (div v) p, f(v) = int v . f (Sec. 2, eq. stokes; Sec. 2.1)
and the same solver: FGMRES with the block-triangular preconditioner, one
GMG V-cycle (degree-4 Chebyshev, Sec. 2.2.1) for A and CG on the
mu^{-1}-weighted pressure mass matrix for S (Sec. 2.2.2).

Readings (the paper fixes none of these):
* support points: Gauss-Lobatto points per direction, {0, (1 - 1/sqrt 5)/2,
  (1 + 1/sqrt 5)/2, 1} for Q3 (the roots of (1 - x^2) P_3'(x) mapped to
  [0, 1]); for Q2 these are {0, 1/2, 1}, the points of the k = 1 velocity;
  local node (i, j, k) has index i + 4 j + 16 k (Q3) or i + 3 j + 9 k (Q2);
  velocity dof (node, component) = 3 node + component;
* quadrature: 4 Gauss points per direction, exact for every form above with
  cell-constant mu on an axis-aligned cube (polynomial degree <= 7 per
  variable); the same points give the cell viscosity (harmonic mean weighted
  by the Gauss weights) and the body force, evaluated pointwise;
* uniform meshes only (n = 2^l cells per edge, every level uniform, no
  hanging nodes): global node index X + m (Y + m Z) on the level's lattice of
  m = 3 n + 1 points per axis; pressure on the Q2 lattice of 2 n + 1 points;
* Dirichlet u = 0 on the boundary; level l viscosity = arithmetic mean of the
  8 children (Sec. 2.3); coarsest level 2 x 2 x 2 cells solved exactly.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe, krylov
from . import multigrid as mg
from .rng import uniform_pm1

GLL3 = np.array([0.0, 0.5 * (1.0 - 1.0 / np.sqrt(5.0)), 0.5 * (1.0 + 1.0 / np.sqrt(5.0)), 1.0])
GLL2 = np.array([0.0, 0.5, 1.0])
NQ = 4


def lagrange_1d(nodes, t):
    """Values [len(nodes), len(t)] of the Lagrange polynomials on ``nodes``."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.ones((len(nodes), len(t)))
    for i, xi in enumerate(nodes):
        for j, xj in enumerate(nodes):
            if i != j:
                out[i] *= (t - xj) / (xi - xj)
    return out


def lagrange_1d_deriv(nodes, t):
    """Derivatives [len(nodes), len(t)] (product rule over the factors)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((n, len(t)))
    for i in range(n):
        for k in range(n):
            if k == i:
                continue
            term = np.full(len(t), 1.0 / (nodes[i] - nodes[k]))
            for j in range(n):
                if j != i and j != k:
                    term = term * (t - nodes[j]) / (nodes[i] - nodes[j])
            out[i] += term
    return out


def basis(nodes, points):
    """Tensor basis on ``nodes`` at points [np, 3]: (phi [n^3, np], grad [n^3, 3, np])."""
    p = np.atleast_2d(np.asarray(points, dtype=np.float64))
    v = [lagrange_1d(nodes, p[:, d]) for d in range(3)]
    g = [lagrange_1d_deriv(nodes, p[:, d]) for d in range(3)]
    phi = fe._tensor(v[0], v[1], v[2])
    grad = np.stack([fe._tensor(g[0], v[1], v[2]), fe._tensor(v[0], g[1], v[2]),
                     fe._tensor(v[0], v[1], g[2])], axis=1)
    return phi, grad


def element_matrices(nq=NQ):
    """Unit-cube element matrices, mu = 1 (the forms of Sec. 2.1 for k = 2):
    K [192, 192] (dof 3 a + c), B [27, 192], M [27, 27] (pressure mass)."""
    pts, w = fe.gauss_points_3d(nq)
    phi, g = basis(GLL3, pts)
    psi, _ = basis(GLL2, pts)
    K = np.zeros((192, 192))
    for c in range(3):
        for d in range(3):
            blk = np.einsum('aq,bq,q->ab', g[:, d, :], g[:, c, :], w)
            if c == d:
                blk = blk + np.einsum('aiq,biq,q->ab', g, g, w)
            K[c::3, d::3] = blk
    B = np.zeros((27, 192))
    for d in range(3):
        B[:, d::3] = -np.einsum('iq,bq,q->ib', psi, g[:, d, :], w)
    M = np.einsum('iq,jq,q->ij', psi, psi, w)
    return K, B, M


_KHAT, _BHAT, _MHAT = element_matrices()


def khat():
    return _KHAT.copy()


class UniformMesh:
    """n = 2^l cells per edge; Q3 velocity lattice m = 3n + 1, Q2 pressure
    lattice 2n + 1 (leaf only)."""

    def __init__(self, level, with_pressure=False):
        self.level = int(level)
        self.n = n = 1 << self.level
        self.m = m = 3 * n + 1
        self.h = 1.0 / n
        self.ncell = n ** 3
        c = np.arange(self.ncell)
        self.cijk = np.stack([c % n, (c // n) % n, c // (n * n)], axis=1)
        loc = np.array([(a, b, cc) for cc in range(4) for b in range(4) for a in range(4)])
        lat = 3 * self.cijk[:, None, :] + loc[None, :, :]
        self.cell_nodes = lat[..., 0] + m * (lat[..., 1] + m * lat[..., 2])      # [ncell, 64]
        self.nnode = m ** 3
        X = np.arange(self.nnode)
        self.lat = np.stack([X % m, (X // m) % m, X // (m * m)], axis=1)
        self.dirichlet = np.any((self.lat == 0) | (self.lat == m - 1), axis=1)
        self.free = ~self.dirichlet
        if with_pressure:
            mp = 2 * n + 1
            ploc = np.array([(a, b, cc) for cc in range(3) for b in range(3) for a in range(3)])
            plat = 2 * self.cijk[:, None, :] + ploc[None, :, :]
            self.cell_pnodes = plat[..., 0] + mp * (plat[..., 1] + mp * plat[..., 2])   # [ncell, 27]
            self.npnode = mp ** 3

    @property
    def n_u(self):
        return 3 * self.nnode

    def positions_1d(self):
        """Physical coordinate of lattice index X (0 .. m-1) along one axis."""
        X = np.arange(self.m)
        cell = np.minimum(X // 3, self.n - 1)
        return (cell + GLL3[X - 3 * cell]) / self.n

    def node_positions(self):
        x = self.positions_1d()
        return np.stack([x[self.lat[:, 0]], x[self.lat[:, 1]], x[self.lat[:, 2]]], axis=1)

    def pressure_positions(self):
        mp = 2 * self.n + 1
        P = np.arange(mp ** 3)
        return np.stack([P % mp, (P // mp) % mp, P // (mp * mp)], axis=1) / (2.0 * self.n)

    def cell_dofs(self):
        return (3 * self.cell_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(self.ncell, 192)

    def free_dofs_mask(self):
        return np.repeat(self.free, 3)

    def gauss_points(self):
        """Physical Gauss points [ncell, 64, 3] (x fastest)."""
        pts, _ = fe.gauss_points_3d(NQ)
        return (self.cijk[:, None, :] + pts[None, :, :]) * self.h

    def dof_key(self):
        """Counter of each velocity dof for seeded vectors: 3 node + component."""
        return 3 * np.arange(self.nnode)[:, None] + np.arange(3)[None, :]


def harmonic_cell_viscosity(mu_qp):
    """mu_K = sum w_q / sum (w_q / mu_q) over the 4^3 Gauss points of a cell."""
    _, w = fe.gauss_points_3d(NQ)
    mu_qp = np.asarray(mu_qp, dtype=np.float64)
    return w.sum() / (w[None, :] / mu_qp).sum(axis=1)


def parent_viscosity(fine, mu_fine):
    """Arithmetic mean of the 8 children (Sec. 2.3) on the next coarser uniform mesh."""
    n = fine.n
    nc = n // 2
    parent = (fine.cijk[:, 0] // 2) + nc * ((fine.cijk[:, 1] // 2) + nc * (fine.cijk[:, 2] // 2))
    return np.bincount(parent, weights=mu_fine, minlength=nc ** 3) / 8.0


def assemble_K(mesh, mu):
    dofs = mesh.cell_dofs()
    scale = np.asarray(mu) * mesh.h
    rows = np.repeat(dofs, 192, axis=1).ravel()
    cols = np.tile(dofs, (1, 192)).ravel()
    vals = (scale[:, None, None] * _KHAT[None]).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n_u, mesh.n_u))


def assemble_A(mesh, mu):
    """D K D + (I - D), D = diag(free dofs): identity rows on Dirichlet dofs."""
    f = mesh.free_dofs_mask().astype(np.float64)
    D = sp.diags(f)
    return (D @ assemble_K(mesh, mu) @ D + sp.diags(1.0 - f)).tocsr()


def assemble_B(mesh):
    dofs = mesh.cell_dofs()
    rows = np.repeat(mesh.cell_pnodes, 192, axis=1).ravel()
    cols = np.tile(dofs, (1, 27)).ravel()
    vals = np.broadcast_to((mesh.h ** 2) * _BHAT, (mesh.ncell, 27, 192)).ravel()
    Bf = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.npnode, mesh.n_u))
    return (Bf @ sp.diags(mesh.free_dofs_mask().astype(np.float64))).tocsr()


def assemble_Mp(mesh, mu):
    pn = mesh.cell_pnodes
    rows = np.repeat(pn, 27, axis=1).ravel()
    cols = np.tile(pn, (1, 27)).ravel()
    vals = ((mesh.h ** 3 / np.asarray(mu))[:, None, None] * _MHAT[None]).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.npnode, mesh.npnode))


def pressure_mean_weights(mesh):
    w1 = _MHAT.sum(axis=1)
    return np.bincount(mesh.cell_pnodes.ravel(), weights=np.broadcast_to(mesh.h ** 3 * w1, (mesh.ncell, 27)).ravel(),
                       minlength=mesh.npnode)


def assemble_rhs(mesh, f_qp):
    """b = D F, F_e[(a, c)] = h^3 sum_q w_q phi_a(xi_q) f_c(x_q); f_qp [ncell, 64, 3]."""
    pts, w = fe.gauss_points_3d(NQ)
    phi, _ = basis(GLL3, pts)
    Fe = np.einsum('aq,nqc->nac', phi * w[None, :], np.asarray(f_qp)) * mesh.h ** 3
    F = np.bincount(mesh.cell_dofs().ravel(), weights=Fe.reshape(-1), minlength=mesh.n_u)
    return F * mesh.free_dofs_mask()


def prolongation_1d(coarse, fine):
    """[m_f, m_c]: the coarse Q3 functions of one axis at the fine lattice points."""
    xf = fine.positions_1d()
    kc = np.minimum(np.floor(xf * coarse.n).astype(np.int64), coarse.n - 1)
    t = xf * coarse.n - kc
    L = lagrange_1d(GLL3, t)                              # [4, m_f]
    rows = np.repeat(np.arange(fine.m), 4)
    cols = (3 * kc[:, None] + np.arange(4)[None, :]).ravel()
    P = sp.csr_matrix((L.T.ravel(), (rows, cols)), shape=(fine.m, coarse.m)).toarray()
    P[np.abs(P) < 1e-15] = 0.0
    return P


def prolongation(coarse, fine):
    """P = D_f (P_z x P_y x P_x) D_c per component (dofs 3 node + c)."""
    P1 = sp.csr_matrix(prolongation_1d(coarse, fine))
    Pn = sp.kron(P1, sp.kron(P1, P1, format='csr'), format='csr')
    Pn = sp.diags(fine.free.astype(np.float64)) @ Pn @ sp.diags(coarse.free.astype(np.float64))
    return sp.kron(Pn.tocsr(), sp.identity(3), format='csr')


class GMG:
    """Uniform Q3 levels 1 .. L with the V-cycle of ``multigrid`` (degree-4
    Chebyshev on [lam/15, lam], lam = 1.2 x 12-step CG-Lanczos from a
    SplitMix64 start vector over counters 3 node + component, Cholesky on
    level 1)."""

    def __init__(self, L, mu_leaf, seed=mg.LAMBDA_SEED):
        self.L = L
        self.mesh = {ell: UniformMesh(ell, with_pressure=(ell == L)) for ell in range(1, L + 1)}
        self.mu = {L: np.asarray(mu_leaf, dtype=np.float64)}
        for ell in range(L - 1, 0, -1):
            self.mu[ell] = parent_viscosity(self.mesh[ell + 1], self.mu[ell + 1])
        self.A, self.minv, self.lam, self.P, self.free = {}, {}, {}, {}, {}
        for ell in range(1, L + 1):
            m = self.mesh[ell]
            A = assemble_A(m, self.mu[ell])
            self.A[ell] = A
            self.free[ell] = m.free_dofs_mask()
            self.minv[ell] = np.where(self.free[ell], 1.0 / A.diagonal(), 1.0)
            if ell >= 2:
                self.P[ell] = prolongation(self.mesh[ell - 1], m)
                r0 = uniform_pm1(seed, m.dof_key().ravel()) * self.free[ell]
                self.lam[ell] = mg.LAMBDA_SAFETY * mg.cg_lanczos_lambda_max(lambda v: self.A[ell] @ v,
                                                                           self.minv[ell], r0)
        self.coarse_free = np.nonzero(self.free[1])[0]
        A1 = self.A[1].toarray()
        self.coarse_chol = sla.cho_factor(A1[np.ix_(self.coarse_free, self.coarse_free)])

    def coarse_solve(self, b):
        x = b.copy()
        x[self.coarse_free] = sla.cho_solve(self.coarse_chol, b[self.coarse_free])
        return x

    def vcycle(self, b, ell=None):
        ell = self.L if ell is None else ell
        if ell == 1:
            return self.coarse_solve(b)
        Aop = lambda v: self.A[ell] @ v
        x = mg.chebyshev(Aop, self.minv[ell], b, None, self.lam[ell], x_is_zero=True)
        r = b - Aop(x)
        x = x + self.P[ell] @ self.vcycle(self.P[ell].T @ r, ell - 1)
        return mg.chebyshev(Aop, self.minv[ell], b, x, self.lam[ell])


class StokesProblem(krylov.StokesProblem):
    """The Q3-Q2 block system [[A, B^T], [B, 0]] on the uniform 2^L mesh with
    the preconditioner and outer solvers of ``krylov.StokesProblem``."""

    def __init__(self, L, mu_leaf, f_qp, with_gmg=True, rhs_p=None):
        self.gmg = GMG(L, mu_leaf) if with_gmg else None
        mesh = self.gmg.mesh[L] if with_gmg else UniformMesh(L, with_pressure=True)
        self.mesh = mesh
        mu = np.asarray(mu_leaf, dtype=np.float64)
        self.A = assemble_A(mesh, mu)
        self.B = assemble_B(mesh)
        self.Mp = assemble_Mp(mesh, mu)
        self.nu, self.np_ = mesh.n_u, mesh.npnode
        self.pfree = np.ones(self.np_, dtype=bool)
        self.b = np.concatenate([assemble_rhs(mesh, f_qp),
                                 np.zeros(self.np_) if rhs_p is None else np.asarray(rhs_p, dtype=np.float64)])
        self.Pi_cp = sp.csr_matrix((self.np_, self.np_))
        self.K = sp.bmat([[self.A, self.B.T], [self.B, self.Pi_cp]], format='csr')
        self.mp_minv = 1.0 / self.Mp.diagonal()
        self.mp_interval = krylov.mass_interval(lambda v: self.Mp @ v, self.mp_minv, self.np_)
        self.inner_cg_its = []

    def solve_direct(self):
        m = pressure_mean_weights(self.mesh)
        n = self.nu + self.np_
        col = sp.csr_matrix(np.concatenate([np.zeros(self.nu), m])[:, None])
        Kb = sp.bmat([[self.K, col], [col.T, None]], format='csc')
        sol = spla.splu(Kb).solve(np.concatenate([self.b, [0.0]]))
        return self.finish(sol[:n])

    def finish(self, x):
        x = x.copy()
        m = pressure_mean_weights(self.mesh)
        p = x[self.nu:]
        x[self.nu:] = p - (m @ p) / m.sum()
        return x

    def distribute(self, x):
        return x[:self.nu].copy(), x[self.nu:].copy()
