"""Outer Stokes solver: FGMRES with the block-triangular preconditioner.

Test infrastructure (see ``oracle/__init``).

Paper, Sec. 2.2: the block system is solved by a Krylov method right
preconditioned with P = [[A, B^T], [0, -S]] (eq. stokes_precond); with exact
blocks the preconditioned matrix is [[I, 0], [B A^{-1}, I]] and GMRES stops
within two iterations.  A^{-1} is replaced by one GMG V-cycle (Sec. 2.2.1) and
S^{-1} by a CG solve with the mu^{-1}-weighted pressure mass matrix
(Sec. 2.2.2); because that inner CG varies between applications the outer
method is flexible GMRES (restart 50, Sec. 3.4).

Readings: x0 = 0; z_p = -S_hat^{-1} r_p, z_u = A_hat^{-1}(r_u - B^T z_p);
inner CG Jacobi-preconditioned to relative tolerance 1e-6 (at most 200
steps); stop once ||b - K x||_2 <= 1e-8 ||b||_2 with the residual recomputed
from scratch; the pressure is reported with zero mean.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operators as ops


def cg(apply_A, b, minv, rtol=1e-6, maxit=200, x0=None):
    """Jacobi-preconditioned conjugate gradients; returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0
    z = minv * r
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = apply_A(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * bn:
            return x, it
        z = minv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


def fgmres(apply_K, apply_P, b, rtol=1e-8, restart=50, maxit=1000):
    """Flexible GMRES (right preconditioning, modified Gram-Schmidt, Givens
    rotations).  Returns (x, stats)."""
    n = len(b)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    its = 0
    r = b.copy()
    beta = np.linalg.norm(r)
    hist = [beta / bn]
    while its < maxit:
        if beta <= rtol * bn:
            break
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            Z[j] = apply_P(V[j])
            w = apply_K(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) <= rtol * bn or its >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
        r = b - apply_K(x)
        beta = np.linalg.norm(r)
    return x, {"iterations": its, "rel_residual": beta / bn, "history": hist}


class StokesProblem:
    """Block system K_S = [[A, B^T], [B, Pi_cp]] on the leaf mesh of a
    hierarchy with its GMG preconditioner (assembled; small meshes)."""

    def __init__(self, hier, mu_leaf, f_qp, gmg=None, gmg_kwargs=None):
        self.hier = hier
        mesh = hier.leaf
        self.mesh = mesh
        self.mus = ops.level_viscosities(hier, mu_leaf)
        self.A = ops.assemble_A(mesh, self.mus[hier.L])
        self.B = ops.assemble_B(mesh)
        self.Mp = ops.assemble_Mp(mesh, self.mus[hier.L])
        self.nu, self.np_ = mesh.n_u, mesh.npnode
        self.pfree = mesh.pfree
        self.b = np.concatenate([ops.assemble_rhs(mesh, f_qp), np.zeros(self.np_)])
        self.Pi_cp = sp.diags((~self.pfree).astype(np.float64))
        self.K = sp.bmat([[self.A, self.B.T], [self.B, self.Pi_cp]], format='csr')
        self.mp_minv = 1.0 / self.Mp.diagonal()
        self.gmg = gmg
        if gmg is None and gmg_kwargs is not None:
            from .multigrid import GMG
            self.gmg = GMG(hier, self.mus, **gmg_kwargs)
        self.inner_cg_its = []

    def apply_K(self, x):
        return self.K @ x

    def precondition(self, r, a_inv=None, s_inv=None):
        ru, rp = r[:self.nu], r[self.nu:]
        if s_inv is None:
            zp_pos, it = cg(lambda v: self.Mp @ v, rp, self.mp_minv, rtol=1e-6, maxit=200)
            self.inner_cg_its.append(it)
        else:
            zp_pos = s_inv(rp)
        zp = -zp_pos
        rhs_u = ru - self.B.T @ zp
        zu = self.gmg.vcycle(rhs_u) if a_inv is None else a_inv(rhs_u)
        return np.concatenate([zu, zp])

    def solve_fgmres(self, rtol=1e-8, restart=50, maxit=1000, **kw):
        x, st = fgmres(self.apply_K, lambda r: self.precondition(r, **kw), self.b,
                       rtol=rtol, restart=restart, maxit=maxit)
        return self.finish(x), st

    def solve_direct(self):
        """Sparse LU of K_S bordered by the zero-mean pressure row m^T p = 0."""
        m = ops.pressure_mean_weights(self.mesh)
        n = self.nu + self.np_
        col = sp.csr_matrix(np.concatenate([np.zeros(self.nu), m])[:, None])
        Kb = sp.bmat([[self.K, col], [col.T, None]], format='csc')
        sol = spla.splu(Kb).solve(np.concatenate([self.b, [0.0]]))
        return self.finish(sol[:n])

    def finish(self, x):
        """Zero-mean pressure (over the free pressure nodes' weights)."""
        x = x.copy()
        m = ops.pressure_mean_weights(self.mesh)
        p = x[self.nu:]
        x[self.nu:] = np.where(self.pfree, p - (m @ p) / m.sum(), 0.0)
        return x

    def residual(self, x):
        return np.linalg.norm(self.b - self.K @ x) / np.linalg.norm(self.b)

    def distribute(self, x):
        """Values at every node (hanging nodes interpolated from masters)."""
        u = self.mesh.Cu() @ x[:self.nu]
        p = self.mesh.Cp @ x[self.nu:]
        return u, p
