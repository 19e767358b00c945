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

The paper's variants for large problems (Sec. 3.4): a Schur approximation that
is a fixed linear operator, so that plain GMRES (storing only the Arnoldi
basis) or IDR(s) (van Gijzen and Sonneveld, short recurrences) can replace
FGMRES; and the block-diagonal preconditioner P_D = diag(A, -S) of
eq. stokes_precond_diag for comparison.  Reading for the linear S_hat^{-1}:
a Chebyshev iteration of fixed degree on the Jacobi-scaled mass matrix (the
matrix-free choice the paper names for S_hat^{-1}, Sec. 2.2.2), over
[b/27, b] with b the row-sum bound max_i (M_p 1)_i / (M_p)_ii (27/8 on
uniform meshes for any viscosity: every Q1 element contributes the ratio
27/8), in place of the paper's one V-cycle on M_p.
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


def chebyshev_fixed(apply_A, minv, b, lo, hi, degree):
    """Chebyshev iteration (Saad, Alg. 12.1) for A x = b from x0 = 0 with the
    preconditioner diag(minv) over [lo, hi]: `degree` updates of x, a fixed
    polynomial in diag(minv) A, hence a linear map of b."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b.copy()
    d = minv * r / theta
    x = d.copy()
    for _ in range(1, degree):
        r = r - apply_A(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (minv * r)
        x = x + d
        rho = rho_new
    return x


def mass_interval(apply_M, minv, n):
    """[b/27, b] with b = max_i (M 1)_i minv_i (a bound on the spectrum of
    diag(minv) M for a matrix with non-negative entries)."""
    hi = float(np.max(minv * apply_M(np.ones(n))))
    return hi / 27.0, hi


def gmres(apply_K, apply_P, b, rtol=1e-8, restart=50, maxit=1000):
    """Right-preconditioned GMRES for a linear preconditioner: Arnoldi on
    K P with only the basis V stored; x += P (V y) at the end of a cycle.
    Modified Gram-Schmidt, Givens rotations.  Returns (x, stats)."""
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
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            w = apply_K(apply_P(V[j]))
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
        x = x + apply_P(V[:j_done].T @ y)
        r = b - apply_K(x)
        beta = np.linalg.norm(r)
    return x, {"iterations": its, "rel_residual": beta / bn, "history": hist}


def shadow_space(keys_u, keys_p, s, seed=4711):
    """IDR shadow space [n][s] for the block vector [u; p]: column i draws
    SplitMix64 values with seed + i over the counters 3 key + component
    (velocity) and 2^40 + key (pressure), then Gram-Schmidt (each column
    against the finished ones in turn) makes the columns orthonormal."""
    from .rng import uniform_pm1
    cu = (3 * np.asarray(keys_u, dtype=np.int64)[:, None] + np.arange(3)[None, :]).ravel()
    cp = (1 << 40) + np.asarray(keys_p, dtype=np.int64)
    c = np.concatenate([cu, cp])
    Q = np.stack([uniform_pm1(seed + i, c) for i in range(s)], axis=1)
    for k in range(s):
        for i in range(k):
            Q[:, k] -= (Q[:, i] @ Q[:, k]) * Q[:, i]
        Q[:, k] /= np.linalg.norm(Q[:, k])
    return Q


def idrs(apply_K, apply_P, b, Q, rtol=1e-8, maxit=1000, kappa=0.7):
    """Right-preconditioned IDR(s) with biorthogonal basis vectors (van Gijzen
    and Sonneveld, ACM TOMS 38:5, 2011), s = Q.shape[1], x0 = 0.  Each cycle
    takes s steps that keep the residual orthogonal to the first columns of
    Q, then one dimension-reduction step with the minimal-residual omega,
    enlarged to |omega| with cos(t, r) = kappa when the angle is larger
    (Sleijpen and van der Vorst).  Stops on the recursive residual; stats
    count K P applications (one preconditioner application each) and report
    the recomputed residual.  Returns (x, stats)."""
    n, s = Q.shape
    x = np.zeros(n)
    r = b.copy()
    bn = np.linalg.norm(b)
    G = np.zeros((n, s))
    U = np.zeros((n, s))
    M = np.eye(s)
    om = 1.0
    its = 0
    rn = np.linalg.norm(r)
    hist = [rn / bn]
    done = rn <= rtol * bn
    while not done and its < maxit:
        f = Q.T @ r
        for k in range(s):
            c = np.linalg.solve(np.tril(M[k:, k:]), f[k:])
            v = r - G[:, k:] @ c
            v = apply_P(v)
            U[:, k] = U[:, k:] @ c + om * v
            G[:, k] = apply_K(U[:, k])
            its += 1
            for i in range(k):
                alpha = (Q[:, i] @ G[:, k]) / M[i, i]
                G[:, k] -= alpha * G[:, i]
                U[:, k] -= alpha * U[:, i]
            M[k:, k] = Q[:, k:].T @ G[:, k]
            beta = f[k] / M[k, k]
            r = r - beta * G[:, k]
            x = x + beta * U[:, k]
            rn = np.linalg.norm(r)
            hist.append(rn / bn)
            if rn <= rtol * bn or its >= maxit:
                done = True
                break
            if k + 1 < s:
                f[k + 1:] -= beta * M[k + 1:, k]
        if done:
            break
        v = apply_P(r)
        t = apply_K(v)
        its += 1
        tt, tr = t @ t, t @ r
        om = tr / tt
        rho = abs(tr) / (np.sqrt(tt) * rn)
        if rho < kappa:
            om *= kappa / rho
        r = r - om * t
        x = x + om * v
        rn = np.linalg.norm(r)
        hist.append(rn / bn)
        done = rn <= rtol * bn
    res = np.linalg.norm(b - apply_K(x)) / bn
    return x, {"iterations": its, "rel_residual": res, "history": hist}


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

    def __init__(self, hier, mu_leaf, f_qp, gmg=None, gmg_kwargs=None, rhs_p=None):
        """rhs_p: right-hand side of the pressure block (B u = rhs_p, i.e.
        div u = g with rhs_p_i = -int psi_i g); zero by default (Sec. 2.1)."""
        self.hier = hier
        mesh = hier.leaf
        self.mesh = mesh
        self.mus = ops.level_viscosities(hier, mu_leaf)
        self.A = ops.assemble_A(mesh, self.mus[hier.L])
        self.B = ops.assemble_B(mesh)
        self.Mp = ops.assemble_Mp(mesh, self.mus[hier.L])
        self.nu, self.np_ = mesh.n_u, mesh.npnode
        self.pfree = mesh.pfree
        self.b = np.concatenate([ops.assemble_rhs(mesh, f_qp),
                                 np.zeros(self.np_) if rhs_p is None else np.asarray(rhs_p, dtype=np.float64)])
        self.Pi_cp = sp.diags((~self.pfree).astype(np.float64))
        self.K = sp.bmat([[self.A, self.B.T], [self.B, self.Pi_cp]], format='csr')
        self.mp_minv = 1.0 / self.Mp.diagonal()
        self.mp_interval = mass_interval(lambda v: self.Mp @ v, self.mp_minv, self.np_)
        self.gmg = gmg
        if gmg is None and gmg_kwargs is not None:
            from .multigrid import GMG
            self.gmg = GMG(hier, self.mus, **gmg_kwargs)
        self.inner_cg_its = []

    def apply_K(self, x):
        return self.K @ x

    def precondition(self, r, a_inv=None, s_inv=None, block="triangular", schur="cg", schur_degree=8,
                     schur_rtol=1e-2, schur_maxit=200):
        """z = P^{-1} r: z_p = -S_hat^{-1} r_p, z_u = A_hat^{-1}(r_u - B^T z_p)
        (block "triangular", eq. stokes_precond) or A_hat^{-1} r_u (block
        "diagonal", eq. stokes_precond_diag).  S_hat^{-1}: Jacobi CG ("cg", to
        schur_rtol or at most schur_maxit iterations) or the fixed Chebyshev
        iteration ("cheb") on M_p.  The default tolerance 1e-2 is the reading
        of Sec. 2.2.2, which states the count (1-5 CG iterations) rather than a
        tolerance."""
        ru, rp = r[:self.nu], r[self.nu:]
        if s_inv is not None:
            zp_pos = s_inv(rp)
        elif schur == "cg":
            zp_pos, it = cg(lambda v: self.Mp @ v, rp, self.mp_minv, rtol=schur_rtol, maxit=schur_maxit)
            self.inner_cg_its.append(it)
        else:
            lo, hi = self.mp_interval
            zp_pos = chebyshev_fixed(lambda v: self.Mp @ v, self.mp_minv, rp, lo, hi, schur_degree)
        zp = -zp_pos
        rhs_u = ru - self.B.T @ zp if block == "triangular" else ru
        zu = self.gmg.vcycle(rhs_u) if a_inv is None else a_inv(rhs_u)
        return np.concatenate([zu, zp])

    def solve_fgmres(self, rtol=1e-8, restart=50, maxit=1000, **kw):
        x, st = fgmres(self.apply_K, lambda r: self.precondition(r, **kw), self.b,
                       rtol=rtol, restart=restart, maxit=maxit)
        return self.finish(x), st

    def solve(self, krylov="fgmres", rtol=1e-8, restart=50, maxit=1000, idr_s=2, **kw):
        """Outer solve with FGMRES, GMRES (linear preconditioner: schur="cheb")
        or IDR(idr_s); keyword arguments go to precondition()."""
        P = lambda r: self.precondition(r, **kw)
        if krylov == "fgmres":
            x, st = fgmres(self.apply_K, P, self.b, rtol=rtol, restart=restart, maxit=maxit)
        elif krylov == "gmres":
            x, st = gmres(self.apply_K, P, self.b, rtol=rtol, restart=restart, maxit=maxit)
        else:
            Q = shadow_space(self.mesh.keys, self.mesh.pkeys, idr_s)
            x, st = idrs(self.apply_K, P, self.b, Q, rtol=rtol, maxit=maxit)
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
