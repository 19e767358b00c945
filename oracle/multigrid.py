"""Geometric multigrid V-cycle for the velocity block A.

Test infrastructure (see ``oracle/__init``).

Paper, Sec. 2.2.1: the velocity block is preconditioned by one V-cycle of a
matrix-free geometric multigrid on the fully coupled operator A (strain-rate
form), smoothed by a degree-4 Chebyshev smoother with one smoothing step per
level.  The paper fixes nothing else.  Readings:

* one pre- and one post-application of the degree-4 polynomial (V(1,1));
* Chebyshev iteration as in Saad, "Iterative Methods for Sparse Linear
  Systems", 2nd ed., Alg. 12.1, preconditioned by M^{-1} = diag(s_i / d_i)
  (s = 1 for the plain smoother), on the interval [lam / 15, lam] with
  lam = 1.2 * (largest eigenvalue of M^{-1} A estimated by 12 steps of
  preconditioned CG-Lanczos from a SplitMix64 start vector);
* pre-smoothing starts from x = 0;
* coarse level G_1 (2x2x2 cells) solved exactly by a Cholesky factorisation of
  its free block;
* restriction R_l = P_l^T with P_l from ``operators.prolongation``.
"""
import numpy as np
import scipy.linalg as sla

from . import operators as ops
from . import rng

CHEB_DEGREE = 4
SMOOTHING_RANGE = 15.0
LAMBDA_SAFETY = 1.2
LANCZOS_STEPS = 12
LAMBDA_SEED = 12345


def cg_lanczos_lambda_max(apply_A, minv, r0, steps=LANCZOS_STEPS):
    """Largest eigenvalue of M^{-1} A from the Lanczos matrix of ``steps`` PCG
    iterations on A x = r0 (x0 = 0, preconditioner M^{-1} = diag(minv)).

    With CG coefficients alpha_k, beta_k the Lanczos tridiagonal matrix is
    T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1},  T_{k,k+1} = sqrt(beta_k)/alpha_k.
    """
    r = np.array(r0, dtype=np.float64)
    z = minv * r
    p = z.copy()
    rz = r @ z
    rz0 = rz
    alphas, betas = [], []
    for _ in range(steps):
        q = apply_A(p)
        pq = p @ q
        if pq <= 0:
            break
        alpha = rz / pq
        alphas.append(alpha)
        r = r - alpha * q
        z = minv * r
        rz_new = r @ z
        beta = rz_new / rz
        if rz_new <= 1e-30 * rz0:
            break
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    return float(np.linalg.eigvalsh(T).max())


def chebyshev(apply_A, minv, b, x, lam, degree=CHEB_DEGREE, x_is_zero=False):
    """``degree`` updates of Chebyshev acceleration (Saad, Alg. 12.1) for
    A x = b with preconditioner M^{-1} = diag(minv) on [lam/15, lam]."""
    a_lo = lam / SMOOTHING_RANGE
    theta = 0.5 * (lam + a_lo)
    delta = 0.5 * (lam - a_lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.zeros_like(b) if x_is_zero else np.array(x, dtype=np.float64)
    r = b.copy() if x_is_zero else b - apply_A(x)
    d = minv * r / theta
    for k in range(degree):
        x = x + d
        if k + 1 < degree:
            r = r - apply_A(d)
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * (minv * r)
            rho = rho_new
    return x


class GMG:
    """Level operators, smoothers, transfers and coarse factor of a hierarchy.

    mus: cell viscosity per level (``operators.level_viscosities``).
    scaling: optional {level: s} per-dof smoother scaling (M^{-1} = s / d).
    assembled_max: largest n_u for which A_l is assembled as a sparse matrix
    (otherwise the cellwise operator is used; both are the same operator).
    """

    def __init__(self, hier, mus, scaling=None, assembled_max=400_000, seed=LAMBDA_SEED):
        self.hier = hier
        self.L = hier.L
        self.A, self.minv, self.lam, self.P = {}, {}, {}, {}
        self.free = {}
        scaling = scaling or {}
        for ell in range(1, self.L + 1):
            mesh = hier.levels[ell]
            if mesh.n_u <= assembled_max:
                Am = ops.assemble_A(mesh, mus[ell])
                diag = Am.diagonal()
                self.A[ell] = Am
            else:
                Am = ops.CellwiseA(mesh, mus[ell])
                diag = Am.diagonal()
                self.A[ell] = Am
            free = mesh.free_dofs_mask()
            self.free[ell] = free
            s = scaling.get(ell, 1.0)
            self.minv[ell] = np.where(free, s / diag, 1.0)
            if ell >= 2:
                self.P[ell] = ops.prolongation(hier, ell)
                r0 = rng.dof_vector(mesh, seed) * free
                lam_hat = cg_lanczos_lambda_max(lambda v: self.A[ell] @ v, self.minv[ell], r0)
                self.lam[ell] = LAMBDA_SAFETY * lam_hat
        # coarse: Cholesky of the free block of A_1
        A1 = self.A[1].toarray() if hasattr(self.A[1], 'toarray') else None
        f1 = self.free[1]
        self.coarse_free = np.nonzero(f1)[0]
        self.coarse_chol = sla.cho_factor(A1[np.ix_(self.coarse_free, self.coarse_free)])

    def apply(self, ell, x):
        return self.A[ell] @ x

    def coarse_solve(self, b):
        x = b.copy()          # identity rows on constrained dofs
        x[self.coarse_free] = sla.cho_solve(self.coarse_chol, b[self.coarse_free])
        return x

    def vcycle(self, b, ell=None):
        """x = V_l(b): pre-smooth from 0, restrict the residual, recurse,
        prolongate and add, post-smooth."""
        ell = self.L if ell is None else ell
        if ell == 1:
            return self.coarse_solve(b)
        Aop = lambda v: self.A[ell] @ v
        x = chebyshev(Aop, self.minv[ell], b, None, self.lam[ell], x_is_zero=True)
        r = b - Aop(x)
        xc = self.vcycle(self.P[ell].T @ r, ell - 1)
        x = x + self.P[ell] @ xc
        x = chebyshev(Aop, self.minv[ell], b, x, self.lam[ell])
        return x
