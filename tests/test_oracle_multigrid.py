"""Pins of the oracle's smoother, eigenvalue estimate, coarse solve and V-cycle.

Fixed by: the closed-form Chebyshev error polynomial on a diagonal matrix,
scale invariance of the preconditioned smoother, dense eigenvalues, exactness
of the coarse factorisation, symmetry of V(1,1) with identical pre/post
polynomials, and an h-independent contraction factor."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import mesh, multigrid as mg, operators as ops, rng
from tests.test_oracle_mesh import adaptive_hierarchy


def cheb_T(k, x):
    return np.cos(k * np.arccos(x)) if abs(x) <= 1 else np.cosh(k * np.arccosh(abs(x))) * np.sign(x) ** k


def test_chebyshev_error_polynomial_closed_form():
    lam_vals = np.linspace(0.05, 2.0, 40)
    A = sp.diags(lam_vals)
    lam = 2.0
    e0 = np.random.default_rng(0).standard_normal(40)
    b = A @ e0
    x = mg.chebyshev(lambda v: A @ v, np.ones(40), b, None, lam, x_is_zero=True)
    a_lo = lam / mg.SMOOTHING_RANGE
    theta, delta = (lam + a_lo) / 2, (lam - a_lo) / 2
    poly = np.array([cheb_T(4, (theta - l) / delta) / cheb_T(4, theta / delta) for l in lam_vals])
    assert np.allclose(e0 - x, poly * e0, atol=1e-13)
    # inside the interval the damping is bounded by 1/T_4(theta/delta)
    inside = lam_vals >= a_lo
    assert np.all(np.abs(poly[inside]) <= 1 / cheb_T(4, theta / delta) + 1e-14)
    # nonzero start vector: same error propagation
    x0 = np.random.default_rng(1).standard_normal(40)
    x1 = mg.chebyshev(lambda v: A @ v, np.ones(40), b, x0, lam)
    assert np.allclose(e0 - x1, poly * (e0 - x0), atol=1e-12)


def test_lanczos_estimate_and_scale_invariance():
    H = adaptive_hierarchy(2, (1, 1, 1), 1)
    m = H.leaf
    rg = np.random.default_rng(5)
    mu = 10 ** rg.uniform(0, 3, m.ncell)
    A = ops.assemble_A(m, mu)
    d = A.diagonal()
    minv = 1.0 / d
    r0 = rng.dof_vector(m, 7) * m.free_dofs_mask()
    lam = mg.cg_lanczos_lambda_max(lambda v: A @ v, minv, r0)
    Dh = np.diag(np.sqrt(minv))
    ev = np.linalg.eigvalsh(Dh @ A.toarray() @ Dh)
    assert lam <= ev.max() * (1 + 1e-12)
    assert lam >= 0.9 * ev.max()
    # scaling M^{-1} by c scales the estimate by c and leaves the smoother unchanged
    lam3 = mg.cg_lanczos_lambda_max(lambda v: A @ v, 3 * minv, r0)
    assert np.isclose(lam3, 3 * lam, rtol=1e-12)
    b = rg.standard_normal(m.n_u)
    x1 = mg.chebyshev(lambda v: A @ v, minv, b, None, 1.2 * lam, x_is_zero=True)
    x3 = mg.chebyshev(lambda v: A @ v, 3 * minv, b, None, 1.2 * lam3, x_is_zero=True)
    assert np.allclose(x1, x3, rtol=1e-11, atol=1e-14)


def _gmg(H, seed=0, spread=3):
    rg = np.random.default_rng(seed)
    mu = 10 ** rg.uniform(0, spread, H.leaf.ncell)
    return mg.GMG(H, ops.level_viscosities(H, mu)), mu


def test_coarse_solve_exact():
    G, _ = _gmg(mesh.Hierarchy.uniform(2))
    b = np.random.default_rng(1).standard_normal(375) * G.free[1]
    x = G.coarse_solve(b)
    assert np.linalg.norm(G.A[1] @ x - b) <= 1e-14 * np.linalg.norm(b) * 10
    assert G.free[1].sum() == 81


def test_vcycle_symmetric_and_contracting():
    for H in (mesh.Hierarchy.uniform(3), adaptive_hierarchy(2, (1, 1, 1), 2)):
        G, _ = _gmg(H)
        n = H.leaf.n_u
        f = G.free[H.L]
        rg = np.random.default_rng(2)
        x = rg.standard_normal(n) * f
        y = rg.standard_normal(n) * f
        a, b = x @ G.vcycle(y), y @ G.vcycle(x)
        assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
        # A-norm contraction of E = I - V A by power iteration
        A = G.A[H.L]
        e = rg.standard_normal(n) * f
        for _ in range(6):
            e_new = e - G.vcycle(A @ e)
            rho = np.sqrt((e_new @ (A @ e_new)) / (e @ (A @ e)))
            e = e_new / np.linalg.norm(e_new)
        # random cellwise jumps of up to 10^3: still a contraction
        assert rho < 0.8, rho


def test_vcycle_factor_h_independent():
    rhos = []
    for L in (2, 3, 4):
        H = mesh.Hierarchy.uniform(L)
        G = mg.GMG(H, ops.level_viscosities(H, np.ones(H.leaf.ncell)))
        A = G.A[L]
        e = rng.dof_vector(H.leaf, 3) * G.free[L]
        for _ in range(8):
            e_new = e - G.vcycle(A @ e)
            rho = np.sqrt((e_new @ (A @ e_new)) / (e @ (A @ e)))
            e = e_new / np.linalg.norm(e_new)
        rhos.append(rho)
    assert max(rhos) < 0.3
    assert rhos[-1] < rhos[-2] * 1.25


def test_chebyshev_residual_form_matches_recurrence():
    """The device smoother forms the residual as b - A x at every step instead
    of by the recurrence r -= A d of Saad's Alg. 12.1; in exact arithmetic the
    iterates are the same.  Written out here in that form, it agrees with the
    oracle's recurrence to rounding, from x = 0 and from a given x."""
    rg = np.random.default_rng(12)
    n = 60
    Q = rg.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    minv = 1.0 / np.diag(A)
    b = rg.standard_normal(n)
    lam = 1.2 * np.linalg.eigvals(minv[:, None] * A).real.max()

    def residual_form(x0, zero):
        lo = lam / 15.0
        theta, delta = 0.5 * (lam + lo), 0.5 * (lam - lo)
        sigma = theta / delta
        rho = 1.0 / sigma
        x = np.zeros(n) if zero else x0.copy()
        d = minv * (b - A @ x) / theta
        x = x + d
        for _ in range(3):
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * (minv * (b - A @ x))
            x = x + d
            rho = rho_new
        return x

    x0 = rg.standard_normal(n)
    for zero in (True, False):
        ref = mg.chebyshev(lambda v: A @ v, minv, b, x0, lam, degree=4, x_is_zero=zero)
        got = residual_form(x0, zero)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref), zero
