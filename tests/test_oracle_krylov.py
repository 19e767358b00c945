"""Pins of the oracle's outer-solver variants (Sec. 3.4 of the paper): the
fixed Chebyshev Schur approximation, plain GMRES, IDR(s) and the
block-diagonal preconditioner P_D (eq. stokes_precond_diag).  Each is checked
against mathematics that does not come from the oracle: closed forms,
textbook algorithms written out here, finite-termination bounds and exact
direct solves."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import krylov, mesh
from tests.test_oracle_mesh import adaptive_hierarchy


def test_chebyshev_fixed_matches_closed_form():
    """For A = diag(lam) and no scaling, degree-k Chebyshev from 0 leaves the
    error p_k(A) A^{-1} b with p_k(l) = T_k((theta - l)/delta) / T_k(theta/delta)."""
    rg = np.random.default_rng(1)
    lo, hi = 0.3, 4.0
    lam = np.concatenate([rg.uniform(lo, hi, 40), [lo, hi]])
    b = rg.standard_normal(lam.size)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    for k in (1, 2, 5, 9):
        x = krylov.chebyshev_fixed(lambda v: lam * v, np.ones_like(lam), b, lo, hi, k)
        Tk = np.zeros(k + 1)
        Tk[k] = 1.0
        p = npcheb.chebval((theta - lam) / delta, Tk) / npcheb.chebval(theta / delta, Tk)
        ref = (1.0 - p) * b / lam
        assert np.allclose(x, ref, rtol=1e-12, atol=1e-13), k


def test_chebyshev_fixed_is_linear():
    rg = np.random.default_rng(2)
    A = rg.standard_normal((20, 20))
    A = A @ A.T + 20 * np.eye(20)
    minv = 1.0 / np.diag(A)
    f = lambda b: krylov.chebyshev_fixed(lambda v: A @ v, minv, b, 0.2, 3.0, 6)
    u, v = rg.standard_normal(20), rg.standard_normal(20)
    assert np.allclose(f(2.0 * u - 3.0 * v), 2.0 * f(u) - 3.0 * f(v), rtol=1e-12, atol=1e-12)


def test_mass_interval_uniform_is_27_over_8():
    """Every Q1 element has (row sum) / (diagonal) = (h^3/8) / (h^3/27) at each
    of its nodes, so on a uniform mesh b = 27/8 for any cell viscosity."""
    H = mesh.Hierarchy.uniform(2)
    m = H.leaf
    mu = 10 ** np.random.default_rng(3).uniform(-2, 3, m.ncell)
    f = np.zeros((m.ncell, 27, 3))
    prob = krylov.StokesProblem(H, mu, f)
    lo, hi = prob.mp_interval
    assert abs(hi - 27.0 / 8.0) < 1e-12 and abs(lo - hi / 27.0) < 1e-15
    # and it bounds the spectrum of diag(M)^{-1} M from above
    Md = prob.Mp.toarray()
    ev = np.linalg.eigvals(Md / np.diag(Md)[:, None]).real
    assert ev.max() <= hi * (1 + 1e-12) and ev.min() >= lo * (1 - 1e-12)


def _problem(H, seed=0, gmg=True):
    m = H.leaf
    rg = np.random.default_rng(seed)
    mu = 10 ** rg.uniform(0, 2, m.ncell)
    f = rg.standard_normal((m.ncell, 27, 3))
    return krylov.StokesProblem(H, mu, f, gmg_kwargs={} if gmg else None)


def test_gmres_equals_fgmres_for_a_linear_preconditioner():
    """With a fixed linear P the flexible and the plain method build the same
    Krylov space: same residual history and the same solution."""
    H = mesh.Hierarchy.uniform(2)
    prob = _problem(H)
    P = lambda r: prob.precondition(r, schur="cheb", schur_degree=6)
    x1, s1 = krylov.fgmres(prob.apply_K, P, prob.b, rtol=1e-10, restart=8)
    x2, s2 = krylov.gmres(prob.apply_K, P, prob.b, rtol=1e-10, restart=8)
    assert s1["iterations"] == s2["iterations"]
    h1, h2 = np.array(s1["history"]), np.array(s2["history"])
    assert np.allclose(h1, h2, rtol=1e-6, atol=1e-13)
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x1)
    assert prob.residual(x2) <= 1e-10


def _bicgstab(A, b, rt, maxit):
    """Textbook BiCGStab (van der Vorst, 1992) from x0 = 0 with shadow r~ = rt;
    residual norms after each full iteration."""
    x = np.zeros_like(b)
    r = b.copy()
    rho = alpha = om = 1.0
    v = p = np.zeros_like(b)
    out = []
    for _ in range(maxit):
        rho_new = rt @ r
        beta = (rho_new / rho) * (alpha / om)
        p = r + beta * (p - om * v)
        v = A @ p
        alpha = rho_new / (rt @ v)
        s = r - alpha * v
        t = A @ s
        om = (t @ s) / (t @ t)
        x = x + alpha * p + om * s
        r = s - om * t
        rho = rho_new
        out.append(np.linalg.norm(r))
    return np.array(out)


def test_idr1_matches_bicgstab():
    """IDR(1) with the minimal-residual omega (kappa = 0) and shadow vector q
    has, after every dimension-reduction step, the residual of BiCGStab with
    shadow r~ = q (van Gijzen and Sonneveld)."""
    rg = np.random.default_rng(4)
    n = 30
    A = np.eye(n) * 4 + rg.standard_normal((n, n)) * 0.4
    b = rg.standard_normal(n)
    q = rg.standard_normal(n)
    Q = (q / np.linalg.norm(q))[:, None]
    _, st = krylov.idrs(lambda v: A @ v, lambda v: v, b, Q, rtol=1e-14, maxit=24, kappa=0.0)
    h = np.array(st["history"]) * np.linalg.norm(b)
    idr_after_reduction = h[2::2]
    ref = _bicgstab(A, b, q, len(idr_after_reduction))
    assert np.allclose(idr_after_reduction, ref, rtol=1e-7, atol=1e-13)


def test_idrs_finite_termination():
    """IDR(s) reaches the solution within n + n/s matrix-vector products
    (exact arithmetic); here n = 12, s = 3: at most 16."""
    rg = np.random.default_rng(5)
    n, s = 12, 3
    A = np.eye(n) + rg.standard_normal((n, n)) * 0.3
    b = rg.standard_normal(n)
    Q = np.linalg.qr(rg.standard_normal((n, s)))[0]
    x, st = krylov.idrs(lambda v: A @ v, lambda v: v, b, Q, rtol=1e-11, maxit=16, kappa=0.0)
    assert st["iterations"] <= 16
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_shadow_space_orthonormal_and_keyed():
    H = mesh.Hierarchy.uniform(2)
    m = H.leaf
    Q = krylov.shadow_space(m.keys, m.pkeys, 3)
    assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-13)
    # column 0 before normalisation is the SplitMix64 draw of its counters
    from oracle.rng import uniform_pm1
    c0 = uniform_pm1(4711, [3 * int(m.keys[5]) + 2])[0]
    q0 = uniform_pm1(4711, np.concatenate([(3 * m.keys[:, None] + np.arange(3)).ravel(),
                                           (1 << 40) + m.pkeys]))
    assert q0[3 * 5 + 2] == c0
    assert np.allclose(Q[:, 0], q0 / np.linalg.norm(q0), rtol=0, atol=1e-15)


@pytest.mark.parametrize("krylov_name", ["gmres", "idrs"])
def test_linear_variants_solve_the_stokes_system(krylov_name):
    for H in (mesh.Hierarchy.uniform(2), adaptive_hierarchy(1, (0, 0, 0), 1)):
        prob = _problem(H, seed=6)
        x, st = prob.solve(krylov=krylov_name, rtol=1e-9, restart=30, maxit=400, schur="cheb",
                           schur_degree=8)
        xd = prob.solve_direct()
        assert prob.residual(x) <= 2e-9, (krylov_name, prob.residual(x))
        assert np.linalg.norm(x - xd) <= 1e-5 * np.linalg.norm(xd)


def test_block_diagonal_exact_three_iterations():
    """With exact blocks, K P_D^{-1} has at most three distinct eigenvalues
    (Murphy, Golub and Wathen), so (F)GMRES stops within three iterations,
    where the block-triangular P needs two."""
    for H in (mesh.Hierarchy.uniform(2), adaptive_hierarchy(1, (0, 0, 0), 1)):
        prob = _problem(H, seed=7, gmg=False)
        m = H.leaf
        Ainv = np.linalg.inv(prob.A.toarray())
        Bd = prob.B.toarray()
        S = Bd @ Ainv @ Bd.T + np.diag((~m.pfree).astype(float))
        Sinv = np.linalg.pinv(S, rcond=1e-12)
        P = lambda r: prob.precondition(r, a_inv=lambda v: Ainv @ v, s_inv=lambda v: Sinv @ v, block="diagonal")
        x, st = krylov.fgmres(prob.apply_K, P, prob.b, rtol=1e-10)
        assert st["iterations"] <= 3, st["iterations"]
        assert prob.residual(x) < 1e-10


def _spd_with_spectrum(lams, seed, dscale=None):
    """SPD matrix A and diagonal preconditioner minv with minv * A similar to
    diag(lams): A = D^-1/2 Q diag(lams) Q^T D^-1/2, minv = diag(D)."""
    rng = np.random.default_rng(seed)
    n = len(lams)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.ones(n) if dscale is None else 10.0 ** rng.uniform(-dscale, dscale, n)
    A = (Q * lams) @ Q.T
    A = A / np.sqrt(d)[:, None] / np.sqrt(d)[None, :]
    return 0.5 * (A + A.T), d


@pytest.mark.parametrize("dscale", [None, 2.0])
def test_cg_terminates_in_k_steps_for_k_distinct_eigenvalues(dscale):
    """Preconditioned CG reaches the exact solution after at most k steps when
    minv * A has k distinct eigenvalues (the Krylov space is then exhausted),
    and not before for a generic right-hand side.  A wrong step length or
    direction update loses the termination."""
    k, n = 5, 40
    lams = np.repeat(np.array([0.5, 1.0, 3.0, 7.0, 20.0]), n // k)
    A, minv = _spd_with_spectrum(lams, 3, dscale)
    b = np.random.default_rng(4).standard_normal(n)
    x, it = krylov.cg(lambda v: A @ v, b, minv, rtol=1e-10, maxit=50)
    assert it == k
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10 * np.abs(x).max())
    x4, it4 = krylov.cg(lambda v: A @ v, b, minv, rtol=1e-10, maxit=k - 1)
    assert it4 == k - 1 and np.linalg.norm(b - A @ x4) > 1e-6 * np.linalg.norm(b)


def test_cg_matches_dense_solve_and_minimises_energy():
    """On a random SPD system CG converges to the dense solution, and each
    iterate minimises the A-norm error over its Krylov space: the error
    decreases monotonically in the A-norm."""
    rng = np.random.default_rng(7)
    n = 60
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    minv = 1.0 / np.diag(A)
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    x, it = krylov.cg(lambda v: A @ v, b, minv, rtol=1e-12, maxit=200)
    assert it < 200 and np.allclose(x, xs, rtol=1e-10, atol=1e-12)
    errs = []
    for m in range(1, 8):
        xm, _ = krylov.cg(lambda v: A @ v, b, minv, rtol=0.0, maxit=m)
        e = xm - xs
        errs.append(e @ (A @ e))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    # a start vector: the same solution, residual measured against b
    x0 = rng.standard_normal(n)
    x2, _ = krylov.cg(lambda v: A @ v, b, minv, rtol=1e-12, maxit=200, x0=x0)
    assert np.allclose(x2, xs, rtol=1e-10, atol=1e-12)
