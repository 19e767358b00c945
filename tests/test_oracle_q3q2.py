"""Pins of the oracle's Q3-Q2 pair (k = 2 of Sec. 2.1) on uniform meshes.

Fixed by:
  * the 1D basis: Lagrange property on the Gauss-Lobatto points, whose
    interior points are the roots of P_3'(2t - 1) (+-1/sqrt 5 on [-1, 1]),
    partition of unity, derivatives against finite differences;
  * the element matrices: the 4-point rule equals the 6-point rule (the
    forms are polynomials of degree <= 7 per variable); K is symmetric with
    exactly the six rigid modes as null space; B annihilates the rigid modes
    and maps u = (x, 0, 0) (div u = 1) to -(M 1); M against the Kronecker
    product of the exact 1D Q2 mass matrix;
  * the transfers reproduce every Q3 polynomial (degree <= 3 per variable)
    that vanishes on the boundary, and any Q3 polynomial without the
    boundary condition;
  * the operator with Dirichlet rows is symmetric positive definite;
  * optimal rates of the pair on the manufactured solution of the k = 1 pins:
    velocity L2 ~ h^4, H1 ~ h^3, pressure L2 ~ h^3;
  * GMG-FGMRES equals the sparse direct solve on a sinker problem."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fe, q3q2
from paper_1907_06696_amd import inputs
from tests.test_oracle_solve import exact_grad_u, exact_p, exact_u, forcing


def test_gauss_lobatto_basis():
    g = q3q2.GLL3
    x = 2 * g[1:3] - 1
    assert np.allclose(15 * x ** 2 - 3, 0.0, atol=1e-14)                 # roots of P_3'
    assert np.allclose(q3q2.lagrange_1d(g, g), np.eye(4), atol=1e-15)
    t = np.linspace(0, 1, 17)
    assert np.allclose(q3q2.lagrange_1d(g, t).sum(axis=0), 1.0, atol=1e-14)
    e = 1e-6
    fd = (q3q2.lagrange_1d(g, t + e) - q3q2.lagrange_1d(g, t - e)) / (2 * e)
    assert np.allclose(q3q2.lagrange_1d_deriv(g, t), fd, atol=1e-7)
    assert np.allclose(q3q2.lagrange_1d_deriv(g, t).sum(axis=0), 0.0, atol=1e-12)
    assert np.allclose(q3q2.GLL2, [0, 0.5, 1])


def _rigid(pos):
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    one, zero = np.ones_like(x), np.zeros_like(x)
    return np.stack([np.stack(r, 1).ravel() for r in
                     [(one, zero, zero), (zero, one, zero), (zero, zero, one),
                      (-y, x, zero), (zero, -z, y), (z, zero, -x)]], 1)


def test_element_matrices():
    K, B, M = q3q2.element_matrices(4)
    K6, B6, M6 = q3q2.element_matrices(6)
    assert np.abs(K - K6).max() < 1e-12 * np.abs(K).max()
    assert np.abs(B - B6).max() < 1e-13 and np.abs(M - M6).max() < 1e-14
    assert np.abs(K - K.T).max() < 1e-13
    loc = np.array([(q3q2.GLL3[a], q3q2.GLL3[b], q3q2.GLL3[c]) for c in range(4) for b in range(4) for a in range(4)])
    R = _rigid(loc)
    assert np.abs(K @ R).max() < 1e-12
    ev = np.linalg.eigvalsh(K)
    assert np.all(ev[:6] < 1e-10) and ev[6] > 1e-3
    assert np.abs(B @ R).max() < 1e-13
    ux = np.stack([loc[:, 0], 0 * loc[:, 0], 0 * loc[:, 0]], 1).ravel()
    assert np.allclose(B @ ux, -M.sum(axis=1), atol=1e-14)
    M1 = fe.Q2_MASS_1D
    assert np.allclose(M, np.kron(M1, np.kron(M1, M1)), atol=1e-15)


def _q3_poly(pos, bc):
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    if bc:
        b = x * (1 - x) * y * (1 - y) * z * (1 - z)
        return np.stack([b * (1 + x), b * (2 - y * z), b * (x - z)], 1).ravel()
    a = 1 + x ** 3 - 2 * y * z + x * x * y * z ** 3 - 3 * z * z * x * y ** 3
    return np.stack([a, 2 - y ** 3 + x * y * z, a * 0 + x ** 2 * y ** 2 * z ** 2], 1).ravel()


def test_transfers_reproduce_q3_polynomials():
    for L in (2, 3):
        c, f = q3q2.UniformMesh(L - 1), q3q2.UniformMesh(L)
        P = q3q2.prolongation(c, f)
        xc = _q3_poly(c.node_positions(), True) * c.free_dofs_mask()
        assert np.allclose(P @ xc, _q3_poly(f.node_positions(), True), atol=1e-14)
        P1 = sp.csr_matrix(q3q2.prolongation_1d(c, f))
        Pn = sp.kron(sp.kron(P1, P1), P1, format='csr')      # (x fastest: symmetric in the axes)
        Pn = sp.kron(Pn, sp.identity(3), format='csr')
        assert np.allclose(Pn @ _q3_poly(c.node_positions(), False), _q3_poly(f.node_positions(), False),
                           atol=1e-13)


def test_operator_spd_and_rigid_null_space_without_bc():
    m = q3q2.UniformMesh(1)
    rg = np.random.default_rng(3)
    mu = 10 ** rg.uniform(0, 3, m.ncell)
    Kf = q3q2.assemble_K(m, mu)
    R = _rigid(m.node_positions())
    assert np.abs(Kf @ R).max() < 1e-11 * abs(Kf).max()
    A = q3q2.assemble_A(m, mu).toarray()
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    sla.cholesky(A)


def _errors(m, u, p, nq=5):
    pts, w = fe.gauss_points_3d(nq)
    phi, g = q3q2.basis(q3q2.GLL3, pts)
    psi, _ = q3q2.basis(q3q2.GLL2, pts)
    X = (m.cijk[:, None, :] + pts[None]) * m.h
    U = u.reshape(-1, 3)[m.cell_nodes]
    uh = np.einsum('aq,nac->nqc', phi, U)
    guh = np.einsum('adq,nac->nqcd', g, U) / m.h
    ph = np.einsum('aq,na->nq', psi, p[m.cell_pnodes])
    jw = w[None, :] * m.h ** 3
    eu = np.sqrt((jw[..., None] * (uh - exact_u(X)) ** 2).sum())
    eg = np.sqrt((jw[..., None, None] * (guh - exact_grad_u(X)) ** 2).sum())
    ep = np.sqrt((jw * (ph - exact_p(X)) ** 2).sum())
    return np.array([eu, eg, ep])


def _solve(L):
    m = q3q2.UniformMesh(L, with_pressure=True)
    if L <= 2:
        prob = q3q2.StokesProblem(L, np.ones(m.ncell), forcing(m.gauss_points()), with_gmg=False)
        x = prob.solve_direct()
        assert prob.residual(x) < 1e-11
    else:
        # the GMG-FGMRES solve (checked against the direct solve below), to round-off level
        prob = q3q2.StokesProblem(L, np.ones(m.ncell), forcing(m.gauss_points()))
        x, st = prob.solve_fgmres(rtol=1e-12)
        assert prob.residual(x) <= 1e-12
    u, p = prob.distribute(x)
    return _errors(prob.mesh, u, p)


@pytest.mark.slow
def test_manufactured_rates():
    e = [_solve(L) for L in (1, 2, 3)]
    r = np.log2(e[1] / e[2])
    assert r[0] > 3.8 and r[1] > 2.85 and r[2] > 2.85, (r, e)
    # below Q2-Q1 on the same mesh (k = 1: velocity L2 error 9.4e-4 at 8^3)
    assert e[2][0] < 3e-4, e


def test_gmg_fgmres_matches_direct_on_sinkers():
    L = 2
    m = q3q2.UniformMesh(L, with_pressure=True)
    cen = inputs.sinker_centres(4, 1)
    X = m.gauss_points().reshape(-1, 3)
    mu = q3q2.harmonic_cell_viscosity(inputs.sinker_mu(X, cen, 1e2).reshape(-1, 64))
    f = inputs.sinker_force(X, cen).reshape(-1, 64, 3)
    prob = q3q2.StokesProblem(L, mu, f)
    x, st = prob.solve_fgmres(rtol=1e-10)
    assert prob.residual(x) <= 1e-10
    xd = prob.solve_direct()
    assert prob.residual(xd) < 1e-12
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-6
    assert st["iterations"] < 100, st["iterations"]
