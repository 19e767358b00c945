"""Pins of the oracle's reference element (Sec. 2.1 bilinear forms).

Each check is fixed by mathematics independent of the oracle's own code path:
exact 1D integrals, a higher-order quadrature, closed-form diagonal entries,
the null space of the strain-rate form, and exactness of the Gauss rule."""
import numpy as np

from oracle import fe


def test_gauss_rule_exact_to_degree_5():
    x, w = fe.gauss_1d(3)
    for p in range(6):
        assert abs((w * x ** p).sum() - 1.0 / (p + 1)) < 1e-15
    assert abs((w * x ** 6).sum() - 1.0 / 7) > 1e-6       # degree 6 is not exact


def test_1d_bases_are_lagrange():
    t = np.array([0.0, 0.5, 1.0])
    assert np.allclose(fe.q2_1d(t), np.eye(3), atol=1e-15)
    assert np.allclose(fe.q1_1d(np.array([0.0, 1.0])), np.eye(2))
    s = np.linspace(0, 1, 11)
    assert np.allclose(fe.q2_1d(s).sum(axis=0), 1.0)
    assert np.allclose(fe.q2_1d_deriv(s).sum(axis=0), 0.0)
    # derivative by central differences
    e = 1e-6
    fd = (fe.q2_1d(s + e) - fe.q2_1d(s - e)) / (2 * e)
    assert np.allclose(fd, fe.q2_1d_deriv(s), atol=1e-8)


def test_closed_form_1d_integrals():
    """The 1D matrices used by the Kronecker route, recomputed by a 10-point rule."""
    x, w = fe.gauss_1d(10)
    L, dL = fe.q2_1d(x), fe.q2_1d_deriv(x)
    assert np.allclose((L * w) @ L.T, fe.Q2_MASS_1D, atol=1e-15)
    assert np.allclose((dL * w) @ dL.T, fe.Q2_STIFF_1D, atol=1e-14)
    assert np.allclose((dL * w) @ L.T, fe.Q2_GRAD_1D, atol=1e-15)


def test_element_matrix_three_routes_agree():
    K3, B3, M3 = fe.element_matrices(3)
    K5, B5, M5 = fe.element_matrices(5)
    Kk = fe.element_matrix_K_kronecker()
    assert np.abs(K3 - K5).max() < 1e-13
    assert np.abs(K3 - Kk).max() < 1e-13
    assert np.abs(B3 - B5).max() < 1e-14
    assert np.abs(M3 - M5).max() < 1e-15


def test_diagonal_closed_forms():
    """diag of the strain-rate matrix = int |grad phi|^2 + (d_c phi)^2:
    vertex node 112/675, cell-centre node 4096/675 (unit cube, mu = 1)."""
    K, _, _ = fe.element_matrices(3)
    for c in range(3):
        assert abs(K[3 * 0 + c, 3 * 0 + c] - 112 / 675) < 1e-14
        assert abs(K[3 * 13 + c, 3 * 13 + c] - 4096 / 675) < 1e-13


def _rigid_modes(pos):
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    one, zero = np.ones_like(x), np.zeros_like(x)
    modes = [(one, zero, zero), (zero, one, zero), (zero, zero, one),
             (-y, x, zero), (zero, -z, y), (z, zero, -x)]
    return [np.stack(m, axis=1).ravel() for m in modes]


def test_strain_form_null_space_is_rigid_motions():
    K, _, _ = fe.element_matrices(3)
    ev = np.linalg.eigvalsh(K)
    assert (np.abs(ev) < 1e-12).sum() == 6
    assert ev.min() > -1e-12
    for r in _rigid_modes(fe.q2_local_positions()):
        assert np.abs(K @ r).max() < 1e-13
    # a non-rigid linear field (pure shear strain) is not in the null space
    pos = fe.q2_local_positions()
    shear = np.stack([pos[:, 1], pos[:, 0], 0 * pos[:, 0]], axis=1).ravel()
    assert np.abs(K @ shear).max() > 0.1


def test_strain_energy_of_linear_field():
    """u = G x with constant G: a(u,u) = int 2 eps:eps = 2 |sym G|^2 on the unit cube."""
    K, _, _ = fe.element_matrices(3)
    rng = np.random.default_rng(0)
    G = rng.standard_normal((3, 3))
    pos = fe.q2_local_positions()
    u = (pos @ G.T).ravel()
    E = 0.5 * (G + G.T)
    assert abs(u @ K @ u - 2 * (E * E).sum()) < 1e-12


def test_divergence_and_mass_closed_forms():
    _, B, M = fe.element_matrices(3)
    m1 = np.array([[2., 1.], [1., 2.]]) / 6
    assert np.allclose(M, np.kron(np.kron(m1, m1), m1), atol=1e-15)
    # u = (x, 2y, -z): div u = 2, so B u = -2 int psi_i = -2 * row sums of M
    pos = fe.q2_local_positions()
    u = np.stack([pos[:, 0], 2 * pos[:, 1], -pos[:, 2]], axis=1).ravel()
    assert np.allclose(B @ u, -2 * M.sum(axis=1), atol=1e-15)
    # rigid rotations are divergence free
    for r in _rigid_modes(pos)[3:]:
        assert np.abs(B @ r).max() < 1e-15
