"""Pins of the oracle's operators, viscosity averaging and transfers.

Fixed by: the rigid-body null space of the strain-rate form (exact for linear
fields, also through hanging-node constraints), symmetry and positive
definiteness with boundary conditions, two independent implementations of A
(assembled vs cellwise), reproduction of Q2 polynomials by the transfers, and
closed forms for the averages."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fe, mesh, operators as ops
from tests.test_oracle_mesh import adaptive_hierarchy


def _rigid(pos):
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    one, zero = np.ones_like(x), np.zeros_like(x)
    return [np.stack(m, 1).ravel() for m in [(one, zero, zero), (zero, one, zero), (zero, zero, one),
                                             (-y, x, zero), (zero, -z, y), (z, zero, -x)]]


def _hierarchies():
    return [mesh.Hierarchy.uniform(2), adaptive_hierarchy(2, (1, 1, 1), 1),
            adaptive_hierarchy(2, (0, 1, 0), 2)]


def test_rigid_modes_in_null_space_without_bc():
    rng = np.random.default_rng(1)
    for H in _hierarchies():
        for m in H.levels.values():
            mu = 10 ** rng.uniform(0, 4, m.ncell)
            hanging, free, Cn = m.C_no_dirichlet()
            Cu = sp.kron(Cn, sp.identity(3), format='csr')
            K = ops.assemble_K(m, mu)
            A = Cu.T @ K @ Cu
            fmask = np.repeat(free, 3)
            nrm = abs(A).max()
            for r in _rigid(m.node_positions()):
                rf = np.where(fmask, r, 0.0)
                # the constraints reproduce the rigid mode at hanging nodes
                assert np.allclose((Cu @ rf), r, atol=1e-13)
                assert np.abs(A @ rf).max() <= 1e-13 * nrm * np.abs(r).max() * 10


def test_spd_with_boundary_conditions():
    rng = np.random.default_rng(2)
    for H in _hierarchies():
        m = H.leaf
        mu = 10 ** rng.uniform(0, 4, m.ncell)
        A = ops.assemble_A(m, mu)
        assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
        sla.cholesky(A.toarray())                       # raises if not SPD
        x = rng.standard_normal(m.n_u)
        assert x @ (A @ x) > 0
        # identity rows on constrained dofs
        c = ~m.free_dofs_mask()
        Ad = A.toarray()
        assert np.allclose(Ad[np.ix_(c, c)], np.eye(c.sum()))
        assert np.abs(Ad[np.ix_(c, ~c)]).max() == 0


def test_cellwise_equals_assembled():
    rng = np.random.default_rng(3)
    for H in _hierarchies():
        for m in H.levels.values():
            mu = 10 ** rng.uniform(0, 4, m.ncell)
            A = ops.assemble_A(m, mu)
            Cw = ops.CellwiseA(m, mu)
            x = rng.uniform(-1, 1, m.n_u)
            assert np.abs(A @ x - Cw.matvec(x, chunk=7)).max() <= 1e-13 * np.abs(A @ x).max()
            assert np.allclose(A.diagonal(), Cw.diagonal(), rtol=1e-13)


def test_operator_scales_with_cell_size_and_viscosity():
    """Uniform 2^l mesh, constant mu: a(u,u) for u = bubble times 3 is
    independent of the mesh once the interpolant is exact (Q2 bubble)."""
    vals = []
    for L in (1, 2, 3):
        m = mesh.Hierarchy.uniform(L).leaf
        p = m.node_positions()
        b = 64 * p[:, 0] * (1 - p[:, 0]) * p[:, 1] * (1 - p[:, 1]) * p[:, 2] * (1 - p[:, 2])
        u = np.stack([b, 2 * b, -b], 1).ravel()
        A = ops.assemble_A(m, np.full(m.ncell, 3.0))
        vals.append(u @ (A @ u))
    assert np.allclose(vals, vals[0], rtol=1e-12)


def test_harmonic_and_parent_averages():
    rng = np.random.default_rng(4)
    mu = np.full((5, 27), 7.5)
    assert np.allclose(ops.harmonic_cell_viscosity(mu), 7.5)
    mu = 10 ** rng.uniform(0, 6, (50, 27))
    _, w = fe.gauss_points_3d(3)
    harm = ops.harmonic_cell_viscosity(mu)
    assert np.all(harm <= (mu * w).sum(1) + 1e-9)
    assert np.all(harm >= mu.min(1) - 1e-12) and np.all(harm <= mu.max(1) + 1e-12)
    # two-valued cell: 1/mu_K = (W_a / a + W_b / b), W the weight share of each value
    m2 = np.where(np.arange(27) % 2 == 0, 2.0, 8.0)[None, :]
    Wa = w[np.arange(27) % 2 == 0].sum()
    assert np.isclose(ops.harmonic_cell_viscosity(m2)[0], 1.0 / (Wa / 2.0 + (1 - Wa) / 8.0))
    H = adaptive_hierarchy(2, (1, 1, 1), 1)
    mul = rng.uniform(1, 2, H.leaf.ncell)
    mus = ops.level_viscosities(H, mul)
    for ell in range(1, H.L + 1):
        vol = 8.0 ** -H.levels[ell].lev.astype(float)
        # arithmetic child means preserve the volume integral of mu
        assert np.isclose((mus[ell] * vol).sum(), (mul * 8.0 ** -H.leaf.lev.astype(float)).sum())
    assert np.allclose(ops.level_viscosities(mesh.Hierarchy.uniform(2), np.full(64, 3.0))[1], 3.0)


def test_prolongation_reproduces_q2_and_is_interpolation():
    for H in _hierarchies() + [adaptive_hierarchy(3, (2, 5, 3), 2)]:
        for ell in range(2, H.L + 1):
            f, c = H.levels[ell], H.levels[ell - 1]
            P = ops.prolongation(H, ell)
            def bub(pos):
                x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
                b = 64 * x * (1 - x) * y * (1 - y) * z * (1 - z)
                return np.stack([b, -2 * b, 0.5 * b], 1).ravel()
            xc = np.where(c.free_dofs_mask(), bub(c.node_positions()), 0.0)
            xf = P @ xc
            ref = bub(f.node_positions())
            ff = f.free_dofs_mask()
            assert np.allclose(xf[ff], ref[ff], atol=1e-14)
            assert np.all(xf[~ff] == 0)
            # without boundary conditions: any Q2 polynomial is reproduced at
            # every fine node that is not hanging
            Pn = ops.prolongation(H, ell, dirichlet=False)
            fh, ffree, _ = f.C_no_dirichlet()
            ch, cfree, _ = c.C_no_dirichlet()
            def q2(pos):
                x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
                a = 1 + x - 2 * y * z + x * x * y * z * z - 3 * z * z * x
                b = 2 - y * y + x * y * z
                return np.stack([a, b, a - b], 1).ravel()
            xc = np.where(np.repeat(cfree, 3), q2(c.node_positions()), 0.0)
            xf = Pn @ xc
            ref = q2(f.node_positions())
            ff = np.repeat(ffree, 3)
            assert np.allclose(xf[ff], ref[ff], atol=1e-13)
            assert np.all(xf[~ff] == 0)


def test_rhs_partition_of_unity_and_divergence():
    H = adaptive_hierarchy(2, (1, 0, 1), 1)
    m = H.leaf
    f = np.zeros((m.ncell, 27, 3))
    f[:, :, 2] = 1.0
    F = ops.assemble_F_full(m, f)
    assert np.isclose(F[2::3].sum(), 1.0) and np.allclose(F[0::3], 0)
    B = ops.assemble_B(m)
    # int div phi_j = 0 for free velocity dofs: constant pressure is in B^T's kernel
    ones = np.where(m.pfree, 1.0, 0.0)
    assert np.abs(B.T @ ones).max() < 1e-14
    Mp = ops.assemble_Mp(m, np.full(m.ncell, 4.0))
    assert np.isclose(ones @ (Mp @ ones), 0.25, rtol=1e-12)
    Cp = m.Cp
    mfull = ops.pressure_mean_weights(m)
    assert np.isclose(mfull.sum(), 1.0)


def _gauss2():
    """2-point Gauss rule on [0, 1] (exact for cubics)."""
    g = 0.5 / np.sqrt(3.0)
    return np.array([0.5 - g, 0.5 + g]), np.array([0.5, 0.5])


def _trilinear_p(pos):
    x, y, z = pos[..., 0], pos[..., 1], pos[..., 2]
    return (1.0 + 2.0 * x) * (2.0 - y) * (1.0 + 0.5 * z) + 0.3 * x * y


@pytest.mark.parametrize("which", ["uniform", "hanging"])
def test_pressure_mass_is_inverse_viscosity_weighted(which):
    """Sec. 2.2.2: [M_p]_ij = int mu^-1 psi_i psi_j with the cell viscosity.
    A global trilinear function is a Q1 function on every cell (and continuous
    across hanging faces), so with its values at the free pressure nodes
    p^T M_p p = sum_K mu_K^-1 int_K p^2, integrated here cell by cell with a
    2x2x2 Gauss rule (exact for the tri-quadratic p^2); and 1^T M_p 1 =
    sum_K h_K^3 / mu_K.  Non-constant mu: a mu where mu^-1 belongs, or a wrong
    power of h, fails."""
    H = mesh.Hierarchy.uniform(2) if which == "uniform" else adaptive_hierarchy(2, (1, 0, 1), 1)
    m = H.leaf
    rng = np.random.default_rng(5)
    mu = 10.0 ** rng.uniform(-2, 2, m.ncell)
    Mp = ops.assemble_Mp(m, mu)
    pos = m.unkey(m.pkeys).astype(np.float64) / m.S
    p = np.where(m.pfree, _trilinear_p(pos), 0.0)
    g, w = _gauss2()
    qx = np.array([(a, b, c) for c in g for b in g for a in g])
    qw = np.array([a * b * c for c in w for b in w for a in w])
    org = m.cell_origin() / m.S
    exact = 0.0
    for K in range(m.ncell):
        X = org[K][None, :] + qx * m.h[K]
        exact += (qw * _trilinear_p(X) ** 2).sum() * m.h[K] ** 3 / mu[K]
    assert np.isclose(p @ (Mp @ p), exact, rtol=1e-12)
    ones = np.where(m.pfree, 1.0, 0.0)
    assert np.isclose(ones @ (Mp @ ones), (m.h ** 3 / mu).sum(), rtol=1e-12)
    if which == "uniform":
        # per-node row sums: each Q1 basis function integrates to h^3/8 over a cell
        rows = np.zeros(m.npnode)
        for K in range(m.ncell):
            rows[m.cell_pnodes[K]] += m.h[K] ** 3 / (8.0 * mu[K])
        assert np.allclose(Mp @ ones, rows, rtol=1e-12, atol=0)


def test_cellwise_B_equals_assembled_and_residual_of_direct_solve():
    """The cellwise B, B^T equal the assembled B on uniform and hanging
    meshes; the cellwise Stokes residual of the direct solve is at round-off,
    and of a perturbed solution it equals ||b - K x|| / ||b|| from the
    assembled block matrix."""
    from oracle import krylov
    for H in _hierarchies():
        m = H.leaf
        B = ops.assemble_B(m)
        Bc = ops.CellwiseB(m)
        rng = np.random.default_rng(3)
        u = rng.uniform(-1, 1, m.n_u) * m.free_dofs_mask()
        p = rng.uniform(-1, 1, m.npnode) * m.pfree
        assert np.abs(Bc.matvec(u) - B @ u).max() <= 1e-14 * np.abs(B @ u).max()
        assert np.abs(Bc.rmatvec(p) - B.T @ p).max() <= 1e-14 * np.abs(B.T @ p).max()
    H = adaptive_hierarchy(2, (1, 0, 1), 1)
    m = H.leaf
    X = ops.gauss_points_of_cells(m).reshape(-1, 3)
    from paper_1907_06696_amd import inputs
    c = inputs.sinker_centres(3, 1)
    mu = ops.harmonic_cell_viscosity(inputs.sinker_mu(X, c, 1e3).reshape(-1, 27))
    f = inputs.sinker_force(X, c).reshape(-1, 27, 3)
    prob = krylov.StokesProblem(H, mu, f)
    x = prob.solve_direct()
    nu = m.n_u
    assert ops.stokes_residual(m, mu, prob.b[:nu], x[:nu], x[nu:]) <= 1e-12
    xp = x + 1e-3 * np.random.default_rng(4).uniform(-1, 1, len(x)) * np.concatenate(
        [m.free_dofs_mask(), m.pfree])
    ref = np.linalg.norm(prob.b - prob.apply_K(xp)) / np.linalg.norm(prob.b)
    assert np.isclose(ops.stokes_residual(m, mu, prob.b[:nu], xp[:nu], xp[nu:]), ref, rtol=1e-10)
