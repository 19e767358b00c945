"""Pins of the oracle's no-normal-flux variant: u . n = 0 on the boundary of
the unit cube (Sec. 2, eq. stokes and the sentence after it: the algorithms
apply unchanged to no-normal-flux constraints).  On the axis-aligned cube the
condition fixes component c on the two faces normal to axis c; the tangential
components stay free and obey the natural condition of the weak form (zero
tangential stress).

Fixed by:
  * the dof count on uniform meshes: with m lattice points per axis each
    component is fixed on its two normal planes only, 3 (m - 2) m^2 free dofs;
  * the rigid modes: all six lie in the null space of the form without a
    boundary condition, none of them (nor any combination) satisfies
    u . n = 0 on all six faces, and the constrained operator is positive
    definite;
  * a Q2 field satisfying the condition is reproduced by the constraints at
    hanging nodes on the boundary (tangential components interpolated, normal
    ones zero) and by the transfers;
  * optimal Taylor-Hood rates (velocity L2 ~ h^3, H1 ~ h^2, pressure L2 ~ h^2)
    on a manufactured solution whose tangential velocity is nonzero on every
    face and whose tangential stress vanishes there, on uniform meshes and on
    meshes with hanging nodes on the boundary: fixing all components, or the
    tangential instead of the normal ones, does not converge to it;
  * the GMG-FGMRES solve (transfers, smoother and coarse solve under the
    condition) agrees with the sparse direct solve on a sinker problem."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fe, krylov, mesh, operators as ops
from paper_1907_06696_amd import inputs

PI = np.pi


def _hier(base, corner=None, times=1, bc="noflux"):
    lev, ijk = mesh.uniform_leaves(base)
    if corner is not None:
        mask = np.all(ijk == list(corner), axis=1)
        lev, ijk = mesh.balance(*mesh.refine(lev, ijk, mask, times))
    return mesh.Hierarchy(lev, ijk, bc=bc)


def _boundary_hanging(m):
    on_b = np.any((m.xyz == 0) | (m.xyz == m.S), axis=1)
    return m.hanging & on_b


def test_uniform_free_dof_count():
    for L in (1, 2, 3):
        H = mesh.Hierarchy.uniform(L, bc="noflux")
        for ell, m in H.levels.items():
            n = 2 ** (ell + 1) + 1
            assert m.free_dofs_mask().sum() == 3 * (n - 2) * n * n
            assert not m.dirichlet.any() and not m.hanging.any()
            # component c is fixed exactly where coordinate c is 0 or 1
            pos = m.node_positions()
            assert np.array_equal(m.fixed, (pos == 0) | (pos == 1))


def test_fixed_components_on_faces_edges_corners():
    m = mesh.Hierarchy.uniform(1, bc="noflux").leaf
    pos = m.node_positions()
    nb = ((pos == 0) | (pos == 1)).sum(axis=1)     # 0 inside, 1 face, 2 edge, 3 corner
    for k in range(4):
        assert np.all(m.fixed[nb == k].sum(axis=1) == k)


def _rigid(pos):
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    one, zero = np.ones_like(x), np.zeros_like(x)
    return np.stack([np.stack(r, 1).ravel() for r in
                     [(one, zero, zero), (zero, one, zero), (zero, zero, one),
                      (-y, x, zero), (zero, -z, y), (z, zero, -x)]], 1)


def test_no_rigid_mode_survives_and_operator_is_spd():
    rg = np.random.default_rng(5)
    for H in (_hier(1), _hier(2), _hier(2, (0, 1, 0), 1)):
        m = H.leaf
        mu = 10 ** rg.uniform(0, 3, m.ncell)
        R = _rigid(m.node_positions())                                # [n_u, 6]
        # every rigid mode is in the null space of the form without condition
        _, free, Cn = m.C_no_dirichlet()
        Cn3 = sp.kron(Cn, sp.identity(3), format='csr')
        An = Cn3.T @ ops.assemble_K(m, mu) @ Cn3
        Rf = R * np.repeat(free, 3)[:, None]
        assert np.abs(An @ Rf).max() <= 1e-11 * abs(An).max()
        # ... and no combination of them vanishes on the fixed components
        sv = np.linalg.svd(R[m.fixed.ravel()], compute_uv=False)
        assert sv.min() > 0.1 * sv.max()
        A = ops.assemble_A(m, mu)
        assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
        f = m.free_dofs_mask()
        ev = sla.eigvalsh(A.toarray()[np.ix_(f, f)])
        assert ev.min() > 1e-6 * ev.max(), (ev.min(), ev.max())
        # identity rows on the fixed components
        Ad = A.toarray()
        c = ~f
        assert np.allclose(Ad[np.ix_(c, c)], np.eye(c.sum())) and np.abs(Ad[np.ix_(c, f)]).max() == 0


def _q2_noflux(pos):
    """A field of Q2 on every cell (degree <= 2 per variable) that satisfies
    u . n = 0 on the cube and has nonzero tangential components there."""
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    return np.stack([x * (1 - x) * (1 + y), y * (1 - y) * (2 - z), z * (1 - z) * (1 + x * y)], 1).ravel()


def test_boundary_hanging_constraints_and_transfers_reproduce_q2_field():
    for H in (_hier(2, (0, 0, 0), 1), _hier(2, (0, 3, 1), 2)):
        for ell in range(1, H.L + 1):
            m = H.levels[ell]
            ref = _q2_noflux(m.node_positions())
            f = m.free_dofs_mask()
            x = np.where(f, ref, 0.0)
            assert np.allclose(m.Cu() @ x, ref, atol=1e-14)
            if ell >= 2:
                c = H.levels[ell - 1]
                xc = np.where(c.free_dofs_mask(), _q2_noflux(c.node_positions()), 0.0)
                xf = ops.prolongation(H, ell) @ xc
                assert np.allclose(xf[f], ref[f], atol=1e-14) and np.all(xf[~f] == 0)
        bh = _boundary_hanging(H.leaf)
        assert bh.any()
        # tangential components of boundary hanging nodes are interpolated, not zero
        full = H.leaf.Cu() @ np.where(H.leaf.free_dofs_mask(), _q2_noflux(H.leaf.node_positions()), 0.0)
        tang = ~H.leaf.fixed[bh]
        assert np.abs(full.reshape(-1, 3)[bh][tang]).min() > 0


# manufactured solution: u = (d_y phi, -d_x phi, 0), phi = sin(pi x) sin(pi y) cos(pi z)
def exact_u(p):
    s, c = np.sin(PI * p), np.cos(PI * p)
    return PI * np.stack([s[..., 0] * c[..., 1] * c[..., 2], -c[..., 0] * s[..., 1] * c[..., 2], 0 * s[..., 0]], -1)


def exact_grad_u(p):
    """[.., component, direction]"""
    s, c = np.sin(PI * p), np.cos(PI * p)
    sx, sy, sz, cx, cy, cz = s[..., 0], s[..., 1], s[..., 2], c[..., 0], c[..., 1], c[..., 2]
    g = np.zeros(p.shape[:-1] + (3, 3))
    k = PI * PI
    g[..., 0, 0], g[..., 0, 1], g[..., 0, 2] = k * cx * cy * cz, -k * sx * sy * cz, -k * sx * cy * sz
    g[..., 1, 0], g[..., 1, 1], g[..., 1, 2] = k * sx * sy * cz, -k * cx * cy * cz, k * cx * sy * sz
    return g


def exact_p(p):
    c = np.cos(PI * p)
    return c[..., 0] * c[..., 1] * c[..., 2]


def forcing(p):
    """f = -div(2 eps(u)) + grad p = 3 pi^2 u + grad p (mu = 1, div u = 0,
    Laplace phi = -3 pi^2 phi)."""
    s, c = np.sin(PI * p), np.cos(PI * p)
    gp = -PI * np.stack([s[..., 0] * c[..., 1] * c[..., 2], c[..., 0] * s[..., 1] * c[..., 2],
                         c[..., 0] * c[..., 1] * s[..., 2]], -1)
    return 3 * PI * PI * exact_u(p) + gp


def test_manufactured_solution_properties():
    """The solution itself: divergence free, u . n = 0 and zero tangential
    stress 2 eps(u) n - (n . 2 eps(u) n) n on each face, nonzero tangential
    velocity there; f matches a finite-difference -div(2 eps(u)) + grad p."""
    rg = np.random.default_rng(3)
    q = rg.uniform(0.05, 0.95, (50, 3))
    g = exact_grad_u(q)
    assert np.abs(np.trace(g, axis1=-2, axis2=-1)).max() < 1e-12
    for ax in range(3):
        for side in (0.0, 1.0):
            pts = q.copy()
            pts[:, ax] = side
            u = exact_u(pts)
            assert np.abs(u[:, ax]).max() < 1e-12
            e = exact_grad_u(pts)
            sig = e + np.swapaxes(e, -1, -2)
            n = np.zeros(3)
            n[ax] = 1.0
            t = sig @ n
            t[:, ax] = 0.0
            assert np.abs(t).max() < 1e-11
        tang = [c for c in range(3) if c != ax and c != 2]
        if tang:
            pts = q.copy()
            pts[:, ax] = 0.0
            assert np.abs(exact_u(pts)[:, tang]).max() > 0.5
    h = 1e-4
    x0 = q[:5]
    div_sig = np.zeros((5, 3))
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        gp, gm = exact_grad_u(x0 + e), exact_grad_u(x0 - e)
        sp_, sm = gp + np.swapaxes(gp, -1, -2), gm + np.swapaxes(gm, -1, -2)
        div_sig += (sp_[:, :, d] - sm[:, :, d]) / (2 * h)
    gradp = np.stack([(exact_p(x0 + h * np.eye(3)[d]) - exact_p(x0 - h * np.eye(3)[d])) / (2 * h)
                      for d in range(3)], -1)
    assert np.allclose(forcing(x0), -div_sig + gradp, atol=1e-5)


def _errors(m, u_full, p_full, nq=4):
    pts, w = fe.gauss_points_3d(nq)
    phi, g = fe.q2_basis(pts)
    psi, _ = fe.q1_basis(pts)
    X = (m.cell_origin() / m.S)[:, None, :] + pts[None] * m.h[:, None, None]
    U = u_full.reshape(-1, 3)[m.cell_nodes]
    uh = np.einsum('aq,nac->nqc', phi, U)
    guh = np.einsum('adq,nac->nqcd', g, U) / m.h[:, None, None, None]
    ph = np.einsum('aq,na->nq', psi, p_full[m.cell_pnodes])
    jw = w[None, :] * (m.h ** 3)[:, None]
    eu = np.sqrt((jw[..., None] * (uh - exact_u(X)) ** 2).sum())
    eg = np.sqrt((jw[..., None, None] * (guh - exact_grad_u(X)) ** 2).sum())
    ep = np.sqrt((jw * (ph - exact_p(X)) ** 2).sum())
    return np.array([eu, eg, ep])


def _solve(H):
    m = H.leaf
    X = ops.gauss_points_of_cells(m)
    if m.n_u < 20000:
        prob = krylov.StokesProblem(H, np.ones(m.ncell), forcing(X))
        x = prob.solve_direct()
    else:
        prob = krylov.StokesProblem(H, np.ones(m.ncell), forcing(X), gmg_kwargs={})
        x, st = prob.solve_fgmres(rtol=1e-11)
        assert prob.residual(x) <= 1e-11
    u, p = prob.distribute(x)
    return _errors(m, u, p)


@pytest.mark.slow
def test_manufactured_rates_uniform():
    e = [_solve(mesh.Hierarchy.uniform(L, bc="noflux")) for L in (2, 3, 4)]
    r = np.log2(e[1] / e[2])
    assert r[0] > 2.8 and r[1] > 1.85 and r[2] > 1.85, r
    # the Dirichlet condition on the same data does not converge to it
    ed = [_solve(mesh.Hierarchy.uniform(L)) for L in (2, 3)]
    assert ed[1][0] > 0.5 * ed[0][0] and ed[1][0] > 20 * e[1][0], (ed, e)


def _adaptive(L):
    """2^L mesh with a slab along the x = 0 face refined once (hanging nodes
    on the boundary faces x = 0, y = 0 and z = 0)."""
    lev, ijk = mesh.uniform_leaves(L)
    n = 1 << L
    mask = np.all(ijk < n // 2, axis=1) & (ijk[:, 0] < n // 4 + 1)
    lev, ijk = mesh.refine(lev, ijk, mask, 1)
    return mesh.Hierarchy(*mesh.balance(lev, ijk), bc="noflux")


@pytest.mark.slow
def test_manufactured_rates_adaptive():
    H2, H3 = _adaptive(2), _adaptive(3)
    assert _boundary_hanging(H3.leaf).any()
    r = np.log2(_solve(H2) / _solve(H3))
    assert r[0] > 2.7 and r[1] > 1.8 and r[2] > 1.8, r


def test_gmg_fgmres_matches_direct_on_sinkers():
    cfg = inputs.CONFIGS['uniform8']
    for H in (mesh.Hierarchy.uniform(cfg['base_level'], bc="noflux"), _hier(2, (0, 2, 3), 1)):
        m = H.leaf
        cen = inputs.sinker_centres(cfg['sinkers'], cfg['centre_seed'])
        X = ops.gauss_points_of_cells(m).reshape(-1, 3)
        mu = ops.harmonic_cell_viscosity(inputs.sinker_mu(X, cen, cfg['dr']).reshape(-1, 27))
        f = inputs.sinker_force(X, cen).reshape(-1, 27, 3)
        prob = krylov.StokesProblem(H, mu, f, gmg_kwargs={})
        x, st = prob.solve_fgmres(rtol=1e-8)
        assert prob.residual(x) <= 1e-8
        xd = prob.solve_direct()
        assert prob.residual(xd) < 1e-12
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-5
        u, _ = prob.distribute(xd)
        assert np.abs(u.reshape(-1, 3)[m.fixed]).max() == 0
        assert np.abs(u.reshape(-1, 3)[~m.fixed & np.any(m.fixed, axis=1)[:, None]]).max() > 0
