"""Pins of the oracle's learned-scaling part: MLP gradients against central
finite differences, the first Adam step in closed form, scaling invariance of
the smoother, the Ritz pair of the lambda estimate (Rayleigh quotient,
exact eigenvalue when converged), the adjoint V-cycle gradient against central
finite differences (lambda held fixed, and lambda re-estimated by a converged
Lanczos run), the invariance of the gradient under y -> y + c, and feature
values on known fields.  The fitted targets themselves have no closed form
(parity unpinned)."""
import numpy as np
import pytest

from oracle import learned as ol, mesh, multigrid as mg, operators as ops
from tests.test_oracle_mesh import adaptive_hierarchy


def test_mlp_backward_matches_finite_differences():
    rg = np.random.default_rng(0)
    w = ol.init_params(1) + rg.normal(0, 0.05, ol.N_PARAMS)
    w[-3 - 192:-3] *= 0.2                        # keep the outputs inside the clamp
    assert len(w) == ol.N_PARAMS == 6147
    x = rg.normal(0, 0.5, (7, 27))
    dy = rg.normal(0, 1, (7, 3))
    y, cache = ol.mlp_forward(w, x)
    assert np.all(np.abs(y) < ol.CLAMP)          # FD is valid away from the clamp
    g = ol.mlp_backward(w, cache, dy)
    idx = rg.choice(ol.N_PARAMS, 60, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(w)
        e[i] = eps
        fd = ((ol.mlp_forward(w + e, x)[0] - ol.mlp_forward(w - e, x)[0]) * dy).sum() / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_gelu_derivative_and_clamp():
    z = np.linspace(-4, 4, 81)
    fd = (ol.gelu(z + 1e-6) - ol.gelu(z - 1e-6)) / 2e-6
    assert np.allclose(fd, ol.gelu_deriv(z), atol=1e-8)
    assert np.isclose(ol.gelu(np.array([0.0]))[0], 0.0) and np.isclose(ol.gelu(np.array([1.0]))[0], 0.8413447460685429)
    w = ol.init_params(0)
    w[-3:] = [5.0, -5.0, 0.5]                        # output biases push two outputs beyond the clamp
    y, cache = ol.mlp_forward(w, np.zeros((2, 27)))
    assert np.allclose(y[:, 0], 2.0) and np.allclose(y[:, 1], -2.0)
    g = ol.mlp_backward(w, cache, np.ones((2, 3)))
    assert g[-3] == 0 and g[-2] == 0 and g[-1] == 2.0


def test_adam_first_step_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = ol.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    # bias-corrected moments equal g and g^2 after one step: update = lr g / (|g| + eps)
    assert np.allclose(w1, w - 0.1 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def _gmg(H, seed=0):
    mu = 10 ** np.random.default_rng(seed).uniform(0, 2, H.leaf.ncell)
    return mg.GMG(H, ops.level_viscosities(H, mu))


def test_constant_scaling_is_invariant():
    H = mesh.Hierarchy.uniform(3)
    G = _gmg(H)
    ell = 3
    nc = H.levels[ell].ncell
    J0, _ = ol.objective(G, ell, np.zeros((nc, 3)), with_grad=False)
    J1, _ = ol.objective(G, ell, np.full((nc, 3), 0.7), with_grad=False)
    assert abs(J0 - J1) <= 1e-10 * abs(J0)
    s = ol.dof_scaling(H.levels[ell], np.full((nc, 3), 0.7))
    assert np.allclose(s, np.exp(0.7))


@pytest.mark.parametrize("which", ["uniform", "adaptive"])
def test_adjoint_gradient_matches_finite_differences(which):
    H = mesh.Hierarchy.uniform(2) if which == "uniform" else adaptive_hierarchy(1, (0, 0, 0), 1)
    G = _gmg(H, 3)
    ell = H.L
    m = H.levels[ell]
    rg = np.random.default_rng(4)
    y = rg.uniform(-0.5, 0.5, (m.ncell, 3))
    lam = ol.ScaledLevel(G, ell, ol.dof_scaling(m, y)).lam
    J, g = ol.objective(G, ell, y, lam=lam)
    eps = 1e-5
    for ci in rg.choice(m.ncell, min(6, m.ncell), replace=False):
        for c in range(3):
            e = np.zeros_like(y)
            e[ci, c] = eps
            fd = (ol.objective(G, ell, y + e, lam=lam, with_grad=False)[0]
                  - ol.objective(G, ell, y - e, lam=lam, with_grad=False)[0]) / (2 * eps)
            assert abs(fd - g[ci, c]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), (ci, c, fd, g[ci, c])


def _scaled_problem():
    H = mesh.Hierarchy.uniform(2)
    G = _gmg(H, 3)
    ell = 2
    m = H.levels[ell]
    y = np.random.default_rng(4).uniform(-0.5, 0.5, (m.ncell, 3))
    return H, G, ell, m, y


def test_ritz_pair_of_lambda_estimate():
    import scipy.linalg as sla
    H, G, ell, m, y = _scaled_problem()
    A, free = G.A[ell], G.free[ell]
    minv = np.where(free, ol.dof_scaling(m, y) / A.diagonal(), 1.0)
    r0 = ol.rng.dof_vector(m, mg.LAMBDA_SEED) * free
    fi = np.nonzero(free)[0]
    exact = sla.eigh(A.toarray()[np.ix_(fi, fi)], np.diag(1.0 / minv[fi]), eigvals_only=True)[-1]
    for steps in (12, 40):
        theta, v = ol.cg_lanczos_ritz(lambda x: A @ x, minv, r0, steps)
        assert abs(theta - mg.cg_lanczos_lambda_max(lambda x: A @ x, minv, r0, steps)) <= 1e-12 * theta
        rq = (v @ (A @ v)) / (v @ np.where(free, v / minv, 0.0))
        assert abs(rq - theta) <= 1e-10 * theta            # a Ritz pair: its Rayleigh quotient is theta
        assert np.all(v[~free] == 0)
        assert theta <= exact * (1 + 1e-12)                 # Ritz values lie inside the spectrum
    assert abs(theta - exact) <= 1e-10 * exact              # 40 steps: converged
    # the eigenvector residual of the converged pair vanishes
    r = A @ v - theta * np.where(free, v / minv, 0.0)
    assert np.linalg.norm(r[free]) <= 1e-6 * np.linalg.norm((A @ v)[free])


def test_gradient_with_reestimated_lambda_matches_finite_differences():
    """With a converged Lanczos estimate lambda(s) is the extreme eigenvalue,
    whose derivative is the Rayleigh-quotient derivative at v: the full
    gradient (fixed-lambda adjoint + lambda term) equals central differences
    of J with lambda re-estimated at every evaluation."""
    H, G, ell, m, y = _scaled_problem()
    J, g = ol.objective(G, ell, y, lanczos_steps=40)
    rg = np.random.default_rng(1)
    eps = 1e-5
    for ci in rg.choice(m.ncell, 4, replace=False):
        for c in range(3):
            e = np.zeros_like(y)
            e[ci, c] = eps
            fd = (ol.objective(G, ell, y + e, with_grad=False, lanczos_steps=40)[0]
                  - ol.objective(G, ell, y - e, with_grad=False, lanczos_steps=40)[0]) / (2 * eps)
            assert abs(fd - g[ci, c]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), (ci, c, fd, g[ci, c])


def test_gradient_is_shift_invariant():
    """J(y + c) = J(y) for a constant c (lambda re-estimated), so the total
    gradient sums to zero; the fixed-lambda gradient alone does not."""
    H, G, ell, m, y = _scaled_problem()
    _, g = ol.objective(G, ell, y)
    assert abs(g.sum()) <= 1e-10 * np.abs(g).sum()
    lam = ol.ScaledLevel(G, ell, ol.dof_scaling(m, y)).lam
    _, g_fixed = ol.objective(G, ell, y, lam=lam)
    assert abs(g_fixed.sum()) > 1e-3 * np.abs(g_fixed).sum()


def test_fitting_decreases_objective():
    H = mesh.Hierarchy.uniform(3)
    G = _gmg(H, 5)
    y, hist = ol.fit_targets(G, 3, steps=8)
    assert hist[-1] < hist[0]
    assert np.all(np.abs(y) <= ol.CLAMP)


def test_features_known_field():
    H = mesh.Hierarchy.uniform(2)
    mu_leaf = np.ones(H.leaf.ncell)
    mus = ops.level_viscosities(H, mu_leaf)
    f = ol.features(H, mus, 2)
    assert np.all(f == 0)
    # one cell with mu = 100 at (1, 1, 1): neighbours see +2 at the mirrored offset
    lf = H.leaf
    hot = np.nonzero(np.all(lf.ijk == [1, 1, 1], axis=1))[0][0]
    mu_leaf[hot] = 100.0
    mus = ops.level_viscosities(H, mu_leaf)
    f = ol.features(H, mus, 2)
    assert np.allclose(f[hot], np.where(np.arange(27) == 13, 0.0, -2.0))
    nb = np.nonzero(np.all(lf.ijk == [2, 1, 1], axis=1))[0][0]     # +x neighbour sees the hot cell at offset -x
    assert np.isclose(f[nb, 12], 2.0) and np.isclose(np.abs(f[nb]).sum(), 2.0)
    corner = np.nonzero(np.all(lf.ijk == [0, 0, 0], axis=1))[0][0]
    assert f[corner, 0] == 0.0                                      # outside the domain
    # coarser level: the parent averages
    f1 = ol.features(H, mus, 1)
    assert np.isclose(f1[0, 13], 0.0)


def test_features_coarser_cell_rule_on_adaptive_mesh():
    """Features on an adaptive mesh, from the definition by brute force: for a
    cell K of level l in the level-ell mesh, the value at neighbour offset o
    is log10 mu(c) - log10 mu_K, where c is the cell of the level-l mesh G_l
    (which holds K: it is a cell of every level mesh from its own level up)
    whose closed box contains the centre of the level-l position K + o; a
    position outside the unit cube gives 0.  In G_l no cell is finer than l,
    so c is either the same-level neighbour or the coarser cell covering it."""
    H = adaptive_hierarchy(2, (1, 0, 1), 2)
    rng = np.random.default_rng(11)
    mu_leaf = 10.0 ** rng.uniform(0, 4, H.leaf.ncell)
    mus = ops.level_viscosities(H, mu_leaf)
    seen_coarser = 0
    for ell in range(2, H.L + 1):
        f = ol.features(H, mus, ell)
        G = H.levels[ell]
        for ci in range(G.ncell):
            l = int(G.lev[ci])
            Gl = H.levels[l]
            lo = Gl.ijk * (1 << (H.L - Gl.lev))[:, None]              # origins in units of 2^-L
            size = (1 << (H.L - Gl.lev))
            me = np.nonzero((Gl.lev == l) & np.all(Gl.ijk == G.ijk[ci], axis=1))[0][0]
            muK = mus[l][me]
            assert muK == mus[ell][ci]
            n = 1 << l
            for o in range(27):
                d = np.array([o % 3, (o // 3) % 3, o // 9]) - 1
                q = G.ijk[ci] + d
                if np.any(q < 0) or np.any(q >= n):
                    assert f[ci, o] == 0.0
                    continue
                centre2 = (2 * q + 1) * (1 << (H.L - l))               # centre in units of 2^-(L+1)
                inside = np.all((2 * lo <= centre2) & (centre2 <= 2 * (lo + size[:, None])), axis=1)
                hit = np.nonzero(inside)[0]
                assert len(hit) == 1
                if Gl.lev[hit[0]] < l:
                    seen_coarser += 1
                assert np.isclose(f[ci, o], np.log10(mus[l][hit[0]]) - np.log10(muK), rtol=0, atol=1e-13)
    assert seen_coarser > 0
