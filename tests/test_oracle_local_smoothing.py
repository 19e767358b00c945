"""Pins of the oracle's local-smoothing V-cycle (the level hierarchy of the
multigrid method the paper cites in Sec. 2.2.1: level meshes of one
refinement level each, Dirichlet on the refinement edge, interface terms).

Fixed by: (i) with a constant viscosity the level operators are Galerkin
products and the level-by-level cycle equals the symmetric multiplicative
subspace correction over the level spaces, computed with level bases built by
evaluating each level basis function at the leaf nodes (no transfer matrices,
no edge operators); (ii) on a uniform mesh there is no refinement edge and
the cycle is the global-coarsening one; (iii) the refinement edge against a
geometric brute force; (iv) symmetry and contraction with variable
viscosity."""
import numpy as np
import pytest

from oracle import local_smoothing as ls, mesh, multigrid as mg, operators as ops
from paper_1907_06696_amd import inputs
from tests.test_oracle_mesh import adaptive_hierarchy

MESHES = [((2, (1, 1, 1), 1)), ((2, (0, 1, 0), 2)), ((3, (7, 0, 3), 1))]


def _sinker_mus(H, dr=1e3, seed=1):
    X = ops.gauss_points_of_cells(H.leaf).reshape(-1, 3)
    mu = ops.harmonic_cell_viscosity(inputs.sinker_mu(X, inputs.sinker_centres(3, seed), dr).reshape(-1, 27))
    return ops.level_viscosities(H, mu)


@pytest.mark.parametrize("base,corner,times", MESHES)
def test_cycle_is_the_multiplicative_subspace_correction(base, corner, times):
    H = adaptive_hierarchy(base, corner, times)
    mus = ops.level_viscosities(H, np.full(H.leaf.ncell, 3.7))
    G = ls.LocalSmoothingGMG(H, mus)
    assert any(G.edge[l].any() for l in G.edge)
    A = ops.assemble_A(H.leaf, mus[H.L])
    E = {l: ls.level_basis(G, l) for l in range(1, H.L + 1)}
    for seed in (5, 6):
        b = inputs.uniform_vector(H.leaf.n_u, seed) * H.leaf.free_dofs_mask()
        xs, gal = ls.subspace_correction(G, A, b, E)
        x = G.vcycle(b)
        assert np.abs(x - xs).max() <= 1e-13 * np.abs(xs).max()
    for l in range(1, H.L + 1):
        dofs = E[l][1]
        ref = G.A[l][np.ix_(dofs, dofs)].toarray()
        assert np.abs(gal[l] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_uniform_mesh_equals_global_coarsening():
    H = mesh.Hierarchy.uniform(3)
    mus = _sinker_mus(H, 1e4)
    G = ls.LocalSmoothingGMG(H, mus)
    assert not any(G.edge[l].any() for l in G.edge)
    b = inputs.uniform_vector(H.leaf.n_u, 3) * H.leaf.free_dofs_mask()
    xg = mg.GMG(H, mus).vcycle(b)
    assert np.abs(G.vcycle(b) - xg).max() <= 1e-13 * np.abs(xg).max()


@pytest.mark.parametrize("base,corner,times", MESHES)
def test_refinement_edge_by_geometry(base, corner, times):
    """A level node lies on the refinement edge iff a point next to it (in
    one of the 8 diagonal directions) is inside the unit cube but inside no
    cell of its level."""
    H = adaptive_hierarchy(base, corner, times)
    for ell in range(1, H.L + 1):
        lev, ijk, _ = ls.level_cells_exact(H, ell)
        T = mesh.LevelMesh(lev, ijk, H.U)
        edge = ls.refinement_edge_mask(T)
        org = T.cell_origin().astype(float)
        size = float(T.cell_size_units()[0])
        eps = 0.25 * size / 2
        ref = np.zeros(T.nnode, dtype=bool)
        for i, p in enumerate(T.xyz.astype(float)):
            if T.dirichlet[i]:
                continue
            for d in np.array([(a, b, c) for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)], float):
                q = p + eps * d
                if np.any(q < 0) or np.any(q > T.S):
                    continue
                inside = np.any(np.all((org <= q) & (q <= org + size), axis=1))
                if not inside:
                    ref[i] = True
                    break
        assert np.array_equal(edge, ref), ell


def test_symmetric_and_contracting_with_variable_viscosity():
    """Symmetric; and a contraction in the A-norm on a mesh that resolves
    the sinkers (8^3 cells, the 20% with the largest |grad log mu| refined
    once, 2:1 balanced; 6 sinkers, contrast 1e3).  On meshes with only 4 to
    16 cells per edge the averaged level viscosities can make it diverge at
    contrast 1e4 (the global-coarsening cycle is at 0.7 there)."""
    c = inputs.sinker_centres(6, 3)
    cells = inputs.refinement_cells(3, c, 1e3, 80.0)
    lev, ijk = mesh.uniform_leaves(3)
    mask = np.isin(mesh.cell_code(lev, ijk), mesh.cell_code(cells[:, 0], cells[:, 1:]))
    lev, ijk = mesh.refine(lev, ijk, mask, 1)
    H = mesh.Hierarchy(*mesh.balance(lev, ijk))
    X = ops.gauss_points_of_cells(H.leaf).reshape(-1, 3)
    mus = ops.level_viscosities(H, ops.harmonic_cell_viscosity(inputs.sinker_mu(X, c, 1e3).reshape(-1, 27)))
    G = ls.LocalSmoothingGMG(H, mus)
    assert any(G.edge[l].any() for l in G.edge)
    lf = H.leaf
    A = ops.CellwiseA(lf, mus[H.L])
    free = lf.free_dofs_mask()
    b = inputs.uniform_vector(lf.n_u, 1) * free
    c2 = inputs.uniform_vector(lf.n_u, 2) * free
    assert abs(c2 @ G.vcycle(b) - b @ G.vcycle(c2)) <= 1e-12 * abs(c2 @ G.vcycle(b))
    e = inputs.uniform_vector(lf.n_u, 3) * free
    for _ in range(8):
        e2 = e - G.vcycle(A @ e)
        rho = np.sqrt((e2 @ (A @ e2)) / (e @ (A @ e)))
        e = e2 / np.sqrt(e2 @ (A @ e2))
    assert rho < 0.95, rho          # 0.84 (the global-coarsening cycle: 0.77)
