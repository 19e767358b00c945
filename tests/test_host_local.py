"""Host layer of the local-smoothing hierarchy (no GPU): the library's level
meshes of one refinement level each, their node kinds (inner, domain
boundary, refinement edge) and their transfers agree with the oracle's,
matched by canonical node keys; the leaf-to-level copy covers every free leaf
node once."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import local_smoothing as ols, mesh as omesh, operators as ops
from tests.test_host_mesh import _pair

CASES = [(2, ((1, 1, 1),), 1), (2, ((0, 1, 0),), 2), (3, ((2, 5, 3), (0, 0, 0)), 2), (3, ((7, 0, 3),), 1)]


@pytest.mark.parametrize("base,corners,times", CASES)
def test_local_levels_match_oracle(base, corners, times):
    s, H = _pair(base, corners, times)
    mus = ops.level_viscosities(H, np.ones(H.leaf.ncell))
    G = ols.LocalSmoothingGMG(H, mus)
    lb, ncell, nnode = s.local_levels()
    uniform = [l for l in range(1, H.L + 1) if not G.edge[l].any() and G.T[l].ncell == 8 ** l]
    assert lb == max(uniform)
    for ell in range(1, H.L + 1):
        assert ncell[ell] == G.T[ell].ncell and nnode[ell] == G.T[ell].nnode, ell
    for ell in range(lb + 1, H.L + 1):
        keys, kinds = s.local_nodes(ell)
        T = G.T[ell]
        pos = np.searchsorted(T.keys, keys)
        assert np.array_equal(T.keys[pos], keys)
        ref = np.where(T.dirichlet, 1, np.where(G.edge[ell][::3], 2, 0))
        assert np.array_equal(kinds, ref[pos]), ell
        # transfer: the library's rows and columns mapped to the oracle's nodes
        ptr, col, w = s.local_transfer(ell)
        if ell - 1 == lb:
            ckeys = s.support_points(ell - 1)
        else:
            ckeys, _ = s.local_nodes(ell - 1)
        cpos = np.searchsorted(G.T[ell - 1].keys, ckeys)
        rows = np.repeat(np.arange(len(keys)), np.diff(ptr))
        P = sp.csr_matrix((w, (pos[rows], cpos[col])), shape=(T.nnode, G.T[ell - 1].nnode))
        Pref = G.P[ell][::3, ::3]
        assert abs(P - Pref).max() <= 1e-15, ell
    s.close()
