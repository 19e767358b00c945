"""Host layer of the Q3-Q2 pair (k = 2 of Sec. 2.1; no GPU): the library's
lattice levels, node kinds, transfers and Gauss points equal the oracle's
(``oracle/q3q2.py``), and the calls that are built for Q2-Q1 only or for
uniform meshes with u = 0 are refused."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fe, q3q2
from paper_1907_06696_amd import mfgmg


def _solver(base):
    s = mfgmg.Solver(base)
    s.set_element(2)
    s.finalize_mesh()
    return s


@pytest.mark.parametrize("base", [1, 2, 3])
def test_levels_transfers_and_points_match_oracle(base):
    s = _solver(base)
    inf = s.info()
    assert inf["element_k"] == 2 and inf["L"] == base
    for ell in range(1, base + 1):
        om = q3q2.UniformMesh(ell, with_pressure=(ell == base))
        assert inf["n_nodes"][ell] == om.nnode and inf["n_u"][ell] == om.n_u
        assert inf["n_free"][ell] == int(om.free_dofs_mask().sum())
        assert np.array_equal(s.support_points(ell), np.arange(om.nnode))
        assert np.array_equal(s.node_types(ell), np.where(om.dirichlet, 1, 0))
        nh, *_ = s.constraints(ell)
        assert len(nh) == 0
        if ell >= 2:
            ptr, col, w = s.transfer(ell)
            rows = np.repeat(np.arange(om.nnode), np.diff(ptr))
            Pl = sp.csr_matrix((w, (rows, col)), shape=(om.nnode, q3q2.UniformMesh(ell - 1).nnode))
            Po = q3q2.prolongation(q3q2.UniformMesh(ell - 1), om)[0::3, 0::3]
            assert abs(Pl - Po).max() < 1e-15
    assert inf["n_p"] == (2 ** (base + 1) + 1) ** 3
    q = s.leaf_quadrature_points()
    om = q3q2.UniformMesh(base)
    assert q.shape == (om.ncell, 64, 3)
    assert np.abs(q - om.gauss_points()).max() < 1e-15
    s.close()


def test_refused_combinations():
    s = mfgmg.Solver(2)
    assert s.lib.mfgmg_set_element(s.h, 3) == mfgmg.ERR_INVALID
    s.set_element(2)
    s.refine(np.array([[2, 0, 0, 0]], dtype=np.int32), 1)
    with pytest.raises(mfgmg.MFGMGError) as e:
        s.finalize_mesh()
    assert e.value.code == mfgmg.ERR_MESH
    s.close()
    t = mfgmg.Solver(2)
    t.set_element(2)
    t.set_boundary("noflux")
    with pytest.raises(mfgmg.MFGMGError) as e:
        t.finalize_mesh()
    assert e.value.code == mfgmg.ERR_MESH
    t.close()
    u = _solver(2)
    assert u.lib.mfgmg_set_element(u.h, 1) == mfgmg.ERR_STATE
    with pytest.raises(mfgmg.MFGMGError) as e:
        u.local_levels()
    assert e.value.code == mfgmg.ERR_INVALID
    u.close()
