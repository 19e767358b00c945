"""Host layer of the C-ABI library (no GPU needed): the library loads, exports
every symbol the header declares, and its meshes, node sets, constraints and
transfers agree with the oracle's, matched by canonical node keys."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mesh as omesh, operators as ops
from paper_1907_06696_amd import mfgmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "mfgmg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mfgmg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = mfgmg.load()
    decl = _declared_functions()
    assert sorted(mfgmg.EXPORTS) == decl
    syms = os.popen(f"nm -D --defined-only {mfgmg.LIB_PATH}").read()
    for name in decl:
        assert re.search(rf"\bT {name}\b", syms), name
        assert hasattr(lib, name)


def _pair(base, corners=(), times=1, bc="dirichlet"):
    """(library solver, oracle hierarchy) for the same mesh."""
    s = mfgmg.Solver(base)
    if bc != "dirichlet":
        s.set_boundary(bc)
    lev, ijk = omesh.uniform_leaves(base)
    if corners:
        cells = np.array([[base, *c] for c in corners], dtype=np.int32)
        s.refine(cells, times)
        mask = np.zeros(len(lev), bool)
        for c in corners:
            mask |= np.all(ijk == list(c), axis=1)
        lev, ijk = omesh.refine(lev, ijk, mask, times)
        lev, ijk = omesh.balance(lev, ijk)
    s.finalize_mesh()
    return s, omesh.Hierarchy(lev, ijk, bc=bc)


CASES = [(2, (), 1), (3, (), 1), (2, ((1, 1, 1),), 1), (2, ((0, 1, 0),), 2), (3, ((2, 5, 3), (0, 0, 0)), 2)]
BCS = ["dirichlet", "noflux"]


def _constraint_dict(keys, node, ptr, master, w):
    out = {}
    for i, n in enumerate(node):
        out[int(keys[n])] = {int(keys[m]): round(float(ww), 14) for m, ww in zip(master[ptr[i]:ptr[i + 1]],
                                                                                 w[ptr[i]:ptr[i + 1]])}
    return out


def _oracle_constraints(keys, hanging, Cmat):
    out = {}
    for i in np.nonzero(hanging)[0]:
        row = Cmat.getrow(i)
        out[int(keys[i])] = {int(keys[m]): round(float(v), 14) for m, v in zip(row.indices, row.data)}
    return out


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("base,corners,times", CASES)
def test_mesh_nodes_constraints_match_oracle(base, corners, times, bc):
    s, H = _pair(base, corners, times, bc)
    inf = s.info()
    assert inf["L"] == H.L and inf["U"] == H.U and inf["boundary"] == bc
    if bc == "noflux":
        assert not any(inf["uniform"])
    for ell in range(1, H.L + 1):
        om = H.levels[ell]
        keys = s.support_points(ell)
        assert len(keys) == om.nnode == inf["n_nodes"][ell]
        assert np.array_equal(np.sort(keys), om.keys)
        # cells
        cl = s.cells(ell)
        ocode = np.sort(omesh.cell_code(om.lev, om.ijk))
        assert np.array_equal(np.sort(omesh.cell_code(cl[:, 0], cl[:, 1:])), ocode)
        # node kinds
        t = s.node_types(ell)
        pos = np.searchsorted(om.keys, keys)
        ot = np.where(om.dirichlet, 1, np.where(om.hanging, 2, 0))[pos]
        assert np.array_equal(t, ot)
        assert inf["n_free"][ell] == int(om.free_dofs_mask().sum())
        # constrained components per node (bit c: dof 3 node + c)
        cm = s.node_types(ell, 2)
        ocm = ((~om.free_dofs_mask()).reshape(-1, 3) * np.array([1, 2, 4])).sum(axis=1)[pos]
        assert np.array_equal(cm, ocm)
        # hanging constraints
        cs = s.constraints(ell)
        assert _constraint_dict(keys, *cs) == _oracle_constraints(om.keys, om.hanging, om.C)
    # pressure nodes and constraints on the leaf
    lf = H.leaf
    pk = s.support_points(H.L, 1)
    assert np.array_equal(np.sort(pk), lf.pkeys)
    pt = s.node_types(H.L, 1)
    assert np.array_equal(pt, np.where(lf.phanging, 2, 0)[np.searchsorted(lf.pkeys, pk)])
    assert _constraint_dict(pk, *s.constraints(H.L, 1)) == _oracle_constraints(lf.pkeys, lf.phanging, lf.Cp)
    s.close()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("base,corners,times", CASES)
def test_transfers_match_oracle(base, corners, times, bc):
    s, H = _pair(base, corners, times, bc)
    for ell in range(2, H.L + 1):
        ptr, col, w = s.transfer(ell)
        fk, ck = s.support_points(ell), s.support_points(ell - 1)
        f, c = H.levels[ell], H.levels[ell - 1]
        rows = np.repeat(np.arange(len(fk)), np.diff(ptr))
        # map library numbering to the oracle's (sorted keys)
        Pl = sp.csr_matrix((w, (np.searchsorted(f.keys, fk)[rows], np.searchsorted(c.keys, ck)[col])),
                           shape=(f.nnode, c.nnode))
        # node level: with u = 0 the component-0 block of the oracle's P; with
        # u . n = 0 the per-dof masks are applied on the device, the node-level
        # CSR is the transfer without boundary condition
        Po = ops.prolongation(H, ell, dirichlet=(bc == "dirichlet"))[0::3, 0::3]
        assert abs(Pl - Po).max() < 1e-15
    s.close()


def test_quadrature_points_and_rejects():
    s, H = _pair(2, ((1, 1, 1),), 1)
    q = s.leaf_quadrature_points()
    cl = s.cells(H.L)
    lf = H.leaf
    oq = ops.gauss_points_of_cells(lf)
    order = np.argsort(omesh.cell_code(lf.lev, lf.ijk))
    lib_codes = omesh.cell_code(cl[:, 0], cl[:, 1:])
    idx = order[np.searchsorted(omesh.cell_code(lf.lev, lf.ijk)[order], lib_codes)]
    assert np.abs(q - oq[idx]).max() < 1e-15
    # failure paths: bad level, refine after finalize, vmult before set_viscosity
    with pytest.raises(mfgmg.MFGMGError) as e:
        s.cells(H.L + 1)
    assert e.value.code == mfgmg.ERR_INVALID
    with pytest.raises(mfgmg.MFGMGError) as e:
        s.refine(np.array([[2, 0, 0, 0]]), 1)
    assert e.value.code == mfgmg.ERR_STATE
    s.close()
    t = mfgmg.Solver(2)
    with pytest.raises(mfgmg.MFGMGError) as e:
        t.refine(np.array([[3, 0, 0, 0]]), 1)      # not an active cell
    assert e.value.code == mfgmg.ERR_INVALID
    with pytest.raises(mfgmg.MFGMGError):
        mfgmg.Solver(0)
    t.close()


def test_boundary_condition_calls():
    """u . n = 0 is chosen before finalize (ERR_STATE after, ERR_INVALID for an
    unknown value); its levels are all general; the local-smoothing hierarchy,
    built for u = 0, is refused."""
    s = mfgmg.Solver(2)
    assert s.lib.mfgmg_set_boundary(s.h, 7) == mfgmg.ERR_INVALID
    with pytest.raises(ValueError):
        s.set_boundary("slip")
    s.set_boundary("noflux")
    s.set_boundary("dirichlet")
    s.set_boundary("noflux")
    s.refine(np.array([[2, 0, 1, 0]], dtype=np.int32), 1)
    s.finalize_mesh()
    inf = s.info()
    assert inf["boundary"] == "noflux" and not any(inf["uniform"][1:])
    assert s.lib.mfgmg_set_boundary(s.h, mfgmg.BC_DIRICHLET) == mfgmg.ERR_STATE
    with pytest.raises(mfgmg.MFGMGError) as e:
        s.local_levels()
    assert e.value.code == mfgmg.ERR_INVALID
    s.close()
    d = mfgmg.Solver(2)
    d.finalize_mesh()
    assert d.info()["boundary"] == "dirichlet" and all(d.info()["uniform"][1:])
    d.close()
