"""Host sanitizer tier: the mesh layer (csrc/mesh.cpp: octree, 2:1 balance,
level meshes, Q2/Q1 nodes, hanging constraints, transfers) built with g++
-fsanitize=address,undefined (no GPU code involved) and run on the meshes of
the host-layer tests; any sanitizer report fails the run.  Its output is
compared with the oracle's node keys, node kinds, constraints and
prolongation, as the library's own host calls are in test_host_mesh."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mesh as omesh, operators as ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_06696_amd", "csrc")

CASES = [(2, (), 1), (3, (), 1), (2, ((1, 1, 1),), 1), (2, ((0, 1, 0),), 2), (3, ((2, 5, 3), (0, 0, 0)), 2),
         (3, ((7, 7, 7), (3, 4, 0), (0, 7, 2)), 1)]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "mesh_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(CSRC, "mesh.cpp"), os.path.join(CSRC, "q3.cpp"),
           os.path.join(ROOT, "tests", "native", "mesh_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, base, corners, times, mode="dirichlet"):
    cells = [f"{base} {c[0]} {c[1]} {c[2]}" for c in corners]
    inp = f"{base} {times} {len(cells)}\n" + "\n".join(cells) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, mode], input=inp, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout.splitlines()


def _oracle(base, corners, times):
    lev, ijk = omesh.uniform_leaves(base)
    if corners:
        mask = np.zeros(len(lev), bool)
        for c in corners:
            mask |= np.all(ijk == list(c), axis=1)
        lev, ijk = omesh.refine(lev, ijk, mask, times)
        lev, ijk = omesh.balance(lev, ijk)
    return omesh.Hierarchy(lev, ijk)


@pytest.mark.parametrize("base,corners,times", CASES)
def test_mesh_layer_under_sanitizers_matches_oracle(driver, base, corners, times):
    out = _run(driver, base, corners, times)
    H = _oracle(base, corners, times)
    assert out[0] == f"L {H.L}"
    pos = 1
    for ell in range(1, H.L + 1):
        om = H.levels[ell]
        head = out[pos].split()
        assert int(head[3]) == om.ncell and int(head[5]) == om.nnode and int(head[7]) == int(om.hanging.sum())
        keys = np.array(out[pos + 1].split()[1:], dtype=np.int64)
        types = np.array(out[pos + 2].split()[1:], dtype=np.int64)
        order = np.argsort(keys)
        assert np.array_equal(keys[order], om.keys)
        ref_t = np.where(om.dirichlet, 1, np.where(om.hanging, 2, 0))
        assert np.array_equal(types[order], ref_t)
        # hanging rows (masters on the boundary omitted, as in the oracle's C)
        C = sp.lil_matrix((om.nnode, om.nnode))
        for tok in out[pos + 3].split()[1:]:
            a, b, w = tok.split(":")
            C[np.searchsorted(om.keys, keys[int(a)]), np.searchsorted(om.keys, keys[int(b)])] = float(w)
        ref = om.C.tolil()
        ref[np.nonzero(om.free)[0], np.nonzero(om.free)[0]] = 0
        assert abs(C.tocsr() - ref.tocsr()).max() <= 1e-14 if C.nnz or ref.nnz else True
        if ell >= 2:
            Pn = sp.lil_matrix((om.nnode, H.levels[ell - 1].nnode))
            ckeys = coarse_keys
            for tok in out[pos + 4].split()[1:]:
                a, b, w = tok.split(":")
                Pn[np.searchsorted(om.keys, keys[int(a)]), np.searchsorted(H.levels[ell - 1].keys, ckeys[int(b)])] \
                    = float(w)
            Pref = ops.prolongation(H, ell)[::3, ::3]
            assert abs(Pn.tocsr() - Pref).max() <= 1e-14
        coarse_keys = keys
        pos += 5
    ph = out[pos].split()
    assert int(ph[2]) == H.leaf.npnode
    assert np.array_equal(np.sort(np.array(out[pos + 1].split()[1:], dtype=np.int64)), H.leaf.pkeys)
    # local-smoothing levels (built under the sanitizers too): sizes against the oracle's
    from oracle import local_smoothing as ols
    G = ols.LocalSmoothingGMG(H, ops.level_viscosities(H, np.ones(H.leaf.ncell)))
    parts = out[pos + 2].split("|")
    base = int(parts[0].split()[2])
    for part in parts[1:-1]:
        ell, nc, nn, ne, _ = (int(v) for v in part.split())
        assert ell > base and nc == G.T[ell].ncell and nn == G.T[ell].nnode and ne == G.edge[ell][::3].sum()
    # every free leaf node copied once (a uniform leaf mesh has no local levels)
    assert int(parts[-1].split()[1]) == (int(H.leaf.free.sum()) if base < H.L else 0)


@pytest.mark.parametrize("base,corners,times", CASES[2:5])
def test_noflux_mesh_layer_under_sanitizers(driver, base, corners, times):
    """u . n = 0: node kinds, fixed-component masks, hanging rows and the
    node-level transfers (no boundary rows dropped) against the oracle."""
    out = _run(driver, base, corners, times, "noflux")
    lev, ijk = omesh.uniform_leaves(base)
    mask = np.zeros(len(lev), bool)
    for c in corners:
        mask |= np.all(ijk == list(c), axis=1)
    H = omesh.Hierarchy(*omesh.balance(*omesh.refine(lev, ijk, mask, times)), bc="noflux")
    assert out[0] == f"L {H.L}"
    pos = 1
    for ell in range(1, H.L + 1):
        om = H.levels[ell]
        keys = np.array(out[pos + 1].split()[1:], dtype=np.int64)
        order = np.argsort(keys)
        assert np.array_equal(keys[order], om.keys)
        types = np.array(out[pos + 2].split()[1:], dtype=np.int64)[order]
        assert np.array_equal(types, np.where(om.hanging, 2, 0))
        fix = np.array(out[pos + 5].split()[1:], dtype=np.int64)[order]
        assert np.array_equal(fix, (om.fixed * np.array([1, 2, 4])).sum(axis=1))
        if ell >= 2:
            Pn = sp.lil_matrix((om.nnode, H.levels[ell - 1].nnode))
            for tok in out[pos + 4].split()[1:]:
                a, b, w = tok.split(":")
                Pn[np.searchsorted(om.keys, keys[int(a)]), np.searchsorted(H.levels[ell - 1].keys, ckeys[int(b)])] \
                    = float(w)
            assert abs(Pn.tocsr() - ops.prolongation(H, ell, dirichlet=False)[::3, ::3]).max() <= 1e-14
        ckeys = keys
        pos += 6


@pytest.mark.parametrize("base", [1, 2, 3])
def test_q3_levels_under_sanitizers(driver, base):
    """Q3-Q2 lattice levels: node counts and kinds, transfers against the oracle."""
    from oracle import q3q2
    out = _run(driver, base, (), 1, "q3")
    assert out[0] == f"L {base}"
    pos = 1
    for ell in range(1, base + 1):
        om = q3q2.UniformMesh(ell)
        head = out[pos].split()
        assert int(head[5]) == om.nnode and int(head[7]) == 0
        assert np.array_equal(np.array(out[pos + 1].split()[1:], dtype=np.int64), np.arange(om.nnode))
        assert np.array_equal(np.array(out[pos + 2].split()[1:], dtype=np.int64), np.where(om.dirichlet, 1, 0))
        if ell >= 2:
            Pn = sp.lil_matrix((om.nnode, q3q2.UniformMesh(ell - 1).nnode))
            for tok in out[pos + 4].split()[1:]:
                a, b, w = tok.split(":")
                Pn[int(a), int(b)] = float(w)
            Pref = q3q2.prolongation(q3q2.UniformMesh(ell - 1), om)[::3, ::3]
            assert abs(Pn.tocsr() - Pref).max() <= 1e-14
        pos += 5
    assert int(out[pos].split()[2]) == (2 ** (base + 1) + 1) ** 3
