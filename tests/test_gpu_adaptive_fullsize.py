"""Device parity at the full size of the adaptive sinker workload: 32^3 base
cells, the cells with |grad log mu| above its 80th percentile refined by two
levels, 2:1 balanced (503,854 leaf cells, 13.06M velocity dofs), 16 sinkers,
viscosity contrast 1e6.  Here the adaptive-level kernels run at scale: the
4^3 and 2^3 block operators with their face-slot gather, the single-cell
kernels, the node-level CSR transfers.

Against the oracle's cellwise operator on every row: the leaf operator
(FP64, FP32), its accumulating form, and on level 6 (136,830 cells, the
first level with hanging nodes below the leaf) the operator, the inverse
diagonal, the Chebyshev bound, the smoother (FP64, FP32) and the transfers
to and from level 7.  Each error is also bounded row by row against
(|C|^T |K| |C| + Pi_c)|x|, which keeps the rows of the cells with viscosity
1 as tight as those with 1e6."""
import time

import numpy as np
import pytest

from oracle import mesh as omesh, multigrid as omg, operators as ops, rng as orng
from paper_1907_06696_amd import inputs, mfgmg
from tests.parity_cases import abs_bound, rel_err, row_err
from tests.test_gpu_parity import ROW32, ROW64

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(msg, t0):
    print(f"[c3 {time.time() - t0:6.1f}s] {msg}", flush=True)


class _Two:
    """The oracle's level meshes 6 and 7 (enough for their transfer)."""

    def __init__(self, levels):
        self.levels = levels


@pytest.fixture(scope="module")
def c3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    t0 = time.time()
    cfg = inputs.CONFIGS["adaptive32p2"]
    centres = inputs.sinker_centres(cfg["sinkers"], cfg["centre_seed"])
    cells = inputs.refinement_cells(cfg["base_level"], centres, cfg["dr"], cfg["refine_percentile"])
    s = mfgmg.Solver(cfg["base_level"])
    s.refine(cells, cfg["refine_levels"])
    s.finalize_mesh()
    info = s.info()
    L = info["L"]
    qp = s.leaf_quadrature_points().reshape(-1, 3)
    s.set_viscosity(inputs.sinker_mu(qp, centres, cfg["dr"]).reshape(-1, 27))
    torch.cuda.synchronize()
    _t(f"library: L={L} leaf cells {info['n_cells'][L]} n_u {info['n_u'][L]}", t0)
    lev, ijk = omesh.uniform_leaves(cfg["base_level"])
    mask = np.isin(omesh.cell_code(lev, ijk), omesh.cell_code(cells[:, 0], cells[:, 1:]))
    lev, ijk = omesh.refine(lev, ijk, mask, cfg["refine_levels"])
    lev, ijk = omesh.balance(lev, ijk)
    lev, ijk = omesh.morton_sort(lev, ijk)
    assert int(lev.max()) == L
    levels = {}
    for ell in (L - 1, L):
        l2, c2 = omesh.level_cells(lev, ijk, ell)
        levels[ell] = omesh.LevelMesh(l2, c2, L + 1)
    H = _Two(levels)
    leaf = levels[L]
    X = ops.gauss_points_of_cells(leaf).reshape(-1, 3)
    mu_leaf = ops.harmonic_cell_viscosity(inputs.sinker_mu(X, centres, cfg["dr"]).reshape(-1, 27))
    # level L-1: the arithmetic mean of the children (a leaf cell of level < L is its own parent)
    up = levels[L - 1]
    pl = np.minimum(leaf.lev, L - 1)
    pc = leaf.ijk >> (leaf.lev - pl)[:, None]
    ucode = omesh.cell_code(up.lev, up.ijk)
    order = np.argsort(ucode)
    pidx = order[np.searchsorted(ucode[order], omesh.cell_code(pl, pc))]
    mu_up = np.bincount(pidx, weights=mu_leaf, minlength=up.ncell) / np.bincount(pidx, minlength=up.ncell)
    mus = {L: mu_leaf, L - 1: mu_up}
    _t("oracle meshes and viscosities", t0)
    yield dict(s=s, info=info, L=L, H=H, mus=mus, t0=t0)
    s.close()


def _perm(c, ell):
    keys = c["s"].support_points(ell)
    node = np.searchsorted(c["H"].levels[ell].keys, keys)
    assert np.array_equal(c["H"].levels[ell].keys[node], keys)
    return (3 * node[:, None] + np.arange(3)[None, :]).ravel()


def _cell_perm(c, ell):
    cl = c["s"].cells(ell)
    om = c["H"].levels[ell]
    oc = omesh.cell_code(om.lev, om.ijk)
    order = np.argsort(oc)
    return order[np.searchsorted(oc[order], omesh.cell_code(cl[:, 0], cl[:, 1:]))]


def _host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("ell_off", [0, 1])
def test_operator_every_row(c3, ell_off):
    s, L = c3["s"], c3["L"]
    ell = L - ell_off
    mesh, mu = c3["H"].levels[ell], c3["mus"][ell]
    assert np.abs(s.cell_viscosity(ell) - mu[_cell_perm(c3, ell)]).max() <= 1e-13 * mu.max()
    A = ops.CellwiseA(mesh, mu)
    perm = _perm(c3, ell)
    n = mesh.n_u
    for dt, npt, tol, rtol in ((torch.float64, np.float64, 1e-12, ROW64), (torch.float32, np.float32, 1e-5, ROW32)):
        x = inputs.uniform_vector(n, 600 + ell).astype(npt).astype(np.float64)
        ref = A @ x
        bound = abs_bound(mesh, mu, x)
        y = torch.empty(n, dtype=dt, device=DEV)
        s.vmult(ell, torch.tensor(x[perm], dtype=dt, device=DEV), y)
        yh = _host(y)
        e, r = rel_err(yh, ref[perm]), row_err(yh, ref[perm], bound[perm])
        _t(f"level {ell} operator {dt}: rel {e:.2e} row {r:.2e}", c3["t0"])
        assert e <= tol and r <= rtol, (ell, dt, e, r)
        if ell == L:
            free = mesh.free_dofs_mask()
            y0 = inputs.uniform_vector(n, 700).astype(npt).astype(np.float64)
            yy = torch.tensor(y0[perm], dtype=dt, device=DEV)
            s.vmult_add(ell, torch.tensor(x[perm], dtype=dt, device=DEV), yy)
            ref2 = y0 + np.where(free, ref, 0.0)
            b2 = np.abs(y0) + np.where(free, bound, 0.0)
            yh = _host(yy)
            e, r = rel_err(yh, ref2[perm]), row_err(yh, ref2[perm], b2[perm])
            _t(f"leaf vmult_add {dt}: rel {e:.2e} row {r:.2e}", c3["t0"])
            assert e <= tol and r <= rtol, (dt, e, r)


def test_level_below_leaf_diagonal_lambda_smoother(c3):
    s, L = c3["s"], c3["L"]
    ell = L - 1
    mesh, mu = c3["H"].levels[ell], c3["mus"][ell]
    A = ops.CellwiseA(mesh, mu)
    perm = _perm(c3, ell)
    free = mesh.free_dofs_mask()
    diag = A.diagonal()
    minv = np.where(free, 1.0 / diag, 1.0)
    _t(f"level {ell}: oracle diagonal", c3["t0"])
    d = torch.empty(mesh.n_u, dtype=torch.float64, device=DEV)
    s.inverse_diagonal(ell, d)
    assert np.abs(_host(d) - minv[perm]).max() <= 1e-12 * np.abs(minv).max()
    # relative to each entry as well: low-viscosity rows have large inverse diagonals
    assert np.abs(_host(d) - minv[perm]).max() <= 1e-12 * np.abs(minv[perm]).max()
    assert (np.abs(_host(d) - minv[perm]) / np.abs(minv[perm])).max() <= 1e-12
    r0 = orng.dof_vector(mesh, omg.LAMBDA_SEED) * free
    lam = omg.LAMBDA_SAFETY * omg.cg_lanczos_lambda_max(lambda v: A @ v, minv, r0)
    lam_dev = s.smoother_lambda(ell)
    _t(f"level {ell}: lambda oracle {lam:.10g} device {lam_dev:.10g}", c3["t0"])
    assert abs(lam_dev - lam) <= 1e-9 * lam
    for dt, npt, tol in ((torch.float64, np.float64, 1e-12), (torch.float32, np.float32, 1e-5)):
        b = (inputs.uniform_vector(mesh.n_u, 31) * free).astype(npt).astype(np.float64)
        x0 = (inputs.uniform_vector(mesh.n_u, 32) * free).astype(npt).astype(np.float64)
        for zero in (True, False):
            ref = omg.chebyshev(lambda v: A @ v, minv, b, None if zero else x0, lam, x_is_zero=zero)
            x = torch.tensor(x0[perm], dtype=dt, device=DEV)
            s.smooth(ell, torch.tensor(b[perm], dtype=dt, device=DEV), x, x_is_zero=zero)
            e = rel_err(_host(x), ref[perm])
            _t(f"level {ell} smoother {dt} from {'zero' if zero else 'x0'}: rel {e:.2e}", c3["t0"])
            assert e <= tol, (dt, zero, e)


def test_transfers_below_leaf(c3):
    s, L = c3["s"], c3["L"]
    P = ops.prolongation(c3["H"], L)
    pf, pc = _perm(c3, L), _perm(c3, L - 1)
    nf, nc = P.shape
    for dt, tol in ((torch.float64, 1e-14), (torch.float32, 1e-6)):
        xc = inputs.uniform_vector(nc, 811).astype(np.float32 if dt == torch.float32 else np.float64)
        xf = torch.empty(nf, dtype=dt, device=DEV)
        s.prolongate(L, torch.tensor(xc[pc], dtype=dt, device=DEV), xf)
        e1 = rel_err(_host(xf), (P @ xc.astype(np.float64))[pf])
        rf = inputs.uniform_vector(nf, 812).astype(np.float32 if dt == torch.float32 else np.float64)
        rc = torch.empty(nc, dtype=dt, device=DEV)
        s.restrict(L, torch.tensor(rf[pf], dtype=dt, device=DEV), rc)
        e2 = rel_err(_host(rc), (P.T @ rf.astype(np.float64))[pc])
        _t(f"transfers {L - 1}<->{L} {dt}: P rel {e1:.2e}, R rel {e2:.2e}", c3["t0"])
        assert e1 <= tol and e2 <= tol, (dt, e1, e2)
