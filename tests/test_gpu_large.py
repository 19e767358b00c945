"""The largest uniform level of the workloads (128^3 cells, 50,923,779 velocity
dofs), FP64 and FP32 operator against the oracle on sampled rows.

The full 128^3 product is beyond what the oracle finishes in seconds, so rows
are checked one by one: for a sampled lattice node the oracle sums
mu_K h K_hat over the cells around it (the cell matrix of the strain-rate
form, Sec. 2.1; K_e = mu_K h K_hat on a cube of side h) applied to the input
restricted to free nodes, and a Dirichlet node's row is the identity.  The
samples cover random nodes and the nodes where the operator kernel's
bricks meet (faces, edges and corners of the 16x16x8 and 16x8x8 node boxes
of the FP32 and FP64 bricks) and the domain boundary.  Viscosity: a smooth
positive field with contrast ~e^6, harmonic-averaged per cell (Sec. 2.3)."""
import numpy as np
import pytest

from oracle import fe, operators as ops
from paper_1907_06696_amd import inputs, mfgmg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
LEVEL = 7


def mu_field(p):
    p = np.asarray(p, dtype=np.float64).reshape(-1, 3)
    return np.exp(3.0 * np.sin(2 * np.pi * p[:, 0]) * np.cos(2 * np.pi * p[:, 1]) * np.sin(2 * np.pi * p[:, 2]))


def sample_nodes(m, rng):
    pts = [rng.integers(0, m, size=(200, 3))]
    for bx, by, bz in ((16, 16, 8), (16, 8, 8)):             # brick node boxes (FP32, FP64)
        for _ in range(40):
            q = rng.integers(1, m - 1, size=3)
            q[:2] = (q[:2] // np.array([bx, by])) * np.array([bx, by])
            q[2] = (q[2] // bz) * bz
            pts.append(np.maximum(q, 1)[None, :])
    pts.append(np.array([[1, 1, 1], [m - 2, m - 2, m - 2], [0, 5, 7], [m - 1, 3, 3], [128, 128, 128],
                         [16, 16, 8], [16, 8, 8], [32, 16, 16], [17, 16, 8]]))
    return np.unique(np.concatenate(pts), axis=0)


def oracle_rows(nodes, x, n, khat):
    """y at the sampled nodes (3 components each), FP64."""
    m = 2 * n + 1
    h = 1.0 / n
    gp, gw = fe.gauss_points_3d(3)
    out = np.zeros((len(nodes), 3))
    for r, (X, Y, Z) in enumerate(nodes):
        node = X + m * (Y + m * Z)
        if min(X, Y, Z) == 0 or max(X, Y, Z) == m - 1:
            out[r] = x[3 * node:3 * node + 3]
            continue
        cx = [X // 2] if X % 2 else [X // 2 - 1, X // 2]
        cy = [Y // 2] if Y % 2 else [Y // 2 - 1, Y // 2]
        cz = [Z // 2] if Z % 2 else [Z // 2 - 1, Z // 2]
        for i in cx:
            for j in cy:
                for k in cz:
                    pts = (np.array([i, j, k]) + gp) * h
                    muc = ops.harmonic_cell_viscosity(mu_field(pts).reshape(1, 27))[0]
                    a = (X - 2 * i) + 3 * (Y - 2 * j) + 9 * (Z - 2 * k)
                    xl = np.zeros(81)
                    for b in range(27):
                        bx_, by_, bz_ = 2 * i + b % 3, 2 * j + (b // 3) % 3, 2 * k + b // 9
                        if min(bx_, by_, bz_) == 0 or max(bx_, by_, bz_) == m - 1:
                            continue
                        nb = bx_ + m * (by_ + m * bz_)
                        xl[3 * b:3 * b + 3] = x[3 * nb:3 * nb + 3]
                    out[r] += muc * h * (khat[3 * a:3 * a + 3] @ xl)
    return out


def test_vmult_128_sampled_rows():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 1 << LEVEL
    m = 2 * n + 1
    s = mfgmg.Solver(LEVEL)
    s.finalize_mesh()
    info = s.info()
    assert info["uniform"][LEVEL] and info["n_u"][LEVEL] == 3 * m ** 3
    qp = s.leaf_quadrature_points().reshape(-1, 3)
    s.set_viscosity(mu_field(qp).reshape(-1, 27))
    del qp
    keys = s.support_points(LEVEL)
    nn = 3 * m ** 3
    rng = np.random.default_rng(5)
    nodes = sample_nodes(m, rng)
    idx = nodes[:, 0] + m * (nodes[:, 1] + m * nodes[:, 2])
    assert np.array_equal(keys[idx], idx)            # lexicographic lattice numbering on uniform levels
    x = inputs.uniform_vector(nn, 77)
    y64 = torch.empty(nn, dtype=torch.float64, device=DEV)
    s.vmult(LEVEL, torch.tensor(x, device=DEV), y64)
    x32 = x.astype(np.float32)
    y32 = torch.empty(nn, dtype=torch.float32, device=DEV)
    s.vmult(LEVEL, torch.tensor(x32, device=DEV), y32)
    torch.cuda.synchronize()
    sel = (3 * idx[:, None] + np.arange(3)[None, :]).ravel()
    g64 = y64[torch.tensor(sel, device=DEV)].cpu().numpy().reshape(-1, 3)
    g32 = y32[torch.tensor(sel, device=DEV)].cpu().numpy().astype(np.float64).reshape(-1, 3)
    s.close()
    khat, _, _ = fe.element_matrices()
    ref64 = oracle_rows(nodes, x, n, khat)
    ref32 = oracle_rows(nodes, x32.astype(np.float64), n, khat)
    scale = np.abs(ref64).max()
    e64 = np.abs(g64 - ref64).max() / scale
    e32 = np.abs(g32 - ref32).max() / scale
    print(f"\n  128^3 sampled rows ({len(nodes)} nodes): fp64 {e64:.2e}, fp32 {e32:.2e}", flush=True)
    assert e64 <= 1e-12
    assert e32 <= 1e-5
