"""Device parity of the learned smoother scaling against the CPU oracle.

* features: <= 1e-6 absolute (FP32 output of FP64 logarithms);
* MLP forward / backward: <= 1e-4 relative against the FP64 numpy oracle on
  the same FP32-rounded weights and inputs; Adam step <= 1e-6;
* fit objective J and its adjoint gradient (FP64 on both sides, lambda
  re-estimated identically from the same SplitMix64 vector): J <= 1e-10
  relative, gradient <= 1e-7 relative in the 2-norm (FP32 output);
* fitted targets after a few Adam steps: J histories <= 1e-8 relative;
* V-cycle with an installed scaling: <= 1e-11 relative (FP64);
* training decreases the loss; the guard reports both contraction factors.
The targets themselves are defined only by the algorithm (parity unpinned
beyond agreement with the oracle's run of the same algorithm)."""
import numpy as np
import pytest

from oracle import learned as ol, multigrid as omg
from paper_1907_06696_amd import inputs, mfgmg
from tests.parity_cases import Case, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"

CASES = {
    "uniform3": dict(base=3, dr=1e4, sinkers=5, seed=2),
    "adaptive2+1": dict(base=2, corners=((1, 1, 1), (0, 0, 1)), times=1, dr=1e3, sinkers=3, seed=4),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = Case(**CASES[request.param])
    print(f"\n[learned case {request.param}] L={c.L} cells={c.info['n_cells'][c.L]}", flush=True)
    c.s.set_viscosity(c.mu_qp_lib)
    c.gmg = omg.GMG(c.H, c.mus)
    yield c
    c.close()


def test_features(case):
    for ell in range(1, case.L + 1):
        f = case.s.features(ell).cpu().numpy()
        ref = ol.features(case.H, case.mus, ell)[case.cell_perm(ell)]
        assert np.abs(f - ref).max() <= 1e-6, ell


def test_mlp_forward_backward_adam():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rg = np.random.default_rng(0)
    w = (ol.init_params(3) * 0.5).astype(np.float32)
    x = rg.normal(0, 0.7, (1000, 27)).astype(np.float32)
    wd, xd = torch.tensor(w, device=DEV), torch.tensor(x, device=DEV)
    y, cache = mfgmg.mlp_forward(wd, xd)
    yr, cr = ol.mlp_forward(w.astype(np.float64), x.astype(np.float64))
    assert rel_err(y.cpu().numpy(), yr) <= 1e-4
    dy = rg.normal(0, 1, (1000, 3)).astype(np.float32)
    dw = mfgmg.mlp_backward(wd, xd, cache, torch.tensor(dy, device=DEV))
    gr = ol.mlp_backward(w.astype(np.float64), cr, dy.astype(np.float64))
    assert rel_err(dw.cpu().numpy(), gr) <= 1e-4
    m = torch.zeros_like(wd)
    v = torch.zeros_like(wd)
    w2 = wd.clone()
    mfgmg.mlp_adam(w2, dw, m, v, 1, 1e-3)
    ref, _, _ = ol.adam_step(w.astype(np.float64), dw.cpu().numpy().astype(np.float64), np.zeros(6147),
                             np.zeros(6147), 1, 1e-3)
    assert np.abs(w2.cpu().numpy() - ref).max() <= 1e-6


def test_fit_objective_and_gradient(case):
    for ell in range(2, case.L + 1):
        m = case.H.levels[ell]
        perm = case.cell_perm(ell)
        rg = np.random.default_rng(ell)
        y_or = rg.uniform(-0.5, 0.5, (m.ncell, 3)).astype(np.float32).astype(np.float64)
        J, lam, g = case.s.fit_objective(ell, torch.tensor(y_or[perm].astype(np.float32), device=DEV))
        Jr, gr = ol.objective(case.gmg, ell, y_or)
        assert abs(J - Jr) <= 1e-10 * abs(Jr), (ell, J, Jr)
        assert rel_err(g.cpu().numpy().astype(np.float64), gr[perm]) <= 1e-6, ell


def test_fit_targets_matches_oracle(case):
    ell = case.L
    y, hist = case.s.fit_targets(ell, steps=4, lr=0.05)
    yr, hr = ol.fit_targets(case.gmg, ell, steps=4, lr=0.05)
    assert np.allclose(hist, hr, rtol=1e-8, atol=0), (hist, hr)
    assert hist[-1] < hist[0]
    assert rel_err(y.cpu().numpy().astype(np.float64), yr[case.cell_perm(ell)]) <= 1e-5


def test_scaled_vcycle_parity(case):
    L = case.L
    rg = np.random.default_rng(9)
    scal, y_by_level = {}, {}
    for ell in range(2, L + 1):
        m = case.H.levels[ell]
        y = rg.uniform(-0.4, 0.4, (m.ncell, 3)).astype(np.float32).astype(np.float64)
        y_by_level[ell] = y
        scal[ell] = ol.dof_scaling(m, y)
        case.s.set_scaling(ell, torch.tensor(y[case.cell_perm(ell)].astype(np.float32), device=DEV))
    G = omg.GMG(case.H, case.mus, scaling=scal)
    n = case.info["n_u"][L]
    perm = case.dof_perm(L)
    b = inputs.uniform_vector(n, 61) * G.free[L]
    ref = G.vcycle(b)[perm]
    x = torch.empty(n, dtype=torch.float64, device=DEV)
    case.s.use_scaling(True)
    case.s.vcycle(torch.tensor(b[perm], device=DEV), x)
    torch.cuda.synchronize()
    case.s.use_scaling(False)
    assert rel_err(x.cpu().numpy(), ref) <= 1e-11
    for ell in range(2, L + 1):
        case.s.set_scaling(ell, None)


def test_training_and_guard(case):
    L = case.L
    feats = case.s.features(L)
    y, _ = case.s.fit_targets(L, steps=3, lr=0.05)
    w = torch.tensor(ol.init_params(0).astype(np.float32), device=DEV)
    hist = mfgmg.mlp_train(w, feats, y.contiguous(), epochs=30, batch=64, lr=3e-3, seed=1)
    assert hist[-1] < hist[0]
    for guard in ("fp64", "fp32"):
        used, fac = case.s.apply_mlp(w, guard=guard)
        assert fac[0] > 0 and fac[1] > 0
        assert used == (fac[1] < 0.95 * fac[0]), (guard, fac)
    used, fac = case.s.apply_mlp(w, guard=None)
    assert used
    for ell in range(2, L + 1):
        case.s.set_scaling(ell, None)
