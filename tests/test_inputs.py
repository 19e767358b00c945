"""Checks of the sinker workload generator (Sec. 3.2 formula)."""
import numpy as np

from paper_1907_06696_amd import inputs


def test_sinker_field_closed_form():
    cen = inputs.sinker_centres(6, 11)
    assert np.all((cen >= 0.1) & (cen <= 0.9))
    p = np.random.default_rng(0).uniform(0, 1, (2000, 3))
    X = inputs.sinker_chi(p, cen)
    assert np.all((X >= 0) & (X <= 1))
    mu = inputs.sinker_mu(p, cen, 1e4)
    assert np.all((mu >= 1) & (mu <= 1e4))
    # at a centre (inside the sinker of diameter omega) X = 0, mu = mu_max
    assert np.allclose(inputs.sinker_chi(cen, cen), 0.0)
    assert np.allclose(inputs.sinker_mu(cen, cen, 1e4), 1e4)
    f = inputs.sinker_force(p, cen)
    assert np.all((f[:, 2] >= -10) & (f[:, 2] <= 0)) and np.all(f[:, :2] == 0)
    # one sinker: X depends on the distance only, 1 - exp(-delta (r - omega/2)^2)
    c1 = np.array([[0.5, 0.5, 0.5]])
    q = np.array([[0.5 + 0.2, 0.5, 0.5]])
    assert np.isclose(inputs.sinker_chi(q, c1)[0], 1 - np.exp(-200 * (0.2 - 0.05) ** 2))


def test_grad_log_mu_matches_finite_differences():
    cen = inputs.sinker_centres(5, 3)
    p = np.random.default_rng(1).uniform(0.05, 0.95, (200, 3))
    g = inputs.grad_log_mu(p, cen, 1e3)
    e = 1e-6
    fd = np.zeros((200, 3))
    for d in range(3):
        dp = np.zeros(3)
        dp[d] = e
        fd[:, d] = (np.log(inputs.sinker_mu(p + dp, cen, 1e3)) - np.log(inputs.sinker_mu(p - dp, cen, 1e3))) / (2 * e)
    assert np.allclose(g, np.linalg.norm(fd, axis=1), rtol=1e-5, atol=1e-6)


def test_refinement_cells_deterministic_fraction():
    cen = inputs.sinker_centres(4, 1)
    cells = inputs.refinement_cells(3, cen, 1e2, 80.0)
    assert cells.shape[1] == 4 and np.all(cells[:, 0] == 3)
    assert len(cells) <= round(512 * 0.2)
    assert np.array_equal(cells, inputs.refinement_cells(3, cen, 1e2, 80.0))


def test_trained_weights_file():
    import os
    from paper_1907_06696_amd import learn
    path = os.path.join(os.path.dirname(learn.__file__), "data", "mlp_sinker32.npz")
    d = np.load(path)
    w = d["weights"]
    assert w.dtype == np.float32 and w.shape == (6147,) and np.all(np.isfinite(w))
    assert not np.array_equal(w, learn.init_weights(0))       # trained, not the initial draw
    assert d["loss"][-1] < d["loss"][0]


def test_learned_field_ranges():
    for seed in (10000, 10255, 20000, 20031):
        c, dr = inputs.learned_field(seed)
        assert 4 <= len(c) <= 32 and 1e2 <= dr <= 1e6
        assert np.all((c >= 0.1) & (c <= 0.9))
