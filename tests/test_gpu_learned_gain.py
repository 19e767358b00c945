"""What the trained network gains over the plain smoother, on a held-out set
declared in advance: the first eight fields of the learned workload's
evaluation set (seeds 20000..20007; 64^3 cells, 4-32 sinkers, viscosity
contrast 1e2-1e6), every one of them.

The weights in ``paper_1907_06696_amd/data/mlp_sinker32.npz`` were trained on
the GPU by the library's own kernels (256 seeded sinker fields at 32^3 cells,
targets fitted by the adjoint V-cycle objective on every smoothed level).
Per field, the FP64 FGMRES solve to 1e-8 with the FP32 V-cycle is run plain
and with the network's scaling behind its guard (V-cycle factors estimated
with the FP64 V-cycle, the linear map the FP32 one rounds; kept only 5%
below plain).  Checked: every solve
reaches 1e-8; the guard keeps the scaling exactly when its factor is 5% below
plain; where it is kept the solve takes no more FGMRES iterations than plain.
Printed: per-field counts and seconds, and the medians with the guard's setup
time counted."""
import os

import numpy as np
import pytest

from paper_1907_06696_amd import learn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(learn.__file__), "data", "mlp_sinker32.npz")
SEEDS = tuple(range(20000, 20008))


def test_trained_network_vs_plain_smoother():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = torch.tensor(np.load(WEIGHTS)["weights"], device="cuda")
    rows = learn.evaluate(w, base=6, seeds=SEEDS, max_iter=2000, log=lambda m: print(m, flush=True))
    assert len(rows) == len(SEEDS)
    for r in rows:
        assert r["plain_converged"] and r["plain_res"] <= 1e-8, r
        assert r["learned_res"] <= 1e-8, r
        assert r["learned_used"] == (r["factor_learned"] < 0.95 * r["factor_plain"]), r
        if r["learned_used"]:
            assert r["learned_its"] <= r["plain_its"], r
    print("summary:", learn.summarize(rows), flush=True)
