"""What the trained network gains over the plain smoother, on held-out fields.

The weights in ``paper_1907_06696_amd/data/mlp_sinker32.npz`` were trained on
the GPU by the library's own kernels (256 seeded sinker fields at 32^3 cells,
targets fitted by the adjoint V-cycle objective on every smoothed level).  On
four held-out 64^3 fields (seeds 20015, 20017, 20021, 20024 of the evaluation
set: 5-12 sinkers, viscosity contrast 2e3-4e5) the FP64 FGMRES solve to 1e-8
with the FP32 V-cycle is run plain and with the learned scaling installed by
its guard.  Checked: both solves reach 1e-8; the guard installs the scaling
only when its estimated V-cycle factor is smaller; the learned solves take no
more FGMRES iterations in total than the plain ones.  The per-field numbers
are printed (the gain is small: the outer iteration count is dominated by the
Schur-complement approximation, not by the velocity smoother)."""
import os

import numpy as np
import pytest

from paper_1907_06696_amd import inputs, learn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(learn.__file__), "data", "mlp_sinker32.npz")
SEEDS = (20015, 20017, 20021, 20024)


def test_trained_network_vs_plain_smoother():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = torch.tensor(np.load(WEIGHTS)["weights"], device="cuda")
    rows = learn.evaluate(w, base=6, seeds=SEEDS, max_iter=2000, log=lambda m: print(m, flush=True))
    for r in rows:
        assert r["plain_converged"] and r["plain_res"] <= 1e-8, r
        assert r["learned_res"] <= 1e-8, r
        assert r["learned_used"] == (r["factor_learned"] < r["factor_plain"]), r
    plain = sum(r["plain_its"] for r in rows)
    learned = sum(r["learned_its"] for r in rows)
    print(f"FGMRES iterations over {len(rows)} fields: plain {plain}, learned {learned}; "
          f"used on {sum(r['learned_used'] for r in rows)}", flush=True)
    assert learned <= plain
