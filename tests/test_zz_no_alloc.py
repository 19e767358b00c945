"""The allocation-free operator entry point (mfgmg_vmult_uniform_noalloc)
against the existing one (mfgmg_vmult on the leaf of a uniform context with
the same cell viscosities): identical results, bit for bit (the same brick
and halo kernels on the same inputs), on two calls in a row, the second on a
smaller mesh (64^3, then 32^3: the second call finds the first call's slot
values in the shared work array, so its zero pad must be cleared), in FP64
and FP32.  Sizes beyond the array's limit are rejected."""
import ctypes as C

import numpy as np
import pytest

from paper_1907_06696_amd import inputs, mfgmg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_noalloc_operator_matches_vmult_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for base in (6, 5):                       # 64^3, then the smaller 32^3
        n = 1 << base
        s = mfgmg.Solver(base)
        s.finalize_mesh()
        qp = s.leaf_quadrature_points().reshape(-1, 3)
        c = inputs.sinker_centres(8, 2)
        s.set_viscosity(inputs.sinker_mu(qp, c, 1e4).reshape(-1, 27))
        mu = s.cell_viscosity(base)             # uniform leaf: cell i + n (j + n k)
        nu = s.info()["n_u"][base]
        for dt in (torch.float64, torch.float32):
            print(f"[noalloc] n={n} {dt}", flush=True)
            mu_d = torch.tensor(mu, dtype=torch.float64, device="cuda").to(dt)
            x = torch.tensor(inputs.uniform_vector(nu, 90 + base), dtype=dt, device="cuda")
            ref = torch.empty_like(x)
            s.vmult(base, x, ref)
            y = torch.full_like(x, float("nan"))
            mfgmg.vmult_uniform_noalloc(n, mu_d, x, y)
            torch.cuda.synchronize()
            assert torch.equal(y, ref), (n, dt, float((y - ref).abs().max()))
        s.close()
    lib = mfgmg.load()
    assert lib.mfgmg_vmult_uniform_noalloc(128, mfgmg.FP64, C.c_void_p(16), C.c_void_p(32), C.c_void_p(64),
                                           None) == mfgmg.ERR_INVALID
    assert b"scratch limit" in lib.mfgmg_last_error(None)
