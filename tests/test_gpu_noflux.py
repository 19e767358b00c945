"""Device Stokes solves under the no-normal-flux condition u . n = 0 (Sec. 2,
eq. stokes and the variants after it) against the CPU oracle.

The sinker problems of the parity suite with u . n = 0 instead of u = 0, on
a uniform mesh and on an adaptive mesh with hanging nodes on the boundary:
the FP64 relative residual of the device solution, recomputed by the
oracle's assembled block system, is <= 1e-8 (1.5e-8 after the oracle's own
rounding) for the FP64 and the FP32 V-cycle, and the solution matches the
oracle's sparse direct solve.  Fixed components of the returned velocity are
exactly zero, tangential ones on the boundary are not.  The local-smoothing
calls, built for u = 0, are refused."""
import numpy as np
import pytest

from paper_1907_06696_amd import inputs, mfgmg
from tests.parity_cases import Case
from tests.test_gpu_solve import _solve_and_check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _velocity(case):
    """Solve once more (FP32 V-cycle) and return the velocity per node [n, 3]
    (library order; hanging values interpolated from their masters)."""
    L = case.L
    nu, npp = case.info["n_u"][L], case.info["n_p"]
    rhs = torch.empty(nu, dtype=torch.float64, device=DEV)
    case.s.assemble_rhs(case.f_qp_lib, rhs)
    u = torch.empty(nu, dtype=torch.float64, device=DEV)
    p = torch.empty(npp, dtype=torch.float64, device=DEV)
    case.s.solve_stokes(rhs, u, p, vcycle_prec="fp32")
    torch.cuda.synchronize()
    return u.cpu().numpy().reshape(-1, 3)


@pytest.mark.parametrize("name,kw", [
    ("uniform8", dict(base=3, sinkers=4, dr=1e2, seed=42)),
    ("adaptive3+1", dict(base=3, corners=((0, 5, 3), (7, 0, 0), (4, 4, 4)), times=1, sinkers=4, dr=1e3, seed=7)),
])
def test_solve_noflux_matches_oracle(name, kw):
    print(f"\n[noflux solve] {name}", flush=True)
    c = Case(bc="noflux", **kw)
    assert c.info["boundary"] == "noflux" and not any(c.info["uniform"])
    c.s.set_viscosity(c.mu_qp_lib)
    _solve_and_check(c)
    u = _velocity(c)
    # the components fixed by u . n = 0 (the oracle's mask, by node key), hanging
    # boundary nodes included, are exactly zero; tangential ones are not
    fixed = c.H.leaf.fixed[c.node_perm(c.L)]
    assert np.abs(u[fixed]).max() == 0.0
    tangential = ~fixed & np.any(fixed, axis=1)[:, None]
    assert np.abs(u[tangential]).max() > 0
    c.close()


def test_local_smoothing_refused_under_noflux():
    c = Case(base=2, corners=((0, 1, 0),), times=1, sinkers=2, dr=1e2, seed=3, build_oracle=False, bc="noflux")
    c.s.set_viscosity(c.mu_qp_lib)
    n = c.info["n_u"][c.L]
    b = torch.tensor(inputs.uniform_vector(n, 1), device=DEV)
    x = torch.empty_like(b)
    with pytest.raises(mfgmg.MFGMGError) as e:
        c.s.vcycle_local(b, x)
    assert e.value.code == mfgmg.ERR_INVALID
    rhs = torch.zeros(n, dtype=torch.float64, device=DEV)
    u = torch.empty_like(rhs)
    p = torch.empty(c.info["n_p"], dtype=torch.float64, device=DEV)
    with pytest.raises(mfgmg.MFGMGError) as e:
        c.s.solve_stokes(rhs, u, p, hierarchy="local")
    assert e.value.code == mfgmg.ERR_INVALID
    c.close()
