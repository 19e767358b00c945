"""Seeded synthetic workloads: the sinker benchmark and random vectors.

This module holds the *problem* definitions only (viscosity field, body
force, refinement flags of the adaptive workloads, random test vectors).  It
contains none of the solver's arithmetic (no basis, quadrature, operator or
smoother) and imports nothing but numpy and the standard library, so that
both the device library's callers and the CPU oracle can draw the same inputs
from it.

Sinker benchmark (paper, Sec. 3.2, after May et al. and Rudi et al.):
    X(x)  = prod_i [1 - exp(-delta max(0, |c_i - x| - omega/2)^2)],
    mu(x) = X mu_min + (1 - X) mu_max,
    f(x)  = (0, 0, beta (X - 1)),
with delta = 200, omega = 0.1, beta = 10 and homogeneous Dirichlet velocity
on the unit cube.  The paper scales mu_min = DR^-1/2, mu_max = DR^1/2; these
workloads use mu_min = 1, mu_max = DR, a global factor that leaves pressure,
relative residuals and iteration counts unchanged (velocity scales by 1/c).
Sinker centres are uniform in [0.1, 0.9]^3 from numpy's default generator.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

DELTA = 200.0
OMEGA = 0.1
BETA = 10.0


def sinker_centres(n, seed):
    return np.random.default_rng(seed).uniform(0.1, 0.9, size=(n, 3))


def _dist_terms(points, centres):
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    diff = p[:, None, :] - centres[None, :, :]                  # [np, n, 3]
    r = np.sqrt((diff ** 2).sum(axis=2))
    s = np.maximum(0.0, r - OMEGA / 2.0)
    e = np.exp(-DELTA * s * s)
    return p, diff, r, s, e


def _chi_chunk(p, centres):
    """X at the points p [m, 3]: the product over the sinkers in their order,
    each factor 1 - exp(-delta max(0, |x - c_i| - omega/2)^2)."""
    X = np.ones(len(p))
    for c in centres:
        d2 = (p[:, 0] - c[0]) ** 2 + (p[:, 1] - c[1]) ** 2 + (p[:, 2] - c[2]) ** 2
        s = np.maximum(0.0, np.sqrt(d2) - OMEGA / 2.0)
        X *= 1.0 - np.exp(-DELTA * s * s)
    return X


def _threads():
    return max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))


def sinker_chi(points, centres, chunk=1 << 18):
    """X at the points, evaluated in chunks on a thread pool (numpy releases
    the interpreter lock inside its array loops)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(p))
    starts = range(0, len(p), chunk)

    def work(a):
        out[a:a + chunk] = _chi_chunk(p[a:a + chunk], centres)

    if len(p) <= chunk:
        work(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, starts))
    return out


def sinker_mu(points, centres, dr):
    X = sinker_chi(points, centres)
    return X * 1.0 + (1.0 - X) * float(dr)


def sinker_force(points, centres):
    X = sinker_chi(points, centres)
    f = np.zeros((len(X), 3))
    f[:, 2] = BETA * (X - 1.0)
    return f


def grad_log_mu(points, centres, dr, chunk=1 << 18):
    """|grad log mu| at points, analytically (product rule on X)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty(len(p))
    for a in range(0, len(p), chunk):
        q, diff, r, s, e = _dist_terms(p[a:a + chunk], centres)
        one_m_e = 1.0 - e
        X = np.prod(one_m_e, axis=1)
        # dX/dx = sum_i (prod_{j != i} (1 - e_j)) * d(1 - e_i)/dx
        # d(1 - e_i)/dx = e_i * 2 delta s_i * (x - c_i) / r_i   (s_i > 0)
        with np.errstate(divide='ignore', invalid='ignore'):
            fac = np.where(s > 0, e * 2.0 * DELTA * s / np.maximum(r, 1e-300), 0.0)
            others = np.where(one_m_e > 0, X[:, None] / one_m_e, 0.0)
        g = (others * fac)[:, :, None] * diff
        gX = g.sum(axis=1)
        mu = X + (1.0 - X) * float(dr)
        gmu = (1.0 - float(dr)) * gX
        out[a:a + chunk] = np.linalg.norm(gmu, axis=1) / mu
    return out


def refinement_cells(base_level, centres, dr, percentile, exclusive=True):
    """Cells (level, i, j, k) of the uniform 2^base_level mesh whose centre has
    |grad log mu| strictly above the given percentile (ties broken by x-fastest
    lexicographic index, so the count is deterministic)."""
    n = 1 << base_level
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing='ij')
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    centres_xyz = (ijk + 0.5) / n
    g = grad_log_mu(centres_xyz, centres, dr)
    n_flag = int(round(len(g) * (1.0 - percentile / 100.0)))
    order = np.lexsort((np.arange(len(g)), -g))
    sel = np.sort(order[:n_flag])
    sel = sel[g[sel] > 0] if exclusive else sel
    out = np.zeros((len(sel), 4), dtype=np.int32)
    out[:, 0] = base_level
    out[:, 1:] = ijk[sel]
    return out


def uniform_vector(n, seed):
    """Seeded uniform[-1, 1] vector in float64."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


# Workload recipes (sizes, seeds) of the five benchmark configurations.
CONFIGS = {
    "uniform8": dict(base_level=3, sinkers=4, dr=1e2, centre_seed=1),
    "uniform64": dict(base_level=6, sinkers=8, dr=1e4, centre_seed=2, vector_seed=42),
    "adaptive32p2": dict(base_level=5, sinkers=16, dr=1e6, centre_seed=3,
                            refine_percentile=80.0, refine_levels=2),
    "learned": dict(train_level=5, eval_level=6, train_fields=256, eval_fields=32,
                       train_seed0=10000, eval_seed0=20000, sinkers=(4, 32), log10_dr=(2.0, 6.0)),
    "uniform128p1": dict(base_level=7, sinkers=32, dr=1e6, centre_seed=5,
                            refine_percentile=97.5, refine_levels=1),
}


def learned_field(seed, sinker_range=(4, 32), log10_dr_range=(2.0, 6.0)):
    """One field of the learned-smoother workload: (centres [n,3], DR) with n
    uniform in sinker_range (inclusive) and log10 DR uniform in the range."""
    g = np.random.default_rng(seed)
    n = int(g.integers(sinker_range[0], sinker_range[1] + 1))
    dr = float(10.0 ** g.uniform(*log10_dr_range))
    centres = g.uniform(0.1, 0.9, size=(n, 3))
    return centres, dr
