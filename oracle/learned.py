"""Learned smoother scaling: features, MLP, per-dof scaling, target fitting.

Test infrastructure (see ``oracle/__init__``).

Not part of the paper.  The paper smooths with a degree-4 Chebyshev iteration
preconditioned by the inverse diagonal (Sec. 2.2.1); the learned extension
replaces M^{-1} = diag(1/d) on a level by diag(s/d), with per-dof scalings s
predicted by a small network from the local viscosity.  Definitions:

* features of a cell K of level l (in the level mesh that holds K): the 27
  values log10 mu_{K'} - log10 mu_K over the 3x3x3 same-level neighbourhood of
  K (offsets (i-1, j-1, k-1), x fastest).  A neighbour position covered by a
  coarser cell takes that cell's viscosity; a position outside the domain
  takes mu_K (feature 0).  Viscosities of level-l positions are those of the
  level-l mesh (children averaged onto parents, Sec. 2.3).
* network: 27 -> 64 -> 64 -> 3, GELU(x) = x Phi(x) (erf form) on both hidden
  layers, output clamped to [-2, 2]: y_K, one log-scaling per velocity
  component.
* per-dof scaling: s_(node, c) = exp(mean of y_{K, c} over the cells K of the
  level that have `node` among their 27 nodes).
* targets: on level l (lower levels plain), y minimises
      J(y) = (1/K) sum_k (1/m) log(||E^m e_k||_A / ||e_k||_A),
  E = I - V_l(y) A_l the error propagation of the V-cycle whose level-l
  smoothers use diag(s/d); m = 2, K = 4 SplitMix64 start vectors.  lambda is
  re-estimated for every y.  The gradient is the adjoint of the linear
  recurrence at fixed lambda (reverse sweep through both Chebyshev smoothers
  and the coarse correction; V_l is symmetric, so E^T = I - A V_l) plus the
  term through lambda(s): the smoother depends on s and lambda only through
  s / lambda (the Chebyshev coefficients scale as 1/lambda, the interval
  ratio is fixed), so dJ/dlambda = -(1/lambda) sum_i s_i dJ/ds_i; and the
  Ritz value theta of the generalized problem A v = theta diag(d/s) v moves
  by s_i dtheta/ds_i = theta pi_i, pi_i = v_i^2 d_i/s_i / sum_j v_j^2 d_j/s_j,
  with v the Ritz vector (derivative of the Rayleigh quotient at v).  In
  log-scaling form the total gradient is q_i - pi_i sum_j q_j with
  q_i = s_i dJ/ds_i at fixed lambda: J is invariant under s -> c s, and so
  is its gradient.
  Adam, lr 0.05, 30 steps from y = 0.
* training: mean squared error of the network output against the targets,
  Adam (lr 1e-3), mini-batches.
"""
import numpy as np
from scipy.special import erf

from . import multigrid as mg
from . import rng
from .mesh import cell_code

LAYERS = (27, 64, 64, 3)
N_PARAMS = 27 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3   # 6147
CLAMP = 2.0
FIT_SEED = 777
FIT_K = 4
FIT_M = 2


# ------------------------------------------------------------------- features
def features(hier, mus, ell):
    """[ncell(l), 27] relative log10 viscosities of the 3x3x3 neighbourhood."""
    mesh = hier.levels[ell]
    lut = {}
    for m in range(1, hier.L + 1):
        lm = hier.levels[m]
        sel = lm.lev == m
        for code, mu in zip(cell_code(lm.lev[sel], lm.ijk[sel]), mus[m][sel]):
            lut[int(code)] = mu
    # coarser leaf cells: their own viscosity at their own level
    for m in range(1, hier.L + 1):
        lm = hier.levels[m]
        for l, c, mu in zip(lm.lev, lm.ijk, mus[m]):
            lut.setdefault(int(cell_code(l, c)), mu)
    out = np.zeros((mesh.ncell, 27))
    for ci in range(mesh.ncell):
        l = int(mesh.lev[ci])
        i, j, k = (int(v) for v in mesh.ijk[ci])
        muK = mus[ell][ci]
        n = 1 << l
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    p = (i + dx - 1, j + dy - 1, k + dz - 1)
                    if min(p) < 0 or max(p) >= n:
                        val = muK
                    else:
                        val = None
                        for up in range(l + 1):
                            code = int(cell_code(l - up, np.array(p) >> up))
                            if code in lut:
                                val = lut[code]
                                break
                        assert val is not None
                    out[ci, dx + 3 * dy + 9 * dz] = np.log10(val) - np.log10(muK)
    return out


# ------------------------------------------------------------------------ MLP
def init_params(seed=0):
    """Flat parameter vector: W1 [64,27], b1 [64], W2 [64,64], b2 [64], W3 [3,64], b3 [3].
    He-uniform weights from numpy's default generator, zero biases."""
    g = np.random.default_rng(seed)
    parts = []
    for fi, fo in zip(LAYERS[:-1], LAYERS[1:]):
        lim = np.sqrt(6.0 / fi)
        parts.append(g.uniform(-lim, lim, (fo, fi)).ravel())
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


def unpack(w):
    out, o = [], 0
    for fi, fo in zip(LAYERS[:-1], LAYERS[1:]):
        W = w[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = w[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_deriv(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def mlp_forward(w, x):
    """Returns (y [n,3] clamped, cache)."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(w)
    z1 = x @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    z3 = h2 @ W3.T + b3
    y = np.clip(z3, -CLAMP, CLAMP)
    return y, (x, z1, h1, z2, h2, z3)


def mlp_backward(w, cache, dy):
    """Gradient of sum(dy * y) w.r.t. the flat parameters (clamp passes
    gradient only strictly inside [-2, 2])."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(w)
    x, z1, h1, z2, h2, z3 = cache
    d3 = dy * ((z3 > -CLAMP) & (z3 < CLAMP))
    gW3, gb3 = d3.T @ h2, d3.sum(0)
    d2 = (d3 @ W3) * gelu_deriv(z2)
    gW2, gb2 = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ W2) * gelu_deriv(z1)
    gW1, gb1 = d1.T @ x, d1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), t >= 1; returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- scaling
def node_counts(mesh):
    return np.bincount(mesh.cell_nodes.ravel(), minlength=mesh.nnode).astype(np.float64)


def dof_scaling(mesh, y):
    """s_(node, c) = exp(mean over cells containing node of y_{K,c})."""
    cnt = node_counts(mesh)
    s = np.zeros((mesh.nnode, 3))
    for c in range(3):
        acc = np.bincount(mesh.cell_nodes.ravel(), weights=np.repeat(y[:, c], 27), minlength=mesh.nnode)
        s[:, c] = np.exp(acc / cnt)
    return s.ravel()


def scaling_grad_to_cells(mesh, s, sbar):
    """ybar_{K,c} = sum over the nodes a of K of sbar_(a,c) s_(a,c) / count_a."""
    cnt = node_counts(mesh)
    g = (sbar * s).reshape(-1, 3) / cnt[:, None]
    return g[mesh.cell_nodes].sum(axis=1)          # [ncell, 3]


# ------------------------------------------------------- differentiable V-cycle
def cheb_coeffs(lam, degree=mg.CHEB_DEGREE):
    lo = lam / mg.SMOOTHING_RANGE
    theta, delta = 0.5 * (lam + lo), 0.5 * (lam - lo)
    sigma = theta / delta
    rho = [1.0 / sigma]
    alpha, beta = [0.0], [1.0 / theta]
    for _ in range(1, degree):
        r = 1.0 / (2.0 * sigma - rho[-1])
        alpha.append(r * rho[-1])
        beta.append(2.0 * r / delta)
        rho.append(r)
    return alpha, beta


def cheb_forward(A, minv, b, x0, lam):
    """The Chebyshev smoother of ``multigrid.chebyshev``, keeping the residuals."""
    alpha, beta = cheb_coeffs(lam)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b.copy() if x0 is None else b - A @ x
    rs = [r]
    d = beta[0] * minv * r
    x = x + d
    for k in range(1, len(alpha)):
        r = r - A @ d
        rs.append(r)
        d = alpha[k] * d + beta[k] * minv * r
        x = x + d
    return x, rs


def cheb_reverse(A, minv, dd, lam, rs, xbar, need_x0bar):
    """Adjoint of ``cheb_forward``: given the adjoint of its output, return
    (bbar, x0bar, sbar) where sbar_i = d/ds_i for M^{-1} = diag(s / dd)."""
    alpha, beta = cheb_coeffs(lam)
    n = len(alpha)
    dbar = np.zeros_like(xbar)
    rbar = np.zeros_like(xbar)
    sbar = np.zeros_like(xbar)
    for k in range(n - 1, -1, -1):
        dbar = dbar + xbar
        rbar = rbar + beta[k] * minv * dbar
        sbar += beta[k] * dbar * rs[k] / dd
        if k > 0:
            dbar = alpha[k] * dbar - A @ rbar
    x0bar = (xbar - A @ rbar) if need_x0bar else None
    return rbar, x0bar, sbar


def cg_lanczos_ritz(apply_A, minv, r0, steps=mg.LANCZOS_STEPS):
    """Largest Ritz pair (theta, v) of M^{-1} A, M^{-1} = diag(minv), from
    ``steps`` PCG iterations on A x = r0 from x = 0.

    The preconditioned residuals z_k = M^{-1} r_k are M-orthogonal; with
    nu_k = sqrt(r_k . z_k), the vectors (-1)^k z_k / nu_k are an M-orthonormal
    Lanczos basis in which M^{-1} A is the tridiagonal matrix T of the CG
    coefficients (diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1}, off-diagonal
    sqrt(beta_k)/alpha_k, both positive).  v = sum_k c_k (-1)^k z_k / nu_k for
    the eigenvector c of T's largest eigenvalue theta."""
    r = np.array(r0, dtype=np.float64)
    z = minv * r
    p = z.copy()
    rz = r @ z
    rz0 = rz
    alphas, betas, basis = [], [], []
    for k in range(steps):
        q = apply_A(p)
        pq = p @ q
        if pq <= 0:
            break
        basis.append((-1) ** k * z / np.sqrt(rz))
        alpha = rz / pq
        alphas.append(alpha)
        r = r - alpha * q
        z = minv * r
        rz_new = r @ z
        if rz_new <= 1e-30 * rz0:
            break
        betas.append(rz_new / rz)
        p = z + betas[-1] * p
        rz = rz_new
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    ev, evec = np.linalg.eigh(T)
    c = evec[:, -1]
    return float(ev[-1]), sum(ci * b for ci, b in zip(c, basis))


def lambda_sensitivity(minv, free, v):
    """pi_i = v_i^2 M_ii / sum_j v_j^2 M_jj over free dofs (M = diag(1/minv)):
    s_i dlambda/ds_i = lambda pi_i for the Ritz-value estimate of lambda."""
    wgt = np.where(free, v * v / minv, 0.0)
    return wgt / wgt.sum()


class ScaledLevel:
    """The V-cycle of ``multigrid.GMG`` whose level-l smoothers use diag(s/d),
    with the forward states needed by its adjoint."""

    def __init__(self, gmg, ell, s, lam=None, lanczos_steps=mg.LANCZOS_STEPS):
        self.g, self.ell = gmg, ell
        A = gmg.A[ell]
        self.A = A
        self.dd = A.diagonal()
        self.free = gmg.free[ell]
        self.minv = np.where(self.free, s / self.dd, 1.0)
        mesh = gmg.hier.levels[ell]
        self.ritz = None
        if lam is None:
            r0 = rng.dof_vector(mesh, mg.LAMBDA_SEED) * self.free
            theta, self.ritz = cg_lanczos_ritz(lambda v: A @ v, self.minv, r0, lanczos_steps)
            lam = mg.LAMBDA_SAFETY * theta
        self.lam = lam

    def coarse(self, r):
        P = self.g.P[self.ell]
        return P @ self.g.vcycle(P.T @ r, self.ell - 1)

    def forward(self, b):
        A = self.A
        x1, rpre = cheb_forward(A, self.minv, b, None, self.lam)
        x2 = x1 + self.coarse(b - A @ x1)
        x3, rpost = cheb_forward(A, self.minv, b, x2, self.lam)
        return x3, (rpre, rpost)

    def reverse(self, states, w):
        """Returns (bbar, sbar) for adjoint w of the output."""
        A = self.A
        rpre, rpost = states
        b1, x2bar, s1 = cheb_reverse(A, self.minv, self.dd, self.lam, rpost, w, True)
        cx = self.coarse(x2bar)
        x1bar = x2bar - A @ cx
        b3, _, s2 = cheb_reverse(A, self.minv, self.dd, self.lam, rpre, x1bar, False)
        return b1 + cx + b3, s1 + s2


def fit_vectors(mesh, free, k=FIT_K, seed=FIT_SEED):
    return [rng.dof_vector(mesh, seed + i) * free for i in range(k)]


def objective(gmg, ell, y, es=None, m=FIT_M, with_grad=True, lam=None, lanczos_steps=mg.LANCZOS_STEPS):
    """J(y) and dJ/dy (per cell, 3 components); lam: hold the Chebyshev bound
    fixed instead of re-estimating it (then the gradient has no lambda term)."""
    mesh = gmg.hier.levels[ell]
    s = dof_scaling(mesh, y)
    lv = ScaledLevel(gmg, ell, s, lam, lanczos_steps)
    A = lv.A
    es = fit_vectors(mesh, lv.free) if es is None else es
    K = len(es)
    J = 0.0
    sbar = np.zeros(mesh.n_u)
    for e in es:
        us, sts = [e], []
        for _ in range(m):
            x, st = lv.forward(A @ us[-1])
            sts.append(st)
            us.append(us[-1] - x)
        nu = us[-1] @ (A @ us[-1])
        ne = e @ (A @ e)
        J += 0.5 * (np.log(nu) - np.log(ne)) / (m * K)
        if not with_grad:
            continue
        # adjoint seed for u_m, then back through the m applications of E:
        # d(E u)/ds with adjoint w is -(reverse of the V-cycle at b = A u)
        w = (A @ us[-1]) / nu / (m * K)
        for j in range(m - 1, -1, -1):
            _, sb = lv.reverse(sts[j], w)
            sbar -= sb
            if j > 0:
                w = w - A @ lv.forward(w)[0]          # E^T w = w - A V w
    if not with_grad:
        return J, None
    sbar = sbar * lv.free
    if lv.ritz is not None:                       # the term through lambda(s)
        pi = lambda_sensitivity(lv.minv, lv.free, lv.ritz)
        sbar = sbar - pi * (s * sbar).sum() / s
    return J, scaling_grad_to_cells(mesh, s, sbar)


def fit_targets(gmg, ell, steps=30, lr=0.05, es=None):
    """Adam on J from y = 0; returns (y, history of J)."""
    mesh = gmg.hier.levels[ell]
    y = np.zeros((mesh.ncell, 3))
    mm, vv = np.zeros_like(y), np.zeros_like(y)
    hist = []
    for t in range(1, steps + 1):
        J, g = objective(gmg, ell, y, es)
        hist.append(J)
        y, mm, vv = adam_step(y, g, mm, vv, t, lr)
        y = np.clip(y, -CLAMP, CLAMP)
    hist.append(objective(gmg, ell, y, es, with_grad=False)[0])
    return y, hist
