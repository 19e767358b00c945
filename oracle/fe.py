"""Reference element for the Q2-Q1 Taylor-Hood pair on the unit cube.

Test infrastructure (see ``oracle/__init__``).

Paper: Sec. 2.1 (Discretization) chooses Taylor-Hood [Q_{k+1}]^3 x Q_k with
k = 1, and defines the bilinear forms
    a(v, u) = int 2 mu eps(v) : eps(u),   b(v, p) = -int (div v) p,
    f(v)    = int v . f,
with eps(u) = (grad u + grad u^T) / 2 (Sec. 2, eq. stokes).  The pressure
Schur approximation uses the mu^{-1}-weighted pressure mass matrix (Sec. 2.2.2).

Readings (the paper fixes none of these):
* basis: Lagrange polynomials on the equispaced points {0, 1/2, 1} (Q2) and
  {0, 1} (Q1), tensorised with x running fastest: local node (i, j, k) has
  index i + 3 j + 9 k (Q2) or i + 2 j + 4 k (Q1);
* local velocity dof (node a, component c) has index 3 a + c;
* quadrature: tensor Gauss-Legendre, 3 points per direction, which integrates
  every product above exactly for a cell-constant mu on an axis-aligned cube.
"""
import numpy as np


def gauss_1d(n):
    """n-point Gauss-Legendre rule mapped to [0, 1]: (points, weights)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def q2_1d(t):
    """Values [3, len(t)] of the 1D Q2 Lagrange basis on nodes 0, 1/2, 1."""
    t = np.asarray(t, dtype=np.float64)
    return np.array([2.0 * (t - 0.5) * (t - 1.0),
                     -4.0 * t * (t - 1.0),
                     2.0 * t * (t - 0.5)])


def q2_1d_deriv(t):
    t = np.asarray(t, dtype=np.float64)
    return np.array([4.0 * t - 3.0, 4.0 - 8.0 * t, 4.0 * t - 1.0])


def q1_1d(t):
    t = np.asarray(t, dtype=np.float64)
    return np.array([1.0 - t, t])


def q1_1d_deriv(t):
    t = np.asarray(t, dtype=np.float64)
    return np.array([-np.ones_like(t), np.ones_like(t)])


def _tensor(vals_x, vals_y, vals_z):
    """Tensor-product values: out[i + n j + n^2 k, p] = vx[i,p] vy[j,p] vz[k,p]."""
    n = vals_x.shape[0]
    out = np.einsum('ip,jp,kp->kjip', vals_x, vals_y, vals_z)
    return out.reshape(n * n * n, -1)


def q2_basis(points):
    """Q2 basis at points [np, 3] in the unit cube.

    Returns (phi [27, np], grad [27, 3, np])."""
    p = np.atleast_2d(np.asarray(points, dtype=np.float64))
    vx, vy, vz = q2_1d(p[:, 0]), q2_1d(p[:, 1]), q2_1d(p[:, 2])
    dx, dy, dz = q2_1d_deriv(p[:, 0]), q2_1d_deriv(p[:, 1]), q2_1d_deriv(p[:, 2])
    phi = _tensor(vx, vy, vz)
    grad = np.stack([_tensor(dx, vy, vz), _tensor(vx, dy, vz), _tensor(vx, vy, dz)], axis=1)
    return phi, grad


def q1_basis(points):
    """Q1 basis at points [np, 3]: (psi [8, np], grad [8, 3, np])."""
    p = np.atleast_2d(np.asarray(points, dtype=np.float64))
    vx, vy, vz = q1_1d(p[:, 0]), q1_1d(p[:, 1]), q1_1d(p[:, 2])
    dx, dy, dz = q1_1d_deriv(p[:, 0]), q1_1d_deriv(p[:, 1]), q1_1d_deriv(p[:, 2])
    psi = _tensor(vx, vy, vz)
    grad = np.stack([_tensor(dx, vy, vz), _tensor(vx, dy, vz), _tensor(vx, vy, dz)], axis=1)
    return psi, grad


def gauss_points_3d(n=3):
    """Tensor Gauss points [n^3, 3] (x fastest) and weights [n^3] on the unit cube."""
    x, w = gauss_1d(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing='ij')
    WZ, WY, WX = np.meshgrid(w, w, w, indexing='ij')
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return pts, (WX * WY * WZ).ravel()


def element_matrices(nq=3):
    """Element matrices on the unit cube with mu = 1, by nq^3 Gauss quadrature.

    K[(a,c),(b,d)] = int 2 eps(phi_a e_c) : eps(phi_b e_d)
                   = int (delta_cd grad phi_a . grad phi_b + d_d phi_a d_c phi_b)
                     (the strain-rate form of a(.,.), Sec. 2.1);
    B[i,(b,d)]     = -int psi_i d_d phi_b          (b(.,.), Sec. 2.1);
    M[i,j]         = int psi_i psi_j               (pressure mass, Sec. 2.2.2).
    Returns (K [81, 81], B [8, 81], M [8, 8]).
    """
    pts, w = gauss_points_3d(nq)
    phi, g = q2_basis(pts)          # [27, nq3], [27, 3, nq3]
    psi, _ = q1_basis(pts)          # [8, nq3]
    K = np.zeros((81, 81))
    for c in range(3):
        for d in range(3):
            blk = np.zeros((27, 27))
            if c == d:
                blk += np.einsum('aiq,biq,q->ab', g, g, w)
            blk += np.einsum('aq,bq,q->ab', g[:, d, :], g[:, c, :], w)
            K[c::3, d::3] = blk
    B = np.zeros((8, 81))
    for d in range(3):
        B[:, d::3] = -np.einsum('iq,bq,q->ib', psi, g[:, d, :], w)
    M = np.einsum('iq,jq,q->ij', psi, psi, w)
    return K, B, M


# Closed-form 1D integrals of the Q2 basis (used as an independent route).
Q2_MASS_1D = np.array([[4., 2., -1.], [2., 16., 2.], [-1., 2., 4.]]) / 30.0
Q2_STIFF_1D = np.array([[7., -8., 1.], [-8., 16., -8.], [1., -8., 7.]]) / 3.0
# G[i, j] = int L_i' L_j over [0, 1]
Q2_GRAD_1D = np.array([[-1/2, -2/3, 1/6], [2/3, 0., -2/3], [-1/6, 2/3, 1/2]])


def element_matrix_K_kronecker():
    """K of ``element_matrices`` from exact 1D integrals and Kronecker products.

    int d_x phi_a d_y phi_b = G[ax,bx] G[by,ay] M[az,bz], and the analogues;
    independent of any quadrature rule.
    """
    M, S, G = Q2_MASS_1D, Q2_STIFF_1D, Q2_GRAD_1D
    idx = np.array([(i, j, k) for k in range(3) for j in range(3) for i in range(3)])

    def one_d(mats):
        # mats[dim] is a 3x3 matrix indexed [a_dim, b_dim]
        return (mats[0][np.ix_(idx[:, 0], idx[:, 0])] * mats[1][np.ix_(idx[:, 1], idx[:, 1])]
                * mats[2][np.ix_(idx[:, 2], idx[:, 2])])

    def dd(p, q):
        """int d_p phi_a d_q phi_b as [27, 27]."""
        mats = [M, M, M]
        if p == q:
            mats = list(mats)
            mats[p] = S
        else:
            mats = list(mats)
            mats[p] = G          # derivative on a in dim p: int L_a' L_b
            mats[q] = G.T        # derivative on b in dim q: int L_a L_b'
        return one_d(mats)

    lap = dd(0, 0) + dd(1, 1) + dd(2, 2)
    K = np.zeros((81, 81))
    for c in range(3):
        for d in range(3):
            blk = dd(d, c).copy()
            if c == d:
                blk += lap
            K[c::3, d::3] = blk
    return K


def element_rhs_weights(nq=3):
    """Per-cell RHS map on the unit cube: Fhat[a, q] = w_q phi_a(xi_q).

    F_e[(a,c)] = h^3 sum_q Fhat[a,q] f_c(x_q), with f evaluated pointwise at
    the Gauss points (reading of the body force of Sec. 3.2).
    """
    pts, w = gauss_points_3d(nq)
    phi, _ = q2_basis(pts)
    return phi * w[None, :]


def q2_local_positions():
    """Local Q2 node positions [27, 3] on the unit cube."""
    return np.array([(i / 2, j / 2, k / 2) for k in range(3) for j in range(3) for i in range(3)])


def q1_local_positions():
    return np.array([(i, j, k) for k in range(2) for j in range(2) for i in range(2)], dtype=float)
