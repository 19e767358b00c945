// Q3-Q2 reference element and lattice levels (see q3.h).
#include "q3.h"

#include <algorithm>
#include <cmath>

namespace mfgmg {

namespace {

// Lagrange polynomial i on the n points x, and its derivative, at t
double lagrange(const double* x, int n, int i, double t) {
  double v = 1.0;
  for (int j = 0; j < n; ++j)
    if (j != i) v *= (t - x[j]) / (x[i] - x[j]);
  return v;
}

double lagrange_deriv(const double* x, int n, int i, double t) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    if (k == i) continue;
    double term = 1.0 / (x[i] - x[k]);
    for (int j = 0; j < n; ++j)
      if (j != i && j != k) term *= (t - x[j]) / (x[i] - x[j]);
    s += term;
  }
  return s;
}

Q3Element make_element() {
  Q3Element E;
  const double r5 = 1.0 / std::sqrt(5.0);
  const double gll[4] = {0.0, 0.5 * (1.0 - r5), 0.5 * (1.0 + r5), 1.0};
  // Gauss-Legendre, 4 points: +-sqrt(3/7 -+ 2/7 sqrt(6/5)) on [-1, 1]
  const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
  const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
  const double xg[4] = {0.5 * (1.0 - b), 0.5 * (1.0 - a), 0.5 * (1.0 + a), 0.5 * (1.0 + b)};
  const double wg[4] = {0.5 * wb, 0.5 * wa, 0.5 * wa, 0.5 * wb};
  const double q2[3] = {0.0, 0.5, 1.0};
  for (int i = 0; i < 4; ++i) E.gll[i] = gll[i], E.xg[i] = xg[i], E.wg[i] = wg[i];
  for (int q = 0; q < 4; ++q) {
    for (int i = 0; i < 4; ++i) {
      E.N[q][i] = lagrange(gll, 4, i, xg[q]);
      E.D[q][i] = lagrange_deriv(xg, 4, i, xg[q]);
    }
    for (int i = 0; i < 3; ++i) E.P2[q][i] = lagrange(q2, 3, i, xg[q]);
  }
  // 1D integrals of the Q3 basis (exact with 4 Gauss points): mass M, stiffness
  // S and G[a][b] = int L_a' L_b
  double M[4][4], S[4][4], G[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      M[i][j] = S[i][j] = G[i][j] = 0.0;
      for (int q = 0; q < 4; ++q) {
        const double li = lagrange(gll, 4, i, xg[q]), lj = lagrange(gll, 4, j, xg[q]);
        const double di = lagrange_deriv(gll, 4, i, xg[q]), dj = lagrange_deriv(gll, 4, j, xg[q]);
        M[i][j] += wg[q] * li * lj;
        S[i][j] += wg[q] * di * dj;
        G[i][j] += wg[q] * di * lj;
      }
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      E.M2[i][j] = 0.0;
      for (int q = 0; q < 4; ++q) E.M2[i][j] += wg[q] * E.P2[q][i] * E.P2[q][j];
    }
  // int d_p phi_A d_q phi_B for tensor nodes A = (a0, a1, a2), B = (b0, b1, b2):
  // per direction S (p = q = dim), G[a][b] (dim = p != q), G[b][a] (dim = q != p), M
  auto dd = [&](int p, int q, const int* A, const int* B) {
    double v = 1.0;
    for (int dim = 0; dim < 3; ++dim) {
      const int ai = A[dim], bi = B[dim];
      if (dim == p && dim == q) v *= S[ai][bi];
      else if (dim == p) v *= G[ai][bi];
      else if (dim == q) v *= G[bi][ai];
      else v *= M[ai][bi];
    }
    return v;
  };
  E.K.assign(192 * 192, 0.0);
  for (int na = 0; na < 64; ++na)
    for (int nb = 0; nb < 64; ++nb) {
      const int A[3] = {na % 4, (na / 4) % 4, na / 16}, B[3] = {nb % 4, (nb / 4) % 4, nb / 16};
      double lap = 0.0;
      for (int e = 0; e < 3; ++e) lap += dd(e, e, A, B);
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d)
          E.K[size_t(3 * na + c) * 192 + 3 * nb + d] = dd(d, c, A, B) + (c == d ? lap : 0.0);
    }
  return E;
}

}  // namespace

const Q3Element& q3_element() {
  static const Q3Element E = make_element();
  return E;
}

void build_q3_level(const Level& cells, bool leaf, Level& lv) {
  const Q3Element& E = q3_element();
  const int ell = cells.ell;
  const int64_t n = int64_t(1) << ell, m = 3 * n + 1;
  lv = Level{};
  lv.ell = ell;
  lv.ncell = cells.ncell;
  lv.clev = cells.clev;
  lv.cijk = cells.cijk;
  lv.uniform = true;
  lv.n_edge = n;
  lv.min_cell_level = ell;
  lv.mu_src = cells.mu_src;
  lv.nnode = m * m * m;
  lv.key.resize(size_t(lv.nnode));
  lv.ntype.assign(size_t(lv.nnode), NODE_FREE);
  lv.hang_index.assign(size_t(lv.nnode), -1);
  for (int64_t Z = 0; Z < m; ++Z)
    for (int64_t Y = 0; Y < m; ++Y)
      for (int64_t X = 0; X < m; ++X) {
        const int64_t id = X + m * (Y + m * Z);
        lv.key[size_t(id)] = id;
        if (X == 0 || Y == 0 || Z == 0 || X == m - 1 || Y == m - 1 || Z == m - 1)
          lv.ntype[size_t(id)] = NODE_DIRICHLET;
      }
  lv.nfree_nodes = (m - 2) * (m - 2) * (m - 2);
  if (ell >= 2) {
    // 1D: fine lattice point X at x = (cell + gll[a]) / n lies in coarse cell
    // kc with local coordinate t; its row holds L_a(t) on coarse points 3 kc + a
    const int64_t nc = n / 2, mc = 3 * nc + 1;
    std::vector<int64_t> c0(static_cast<size_t>(m));
    std::vector<double> w1(static_cast<size_t>(4 * m));
    for (int64_t X = 0; X < m; ++X) {
      const int64_t cell = std::min<int64_t>(X / 3, n - 1);
      const double x = (double(cell) + E.gll[X - 3 * cell]) / double(n);
      const int64_t kc = std::min<int64_t>(int64_t(std::floor(x * double(nc))), nc - 1);
      const double t = x * double(nc) - double(kc);
      c0[size_t(X)] = 3 * kc;
      for (int a = 0; a < 4; ++a) w1[size_t(4 * X + a)] = lagrange(E.gll, 4, a, t);
    }
    lv.p1_c0.assign(c0.begin(), c0.end());
    lv.p1_w = w1;
    lv.P_ptr.assign(size_t(lv.nnode) + 1, 0);
    for (int64_t Z = 0; Z < m; ++Z)
      for (int64_t Y = 0; Y < m; ++Y)
        for (int64_t X = 0; X < m; ++X) {
          const int64_t f = X + m * (Y + m * Z);
          if (lv.ntype[size_t(f)] == NODE_FREE) {
            for (int cz = 0; cz < 4; ++cz)
              for (int cy = 0; cy < 4; ++cy)
                for (int cx = 0; cx < 4; ++cx) {
                  const double w = w1[size_t(4 * X + cx)] * w1[size_t(4 * Y + cy)] * w1[size_t(4 * Z + cz)];
                  if (std::fabs(w) < 1e-15) continue;
                  const int64_t XC = c0[size_t(X)] + cx, YC = c0[size_t(Y)] + cy, ZC = c0[size_t(Z)] + cz;
                  if (XC == 0 || YC == 0 || ZC == 0 || XC == mc - 1 || YC == mc - 1 || ZC == mc - 1) continue;
                  lv.P_col.push_back(int32_t(XC + mc * (YC + mc * ZC)));
                  lv.P_w.push_back(w);
                }
          }
          lv.P_ptr[size_t(f) + 1] = int64_t(lv.P_col.size());
        }
    const int64_t ncn = mc * mc * mc;
    lv.R_ptr.assign(size_t(ncn) + 1, 0);
    for (int32_t c : lv.P_col) ++lv.R_ptr[size_t(c) + 1];
    for (int64_t c = 0; c < ncn; ++c) lv.R_ptr[size_t(c) + 1] += lv.R_ptr[size_t(c)];
    lv.R_col.resize(lv.P_col.size());
    lv.R_w.resize(lv.P_col.size());
    std::vector<int64_t> pos(lv.R_ptr.begin(), lv.R_ptr.end() - 1);
    for (int64_t f = 0; f < lv.nnode; ++f)
      for (int64_t q = lv.P_ptr[size_t(f)]; q < lv.P_ptr[size_t(f) + 1]; ++q) {
        const int64_t d = pos[size_t(lv.P_col[size_t(q)])]++;
        lv.R_col[size_t(d)] = int32_t(f);
        lv.R_w[size_t(d)] = lv.P_w[size_t(q)];
      }
  }
  if (leaf) {
    const int64_t mp = 2 * n + 1;
    lv.npnode = mp * mp * mp;
    lv.pkey.resize(size_t(lv.npnode));
    for (int64_t i = 0; i < lv.npnode; ++i) lv.pkey[size_t(i)] = i;
    lv.ptype.assign(size_t(lv.npnode), NODE_FREE);
    lv.phang_index.assign(size_t(lv.npnode), -1);
  }
}

}  // namespace mfgmg
