// Learned smoother scaling: host drivers and C-ABI entry points.
//
// Target fitting: on level l (lower levels plain) the per-cell log-scalings y
// minimise J(y) = (1/K) sum_k (1/m) log(||E^m e_k||_A / ||e_k||_A), E = I - V A,
// V the V-cycle whose level-l Chebyshev smoothers use diag(s/d).  lambda is
// re-estimated for every y (12-step CG-Lanczos with diag(s/d)) and held
// constant in the gradient.  The gradient is the adjoint of the linear
// recurrence: a reverse sweep through the post-smoother, the coarse
// correction (symmetric: P V_{l-1} P^T) and the pre-smoother, with the
// forward residuals of each smoother kept; since V is symmetric,
// E^T = I - A V.  Adam (Kingma & Ba) updates y, clipped to [-2, 2].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "ctx.h"
#include "learned.h"

using namespace mfgmg;
using namespace mfgmg::detail;
using namespace mfgmg::learned;

namespace {

constexpr int kFitK = 4;
constexpr int kFitM = 2;
constexpr uint64_t kFitSeed = 777;
constexpr uint64_t kGuardSeed = 4242;
// Guard: power steps per factor estimate, and the relative margin by which the
// learned factor must undercut the plain one.  Three steps from the same start
// vector leave the two estimates' ratio uncertain by a few per cent; a 0.3%
// lower learned estimate once came with two more outer iterations than plain.
constexpr int kGuardSteps = 6;
constexpr double kGuardMargin = 0.05;

struct DBuf {
  std::vector<double*> v;
  ~DBuf() {
    for (double* p : v)
      if (p) (void)hipFree(p);
  }
  double* get(size_t n) {
    double* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)) != hipSuccess) return nullptr;
    v.push_back(p);
    return p;
  }
};

void cheb_coeffs(double lam, double alpha[4], double beta[4]) {
  const double lo = lam / 15.0, theta = 0.5 * (lam + lo), delta = 0.5 * (lam - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  alpha[0] = 0.0;
  beta[0] = 1.0 / theta;
  for (int k = 1; k < 4; ++k) {
    const double r = 1.0 / (2.0 * sigma - rho);
    alpha[k] = r * rho;
    beta[k] = 2.0 * r / delta;
    rho = r;
  }
}

// Level-l work for the objective and its adjoint (FP64).
struct Fit {
  mfgmg_ctx* ctx;
  int ell;
  int64_t n;       // 3 * nnode
  hipStream_t s;
  DBuf buf;
  double *acc, *cnt, *sdof, *minv_s, *sbar, *ybar;
  double *d, *t, *x, *w, *u1, *u2, *dbar, *rbar, *cx, *x1bar, *x2bar, *xb, *bv;
  double *ritz, *basis;   // Ritz vector of lambda and the Lanczos basis it is built from
  double* es[kFitK];
  double* rs[2][2][4];   // [application][pre, post][k]
  double ne[kFitK];
  double lam = 0.0;
  bool lam_free = false;  // lambda re-estimated from the scaling (gradient has a lambda term)

  bool init(mfgmg_ctx* c, int l, hipStream_t st) {
    ctx = c, ell = l, s = st;
    const LevelDev& L = ctx->lv[size_t(l)];
    n = 3 * L.v.nnode;
    const size_t N = size_t(n);
    acc = buf.get(N), cnt = buf.get(size_t(L.v.nnode)), sdof = buf.get(N), minv_s = buf.get(N), sbar = buf.get(N);
    ybar = buf.get(size_t(3 * L.v.ncell));
    d = buf.get(N), t = buf.get(N), x = buf.get(N), w = buf.get(N), u1 = buf.get(N), u2 = buf.get(N);
    dbar = buf.get(N), rbar = buf.get(N), cx = buf.get(N), x1bar = buf.get(N), x2bar = buf.get(N), xb = buf.get(N);
    bv = buf.get(N);
    ritz = buf.get(N), basis = buf.get(N * kLanczosSteps);
    for (auto& e : es) e = buf.get(N);
    for (auto& a : rs)
      for (auto& b : a)
        for (auto& r : b) r = buf.get(N);
    for (double* p : buf.v)
      if (!p) return false;
    // start vectors: SplitMix64 over 3 key + component, free dofs only
    const Level& h = ctx->mesh->level(l);
    std::vector<double> hv(N);
    for (int k = 0; k < kFitK; ++k) {
      for (int64_t i = 0; i < h.nnode; ++i)
        for (int q = 0; q < 3; ++q)
          hv[size_t(3 * i + q)] =
              h.dof_free(i, q) ? splitmix_pm1(kFitSeed + k, uint64_t(3 * h.key[size_t(i)] + q)) : 0.0;
      (void)hipMemcpyAsync(es[k], hv.data(), N * sizeof(double), hipMemcpyHostToDevice, s);
      (void)hipStreamSynchronize(s);   // hv is refilled for the next vector
    }
    // cells per free node
    launch_fill(L.v.nnode, 0.0, cnt, s);
    launch_fill(n, 0.0, acc, s);
    launch_fill(3 * L.v.ncell, 0.0, ybar, s);
    launch_scaling_accum(L.v, ybar, acc, cnt, s);
    for (int k = 0; k < kFitK; ++k) {
      launch_vmult<double>(L.v, es[k], t, s);
      ne[k] = dot_sync(ctx, n, es[k], t, s);
    }
    return true;
  }

  const DevLevel& lv() const { return ctx->lv[size_t(ell)].v; }
  void A(const double* in, double* out) { launch_vmult<double>(lv(), in, out, s); }

  // C v = P V_{l-1} P^T v (plain lower levels)
  void coarse(const double* v, double* out, bool add) {
    LevelDev& F = ctx->lv[size_t(ell)];
    LevelDev& Cl = ctx->lv[size_t(ell - 1)];
    double* bc = static_cast<double*>(Cl.work[1][0]);
    double* xc = static_cast<double*>(Cl.work[1][1]);
    // scratch of the restriction: the level's FP64 smoother vectors (this
    // context keeps its own)
    launch_restrict_level<double>(F.v, Cl.v, F.R_ptr, F.R_col, F.R_w, v, nullptr, bc,
                                  static_cast<double*>(F.work[1][2]), static_cast<double*>(F.work[1][3]), s);
    vcycle<double>(ctx, ell - 1, bc, xc, s);
    launch_prolong_level<double>(F.v, Cl.v, F.P_ptr, F.P_col, F.P_w, xc, out, add, s);
  }

  // Chebyshev smoother with diag(minv_s), residuals stored in r[0..3]
  void cheb(const double* b, double* xx, bool zero, double* const r[4]) {
    double al[4], be[4];
    cheb_coeffs(lam, al, be);
    if (zero) {
      launch_cheb_init0<double>(n, b, minv_s, r[0], d, xx, be[0], s);
    } else {
      A(xx, t);
      launch_cheb_init<double>(n, b, t, minv_s, r[0], d, xx, be[0], s);
    }
    for (int k = 1; k < 4; ++k) {
      A(d, t);
      (void)hipMemcpyAsync(r[k], r[k - 1], size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s);
      launch_cheb_step<double>(n, t, minv_s, r[k], d, xx, al[k], be[k], s);
    }
  }

  // xx = V b, states kept in rs[app]
  void forward(const double* b, double* xx, int app) {
    cheb(b, xb, true, rs[app][0]);
    A(xb, t);
    // xx = xb + C (b - A xb)
    launch_axpby(n, 1.0, b, 0.0, x2bar, s);       // x2bar used as scratch: b
    launch_axpby(n, -1.0, t, 1.0, x2bar, s);      // b - A xb
    (void)hipMemcpyAsync(xx, xb, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s);
    coarse(x2bar, xx, true);
    cheb(b, xx, false, rs[app][1]);
  }

  // adjoint of the smoother: sbar += sgn * (d/ds of <xbar, smoother output>)
  void cheb_rev(double* const r[4], const double* xbar_in, bool need_x0bar, double* x0bar, double sgn) {
    double al[4], be[4];
    cheb_coeffs(lam, al, be);
    launch_fill(n, 0.0, dbar, s);
    launch_fill(n, 0.0, rbar, s);
    const double* mp = ctx->lv[size_t(ell)].minv_d;
    for (int k = 3; k >= 0; --k) {
      launch_chebrev_a(n, xbar_in, minv_s, mp, r[k], dbar, rbar, sbar, be[k], sgn, s);
      if (k > 0) {
        A(rbar, t);
        launch_chebrev_b(n, dbar, t, al[k], s);
      }
    }
    if (need_x0bar) {
      A(rbar, t);
      launch_axpby(n, 1.0, xbar_in, 0.0, x0bar, s);
      launch_axpby(n, -1.0, t, 1.0, x0bar, s);
    }
  }

  // sbar += sgn * d/ds <wbar, V_s b> for the application `app`
  void reverse(int app, const double* wbar, double sgn) {
    cheb_rev(rs[app][1], wbar, true, x2bar, sgn);
    launch_fill(n, 0.0, cx, s);
    coarse(x2bar, cx, false);
    A(cx, t);
    launch_axpby(n, 1.0, x2bar, 0.0, x1bar, s);
    launch_axpby(n, -1.0, t, 1.0, x1bar, s);
    cheb_rev(rs[app][0], x1bar, false, nullptr, sgn);
  }

  // scaling from y (double, [ncell][3]) and lambda (re-estimated unless lam_fixed > 0)
  int set_y(const double* yd, double lam_fixed) {
    LevelDev& L = ctx->lv[size_t(ell)];
    launch_fill(n, 0.0, acc, s);
    launch_scaling_accum(L.v, yd, acc, nullptr, s);
    launch_scaling_finish(L.v.nnode, acc, cnt, L.minv_d, sdof, minv_s, nullptr, s);
    lam_free = !(lam_fixed > 0);
    if (!lam_free) {
      lam = lam_fixed;
      return MFGMG_OK;
    }
    return lanczos_lambda(ctx, ell, minv_s, &lam, s, basis, ritz);
  }

  // J depends on s and lambda only through s / lambda, so dJ/dlambda = -(s . sbar) / lambda;
  // the Ritz value moves by s_i dlambda/ds_i = lambda pi_i, pi_i = v_i^2 M_ii / (v . M v)
  void add_lambda_term() {
    const double q = dot_sync(ctx, n, sdof, sbar, s);
    launch_ritz_mass(n, ritz, minv_s, t, s);
    const double vmv = dot_sync(ctx, n, ritz, t, s);
    if (vmv > 0) launch_lambda_term(n, ritz, minv_s, sdof, q / vmv, sbar, s);
  }

  // J and (optionally) ybar
  int objective(const double* yd, double lam_fixed, bool grad, double* J_out) {
    int st = set_y(yd, lam_fixed);
    if (st) return st;
    launch_fill(n, 0.0, sbar, s);
    double J = 0.0;
    for (int k = 0; k < kFitK; ++k) {
      A(es[k], bv);   // forward() overwrites t: the right-hand side needs its own buffer
      forward(bv, x, 0);
      launch_axpby(n, 1.0, es[k], 0.0, u1, s);
      launch_axpby(n, -1.0, x, 1.0, u1, s);          // u1 = e - V A e
      A(u1, bv);
      forward(bv, x, 1);
      launch_axpby(n, 1.0, u1, 0.0, u2, s);
      launch_axpby(n, -1.0, x, 1.0, u2, s);          // u2 = u1 - V A u1
      A(u2, t);
      const double nu = dot_sync(ctx, n, u2, t, s);
      if (!(nu > 0) || !std::isfinite(nu)) return ctx->set(MFGMG_ERR_NOCONV, "objective: non-finite error norm");
      J += 0.5 * (std::log(nu) - std::log(ne[k])) / double(kFitM * kFitK);
      if (!grad) continue;
      launch_scale_copy(n, 1.0 / (nu * kFitM * kFitK), t, w, s);   // dJ/du2
      reverse(1, w, -1.0);
      forward(w, x, 1);                                             // E^T w = w - A V w
      A(x, t);
      launch_axpby(n, -1.0, t, 1.0, w, s);
      reverse(0, w, -1.0);
    }
    if (grad && lam_free) add_lambda_term();
    if (grad) launch_scaling_grad(lv(), sbar, sdof, cnt, ybar, s);
    *J_out = J;
    return MFGMG_OK;
  }
};

int check_ready(mfgmg_ctx* ctx, int32_t level, bool need_smoother) {
  int st = check_level(ctx, level);
  if (st) return st;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  if (need_smoother && level < 2) return ctx->set(MFGMG_ERR_INVALID, "level 1 has no smoother");
  return MFGMG_OK;
}

inline uint64_t cell_code(int l, int64_t i, int64_t j, int64_t k) {
  const uint64_t off = ((uint64_t(1) << (3 * l)) - 1) / 7;
  const uint64_t nl = uint64_t(1) << l;
  return off + uint64_t(i) + nl * (uint64_t(j) + nl * uint64_t(k));
}

// V-cycle contraction estimate: three power steps of E = I - V A in the A-norm (FP64)
// A-norm contraction of E = I - V A on the leaf by `steps` power steps from
// a SplitMix64 vector (seed 4242), the V-cycle in precision `prec` (the
// residual and the error in FP64).  Negative on allocation failure.
double vcycle_factor(mfgmg_ctx* ctx, hipStream_t s, int prec, int steps) {
  const int L = ctx->mesh->L();
  const Level& h = ctx->mesh->level(L);
  const DevLevel& v = ctx->lv[size_t(L)].v;
  const int64_t n = 3 * h.nnode;
  DBuf buf;
  double *e = buf.get(size_t(n)), *t = buf.get(size_t(n)), *x = buf.get(size_t(n));
  // FP32 V-cycle: its right-hand side and result in the two halves of one buffer
  double* fbuf = prec == MFGMG_FP32 ? buf.get(size_t(n)) : nullptr;
  if (!e || !t || !x || (prec == MFGMG_FP32 && !fbuf)) return -1.0;
  float* tf = reinterpret_cast<float*>(fbuf);
  float* xf = tf + n;
  std::vector<double> hv(static_cast<size_t>(n));
  for (int64_t i = 0; i < h.nnode; ++i)
    for (int q = 0; q < 3; ++q)
      hv[size_t(3 * i + q)] =
          h.dof_free(i, q) ? splitmix_pm1(kGuardSeed, uint64_t(3 * h.key[size_t(i)] + q)) : 0.0;
  (void)hipMemcpyAsync(e, hv.data(), size_t(n) * sizeof(double), hipMemcpyHostToDevice, s);
  double rho = 0.0;
  for (int it = 0; it < steps; ++it) {
    launch_vmult<double>(v, e, t, s);
    const double ne = dot_sync(ctx, n, e, t, s);
    if (prec == MFGMG_FP32) {
      launch_to_float(n, t, tf, s);
      vcycle<float>(ctx, L, tf, xf, s);
      launch_to_double(n, xf, x, s);
    } else {
      vcycle<double>(ctx, L, t, x, s);
    }
    launch_axpby(n, -1.0, x, 1.0, e, s);
    launch_vmult<double>(v, e, t, s);
    const double nn = dot_sync(ctx, n, e, t, s);
    rho = std::sqrt(nn / ne);
    launch_scale_copy(n, 1.0 / std::sqrt(nn), e, e, s);
  }
  return rho;
}

}  // namespace

extern "C" {

int mfgmg_features(mfgmg_ctx* ctx, int32_t level, float* feat, void* stream) {
  if (ctx && ctx->mesh && ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "the learned scaling is built for Q2-Q1");
  int st = check_ready(ctx, level, false);
  if (st) return st;
  if (!feat) return MFGMG_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Mesh& m = *ctx->mesh;
  const int L = m.L();
  // all level viscosities in one array; cell code -> index (level-l cells at their own level)
  std::vector<int64_t> off(size_t(L + 2), 0);
  for (int l = 1; l <= L; ++l) off[size_t(l + 1)] = off[size_t(l)] + m.level(l).ncell;
  std::unordered_map<uint64_t, int32_t> code2idx;
  code2idx.reserve(size_t(off[size_t(L + 1)]));
  for (int l = 1; l <= L; ++l) {
    const Level& h = m.level(l);
    for (int64_t c = 0; c < h.ncell; ++c)
      code2idx.emplace(cell_code(h.clev[size_t(c)], h.cijk[size_t(3 * c)], h.cijk[size_t(3 * c + 1)],
                                 h.cijk[size_t(3 * c + 2)]),
                       int32_t(off[size_t(l)] + c));
  }
  const Level& h = m.level(level);
  std::vector<int32_t> nbr(static_cast<size_t>(27 * h.ncell)), self(static_cast<size_t>(h.ncell));
  for (int64_t c = 0; c < h.ncell; ++c) {
    const int l = h.clev[size_t(c)];
    const int64_t i = h.cijk[size_t(3 * c)], j = h.cijk[size_t(3 * c + 1)], k = h.cijk[size_t(3 * c + 2)];
    const int32_t me = int32_t(off[size_t(level)] + c);
    self[size_t(c)] = me;
    const int64_t nl = int64_t(1) << l;
    for (int dz = 0; dz < 3; ++dz)
      for (int dy = 0; dy < 3; ++dy)
        for (int dx = 0; dx < 3; ++dx) {
          const int64_t p[3] = {i + dx - 1, j + dy - 1, k + dz - 1};
          int32_t idx = me;
          if (p[0] >= 0 && p[1] >= 0 && p[2] >= 0 && p[0] < nl && p[1] < nl && p[2] < nl) {
            idx = -1;
            for (int up = 0; up <= l && idx < 0; ++up) {
              auto it = code2idx.find(cell_code(l - up, p[0] >> up, p[1] >> up, p[2] >> up));
              if (it != code2idx.end()) idx = it->second;
            }
            if (idx < 0) return ctx->set(MFGMG_ERR_MESH, "features: neighbour not found");
          }
          nbr[size_t(27 * c + dx + 3 * dy + 9 * dz)] = idx;
        }
  }
  double* mu_all = nullptr;
  int32_t *dn = nullptr, *ds = nullptr;
  HIPCHK(hipMalloc(&mu_all, size_t(off[size_t(L + 1)]) * sizeof(double)));
  HIPCHK(hipMalloc(&dn, nbr.size() * sizeof(int32_t)));
  HIPCHK(hipMalloc(&ds, self.size() * sizeof(int32_t)));
  for (int l = 1; l <= L; ++l)
    HIPCHK(hipMemcpyAsync(mu_all + off[size_t(l)], ctx->lv[size_t(l)].mu_d, size_t(m.level(l).ncell) * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(dn, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ds, self.data(), self.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  launch_features(h.ncell, dn, ds, mu_all, feat, s);
  HIPCHK(hipStreamSynchronize(s));
  (void)hipFree(mu_all);
  (void)hipFree(dn);
  (void)hipFree(ds);
  return MFGMG_OK;
}

int mfgmg_fit_objective(mfgmg_ctx* ctx, int32_t level, const float* y, double lam_fixed, double* J, double* lam_out,
                        float* grad, void* stream) {
  if (ctx && ctx->mesh && ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "the learned scaling is built for Q2-Q1");
  int st = check_ready(ctx, level, true);
  if (st) return st;
  if (!y || !J) return MFGMG_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool saved = ctx->use_scaling;
  ctx->use_scaling = false;   // lower levels plain
  Fit f;
  if (!f.init(ctx, level, s)) {
    ctx->use_scaling = saved;
    return ctx->set(MFGMG_ERR_NOMEM, "fit: device allocation failed");
  }
  const int64_t nc = ctx->lv[size_t(level)].v.ncell;
  double* yd = f.buf.get(size_t(3 * nc));
  launch_f2d(3 * nc, y, yd, s);
  st = f.objective(yd, lam_fixed, grad != nullptr, J);
  if (!st && grad) launch_d2f(3 * nc, f.ybar, grad, s);
  if (lam_out) *lam_out = f.lam;
  (void)hipStreamSynchronize(s);
  ctx->use_scaling = saved;
  return st;
}

int mfgmg_fit_targets(mfgmg_ctx* ctx, int32_t level, int32_t steps, double lr, float* y_out, double* J_hist,
                      void* stream) {
  if (ctx && ctx->mesh && ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "the learned scaling is built for Q2-Q1");
  int st = check_ready(ctx, level, true);
  if (st) return st;
  if (!y_out || steps < 0 || !(lr > 0)) return MFGMG_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool saved = ctx->use_scaling;
  ctx->use_scaling = false;
  Fit f;
  if (!f.init(ctx, level, s)) {
    ctx->use_scaling = saved;
    return ctx->set(MFGMG_ERR_NOMEM, "fit: device allocation failed");
  }
  const int64_t nc = ctx->lv[size_t(level)].v.ncell;
  double *yd = f.buf.get(size_t(3 * nc)), *mm = f.buf.get(size_t(3 * nc)), *vv = f.buf.get(size_t(3 * nc));
  if (!yd || !mm || !vv) {
    ctx->use_scaling = saved;
    return ctx->set(MFGMG_ERR_NOMEM, "fit: device allocation failed");
  }
  launch_fill(3 * nc, 0.0, yd, s);
  launch_fill(3 * nc, 0.0, mm, s);
  launch_fill(3 * nc, 0.0, vv, s);
  for (int t = 1; t <= steps && !st; ++t) {
    double J = 0.0;
    st = f.objective(yd, 0.0, true, &J);
    if (st) break;
    if (J_hist) J_hist[t - 1] = J;
    launch_adam<double>(3 * nc, yd, f.ybar, mm, vv, lr, 0.9, 0.999, 1e-8, t, double(kClamp), s);
  }
  if (!st) {
    double J = 0.0;
    st = f.objective(yd, 0.0, false, &J);
    if (!st && J_hist) J_hist[steps] = J;
  }
  if (!st) launch_d2f(3 * nc, yd, y_out, s);
  (void)hipStreamSynchronize(s);
  ctx->use_scaling = saved;
  return st;
}

int mfgmg_set_scaling(mfgmg_ctx* ctx, int32_t level, const float* y, void* stream) {
  if (ctx && ctx->mesh && ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "the learned scaling is built for Q2-Q1");
  int st = check_ready(ctx, level, true);
  if (st) return st;
  LevelDev& L = ctx->lv[size_t(level)];
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!y) {
    L.scaled = false;
    return MFGMG_OK;
  }
  const int64_t n = 3 * L.v.nnode, nc = L.v.ncell;
  if (!L.minv_s_d) L.minv_s_d = ctx->dalloc<double>(size_t(n));
  if (!L.minv_s_f) L.minv_s_f = ctx->dalloc<float>(size_t(n));
  if (!L.node_count) {
    L.node_count = ctx->dalloc<double>(size_t(L.v.nnode));
    if (!L.node_count) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
    double* acc0 = nullptr;
    double* y0 = nullptr;
    HIPCHK(hipMalloc(&acc0, size_t(n) * sizeof(double)));
    HIPCHK(hipMalloc(&y0, size_t(3 * nc) * sizeof(double)));
    launch_fill(L.v.nnode, 0.0, L.node_count, s);
    launch_fill(3 * nc, 0.0, y0, s);
    launch_scaling_accum(L.v, y0, acc0, L.node_count, s);
    HIPCHK(hipStreamSynchronize(s));
    (void)hipFree(acc0);
    (void)hipFree(y0);
  }
  if (!L.minv_s_d || !L.minv_s_f) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
  double *acc = nullptr, *yd = nullptr;
  HIPCHK(hipMalloc(&acc, size_t(n) * sizeof(double)));
  HIPCHK(hipMalloc(&yd, size_t(3 * nc) * sizeof(double)));
  launch_f2d(3 * nc, y, yd, s);
  launch_fill(n, 0.0, acc, s);
  launch_scaling_accum(L.v, yd, acc, nullptr, s);
  launch_scaling_finish(L.v.nnode, acc, L.node_count, L.minv_d, nullptr, L.minv_s_d, L.minv_s_f, s);
  st = lanczos_lambda(ctx, level, L.minv_s_d, &L.lambda_s, s);
  (void)hipFree(acc);
  (void)hipFree(yd);
  if (st) return st;
  L.scaled = true;
  return MFGMG_OK;
}

int mfgmg_use_scaling(mfgmg_ctx* ctx, int32_t on) {
  if (!ctx) return MFGMG_ERR_INVALID;
  ctx->use_scaling = on != 0;
  return MFGMG_OK;
}

int mfgmg_vcycle_factor(mfgmg_ctx* ctx, double* rho, void* stream) {
  if (!ctx || !rho) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  *rho = vcycle_factor(ctx, static_cast<hipStream_t>(stream), MFGMG_FP64, 3);
  return *rho >= 0 ? MFGMG_OK : ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
}

int mfgmg_mlp_forward(const float* w, const float* x, int64_t n, float* y, float* cache, void* stream) {
  if (!w || !x || !y || !cache || n < 0) return MFGMG_ERR_INVALID;
  launch_mlp_forward(w, x, n, y, cache, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? MFGMG_OK : MFGMG_ERR_HIP;
}

int mfgmg_mlp_backward(const float* w, const float* x, const float* cache, const float* dy, int64_t n, float* dw,
                       float* work, void* stream) {
  if (!w || !x || !cache || !dy || !dw || !work || n < 1) return MFGMG_ERR_INVALID;
  float* part = work + 260 * n;
  launch_mlp_backward(w, x, cache, dy, n, dw, work, part, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? MFGMG_OK : MFGMG_ERR_HIP;
}

int64_t mfgmg_mlp_work_size(int64_t n) { return 260 * n + ((n + 63) / 64) * kParams; }

int mfgmg_mlp_adam(float* w, const float* dw, float* m, float* v, int64_t step, double lr, void* stream) {
  if (!w || !dw || !m || !v || step < 1 || !(lr > 0)) return MFGMG_ERR_INVALID;
  launch_adam<float>(kParams, w, dw, m, v, lr, 0.9, 0.999, 1e-8, step, 0.0, static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? MFGMG_OK : MFGMG_ERR_HIP;
}

int mfgmg_mlp_train(float* w, const float* feats, const float* targets, int64_t n, int32_t epochs, int32_t batch,
                    double lr, uint64_t seed, double* loss_hist, void* stream) {
  if (!w || !feats || !targets || n < 1 || epochs < 0 || batch < 1) return MFGMG_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t B = std::min<int64_t>(batch, n);
  float *m = nullptr, *v = nullptr, *xb = nullptr, *tb = nullptr, *yb = nullptr, *cache = nullptr, *dy = nullptr,
        *dw = nullptr, *work = nullptr;
  int64_t* idx = nullptr;
  double* loss = nullptr;
  auto fail = [&]() {
    for (void* p : {(void*)m, (void*)v, (void*)xb, (void*)tb, (void*)yb, (void*)cache, (void*)dy, (void*)dw,
                    (void*)work, (void*)idx, (void*)loss})
      if (p) (void)hipFree(p);
  };
  if (hipMalloc(&m, kParams * sizeof(float)) || hipMalloc(&v, kParams * sizeof(float)) ||
      hipMalloc(&xb, size_t(B) * kIn * sizeof(float)) || hipMalloc(&tb, size_t(B) * kOut * sizeof(float)) ||
      hipMalloc(&yb, size_t(B) * kOut * sizeof(float)) || hipMalloc(&cache, size_t(B) * kCache * sizeof(float)) ||
      hipMalloc(&dy, size_t(B) * kOut * sizeof(float)) || hipMalloc(&dw, kParams * sizeof(float)) ||
      hipMalloc(&work, size_t(mfgmg_mlp_work_size(B)) * sizeof(float)) ||
      hipMalloc(&idx, size_t(n) * sizeof(int64_t)) || hipMalloc(&loss, sizeof(double))) {
    fail();
    return MFGMG_ERR_NOMEM;
  }
  (void)hipMemsetAsync(m, 0, kParams * sizeof(float), s);
  (void)hipMemsetAsync(v, 0, kParams * sizeof(float), s);
  std::vector<int64_t> perm(static_cast<size_t>(n));
  int64_t step = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    // Fisher-Yates shuffle driven by SplitMix64 (seed, epoch, position)
    for (int64_t i = 0; i < n; ++i) perm[size_t(i)] = i;
    for (int64_t i = n - 1; i > 0; --i) {
      const double u = 0.5 * (splitmix_pm1(seed + 1000003ULL * uint64_t(ep), uint64_t(i)) + 1.0);
      int64_t j = int64_t(u * double(i + 1));
      if (j > i) j = i;
      std::swap(perm[size_t(i)], perm[size_t(j)]);
    }
    (void)hipMemcpyAsync(idx, perm.data(), size_t(n) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    (void)hipMemsetAsync(loss, 0, sizeof(double), s);
    for (int64_t b0 = 0; b0 < n; b0 += B) {
      const int64_t nb = std::min(B, n - b0);
      launch_gather_rows(feats, kIn, idx + b0, nb, xb, s);
      launch_gather_rows(targets, kOut, idx + b0, nb, tb, s);
      launch_mlp_forward(w, xb, nb, yb, cache, s);
      launch_mse(nb * kOut, yb, tb, dy, 2.0f / float(nb * kOut), loss, s);
      launch_mlp_backward(w, xb, cache, dy, nb, dw, work, work + 260 * nb, s);
      ++step;
      launch_adam<float>(kParams, w, dw, m, v, lr, 0.9, 0.999, 1e-8, step, 0.0, s);
    }
    if (loss_hist) {
      double l = 0.0;
      (void)hipMemcpyAsync(&l, loss, sizeof(double), hipMemcpyDeviceToHost, s);
      (void)hipStreamSynchronize(s);
      loss_hist[ep] = l / double(n * kOut);
    }
  }
  (void)hipStreamSynchronize(s);
  const bool ok = hipGetLastError() == hipSuccess;
  fail();
  return ok ? MFGMG_OK : MFGMG_ERR_HIP;
}

int mfgmg_apply_mlp(mfgmg_ctx* ctx, const float* w, int32_t guard, int32_t* used, double* factors, void* stream) {
  if (ctx && ctx->mesh && ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "the learned scaling is built for Q2-Q1");
  if (!ctx || !w || guard < MFGMG_GUARD_NONE || guard > MFGMG_GUARD_FP32) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int L = ctx->mesh->L();
  for (int l = 2; l <= L; ++l) {
    const int64_t nc = ctx->lv[size_t(l)].v.ncell;
    float *feat = nullptr, *y = nullptr, *cache = nullptr;
    HIPCHK(hipMalloc(&feat, size_t(nc) * kIn * sizeof(float)));
    HIPCHK(hipMalloc(&y, size_t(nc) * kOut * sizeof(float)));
    HIPCHK(hipMalloc(&cache, size_t(nc) * kCache * sizeof(float)));
    int st = mfgmg_features(ctx, l, feat, stream);
    if (!st) {
      launch_mlp_forward(w, feat, nc, y, cache, s);
      st = mfgmg_set_scaling(ctx, l, y, stream);
    }
    (void)hipFree(feat);
    (void)hipFree(y);
    (void)hipFree(cache);
    if (st) return st;
  }
  int32_t use = 1;
  if (guard) {
    // both factors with the V-cycle precision of the solve the scaling is for
    const int prec = guard == MFGMG_GUARD_FP32 ? MFGMG_FP32 : MFGMG_FP64;
    const bool saved = ctx->use_scaling;
    ctx->use_scaling = false;
    const double plain = vcycle_factor(ctx, s, prec, kGuardSteps);
    ctx->use_scaling = true;
    const double lrn = vcycle_factor(ctx, s, prec, kGuardSteps);
    ctx->use_scaling = saved;
    if (plain < 0 || lrn < 0) return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
    if (factors) factors[0] = plain, factors[1] = lrn;
    if (!(lrn < (1.0 - kGuardMargin) * plain)) {
      use = 0;
      for (int l = 2; l <= L; ++l) ctx->lv[size_t(l)].scaled = false;
    }
  }
  if (used) *used = use;
  return MFGMG_OK;
}

}  // extern "C"
