// Local-smoothing V-cycle on the device: the multigrid hierarchy of level
// meshes that hold the cells of one refinement level each (the method the
// paper cites in Sec. 2.2.1), beside the global-coarsening V-cycle of api.hip.
//
// Levels 1 .. base are the uniform global-coarsening levels (every cell of
// the level exists, no refinement edge: there the local cycle is the global
// one).  A finer level l holds the cells of level exactly l; its smoother
// works with the refinement-edge nodes fixed (operator `a`), and the same
// cells with those nodes free (operator `k`) give the interface terms:
//   copy:  every free leaf node to the finest level holding it (defect d_l);
//   level l:  y = S_l(d on inner nodes), t = d - K y on all level nodes,
//             d_{l-1} += R t, recursion, z = P y_{l-1} (edge rows kept),
//             y += z, post-smoothing of A_II y_I = d_I - K_IE y_E from y;
//   copy back: every free leaf node from the finest level holding it.
// Level vectors are node-major like the global-coarsening ones.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mfgmg.h"
#include "ctx.h"
#include "mesh.h"
#include "ops.h"

namespace mfgmg {
namespace detail {

namespace {

constexpr int kLsBlock = 256;
inline unsigned ls_grid(int64_t n) {
  const int64_t g = (n + kLsBlock - 1) / kLsBlock;
  return unsigned(g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g));
}

// d[3 node[i] + c] = b[3 leaf[i] + c]
template <typename T>
__global__ void k_ls_copy_in(int64_t n, const int32_t* __restrict__ leaf, const int32_t* __restrict__ node,
                             const T* __restrict__ b, T* __restrict__ d) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < 3 * n; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / 3, c = e - 3 * i;
    d[3 * int64_t(node[i]) + c] = b[3 * int64_t(leaf[i]) + c];
  }
}

// x[3 leaf[i] + c] = y[3 node[i] + c]
template <typename T>
__global__ void k_ls_copy_out(int64_t n, const int32_t* __restrict__ leaf, const int32_t* __restrict__ node,
                              const T* __restrict__ y, T* __restrict__ x) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < 3 * n; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e / 3, c = e - 3 * i;
    x[3 * int64_t(leaf[i]) + c] = y[3 * int64_t(node[i]) + c];
  }
}

// out = a on nodes of kind `keep`, 0 elsewhere
template <typename T>
__global__ void k_ls_mask(int64_t nn, const uint8_t* __restrict__ kind, int keep, const T* __restrict__ a,
                          T* __restrict__ out) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < 3 * nn; e += int64_t(gridDim.x) * blockDim.x)
    out[e] = kind[e / 3] == keep ? a[e] : T(0);
}

// t = d - t
template <typename T>
__global__ void k_ls_sub(int64_t n, const T* __restrict__ d, T* __restrict__ t) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    t[e] = d[e] - t[e];
}

// y += a
template <typename T>
__global__ void k_ls_add(int64_t n, const T* __restrict__ a, T* __restrict__ y) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    y[e] += a[e];
}

// post-smoothing right-hand side: inner d - w (w = K y_E), edge y (kept), boundary 0
template <typename T>
__global__ void k_ls_post_rhs(int64_t nn, const uint8_t* __restrict__ kind, const T* __restrict__ d,
                              const T* __restrict__ w, const T* __restrict__ y, T* __restrict__ rhs) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < 3 * nn; e += int64_t(gridDim.x) * blockDim.x) {
    const int k = kind[e / 3];
    rhs[e] = k == 0 ? d[e] - w[e] : (k == 2 ? y[e] : T(0));
  }
}

template <typename T>
__global__ void k_ls_zero(int64_t n, T* __restrict__ y) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    y[e] = T(0);
}

// cell viscosity of a local level from the global-coarsening level (the same octree node)
__global__ void k_ls_gather_mu(int64_t nc, const int32_t* __restrict__ gc, const double* __restrict__ mu_g,
                               double* __restrict__ mu, float* __restrict__ mu_f) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < nc; c += int64_t(gridDim.x) * blockDim.x) {
    const double v = mu_g[gc[c]];
    mu[c] = v;
    mu_f[c] = float(v);
  }
}

template <typename T>
constexpr int pidx() {
  return sizeof(T) == 4 ? 0 : 1;
}

template <typename T>
T* wk(LevelDev& d, int k) {
  return static_cast<T*>(d.work[pidx<T>()][k]);
}

// the level vectors of level `ell` (a local level or the uniform base):
// defect, correction, and a scratch vector of the level's size
template <typename T>
void level_vectors(mfgmg_ctx* ctx, int ell, T** d, T** y, T** tmp, int64_t* n) {
  const int base = ctx->mesh->local_base();
  if (ell == base) {
    LevelDev& g = ctx->lv[size_t(ell)];
    *d = wk<T>(g, 0), *y = wk<T>(g, 1), *tmp = wk<T>(g, 2);
    *n = 3 * g.v.nnode;
  } else {
    LocalDev& l = ctx->ls[size_t(ell)];
    *d = wk<T>(l.a, 0), *y = wk<T>(l.a, 1), *tmp = static_cast<T*>(l.ext[pidx<T>()][0]);
    *n = 3 * l.a.v.nnode;
  }
}

template <typename T>
void ls_level(mfgmg_ctx* ctx, int ell, hipStream_t s) {
  const int base = ctx->mesh->local_base();
  if (ell == base) {
    LevelDev& g = ctx->lv[size_t(ell)];
    vcycle<T>(ctx, ell, wk<T>(g, 0), wk<T>(g, 1), s);
    return;
  }
  LocalDev& l = ctx->ls[size_t(ell)];
  const int64_t nn = l.a.v.nnode, n = 3 * nn;
  T *d = wk<T>(l.a, 0), *y = wk<T>(l.a, 1), *t = wk<T>(l.a, 2);
  T *z = static_cast<T*>(l.ext[pidx<T>()][0]), *w = static_cast<T*>(l.ext[pidx<T>()][1]);
  T *dc, *yc, *tc;
  int64_t ncn;
  level_vectors<T>(ctx, ell - 1, &dc, &yc, &tc, &ncn);
  // pre-smoothing on the inner nodes, from zero
  k_ls_mask<T><<<ls_grid(n), kLsBlock, 0, s>>>(nn, l.kind, 0, d, t);
  smooth_on<T>(ctx, l.a, t, y, true, s);
  // residual on every level node, the interface rows included: t = d - K y
  launch_vmult<T>(l.k.v, y, t, s);
  k_ls_sub<T><<<ls_grid(n), kLsBlock, 0, s>>>(n, d, t);
  launch_restrict<T>(ncn / 3, l.a.R_ptr, l.a.R_col, l.a.R_w, t, nullptr, tc, s);
  k_ls_add<T><<<ls_grid(ncn), kLsBlock, 0, s>>>(ncn, tc, dc);
  ls_level<T>(ctx, ell - 1, s);
  // coarse correction, kept on the refinement edge
  launch_prolong<T>(nn, l.a.P_ptr, l.a.P_col, l.a.P_w, yc, z, false, s);
  k_ls_add<T><<<ls_grid(n), kLsBlock, 0, s>>>(n, z, y);
  // post-smoothing of A_II y_I = d_I - K_IE y_E, the edge values kept
  k_ls_mask<T><<<ls_grid(n), kLsBlock, 0, s>>>(nn, l.kind, 2, y, t);
  launch_vmult<T>(l.k.v, t, w, s);
  k_ls_post_rhs<T><<<ls_grid(n), kLsBlock, 0, s>>>(nn, l.kind, d, w, y, t);
  smooth_on<T>(ctx, l.a, t, y, false, s);
}

}  // namespace

// Device data of the local levels (once per mesh) and their viscosity,
// inverse diagonals and Chebyshev bounds (once per viscosity).
int local_setup(mfgmg_ctx* ctx, hipStream_t s) {
  const Mesh& m = *ctx->mesh;
  const int L = m.L(), base = m.local_base();
  if (base >= L) return MFGMG_OK;   // uniform leaf: the local cycle is the global one
  if (!ctx->ls_ready) {
    ctx->ls.assign(size_t(L + 1), LocalDev{});
    for (int ell = base + 1; ell <= L; ++ell) {
      const LocalLevel& h = m.local_level(ell);
      LocalDev& l = ctx->ls[size_t(ell)];
      int st = upload_level(ctx, h.mesh, l.a, false, false, true, true);
      if (st) return st;
      Level free_edge = h.mesh;   // the same cells with the refinement edge free
      for (int64_t i = 0; i < free_edge.nnode; ++i)
        if (h.kind[size_t(i)] == 2) free_edge.ntype[size_t(i)] = NODE_FREE;
      free_edge.P_ptr.clear(), free_edge.P_col.clear(), free_edge.P_w.clear();
      free_edge.R_ptr.clear(), free_edge.R_col.clear(), free_edge.R_w.clear();
      st = upload_level(ctx, free_edge, l.k, false, false, false, false);
      if (st) return st;
      l.k.v.mu_d = l.a.mu_d;
      l.k.v.mu_f = l.a.mu_f;
      l.kind = ctx->upload(h.kind);
      l.gc_cell = ctx->upload(h.gc_cell);
      l.copy_leaf = ctx->upload(h.copy_leaf);
      l.copy_node = ctx->upload(h.copy_node);
      l.ncopy = int64_t(h.copy_leaf.size());
      const size_t n = size_t(3 * h.mesh.nnode);
      l.ext[0][0] = ctx->dalloc<float>(n), l.ext[0][1] = ctx->dalloc<float>(n);
      l.ext[1][0] = ctx->dalloc<double>(n), l.ext[1][1] = ctx->dalloc<double>(n);
      if (!l.kind || !l.gc_cell || !l.ext[0][0] || !l.ext[0][1] || !l.ext[1][0] || !l.ext[1][1] ||
          (l.ncopy && (!l.copy_leaf || !l.copy_node)))
        return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
    }
    ctx->ls_base_leaf = ctx->upload(m.local_base_copy_leaf());
    ctx->ls_base_node = ctx->upload(m.local_base_copy_node());
    ctx->ls_base_ncopy = int64_t(m.local_base_copy_leaf().size());
    if (ctx->ls_base_ncopy && (!ctx->ls_base_leaf || !ctx->ls_base_node))
      return ctx->set(MFGMG_ERR_NOMEM, "device allocation failed");
    ctx->ls_ready = true;
  }
  if (!ctx->ls_mu_ready) {
    int64_t nmax = 0;
    for (int ell = base + 1; ell <= L; ++ell) nmax = std::max(nmax, 3 * ctx->ls[size_t(ell)].a.v.nnode);
    double* dtmp = nullptr;
    HIPCHK(hipMalloc(&dtmp, size_t(nmax) * sizeof(double)));
    for (int ell = base + 1; ell <= L; ++ell) {
      LocalDev& l = ctx->ls[size_t(ell)];
      const int64_t nc = l.a.v.ncell;
      k_ls_gather_mu<<<ls_grid(nc), kLsBlock, 0, s>>>(nc, l.gc_cell, ctx->lv[size_t(ell)].mu_d, l.a.mu_d, l.a.mu_f);
      launch_fill(3 * l.a.v.nnode, 0.0, dtmp, s);
      launch_diag(l.a.v, ctx->khat_d, dtmp, s);
      launch_invert_diag(l.a.v, dtmp, l.a.minv_d, l.a.minv_f, s);
      const int st = lanczos_on(ctx, l.a, m.local_level(ell).mesh, l.a.minv_d, &l.a.lambda, s);
      if (st) {
        (void)hipFree(dtmp);
        return st;
      }
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipFree(dtmp));
    ctx->ls_mu_ready = true;
  }
  return MFGMG_OK;
}

// x = V_local(b) on leaf vectors (x zero on constrained leaf dofs)
template <typename T>
void local_vcycle(mfgmg_ctx* ctx, const T* b, T* x, hipStream_t s) {
  const Mesh& m = *ctx->mesh;
  const int L = m.L(), base = m.local_base();
  if (base >= L) {
    vcycle<T>(ctx, L, b, x, s);
    return;
  }
  for (int ell = base; ell <= L; ++ell) {
    T *d, *y, *tmp;
    int64_t n;
    level_vectors<T>(ctx, ell, &d, &y, &tmp, &n);
    k_ls_zero<T><<<ls_grid(n), kLsBlock, 0, s>>>(n, d);
    if (ell == base) {
      if (ctx->ls_base_ncopy)
        k_ls_copy_in<T><<<ls_grid(3 * ctx->ls_base_ncopy), kLsBlock, 0, s>>>(ctx->ls_base_ncopy, ctx->ls_base_leaf,
                                                                               ctx->ls_base_node, b, d);
    } else {
      const LocalDev& l = ctx->ls[size_t(ell)];
      if (l.ncopy) k_ls_copy_in<T><<<ls_grid(3 * l.ncopy), kLsBlock, 0, s>>>(l.ncopy, l.copy_leaf, l.copy_node, b, d);
    }
  }
  ls_level<T>(ctx, L, s);
  const int64_t nleaf = 3 * ctx->lv[size_t(L)].v.nnode;
  k_ls_zero<T><<<ls_grid(nleaf), kLsBlock, 0, s>>>(nleaf, x);
  for (int ell = base; ell <= L; ++ell) {
    T *d, *y, *tmp;
    int64_t n;
    level_vectors<T>(ctx, ell, &d, &y, &tmp, &n);
    if (ell == base) {
      if (ctx->ls_base_ncopy)
        k_ls_copy_out<T><<<ls_grid(3 * ctx->ls_base_ncopy), kLsBlock, 0, s>>>(ctx->ls_base_ncopy, ctx->ls_base_leaf,
                                                                                ctx->ls_base_node, y, x);
    } else {
      const LocalDev& l = ctx->ls[size_t(ell)];
      if (l.ncopy) k_ls_copy_out<T><<<ls_grid(3 * l.ncopy), kLsBlock, 0, s>>>(l.ncopy, l.copy_leaf, l.copy_node, y, x);
    }
  }
}

template void local_vcycle<float>(mfgmg_ctx*, const float*, float*, hipStream_t);
template void local_vcycle<double>(mfgmg_ctx*, const double*, double*, hipStream_t);

}  // namespace detail
}  // namespace mfgmg

using namespace mfgmg;
using namespace mfgmg::detail;

extern "C" {

int mfgmg_local_levels(const mfgmg_ctx* ctx, int32_t* base, int64_t* n_cells, int64_t* n_nodes) {
  if (!ctx || !base || !n_cells || !n_nodes) return MFGMG_ERR_INVALID;
  if (!ctx->mesh || !ctx->mesh->finalized()) return MFGMG_ERR_STATE;
  // local smoothing: Q2-Q1 with u = 0 only
  if (ctx->mesh->noflux() || ctx->mesh->velocity_degree() != 2) return MFGMG_ERR_INVALID;
  const Mesh& m = *ctx->mesh;
  *base = m.local_base();
  for (int ell = 0; ell <= MFGMG_MAX_LEVELS; ++ell) n_cells[ell] = n_nodes[ell] = 0;
  for (int ell = 1; ell <= m.L(); ++ell) {
    const Level& h = ell <= m.local_base() ? m.level(ell) : m.local_level(ell).mesh;
    n_cells[ell] = h.ncell;
    n_nodes[ell] = h.nnode;
  }
  return MFGMG_OK;
}

int mfgmg_local_nodes(const mfgmg_ctx* ctx, int32_t level, int64_t* keys, uint8_t* kinds) {
  if (!ctx || !keys || !kinds) return MFGMG_ERR_INVALID;
  if (!ctx->mesh || !ctx->mesh->finalized()) return MFGMG_ERR_STATE;
  // local smoothing: Q2-Q1 with u = 0 only
  if (ctx->mesh->noflux() || ctx->mesh->velocity_degree() != 2) return MFGMG_ERR_INVALID;
  const Mesh& m = *ctx->mesh;
  if (level <= m.local_base() || level > m.L()) return MFGMG_ERR_INVALID;
  const LocalLevel& h = m.local_level(level);
  for (int64_t i = 0; i < h.mesh.nnode; ++i) keys[i] = h.mesh.key[size_t(i)], kinds[i] = h.kind[size_t(i)];
  return MFGMG_OK;
}

int mfgmg_local_transfer(const mfgmg_ctx* ctx, int32_t level, int64_t* nnz, int64_t* ptr, int64_t* col, double* w) {
  if (!ctx || !nnz) return MFGMG_ERR_INVALID;
  if (!ctx->mesh || !ctx->mesh->finalized()) return MFGMG_ERR_STATE;
  // local smoothing: Q2-Q1 with u = 0 only
  if (ctx->mesh->noflux() || ctx->mesh->velocity_degree() != 2) return MFGMG_ERR_INVALID;
  const Mesh& m = *ctx->mesh;
  if (level <= m.local_base() || level > m.L()) return MFGMG_ERR_INVALID;
  const Level& h = m.local_level(level).mesh;
  *nnz = int64_t(h.P_col.size());
  if (!ptr && !col && !w) return MFGMG_OK;
  if (!ptr || !col || !w) return MFGMG_ERR_INVALID;
  for (size_t i = 0; i < h.P_ptr.size(); ++i) ptr[i] = h.P_ptr[i];
  for (size_t i = 0; i < h.P_col.size(); ++i) col[i] = h.P_col[i], w[i] = h.P_w[i];
  return MFGMG_OK;
}

int mfgmg_vcycle_local(mfgmg_ctx* ctx, mfgmg_prec prec, const void* rhs, void* x, void* stream) {
  if (!ctx || !rhs || !x || rhs == x || (prec != MFGMG_FP32 && prec != MFGMG_FP64)) return MFGMG_ERR_INVALID;
  if (!ctx->mu_ready) return ctx->set(MFGMG_ERR_STATE, "set_viscosity first");
  if (ctx->mesh->noflux() || ctx->mesh->velocity_degree() != 2)
    return ctx->set(MFGMG_ERR_INVALID, "local smoothing is built for Q2-Q1 with the Dirichlet condition");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int st = local_setup(ctx, s);
  if (st) return st;
  if (prec == MFGMG_FP64)
    local_vcycle<double>(ctx, static_cast<const double*>(rhs), static_cast<double*>(x), s);
  else
    local_vcycle<float>(ctx, static_cast<const float*>(rhs), static_cast<float*>(x), s);
  HIPCHK(hipGetLastError());
  return MFGMG_OK;
}

}  // extern "C"
