// Device kernels and their launchers (host-callable, async on a stream).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfgmg {

// Velocity slots (cell tables and block lattices) hold node >= 0 for a free
// node, -1 for a Dirichlet node, -(2+h) for hanging row h (-2 in blocks).  A
// free node's slot carries in bits 28..30 the components fixed by the
// no-normal-flux condition (bit 28 + c: component c), zero under u = 0;
// node indices stay below 2^28.
constexpr int kSlotFixShift = 28;
constexpr int32_t kSlotNodeMask = (int32_t(1) << kSlotFixShift) - 1;
__host__ __device__ __forceinline__ int32_t slot_node(int32_t s) { return s & kSlotNodeMask; }
// for a free slot: true when component c is fixed
__host__ __device__ __forceinline__ bool slot_fixed(int32_t s, int c) { return (s >> (kSlotFixShift + c)) & 1; }

// Blocks of B^3 same-level cells of a non-uniform level: node-box slots
// [(2B+1)^3] per block (x fastest; node >= 0 free, -1 Dirichlet, -2
// hanging), cell indices [B^3], and the hanging points' masters as lattice
// points of the same block: entries hoff[b] .. hoff[b+1] of block b pack
// (point | master << 10 | (b mod blocks-per-workgroup) << 20) with weight hw.
struct DevBlocks {
  const int32_t* slots = nullptr;
  const int32_t* cells = nullptr;
  const int32_t* hoff = nullptr;
  const int32_t* hent = nullptr;
  const double* hw_d = nullptr;
  const float* hw_f = nullptr;
  // the same entries grouped per workgroup for the velocity kernel, without
  // atomics: by hanging point (consecutive in hent; group k of workgroup g is
  // [g1[k], g1[k + 1]) for k in [g1off[g], g1off[g + 1] - 1)), and sorted by
  // master (hent2 / hw2_*, groups g2 / g2off)
  const int32_t* g1off = nullptr;
  const int32_t* g1 = nullptr;
  const int32_t* hent2 = nullptr;
  const double* hw2_d = nullptr;
  const float* hw2_f = nullptr;
  const int32_t* g2off = nullptr;
  const int32_t* g2 = nullptr;
  int64_t n = 0;
  // leaf only: the Q1 pressure lattice [(B+1)^3] of each block (node >= 0,
  // -2 hanging) and its hanging points' masters, packed as above
  const int32_t* pslots = nullptr;
  const int32_t* phoff = nullptr;
  const int32_t* phent = nullptr;
  const double* phw = nullptr;
};

// Device view of one level mesh.
struct DevLevel {
  int ell = 0;
  int64_t ncell = 0, nnode = 0;
  bool uniform = false;
  int64_t n_edge = 0;
  // general (non-uniform) levels
  const int32_t* slots = nullptr;   // [27*ncell]: node >= 0 free, -1 Dirichlet, -(2+h) hanging row h
  const int8_t* clev = nullptr;     // [ncell]
  // [nnode]: bit c set when dof (node, c) is constrained (Dirichlet and
  // hanging nodes: all three; fixed components of no-normal-flux nodes)
  const uint8_t* cmask = nullptr;
  bool noflux = false;              // u . n = 0 on the boundary (general levels only)
  // Q3-Q2 lattice levels (k = 2): the Q3 kernels, FP64 transfer weights of
  // the prolongation from the level below (CSR of the LevelDev) and of its
  // transpose, the diagonal of the unit element matrix [192]
  bool q3 = false;
  float* q3_halo_f = nullptr;       // operator halo slots (q3_halo_words entries)
  double* q3_halo_d = nullptr;
  const double* q3_Pw = nullptr;
  const double* q3_Rw = nullptr;
  // separable transfers from the level below: the 1D factor (fine coordinate
  // -> 4 coarse coordinates from q3_pc0, weights q3_pw) and its transpose as
  // CSR over coarse coordinates
  const int32_t* q3_pc0 = nullptr;
  const double* q3_pw = nullptr;
  const int32_t* q3_rptr = nullptr;
  const int32_t* q3_rcol = nullptr;
  const double* q3_rw = nullptr;
  // two scratch vectors of this level's size for the separable transfers
  // from the level below (the smoother's r and d, free while a transfer runs)
  float* tr_s1_f = nullptr;
  float* tr_s2_f = nullptr;
  double* tr_s1_d = nullptr;
  double* tr_s2_d = nullptr;
  const double* q3_kdiag = nullptr;
  const int64_t* hptr = nullptr;    // hanging CSR
  const int32_t* hmaster = nullptr;
  const float* hw_f = nullptr;
  const double* hw_d = nullptr;
  const int32_t* hang_cells = nullptr;  // cells with at least one hanging node
  int64_t n_hang_cells = 0;
  const int32_t* reg_cells = nullptr;   // the other cells
  int64_t n_reg_cells = 0;
  // operator partition: blocks of 4^3 and 2^3 same-level cells, and the
  // remaining single cells with and without hanging nodes
  DevBlocks blk4, blk2;
  const int32_t* single_reg = nullptr;
  int64_t n_single_reg = 0;
  const int32_t* single_hang = nullptr;
  int64_t n_single_hang = 0;
  const int64_t* cons_dofs = nullptr;   // constrained velocity dofs (3 node + c)
  int64_t n_cons = 0;
  const int64_t* hnode = nullptr;       // node of each hanging row
  int64_t nhang = 0;
  // per-cell viscosity
  const double* mu_d = nullptr;
  const float* mu_f = nullptr;
  // uniform levels: halo slots of the brick kernel (brick_halo_words entries)
  float* halo_f = nullptr;
  double* halo_d = nullptr;
  // non-uniform levels: the block kernels write the values of their free
  // face points to slots (3 values per lattice point of every block: 4^3
  // blocks first, then 2^3 blocks), and a gather kernel adds, for every node
  // that is a free face point of some block, its slots into y:
  // face_ent[face_ptr[i] .. face_ptr[i+1]) are the slots of node face_node[i]
  float* fslot_f = nullptr;
  double* fslot_d = nullptr;
  int64_t fslot_blk2 = 0;               // first slot of the 2^3 blocks
  const int32_t* face_node = nullptr;
  const int32_t* face_ptr = nullptr;
  const int32_t* face_ent = nullptr;
  int64_t n_face = 0;
  // the leaf's pressure mass blocks do the same on their Q1 lattices (one
  // value per lattice point of every block)
  double* pfslot = nullptr;
  int64_t pfslot_blk2 = 0;
  const int32_t* pface_node = nullptr;
  const int32_t* pface_ptr = nullptr;
  const int32_t* pface_ent = nullptr;
  int64_t n_pface = 0;
};

// entries of the brick kernel's halo buffer on a uniform level of n cells per
// edge (0 when the brick kernel does not apply)
template <typename T>
int64_t brick_halo_words(int64_t n);

template <typename T>
const T* mu_of(const DevLevel& L);

// y = A x on a level (identity on constrained dofs).  x, y must not alias.
// init = false: y += cell contributions only (constrained entries untouched)
template <typename T>
void launch_vmult(const DevLevel& L, const T* x, T* y, hipStream_t s, bool init = true);

// diag(A) accumulation (free dofs) into d (zeroed by the caller), then
// minv = 1/d on free dofs and 1 on constrained dofs.
void launch_diag(const DevLevel& L, const double* khat_full_dev, double* d, hipStream_t s);
void launch_invert_diag(const DevLevel& L, const double* d, double* minv_d, float* minv_f, hipStream_t s);

// Chebyshev updates in the residual-recurrence form of Saad's Alg. 12.1
// (r -= t; d = alpha d + beta minv r; x += d), used by the learned-scaling
// fit and the pressure Chebyshev map.
template <typename T>
void launch_cheb_init0(int64_t n, const T* b, const T* minv, T* r, T* d, T* x, double inv_theta, hipStream_t s);
template <typename T>
void launch_cheb_init(int64_t n, const T* b, const T* t, const T* minv, T* r, T* d, T* x, double inv_theta,
                      hipStream_t s);
template <typename T>
void launch_cheb_step(int64_t n, const T* t, const T* minv, T* r, T* d, T* x, double alpha, double beta,
                      hipStream_t s);
// With p.tn set, the smoother's updates (launch_chebx_*) also prepare the
// output of the next operator call on a level whose operator starts with an
// initialisation kernel: tn = (constrained ? src : 0), src the new x (from_x)
// or the new d; that call is then launch_vmult_prepared.  cmask: the level's
// constrained-component masks (general levels), else null and m = 2n + 1
// (uniform levels).
struct ChebPrep {
  void* tn = nullptr;
  const uint8_t* cmask = nullptr;
  int64_t m = 0;
  bool from_x = false;
};
// the smoother's form (residual b - A x formed each step, r not stored):
// init0 from x = 0; step: d = alpha d + beta minv (b - t), x += d (alpha = 0:
// d is not read).  p prepares t for the next operator call on x (from_x).
template <typename T>
void launch_chebx_init0(int64_t n, const T* b, const T* minv, T* d, T* x, double inv_theta, hipStream_t s,
                        const ChebPrep& p = ChebPrep());
template <typename T>
void launch_chebx_step(int64_t n, const T* b, const T* t, const T* minv, T* d, T* x, double alpha, double beta,
                       hipStream_t s, const ChebPrep& p = ChebPrep());
// true when launch_vmult<T> on L starts with an output initialisation kernel
// (every level but the uniform ones the brick kernel takes and the Q3 lattice
// levels)
template <typename T>
bool vmult_has_init(const DevLevel& L);
// y = A x like launch_vmult (init), for a y already holding x on the
// constrained dofs and 0 elsewhere (the initialisation kernel is skipped)
template <typename T>
void launch_vmult_prepared(const DevLevel& L, const T* x, T* y, hipStream_t s);

// transfers (node-level CSR, 3 components).  cm_fine / cm_coarse (may be
// null): constrained-component masks of the two levels; a masked component
// neither carries nor receives anything (no-normal-flux levels, where the
// node-level rows do not express the per-component condition)
template <typename T>
void launch_prolong(int64_t nfine, const int64_t* ptr, const int32_t* col, const float* w, const T* coarse, T* fine,
                    bool add, hipStream_t s, const uint8_t* cm_fine = nullptr, const uint8_t* cm_coarse = nullptr);
// coarse = R (b - t) (t may be null: coarse = R b)
template <typename T>
void launch_restrict(int64_t ncoarse, const int64_t* ptr, const int32_t* col, const float* w, const T* b, const T* t,
                     T* coarse, hipStream_t s, const uint8_t* cm_fine = nullptr, const uint8_t* cm_coarse = nullptr);

// level-aware transfers: structured kernels between two uniform levels,
// the CSR kernels otherwise
template <typename T>
void launch_prolong_level(const DevLevel& fine, const DevLevel& coarse, const int64_t* ptr, const int32_t* col,
                          const float* w, const T* xc, T* xf, bool add, hipStream_t s);
// (between two uniform levels the restriction runs in three one-axis passes
// through the scratch vectors s1 and s2, each of the fine level's size; they
// are not read elsewhere)
template <typename T>
void launch_restrict_level(const DevLevel& fine, const DevLevel& coarse, const int64_t* ptr, const int32_t* col,
                           const float* w, const T* b, const T* t, T* xc, T* s1, T* s2, hipStream_t s);

// coarse solve: x[free] = Ainv b[free], x[constrained] = b
template <typename T>
void launch_coarse(const T* Ainv, const int32_t* free_dofs, int nfree, int n, const T* b, T* x, hipStream_t s);
// One V-cycle on the uniform 4^3 level L with the coarse solve of the 2^3
// level Lc below it (Ainv, free_dofs, nfree as for launch_coarse), smoother
// M^-1 = minv on [lam / 15, lam], in a single workgroup; the same steps as
// smoothing, residual, restriction, coarse solve, prolongation and smoothing
// launched one by one.  Returns false (nothing launched) when L, Lc are not
// such levels (no-normal-flux and Q3 lattice levels are not).
template <typename T>
bool launch_vcycle_tail(const DevLevel& L, const DevLevel& Lc, const T* minv, const T* Ainv, const int32_t* free_dofs,
                        int nfree, double lam, const T* b, T* x, hipStream_t s);

// viscosity
void launch_harmonic_mu(int64_t ncell, const double* mu_qp, double* mu, hipStream_t s);
void launch_restrict_mu(int64_t ncell, const int32_t* src, const double* mu_fine, double* mu_coarse, hipStream_t s);
void launch_to_float(int64_t n, const double* a, float* b, hipStream_t s);
void launch_to_double(int64_t n, const float* a, double* b, hipStream_t s);

// reductions: result[0] = sum a*b (two-stage, deterministic); partial has >= 1024 doubles
void launch_dot(int64_t n, const double* a, const double* b, double* partial, double* result, hipStream_t s);
// result[j] = sum_i V[j*ldv + i] w[i], j < nv, and with_norm: result[nv] =
// w . w; partial has >= (nv + 1)*256 doubles
void launch_mdot(int64_t n, int nv, const double* V, int64_t ldv, const double* w, double* partial, double* result,
                 hipStream_t s, bool with_norm = false);
// w -= sum_j h[j] V[j*ldv + i] (j < nv), reading V once, and the products of
// the new w: dots: result[j] = V_j . w (j < nv), result[nv] = w . w; else
// result[0] = w . w.  partial has >= 65536 doubles.  Returns false (nothing
// launched) unless 1 <= nv <= kMupdateDotsMax.
constexpr int kMupdateDotsMax = 128;
bool launch_mupdate_dots(int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w, double* partial,
                         double* result, bool dots, hipStream_t s);
// w -= sum_j h[j] V[j*ldv + i]
void launch_mupdate(int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w, hipStream_t s);
// y = a*x + b*y
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
void launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s);
void launch_fill(int64_t n, double v, double* y, hipStream_t s);
void launch_fill_f(int64_t n, float v, float* y, hipStream_t s);
void launch_mul(int64_t n, const double* a, const double* b, double* y, hipStream_t s);

// leaf pressure operators (FP64)
struct DevPressure {
  int64_t np = 0;
  const int32_t* pslots = nullptr;   // [8*ncell]: node >= 0 free, -(2+h) hanging row h
  const int64_t* hptr = nullptr;
  const int32_t* hmaster = nullptr;
  const double* hw = nullptr;
  const int64_t* hang_nodes = nullptr;
  int64_t nh = 0;
  // uniform leaf only: pressure node of lattice point (Px, Py, Pz) of the
  // (n+1)^3 Q1 lattice, Px fastest
  const int32_t* plat = nullptr;
};
void launch_div(const DevLevel& L, const DevPressure& P, const double* u, double* p_out, hipStream_t s);
void launch_grad_add(const DevLevel& L, const DevPressure& P, const double* p, double* u_out, hipStream_t s);
// u_out = src + B^T p (src and u_out distinct)
void launch_grad_from(const DevLevel& L, const DevPressure& P, const double* p, const double* src, double* u_out,
                      hipStream_t s);
// p_out = M_p p; gate (device, may be null): when *gate != 0 the cell kernel is skipped
void launch_pmass(const DevLevel& L, const DevPressure& P, const double* p, double* p_out, hipStream_t s,
                  const double* gate = nullptr);
// the same without clearing p_out first (p_out must be zero on entry)
void launch_pmass_add(const DevLevel& L, const DevPressure& P, const double* p, double* p_out, hipStream_t s,
                      const double* gate = nullptr);
// Jacobi-CG on M_p with its scalars on the device (see ops.hip): setup of the
// scalars (sc[0] must hold r.z, q must be zero), and iteration k = 0, 1, ...
// (no host synchronisation; a no-op once sc[5] is set).  part holds
// kRedPartWords doubles.  p holds p_0 at iteration 0; on a uniform leaf the
// direction alternates between p (even k) and p_alt (odd k), elsewhere p_alt
// is not used.  On a uniform leaf the test of iteration k's residual runs at
// the start of iteration k + 1 (a batch that ends on the converging iteration
// leaves sc[5] for the next one to set); the iteration count in sc[6] is the
// same on both paths.
constexpr int64_t kRedPartWords = 256 * 256;
// start vectors: r = rhs, z = p = minv rhs, x = q = 0
void launch_cg_start(int64_t n, const double* rhs, const double* minv, double* r, double* z, double* p, double* x,
                     double* q, hipStream_t s);
// scalars: sc[0] must hold r.z and sc[7] r.r of the start residual; the
// threshold on r.r becomes rtol2 r.r (a zero r is done at once)
void launch_cg_setup(double* sc, double rtol2, hipStream_t s);
void launch_cg_pmass_iteration(const DevLevel& L, const DevPressure& P, const double* minv, double* x, double* r,
                               double* z, double* p, double* p_alt, double* q, double* part, double* sc, int k,
                               hipStream_t s);
// copy p_in on hanging pressure nodes into p_out
void launch_p_identity(const DevPressure& P, const double* p_in, double* p_out, hipStream_t s);
// resolve hanging values: u[h] = sum w u[m] (velocity) and p likewise
void launch_distribute_u(const DevLevel& L, double* u, hipStream_t s);
void launch_distribute_p(const DevPressure& P, double* p, hipStream_t s);
// zero the constrained velocity entries
void launch_zero_constrained(const DevLevel& L, double* u, hipStream_t s);
// rhs: b_u = C^T F from f at the Gauss points [ncell][27][3]
void launch_rhs(const DevLevel& L, const double* f_qp, double* b, hipStream_t s);

// upload element constants (K_hat diagonal, B_hat, M_hat) to constant memory
void set_element_constants(const double* khat_diag81, const double* bhat8x81, const double* mhat8x8);

// Q3-Q2 lattice levels (q3_ops.hip): 1D tables N [4x4], D [4x4], Gauss
// weights [4], P2 [4x3], Q2 mass M2 [3x3]; operator, diagonal, harmonic viscosity over 4^3
// Gauss points, right-hand side (b zeroed by the caller) and the Q2 pressure
// side on the leaf (B u, B^T p added; M_p p added; diag(M_p) added).  The
// operator writes every entry of y (identity rows on constrained dofs), or
// adds the cell terms to the free entries when accumulating.
void set_q3_constants(const double* N, const double* D, const double* w, const double* P2, const double* M2);
template <typename T>
void launch_vmult_q3(const DevLevel& L, const T* x, T* y, bool accumulate, hipStream_t s);
// scratch vector k (0 or 1) of level L's separable transfers, precision T
template <typename T>
inline T* tr_scratch(const DevLevel& L, int k);
template <>
inline float* tr_scratch<float>(const DevLevel& L, int k) {
  return k ? L.tr_s2_f : L.tr_s1_f;
}
template <>
inline double* tr_scratch<double>(const DevLevel& L, int k) {
  return k ? L.tr_s2_d : L.tr_s1_d;
}

// entries of a Q3 level's operator halo buffer (n cells per edge)
int64_t q3_halo_words(int64_t n);
// separable transfers between a Q3 lattice level F and the level below
// (three one-axis passes through F's scratch vectors); t may be null
template <typename T>
void launch_prolong_q3(const DevLevel& F, const T* xc, T* xf, bool add, hipStream_t s);
template <typename T>
void launch_restrict_q3(const DevLevel& F, const T* b, const T* t, T* xc, hipStream_t s);
void launch_diag_q3(const DevLevel& L, const double* kdiag, double* d, hipStream_t s);
void launch_harmonic_mu64(int64_t ncell, const double* mu_qp, double* mu, hipStream_t s);
void launch_rhs_q3(const DevLevel& L, const double* f_qp, double* b, hipStream_t s);
void launch_div_q3(const DevLevel& L, const double* u, double* p_out, hipStream_t s);
void launch_grad_q3(const DevLevel& L, const double* p, double* u_out, hipStream_t s);
void launch_pmass_q2(const DevLevel& L, const double* p, double* p_out, hipStream_t s, const double* gate = nullptr);
void launch_pmass_diag_q2(const DevLevel& L, double* dg, hipStream_t s);

}  // namespace mfgmg
