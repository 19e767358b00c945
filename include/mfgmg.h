/*
 * mfgmg.h -- matrix-free geometric multigrid for the variable-viscosity Stokes
 * problem on adaptive hexahedral meshes of the unit cube, on AMD MI355X (gfx950).
 *
 * Method: Clevenger & Heister, "Comparison between algebraic and matrix-free
 * geometric multigrid for a Stokes problem on adaptive meshes with variable
 * viscosity" (arXiv 1907.06696).
 *   - problem: -div(2 mu eps(u)) + grad p = f, div u = 0, u = 0 on the boundary
 *     (Sec. 2, eq. stokes), Taylor-Hood Q2-Q1 (Sec. 2.1, eq. weak_form); also
 *     div u = g (a pressure right-hand side) and the no-normal-flux condition
 *     u . n = 0 (Sec. 2, the variants named after eq. stokes);
 *   - block system [A B^T; B 0] (Sec. 2.1, eq. stokes_linear_system);
 *   - FGMRES right-preconditioned by P = [A B^T; 0 -S] (Sec. 2.2,
 *     eq. stokes_precond), A^{-1} ~ one matrix-free GMG V-cycle with a degree-4
 *     Chebyshev smoother (Sec. 2.2.1), S^{-1} ~ CG on the mu^{-1}-weighted
 *     pressure mass matrix (Sec. 2.2.2);
 *   - cellwise viscosity by harmonic averaging over the quadrature points,
 *     children averaged onto parents (Sec. 2.3).
 *
 * Conventions used by every call:
 *   - Every function returns an int status: MFGMG_OK (0) or a negative
 *     MFGMG_ERR_* code; mfgmg_last_error() gives a message.  No exception
 *     crosses the interface.
 *   - Levels are numbered 1..L: level 1 is the 2x2x2-cell coarse mesh, level L
 *     the leaf (active) mesh; level l is the leaf mesh with every finer cell
 *     replaced by its level-l ancestor (global coarsening).
 *   - Velocity vectors of a level hold 3 values per Q2 node, node-major:
 *     entry 3*node + component.  Every node is stored, constrained ones
 *     included.  Pressure vectors hold one value per leaf Q1 node.
 *   - Nodes are identified across layouts by a canonical key: with U = L + 1,
 *     integer coordinates (X, Y, Z) in units of 2^-U, key = X + (S+1)(Y + (S+1)Z),
 *     S = 2^U.
 *   - Constrained dofs (Dirichlet boundary, hanging nodes, and under
 *     u . n = 0 the normal component on each boundary face) have identity
 *     rows: (A x)_i = x_i.  Hanging values are interpolated from their masters
 *     (Lagrange basis on {0, 1/2, 1} / {0, 1}) when a solution is returned.
 *   - Pointers named *_dev are device pointers (e.g. torch CUDA tensors on the
 *     current device); *_host are host pointers.  The caller owns them; device
 *     arrays must stay alive until the work on `stream` has completed.
 *     `stream` is a hipStream_t (NULL = default stream).  Calls marked async
 *     only enqueue work on that stream.
 *   - One context per host thread; a context is bound to the device that is
 *     current when mfgmg_set_viscosity is first called.  Device calls of one
 *     context share its internal work vectors: work enqueued on different
 *     streams of one context must not overlap in time.
 */
#ifndef MFGMG_H
#define MFGMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MFGMG_OK = 0,
  MFGMG_ERR_INVALID = -1, /* bad argument: null pointer, size, level, flag */
  MFGMG_ERR_STATE = -2,   /* call out of order (e.g. vmult before set_viscosity) */
  MFGMG_ERR_NOMEM = -3,   /* host or device allocation failed */
  MFGMG_ERR_HIP = -4,     /* a HIP runtime call failed */
  MFGMG_ERR_NOCONV = -5,  /* solver did not reach the tolerance, or NaN/Inf */
  MFGMG_ERR_MESH = -6     /* mesh cannot be built (too deep, bad cell) */
};

typedef enum { MFGMG_FP32 = 0, MFGMG_FP64 = 1 } mfgmg_prec;

#define MFGMG_MAX_LEVELS 14

typedef struct mfgmg_ctx mfgmg_ctx; /* opaque, owned by the library */

typedef struct {
  int32_t n_levels;      /* L */
  int32_t unit_exponent; /* U = L + 1 */
  /* arrays indexed by level (entry 0 unused) */
  int64_t n_cells[MFGMG_MAX_LEVELS + 1];
  int64_t n_nodes[MFGMG_MAX_LEVELS + 1];    /* Q2 nodes */
  int64_t n_u[MFGMG_MAX_LEVELS + 1];        /* 3 * n_nodes */
  int64_t n_free[MFGMG_MAX_LEVELS + 1];     /* free velocity dofs */
  int64_t n_hanging[MFGMG_MAX_LEVELS + 1];  /* hanging Q2 nodes */
  int32_t uniform[MFGMG_MAX_LEVELS + 1];    /* 1: all 8^l cells of level l */
  int64_t n_p;                              /* leaf Q1 nodes */
  int64_t n_p_hanging;                      /* hanging leaf Q1 nodes */
  int32_t boundary;                         /* MFGMG_BC_DIRICHLET or MFGMG_BC_NOFLUX */
  int32_t element_k;                        /* 1: Q2-Q1, 2: Q3-Q2 (mfgmg_set_element) */
} mfgmg_info_t;

/* velocity boundary conditions */
enum { MFGMG_BC_DIRICHLET = 0, MFGMG_BC_NOFLUX = 1 };

/* ---------------------------------------------------------------- mesh setup
 * The mesh is the unit cube as an octree (abstract; Sec. 3.2 domain).  Host
 * only; these calls touch no GPU. */

/* Unit cube refined uniformly to 2^base_level cells per edge
 * (1 <= base_level <= MFGMG_MAX_LEVELS - 2).  *out receives a new context. */
int mfgmg_create(int32_t base_level, mfgmg_ctx** out);

/* Velocity boundary condition (Sec. 2, eq. stokes and the variants after it),
 * before mfgmg_finalize_mesh:
 *   MFGMG_BC_DIRICHLET (default): u = 0 on the boundary;
 *   MFGMG_BC_NOFLUX: u . n = 0.  On the unit cube component c is fixed (zero)
 *     on the two faces normal to axis c, at edge and corner nodes two or three
 *     components; tangential components are unknowns whose condition (zero
 *     tangential stress) is the natural one of the weak form.  Every level is
 *     then stored as a general level (mfgmg_info uniform[] = 0) and the local
 *     smoothing calls are not available (ERR_INVALID).
 * Errors: ERR_INVALID for another value, ERR_STATE after finalize. */
int mfgmg_set_boundary(mfgmg_ctx* ctx, int32_t bc);

/* Taylor-Hood pair [Q_{k+1}]^3 x Q_k (Sec. 2.1), before mfgmg_finalize_mesh:
 * k = 1: Q2-Q1 (default, every call of this header);
 * k = 2: Q3-Q2 on uniform meshes (no mfgmg_refine) with u = 0.  Support points
 *   are the Gauss-Lobatto points of each direction, 4 Gauss points per
 *   direction integrate the forms.  A level of n = 2^l cells per edge stores
 *   its Q3 nodes X + m (Y + m Z), m = 3n + 1 (cell (i, j, k), local node (a, b,
 *   c): X = 3i + a, ...), and the leaf its Q2 pressure nodes on the (2n + 1)^3
 *   lattice; these lattice indices are the keys mfgmg_support_points returns.
 *   Viscosity and body force are given at the 64 Gauss points of each leaf
 *   cell (mfgmg_leaf_quadrature_points: [n_cells][64][3]); node kinds,
 *   transfers, vmult, vmult_add, the diagonal, smoother, transfers, coarse
 *   solve, V-cycle, right-hand side, B, B^T, M_p and mfgmg_solve_stokes (FGMRES
 *   with the CG Schur solve, either block preconditioner) work as for k = 1;
 *   the Chebyshev Schur map (its interval is the Q1 one), the local smoothing
 *   and the learned scaling return ERR_INVALID.
 * Errors: ERR_INVALID for another k; ERR_STATE after finalize; ERR_MESH from
 * finalize for k = 2 on a refined mesh or with MFGMG_BC_NOFLUX. */
int mfgmg_set_element(mfgmg_ctx* ctx, int32_t k);

/* Refine the listed active cells `levels_up` times (each becomes 8^levels_up
 * cells), then restore 2:1 balance across faces, edges and vertices by
 * refining further cells.  cells_host: [n][4] int32 (level, i, j, k) of active
 * cells.  Errors: ERR_INVALID if a listed cell is not active, ERR_STATE after
 * mfgmg_finalize_mesh. */
int mfgmg_refine(mfgmg_ctx* ctx, const int32_t* cells_host, int64_t n, int32_t levels_up);

/* Build the level meshes 1..L, Q2/Q1 node numbering, Dirichlet and hanging
 * constraints, and the level transfers.  Host only. */
int mfgmg_finalize_mesh(mfgmg_ctx* ctx);

int mfgmg_info(const mfgmg_ctx* ctx, mfgmg_info_t* out);

/* Cells of a level: [n_cells[level]][4] int32 (level, i, j, k). */
int mfgmg_cells(const mfgmg_ctx* ctx, int32_t level, int32_t* cells_host);

/* Canonical keys of the nodes of a level, in the library's storage order.
 * field 0: Q2 velocity nodes of `level` ([n_nodes[level]]);
 * field 1: Q1 pressure nodes of the leaf ([n_p]; level must be L). */
int mfgmg_support_points(const mfgmg_ctx* ctx, int32_t level, int32_t field, int64_t* keys_host);

/* Node kinds of a level: 0 free, 1 Dirichlet, 2 hanging.  field as above;
 * field 2: per Q2 node of `level`, the constrained components as bits
 * (bit c: dof 3*node + c has an identity row): 7 for Dirichlet and hanging
 * nodes, the fixed components of a no-normal-flux boundary node, else 0. */
int mfgmg_node_types(const mfgmg_ctx* ctx, int32_t level, int32_t field, uint8_t* types_host);

/* Hanging-node constraints of a level as CSR over the hanging nodes, in the
 * order of increasing node index: node_host[nh], ptr_host[nh+1],
 * master_host[nnz], weight_host[nnz] (masters on the boundary are omitted:
 * they carry zero).  Call with all arrays NULL to get *nh and *nnz only. */
int mfgmg_constraints(const mfgmg_ctx* ctx, int32_t level, int32_t field, int64_t* nh, int64_t* nnz,
                      int64_t* node_host, int64_t* ptr_host, int64_t* master_host, double* weight_host);

/* Node-level prolongation from level-1 to level (2 <= level <= L) as CSR
 * over fine nodes: ptr_host[n_nodes[level]+1], col_host[nnz] (coarse nodes),
 * weight_host[nnz].  The velocity prolongation applies it to each component
 * (under u . n = 0, with the fixed components of either level masked out).
 * Rows of constrained fine nodes are empty.  NULL arrays: *nnz only. */
int mfgmg_transfer(const mfgmg_ctx* ctx, int32_t level, int64_t* nnz, int64_t* ptr_host, int64_t* col_host,
                   double* weight_host);

/* Physical coordinates of the 3x3x3 Gauss points of the leaf cells,
 * [n_cells[L]][27][3] (points x-fastest), for evaluating the viscosity and
 * body force the caller wants to solve with. */
int mfgmg_leaf_quadrature_points(const mfgmg_ctx* ctx, double* xyz_host);

/* --------------------------------------------------------------- device data */

/* Viscosity at the leaf Gauss points, mu_qp_host [n_cells[L]][27] (> 0).
 * On the GPU: harmonic mean per leaf cell, arithmetic child mean on every
 * coarser level (Sec. 2.3); inverse diagonals of every level operator;
 * Chebyshev eigenvalue estimates; coarse factorisation.  Allocates the
 * library's device memory on first use.  Synchronises `stream`.
 * Errors: ERR_INVALID for non-positive or non-finite values. */
int mfgmg_set_viscosity(mfgmg_ctx* ctx, const double* mu_qp_host, void* stream);

/* Cell viscosities of a level after averaging: [n_cells[level]] (host copy). */
int mfgmg_cell_viscosity(const mfgmg_ctx* ctx, int32_t level, double* mu_host);

/* Chebyshev upper bound lambda = 1.2 * estimated max eig of D^{-1} A of a level. */
int mfgmg_smoother_lambda(const mfgmg_ctx* ctx, int32_t level, double* lambda_out);

/* Inverse diagonal of the level operator (1 on constrained dofs), device,
 * [n_u[level]] in the given precision.  Async. */
int mfgmg_inverse_diagonal(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, void* dst_dev, void* stream);

/* dst = A_level src: the matrix-free Q2 strain-rate operator of Sec. 2.1
 * (A_ij = int 2 mu eps(phi_i):eps(phi_j)) by sum factorisation at the 3x3x3
 * Gauss points of each cell, hanging nodes resolved in the gather and
 * condensed in the scatter, identity on constrained dofs.  src_dev, dst_dev:
 * [n_u[level]] of type float (FP32) or double (FP64); must not alias.  Async. */
int mfgmg_vmult(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* src_dev, void* dst_dev,
                void* stream);

/* dst += (cell contributions of A_level) src: the same cell loop as
 * mfgmg_vmult but without initialising dst and without the identity rows of
 * constrained dofs (their entries of dst are left unchanged).  One kernel
 * launch per call on uniform levels; used to accumulate and to time the cell
 * loop alone.  Async. */
int mfgmg_vmult_add(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* src_dev, void* dst_dev,
                    void* stream);

/* x = V(b): one V(1,1)-cycle on the leaf level (Sec. 2.2.1) with degree-4
 * Chebyshev smoothing (Saad, Alg. 12.1) preconditioned by the (scaled)
 * inverse diagonal, global-coarsening transfers, exact coarse solve.
 * rhs_dev, x_dev: [n_u[L]] in `prec`; x is overwritten.  Async. */
int mfgmg_vcycle(mfgmg_ctx* ctx, mfgmg_prec prec, const void* rhs_dev, void* x_dev, void* stream);

/* Level transfers (velocity, `prec`):  fine = P_level coarse (overwrite) and
 * coarse = P_level^T fine.  Async. */
int mfgmg_prolongate(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* coarse_dev, void* fine_dev,
                     void* stream);
int mfgmg_restrict(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* fine_dev, void* coarse_dev,
                   void* stream);

/* Chebyshev smoothing on a level: `degree`-4 polynomial applied to
 * A x = b starting from x (x_is_zero: ignore x's content).  Async. */
int mfgmg_smooth(mfgmg_ctx* ctx, int32_t level, mfgmg_prec prec, const void* b_dev, void* x_dev,
                 int32_t x_is_zero, void* stream);

/* Exact coarse solve on level 1 (375 entries): x = A_1^{-1} b.  Async. */
int mfgmg_coarse_solve(mfgmg_ctx* ctx, mfgmg_prec prec, const void* b_dev, void* x_dev, void* stream);

/* ------------------------------------------------------------ Stokes solve */

/* Right-hand side b_u = C^T F, F_(a,c) = int phi_a f_c, from the body force at
 * the leaf Gauss points f_qp_host [n_cells[L]][27][3]; constrained entries 0.
 * rhs_u_dev: double [n_u[L]].  Synchronises `stream`. */
int mfgmg_assemble_rhs(mfgmg_ctx* ctx, const double* f_qp_host, double* rhs_u_dev, void* stream);

/* Leaf operators in FP64 (Sec. 2.1, 2.2.2), async:
 *   div:  p_out = B u      (B_ij = -int psi_i div phi_j), [n_p] <- [n_u[L]]
 *   grad: u_out = B^T p                                  , [n_u[L]] <- [n_p]
 *   mass: p_out = M_p p    ([M_p]_ij = int mu^-1 psi_i psi_j, identity on
 *                           hanging pressure nodes). */
int mfgmg_apply_div(mfgmg_ctx* ctx, const double* u_dev, double* p_out_dev, void* stream);
int mfgmg_apply_grad(mfgmg_ctx* ctx, const double* p_dev, double* u_out_dev, void* stream);
int mfgmg_apply_pmass(mfgmg_ctx* ctx, const double* p_dev, double* p_out_dev, void* stream);

typedef struct {
  double rtol;            /* stop when ||b - K x||_2 <= rtol ||b||_2 (1e-8) */
  int32_t restart;        /* FGMRES restart length (50) */
  int32_t max_iter;       /* total outer iterations (1000) */
  int32_t vcycle_prec;    /* MFGMG_FP32 or MFGMG_FP64 */
  double schur_rtol;      /* inner pressure-mass CG tolerance (1e-2: the
                             1-5 inner iterations of Sec. 2.2.2) */
  int32_t schur_max_iter; /* (200) */
  int32_t use_scaling;    /* 1: use the installed smoother scaling */
  int32_t verbose;        /* > 0: every `verbose` outer iterations print the
                             iteration, the residual estimate and the elapsed
                             time to stderr (0) */
  int32_t use_graph;      /* 1: the V-cycle is captured once per solve as a HIP
                             graph (on a stream of the context) and replayed on
                             `stream`; 0: launched kernel by kernel (1) */
  /* Sec. 3.4 variants.  A Schur approximation that is a fixed linear map lets
   * plain GMRES (basis only, half the vectors of FGMRES) or IDR(s) (short
   * recurrences, 4 + 3s vectors) replace FGMRES. */
  int32_t krylov;         /* MFGMG_FGMRES, MFGMG_GMRES or MFGMG_IDR; the last
                             two need schur = MFGMG_SCHUR_CHEB (FGMRES) */
  int32_t idr_s;          /* IDR shadow-space dimension, 1..8 (2) */
  int32_t block;          /* MFGMG_BLOCK_TRIANGULAR: P of eq. stokes_precond;
                             MFGMG_BLOCK_DIAGONAL: P_D = diag(A, -S) of
                             eq. stokes_precond_diag, z_u = V(v_u) (triangular) */
  int32_t schur;          /* MFGMG_SCHUR_CG: Jacobi CG on M_p to schur_rtol;
                             MFGMG_SCHUR_CHEB: Chebyshev iteration (Saad,
                             Alg. 12.1) of degree schur_degree from 0 with
                             diag(M_p)^-1 over [b/27, b], b = max_i
                             (M_p 1)_i / (M_p)_ii, a fixed linear map (CG) */
  int32_t schur_degree;   /* 1..64 (8) */
  int32_t hierarchy;      /* MFGMG_GLOBAL_COARSENING: level l = the leaf mesh
                             with finer cells replaced by their level-l
                             ancestors (hanging nodes on every level);
                             MFGMG_LOCAL_SMOOTHING: level l = the cells of
                             refinement level exactly l, smoothed with the
                             refinement edge fixed (mfgmg_vcycle_local)
                             (MFGMG_GLOBAL_COARSENING) */
  int32_t idr_fp64_from;  /* IDR with the FP32 V-cycle: go on with the FP64
                             V-cycle from this iteration at the latest (from
                             the best iterate, with the true residual, as
                             where the run stalls); 0: only where it stalls (0) */
} mfgmg_solve_opts;

enum { MFGMG_FGMRES = 0, MFGMG_GMRES = 1, MFGMG_IDR = 2 };
enum { MFGMG_BLOCK_TRIANGULAR = 0, MFGMG_BLOCK_DIAGONAL = 1 };
enum { MFGMG_SCHUR_CG = 0, MFGMG_SCHUR_CHEB = 1 };
enum { MFGMG_GLOBAL_COARSENING = 0, MFGMG_LOCAL_SMOOTHING = 1 };

typedef struct {
  int32_t iterations;    /* outer iterations: Arnoldi steps ((F)GMRES) or
                            K P applications (IDR), one V-cycle each */
  int32_t vcycles;
  int64_t inner_cg_iterations;
  double rel_residual;   /* ||b - K x|| / ||b||, recomputed in FP64 at the end */
  double seconds;        /* wall time of the solve */
  int32_t converged;
  int32_t fp64_from;     /* IDR with the FP32 V-cycle: the iteration from which
                            the stalled solve went on with the FP64 V-cycle,
                            restarted from its best iterate; -1 otherwise */
} mfgmg_solve_stats;

/* Fill opts with the defaults above. */
int mfgmg_default_opts(mfgmg_solve_opts* opts);

/* Solve the block system (Sec. 2.2) with FGMRES (x0 = 0; GMRES or IDR(s) by
 * opts->krylov) right preconditioned by the block-triangular z_p =
 * -S^{-1} r_p, z_u = V(r_u - B^T z_p) (or the block-diagonal P_D).  IDR uses
 * the shadow space of SplitMix64 columns (seeds 4711 + i over the counters
 * 3 key + component for velocity dofs and 2^40 + key for pressure nodes),
 * orthonormalised by Gram-Schmidt (each column against the finished ones).  Outputs have hanging values
 * interpolated and the pressure shifted to zero mean.  rhs_p_dev may be
 * NULL (zero).  Synchronises `stream`.  Returns ERR_INVALID for options out
 * of range (GMRES or IDR without the Chebyshev Schur map), ERR_NOCONV
 * (stats and outputs filled) if rtol is not reached. */
int mfgmg_solve_stokes(mfgmg_ctx* ctx, const double* rhs_u_dev, const double* rhs_p_dev, double* u_dev,
                       double* p_dev, const mfgmg_solve_opts* opts, mfgmg_solve_stats* stats, void* stream);

/* ------------------------------------------------ local smoothing
 * The level hierarchy of the multigrid method cited in Sec. 2.2.1 (local
 * smoothing): levels 1 .. base are the uniform levels (every cell of the
 * level exists; there it equals the global-coarsening hierarchy); a finer
 * level l holds only the cells of refinement level l.  Its smoother keeps the
 * nodes on the refinement edge (on the boundary of the refined part, inside
 * the domain) fixed; the coupling of inner and edge nodes is carried between
 * the levels: t = d - K y (edge rows included) is restricted, the coarse
 * correction is kept on the edge, and the post-smoothing solves
 * A_II y_I = d_I - K_IE y_E.  Every free leaf node is copied to and from the
 * finest level whose cells hold it.  Level cell viscosities are those of the
 * same octree nodes on the global-coarsening levels (Sec. 2.3). */

/* Host only.  *base_host: the finest uniform level (L for a uniform leaf
 * mesh); n_cells_host[l], n_nodes_host[l] ([MFGMG_MAX_LEVELS + 1]) of every
 * level (the uniform ones included). */
int mfgmg_local_levels(const mfgmg_ctx* ctx, int32_t* base_host, int64_t* n_cells_host, int64_t* n_nodes_host);

/* Host only.  Canonical keys and kinds (0 inner, 1 domain boundary,
 * 2 refinement edge) of the Q2 nodes of local level `level` (base < level
 * <= L), in storage order: keys_host, kinds_host [n_nodes[level]]. */
int mfgmg_local_nodes(const mfgmg_ctx* ctx, int32_t level, int64_t* keys_host, uint8_t* kinds_host);

/* Host only.  Node-level prolongation to local level `level` from the level
 * below (the base level or the local level below) as CSR over the level's
 * nodes (as mfgmg_transfer): boundary rows empty, edge rows kept.
 * NULL arrays: *nnz only. */
int mfgmg_local_transfer(const mfgmg_ctx* ctx, int32_t level, int64_t* nnz, int64_t* ptr_host, int64_t* col_host,
                         double* weight_host);

/* x = one local-smoothing V(1,1)-cycle on leaf vectors (same smoother,
 * Chebyshev bounds rule and coarse solve as mfgmg_vcycle; x is zero on the
 * constrained leaf dofs).  The first call after mfgmg_set_viscosity sets up
 * the local levels (synchronises `stream`).  Async otherwise. */
int mfgmg_vcycle_local(mfgmg_ctx* ctx, mfgmg_prec prec, const void* rhs_dev, void* x_dev, void* stream);

/* ------------------------------------------- learned smoother scaling
 * Not part of the paper: the degree-4 Chebyshev smoother of Sec. 2.2.1 is
 * preconditioned by diag(s/d) instead of diag(1/d) on chosen levels, with
 * s_(node, c) = exp(mean of y_{K,c} over the cells K of the level holding the
 * node) and y_K = MLP(27 relative log10 viscosities of K's 3x3x3
 * neighbourhood); MLP 27 -> 64 -> 64 -> 3, GELU (erf form), output clamped to
 * [-2, 2], 6147 FP32 parameters W1[64][27], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3] (row-major [out][in]). */

/* Features of the cells of a level, feat_dev [n_cells[level]][27] FP32:
 * log10 mu_{K'} - log10 mu_K over the 3x3x3 same-level neighbourhood
 * (offsets (i-1, j-1, k-1), x fastest); a position covered by a coarser cell
 * takes that cell's viscosity, one outside the domain takes mu_K.
 * Synchronises `stream`. */
int mfgmg_features(mfgmg_ctx* ctx, int32_t level, float* feat_dev, void* stream);

/* Objective of the target fit on a level (2 <= level <= L) for per-cell
 * log-scalings y_dev [n_cells][3] (FP32 in, FP64 arithmetic):
 * J = (1/4) sum_k (1/2) log(||E^2 e_k||_A / ||e_k||_A), E = I - V A, V the
 * V-cycle whose level-`level` smoothers use diag(s/d) (coarser levels plain),
 * e_k SplitMix64 vectors (seeds 777..780 over 3 key + component).
 * lam_fixed > 0 holds the Chebyshev bound fixed, else it is re-estimated
 * (*lam_out receives the value used).  grad_dev (may be NULL):
 * dJ/dy [n_cells][3] FP32: the adjoint of the V-cycle at fixed lambda plus,
 * when lambda is re-estimated, its dependence on the scaling through the
 * Ritz pair (theta, v) of the estimate: s_i dlambda/ds_i = lambda v_i^2 M_ii /
 * (v . M v), M = diag(d/s), with dJ/dlambda = -(s . dJ/ds) / lambda (the
 * smoother depends on s / lambda only).  Synchronises `stream`. */
int mfgmg_fit_objective(mfgmg_ctx* ctx, int32_t level, const float* y_dev, double lam_fixed, double* J_host,
                        double* lam_out_host, float* grad_dev, void* stream);

/* Targets of a level: Adam (lr, beta 0.9/0.999, eps 1e-8) on J from y = 0 for
 * `steps` steps, y clipped to [-2, 2].  y_dev [n_cells][3] FP32 out;
 * J_hist_host [steps + 1] (may be NULL).  Synchronises `stream`. */
int mfgmg_fit_targets(mfgmg_ctx* ctx, int32_t level, int32_t steps, double lr, float* y_dev, double* J_hist_host,
                      void* stream);

/* Install the scaling of a level from per-cell y_dev [n_cells][3] FP32
 * (re-estimates lambda); y_dev NULL removes it.  Synchronises `stream`. */
int mfgmg_set_scaling(mfgmg_ctx* ctx, int32_t level, const float* y_dev, void* stream);

/* Whether mfgmg_vcycle / mfgmg_smooth use the installed scalings (default 0);
 * mfgmg_solve_stokes follows opts->use_scaling instead. */
int mfgmg_use_scaling(mfgmg_ctx* ctx, int32_t on);

/* A-norm contraction of E = I - V A on the leaf level estimated by three
 * power steps from a SplitMix64 vector (seed 4242), FP64.  Synchronises. */
int mfgmg_vcycle_factor(mfgmg_ctx* ctx, double* rho_host, void* stream);

/* MLP over n samples: x_dev [n][27] -> y_dev [n][3]; cache_dev [n][131]
 * keeps the pre-activations for the backward pass.  Async. */
int mfgmg_mlp_forward(const float* w_dev, const float* x_dev, int64_t n, float* y_dev, float* cache_dev, void* stream);

/* dw_dev[6147] = gradient of sum(dy * y) w.r.t. the parameters (the clamp
 * passes gradient strictly inside [-2, 2]); work_dev holds
 * mfgmg_mlp_work_size(n) floats.  Async. */
int mfgmg_mlp_backward(const float* w_dev, const float* x_dev, const float* cache_dev, const float* dy_dev, int64_t n,
                       float* dw_dev, float* work_dev, void* stream);
int64_t mfgmg_mlp_work_size(int64_t n);

/* One Adam step (beta 0.9/0.999, eps 1e-8, bias-corrected, step >= 1) on the
 * 6147 parameters.  Async. */
int mfgmg_mlp_adam(float* w_dev, const float* dw_dev, float* m_dev, float* v_dev, int64_t step, double lr,
                   void* stream);

/* Train on n (feature, target) pairs: mean-squared error, Adam (lr), epochs of
 * mini-batches of `batch` samples shuffled by a SplitMix64-driven
 * Fisher-Yates permutation (seed, epoch).  loss_hist_host [epochs] receives
 * the mean squared error of each epoch (may be NULL).  w_dev updated in
 * place.  Synchronises `stream`. */
int mfgmg_mlp_train(float* w_dev, const float* feats_dev, const float* targets_dev, int64_t n, int32_t epochs,
                    int32_t batch, double lr, uint64_t seed, double* loss_hist_host, void* stream);

/* Features -> MLP -> scaling on every level 2..L, then the guard:
 *   MFGMG_GUARD_NONE: keep the scalings;
 *   MFGMG_GUARD_FP64 / MFGMG_GUARD_FP32: estimate the A-norm contraction of
 *   E = I - V A on the leaf with and without the scalings (6 power steps from
 *   a SplitMix64 vector, seed 4242, the V-cycle in FP64 / FP32: pass the
 *   precision of the solve the scaling is for) and keep the scalings only if
 *   the learned factor is below 0.95 times the plain one.
 * factors_host[0] plain, [1] learned (may be NULL); *used_host = 1 if kept.
 * ERR_INVALID for another guard value.  Synchronises `stream`. */
enum { MFGMG_GUARD_NONE = 0, MFGMG_GUARD_FP64 = 1, MFGMG_GUARD_FP32 = 2 };
int mfgmg_apply_mlp(mfgmg_ctx* ctx, const float* w_dev, int32_t guard, int32_t* used_host, double* factors_host,
                    void* stream);

/* ------------------------------------------- operator without allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * operator of mfgmg_vmult on the uniform n x n x n mesh of the unit cube
 * (n_edge = 32 or 64), without a context.  mu_dev: cell viscosity [n^3]
 * (cell i + n (j + n k)), src_dev, dst_dev: [3 (2n+1)^3] velocity values,
 * node X + (2n+1)(Y + (2n+1) Z) with X, Y, Z the lattice coordinates in units
 * of 1/(2n), all in the precision `prec`; boundary nodes are Dirichlet
 * (identity rows: dst = src there).  Identical results to mfgmg_vmult on the
 * leaf of a uniform context with the same cell viscosities.  Work memory:
 * the library's static device array (71.4 MB per GPU, held until the process
 * ends); no allocation, no host synchronisation.  Calls on one GPU share that
 * array: calls whose work overlaps in time (other streams or threads) race.
 * Errors: ERR_INVALID for n_edge above 64 (the array's limit) or other than
 * 32 and 64, null or aliased pointers; ERR_HIP if the array's device address
 * cannot be found.  Async. */
int mfgmg_vmult_uniform_noalloc(int32_t n_edge, mfgmg_prec prec, const void* mu_dev, const void* src_dev,
                                void* dst_dev, void* stream);

/* ---------------------------------------------------------------- misc */

const char* mfgmg_last_error(const mfgmg_ctx* ctx); /* ctx may be NULL */
void mfgmg_destroy(mfgmg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MFGMG_H */
