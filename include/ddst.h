/*
 * ddst.h -- C-ABI of the MI355X solution-transfer domain-decomposition library.
 *
 * The library implements the data-parallel hot path of the overlapping
 * solution-transfer DD method (Dirckx, Yesypenko, Martinsson, arXiv 2510.25991)
 * for the finite-difference model problem of Section 2.1:
 *
 *     -div(kappa grad u) + b . grad u + c u = f   in the unit square / cube,
 *                                        u = g   on its boundary,
 *
 * discretised on n interior nodes per axis (h = 1/(n+1)) with the 5-point /
 * 7-point stencil.  The coefficient kappa is cellwise ((n+1)^dim cells); the
 * coefficient of a grid edge is the mean of the 2^(dim-1) cells sharing it;
 * convection uses centred differences.  The domain is cut along x into
 * n_slabs equispaced slabs of m = (n+1)/n_slabs cells; the N_ds = n_slabs-1
 * interfaces Gamma_j sit on node planes x-index j*m and carry M = n^(dim-1)
 * nodes each (Section 2, equispaced slabs).
 *
 * Layouts (all arrays are caller-owned DEVICE memory unless stated):
 *   interior nodal arrays: n^dim float64, C order, x slowest (node (i,j[,k])
 *       with 1-based indices sits at ((i-1)*n + (j-1))[*n + (k-1)]);
 *   kappa: (n+1)^dim float64 cells, C order (cell c spans nodes c..c+1);
 *   g: (n+2)^dim float64 node box, C order; only boundary entries are read;
 *   interface vectors: N_ds*M float64, interface-major (Gamma_1 first).
 *
 * Every call is ordered on the given HIP stream.  Calls whose return status
 * depends on device results (pivot breakdown, ranks, convergence) synchronise
 * the stream before returning.  No C++ exception crosses this boundary.
 *
 * Status codes: 0 success; DDST_ENOTCONV (+1) means outputs were written but
 * the requested tolerance was not met; negative values are errors, and after
 * an error the text of ddst_last_error() (thread-local) says what failed.
 */
#ifndef DDST_H
#define DDST_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DDST_OK = 0,
  DDST_ENOTCONV = 1,     /* outputs written, tolerance not reached            */
  DDST_EINVAL = -1,      /* bad shape, divisibility, NaN or kappa <= 0, NULL  */
  DDST_ENOMEM = -2,      /* device allocation failed                          */
  DDST_EHIP = -3,        /* a HIP runtime call failed                         */
  DDST_EBREAKDOWN = -4,  /* non-finite (or, by default, non-positive) pivot in a
                            local solve */
  DDST_ERANK = -5,       /* HODLR rank cap exceeded                           */
  DDST_ESTATE = -6       /* operation not available in this operator state    */
};

/* Arithmetic of the local eliminations, transfer blocks and factors. */
enum { DDST_FP64 = 0, DDST_FP32 = 1 };
/* Local elimination: symmetric when the operator is (automatic), or always
 * the general one. */
enum { DDST_ELIM_AUTO = 0, DDST_ELIM_GENERAL = 1 };
/* Cluster tree for hierarchical compression. */
enum { DDST_TREE_BINARY = 0, DDST_TREE_QUAD = 1 };
/* Storage type of the compressed low-rank factors. */
enum { DDST_FACTOR_BF16 = 0, DDST_FACTOR_FP32 = 1, DDST_FACTOR_FP64 = 2 };
/* Largest number of right-hand sides of ddst_solve_many. */
enum { DDST_MAX_RHS = 16 };
/* Which representation ddst_apply uses: the dense transfer blocks, their
 * HODLR compression, no blocks at all (matrix-free: sweeps with the stored
 * single-slab factors and the interface blocks, Sections 2.2 and 5.1), or
 * the HBS form built from samples without the blocks (Section 2.4,
 * Algorithm 1; ddst_compress_hbs). */
enum { DDST_APPLY_DENSE = 0, DDST_APPLY_HODLR = 1, DDST_APPLY_MATFREE = 2, DDST_APPLY_HBS = 3 };

typedef struct ddst_op ddst_op_t; /* opaque, library-owned */

/* The PDE operator (eq. basic of the paper, FD form of Section 2.1). */
typedef struct {
  int32_t dim;          /* 2 or 3                                              */
  int32_t n;            /* interior nodes per axis, >= 3                       */
  int32_t n_slabs;      /* >= 2, (n+1) % n_slabs == 0, m = (n+1)/n_slabs >= 2  */
  const double *kappa;  /* device, (n+1)^dim cells, > 0; NULL means kappa = 1  */
  double bvec[3];       /* constant convection velocity (unused entries 0)     */
  const double *c;      /* device, n^dim nodal zeroth-order term; NULL means 0 */
} ddst_problem_t;

typedef struct {
  int32_t precision;        /* DDST_FP64 (plain path) or DDST_FP32 (mixed path) */
  int32_t keep_factors;     /* 1: keep the per-slab elimination factors for the
                               solve (required by ddst_solve); 0: drop them     */
  int32_t transpose;        /* must be 0 (reserved; the adjoint works from the
                               forward operator's transposed structure)       */
  int32_t skip_transfer;    /* 1: matrix-free set-up (Section 5.1): slab factors
                               and interface blocks only, no transfer blocks;
                               needs keep_factors; solves then set
                               matrix_free, and the dense form, the compressed
                               form and ddst_get_transfer report ESTATE       */
  int32_t indefinite;       /* 0: a non-positive pivot is a breakdown (the local
                               problems are taken to be definite, as for
                               diffusion and low-frequency Helmholtz); 1:
                               negative pivots are accepted, for indefinite but
                               nonsingular local problems (Helmholtz above the
                               first double-slab resonance, Section 5.2); the
                               elimination still does not pivot, so every
                               partial-slab Schur complement D_k (the planes
                               1..k of a single slab, k < m) must be
                               nonsingular too, not only the double slab: a
                               pivot growth (ddst_stats_t) above 1e12 (FP64)
                               or 1e5 (FP32) is reported as EBREAKDOWN        */
  int32_t elimination;      /* DDST_ELIM_AUTO (0): when the operator is
                               symmetric (no convection: bvec = 0) and the
                               local problems definite (indefinite = 0), its
                               plane blocks and interface blocks are
                               symmetric and the local inverses are formed
                               by the symmetric elimination, which updates
                               only the lower triangle (about half the work,
                               the factorisation remark of Section 2.5);
                               DDST_ELIM_GENERAL (1): always the general
                               elimination                                    */
} ddst_build_opts_t;

typedef struct {
  int32_t tree;             /* DDST_TREE_BINARY (dim 2) or DDST_TREE_QUAD (dim 3) */
  int32_t leaf;             /* maximum leaf cluster size, e.g. 128             */
  int32_t oversample;       /* p, extra Gaussian samples beyond the rank, e.g. 10 */
  int32_t max_rank;         /* rank cap per admissible block, max_rank +
                               oversample <= 128                               */
  int32_t factor_dtype;     /* DDST_FACTOR_BF16 / FP32 / FP64                  */
  int32_t reserved;
  double tol;               /* keep sigma_i > tol * ||S_{j,j'}||_2             */
  uint64_t seed;            /* Gaussian test matrices                          */
} ddst_compress_opts_t;

typedef struct {
  double tol;               /* target relative error of the refined solution   */
  double inner_tol;         /* relative residual of the interface GMRES per    */
                            /* refinement pass (default 1e-4 FP32, 1e-12 FP64) */
  int32_t max_iter;         /* GMRES iteration cap per pass (<= 20000; the     */
                            /* basis takes (max_iter+1)*N_ds*ld*8 device bytes) */
  int32_t max_outer;        /* FP64 refinement passes (>= 1)                   */
  int32_t use_hodlr;        /* 1: apply S through the compressed form          */
  int32_t matrix_free;      /* 1: apply S by sweeps with the stored factors,
                               without its blocks (exclusive with use_hodlr)   */
  int32_t restart;          /* 0: unrestarted GMRES (the paper's); k > 0:
                               restart every k iterations from the explicit
                               residual (0 <= k <= max_iter)                   */
  int32_t use_hbs;          /* 1: apply S through the HBS form of
                               ddst_compress_hbs (exclusive with use_hodlr and
                               matrix_free)                                    */
  int32_t basis_fp32;       /* 1: GMRES passes whose tolerance is >= 1e-6 keep
                               the finalized Krylov vectors in FP32 (the
                               operator's input and every sum stay FP64; half
                               the bytes of the Gram-Schmidt passes); 0 (the
                               default): FP64 basis                            */
  int32_t reserved_;
} ddst_solve_opts_t;

typedef struct {
  int32_t outer_iters;      /* refinement passes taken                         */
  int32_t gmres_iters;      /* GMRES iterations summed over passes             */
  int32_t last_gmres_iters; /* GMRES iterations of the last pass               */
  int32_t converged;        /* 1 if the stopping rule was met                  */
  double gmres_relres;      /* last GMRES relative residual estimate           */
  double residual_rel;      /* ||f - A u||_2 / ||f - A 0||_2, FP64 stencil     */
  double correction_rel;    /* ||last correction|| / ||u||                     */
  double t_build_ms, t_compress_ms, t_solve_ms, t_adjoint_ms; /* phase times   */
  double bytes_factors, bytes_transfer, bytes_hodlr;          /* storage       */
  int32_t max_rank, min_rank;                                  /* HODLR ranks   */
  double pivot_growth;      /* largest |entry| of an inverted pivot block times
                               the largest |entry| of the FD matrix, over the
                               local eliminations of the build: of order
                               1 / (eps ||A||) ||A|| when a local problem is
                               singular to working precision                  */
  int32_t symmetric;        /* 1 if the build used the symmetric elimination   */
  int32_t reserved_;
} ddst_stats_t;

/*
 * ddst_build_transfer -- form every dense solution-transfer block
 *   S_{j,j'} = -R_{C_j} A_j(I_j,I_j)^{-1} A_j(I_j,J_{j,j'})   (eq. defS)
 * of every double slab Psi_j (Section 2.5, local and global assembly), by
 * batched block-tridiagonal elimination across the thin x direction of all
 * slabs at once, plus the inverse of each interface Schur block
 * T_jj (Section 2.1, eq. efewin) and, if keep_factors, the per-plane inverse
 * Schur complements of a left-to-right sweep of every single slab.
 * prob: host struct; its device arrays are read during the call only.
 * opts: host struct or NULL (defaults: FP32, keep_factors=1, the rest 0).
 * out: receives the new operator, or NULL on error.
 * Errors: EINVAL (shape/divisibility, kappa <= 0 or non-finite, c non-finite),
 *         ENOMEM, EHIP, EBREAKDOWN (a local elimination met a non-finite pivot,
 *         or a non-positive one unless opts->indefinite: the local problem is
 *         degenerate, cf. the remark on degenerate local problems in Section
 *         2.2, or indefinite).
 */
int ddst_build_transfer(const ddst_problem_t *prob, const ddst_build_opts_t *opts,
                        hipStream_t stream, ddst_op_t **out);

/*
 * ddst_compress -- compress every transfer block as a weak-admissibility
 * hierarchical matrix (Section 2.4; HODLR form): on a cluster tree shared by
 * source and target interface, every interaction between distinct children
 * of a tree node is a low-rank block U V^T obtained from a randomized range
 * finder with Gaussian probes (Algorithm 1, sampling step), a Householder QR
 * and a small SVD, truncated at sigma_i > tol * ||S_{j,j'}||_2; leaves stay
 * dense.  The dense blocks are kept (ddst_apply can use either form).
 * Errors: EINVAL, ENOMEM, EHIP, ERANK (a block needs more than max_rank).
 */
int ddst_compress(ddst_op_t *op, const ddst_compress_opts_t *opts, hipStream_t stream);

/*
 * ddst_solve -- solve the FD problem through the equilibrium system
 *   u_j - S_{j,j-1} u_{j-1} - S_{j,j+1} u_{j+1} = hhat_j   (eq. modelS)
 * by unrestarted GMRES (Section 5), with FP64 iterative refinement on the FP64
 * stencil residual: each pass forms r = f - A u, computes the equivalent loads
 * of r (eq. equilib1) with the stored slab factors, solves the interface
 * system, recovers the volume correction slab by slab and adds it in FP64.
 * f: device n^dim (NULL means 0); g: device (n+2)^dim node box (NULL means 0).
 * u_gamma: device N_ds*M output (interface traces), may be NULL.
 * u_vol: device n^dim output (full solution), may be NULL.
 * stats: host, may be NULL.
 * Stops when the predicted relative error (correction size times the
 * observed contraction) is <= tol, or after max_outer passes.
 * Errors: EINVAL, ESTATE (factors dropped), ENOMEM, EHIP; ENOTCONV (+1) if
 * GMRES hit max_iter or the stopping rule was not met.
 */
int ddst_solve(const ddst_op_t *op, const double *f, const double *g,
               const ddst_solve_opts_t *opts, double *u_gamma, double *u_vol,
               ddst_stats_t *stats, hipStream_t stream);

/*
 * ddst_solve_many -- nrhs problems with the same operator and different data
 * solved together: the case of many right-hand sides for which forming the
 * transfer blocks pays (Section 2.2, the first reason listed for forming S;
 * Example 1 reuses S over time steps).  The interface systems of all of them
 * form one block-diagonal system diag(S, ..., S) solved by one GMRES (one
 * Krylov polynomial, inner products summed over all right-hand sides), so
 * each product reads every block of S, and each slab sweep every factor, once
 * for all of them; the FP64 refinement runs until every right-hand side meets
 * the stopping rule of ddst_solve.
 * nrhs: 1..DDST_MAX_RHS.  f: device nrhs * n^dim, right-hand side v at
 * f + v n^dim (NULL: all 0); g: device nrhs * (n+2)^dim node boxes, likewise
 * (NULL: all 0); u_vol: device nrhs * n^dim output.  stats: as ddst_solve,
 * with correction_rel and residual_rel the largest over the right-hand sides.
 * Errors: as ddst_solve.
 */
int ddst_solve_many(const ddst_op_t *op, int32_t nrhs, const double *f, const double *g,
                    const ddst_solve_opts_t *opts, double *u_vol, ddst_stats_t *stats,
                    hipStream_t stream);

/*
 * ddst_adjoint -- gradient of a loss L(u) with respect to the cellwise
 * coefficient kappa, for the solution u of ddst_solve with the same g.
 * Solves A^T lambda = gbar through the transposed Schur structure of the
 * slab decomposition: transposed single-slab solves, the transposed
 * equilibrium system S^T (GMRES; (S^T)_{j,j'} = S_{j',j}^T) and the transposed
 * interface blocks, with FP64 refinement on the A^T stencil residual.  The
 * slab factors are recomputed (not read from the operator) when the operator
 * holds none.  Then
 *   dL/dkappa_c = -1/(2^(dim-1) h^2) sum_{edges (p,q) of cell c}
 *                  (lambda_p - lambda_q)(u_p - u_q),
 * with lambda = 0 and u = g on the boundary.
 * u_vol: device n^dim; gbar: device n^dim (dL/du); g: as in ddst_solve;
 * dkappa: device (n+1)^dim output (overwritten); lambda: device n^dim output
 * or NULL.  Errors: as ddst_solve.
 */
int ddst_adjoint(const ddst_op_t *op, const double *u_vol, const double *g,
                 const double *gbar, const ddst_solve_opts_t *opts, double *dkappa,
                 double *lambda, ddst_stats_t *stats, hipStream_t stream);

/* Options of the sampled HBS compression. */
typedef struct {
  int32_t rank;             /* k: rank of every cluster basis (the paper's fixed
                               HBS rank, e.g. 64)                              */
  int32_t oversample;       /* q: s = 3 k + q samples per side (Algorithm 1:
                               alpha = 3, typically q = 10)                    */
  int32_t leaf;             /* largest leaf cluster, 0 means 2 k; every
                               cluster needs s >= its size + k                 */
  int32_t factor_dtype;     /* DDST_FACTOR_BF16 / FP32 / FP64                  */
  uint64_t seed;            /* probes drawn by the library (Philox-4x32-10, Box-
                               Muller) when omega / psi are NULL               */
} ddst_hbs_opts_t;

/*
 * ddst_compress_hbs -- every transfer block S_{j,j'} in Hierarchically Block
 * Separable form (Section 2.4), built from s = 3 k + q two-sided samples
 * Y = S Omega and Z = S^T Psi obtained by local solves with the stored
 * factors of the single slabs (Algorithm 1's sampling step: forward and
 * transposed chains of products with the inverse plane Schur complements,
 * then the inverse interface blocks), so the dense blocks are never needed:
 * it works on an operator built with skip_transfer = 1 (whose memory is the
 * slab factors only) as well as on one that holds the blocks.  The
 * compression is the single-pass randomized HBS construction from Y and Z
 * alone, on a binary cluster tree of uniform depth shared by rows and
 * columns (2D: index ranges split at the midpoint; 3D: the n x n interface
 * grid split at the midpoint of the longer side), rank k at every node; the
 * form stores O(k M) numbers per block and applies in O(k M) (solve option
 * use_hbs, ddst_apply with DDST_APPLY_HBS).
 * omega, psi: device M x s float64 row-major probes, or NULL (the library
 * draws them from opts->seed); read during the call only.
 * Errors: EINVAL (bad options; a cluster with more points than s - k),
 * ESTATE (slab factors dropped), ENOMEM, EHIP, EBREAKDOWN (a probe Gram
 * matrix is not positive definite).
 */
int ddst_compress_hbs(ddst_op_t *op, const ddst_hbs_opts_t *opts, const double *omega,
                      const double *psi, hipStream_t stream);

/* HBS summary: factor bytes, rank k, sampling and compression times (ms) of
 * the last ddst_compress_hbs.  ESTATE if none. */
int ddst_hbs_info(const ddst_op_t *op, double *bytes, int32_t *rank, double *t_sample_ms,
                  double *t_compress_ms);

/*
 * ddst_sample_blocks -- test hook of the sampling step: Y_b = S_b X and
 * Z_b = S_b^T X for every transfer block by the chains of ddst_compress_hbs.
 * Blocks b = 2 (s - 1) (S_{s+1,s}) and 2 (s - 1) + 1 (S_{s,s+1}) for the
 * slabs s = 1 .. N_ds - 1; X: device M x ncols float64 row-major; Y, Z:
 * device 2 (N_ds - 1) x M x ncols outputs.  1 <= ncols <= 512.
 */
int ddst_sample_blocks(const ddst_op_t *op, int32_t ncols, const double *X, double *Y,
                       double *Z, hipStream_t stream);

/* Compressed-form summary: factor bytes, largest / smallest admissible rank,
 * compression time of the last ddst_compress (ms).  ESTATE if none. */
int ddst_compress_info(const ddst_op_t *op, double *bytes, int32_t *max_rank,
                       int32_t *min_rank, double *ms);

/* Drop the per-slab factors (frees device memory); the adjoint recomputes. */
int ddst_release_factors(ddst_op_t *op);

/* Destroy an operator; NULL is a no-op.  Synchronises the device. */
void ddst_destroy(ddst_op_t *op);

/*
 * ddst_set_allocator -- device memory for everything the library allocates
 * (operators, factors, compressed forms, workspaces, temporaries) from the
 * caller's allocator, e.g. a framework's caching allocator, instead of
 * hipMalloc / hipFree.  alloc(bytes, ctx) returns device memory on the
 * current device, 256-byte aligned, or NULL (reported as ENOMEM);
 * free(ptr, ctx) releases it.  Both NULL restores hipMalloc / hipFree.  As
 * with hipFree, the device is synchronized before every free, so the block
 * may be reused at once.  Process-wide; call it while no operator
 * exists and no other call is running (ESTATE otherwise); EINVAL if exactly
 * one of alloc and free is NULL.
 */
typedef void *(*ddst_alloc_fn)(size_t bytes, void *ctx);
typedef void (*ddst_free_fn)(void *ptr, void *ctx);
int ddst_set_allocator(ddst_alloc_fn alloc, ddst_free_fn free_fn, void *ctx);

/* Text of the last error on this thread ("" if none). */
const char *ddst_last_error(void);

/* Figures of the build (phase times, storage, ranks, pivot growth) in the
 * fields of ddst_stats_t that ddst_build_transfer and ddst_compress set; the
 * solve fields are zero.  stats: host. */
int ddst_build_stats(const ddst_op_t *op, ddst_stats_t *stats);

/* Geometry of an operator: M, N_ds, padded leading dimension, precision. */
int ddst_op_info(const ddst_op_t *op, int32_t *M, int32_t *n_ds, int32_t *ld,
                 int32_t *precision);

/*
 * Test hooks.
 * ddst_get_transfer: copy S_{j,j-1} and S_{j,j+1} (1-based j) into M x M
 *   row-major float64 device buffers (a block that does not exist -- next to
 *   the physical boundary -- is written as zeros); either pointer may be NULL.
 * ddst_apply: y = S x (transpose 0) or S^T x (transpose 1) for the equilibrium
 *   matrix S = I - K, x and y device N_ds*M float64, through the dense blocks
 *   (which = DDST_APPLY_DENSE), the compressed form (DDST_APPLY_HODLR) or
 *   matrix-free (DDST_APPLY_MATFREE: for every single slab between two
 *   interfaces, two chains of m-1 products with its stored factors, then
 *   Sigma_j^{-1}; the paper's matrix-free alternative, Section 5.1).
 *   ESTATE if the chosen form is not held (no compression; factors dropped).
 * ddst_loads: equivalent loads hhat (eq. equilib1) of the load f and boundary
 *   data g, device N_ds*M output.
 */
int ddst_get_transfer(const ddst_op_t *op, int32_t j, double *S_left, double *S_right,
                      hipStream_t stream);
int ddst_apply(const ddst_op_t *op, int32_t transpose, int32_t which, const double *x,
               double *y, hipStream_t stream);
int ddst_loads(const ddst_op_t *op, const double *f, const double *g, double *hhat,
               hipStream_t stream);

/*
 * ddst_apply_noalloc -- for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the product of ddst_apply, y = S x or S^T x, through the
 * dense blocks (which = DDST_APPLY_DENSE) or a compressed form
 * (DDST_APPLY_HODLR, DDST_APPLY_HBS), with no hipMalloc, hipFree or other
 * allocation and no
 * synchronisation (the work is ordered on `stream`; the call returns once
 * it is enqueued).  Its temporaries (padded copies of x and y, the product's
 * job table, the partial sums of the transposed product) live in a static
 * device array of 16 MiB per GPU, held until the process ends; the first
 * call on a device looks up its address.  x, y: device N_ds*M float64,
 * caller-owned.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or threads without ordering between
 * them) race.  Errors: EINVAL (NULL pointers, which MATFREE, or a
 * product that needs more than the 16 MiB: the dense product needs
 * 16 N_ds ld bytes plus, transposed, 8 N_ds min(ld/32, 64) ld, with ld = M
 * rounded up to a multiple of 128), ESTATE (form not held), EHIP.
 */
int ddst_apply_noalloc(const ddst_op_t *op, int32_t transpose, int32_t which, const double *x,
                       double *y, hipStream_t stream);

/*
 * Diagnostics of the equilibrium system (the iteration counts and condition
 * numbers of Section 5.2, Tables fd_poisson_fixedH, fd_shrinkingH and
 * fd_other_models).
 * ddst_gmres: x = S^{-1} b (transpose 1: S^{-T} b) by unrestarted GMRES from
 *   x = 0 to a relative residual <= tol (FP64 Arnoldi), S applied through form
 *   `which` (DDST_APPLY_*); b, x device N_ds*M float64; iters, relres: host,
 *   may be NULL.  ENOTCONV (+1) if max_iter (<= 20000) was reached first.
 * ddst_cond_est: the extreme singular values of S by power iteration on
 *   S^T S and inverse iteration on (S^T S)^{-1} (two GMRES solves to
 *   gmres_tol per step), each stopped when the eigenvalue estimate changes by
 *   <= tol relative or after max_iter steps, from a fixed pseudo-random start;
 *   kappa_2(S) = smax / smin.  iters: host, steps of the last iteration.
 * Errors: EINVAL, ESTATE (form not held), ENOMEM, EHIP.
 */
int ddst_gmres(const ddst_op_t *op, int32_t transpose, int32_t which, const double *b,
               double *x, double tol, int32_t max_iter, int32_t *iters, double *relres,
               hipStream_t stream);
int ddst_cond_est(const ddst_op_t *op, int32_t which, int32_t max_iter, double tol,
                  double gmres_tol, double *smax, double *smin, int32_t *iters,
                  hipStream_t stream);

/*
 * Inspection hooks for the intermediate state of the build.
 * ddst_get_factor: G_k = D_k^{-1}, the inverse Schur complement after k
 *   planes of the left-to-right elimination of single slab `slab`
 *   (0-based, 0..n_slabs-1), k = 1..m-1, into an M x M float64 device buffer.
 *   ESTATE if the factors were dropped.
 * ddst_get_center_inverse: inverse of the interface Schur block
 *   T_jj (eq. efewin), j = 1..N_ds, M x M float64 device buffer.
 */
int ddst_get_factor(const ddst_op_t *op, int32_t slab, int32_t k, double *out,
                    hipStream_t stream);
int ddst_get_center_inverse(const ddst_op_t *op, int32_t j, double *out, hipStream_t stream);

/*
 * Kernel unit hooks (the batched dense kernels of the build, on caller data).
 * Matrices are `batch` contiguous ld x ld row-major device arrays of the
 * given precision (float for DDST_FP32, double for DDST_FP64); ld must be a
 * positive multiple of 128.
 * ddst_test_gemm: C_b = alpha * A_b * diag(bscale_b) * B_b + beta * C_b;
 *   bscale: device float64 batch x ld, or NULL for no scaling.
 * ddst_test_invert: in-place inverse of every A_b by Gauss-Jordan without
 *   pivoting; EBREAKDOWN if a pivot is non-positive or non-finite.
 */
int ddst_test_gemm(int32_t precision, int32_t ld, int32_t batch, const void *A, const void *B,
                   void *C, const double *bscale, double alpha, double beta,
                   hipStream_t stream);
int ddst_test_invert(int32_t precision, int32_t ld, int32_t batch, void *A, hipStream_t stream);
/* ddst_test_invert_sym: the same by the symmetric elimination (each A_b must
 *   be symmetric; of its 128 x 128 tiles only those on and below the
 *   diagonal are read, the inverse is written in full). */
int ddst_test_invert_sym(int32_t precision, int32_t ld, int32_t batch, void *A,
                         hipStream_t stream);

/*
 * Per-kernel-class timing.  ddst_profile_select(kinds) clears the counters
 * and times the classes whose bit (1 << DDST_K_...) is set in `kinds`
 * (0 stops timing and keeps the counters); ddst_profile_enable(1) selects
 * every class, (0) stops.  Each timed launch carries a start and a stop HIP
 * event on the stream it is launched on, attached to the dispatch itself
 * where the launch is a single kernel (or to its first and last kernel), so
 * timing adds no packets to the stream.  ddst_profile_read drains pending
 * events and returns, for one class, the number of launches, their summed
 * duration in ms and their summed algorithmic work (flops for the
 * matrix-core classes, bytes for the others; padding excluded).  Returns
 * DDST_EINVAL for a class index out of range.  Timing state is
 * process-wide, shared by every operator.
 */
enum {
  DDST_K_GJ_PANEL = 0,  /* Gauss-Jordan pivot block inverse + panel   (flops) */
  DDST_K_GJ_UPDATE = 1, /* Gauss-Jordan rank-128 update, MFMA         (flops) */
  DDST_K_GEMM = 2,      /* transfer chains / blocks, MFMA             (flops) */
  DDST_K_ASSEMBLE = 3,  /* plane-block (Schur recursion) assembly     (bytes) */
  DDST_K_GEMV = 4,      /* slab sweeps and interface products         (bytes) */
  DDST_K_GEMV_MANY = 5  /* the same for several right-hand sides: matrix
                           bytes, once per group of 8 vectors         (bytes) */
};
int ddst_profile_select(uint32_t kinds);
int ddst_profile_enable(int32_t on);
int ddst_profile_read(int32_t kind, int64_t *launches, double *total_ms, double *work);
/* Union of the time intervals of the timed launches of one class (ms): less
 * than total_ms when launches of the class overlap on different streams.
 * DDST_EINVAL for a class index out of range or a NULL pointer. */
int ddst_profile_busy(int32_t kind, double *busy_ms);

#ifdef __cplusplus
}
#endif

#endif /* DDST_H */
