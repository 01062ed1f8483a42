// Internal declarations shared by the HIP sources of libddst.
//
// Data layout on the device (ld = M rounded up to a multiple of 128):
//  * every dense interface/plane matrix is ld x ld, row-major; rows/columns
//    >= M are padding: zero coupling, identity on the diagonal, so a padded
//    matrix inverts to blockdiag(inverse, I) and no kernel needs edge tests;
//  * volume vectors are padded per node plane: plane i (1..n) occupies
//    [(i-1)*ld, i*ld), entries >= M are zero;
//  * interface vectors: interface j (1..N_ds) occupies [(j-1)*ld, j*ld).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ddst.h"

struct ddst_op;

namespace ddst {
struct Hodlr;

constexpr int kTile = 128;   // GEMM / update output tile (rows and cols)
constexpr int kNB = 128;     // Gauss-Jordan block width (= kTile)
constexpr int kMaxGmresIter = 20000;  // unrestarted GMRES: basis kept in HBM
constexpr int kGemvChunk = 32;  // rows per partial sum in the transposed GEMV

// Stencil coefficient slots: coef[slot * N + node], node = interior C-order.
// slot 0: diagonal; slot 1+2a: neighbour p - e_a; slot 2+2a: neighbour p + e_a.
inline int coef_slots(int dim) { return 2 * dim + 1; }

// One batched plane-block assembly:
//   D = A_plane - diag(r1) G1 diag(c1) - diag(r2) G2 diag(c2)
// (G1 / G2 may be null).  A_plane is the in-plane FD operator of node plane
// `plane` (1-based); padding rows/cols are set to the identity.
struct AsmJob {
  void *D;
  const void *G1;
  const double *r1, *c1;
  const void *G2;
  const double *r2, *c2;
  int plane;
  int pad_;
};

// One batched GEMM job: C = alpha * A * diag(bscale) * B + beta * C
// (all ld x ld; bscale may be null).
struct GemmJob {
  const void *A;
  const void *B;
  void *C;
  const double *bscale;
};

// One batched GEMV job (vectors float64, matrix type T):
//   out = w + alpha * ( op(G) (x1 - e .* x2) + op(G2) x3 )
// any of x1, e/x2, w, G2/x3 may be null (treated as zero); G may be null
// (then only the G2 term contributes).
struct GemvJob {
  const void *G;
  const double *x1;
  const double *e;
  const double *x2;
  const void *G2;
  const double *x3;
  const double *w;
  double *out;
};

// ---- global-memory access helpers (device code) ---------------------------
// Pointers read from job tables are generic to the compiler, which then
// emits flat loads and stores; those also count against the LDS counter, so
// every wait for LDS data would also wait for outstanding matrix loads.  All
// matrices and vectors live in device memory: these helpers access them
// through global-address-space pointers (16-byte vectors of native vector
// type, which keep the address space through the copy).
template <typename T> struct V16;
template <> struct V16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct V16<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gp(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ typename V16<T>::type ld16(const T *p) {
  return *(__attribute__((address_space(1))) const typename V16<T>::type *)p;
}
template <typename T>
__device__ __forceinline__ void st16(T *p, typename V16<T>::type v) {
  *(__attribute__((address_space(1))) typename V16<T>::type *)p = v;
}

// ---- per-kernel timing (prof.hip) ----------------------------------------
// Kernel classes; the numbering is part of the C-ABI (ddst_profile_read).
enum KernelKind {
  KK_GJ_PANEL = 0,   // Gauss-Jordan pivot block + panel (work: flops)
  KK_GJ_UPDATE = 1,  // Gauss-Jordan rank-kNB update on MFMA (work: flops)
  KK_GEMM = 2,       // transfer-chain / transfer-block GEMM on MFMA (flops)
  KK_ASSEMBLE = 3,   // plane-block assembly (work: bytes)
  KK_GEMV = 4,       // slab sweeps and interface products (work: bytes)
  KK_GEMV_MANY = 5,  // the same products for several right-hand sides (bytes)
  KK_COUNT = 6
};
// Start/stop events of one timed launch (both null when its class is off).
// Single-kernel launches pass them to hipExtLaunchKernelGGL; a sequence of
// kernels gives the start to its first and the stop to its last dispatch.
struct ProfSpan {
  hipEvent_t a = nullptr, b = nullptr;
};
ProfSpan prof_open(int kind);
void prof_close(const ProfSpan &sp, int kind, double work);
// Marker form for sequences whose last kernel is chosen at run time: events
// recorded on s before and after.
void prof_begin(int kind, hipStream_t s);
void prof_end(int kind, hipStream_t s, double work);

// ---- dense kernels (dense.hip) -------------------------------------------
template <typename T>
void launch_assemble(const AsmJob *jobs, int njobs, const double *coef, int n, int dim,
                     int M, int ld, hipStream_t s);
// M (the unpadded size) only enters the algorithmic work recorded by the
// profiler: 2 M^3 flops per GEMM, 2 M^2 kNB per Gauss-Jordan update.
template <typename T>
void launch_scale_cols(const GemmJob *jobs, int njobs, int ld, double alpha, hipStream_t s);
template <typename T>
void launch_gemm(const GemmJob *jobs, int njobs, int ld, int M, double alpha, double beta,
                 hipStream_t s);
// C (ld x ldc) = alpha op(A) diag(bscale) B + beta C: A ld x ld (op = A, or
// A^T when trans), B and C ld x ldc row-major, ldc a multiple of 128 (the
// block products of the sampling chains).  M and ncols (the unpadded sizes)
// only enter the profiler's work: 2 M^2 ncols flops per job.
template <typename T>
void launch_gemm_rect(const GemmJob *jobs, int njobs, int ld, int ldc, int M, int ncols,
                      int trans, double alpha, double beta, hipStream_t s);
// Helper stream and events of the look-ahead Gauss-Jordan schedule, created
// once and reused by every inversion of a build (destroyed with the object).
// Events are created without timing and with device-scope release only (a
// system-scope release writes back the L2 caches, which after an update
// launch holds megabytes of dirty lines); they are attached to the
// dispatches they follow where possible.
struct GjStreams {
  hipStream_t h = nullptr;   // bulk of each update
  hipStream_t x = nullptr;   // the next pivot's row and column blocks
  hipEvent_t panel = nullptr;
  hipEvent_t rest[2] = {nullptr, nullptr};
  hipEvent_t cross[2] = {nullptr, nullptr};
  GjStreams() = default;
  GjStreams(const GjStreams &) = delete;
  GjStreams &operator=(const GjStreams &) = delete;
  hipError_t create();
  ~GjStreams();
};
// Device status words of the local eliminations (32 bytes, zeroed at set-up):
// a breakdown flag, the largest |entry| of any inverted pivot block, and the
// largest |entry| of the FD matrix (bit patterns of non-negative doubles).
// Their product is the pivot growth: a local problem that is singular to
// working precision makes some pivot block's inverse of the order of
// 1 / (eps ||A||), while the entries of a well-posed one stay far below.
struct ElimStatus {
  int bad;
  int pad_;
  unsigned long long inv_max;
  unsigned long long a_max;
  unsigned long long pad2_;
};
static_assert(sizeof(ElimStatus) == 32, "ElimStatus is 32 bytes");
// In-place Gauss-Jordan inversion (no pivoting) of `nmat` ld x ld matrices
// with look-ahead: the pivot and panel kernels of step p + 1 apply step p's
// update to their own row block (on s), while the update of every other
// tile of step p runs on gs.h.  work: gj_workspace_bytes
// bytes (two R and two column panels, the pivot inverses); flag: device
// ElimStatus: bad set to 1 when a pivot is non-finite, or non-positive
// unless any_sign is non-zero, inv_max raised to the largest |entry| of
// the inverted pivot blocks; sym non-zero: the matrices are symmetric and
// only their lower triangle is eliminated (the inverse is mirrored at the
// end).  Everything is ordered before later work on s when the call
// returns.
template <typename T>
hipError_t gj_invert(void *const *mats, int nmat, int ld, int M, void *work, int *flag,
                     int any_sign, int sym, GjStreams &gs, hipStream_t s);
// Bytes of Gauss-Jordan workspace for nmat matrices.
inline size_t gj_workspace_bytes(int nmat, int ld, size_t esz) {
  return (size_t)nmat * kNB * ld * esz * 4 + (size_t)nmat * kNB * kNB * esz;
}

// ---- vector kernels (vec.hip) --------------------------------------------
void launch_setup_coef(const double *kappa, const double *c, const double *bvec3,
                       int dim, int n, double h, double *coef, int *bad, hipStream_t s);
void launch_fill_couplings(const double *coef, int dim, int n, int M, int ld,
                           double *Em, double *Ep, hipStream_t s);
// r = f - A_full(x; g)  (transpose: r = f - A^T x with x = 0 on the boundary,
// g ignored).  x, r padded volumes; f unpadded n^d (nullable); g box (nullable).
void launch_residual(const double *coef, int dim, int n, int M, int ld, const double *f,
                     const double *g, const double *x, double *r, int transpose,
                     hipStream_t s);
void launch_pad(const double *src, double *dst, int rows, int M, int ld, hipStream_t s);
void launch_unpad(const double *src, double *dst, int rows, int M, int ld, hipStream_t s);
template <typename T>
void launch_gemv(const GemvJob *jobs, int njobs, int ld, int M, int transpose, double alpha,
                 double *partial, hipStream_t s);
// Device memory of the library: hipMalloc / hipFree, or the caller's
// allocator set with ddst_set_allocator.  0 bytes gives nullptr.
hipError_t dev_malloc(void **p, size_t bytes);
void dev_free(void *p);

// The same non-transposed products for nv right-hand sides, vector v of every
// job shifted by v * vs (matrices and couplings shared), nv <= 16 (matrix
// cores); nv <= 1 is launch_gemv.
template <typename T>
void launch_gemv_many(const GemvJob *jobs, int njobs, int ld, int M, double alpha, int nv,
                      size_t vs, double *partial, hipStream_t s);
// Interface right-hand sides from the planes next to each interface:
//   out[j] = v[pl] - Ea[pl + a_off] .* Zl[pl - 1] - Eb[pl + b_off] .* Zr[pl + 1],
// pl = j m the interface plane (1-based), v = vol (0 if vol is NULL).
void launch_interface_rhs(const double *vol, const double *Zl, const double *Zr,
                          const double *Ea, const double *Eb, int n_ds, int m, int ld,
                          int a_off, int b_off, double *out, hipStream_t s);
void launch_copy_planes(const double *src, int src_stride, int src_off, double *dst,
                        int dst_stride, int dst_off, int count, int ld, int M,
                        hipStream_t s);
void launch_axpy(double *y, const double *x, double a, size_t len, hipStream_t s);
void launch_fill(double *y, double v, size_t len, hipStream_t s);
// part: at least dots_part_len(len, nvec) doubles of workspace
inline size_t dots_part_len(size_t len, int nvec) { return ((len + 255) / 256) * (size_t)nvec; }
// w += sign V h over nvec basis vectors of stride `stride` (FP64 or FP32
// storage, FP64 arithmetic)
template <typename B>
void launch_mgs_update(double *w, const B *V, size_t stride, int nvec,
                       const double *h, double sign, size_t len, hipStream_t s);
// dst = src rounded to FP32
void launch_to_float(float *dst, const double *src, size_t len, hipStream_t s);
void launch_norm(const double *w, size_t len, double *out, double *part, hipStream_t s);
// GMRES state on the device: packed Hessenberg columns (column k, k + 2
// entries, from offset k (k + 3) / 2), Givens pairs, the rotated right-hand
// side g and per-iteration residual estimates.
__host__ __device__ inline size_t gmres_hoff(int k) { return (size_t)k * (k + 3) / 2; }
// The unrotated Hessenberg matrix by rows (for products H a): row i holds
// columns max(i - 1, 0) .. mi - 1, rows 0 .. mi.
__host__ __device__ inline size_t gmres_roff(int i, int mi) {
  return i == 0 ? 0 : (size_t)mi + (size_t)(i - 1) * (mi + 1) - (size_t)(i - 1) * i / 2;
}
__host__ __device__ inline size_t gmres_rix(int i, int j, int mi) {
  return gmres_roff(i, mi) + (size_t)(j - (i > 0 ? i - 1 : 0));
}
struct GmresDev {
  double *H, *cs, *sn, *g, *res, *y;
  // lagged reorthogonalization (launch_arnoldi_lagged): unrotated columns
  // by rows, the provisional column of the previous step, coefficients and
  // scalars of the current step, pass-A dot products, H a
  double *Hraw, *prov, *cf, *sc, *dA, *dv;
  int maxit;
  static size_t doubles(int max_iter) {
    return gmres_hoff(max_iter) + 6 * (size_t)max_iter + 8 + gmres_roff(max_iter + 1, max_iter) +
           5 * (size_t)(max_iter + 2) + 16;
  }
  void carve(double *base, int max_iter) {
    maxit = max_iter;
    H = base;
    cs = H + gmres_hoff(max_iter);
    sn = cs + max_iter;
    g = sn + max_iter;
    res = g + max_iter + 1;  // pairs (estimate, breakdown flag) per iteration
    y = res + 2 * (size_t)max_iter;
    Hraw = y + max_iter + 8;
    prov = Hraw + gmres_roff(max_iter + 1, max_iter);
    cf = prov + (max_iter + 2);
    dv = cf + (max_iter + 2);
    dA = dv + (max_iter + 2);  // 2 (max_iter + 2)
    sc = dA + 2 * (size_t)(max_iter + 2);  // 16
  }
};
// GMRES iteration k after the matvec w = S v_k: one Arnoldi step by
// classical Gram-Schmidt applied twice (FP64 arithmetic), V the k + 1 basis
// vectors of stride `stride` (stored in FP64 or FP32),
//   h1 = V^T w; w -= V h1; h2 = V^T w; w -= V h2; vnext = w / |w|
// (vnext in FP64; with an FP32 basis also rounded into vslot, slot k + 1;
// vslot null otherwise, vnext being slot k + 1 itself)
// (hd[0..k] = h1, hd[k+1 .. 2k+1] = h2, hd[2k+2] = |w|), then column k of H
// from them: previous rotations applied, the new one formed, g updated;
// res[2k] = |g[k+1]| / beta, res[2k+1] = 1 when the new norm is not
// positive and finite (breakdown: the Krylov space is exhausted; a zero norm
// makes the estimate exactly 0), else 0.  part: dots_part_len(len, k + 1).
template <typename B>
void launch_arnoldi_step(const B *V, size_t stride, int k, double *w, size_t len, double *hd,
                         double *vnext, float *vslot, double *part, GmresDev gd, double beta,
                         hipStream_t s);
// GMRES iteration k with lagged reorthogonalization (two passes over the
// basis instead of four).  V slots 0..k-1 hold the orthonormal q_0..q_{k-1}
// (FP64 or FP32 storage); u (FP64: slot k itself with an FP64 basis, else a
// separate vector) holds the candidate (q_k after one Gram-Schmidt pass,
// normalized); w = S u.  Pass A: a = Q^T u, |u|^2, b = Q^T w, u.w in one sweep; then
// nu = |u - Q a|, column k - 1 of H is finalized (its provisional
// coefficients plus rho a, subdiagonal rho nu) and rotated (res[2(k-1)]);
// q_k = (u - Q a) / nu, and, with d = H a (S Q = Q H), the first pass of
// S q_k = (w - [Q, q_k] d) / nu against [Q, q_k] gives the provisional
// column h of step k and z = S q_k - [Q, q_k] h, formed from w, u and Q in
// pass B (one sweep, which also writes q_k into slot k); unext = z / |z|
// (FP64: slot k + 1, or the separate candidate vector, overwriting u),
// rho = |z|.  col_final: column k - 1 is already final (the previous step
// was a classical one); finalize_only: only pass A for a and nu and the
// finalization of column k - 1 (w unused), to close the last column.
// part: dots_part_len(len, 2 (k + 1)).
template <typename B>
void launch_arnoldi_lagged(B *V, size_t stride, int k, const double *u, double *w,
                           double *unext, size_t len, double *part, GmresDev gd, double beta,
                           int col_final, int finalize_only, hipStream_t s);
// y = R^{-1} g over the first k columns (one work-group), then x = V y.
template <typename B>
void launch_gmres_solution(GmresDev d, int k, double *x, const B *V, size_t len, hipStream_t s);
void launch_scale_by_inv(double *dst, const double *src, const double *nrm, size_t len,
                         hipStream_t s);
void launch_cell_gradient(const double *u, const double *lam, const double *g, int dim,
                          int n, int M, int ld, double h, double *grad, hipStream_t s);
void launch_check_finite(const double *x, size_t len, double lo_exclusive, int *bad,
                         hipStream_t s);
// *out = max(*out, max_e |x_e|) as the bit pattern of a non-negative double
void launch_maxabs(const double *x, size_t len, unsigned long long *out, hipStream_t s);
// dst (M x M float64, row-major) = src (ld x ld of the operator precision)
void launch_extract_block(const void *src, int prec, int M, int ld, double *dst,
                          hipStream_t s);

// ---- allocation-free product (noalloc.hip) ---------------------------------
// Size of the static per-GPU scratch array, the bytes one product needs from
// it (0: form not supported), and the product itself (no allocation, no
// synchronisation).
size_t noalloc_scratch_bytes();
size_t noalloc_need(const ddst_op *op, int which, int trans);
hipError_t noalloc_apply(const ddst_op *op, int which, int trans, const double *x, double *y,
                         hipStream_t s);

// ---- HBS form from samples (hbs.hip) --------------------------------------
struct Hbs;
void hbs_free(ddst_op *op);
bool hbs_ready(const ddst_op *op);
// rank k, s = 3 k + q samples, leaf (<= 0: 2 k), factor storage type;
// omega / psi: caller's M x s probes (device, row-major) or null (Philox,
// seed).  DDST_OK, DDST_EINVAL (*msg says why) or DDST_EBREAKDOWN.
int hbs_compress(ddst_op *op, int k, int q, int leaf, int dtype, const double *omega,
                 const double *psi, uint64_t seed, hipStream_t st, std::string *msg);
void hbs_info(const ddst_op *op, double *bytes, int *rank, double *t_sample_ms,
              double *t_compress_ms);
// y = S x or S^T x through the HBS form (padded interface vectors)
int hbs_apply(const ddst_op *op, const double *x, double *y, int transpose, hipStream_t st);
// Y_b = S_b X and Z_b = S_b^T X for every transfer block b (natural order,
// M x ncols each, b-major) by the sampling chains (test hook).
int hbs_sample_blocks(ddst_op *op, int ncols, const double *X, double *Y, double *Z,
                      hipStream_t st);
// Gaussian rows x cols (row-major) from the Philox-4x32-10 counter generator
// with Box-Muller, counter (row, col, stream_id, 0), key = seed.
void launch_gaussian(double *out, int rows, int cols, uint64_t seed, unsigned stream_id,
                     hipStream_t st);

// ---- compressed form (hodlr.hip) -----------------------------------------
void hodlr_free(ddst_op *op);
bool hodlr_ready(const ddst_op *op);
// returns DDST_OK or DDST_ERANK (then *overflow = the largest rank found)
int hodlr_compress(ddst_op *op, const ddst_compress_opts_t &o, hipStream_t s, int *overflow);
void hodlr_info(const ddst_op *op, double *bytes, int *max_rank, int *min_rank);
// y = S x or S^T x through the compressed blocks (padded interface vectors)
int hodlr_apply_jobs(const ddst_op *op, const double *x, double *y, int transpose,
                     hipStream_t s);

}  // namespace ddst

// The operator object behind the opaque C handle.
struct ddst_op {
  int dim = 0, n = 0, n_slabs = 0, m = 0, M = 0, ld = 0, n_ds = 0, prec = 0;
  double h = 0;
  double bvec[3] = {0, 0, 0};
  size_t N = 0;          // n^dim
  size_t mat_bytes = 0;  // ld*ld*sizeof(T)
  // persistent device storage
  void *arena = nullptr;      // one allocation for everything below
  double *kappa = nullptr;    // (n+1)^dim copy (or null)
  double *c = nullptr;        // n^dim copy (or null)
  double *coef = nullptr;     // (2 dim + 1) * N stencil coefficients
  double *Em = nullptr;       // (n+2) * ld coupling to plane i-1
  double *Ep = nullptr;       // (n+2) * ld coupling to plane i+1
  void *Sinv = nullptr;       // n_ds matrices: inverse interface Schur blocks
  void *S = nullptr;          // 2 n_ds matrices: S_{j,j-1}, S_{j,j+1}
  void *G = nullptr;          // n_slabs*(m-1) factor matrices (own allocation)
  int *flag = nullptr;        // device ElimStatus (breakdown flag, pivot growth)
  double pivot_growth = 0;    // largest pivot growth seen by the last build
  int indefinite = 0;         // 1: negative pivots accepted (indefinite local problems)
  int sym = 0;                // 1: symmetric operator, symmetric local eliminations
  // compressed forms (hodlr.hip: from the dense blocks; hbs.hip: from samples)
  ddst::Hodlr *hodlr = nullptr;
  ddst::Hbs *hbs = nullptr;
  // reusable solve workspace (grown on demand)
  void *ws = nullptr;
  size_t ws_bytes = 0;
  double *hbuf_host = nullptr;  // pinned host staging for GMRES scalars
  size_t hbuf_bytes = 0;
  ddst_stats_t last_build{};
};
