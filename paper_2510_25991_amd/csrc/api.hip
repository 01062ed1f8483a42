// Host side of libddst: the C-ABI entry points of include/ddst.h.
//
// Build (eq. defS, Algorithms 1-2 of the paper, dense form): every single
// slab is swept across its thin x direction by block-tridiagonal elimination,
// all sweeps of all slabs batched into each launch.  Sweep of slab s towards
// an interface, local planes k = 1..m-1 (plane P(k)):
//     D_1 = A_P(1),  G_k = D_k^{-1},
//     D_k = A_P(k) - diag(Eb(P(k))) G_{k-1} diag(Ef(P(k-1))),
//     Y_1 = -G_1 diag(Eb(P(1))),  Y_k = -G_k diag(Eb(P(k))) Y_{k-1},
// with Eb / Ef the couplings towards / away from the sweep's start plane.
// At interface j (plane c = j m) the two sweeps that end there give
//     Sigma_j = A_c - Em(c) G^L Ep(c-1) - Ep(c) G^R Em(c+1)   (= T_jj),
//     S_{j,j-1} = Sigma_j^{-1} (-diag(Em(c)) Y^L),
//     S_{j,j+1} = Sigma_j^{-1} (-diag(Ep(c)) Y^R).
// The left-to-right G_k of every slab are kept for the solve.
//
// Solve (eq. modelS, Section 5): FP64 refinement around the DD solve
//     r = f - A u;   z = A_II^{-1} r_I (slab sweeps);
//     hhat = Sigma^{-1} (r_J - A_JI z);   S delta_J = hhat (GMRES, CGS2, FP64);
//     delta_I = A_II^{-1}(r_I - A_IJ delta_J);   u += delta.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"

namespace ddst {
namespace {
// device allocator: hipMalloc / hipFree unless the caller set hooks
ddst_alloc_fn g_alloc = nullptr;
ddst_free_fn g_free = nullptr;
void *g_ctx = nullptr;
std::atomic<long long> g_live{0};  // library allocations not yet freed
}  // namespace

hipError_t dev_malloc(void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  if (g_alloc) {
    *p = g_alloc(bytes, g_ctx);
    if (!*p) return hipErrorOutOfMemory;
    if (reinterpret_cast<uintptr_t>(*p) & 255) {  // the kernels need 256-byte alignment
      g_free(*p, g_ctx);
      *p = nullptr;
      return hipErrorInvalidValue;
    }
  } else {
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return e;
    }
  }
  ++g_live;
  return hipSuccess;
}

void dev_free(void *p) {
  if (!p) return;
  if (g_free) {
    // as hipFree does: no work that may still read the block is in flight
    (void)hipDeviceSynchronize();
    g_free(p, g_ctx);
  } else {
    (void)hipFree(p);
  }
  --g_live;
}
}  // namespace ddst

using namespace ddst;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw HipError(std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

struct DeviceMem {
  void *p = nullptr;
  size_t bytes = 0;
  DeviceMem() = default;
  explicit DeviceMem(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    if (dev_malloc(&p, b) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    bytes = b;
  }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  ~DeviceMem() { release(); }
  DeviceMem(const DeviceMem &) = delete;
  DeviceMem &operator=(const DeviceMem &) = delete;
};

// Bump allocator over one device allocation (256-byte aligned slices).
struct Carve {
  size_t off = 0;
  size_t take(size_t b) {
    const size_t o = off;
    off += (b + 255) & ~size_t(255);
    return o;
  }
};

// A table of plain structs staged to the device in one copy.
struct JobTable {
  std::vector<unsigned char> host;
  DeviceMem dev;
  template <typename J>
  size_t add(const std::vector<J> &v) {
    const size_t o = (host.size() + 63) & ~size_t(63);
    host.resize(o + v.size() * sizeof(J));
    if (!v.empty()) std::memcpy(host.data() + o, v.data(), v.size() * sizeof(J));
    return o;
  }
  void upload(hipStream_t s) {
    if (host.empty()) return;
    dev.alloc(host.size());
    HIPCHK(hipMemcpyAsync(dev.p, host.data(), host.size(), hipMemcpyHostToDevice, s));
  }
  template <typename J>
  const J *at(size_t o) const {
    return reinterpret_cast<const J *>(static_cast<unsigned char *>(dev.p) + o);
  }
};

inline size_t esize(int prec) { return prec == DDST_FP32 ? sizeof(float) : sizeof(double); }

inline void *mat(void *base, size_t idx, size_t bytes) {
  return static_cast<unsigned char *>(base) + idx * bytes;
}

// ---- sweeps ----------------------------------------------------------------
struct Sweep {
  int slab;
  int dir;      // +1 left-to-right (towards plane (s+1)m), -1 right-to-left
  int y_index;  // index into the transfer-chain buffers, -1 if no chain
  int work;     // first of its work buffers, -1 if stored in the factor store
  int nbuf;     // work buffers: 2 (ping-pong: a transfer chain reads G_k while
                // plane k+1 is formed) or 1 (no chain: plane k+1 is assembled
                // over G_k in place, element by element)
};

struct SweepPlan {
  std::vector<Sweep> sw;
  int n_y = 0, n_work = 0;  // chain buffer pairs, work buffers
};

// Plane (1-based) of local step k of a sweep.
inline int sweep_plane(const ddst_op *op, const Sweep &w, int k) {
  return w.dir > 0 ? w.slab * op->m + k : (w.slab + 1) * op->m - k;
}

struct SweepBuffers {
  void *store = nullptr;  // factor store (n_slabs*(m-1) matrices) or null
  void *work = nullptr;   // n_work matrices
  void *ybuf = nullptr;   // 2 * n_y matrices
};

inline void *sweep_G(const ddst_op *op, const Sweep &w, int k, const SweepBuffers &b) {
  if (w.work < 0) return mat(b.store, (size_t)w.slab * (op->m - 1) + (k - 1), op->mat_bytes);
  return mat(b.work, (size_t)w.work + (w.nbuf == 2 ? (k & 1) : 0), op->mat_bytes);
}
inline void *sweep_Y(const ddst_op *op, const Sweep &w, int k, const SweepBuffers &b) {
  return mat(b.ybuf, (size_t)w.y_index * 2 + (k & 1), op->mat_bytes);
}
inline const double *Ebwd(const ddst_op *op, const Sweep &w, int plane) {
  return (w.dir > 0 ? op->Em : op->Ep) + (size_t)plane * op->ld;
}
inline const double *Efwd(const ddst_op *op, const Sweep &w, int plane) {
  return (w.dir > 0 ? op->Ep : op->Em) + (size_t)plane * op->ld;
}

// Run all sweeps of a plan, batched per local step.  Returns nothing; the
// breakdown flag on the device records pivot failures.
template <typename T>
void run_sweeps(ddst_op *op, const SweepPlan &plan, const SweepBuffers &buf, hipStream_t s) {
  const int m = op->m, ld = op->ld;
  const int nsw = (int)plan.sw.size();
  JobTable tab;
  std::vector<size_t> off_asm(m), off_mats(m), off_y(m);
  std::vector<int> ny_at(m, 0);
  for (int k = 1; k <= m - 1; ++k) {
    std::vector<AsmJob> aj;
    std::vector<void *> mats;
    std::vector<GemmJob> yj;
    for (const Sweep &w : plan.sw) {
      const int P = sweep_plane(op, w, k);
      AsmJob a{};
      a.D = sweep_G(op, w, k, buf);
      a.plane = P;
      if (k > 1) {
        a.G1 = sweep_G(op, w, k - 1, buf);
        a.r1 = Ebwd(op, w, P);
        a.c1 = Efwd(op, w, sweep_plane(op, w, k - 1));
      }
      aj.push_back(a);
      mats.push_back(a.D);
      if (w.y_index >= 0) {
        GemmJob g{};
        g.A = a.D;
        g.B = (k > 1) ? sweep_Y(op, w, k - 1, buf) : nullptr;
        g.C = sweep_Y(op, w, k, buf);
        g.bscale = Ebwd(op, w, P);
        yj.push_back(g);
      }
    }
    off_asm[k - 1] = tab.add(aj);
    off_mats[k - 1] = tab.add(mats);
    off_y[k - 1] = tab.add(yj);
    ny_at[k - 1] = (int)yj.size();
  }
  tab.upload(s);
  DeviceMem gjw(gj_workspace_bytes(nsw, ld, sizeof(T)));
  GjStreams gs;
  HIPCHK(gs.create());
  // The transfer chain of plane k needs only G_k: it runs on a second
  // stream, overlapping the inversion of plane k+1 with its
  // (matrix-core-bound) GEMM.  Before plane k+2 is assembled into the
  // ping-pong slot that held G_k, the main stream waits for that GEMM.
  const bool chains = plan.n_y > 0;
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> ev_gj(m, nullptr), ev_y(m, nullptr);
  auto release = [&]() {
    for (auto e : ev_gj) if (e) (void)hipEventDestroy(e);
    for (auto e : ev_y) if (e) (void)hipEventDestroy(e);
    if (s2) (void)hipStreamDestroy(s2);
  };
  try {
    if (chains) {
      HIPCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
      // stream ordering only: no timing, device-scope release
      const unsigned evf = hipEventDisableTiming | hipEventDisableSystemFence;
      for (int k = 1; k <= m - 1; ++k) {
        HIPCHK(hipEventCreateWithFlags(&ev_gj[k], evf));
        HIPCHK(hipEventCreateWithFlags(&ev_y[k], evf));
      }
    }
    // the chain GEMM of plane k is released after the assembly of plane
    // k + 1 has been enqueued: the (HBM-bound, critical-path) assembly then
    // runs alone and the GEMM overlaps the elimination steps of plane k + 1
    auto chain = [&](int k) {
      if (ny_at[k - 1] <= 0) return;
      HIPCHK(hipEventRecord(ev_gj[k], s));
      HIPCHK(hipStreamWaitEvent(s2, ev_gj[k], 0));
      if (k == 1)
        launch_scale_cols<T>(tab.at<GemmJob>(off_y[0]), ny_at[0], ld, -1.0, s2);
      else
        launch_gemm<T>(tab.at<GemmJob>(off_y[k - 1]), ny_at[k - 1], ld, op->M, -1.0, 0.0, s2);
      HIPCHK(hipEventRecord(ev_y[k], s2));
    };
    for (int k = 1; k <= m - 1; ++k) {
      if (chains && k >= 3) HIPCHK(hipStreamWaitEvent(s, ev_y[k - 2], 0));
      launch_assemble<T>(tab.at<AsmJob>(off_asm[k - 1]), nsw, op->coef, op->n, op->dim, op->M,
                         ld, s);
      if (k >= 2) chain(k - 1);
      HIPCHK(gj_invert<T>(tab.at<void *>(off_mats[k - 1]), nsw, ld, op->M, gjw.p, op->flag,
                          op->indefinite, op->sym, gs, s));
    }
    chain(m - 1);
    if (chains) HIPCHK(hipStreamWaitEvent(s, ev_y[m - 1], 0));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));  // keeps the job tables alive until done
  } catch (...) {
    if (s2) (void)hipStreamSynchronize(s2);
    release();
    throw;
  }
  release();
}

// Left-to-right factor sweeps of every slab (no transfer chains): the part
// of the build the solve and the adjoint need.
SweepPlan factor_plan(const ddst_op *op) {
  SweepPlan p;
  for (int s = 0; s < op->n_slabs; ++s) p.sw.push_back({s, +1, -1, -1, 0});
  return p;
}

// Pivot growth above which an indefinite local problem counts as singular
// to working precision: the inverse of a pivot block of a matrix that is
// singular up to rounding has entries of order 1 / (c eps ||A||).  Measured:
// the definite and indefinite test problems (2D and 3D, up to the first
// double-slab resonances and past them) stay between 1.3 and 1e2; a slab
// whose planes 1..4 have a singular Schur complement gives 1e14 with FP64
// blocks and 7e6 with FP32 ones (whose rounding keeps the pivot near
// 1e-7 ||A|| instead of 1e-16 ||A||).
inline double growth_limit(int prec) { return prec == DDST_FP32 ? 1e5 : 1e12; }

int check_flag(ddst_op *op, hipStream_t s, const char *what) {
  ElimStatus h{};
  HIPCHK(hipMemcpyAsync(&h, op->flag, sizeof(ElimStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double inv_max, a_max;
  std::memcpy(&inv_max, &h.inv_max, 8);
  std::memcpy(&a_max, &h.a_max, 8);
  const double growth = inv_max * a_max;
  op->pivot_growth = std::max(op->pivot_growth, growth);
  // clear the flag and the inverse maximum for the next elimination
  HIPCHK(hipMemsetAsync(op->flag, 0, 16, s));
  if (!h.bad && op->indefinite && !(growth <= growth_limit(op->prec))) {
    char buf[160];
    std::snprintf(buf, sizeof buf,
                  ": local elimination numerically singular (pivot growth %.3g > %.3g): a "
                  "partial-slab Schur complement is singular to working precision",
                  growth, growth_limit(op->prec));
    return fail(DDST_EBREAKDOWN, std::string(what) + buf);
  }
  if (h.bad) {
    return fail(DDST_EBREAKDOWN,
                std::string(what) +
                    (op->indefinite ? ": zero or non-finite pivot in a local elimination "
                                      "(degenerate local problem)"
                                    : ": non-positive or non-finite pivot in a local "
                                      "elimination (degenerate or indefinite local problem; "
                                      "indefinite = 1 accepts the latter)"));
  }
  return DDST_OK;
}

// blocks = 0: the matrix-free set-up (slab factors and interface blocks
// only; no transfer chains, no transfer blocks).
template <typename T>
int build_impl(ddst_op *op, int keep, int blocks, hipStream_t s) {
  const int m = op->m, nsl = op->n_slabs, nds = op->n_ds;
  SweepPlan plan;
  int nwork = 0, ny = 0;
  auto take = [&](bool hasY) {  // work buffers of a sweep that is not stored
    const int first = nwork;
    nwork += hasY ? 2 : 1;
    return first;
  };
  for (int sl = 0; sl < nsl; ++sl) {  // left-to-right, towards Gamma_{sl+1}
    const bool hasY = blocks && sl >= 1 && sl <= nsl - 2;
    const int wk = keep ? -1 : take(hasY);
    plan.sw.push_back({sl, +1, hasY ? ny++ : -1, wk, hasY ? 2 : 1});
  }
  for (int sl = 1; sl < nsl; ++sl) {  // right-to-left, towards Gamma_sl
    const bool hasY = blocks && sl <= nsl - 2;
    const int wk = take(hasY);
    plan.sw.push_back({sl, -1, hasY ? ny++ : -1, wk, hasY ? 2 : 1});
  }
  plan.n_y = ny;
  plan.n_work = nwork;
  SweepBuffers buf;
  if (keep) {
    if (dev_malloc(&op->G, (size_t)nsl * (m - 1) * op->mat_bytes) != hipSuccess) {
      op->G = nullptr;
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    buf.store = op->G;
  }
  DeviceMem work((size_t)nwork * op->mat_bytes);
  DeviceMem ybuf((size_t)2 * std::max(ny, 1) * op->mat_bytes);
  buf.work = work.p;
  buf.ybuf = ybuf.p;
  run_sweeps<T>(op, plan, buf, s);

  // interface centres and transfer blocks
  std::vector<AsmJob> cj;
  std::vector<void *> smats;
  std::vector<GemmJob> sj;
  for (int j = 1; j <= nds; ++j) {
    const int c = j * m;
    const Sweep &L = plan.sw[j - 1];        // slab j-1, left-to-right
    const Sweep &R = plan.sw[nsl + j - 1];  // slab j, right-to-left
    AsmJob a{};
    a.D = mat(op->Sinv, j - 1, op->mat_bytes);
    a.plane = c;
    a.G1 = sweep_G(op, L, m - 1, buf);
    a.r1 = op->Em + (size_t)c * op->ld;
    a.c1 = op->Ep + (size_t)(c - 1) * op->ld;
    a.G2 = sweep_G(op, R, m - 1, buf);
    a.r2 = op->Ep + (size_t)c * op->ld;
    a.c2 = op->Em + (size_t)(c + 1) * op->ld;
    cj.push_back(a);
    smats.push_back(a.D);
    if (!blocks) continue;
    if (j >= 2) {
      GemmJob g{};
      g.A = a.D;
      g.B = sweep_Y(op, L, m - 1, buf);
      g.C = mat(op->S, 2 * (j - 1) + 0, op->mat_bytes);
      g.bscale = op->Em + (size_t)c * op->ld;
      sj.push_back(g);
    }
    if (j <= nds - 1) {
      GemmJob g{};
      g.A = a.D;
      g.B = sweep_Y(op, R, m - 1, buf);
      g.C = mat(op->S, 2 * (j - 1) + 1, op->mat_bytes);
      g.bscale = op->Ep + (size_t)c * op->ld;
      sj.push_back(g);
    }
  }
  JobTable tab;
  const size_t oc = tab.add(cj), om = tab.add(smats), os = tab.add(sj);
  tab.upload(s);
  launch_assemble<T>(tab.at<AsmJob>(oc), nds, op->coef, op->n, op->dim, op->M, op->ld, s);
  DeviceMem gjw(gj_workspace_bytes(nds, op->ld, sizeof(T)));
  GjStreams gs;
  HIPCHK(gs.create());
  HIPCHK(gj_invert<T>(tab.at<void *>(om), nds, op->ld, op->M, gjw.p, op->flag, op->indefinite,
                      op->sym, gs, s));
  if (!sj.empty())
    launch_gemm<T>(tab.at<GemmJob>(os), (int)sj.size(), op->ld, op->M, -1.0, 0.0, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return check_flag(op, s, "ddst_build_transfer");
}

int validate_problem(const ddst_problem_t *p) {
  if (!p) return fail(DDST_EINVAL, "problem is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(DDST_EINVAL, "dim must be 2 or 3");
  if (p->n < 3) return fail(DDST_EINVAL, "n must be >= 3");
  if (p->n_slabs < 2) return fail(DDST_EINVAL, "n_slabs must be >= 2");
  if ((p->n + 1) % p->n_slabs != 0) return fail(DDST_EINVAL, "(n+1) % n_slabs != 0");
  if ((p->n + 1) / p->n_slabs < 2) return fail(DDST_EINVAL, "slab width m must be >= 2");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->bvec[a])) return fail(DDST_EINVAL, "bvec not finite");
  const double M = std::pow((double)p->n, p->dim - 1);
  if (M > 65536.0) return fail(DDST_EINVAL, "interface too large (M > 65536)");
  return DDST_OK;
}

void destroy_op(ddst_op *op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  hodlr_free(op);
  hbs_free(op);
  if (op->G) dev_free(op->G);
  if (op->arena) dev_free(op->arena);
  if (op->ws) dev_free(op->ws);
  if (op->hbuf_host) (void)hipHostFree(op->hbuf_host);
  delete op;
}

int build_entry(const ddst_problem_t *prob, const ddst_build_opts_t *opts, hipStream_t s,
                ddst_op_t **out) {
  if (!out) return fail(DDST_EINVAL, "out is NULL");
  *out = nullptr;
  int st = validate_problem(prob);
  if (st) return st;
  ddst_build_opts_t o{DDST_FP32, 1, 0, 0, 0, DDST_ELIM_AUTO};
  if (opts) o = *opts;
  if (o.precision != DDST_FP32 && o.precision != DDST_FP64)
    return fail(DDST_EINVAL, "precision must be DDST_FP32 or DDST_FP64");
  if (o.transpose != 0) return fail(DDST_EINVAL, "transpose builds are not supported");
  if (o.skip_transfer != 0 && o.skip_transfer != 1)
    return fail(DDST_EINVAL, "skip_transfer must be 0 or 1");
  if (o.skip_transfer && !o.keep_factors)
    return fail(DDST_EINVAL, "skip_transfer needs keep_factors (the matrix-free apply reads them)");
  if (o.indefinite != 0 && o.indefinite != 1)
    return fail(DDST_EINVAL, "indefinite must be 0 or 1");
  if (o.elimination != DDST_ELIM_AUTO && o.elimination != DDST_ELIM_GENERAL)
    return fail(DDST_EINVAL, "elimination must be DDST_ELIM_AUTO or DDST_ELIM_GENERAL");
  const int blocks = o.skip_transfer ? 0 : 1;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  ddst_op *op = new ddst_op();
  try {
    op->dim = prob->dim;
    op->n = prob->n;
    op->n_slabs = prob->n_slabs;
    op->m = (prob->n + 1) / prob->n_slabs;
    op->n_ds = prob->n_slabs - 1;
    op->M = prob->dim == 2 ? prob->n : prob->n * prob->n;
    op->ld = (op->M + kTile - 1) / kTile * kTile;
    op->N = (size_t)op->M * op->n;
    op->h = 1.0 / (prob->n + 1);
    op->prec = o.precision;
    op->indefinite = o.indefinite;
    for (int a = 0; a < 3; ++a) op->bvec[a] = prob->bvec[a];
    // the FD matrix is symmetric without convection (diffusion with
    // edge-averaged coefficients and a diagonal zeroth-order term), and so
    // are its plane blocks, their Schur complements and the interface
    // blocks.  Indefinite local problems keep the general elimination: past
    // a double-slab resonance the transfer blocks amplify the rounding of
    // the local inverses, and the symmetric one (which projects each input
    // onto symmetric matrices) lost a factor ~30 there in FP64.
    op->sym = o.elimination == DDST_ELIM_AUTO && !o.indefinite && prob->bvec[0] == 0.0 &&
              prob->bvec[1] == 0.0 && (prob->dim == 2 || prob->bvec[2] == 0.0);
    op->mat_bytes = (size_t)op->ld * op->ld * esize(op->prec);
    const size_t ncell = (size_t)std::pow((double)(op->n + 1), op->dim) + 0.5;
    Carve cv;
    const size_t o_kap = prob->kappa ? cv.take(ncell * 8) : 0;
    const size_t o_c = prob->c ? cv.take(op->N * 8) : 0;
    const size_t o_coef = cv.take((size_t)coef_slots(op->dim) * op->N * 8);
    const size_t o_em = cv.take((size_t)(op->n + 2) * op->ld * 8);
    const size_t o_ep = cv.take((size_t)(op->n + 2) * op->ld * 8);
    const size_t o_si = cv.take((size_t)op->n_ds * op->mat_bytes);
    const size_t o_s = blocks ? cv.take((size_t)2 * op->n_ds * op->mat_bytes) : 0;
    const size_t o_fl = cv.take(sizeof(ElimStatus));
    if (dev_malloc(&op->arena, cv.off) != hipSuccess) {
      op->arena = nullptr;
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    auto at = [&](size_t o) { return static_cast<unsigned char *>(op->arena) + o; };
    op->kappa = prob->kappa ? reinterpret_cast<double *>(at(o_kap)) : nullptr;
    op->c = prob->c ? reinterpret_cast<double *>(at(o_c)) : nullptr;
    op->coef = reinterpret_cast<double *>(at(o_coef));
    op->Em = reinterpret_cast<double *>(at(o_em));
    op->Ep = reinterpret_cast<double *>(at(o_ep));
    op->Sinv = at(o_si);
    op->S = blocks ? at(o_s) : nullptr;
    op->flag = reinterpret_cast<int *>(at(o_fl));
    HIPCHK(hipMemsetAsync(op->flag, 0, sizeof(ElimStatus), s));
    if (op->S) HIPCHK(hipMemsetAsync(op->S, 0, (size_t)2 * op->n_ds * op->mat_bytes, s));
    if (op->kappa) {
      HIPCHK(hipMemcpyAsync(op->kappa, prob->kappa, ncell * 8, hipMemcpyDeviceToDevice, s));
      launch_check_finite(op->kappa, ncell, 0.0, op->flag, s);
    }
    if (op->c) {
      HIPCHK(hipMemcpyAsync(op->c, prob->c, op->N * 8, hipMemcpyDeviceToDevice, s));
      launch_check_finite(op->c, op->N, -1.7976931348623157e308, op->flag, s);
    }
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, op->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) {
      destroy_op(op);
      return fail(DDST_EINVAL, "kappa must be finite and > 0, c finite");
    }
    launch_setup_coef(op->kappa, op->c, op->bvec, op->dim, op->n, op->h, op->coef, nullptr, s);
    launch_maxabs(op->coef, (size_t)coef_slots(op->dim) * op->N,
                  &reinterpret_cast<ElimStatus *>(op->flag)->a_max, s);
    launch_fill_couplings(op->coef, op->dim, op->n, op->M, op->ld, op->Em, op->Ep, s);
    HIPCHK(hipGetLastError());
    const int keep = o.keep_factors ? 1 : 0;
    st = (op->prec == DDST_FP32) ? build_impl<float>(op, keep, blocks, s)
                                 : build_impl<double>(op, keep, blocks, s);
    if (st) {
      destroy_op(op);
      return st;
    }
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    op->last_build.t_build_ms = ms;
    op->last_build.bytes_transfer = op->S ? (double)2 * op->n_ds * op->mat_bytes : 0;
    op->last_build.bytes_factors = op->G ? (double)op->n_slabs * (op->m - 1) * op->mat_bytes : 0;
    op->last_build.pivot_growth = op->pivot_growth;
    op->last_build.symmetric = op->sym;
  } catch (...) {
    destroy_op(op);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *out = op;
  return DDST_OK;
}

// ---- solve ------------------------------------------------------------------
struct SolveWs {
  double *X, *R, *Z, *D;     // padded volumes (n*ld)
  double *fJ, *hh, *W, *xg;  // interface vectors (n_ds*ld)
  double *Zf, *Zb;           // padded volumes of the matrix-free apply's chains
  double *mfx, *mfv, *mff;   // interface vectors of the matrix-free apply
  double *rr, *dx;           // restarted GMRES: residual and cycle correction
  double *V;                 // Krylov basis (max_iter+1) * n_ds*ld
  double *hd;                // small scalars
  double *part;              // transposed-GEMV partial sums
  double *dpart;             // dot-product partial sums
  double *nrm;               // norms
  GmresDev gm;               // device GMRES state
  size_t vol, ifc;           // one right-hand side's volume / interface length
  int nr;                    // right-hand sides held (vectors nr * vol, nr * ifc)
  bool basis32 = false;      // FP32 Krylov basis allowed (ddst_solve_opts_t::basis_fp32)
};

void ensure_ws(ddst_op *op, size_t bytes) {
  if (op->ws_bytes >= bytes) return;
  if (op->ws) dev_free(op->ws);
  op->ws = nullptr;
  op->ws_bytes = 0;
  if (dev_malloc(&op->ws, bytes) != hipSuccess) {
    op->ws = nullptr;
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  op->ws_bytes = bytes;
}

SolveWs carve_ws(ddst_op *op, int max_iter, int nr = 1) {
  const size_t vol1 = (size_t)op->n * op->ld, ifc1 = (size_t)op->n_ds * op->ld;
  const size_t vol = vol1 * nr, ifc = ifc1 * nr;
  const int nchunk = std::min(op->ld / kGemvChunk, 64);
  // transposed GEMVs: at most 2 n_slabs jobs (the matrix-free chains)
  const size_t part = (size_t)2 * op->n_slabs * nchunk * op->ld;
  Carve cv;
  size_t o[13];
  o[0] = cv.take(vol * 8); o[1] = cv.take(vol * 8); o[2] = cv.take(vol * 8);
  o[3] = cv.take(vol * 8);
  o[4] = cv.take(ifc * 8); o[5] = cv.take(ifc * 8); o[6] = cv.take(ifc * 8);
  o[7] = cv.take(ifc * 8);
  o[8] = cv.take((size_t)(max_iter + 1) * ifc * 8);
  o[9] = cv.take((size_t)(4 * max_iter + 16) * 8);
  o[10] = cv.take(part * 8);
  o[11] = cv.take(64 * 8);
  // partial sums: up to 2 (max_iter + 2) interface-length dots (the lagged
  // Arnoldi step's pass A), or one volume norm
  o[12] = cv.take(std::max(dots_part_len(ifc, 2 * (max_iter + 2)), dots_part_len(vol, 1)) * 8);
  const size_t o_gm = cv.take(GmresDev::doubles(max_iter) * 8);
  const size_t o_zf = cv.take(vol * 8), o_zb = cv.take(vol * 8);
  const size_t o_mx = cv.take(ifc * 8), o_mv = cv.take(ifc * 8), o_mf = cv.take(ifc * 8);
  const size_t o_rr = cv.take(ifc * 8), o_dx = cv.take(ifc * 8);
  ensure_ws(op, cv.off);
  auto at = [&](size_t x) {
    return reinterpret_cast<double *>(static_cast<unsigned char *>(op->ws) + x);
  };
  SolveWs w;
  w.X = at(o[0]); w.R = at(o[1]); w.Z = at(o[2]); w.D = at(o[3]);
  w.fJ = at(o[4]); w.hh = at(o[5]); w.W = at(o[6]); w.xg = at(o[7]);
  w.V = at(o[8]); w.hd = at(o[9]); w.part = at(o[10]); w.nrm = at(o[11]); w.dpart = at(o[12]);
  w.gm.carve(at(o_gm), max_iter);
  w.Zf = at(o_zf); w.Zb = at(o_zb);
  w.mfx = at(o_mx); w.mfv = at(o_mv); w.mff = at(o_mf);
  w.rr = at(o_rr); w.dx = at(o_dx);
  w.vol = vol1;
  w.ifc = ifc1;
  w.nr = nr;
  return w;
}

// Slab-solve job tables: forward and backward block-Thomas sweeps of every
// single slab with the stored left-to-right factors (or their transposes).
//   forward  : y_k = op(G_k) (r_P(k) - e_f(k) .* y_{k-1}),  y_0 = left trace
//   backward : z_k = y_k - op(G_k) (e_b(k) .* z_{k+1}),      z_m = right trace
// e_f(k) = Em(P(k)), e_b(k) = Ep(P(k)) for A; Ep(P(k)-1), Em(P(k)+1) for A^T.
struct SlabTables {
  JobTable tab;
  std::vector<size_t> fwd, bwd;
  std::vector<int> nfwd, nbwd;
};

void make_slab_tables(const ddst_op *op, const void *G, const double *R, double *Vol,
                      bool with_traces, bool transpose, SlabTables &t) {
  const int m = op->m, ld = op->ld;
  const size_t mb = op->mat_bytes;
  t.fwd.assign(m, 0);
  t.bwd.assign(m, 0);
  t.nfwd.assign(m, 0);
  t.nbwd.assign(m, 0);
  for (int k = 1; k <= m - 1; ++k) {
    std::vector<GemvJob> jf, jb;
    for (int s = 0; s < op->n_slabs; ++s) {
      const int P = s * m + k;
      const void *Gk = mat(const_cast<void *>(G), (size_t)s * (m - 1) + (k - 1), mb);
      GemvJob f{};
      f.G = Gk;
      f.x1 = R + (size_t)(P - 1) * ld;
      const bool left = (k > 1) || (with_traces && s >= 1);
      if (left) {
        f.e = transpose ? op->Ep + (size_t)(P - 1) * ld : op->Em + (size_t)P * ld;
        f.x2 = Vol + (size_t)(P - 2) * ld;
      }
      f.out = Vol + (size_t)(P - 1) * ld;
      jf.push_back(f);
      GemvJob b{};
      const bool right = (k < m - 1) || (with_traces && s + 1 <= op->n_ds);
      b.G = right ? Gk : nullptr;
      if (right) {
        b.e = transpose ? op->Em + (size_t)(P + 1) * ld : op->Ep + (size_t)P * ld;
        b.x2 = Vol + (size_t)P * ld;
      }
      b.w = Vol + (size_t)(P - 1) * ld;
      b.out = Vol + (size_t)(P - 1) * ld;
      jb.push_back(b);
    }
    t.fwd[k] = t.tab.add(jf);
    t.nfwd[k] = (int)jf.size();
    if (k < m - 1 || with_traces) {
      t.bwd[k] = t.tab.add(jb);
      t.nbwd[k] = (int)jb.size();
    }
  }
}

// nr right-hand sides: volume v of each is v * vs after the tables' volumes
// (transposed sweeps take one).
template <typename T>
void run_slab_solve(const ddst_op *op, const SlabTables &t, bool transpose, double *part,
                    hipStream_t s, int nr = 1, size_t vs = 0) {
  const int m = op->m;
  if (transpose && nr > 1) throw std::logic_error("transposed sweeps take one right-hand side");
  auto go = [&](size_t off, int n) {
    if (transpose)
      launch_gemv<T>(t.tab.at<GemvJob>(off), n, op->ld, op->M, 1, 1.0, part, s);
    else
      launch_gemv_many<T>(t.tab.at<GemvJob>(off), n, op->ld, op->M, 1.0, nr, vs, part, s);
  };
  for (int k = 1; k <= m - 1; ++k) go(t.fwd[k], t.nfwd[k]);
  for (int k = m - 1; k >= 1; --k)
    if (t.nbwd[k] > 0) go(t.bwd[k], t.nbwd[k]);
}

// Interface operator jobs: y = S x (or S^T x) for a fixed pair (x, y).
std::vector<GemvJob> interface_jobs(const ddst_op *op, const double *x, double *y, bool trans) {
  std::vector<GemvJob> jobs;
  const int nds = op->n_ds, ld = op->ld;
  const size_t mb = op->mat_bytes;
  for (int j = 1; j <= nds; ++j) {
    GemvJob g{};
    if (!trans) {
      if (j >= 2) { g.G = mat(op->S, 2 * (j - 1) + 0, mb); g.x1 = x + (size_t)(j - 2) * ld; }
      if (j <= nds - 1) { g.G2 = mat(op->S, 2 * (j - 1) + 1, mb); g.x3 = x + (size_t)j * ld; }
    } else {
      if (j >= 2) { g.G = mat(op->S, 2 * (j - 2) + 1, mb); g.x1 = x + (size_t)(j - 2) * ld; }
      if (j <= nds - 1) { g.G2 = mat(op->S, 2 * j + 0, mb); g.x3 = x + (size_t)j * ld; }
    }
    g.w = x + (size_t)(j - 1) * ld;
    g.out = y + (size_t)(j - 1) * ld;
    jobs.push_back(g);
  }
  return jobs;
}

std::vector<GemvJob> sinv_jobs(const ddst_op *op, const double *x, double *y) {
  std::vector<GemvJob> jobs;
  for (int j = 1; j <= op->n_ds; ++j) {
    GemvJob g{};
    g.G = mat(op->Sinv, j - 1, op->mat_bytes);
    g.x1 = x + (size_t)(j - 1) * op->ld;
    g.out = y + (size_t)(j - 1) * op->ld;
    jobs.push_back(g);
  }
  return jobs;
}

// Matrix-free application of the equilibrium matrix (the alternative to
// forming the transfer blocks, Sections 2.2 and 5.1): only the stored
// left-to-right factors G_k of the single slabs and the interface blocks
// Sigma_j^{-1} are read.  With O the couplings between different interfaces
// of the interface Schur complement, S x = x + Sigma^{-1} O x and
//   (O x)_j = Em(c) .* a_{j-1} + Ep(c) .* b_j        (c = j m),
// where a_s is the plane next to the right interface of slab s for Dirichlet
// data x on its left interface only and b_s the plane next to its left
// interface for data on its right interface only:
//   a: y_1 = G_1 (-Em(P(1)) .* x_s),  y_k = G_k (-Em(P(k)) .* y_{k-1}),  a_s = y_{m-1};
//   b: z_{m-1} = G_{m-1} (-Ep(P(m-1)) .* x_{s+1}),  z_k = G_k (-Ep(P(k)) .* z_{k+1}),
//      b_s = z_1.
// The interface sum is -f with f = interface_rhs(0, a, b).  Transposed:
// S^T x = x + O^T Sigma^{-T} x, and O^T is the same two chains with G_k^T
// and the couplings of A^T (Ep(P-1) towards P-1, Em(P+1) towards P+1).
// Slabs next to the physical boundary have one interface and no chain; the
// planes they would fill stay zero.  Launch i = 1..m-1 takes step k = i of
// every a-chain and step k = m-i of every b-chain (2 (n_slabs - 2) jobs).
struct MatfreeTables {
  JobTable tab;
  std::vector<size_t> chain;  // per launch i = 1..m-1 (index i-1)
  int nchain = 0;             // jobs per chain launch
  size_t sinv = 0;            // n_ds jobs with Sigma_j^{-1}
};

struct MatfreeBufs {
  double *X, *V, *F;  // input copy, Sigma^{-T} X (transposed only), f
  double *Zf, *Zb;    // padded volumes: a-chain and b-chain planes
  double *y;          // output
};

void make_matfree_tables(const ddst_op *op, const void *G, bool trans, const MatfreeBufs &b,
                         MatfreeTables &t) {
  const int m = op->m, ld = op->ld;
  const size_t mb = op->mat_bytes;
  const double *data = trans ? b.V : b.X;  // Dirichlet data of the chains
  t.chain.assign(m - 1, 0);
  t.nchain = 2 * std::max(op->n_slabs - 2, 0);
  for (int i = 1; i <= m - 1; ++i) {
    std::vector<GemvJob> jobs;
    for (int s = 1; s <= op->n_slabs - 2; ++s) {
      int k = i, P = s * m + k;
      GemvJob a{};
      a.G = mat(const_cast<void *>(G), (size_t)s * (m - 1) + (k - 1), mb);
      a.e = trans ? op->Ep + (size_t)(P - 1) * ld : op->Em + (size_t)P * ld;
      a.x2 = (k == 1) ? data + (size_t)(s - 1) * ld : b.Zf + (size_t)(P - 2) * ld;
      a.out = b.Zf + (size_t)(P - 1) * ld;
      jobs.push_back(a);
      k = m - i;
      P = s * m + k;
      GemvJob z{};
      z.G = mat(const_cast<void *>(G), (size_t)s * (m - 1) + (k - 1), mb);
      z.e = trans ? op->Em + (size_t)(P + 1) * ld : op->Ep + (size_t)P * ld;
      z.x2 = (k == m - 1) ? data + (size_t)s * ld : b.Zb + (size_t)P * ld;
      z.out = b.Zb + (size_t)(P - 1) * ld;
      jobs.push_back(z);
    }
    t.chain[i - 1] = t.tab.add(jobs);
  }
  std::vector<GemvJob> sj;
  for (int j = 1; j <= op->n_ds; ++j) {
    GemvJob g{};
    g.G = mat(op->Sinv, j - 1, mb);
    if (!trans) {  // y = X - Sigma^{-1} f
      g.x1 = b.F + (size_t)(j - 1) * ld;
      g.w = b.X + (size_t)(j - 1) * ld;
      g.out = b.y + (size_t)(j - 1) * ld;
    } else {  // V = Sigma^{-T} X
      g.x1 = b.X + (size_t)(j - 1) * ld;
      g.out = b.V + (size_t)(j - 1) * ld;
    }
    sj.push_back(g);
  }
  t.sinv = t.tab.add(sj);
}

// y = S X (or S^T X) with the tables above; Zf and Zb must hold zeros in
// the planes no chain writes (fill them once per set of tables).
template <typename T>
void run_matfree(const ddst_op *op, const MatfreeTables &t, bool trans, const MatfreeBufs &b,
                 double *part, hipStream_t s) {
  const int ld = op->ld, M = op->M;
  const size_t len = (size_t)op->n_ds * ld;
  if (trans) launch_gemv<T>(t.tab.at<GemvJob>(t.sinv), op->n_ds, ld, M, 1, 1.0, part, s);
  if (t.nchain > 0)
    for (int i = 1; i <= op->m - 1; ++i)
      launch_gemv<T>(t.tab.at<GemvJob>(t.chain[i - 1]), t.nchain, ld, M, trans ? 1 : 0, 1.0,
                     part, s);
  if (!trans) {
    launch_interface_rhs(nullptr, b.Zf, b.Zb, op->Em, op->Ep, op->n_ds, op->m, ld, 0, 0, b.F,
                         s);
    launch_gemv<T>(t.tab.at<GemvJob>(t.sinv), op->n_ds, ld, M, 0, -1.0, part, s);
  } else {
    launch_interface_rhs(nullptr, b.Zf, b.Zb, op->Ep, op->Em, op->n_ds, op->m, ld, -1, +1,
                         b.F, s);
    HIPCHK(hipMemcpyAsync(b.y, b.X, len * 8, hipMemcpyDeviceToDevice, s));
    launch_axpy(b.y, b.F, -1.0, len, s);
  }
}

// Unrestarted GMRES with classical Gram-Schmidt applied twice (FP64).
// Basis vectors are padded interface vectors.  The Givens rotations run on
// the device (one tiny kernel per iteration) and the host reads the
// residual estimates back at most every kGmresCheck iterations (sooner when
// the observed reduction rate predicts the tolerance), so the GPU is fed
// several iterations ahead; iterations past the stopping point are computed
// and discarded (they touch only later columns).
// With several right-hand sides (w.nr > 1) the basis vectors are their
// interface vectors stacked, i.e. GMRES on the block-diagonal system
// diag(S, ..., S) (one Krylov polynomial for all, inner products summed
// over all: the "global" GMRES of several right-hand sides), so that each
// product reads every block of S once for all of them.
// Once the basis holds more than kLagBytes, each step orthogonalizes with
// lagged reorthogonalization (launch_arnoldi_lagged: two passes over the
// basis instead of four, one column of H finalized a step later); below
// that, the classical twice-applied Gram-Schmidt step, whose fewer launches
// cost less than the passes saved.
// When the caller allows it (basis_fp32) and the tolerance is at least
// kBasis32Tol the basis is stored in FP32
// (half the bytes of the passes over it, which dominate long runs): each
// q_j is rounded once when it is final (2^-24 relative), while the candidate
// vector the operator is applied to and every sum stay FP64 (the candidate
// in a separate FP64 vector after the FP32 slots).  The Arnoldi relation and
// the solution x = V y then hold to about 1e-7 relative, far below such a
// tolerance; an inner solve of iterative refinement at 1e-4 is the case.
// Returns the iterations used.
constexpr int kGmresCheck = 8;
constexpr size_t kLagBytes = (size_t)16 << 20;
constexpr double kBasis32Tol = 1e-6;

template <typename T>
int gmres_cycle(ddst_op *op, SolveWs &w, const void *G, const double *rhs, double *x, double tol,
                int max_iter, bool trans, int form, double *relres, hipStream_t s) {
  const int nr = w.nr;
  if (trans && nr > 1) throw std::logic_error("the transposed solve takes one right-hand side");
  const size_t len = w.ifc * nr;
  double *hh = op->hbuf_host;
  launch_norm(rhs, len, w.nrm, w.dpart, s);
  HIPCHK(hipMemcpyAsync(hh, w.nrm, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double beta = hh[0];
  launch_fill(x, 0.0, len, s);
  *relres = 0.0;
  if (!(beta > 0.0)) return 0;
  // FP32 basis: (max_iter + 1) FP32 slots, then the FP64 candidate (the
  // region holds max_iter + 1 FP64 slots, so both fit for max_iter >= 2)
  const bool b32 = w.basis32 && tol >= kBasis32Tol && max_iter >= 2 && len >= 64;
  float *V32 = reinterpret_cast<float *>(w.V);
  double *ucur =
      b32 ? reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(w.V) +
                                       ((size_t)(max_iter + 1) * len * 4 + 255) / 256 * 256)
          : nullptr;
  launch_scale_by_inv(b32 ? ucur : w.V, rhs, w.nrm, len, s);
  if (b32) launch_to_float(V32, ucur, len, s);
  // operator input of step k: slot k, or the FP64 candidate
  auto vin = [&](int k) -> double * { return b32 ? ucur : w.V + (size_t)k * len; };
  // matvec tables for every basis vector
  JobTable tab;
  std::vector<size_t> offs(max_iter);
  if (form == DDST_APPLY_DENSE)
    for (int k = 0; k < max_iter; ++k)
      offs[k] = (b32 && k > 0) ? offs[0] : tab.add(interface_jobs(op, vin(k), w.W, trans));
  tab.upload(s);
  std::vector<MatfreeTables> mf(form == DDST_APPLY_MATFREE ? nr : 0);
  std::vector<MatfreeBufs> mb;
  for (int v = 0; v < (int)mf.size(); ++v) {
    const size_t oi = (size_t)v * w.ifc, ov = (size_t)v * w.vol;
    mb.push_back({w.mfx + oi, w.mfv + oi, w.mff + oi, w.Zf + ov, w.Zb + ov, w.W + oi});
    make_matfree_tables(op, G, trans, mb[v], mf[v]);
    mf[v].tab.upload(s);
  }
  if (!mf.empty()) {
    launch_fill(w.Zf, 0.0, w.vol * nr, s);
    launch_fill(w.Zb, 0.0, w.vol * nr, s);
  }
  GmresDev d = w.gm;
  int used = 0;
  double res = 1.0;
  int checked = 0;  // columns whose estimates were read back
  int nfinal = 0;   // columns of H finalized by the steps enqueued so far
  int next_check = std::min(kGmresCheck, max_iter);
  double prev_res = 1.0;
  auto lagged = [&](int k) { return (size_t)(k + 1) * len * (b32 ? 4 : 8) >= kLagBytes; };
  // read back the estimates of the columns finalized since the last check
  auto check = [&]() {
    const int n = nfinal - checked;
    if (n <= 0) return;
    HIPCHK(hipMemcpyAsync(hh, d.res + 2 * (size_t)checked, (size_t)n * 16,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
      res = hh[2 * i];
      // stop at the tolerance or at a breakdown (the new direction
      // vanished: the Krylov space is exhausted)
      if (res <= tol || hh[2 * i + 1] != 0.0) {
        used = checked + i + 1;
        break;
      }
    }
    if (used == 0) {
      // next read-back: when the reduction rate seen over this window
      // predicts the tolerance, at most kGmresCheck iterations ahead
      int step = kGmresCheck;
      if (res > 0.0 && res < prev_res) {
        const double rate = std::log(res / prev_res) / n;  // per iteration, < 0
        const double need = std::ceil(std::log(tol / res) / rate);
        if (need < step) step = std::max(1, (int)need);
      }
      prev_res = res;
      next_check = std::min(nfinal + step, max_iter);
    }
    checked = nfinal;
  };
  for (int k = 0; k < max_iter && used == 0; ++k) {
    const double *vk = vin(k);
    if (form == DDST_APPLY_HODLR || form == DDST_APPLY_HBS) {
      for (int v = 0; v < nr; ++v) {
        const size_t oi = (size_t)v * w.ifc;
        const int st = form == DDST_APPLY_HBS
                           ? hbs_apply(op, vk + oi, w.W + oi, trans ? 1 : 0, s)
                           : hodlr_apply_jobs(op, vk + oi, w.W + oi, trans ? 1 : 0, s);
        if (st) throw HipError("compressed apply failed");
      }
    } else if (form == DDST_APPLY_MATFREE) {
      HIPCHK(hipMemcpyAsync(w.mfx, vk, len * 8, hipMemcpyDeviceToDevice, s));
      for (int v = 0; v < nr; ++v) run_matfree<T>(op, mf[v], trans, mb[v], w.part, s);
    } else if (trans) {
      launch_gemv<T>(tab.at<GemvJob>(offs[k]), op->n_ds, op->ld, op->M, 1, -1.0, w.part, s);
    } else {
      launch_gemv_many<T>(tab.at<GemvJob>(offs[k]), op->n_ds, op->ld, op->M, -1.0, nr, w.ifc,
                          w.part, s);
    }
    if (lagged(k)) {
      const int cf = (k >= 1 && !lagged(k - 1)) ? 1 : 0;
      if (b32)
        launch_arnoldi_lagged<float>(V32, len, k, ucur, w.W, ucur, len, w.dpart, d, beta, cf, 0,
                                     s);
      else
        launch_arnoldi_lagged<double>(w.V, len, k, w.V + (size_t)k * len, w.W,
                                      w.V + (size_t)(k + 1) * len, len, w.dpart, d, beta, cf, 0,
                                      s);
      nfinal = k;
    } else {
      if (b32)
        launch_arnoldi_step<float>(V32, len, k, w.W, len, w.hd, ucur, V32 + (size_t)(k + 1) * len,
                                   w.dpart, d, beta, s);
      else
        launch_arnoldi_step<double>(w.V, len, k, w.W, len, w.hd, w.V + (size_t)(k + 1) * len,
                                    nullptr, w.dpart, d, beta, s);
      nfinal = k + 1;
    }
    if (nfinal >= next_check) check();
  }
  if (used == 0 && nfinal < max_iter && max_iter > 0 && lagged(max_iter - 1)) {
    // close the last column (its reorthogonalization coefficients)
    const int cf = (max_iter >= 1 && !lagged(max_iter - 1)) ? 1 : 0;
    if (b32)
      launch_arnoldi_lagged<float>(V32, len, max_iter, ucur, nullptr, nullptr, len, w.dpart, d,
                                   beta, cf, 1, s);
    else
      launch_arnoldi_lagged<double>(w.V, len, max_iter, w.V + (size_t)max_iter * len, nullptr,
                                    nullptr, len, w.dpart, d, beta, cf, 1, s);
    nfinal = max_iter;
  }
  if (used == 0) check();
  if (used == 0) used = checked;
  if (b32)
    launch_gmres_solution<float>(d, used, x, V32, len, s);
  else
    launch_gmres_solution<double>(d, used, x, w.V, len, s);
  HIPCHK(hipStreamSynchronize(s));
  *relres = res;
  return used;
}

// out = S in (or S^T in) for the w.nr stacked interface vectors, through
// form `form` (tables built per call: once per restart cycle).
template <typename T>
void stacked_apply(ddst_op *op, SolveWs &w, const void *G, int form, bool trans,
                   const double *in, double *out, hipStream_t s) {
  const int nr = w.nr;
  if (form == DDST_APPLY_HODLR || form == DDST_APPLY_HBS) {
    for (int v = 0; v < nr; ++v) {
      const size_t oi = (size_t)v * w.ifc;
      const int st = form == DDST_APPLY_HBS
                         ? hbs_apply(op, in + oi, out + oi, trans ? 1 : 0, s)
                         : hodlr_apply_jobs(op, in + oi, out + oi, trans ? 1 : 0, s);
      if (st) throw HipError("compressed apply failed");
    }
  } else if (form == DDST_APPLY_MATFREE) {
    launch_fill(w.Zf, 0.0, w.vol * nr, s);
    launch_fill(w.Zb, 0.0, w.vol * nr, s);
    for (int v = 0; v < nr; ++v) {
      const size_t oi = (size_t)v * w.ifc, ov = (size_t)v * w.vol;
      const MatfreeBufs b{const_cast<double *>(in) + oi, w.mfv + oi, w.mff + oi, w.Zf + ov,
                          w.Zb + ov, out + oi};
      MatfreeTables t;
      make_matfree_tables(op, G, trans, b, t);
      t.tab.upload(s);
      run_matfree<T>(op, t, trans, b, w.part, s);
      HIPCHK(hipStreamSynchronize(s));  // keeps the tables alive until done
    }
  } else {
    JobTable t;
    const size_t o = t.add(interface_jobs(op, in, out, trans));
    t.upload(s);
    if (trans)
      launch_gemv<T>(t.at<GemvJob>(o), op->n_ds, op->ld, op->M, 1, -1.0, w.part, s);
    else
      launch_gemv_many<T>(t.at<GemvJob>(o), op->n_ds, op->ld, op->M, -1.0, nr, w.ifc, w.part,
                          s);
    HIPCHK(hipStreamSynchronize(s));
  }
}

// GMRES for S x = rhs from x = 0: unrestarted (restart 0, or >= max_iter),
// else cycles of at most `restart` iterations, each started from the
// explicit residual rhs - S x, until the residual relative to ||rhs|| is
// <= tol or max_iter iterations in all.  Returns the iterations used.
template <typename T>
int gmres(ddst_op *op, SolveWs &w, const void *G, const double *rhs, double *x, double tol,
          int max_iter, bool trans, int form, double *relres, hipStream_t s, int restart = 0) {
  if (restart <= 0 || restart >= max_iter)
    return gmres_cycle<T>(op, w, G, rhs, x, tol, max_iter, trans, form, relres, s);
  const size_t len = w.ifc * w.nr;
  launch_norm(rhs, len, w.nrm, w.dpart, s);
  HIPCHK(hipMemcpyAsync(op->hbuf_host, w.nrm, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double beta0 = op->hbuf_host[0];
  launch_fill(x, 0.0, len, s);
  *relres = 0.0;
  if (!(beta0 > 0.0)) return 0;
  HIPCHK(hipMemcpyAsync(w.rr, rhs, len * 8, hipMemcpyDeviceToDevice, s));
  double rnorm = beta0, res = 1.0;
  int total = 0;
  while (total < max_iter) {
    const int m = std::min(restart, max_iter - total);
    double rc = 0.0;
    const int it = gmres_cycle<T>(op, w, G, w.rr, w.dx, tol * beta0 / rnorm, m, trans, form,
                                  &rc, s);
    launch_axpy(x, w.dx, 1.0, len, s);
    total += it;
    res = rc * rnorm / beta0;
    if (res <= tol || it < m) break;  // converged, or the Krylov space ran out
    // explicit residual for the next cycle
    stacked_apply<T>(op, w, G, form, trans, x, w.W, s);
    HIPCHK(hipMemcpyAsync(w.rr, rhs, len * 8, hipMemcpyDeviceToDevice, s));
    launch_axpy(w.rr, w.W, -1.0, len, s);
    launch_norm(w.rr, len, w.nrm, w.dpart, s);
    HIPCHK(hipMemcpyAsync(op->hbuf_host, w.nrm, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    rnorm = op->hbuf_host[0];
    res = rnorm / beta0;
    if (res <= tol) break;
  }
  HIPCHK(hipStreamSynchronize(s));
  *relres = res;
  return total;
}

// Pinned host staging for GMRES scalars: 2 (max_iter + 1) + 1 doubles per
// Arnoldi step and max_iter coefficients at the end.
void ensure_host(ddst_op *op, int max_iter) {
  const size_t need = std::max<size_t>((size_t)(2 * max_iter + 16) * 8, 1 << 16);
  if (op->hbuf_host && op->hbuf_bytes >= need) return;
  if (op->hbuf_host) (void)hipHostFree(op->hbuf_host);
  op->hbuf_host = nullptr;
  op->hbuf_bytes = 0;
  void *p = nullptr;
  HIPCHK(hipHostMalloc(&p, need, hipHostMallocDefault));
  op->hbuf_host = static_cast<double *>(p);
  op->hbuf_bytes = need;
}

// One DD solve of A d = r (transpose: A^T d = r) with zero boundary data,
// writing the correction volume into w.D (for each of the w.nr right-hand
// sides; the transposed solve takes one); returns GMRES iterations.
template <typename T>
int dd_correction(ddst_op *op, SolveWs &w, const void *G, bool trans, const double *tol_inner,
                  int max_iter, int form, double *relres, SlabTables &loads,
                  SlabTables &recon, hipStream_t s, int restart) {
  const int nr = w.nr;
  // z = A_II^{-1} r_I
  run_slab_solve<T>(op, loads, trans, w.part, s, nr, w.vol);
  // f_J = r_J - A_JI z
  for (int v = 0; v < nr; ++v) {
    const size_t ov = (size_t)v * w.vol, oi = (size_t)v * w.ifc;
    if (!trans)
      launch_interface_rhs(w.R + ov, w.Z + ov, w.Z + ov, op->Em, op->Ep, op->n_ds, op->m, op->ld,
                           0, 0, w.fJ + oi, s);
    else
      launch_interface_rhs(w.R + ov, w.Z + ov, w.Z + ov, op->Ep, op->Em, op->n_ds, op->m, op->ld,
                           -1, +1, w.fJ + oi, s);
  }
  int it;
  if (!trans) {
    // hhat = Sigma^{-1} f_J ; S d_J = hhat
    JobTable tb;
    const size_t o = tb.add(sinv_jobs(op, w.fJ, w.hh));
    tb.upload(s);
    launch_gemv_many<T>(tb.at<GemvJob>(o), op->n_ds, op->ld, op->M, 1.0, nr, w.ifc, w.part, s);
    it = gmres<T>(op, w, G, w.hh, w.xg, *tol_inner, max_iter, false, form, relres, s, restart);
  } else {
    // S^T mu = f_J ; d_J = Sigma^{-T} mu
    it = gmres<T>(op, w, G, w.fJ, w.hh, *tol_inner, max_iter, true, form, relres, s, restart);
    JobTable tb;
    const size_t o = tb.add(sinv_jobs(op, w.hh, w.xg));
    tb.upload(s);
    launch_gemv<T>(tb.at<GemvJob>(o), op->n_ds, op->ld, op->M, 1, 1.0, w.part, s);
    HIPCHK(hipStreamSynchronize(s));
  }
  // traces into the correction volume, then the slab interiors
  for (int v = 0; v < nr; ++v)
    launch_copy_planes(w.xg + (size_t)v * w.ifc, 1, 0, w.D + (size_t)v * w.vol, op->m, op->m - 1,
                       op->n_ds, op->ld, op->M, s);
  run_slab_solve<T>(op, recon, trans, w.part, s, nr, w.vol);
  return it;
}

// How GMRES applies S: the dense blocks, the compressed form or the
// matrix-free sweeps.
inline int apply_form(const ddst_solve_opts_t &o) {
  return o.use_hodlr ? DDST_APPLY_HODLR
         : o.use_hbs ? DDST_APPLY_HBS
         : o.matrix_free ? DDST_APPLY_MATFREE
                         : DDST_APPLY_DENSE;
}

struct RefineOut {
  int outer = 0, gm_total = 0, gm_last = 0, converged = 0;
  double relres = 0, corr = 0, resrel = 0;  // the largest over right-hand sides
};

// Norms of `count` vectors of length len, stride apart, into host out[]
// (one read-back).
void dev_norms(ddst_op *op, SolveWs &w, const double *v, size_t stride, size_t len, int count,
               double *out, hipStream_t s) {
  for (int i = 0; i < count; ++i) launch_norm(v + (size_t)i * stride, len, w.nrm + i, w.dpart, s);
  HIPCHK(hipMemcpyAsync(op->hbuf_host, w.nrm, (size_t)count * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::memcpy(out, op->hbuf_host, (size_t)count * 8);
}

// FP64 refinement loop shared by the solve (A) and the adjoint (A^T), for
// the w.nr right-hand sides f + v N, g + v (n+2)^dim; passes run until every
// one meets the stopping rule.
template <typename T>
int refine(ddst_op *op, const void *G, const double *f, const double *g, bool trans,
           const ddst_solve_opts_t &o, SolveWs &w, RefineOut &ro, hipStream_t s) {
  const int nr = w.nr;
  const size_t box = (size_t)std::pow((double)(op->n + 2), op->dim) + 0.5;
  SlabTables loads, recon;
  make_slab_tables(op, G, w.R, w.Z, false, trans, loads);
  make_slab_tables(op, G, w.R, w.D, true, trans, recon);
  loads.tab.upload(s);
  recon.tab.upload(s);
  launch_fill(w.X, 0.0, w.vol * nr, s);
  launch_fill(w.Z, 0.0, w.vol * nr, s);
  launch_fill(w.R, 0.0, w.vol * nr, s);  // padding of R must stay zero
  auto residuals = [&]() {
    for (int v = 0; v < nr; ++v)
      launch_residual(op->coef, op->dim, op->n, op->M, op->ld, f ? f + (size_t)v * op->N : nullptr,
                      (trans || !g) ? nullptr : g + (size_t)v * box, w.X + (size_t)v * w.vol,
                      w.R + (size_t)v * w.vol, trans ? 1 : 0, s);
  };
  std::vector<double> prev(nr, 0.0), r0(nr, 0.0), dn(nr), xn(nr), rf(nr);
  int status = DDST_OK;
  for (int outer = 0; outer < o.max_outer; ++outer) {
    residuals();
    if (outer == 0) dev_norms(op, w, w.R, w.vol, w.vol, nr, r0.data(), s);
    launch_fill(w.D, 0.0, w.vol * nr, s);
    double rr = 0;
    const int it = dd_correction<T>(op, w, G, trans, &o.inner_tol, o.max_iter, apply_form(o),
                                    &rr, loads, recon, s, o.restart);
    ro.gm_total += it;
    ro.gm_last = it;
    ro.relres = rr;
    if (rr > o.inner_tol) status = DDST_ENOTCONV;
    launch_axpy(w.X, w.D, 1.0, w.vol * nr, s);
    dev_norms(op, w, w.D, w.vol, w.vol, nr, dn.data(), s);
    dev_norms(op, w, w.X, w.vol, w.vol, nr, xn.data(), s);
    ro.outer = outer + 1;
    ro.corr = 0.0;
    bool all_done = true;
    for (int v = 0; v < nr; ++v) {
      const double corr = (xn[v] > 0) ? dn[v] / xn[v] : 0.0;
      ro.corr = std::max(ro.corr, corr);
      bool done = corr <= o.tol;
      if (outer >= 1 && prev[v] > 0 && dn[v] < prev[v] && (dn[v] / prev[v]) * corr <= o.tol)
        done = true;
      if (xn[v] == 0.0) done = true;
      prev[v] = dn[v];
      all_done = all_done && done;
    }
    if (all_done) {
      ro.converged = 1;
      break;
    }
  }
  residuals();
  dev_norms(op, w, w.R, w.vol, w.vol, nr, rf.data(), s);
  ro.resrel = 0.0;
  for (int v = 0; v < nr; ++v) ro.resrel = std::max(ro.resrel, r0[v] > 0 ? rf[v] / r0[v] : 0.0);
  if (!ro.converged) status = DDST_ENOTCONV;
  return status;
}

ddst_solve_opts_t solve_defaults(const ddst_op *op) {
  ddst_solve_opts_t o{};
  o.tol = 1e-10;
  // FP32 operators: the inner solve need not beat the contraction one
  // refinement pass gets from the FP32 build (about 1e-4 per pass)
  o.inner_tol = (op->prec == DDST_FP32) ? 1e-4 : 1e-12;
  o.max_iter = 300;
  o.max_outer = 4;
  o.use_hodlr = 0;
  o.matrix_free = 0;
  o.restart = 0;
  o.use_hbs = 0;
  o.basis_fp32 = 0;
  o.reserved_ = 0;
  return o;
}

int check_solve_opts(const ddst_solve_opts_t &o) {
  if (!(o.tol > 0) || !(o.inner_tol > 0)) return fail(DDST_EINVAL, "tolerances must be > 0");
  if (o.max_iter < 1 || o.max_iter > kMaxGmresIter)
    return fail(DDST_EINVAL, "max_iter in [1, " + std::to_string(kMaxGmresIter) + "]");
  if (o.max_outer < 1 || o.max_outer > 100) return fail(DDST_EINVAL, "max_outer in [1, 100]");
  if ((o.use_hodlr != 0 && o.use_hodlr != 1) || (o.matrix_free != 0 && o.matrix_free != 1) ||
      (o.use_hbs != 0 && o.use_hbs != 1))
    return fail(DDST_EINVAL, "use_hodlr, use_hbs and matrix_free must be 0 or 1");
  if (o.basis_fp32 != 0 && o.basis_fp32 != 1)
    return fail(DDST_EINVAL, "basis_fp32 must be 0 or 1");
  if (o.use_hodlr + o.matrix_free + o.use_hbs > 1)
    return fail(DDST_EINVAL, "use_hodlr, use_hbs and matrix_free are exclusive");
  if (o.restart < 0 || o.restart > o.max_iter)
    return fail(DDST_EINVAL, "restart in [0, max_iter]");
  return DDST_OK;
}

template <typename T>
int solve_impl(ddst_op *op, const double *f, const double *g, const ddst_solve_opts_t &o,
               double *u_gamma, double *u_vol, ddst_stats_t *st, hipStream_t s, int nr = 1) {
  if (!op->G) return fail(DDST_ESTATE, "slab factors were dropped; rebuild with keep_factors");
  if (o.use_hodlr && !hodlr_ready(op)) return fail(DDST_ESTATE, "no compressed form: call ddst_compress");
  if (o.use_hbs && !hbs_ready(op)) return fail(DDST_ESTATE, "no HBS form: call ddst_compress_hbs");
  if (apply_form(o) == DDST_APPLY_DENSE && !op->S)
    return fail(DDST_ESTATE, "no transfer blocks (matrix-free build): set matrix_free or use_hbs");
  ensure_host(op, o.max_iter);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  SolveWs w = carve_ws(op, o.max_iter, nr);
  w.basis32 = o.basis_fp32 != 0;
  RefineOut ro;
  const int status = refine<T>(op, op->G, f, g, false, o, w, ro, s);
  if (u_vol)
    for (int v = 0; v < nr; ++v)
      launch_unpad(w.X + (size_t)v * w.vol, u_vol + (size_t)v * op->N, op->n, op->M, op->ld, s);
  if (u_gamma && nr == 1) {
    launch_copy_planes(w.X, op->m, op->m - 1, w.xg, 1, 0, op->n_ds, op->ld, op->M, s);
    launch_unpad(w.xg, u_gamma, op->n_ds, op->M, op->ld, s);
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    *st = op->last_build;
    st->outer_iters = ro.outer;
    st->gmres_iters = ro.gm_total;
    st->last_gmres_iters = ro.gm_last;
    st->converged = ro.converged;
    st->gmres_relres = ro.relres;
    st->residual_rel = ro.resrel;
    st->correction_rel = ro.corr;
    st->t_solve_ms = ms;
  }
  return status;
}

template <typename T>
int adjoint_impl(ddst_op *op, const double *u_vol, const double *g, const double *gbar,
                 const ddst_solve_opts_t &o, double *dkappa, double *lambda, ddst_stats_t *st,
                 hipStream_t s) {
  if (o.use_hodlr && !hodlr_ready(op)) return fail(DDST_ESTATE, "no compressed form: call ddst_compress");
  if (o.use_hbs && !hbs_ready(op)) return fail(DDST_ESTATE, "no HBS form: call ddst_compress_hbs");
  if (apply_form(o) == DDST_APPLY_DENSE && !op->S)
    return fail(DDST_ESTATE, "no transfer blocks (matrix-free build): set matrix_free or use_hbs");
  ensure_host(op, o.max_iter);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  // factors: stored ones, or recomputed left-to-right sweeps of every slab
  DeviceMem tmp;
  const void *G = op->G;
  if (!G) {
    tmp.alloc((size_t)op->n_slabs * (op->m - 1) * op->mat_bytes);
    SweepBuffers b;
    b.store = tmp.p;
    run_sweeps<T>(op, factor_plan(op), b, s);
    const int fs = check_flag(op, s, "ddst_adjoint");
    if (fs) return fs;
    G = tmp.p;
  }
  SolveWs w = carve_ws(op, o.max_iter);
  w.basis32 = o.basis_fp32 != 0;
  RefineOut ro;
  const int status = refine<T>(op, G, gbar, nullptr, true, o, w, ro, s);
  launch_cell_gradient(u_vol, w.X, g, op->dim, op->n, op->M, op->ld, op->h, dkappa, s);
  if (lambda) launch_unpad(w.X, lambda, op->n, op->M, op->ld, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    *st = op->last_build;
    st->outer_iters = ro.outer;
    st->gmres_iters = ro.gm_total;
    st->last_gmres_iters = ro.gm_last;
    st->converged = ro.converged;
    st->gmres_relres = ro.relres;
    st->residual_rel = ro.resrel;
    st->correction_rel = ro.corr;
    st->t_adjoint_ms = ms;
  }
  return status;
}

// The form `which` is held by the operator (0), or the error to report.
int check_form(const ddst_op *op, int which) {
  if (which != DDST_APPLY_DENSE && which != DDST_APPLY_HODLR && which != DDST_APPLY_MATFREE &&
      which != DDST_APPLY_HBS)
    return fail(DDST_EINVAL, "which must be DENSE, HODLR, MATFREE or HBS");
  if (which == DDST_APPLY_HODLR && !hodlr_ready(op))
    return fail(DDST_ESTATE, "no compressed form: call ddst_compress");
  if (which == DDST_APPLY_HBS && !hbs_ready(op))
    return fail(DDST_ESTATE, "no HBS form: call ddst_compress_hbs");
  if (which == DDST_APPLY_MATFREE && !op->G)
    return fail(DDST_ESTATE, "slab factors were dropped; rebuild with keep_factors");
  if (which == DDST_APPLY_DENSE && !op->S)
    return fail(DDST_ESTATE, "no transfer blocks (matrix-free build)");
  return DDST_OK;
}

// yp = S xp (or S^T xp), padded interface vectors, through form `which`
// (temporaries allocated per call).
int apply_padded(ddst_op *op, int which, bool trans, const double *xp, double *yp,
                 hipStream_t stream) {
  const bool f32 = op->prec == DDST_FP32;
  if (which == DDST_APPLY_DENSE) {
    JobTable t;
    const size_t o = t.add(interface_jobs(op, xp, yp, trans));
    t.upload(stream);
    const int nchunk = std::min(op->ld / kGemvChunk, 64);
    DeviceMem part((size_t)op->n_ds * nchunk * op->ld * 8);
    double *pp = static_cast<double *>(part.p);
    if (f32)
      launch_gemv<float>(t.at<GemvJob>(o), op->n_ds, op->ld, op->M, trans, -1.0, pp, stream);
    else
      launch_gemv<double>(t.at<GemvJob>(o), op->n_ds, op->ld, op->M, trans, -1.0, pp, stream);
    HIPCHK(hipStreamSynchronize(stream));  // keeps the job table alive until done
    return DDST_OK;
  }
  if (which == DDST_APPLY_HODLR) return hodlr_apply_jobs(op, xp, yp, trans ? 1 : 0, stream);
  if (which == DDST_APPLY_HBS) return hbs_apply(op, xp, yp, trans ? 1 : 0, stream);
  const size_t ifc = (size_t)op->n_ds * op->ld, vol = (size_t)op->n * op->ld;
  const int nchunk = std::min(op->ld / kGemvChunk, 64);
  const size_t npart = (size_t)2 * op->n_slabs * nchunk * op->ld;
  DeviceMem tmp((2 * vol + 3 * ifc + npart) * 8);
  double *Zf = static_cast<double *>(tmp.p), *Zb = Zf + vol, *X = Zb + vol, *V = X + ifc;
  double *F = V + ifc, *part = F + ifc;
  HIPCHK(hipMemcpyAsync(X, xp, ifc * 8, hipMemcpyDeviceToDevice, stream));
  const MatfreeBufs b{X, V, F, Zf, Zb, yp};
  MatfreeTables t;
  make_matfree_tables(op, op->G, trans, b, t);
  t.tab.upload(stream);
  launch_fill(Zf, 0.0, 2 * vol, stream);
  if (f32)
    run_matfree<float>(op, t, trans, b, part, stream);
  else
    run_matfree<double>(op, t, trans, b, part, stream);
  HIPCHK(hipStreamSynchronize(stream));
  return DDST_OK;
}

template <typename Fn>
int guarded(Fn &&fn) {
  try {
    return fn();
  } catch (const std::bad_alloc &) {
    return fail(DDST_ENOMEM, "device or host allocation failed");
  } catch (const HipError &e) {
    return fail(DDST_EHIP, e.what());
  } catch (const std::exception &e) {
    return fail(DDST_EHIP, e.what());
  } catch (...) {
    return fail(DDST_EHIP, "unknown error");
  }
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

int ddst_build_transfer(const ddst_problem_t *prob, const ddst_build_opts_t *opts,
                        hipStream_t stream, ddst_op_t **out) {
  g_err.clear();
  return guarded([&]() -> int { return build_entry(prob, opts, stream, out); });
}

int ddst_solve(const ddst_op_t *cop, const double *f, const double *g,
               const ddst_solve_opts_t *opts, double *u_gamma, double *u_vol,
               ddst_stats_t *stats, hipStream_t stream) {
  g_err.clear();
  if (!cop) return fail(DDST_EINVAL, "op is NULL");
  ddst_op *op = const_cast<ddst_op *>(cop);
  ddst_solve_opts_t o = opts ? *opts : solve_defaults(op);
  int st = check_solve_opts(o);
  if (st) return st;
  return guarded([&]() -> int {
    return op->prec == DDST_FP32 ? solve_impl<float>(op, f, g, o, u_gamma, u_vol, stats, stream)
                                 : solve_impl<double>(op, f, g, o, u_gamma, u_vol, stats, stream);
  });
}

int ddst_solve_many(const ddst_op_t *cop, int32_t nrhs, const double *f, const double *g,
                    const ddst_solve_opts_t *opts, double *u_vol, ddst_stats_t *stats,
                    hipStream_t stream) {
  g_err.clear();
  if (!cop) return fail(DDST_EINVAL, "op is NULL");
  if (nrhs < 1 || nrhs > DDST_MAX_RHS)
    return fail(DDST_EINVAL, "nrhs in [1, " + std::to_string(DDST_MAX_RHS) + "]");
  ddst_op *op = const_cast<ddst_op *>(cop);
  ddst_solve_opts_t o = opts ? *opts : solve_defaults(op);
  int st = check_solve_opts(o);
  if (st) return st;
  return guarded([&]() -> int {
    return op->prec == DDST_FP32
               ? solve_impl<float>(op, f, g, o, nullptr, u_vol, stats, stream, nrhs)
               : solve_impl<double>(op, f, g, o, nullptr, u_vol, stats, stream, nrhs);
  });
}

int ddst_adjoint(const ddst_op_t *cop, const double *u_vol, const double *g, const double *gbar,
                 const ddst_solve_opts_t *opts, double *dkappa, double *lambda,
                 ddst_stats_t *stats, hipStream_t stream) {
  g_err.clear();
  if (!cop || !u_vol || !gbar || !dkappa)
    return fail(DDST_EINVAL, "op, u_vol, gbar and dkappa must be non-NULL");
  ddst_op *op = const_cast<ddst_op *>(cop);
  ddst_solve_opts_t o = opts ? *opts : solve_defaults(op);
  int st = check_solve_opts(o);
  if (st) return st;
  return guarded([&]() -> int {
    return op->prec == DDST_FP32
               ? adjoint_impl<float>(op, u_vol, g, gbar, o, dkappa, lambda, stats, stream)
               : adjoint_impl<double>(op, u_vol, g, gbar, o, dkappa, lambda, stats, stream);
  });
}

int ddst_compress(ddst_op_t *op, const ddst_compress_opts_t *opts, hipStream_t stream) {
  g_err.clear();
  if (!op || !opts) return fail(DDST_EINVAL, "op and opts must be non-NULL");
  if (!op->S) return fail(DDST_ESTATE, "no transfer blocks to compress (matrix-free build)");
  const ddst_compress_opts_t &o = *opts;
  if (o.tree != DDST_TREE_BINARY && o.tree != DDST_TREE_QUAD)
    return fail(DDST_EINVAL, "tree must be BINARY or QUAD");
  if (o.tree == DDST_TREE_QUAD && op->dim != 3)
    return fail(DDST_EINVAL, "the quadtree needs a 3D problem (planar interfaces)");
  if (o.leaf < 4) return fail(DDST_EINVAL, "leaf must be >= 4");
  if (o.oversample < 2 || o.max_rank < 1 || o.max_rank + o.oversample > 128)
    return fail(DDST_EINVAL, "need oversample >= 2, max_rank >= 1, max_rank + oversample <= 128");
  if (!(o.tol > 0) || !std::isfinite(o.tol)) return fail(DDST_EINVAL, "tol must be > 0");
  if (o.factor_dtype < DDST_FACTOR_BF16 || o.factor_dtype > DDST_FACTOR_FP64)
    return fail(DDST_EINVAL, "bad factor_dtype");
  return guarded([&]() -> int {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, stream));
    int overflow = 0;
    const int st = hodlr_compress(op, o, stream, &overflow);
    HIPCHK(hipEventRecord(e1, stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == DDST_ERANK)
      return fail(DDST_ERANK, "an admissible block needs rank " + std::to_string(overflow) +
                                  ", beyond max_rank (" + std::to_string(o.max_rank) +
                                  ") with oversampling " + std::to_string(o.oversample));
    if (st) return fail(st, "compression failed");
    op->last_build.t_compress_ms = ms;
    hodlr_info(op, &op->last_build.bytes_hodlr, &op->last_build.max_rank,
               &op->last_build.min_rank);
    return DDST_OK;
  });
}

int ddst_compress_hbs(ddst_op_t *op, const ddst_hbs_opts_t *opts, const double *omega,
                      const double *psi, hipStream_t stream) {
  g_err.clear();
  if (!op || !opts) return fail(DDST_EINVAL, "op and opts must be non-NULL");
  if (!op->G) return fail(DDST_ESTATE, "slab factors were dropped; rebuild with keep_factors");
  const ddst_hbs_opts_t &o = *opts;
  if (o.factor_dtype < DDST_FACTOR_BF16 || o.factor_dtype > DDST_FACTOR_FP64)
    return fail(DDST_EINVAL, "bad factor_dtype");
  if (o.leaf < 0) return fail(DDST_EINVAL, "leaf must be >= 0 (0: 2 rank)");
  return guarded([&]() -> int {
    std::string msg;
    const int st = hbs_compress(op, o.rank, o.oversample, o.leaf, o.factor_dtype, omega, psi,
                                o.seed, stream, &msg);
    if (st) return fail(st, "ddst_compress_hbs: " + msg);
    return DDST_OK;
  });
}

int ddst_hbs_info(const ddst_op_t *op, double *bytes, int32_t *rank, double *t_sample_ms,
                  double *t_compress_ms) {
  g_err.clear();
  if (!op) return fail(DDST_EINVAL, "op is NULL");
  if (!hbs_ready(op)) return fail(DDST_ESTATE, "no HBS form: call ddst_compress_hbs");
  int k = 0;
  hbs_info(op, bytes, &k, t_sample_ms, t_compress_ms);
  if (rank) *rank = k;
  return DDST_OK;
}

int ddst_sample_blocks(const ddst_op_t *cop, int32_t ncols, const double *X, double *Y,
                       double *Z, hipStream_t stream) {
  g_err.clear();
  if (!cop || !X || !Y || !Z || ncols < 1 || ncols > 512)
    return fail(DDST_EINVAL, "op, X, Y, Z must be non-NULL and 1 <= ncols <= 512");
  ddst_op *op = const_cast<ddst_op *>(cop);
  if (!op->G) return fail(DDST_ESTATE, "slab factors were dropped");
  return guarded([&]() -> int { return hbs_sample_blocks(op, ncols, X, Y, Z, stream); });
}

int ddst_compress_info(const ddst_op_t *op, double *bytes, int32_t *max_rank,
                       int32_t *min_rank, double *ms) {
  g_err.clear();
  if (!op) return fail(DDST_EINVAL, "op is NULL");
  if (!hodlr_ready(op)) return fail(DDST_ESTATE, "no compressed form: call ddst_compress");
  int mx = 0, mn = 0;
  hodlr_info(op, bytes, &mx, &mn);
  if (max_rank) *max_rank = mx;
  if (min_rank) *min_rank = mn;
  if (ms) *ms = op->last_build.t_compress_ms;
  return DDST_OK;
}

int ddst_release_factors(ddst_op_t *op) {
  g_err.clear();
  if (!op) return fail(DDST_EINVAL, "op is NULL");
  if (op->G) {
    (void)hipDeviceSynchronize();
    dev_free(op->G);
    op->G = nullptr;
  }
  return DDST_OK;
}

void ddst_destroy(ddst_op_t *op) { destroy_op(op); }

const char *ddst_last_error(void) { return g_err.c_str(); }

int ddst_build_stats(const ddst_op_t *op, ddst_stats_t *stats) {
  g_err.clear();
  if (!op || !stats) return fail(DDST_EINVAL, "op and stats must be non-NULL");
  *stats = op->last_build;
  return DDST_OK;
}

int ddst_op_info(const ddst_op_t *op, int32_t *M, int32_t *n_ds, int32_t *ld,
                 int32_t *precision) {
  if (!op) return fail(DDST_EINVAL, "op is NULL");
  if (M) *M = op->M;
  if (n_ds) *n_ds = op->n_ds;
  if (ld) *ld = op->ld;
  if (precision) *precision = op->prec;
  return DDST_OK;
}

int ddst_get_transfer(const ddst_op_t *op, int32_t j, double *S_left, double *S_right,
                      hipStream_t stream) {
  g_err.clear();
  if (!op) return fail(DDST_EINVAL, "op is NULL");
  if (j < 1 || j > op->n_ds) return fail(DDST_EINVAL, "interface index out of range");
  if (!op->S) return fail(DDST_ESTATE, "no transfer blocks (matrix-free build)");
  return guarded([&]() -> int {
    if (S_left)
      launch_extract_block(mat(op->S, 2 * (j - 1) + 0, op->mat_bytes), op->prec, op->M, op->ld,
                           S_left, stream);
    if (S_right)
      launch_extract_block(mat(op->S, 2 * (j - 1) + 1, op->mat_bytes), op->prec, op->M, op->ld,
                           S_right, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return DDST_OK;
  });
}

int ddst_set_allocator(ddst_alloc_fn alloc, ddst_free_fn free_fn, void *ctx) {
  g_err.clear();
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(DDST_EINVAL, "alloc and free must both be set or both be NULL");
  if (g_live.load() != 0)
    return fail(DDST_ESTATE, "library memory is allocated: destroy every operator first");
  g_alloc = alloc;
  g_free = free_fn;
  g_ctx = ctx;
  return DDST_OK;
}

int ddst_apply(const ddst_op_t *cop, int32_t transpose, int32_t which, const double *x,
               double *y, hipStream_t stream) {
  g_err.clear();
  if (!cop || !x || !y) return fail(DDST_EINVAL, "op, x and y must be non-NULL");
  ddst_op *op = const_cast<ddst_op *>(cop);
  const int st = check_form(op, which);
  if (st) return st;
  return guarded([&]() -> int {
    DeviceMem buf((size_t)op->n_ds * op->ld * 8 * 2);
    double *xp = static_cast<double *>(buf.p), *yp = xp + (size_t)op->n_ds * op->ld;
    launch_pad(x, xp, op->n_ds, op->M, op->ld, stream);
    const int r = apply_padded(op, which, transpose != 0, xp, yp, stream);
    if (r) return r;
    launch_unpad(yp, y, op->n_ds, op->M, op->ld, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return DDST_OK;
  });
}

int ddst_apply_noalloc(const ddst_op_t *cop, int32_t transpose, int32_t which, const double *x,
                       double *y, hipStream_t stream) {
  g_err.clear();
  if (!cop || !x || !y) return fail(DDST_EINVAL, "op, x and y must be non-NULL");
  if (which != DDST_APPLY_DENSE && which != DDST_APPLY_HODLR && which != DDST_APPLY_HBS)
    return fail(DDST_EINVAL, "which must be DENSE, HODLR or HBS (the matrix-free product "
                             "needs volume-sized temporaries)");
  const int st = check_form(cop, which);
  if (st) return st;
  const size_t need = noalloc_need(cop, which, transpose != 0);
  if (need > noalloc_scratch_bytes())
    return fail(DDST_EINVAL, "this product needs " + std::to_string(need) +
                                 " bytes of scratch; the static buffer holds " +
                                 std::to_string(noalloc_scratch_bytes()) + " (use ddst_apply)");
  const hipError_t e = noalloc_apply(cop, which, transpose != 0, x, y, stream);
  if (e != hipSuccess) return fail(DDST_EHIP, std::string("ddst_apply_noalloc: ") +
                                                  hipGetErrorString(e));
  return DDST_OK;
}

int ddst_gmres(const ddst_op_t *cop, int32_t transpose, int32_t which, const double *b, double *x,
               double tol, int32_t max_iter, int32_t *iters, double *relres,
               hipStream_t stream) {
  g_err.clear();
  if (!cop || !b || !x) return fail(DDST_EINVAL, "op, b and x must be non-NULL");
  if (!(tol > 0)) return fail(DDST_EINVAL, "tol must be > 0");
  if (max_iter < 1 || max_iter > kMaxGmresIter)
    return fail(DDST_EINVAL, "max_iter in [1, " + std::to_string(kMaxGmresIter) + "]");
  ddst_op *op = const_cast<ddst_op *>(cop);
  const int st = check_form(op, which);
  if (st) return st;
  return guarded([&]() -> int {
    ensure_host(op, max_iter);
    SolveWs w = carve_ws(op, max_iter);
    launch_pad(b, w.fJ, op->n_ds, op->M, op->ld, stream);
    double rr = 0.0;
    const int it = op->prec == DDST_FP32
                       ? gmres<float>(op, w, op->G, w.fJ, w.xg, tol, max_iter, transpose != 0,
                                      which, &rr, stream)
                       : gmres<double>(op, w, op->G, w.fJ, w.xg, tol, max_iter, transpose != 0,
                                       which, &rr, stream);
    launch_unpad(w.xg, x, op->n_ds, op->M, op->ld, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    if (iters) *iters = it;
    if (relres) *relres = rr;
    return rr <= tol ? DDST_OK : DDST_ENOTCONV;
  });
}

int ddst_cond_est(const ddst_op_t *cop, int32_t which, int32_t max_iter, double tol,
                  double gmres_tol, double *smax, double *smin, int32_t *iters,
                  hipStream_t stream) {
  g_err.clear();
  if (!cop || !smax || !smin) return fail(DDST_EINVAL, "op, smax and smin must be non-NULL");
  if (max_iter < 1 || !(tol > 0) || !(gmres_tol > 0))
    return fail(DDST_EINVAL, "need max_iter >= 1, tol > 0, gmres_tol > 0");
  ddst_op *op = const_cast<ddst_op *>(cop);
  const int st = check_form(op, which);
  if (st) return st;
  return guarded([&]() -> int {
    const int kInner = 2000;  // GMRES cap of each inverse-iteration solve
    ensure_host(op, kInner);
    SolveWs w = carve_ws(op, kInner);
    const size_t len = w.ifc;
    // fixed start vector: uniform in (-1, 1) from a 64-bit xorshift, zero
    // in the padding
    std::vector<double> h0(len, 0.0);
    uint64_t r = 0x9E3779B97F4A7C15ull;
    for (int j = 0; j < op->n_ds; ++j)
      for (int i = 0; i < op->M; ++i) {
        r ^= r << 13;
        r ^= r >> 7;
        r ^= r << 17;
        h0[(size_t)j * op->ld + i] = (double)(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
      }
    double *v = w.hh, *y = w.D, *z = w.Z;  // buffers GMRES does not touch
    // largest eigenvalue of S^T S by power iteration (forward), of
    // (S^T S)^{-1} = S^{-1} S^{-T} by inverse iteration (GMRES solves)
    for (int inv = 0; inv < 2; ++inv) {
      HIPCHK(hipMemcpyAsync(v, h0.data(), len * 8, hipMemcpyHostToDevice, stream));
      launch_norm(v, len, w.nrm, w.dpart, stream);
      launch_scale_by_inv(v, v, w.nrm, len, stream);
      double lam = 0.0, prev = 0.0;
      for (int k = 0; k < max_iter; ++k) {
        if (!inv) {
          int e = apply_padded(op, which, false, v, y, stream);
          if (!e) e = apply_padded(op, which, true, y, z, stream);
          if (e) return e;
        } else {
          double rr = 0.0;
          HIPCHK(hipMemcpyAsync(w.fJ, v, len * 8, hipMemcpyDeviceToDevice, stream));
          const bool f32 = op->prec == DDST_FP32;
          if (f32)
            gmres<float>(op, w, op->G, w.fJ, w.xg, gmres_tol, kInner, true, which, &rr, stream);
          else
            gmres<double>(op, w, op->G, w.fJ, w.xg, gmres_tol, kInner, true, which, &rr, stream);
          HIPCHK(hipMemcpyAsync(w.fJ, w.xg, len * 8, hipMemcpyDeviceToDevice, stream));
          if (f32)
            gmres<float>(op, w, op->G, w.fJ, w.xg, gmres_tol, kInner, false, which, &rr, stream);
          else
            gmres<double>(op, w, op->G, w.fJ, w.xg, gmres_tol, kInner, false, which, &rr, stream);
          HIPCHK(hipMemcpyAsync(z, w.xg, len * 8, hipMemcpyDeviceToDevice, stream));
        }
        // v has unit norm, so ||z|| -> the dominant eigenvalue
        launch_norm(z, len, w.nrm, w.dpart, stream);
        HIPCHK(hipMemcpyAsync(op->hbuf_host, w.nrm, 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        lam = op->hbuf_host[0];
        if (!(lam > 0.0) || !std::isfinite(lam)) return fail(DDST_EHIP, "power iteration failed");
        launch_scale_by_inv(v, z, w.nrm, len, stream);
        if (iters) *iters = k + 1;
        if (k > 0 && std::fabs(lam - prev) <= tol * lam) break;
        prev = lam;
      }
      if (!inv)
        *smax = std::sqrt(lam);
      else
        *smin = 1.0 / std::sqrt(lam);
    }
    HIPCHK(hipStreamSynchronize(stream));
    return DDST_OK;
  });
}

int ddst_loads(const ddst_op_t *cop, const double *f, const double *g, double *hhat,
               hipStream_t stream) {
  g_err.clear();
  if (!cop || !hhat) return fail(DDST_EINVAL, "op and hhat must be non-NULL");
  ddst_op *op = const_cast<ddst_op *>(cop);
  if (!op->G) return fail(DDST_ESTATE, "slab factors were dropped");
  return guarded([&]() -> int {
    SolveWs w = carve_ws(op, 1);
    launch_fill(w.X, 0.0, w.vol, stream);
    launch_fill(w.Z, 0.0, w.vol, stream);
    launch_fill(w.R, 0.0, w.vol, stream);
    launch_residual(op->coef, op->dim, op->n, op->M, op->ld, f, g, w.X, w.R, 0, stream);
    SlabTables loads;
    make_slab_tables(op, op->G, w.R, w.Z, false, false, loads);
    loads.tab.upload(stream);
    JobTable tb;
    const size_t o = tb.add(sinv_jobs(op, w.fJ, w.hh));
    tb.upload(stream);
    if (op->prec == DDST_FP32) {
      run_slab_solve<float>(op, loads, false, w.part, stream);
      launch_interface_rhs(w.R, w.Z, w.Z, op->Em, op->Ep, op->n_ds, op->m, op->ld, 0, 0, w.fJ,
                           stream);
      launch_gemv<float>(tb.at<GemvJob>(o), op->n_ds, op->ld, op->M, 0, 1.0, w.part, stream);
    } else {
      run_slab_solve<double>(op, loads, false, w.part, stream);
      launch_interface_rhs(w.R, w.Z, w.Z, op->Em, op->Ep, op->n_ds, op->m, op->ld, 0, 0, w.fJ,
                           stream);
      launch_gemv<double>(tb.at<GemvJob>(o), op->n_ds, op->ld, op->M, 0, 1.0, w.part, stream);
    }
    launch_unpad(w.hh, hhat, op->n_ds, op->M, op->ld, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return DDST_OK;
  });
}

}  // extern "C"

extern "C" {

int ddst_get_factor(const ddst_op_t *op, int32_t slab, int32_t k, double *out,
                    hipStream_t stream) {
  g_err.clear();
  if (!op || !out) return fail(DDST_EINVAL, "op and out must be non-NULL");
  if (!op->G) return fail(DDST_ESTATE, "slab factors were dropped");
  if (slab < 0 || slab >= op->n_slabs || k < 1 || k > op->m - 1)
    return fail(DDST_EINVAL, "slab or plane index out of range");
  return guarded([&]() -> int {
    launch_extract_block(mat(op->G, (size_t)slab * (op->m - 1) + (k - 1), op->mat_bytes),
                         op->prec, op->M, op->ld, out, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return DDST_OK;
  });
}

int ddst_get_center_inverse(const ddst_op_t *op, int32_t j, double *out, hipStream_t stream) {
  g_err.clear();
  if (!op || !out) return fail(DDST_EINVAL, "op and out must be non-NULL");
  if (j < 1 || j > op->n_ds) return fail(DDST_EINVAL, "interface index out of range");
  return guarded([&]() -> int {
    launch_extract_block(mat(op->Sinv, j - 1, op->mat_bytes), op->prec, op->M, op->ld, out,
                         stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return DDST_OK;
  });
}

int ddst_test_gemm(int32_t precision, int32_t ld, int32_t batch, const void *A, const void *B,
                   void *C, const double *bscale, double alpha, double beta,
                   hipStream_t stream) {
  g_err.clear();
  if (!A || !B || !C || batch < 1 || ld < kTile || ld % kTile != 0 ||
      (precision != DDST_FP32 && precision != DDST_FP64))
    return fail(DDST_EINVAL, "bad arguments");
  return guarded([&]() -> int {
    const size_t mb = (size_t)ld * ld * esize(precision);
    std::vector<GemmJob> jobs;
    for (int b = 0; b < batch; ++b) {
      GemmJob g{};
      g.A = mat(const_cast<void *>(A), b, mb);
      g.B = mat(const_cast<void *>(B), b, mb);
      g.C = mat(C, b, mb);
      g.bscale = bscale ? bscale + (size_t)b * ld : nullptr;
      jobs.push_back(g);
    }
    JobTable t;
    const size_t o = t.add(jobs);
    t.upload(stream);
    if (precision == DDST_FP32)
      launch_gemm<float>(t.at<GemmJob>(o), batch, ld, ld, alpha, beta, stream);
    else
      launch_gemm<double>(t.at<GemmJob>(o), batch, ld, ld, alpha, beta, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return DDST_OK;
  });
}

static int test_invert(int32_t precision, int32_t ld, int32_t batch, void *A, int sym,
                       hipStream_t stream) {
  g_err.clear();
  if (!A || batch < 1 || ld < kTile || ld % kTile != 0 ||
      (precision != DDST_FP32 && precision != DDST_FP64))
    return fail(DDST_EINVAL, "bad arguments");
  return guarded([&]() -> int {
    const size_t mb = (size_t)ld * ld * esize(precision);
    std::vector<void *> mats;
    for (int b = 0; b < batch; ++b) mats.push_back(mat(A, b, mb));
    JobTable t;
    const size_t o = t.add(mats);
    t.upload(stream);
    DeviceMem fl(sizeof(ElimStatus));
    HIPCHK(hipMemsetAsync(fl.p, 0, sizeof(ElimStatus), stream));
    DeviceMem w(gj_workspace_bytes(batch, ld, esize(precision)));
    GjStreams gs;
    HIPCHK(gs.create());
    int *flag = static_cast<int *>(fl.p);
    if (precision == DDST_FP32)
      HIPCHK(gj_invert<float>(t.at<void *>(o), batch, ld, ld, w.p, flag, 0, sym, gs, stream));
    else
      HIPCHK(gj_invert<double>(t.at<void *>(o), batch, ld, ld, w.p, flag, 0, sym, gs, stream));
    HIPCHK(hipGetLastError());
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, fl.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (h) return fail(DDST_EBREAKDOWN, "non-positive or non-finite pivot");
    return DDST_OK;
  });
}

int ddst_test_invert(int32_t precision, int32_t ld, int32_t batch, void *A, hipStream_t stream) {
  return test_invert(precision, ld, batch, A, 0, stream);
}

int ddst_test_invert_sym(int32_t precision, int32_t ld, int32_t batch, void *A,
                         hipStream_t stream) {
  return test_invert(precision, ld, batch, A, 1, stream);
}

}  // extern "C"
