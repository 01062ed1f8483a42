// ddst_apply_noalloc: the product with the equilibrium matrix S (dense
// transfer blocks or a compressed form) without any allocation, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid it).
//
// ddst_apply allocates its temporaries per call (the padded copies of x and
// y, the GEMV job table, the partial sums of the transposed product).  Here
// they live in one file-scope device array of fixed size, `scratch`, which
// every GPU that loads the library holds until the process ends.  Its
// device address is looked up once per device with hipGetSymbolAddress
// (the array's name in host code is a host-side stand-in, not a device
// address) and kept; kernels receive that address.  Every call on one GPU
// shares that GPU's array: calls that overlap on one GPU (different streams
// or threads without ordering between them) race.  Nothing in the array has
// to start at zero: the job table and the padded input are written in full
// before they are read, and the partial sums are written before they are
// reduced.
#include <mutex>
#include <string>

#include "internal.h"

namespace ddst {
namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
hipError_t scratch_ptr(void **out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// The GEMV jobs of y = S x (or S^T x) over padded interface vectors, written
// on the device (the job table of the allocating entry point, built there on
// the host): interface j gets the blocks of its neighbours j-1 and j+1,
//   forward:    S_{j,j-1} x_{j-1} + S_{j,j+1} x_{j+1}
//   transposed: S_{j-1,j}^T x_{j-1} + S_{j+1,j}^T x_{j+1},
// and y_j = x_j - (that sum).  Block storage: S_{j,j-1} at 2(j-1),
// S_{j,j+1} at 2(j-1)+1 (ld x ld matrices of mat_bytes each).
__global__ void k_interface_jobs(GemvJob *__restrict__ jobs, const unsigned char *S,
                                 size_t mat_bytes, int n_ds, int ld, const double *xp,
                                 double *yp, int trans) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x + 1;  // 1-based interface
  if (j > n_ds) return;
  GemvJob g{};
  if (!trans) {
    if (j >= 2) {
      g.G = S + (size_t)(2 * (j - 1) + 0) * mat_bytes;
      g.x1 = xp + (size_t)(j - 2) * ld;
    }
    if (j <= n_ds - 1) {
      g.G2 = S + (size_t)(2 * (j - 1) + 1) * mat_bytes;
      g.x3 = xp + (size_t)j * ld;
    }
  } else {
    if (j >= 2) {
      g.G = S + (size_t)(2 * (j - 2) + 1) * mat_bytes;
      g.x1 = xp + (size_t)(j - 2) * ld;
    }
    if (j <= n_ds - 1) {
      g.G2 = S + (size_t)(2 * j + 0) * mat_bytes;
      g.x3 = xp + (size_t)j * ld;
    }
  }
  g.w = xp + (size_t)(j - 1) * ld;
  g.out = yp + (size_t)(j - 1) * ld;
  jobs[j - 1] = g;
}

inline size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Bytes of scratch one call needs (0 for a form it does not support).
size_t noalloc_need(const ddst_op *op, int which, int trans) {
  const size_t ifc = (size_t)op->n_ds * op->ld * sizeof(double);
  if (which == DDST_APPLY_HODLR || which == DDST_APPLY_HBS) return 2 * up256(ifc);
  if (which != DDST_APPLY_DENSE) return 0;
  size_t need = up256((size_t)op->n_ds * sizeof(GemvJob)) + 2 * up256(ifc);
  if (trans) {
    const int nchunk = std::min(op->ld / kGemvChunk, 64);
    need += up256((size_t)op->n_ds * nchunk * op->ld * sizeof(double));
  }
  return need;
}

// y = S x (or S^T x), x and y unpadded N_ds*M device vectors; the caller has
// checked the operator state, the form and the scratch size.  No allocation,
// no synchronisation: the work is ordered on s.
hipError_t noalloc_apply(const ddst_op *op, int which, int trans, const double *x, double *y,
                         hipStream_t s) {
  void *base = nullptr;
  hipError_t e = scratch_ptr(&base);
  if (e != hipSuccess) return e;
  unsigned char *p = static_cast<unsigned char *>(base);
  const size_t ifc = (size_t)op->n_ds * op->ld * sizeof(double);
  GemvJob *jobs = nullptr;
  if (which == DDST_APPLY_DENSE) {
    jobs = reinterpret_cast<GemvJob *>(p);
    p += up256((size_t)op->n_ds * sizeof(GemvJob));
  }
  double *xp = reinterpret_cast<double *>(p);
  double *yp = reinterpret_cast<double *>(p + up256(ifc));
  double *part = reinterpret_cast<double *>(p + 2 * up256(ifc));
  launch_pad(x, xp, op->n_ds, op->M, op->ld, s);
  if (which == DDST_APPLY_DENSE) {
    hipLaunchKernelGGL(k_interface_jobs, dim3((op->n_ds + 63) / 64), dim3(64), 0, s, jobs,
                       static_cast<const unsigned char *>(op->S), op->mat_bytes, op->n_ds,
                       op->ld, xp, yp, trans);
    if (op->prec == DDST_FP32)
      launch_gemv<float>(jobs, op->n_ds, op->ld, op->M, trans, -1.0, part, s);
    else
      launch_gemv<double>(jobs, op->n_ds, op->ld, op->M, trans, -1.0, part, s);
  } else {
    const int st = which == DDST_APPLY_HBS ? hbs_apply(op, xp, yp, trans, s)
                                           : hodlr_apply_jobs(op, xp, yp, trans, s);
    if (st != DDST_OK) return hipErrorInvalidValue;
  }
  launch_unpad(yp, y, op->n_ds, op->M, op->ld, s);
  return hipGetLastError();
}

}  // namespace ddst
