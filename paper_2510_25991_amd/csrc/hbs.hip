// Hierarchically block separable (HBS) form of the transfer blocks, built
// from two-sided random samples without forming the blocks (Section 2.4,
// Algorithm 1 of the paper: s = alpha k + q samples, alpha = 3).
//
// Sampling.  For a single slab s between interfaces s and s + 1 the stored
// left-to-right factors G_k (inverse plane Schur complements, k = 1..m-1)
// and the inverse interface blocks Sigma_j^{-1} give, for an ld x sp block
// of sample columns (P(k) = s m + k the planes, c_j = j m the interfaces,
// Em / Ep the couplings towards the previous / next plane):
//   S_{s+1,s} Om = -Sigma_{s+1}^{-1} Em(c_{s+1}) a,  a = y_{m-1},
//       y_0 = Om,  y_k = -G_k Em(P(k)) y_{k-1};
//   S_{s,s+1} Om = -Sigma_s^{-1} Ep(c_s) b,  b = z_1,
//       z_m = Om,  z_k = -G_k Ep(P(k)) z_{k+1};
//   S_{s+1,s}^T Ps = -Em(P(1)) r_1,  r_{m-1} = -G_{m-1}^T Em(c_{s+1}) W_{s+1},
//       r_{k-1} = -G_{k-1}^T Em(P(k)) r_k,  W_j = Sigma_j^{-T} Ps;
//   S_{s,s+1}^T Ps = -Ep(P(m-1)) r_{m-1},  r_1 = -G_1^T Ep(c_s) W_s,
//       r_k = -G_k^T Ep(P(k-1)) r_{k-1}
// (the local solves of Algorithm 1 with the factorisation of the slabs,
// forward for Y = S Om and transposed for Z = S^T Ps), every chain step of
// every slab one batched matrix-core product.
//
// Compression (FP64), level by level from the leaves of a uniform-depth
// binary cluster tree shared by rows and columns; for every node tau and
// block, with its rows Om, Ps, Y, Z of the current sketches (n x s):
//   Yh = Y Om^+ (Gram matrix Om Om^T, Cholesky), W = Y - Yh Om,
//   U = the first k columns of the column-pivoted Householder QR of W,
//   likewise Zh, V from Z, Ps;
//   D = Yh + U U^T (Zh^T - Yh) - U (U^T Zh^T V) V^T;
//   the parent's rows: V^T Om, U^T Ps, U^T (Y - D Om), V^T (Z - D^T Ps);
// at the root D = Y Om^+.  This is the single-pass construction of the
// public literature (Levitt and Martinsson); a node needs s >= n + k.
//
// Apply: upward pass x^_tau = V^T x_tau (leaves) or V^T [x^_children],
// root [y^_children] = D_root x^, downward [y^_children] = U y^_tau +
// D [x^_children], leaves y_tau = U y^_tau + D x_tau; transposed with U and
// V exchanged and D^T.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"

namespace ddst {

struct HbsNodeDev {
  int n, r;        // rows of the node's sketch (its size at this level), rank
  int lo;          // leaves: first cluster-order index
  int roff;        // offset of the node's rank entries in its level's hat vector
  int coff;        // offset of its children's entries in the next level's hat vector
  int ldr, ldn;    // stored row lengths of U, V and of D (r, n rounded up to 8)
  int pad_;
  long long fU, fV, fD;  // element offsets (within one block) of U, V (n x r), D (n x n)
                         // in the FP64 compression output (unpadded rows)
  long long pU, pV, pD;  // the same in the stored factors (rows of ldr, ldn entries)
};

struct Hbs {
  int k = 0, s = 0, sp = 0, leaf = 0, depth = 0, dtype = 0, nblk = 0;
  std::vector<std::vector<HbsNodeDev>> lv;  // depth d = 0 .. depth (0: root)
  std::vector<int> nhat;                    // hat entries per level (sum of ranks)
  std::vector<size_t> hoff;                 // per-level offset in one block's hat vector
  size_t hat_per_block = 0;
  size_t block_elems = 0, root_off = 0;     // FP64 compression output per block; root D offset
  size_t stored_elems = 0;                  // stored factor elements per block (padded rows)
  std::vector<int> perm;
  int *d_perm = nullptr;
  void *factors = nullptr;
  size_t bytes = 0;
  void *nodes = nullptr;                    // device copies of the level node tables
  std::vector<size_t> node_off;             // byte offset of level d's table
  double *hat = nullptr;                    // apply workspace: x^ and y^ per block
  double t_sample_ms = 0, t_compress_ms = 0;
};

namespace {

struct HbsErr : std::runtime_error {
  using std::runtime_error::runtime_error;
};
#define BCHK(x)                                                                        \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw HbsErr(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct BMem {
  void *p = nullptr;
  explicit BMem(size_t b) {
    if (b && dev_malloc(&p, b) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
  }
  ~BMem() {
    if (p) dev_free(p);
  }
  BMem(const BMem &) = delete;
  BMem &operator=(const BMem &) = delete;
  template <typename X>
  X *as() const { return static_cast<X *>(p); }
};

inline unsigned nblk1(size_t n, unsigned b = 256) { return (unsigned)((n + b - 1) / b); }

constexpr int WG = 256;
constexpr int GT = 64;   // work-group GEMM output tile
constexpr int GK = 16;   // its k-chunk
constexpr int kMaxS = 512;  // largest sample count
constexpr int kMaxN = 256;  // largest node size

// ------------------------------------------------ work-group dense helpers
// C (m x n) = alpha op(A) op(B) + beta C, FP64, by the whole work-group,
// operands in global memory (row-major): op(A) is m x K, stored as A (m x K,
// lda) or, TA, as its transpose (K x m); op(B) is K x n, stored as B (K x n,
// ldb) or, TB, as its transpose (n x K).  C must not alias A or B.  beta = 0
// does not read C.  lds: 2 GK (GT + 1) doubles.
template <bool TA, bool TB>
__device__ void wg_gemm(int m, int n, int K, double alpha, const double *A, int lda,
                        const double *B, int ldb, double beta, double *C, int ldc,
                        double *lds) {
  double *As = lds, *Bs = lds + GK * (GT + 1);
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  for (int i0 = 0; i0 < m; i0 += GT)
    for (int j0 = 0; j0 < n; j0 += GT) {
      double acc[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
      for (int k0 = 0; k0 < K; k0 += GK) {
        __syncthreads();
        for (int e = tid; e < GT * GK; e += WG) {
          int i, k;
          if (TA) {
            k = e / GT;
            i = e % GT;
          } else {
            i = e / GK;
            k = e % GK;
          }
          const int gi = i0 + i, gk = k0 + k;
          double v = 0.0;
          if (gi < m && gk < K) v = TA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
          As[k * (GT + 1) + i] = v;
        }
        for (int e = tid; e < GT * GK; e += WG) {
          int j, k;
          if (TB) {
            j = e / GK;
            k = e % GK;
          } else {
            k = e / GT;
            j = e % GT;
          }
          const int gj = j0 + j, gk = k0 + k;
          double v = 0.0;
          if (gj < n && gk < K) v = TB ? B[(size_t)gj * ldb + gk] : B[(size_t)gk * ldb + gj];
          Bs[k * (GT + 1) + j] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < GK; ++k) {
          double a[4], b[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) a[q] = As[k * (GT + 1) + ti + 16 * q];
#pragma unroll
          for (int q = 0; q < 4; ++q) b[q] = Bs[k * (GT + 1) + tj + 16 * q];
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
        }
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + ti + 16 * p, j = j0 + tj + 16 * q;
          if (i < m && j < n) {
            double v = alpha * acc[p][q];
            if (beta != 0.0) v += beta * C[(size_t)i * ldc + j];
            C[(size_t)i * ldc + j] = v;
          }
        }
    }
  __syncthreads();
}

// Work-group sum of one double per thread (every thread gets the sum).
__device__ double wg_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < WG / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

// ------------------------------------------------------ compression kernels
struct HbsJob {
  const double *om, *ps, *y, *z;  // node sketch rows (n x s, leading dimension s)
  double *G[2];                   // n x n: Gram matrix, then its Cholesky factor
  double *H[2];                   // n x n: X = Y Om^T, then Yh (side 0) / Zh (side 1)
  double *W[2];                   // n x s: residual sketches, CPQR in place; then scratch
  double *B[2];                   // outputs U (side 0), V (side 1): n x r
  double *D;                      // output n x n
  double *T;                      // n x s scratch
  double *out[4];                 // parent rows: Om', Ps', Y', Z' (r x s), or null
  int n, r;
};

// side 0: G = Om Om^T, H = Y Om^T;  side 1: G = Ps Ps^T, H = Z Ps^T.
__global__ __launch_bounds__(WG) void k_hbs_gram(const HbsJob *__restrict__ jobs, int s) {
  __shared__ double lds[2 * GK * (GT + 1)];
  const HbsJob J = jobs[blockIdx.x];
  const int side = blockIdx.y;
  const double *om = side ? J.ps : J.om, *y = side ? J.z : J.y;
  wg_gemm<false, true>(J.n, J.n, s, 1.0, om, s, om, s, 0.0, J.G[side], J.n, lds);
  wg_gemm<false, true>(J.n, J.n, s, 1.0, y, s, om, s, 0.0, J.H[side], J.n, lds);
}

// Cholesky G = L L^T (in place, lower), then H <- H G^{-1} row by row.
__global__ __launch_bounds__(WG) void k_hbs_solve(const HbsJob *__restrict__ jobs,
                                                  int *__restrict__ flag) {
  const HbsJob J = jobs[blockIdx.x];
  const int side = blockIdx.y, n = J.n, tid = threadIdx.x;
  double *G = J.G[side], *H = J.H[side];
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    const double d = G[(size_t)j * n + j];
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) atomicOr(flag, 1);
      return;  // uniform: every thread read the same d
    }
    const double sd = sqrt(d);
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += WG) G[(size_t)i * n + j] /= sd;
    if (tid == 0) G[(size_t)j * n + j] = sd;
    __syncthreads();
    const int nt = n - j - 1;
    for (int e = tid; e < nt * nt; e += WG) {
      const int i = j + 1 + e / nt, l = j + 1 + e % nt;
      if (l <= i) G[(size_t)i * n + l] -= G[(size_t)i * n + j] * G[(size_t)l * n + j];
    }
  }
  __syncthreads();
  // rows of H: h <- h G^{-1}: solve L w = h^T, then L^T v = w
  for (int i = tid; i < n; i += WG) {
    double *h = H + (size_t)i * n;
    for (int a = 0; a < n; ++a) {
      double v = h[a];
      for (int b = 0; b < a; ++b) v -= G[(size_t)a * n + b] * h[b];
      h[a] = v / G[(size_t)a * n + a];
    }
    for (int a = n - 1; a >= 0; --a) {
      double v = h[a];
      for (int b = a + 1; b < n; ++b) v -= G[(size_t)b * n + a] * h[b];
      h[a] = v / G[(size_t)a * n + a];
    }
  }
}

// side 0: W = Y - Yh Om;  side 1: W = Z - Zh Ps.
__global__ __launch_bounds__(WG) void k_hbs_resid(const HbsJob *__restrict__ jobs, int s) {
  __shared__ double lds[2 * GK * (GT + 1)];
  const HbsJob J = jobs[blockIdx.x];
  const int side = blockIdx.y;
  const double *om = side ? J.ps : J.om, *y = side ? J.z : J.y;
  double *W = J.W[side];
  for (size_t e = threadIdx.x; e < (size_t)J.n * s; e += WG) W[e] = y[e];
  __syncthreads();
  wg_gemm<false, false>(J.n, s, J.n, -1.0, J.H[side], J.n, om, s, 1.0, W, s, lds);
}

// Householder QR with column pivoting of W (n x s), r steps; writes the
// orthonormal n x r factor of the first r reflectors to B[side].
__global__ __launch_bounds__(WG) void k_hbs_cpqr(const HbsJob *__restrict__ jobs, int s) {
  __shared__ double nrm[kMaxS], nrm0[kMaxS], beta[kMaxN], red[WG / 64];
  __shared__ double bestv[WG];
  __shared__ int besti[WG];
  const HbsJob J = jobs[blockIdx.x];
  const int side = blockIdx.y, n = J.n, r = J.r, tid = threadIdx.x;
  double *W = J.W[side], *Q = J.B[side];
  for (int c = tid; c < s; c += WG) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += W[(size_t)i * s + c] * W[(size_t)i * s + c];
    nrm[c] = t;
    nrm0[c] = t;
  }
  __syncthreads();
  for (int i = 0; i < r; ++i) {
    // pivot: the largest remaining column norm (the first on ties)
    double bv = -1.0;
    int bi = s;
    for (int c = i + tid; c < s; c += WG)
      if (nrm[c] > bv) {
        bv = nrm[c];
        bi = c;
      }
    bestv[tid] = bv;
    besti[tid] = bi;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
      if (tid < h) {
        const double ov = bestv[tid + h];
        const int oi = besti[tid + h];
        if (ov > bestv[tid] || (ov == bestv[tid] && oi < besti[tid])) {
          bestv[tid] = ov;
          besti[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int p = besti[0];
    __syncthreads();
    if (p != i) {
      for (int row = tid; row < n; row += WG) {
        const double t = W[(size_t)row * s + i];
        W[(size_t)row * s + i] = W[(size_t)row * s + p];
        W[(size_t)row * s + p] = t;
      }
      if (tid == 0) {
        double t = nrm[i];
        nrm[i] = nrm[p];
        nrm[p] = t;
        t = nrm0[i];
        nrm0[i] = nrm0[p];
        nrm0[p] = t;
      }
    }
    __syncthreads();
    // reflector of column i, rows i..n-1: v = w - alpha e_i, alpha = -sign(w_i) |w|
    double part = 0.0;
    for (int row = i + tid; row < n; row += WG) part += W[(size_t)row * s + i] * W[(size_t)row * s + i];
    const double nn = wg_sum(part, red);
    const double wi = W[(size_t)i * s + i];
    const double alpha = wi >= 0.0 ? -sqrt(nn) : sqrt(nn);
    const double vi = wi - alpha;
    const double vtv = nn - wi * wi + vi * vi;
    const double bt = vtv > 0.0 ? 2.0 / vtv : 0.0;
    __syncthreads();
    if (tid == 0) {
      W[(size_t)i * s + i] = vi;
      beta[i] = bt;
    }
    __syncthreads();
    // apply to the columns right of i; downdate their norms
    for (int c = i + 1 + tid; c < s; c += WG) {
      double dot = 0.0;
      for (int row = i; row < n; ++row) dot += W[(size_t)row * s + i] * W[(size_t)row * s + c];
      const double f = bt * dot;
      for (int row = i; row < n; ++row) W[(size_t)row * s + c] -= f * W[(size_t)row * s + i];
      const double top = W[(size_t)i * s + c];
      double nv = nrm[c] - top * top;
      if (!(nv > 1e-10 * nrm0[c])) {  // cancellation: recompute from the rows below
        nv = 0.0;
        for (int row = i + 1; row < n; ++row) nv += W[(size_t)row * s + c] * W[(size_t)row * s + c];
        nrm0[c] = nv;
      }
      nrm[c] = nv;
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{r-1} [I_r; 0]
  for (size_t e = tid; e < (size_t)n * r; e += WG) Q[e] = (e / r == e % r) ? 1.0 : 0.0;
  __syncthreads();
  for (int i = r - 1; i >= 0; --i) {
    const double bt = beta[i];
    for (int c = i + tid; c < r; c += WG) {
      double dot = 0.0;
      for (int row = i; row < n; ++row) dot += W[(size_t)row * s + i] * Q[(size_t)row * r + c];
      const double f = bt * dot;
      for (int row = i; row < n; ++row) Q[(size_t)row * r + c] -= f * W[(size_t)row * s + i];
    }
    __syncthreads();
  }
}

// D = Yh + U U^T (Zh^T - Yh) - U (U^T Zh^T V) V^T.
__global__ __launch_bounds__(WG) void k_hbs_diag(const HbsJob *__restrict__ jobs) {
  __shared__ double lds[2 * GK * (GT + 1)];
  const HbsJob J = jobs[blockIdx.x];
  const int n = J.n, r = J.r;
  const double *Yh = J.H[0], *Zh = J.H[1], *U = J.B[0], *V = J.B[1];
  double *T1 = J.T, *T2 = J.T + (size_t)n * n;
  for (size_t e = threadIdx.x; e < (size_t)n * n; e += WG) {
    const size_t a = e / n, b = e % n;
    T1[e] = Zh[b * n + a] - Yh[e];
    J.D[e] = Yh[e];
  }
  __syncthreads();
  wg_gemm<true, false>(r, n, n, 1.0, U, r, T1, n, 0.0, T2, n, lds);    // U^T T1
  wg_gemm<false, false>(n, n, r, 1.0, U, r, T2, n, 1.0, J.D, n, lds);  // D += U T2
  double *T3 = J.T, *T4 = J.T + (size_t)r * n, *T5 = T4 + (size_t)r * r;
  wg_gemm<true, true>(r, n, n, 1.0, U, r, Zh, n, 0.0, T3, n, lds);     // U^T Zh^T
  wg_gemm<false, false>(r, r, n, 1.0, T3, n, V, r, 0.0, T4, r, lds);   // (U^T Zh^T) V
  wg_gemm<false, true>(r, n, r, 1.0, T4, r, V, r, 0.0, T5, n, lds);    // ... V^T
  wg_gemm<false, false>(n, n, r, -1.0, U, r, T5, n, 1.0, J.D, n, lds); // D -= U T5
}

// Rows of the parent level: side 0: Om' = V^T Om, Y' = U^T (Y - D Om);
// side 1: Ps' = U^T Ps, Z' = V^T (Z - D^T Ps).
__global__ __launch_bounds__(WG) void k_hbs_reduce(const HbsJob *__restrict__ jobs, int s) {
  __shared__ double lds[2 * GK * (GT + 1)];
  const HbsJob J = jobs[blockIdx.x];
  const int side = blockIdx.y, n = J.n, r = J.r;
  const double *om = side ? J.ps : J.om, *y = side ? J.z : J.y;
  const double *Bo = side ? J.B[0] : J.B[1];  // basis that meets Om (V) or Ps (U)
  const double *By = side ? J.B[1] : J.B[0];  // basis of the output side
  double *W = J.W[side];
  wg_gemm<true, false>(r, s, n, 1.0, Bo, r, om, s, 0.0, J.out[side], s, lds);
  for (size_t e = threadIdx.x; e < (size_t)n * s; e += WG) W[e] = y[e];
  __syncthreads();
  if (side == 0)
    wg_gemm<false, false>(n, s, n, -1.0, J.D, n, om, s, 1.0, W, s, lds);
  else
    wg_gemm<true, false>(n, s, n, -1.0, J.D, n, om, s, 1.0, W, s, lds);
  wg_gemm<true, false>(r, s, n, 1.0, By, r, W, s, 0.0, J.out[2 + side], s, lds);
}

// -------------------------------------------------------- sample handling
// dst[i][c] = (T) src[i][c] for i < M, c < s; 0 in the padding (ld x sp).
template <typename T>
__global__ void k_pad_samples(const double *__restrict__ src, int M, int s, int ld, int sp,
                              T *__restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ld * sp) return;
  const int i = (int)(e / sp), c = (int)(e % sp);
  dst[e] = (i < M && c < s) ? (T)src[(size_t)i * s + c] : T(0);
}

// Cluster-order FP64 rows: dst[i][c] = sc(perm[i]) src[perm[i]][c] for
// i < M, c < s (sc = -e[.] when e is given, else 1).
template <typename T>
__global__ void k_gather_samples(const T *__restrict__ src, int sp, const int *__restrict__ perm,
                                 const double *__restrict__ e, int M, int s,
                                 double *__restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)M * s) return;
  const int i = (int)(t / s), c = (int)(t % s);
  const int p = perm ? perm[i] : i;
  const double v = (double)src[(size_t)p * sp + c];
  dst[t] = e ? -e[p] * v : v;
}

// Natural-order FP64 rows gathered to cluster order (Om, Ps of the leaves).
__global__ void k_gather_rows(const double *__restrict__ src, const int *__restrict__ perm, int M,
                              int s, double *__restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)M * s) return;
  const int i = (int)(t / s), c = (int)(t % s);
  dst[t] = src[(size_t)(perm ? perm[i] : i) * s + c];
}

// ------------------------------------------------------------ factor I/O
__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
  const unsigned lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest even
  return (unsigned short)(u >> 16);
}
template <typename F> struct FIO;
template <> struct FIO<unsigned short> {
  static __device__ __forceinline__ unsigned short put(double v) { return to_bf16((float)v); }
  static __device__ __forceinline__ double get(unsigned short v) {
    return (double)__uint_as_float(((unsigned)v) << 16);
  }
};
template <> struct FIO<float> {
  static __device__ __forceinline__ float put(double v) { return (float)v; }
  static __device__ __forceinline__ double get(float v) { return (double)v; }
};
template <> struct FIO<double> {
  static __device__ __forceinline__ double put(double v) { return v; }
  static __device__ __forceinline__ double get(double v) { return v; }
};

template <typename F>
__global__ void k_pack_factors(const double *__restrict__ src, size_t len, F *__restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) dst[e] = FIO<F>::put(src[e]);
}

// ---------------------------------------------------------------- apply
// Block b = 2 (s - 1) + 0 is S_{s+1,s} (input interface s, output s + 1),
// b = 2 (s - 1) + 1 is S_{s,s+1} (input s + 1, output s); 1-based
// interfaces, s = 1 .. n_slabs - 2.  Transposed: input and output exchange.
__device__ __forceinline__ int blk_in(int b, int trans) {
  const int s = b / 2 + 1;
  const bool a = (b & 1) == 0;
  return trans ? (a ? s + 1 : s) : (a ? s : s + 1);
}

// Stored factors: every row of U, V (r entries) and D (n entries) starts on
// an 8-element boundary (rows padded with zeros to ldr and ldn entries), so
// a thread reads eight entries of a row with 16-byte loads (one for BF16).
template <typename F>
__device__ __forceinline__ void load8(const F *p, double (&v)[8]) {
  if constexpr (sizeof(F) == 2) {
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 q = *reinterpret_cast<const __attribute__((address_space(1))) u32x4 *>(gp(p));
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[2 * e] = (double)__uint_as_float(q[e] << 16);
      v[2 * e + 1] = (double)__uint_as_float(q[e] & 0xffff0000u);
    }
  } else if constexpr (sizeof(F) == 4) {
    const auto a = ld16(p), c = ld16(p + 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = (double)a[e];
      v[4 + e] = (double)c[e];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const auto a = ld16(p + 2 * q);
      v[2 * q] = a[0];
      v[2 * q + 1] = a[1];
    }
  }
}

// smallest power of two >= n (n <= 32 here)
__device__ __forceinline__ int pow2_ge(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// out[i] += sum_c A[i][c] v[c] (i < rows, c < cols; rows of A padded to lda,
// a multiple of 8): a group of lp lanes per row, eight entries per lane and
// load, the row's partial sums reduced across the group.  Called by all
// threads with the same arguments.
template <typename F>
__device__ __forceinline__ void mv_rows(const F *A, int lda, int rows, int cols, const double *v,
                                        double *out) {
  const int nch = (cols + 7) >> 3;
  const int lp = pow2_ge(nch);
  const int g = threadIdx.x / lp, l = threadIdx.x % lp, G = WG / lp;
  for (int i0 = 0; i0 < rows; i0 += G) {
    const int i = i0 + g;
    double t = 0.0;
    if (i < rows)
      for (int ch = l; ch < nch; ch += lp) {
        double a[8];
        load8(A + (size_t)i * lda + 8 * ch, a);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (8 * ch + e < cols) t += a[e] * v[8 * ch + e];
      }
    for (int off = lp >> 1; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (i < rows && l == 0) out[i] += t;
  }
}

// out[c] += sum_i B[i][c] v[i] (i < rows, c < cols): lane l of a group of lp
// takes columns 8 l .. 8 l + 7 of the rows g, g + G, ...; a column's partial
// sums are reduced across the wavefront's groups by shuffles and across the
// four wavefronts through red.  Called by all threads with the same
// arguments; out is complete on return.
template <typename F>
__device__ __forceinline__ void mv_cols(const F *B, int ldb, int rows, int cols, const double *v,
                                        double *out, double (*red)[kMaxN]) {
  const int nch = (cols + 7) >> 3;
  const int lp = pow2_ge(nch);
  const int g = threadIdx.x / lp, l = threadIdx.x % lp, G = WG / lp;
  double t[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) t[e] = 0.0;
  if (l < nch)
    for (int i = g; i < rows; i += G) {
      double a[8];
      load8(B + (size_t)i * ldb + 8 * l, a);
      const double vi = v[i];
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] += a[e] * vi;
    }
  for (int off = lp; off < 64; off <<= 1)
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] += __shfl_xor(t[e], off);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane < lp && l < nch)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (8 * l + e < cols) red[w][8 * l + e] = t[e];
  __syncthreads();
  for (int c = threadIdx.x; c < cols; c += WG) out[c] += red[0][c] + red[1][c] + red[2][c] + red[3][c];
  __syncthreads();
}

// out[c] = sum_i B[i][c] v[i] (i < rows, c < cols) by one wavefront: lane
// l of a group of lp takes the 8-column chunk l of the rows g, g + G, ...;
// the groups' partial sums are reduced by shuffles.
template <typename F>
__device__ __forceinline__ void wave_mv_cols(const F *B, int ldb, int rows, int cols,
                                             const double *v, double *out) {
  const int lane = threadIdx.x & 63;
  const int nch = (cols + 7) >> 3;
  const int lp = pow2_ge(nch);
  const int g = lane / lp, l = lane % lp, G = 64 / lp;
  double t[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) t[e] = 0.0;
  if (l < nch)
    for (int i = g; i < rows; i += G) {
      double a[8];
      load8(B + (size_t)i * ldb + 8 * l, a);
      const double vi = v[i];
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] += a[e] * vi;
    }
  for (int off = lp; off < 64; off <<= 1)
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] += __shfl_xor(t[e], off);
  if (lane < lp && l < nch)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (8 * l + e < cols) out[8 * l + e] = t[e];
}

// Up, leaf level, four leaves per work-group (one per wavefront):
// xh[b][L][t] = B^T x_in[perm[lo..lo+n)] (B = V, or U if trans).
template <typename F>
__global__ __launch_bounds__(WG) void k_hbs_up_leaf4(const HbsNodeDev *__restrict__ nodes, int nl,
                                                     const F *__restrict__ fac, size_t bstride,
                                                     const int *__restrict__ perm,
                                                     const double *__restrict__ x, int ld,
                                                     double *__restrict__ hat, size_t hstride,
                                                     size_t hoff, int trans) {
  __shared__ double v[WG / 64][kMaxN];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * (WG / 64) + w, b = blockIdx.y;
  const bool has = t < nl;
  HbsNodeDev N{};
  if (has) {
    N = nodes[t];
    const double *xin = x + (size_t)(blk_in(b, trans) - 1) * ld;
    for (int i = lane; i < N.n; i += 64) v[w][i] = xin[perm ? perm[N.lo + i] : N.lo + i];
  }
  __syncthreads();
  if (has)
    wave_mv_cols(fac + b * bstride + (trans ? N.pU : N.pV), N.ldr, N.n, N.r, v[w],
                 hat + b * hstride + hoff + N.roff);
}

// Up, internal level: xh[b][d][t] = B^T xh[b][d+1][children].
template <typename F>
__global__ __launch_bounds__(WG) void k_hbs_up(const HbsNodeDev *__restrict__ nodes,
                                               const F *__restrict__ fac, size_t bstride,
                                               double *__restrict__ hat, size_t hstride,
                                               size_t hoff, size_t hoff_child, int trans) {
  __shared__ double v[kMaxN], out[kMaxN], red[WG / 64][kMaxN];
  const HbsNodeDev N = nodes[blockIdx.x];
  const int b = blockIdx.y;
  const double *in = hat + b * hstride + hoff_child + N.coff;
  for (int i = threadIdx.x; i < N.n; i += WG) v[i] = in[i];
  for (int c = threadIdx.x; c < N.r; c += WG) out[c] = 0.0;
  __syncthreads();
  mv_cols(fac + b * bstride + (trans ? N.pU : N.pV), N.ldr, N.n, N.r, v, out, red);
  double *h = hat + b * hstride + hoff + N.roff;
  for (int c = threadIdx.x; c < N.r; c += WG) h[c] = out[c];
}

// Root: yh[b][1] = D_root xh[b][1] (or D_root^T).
template <typename F>
__global__ __launch_bounds__(WG) void k_hbs_root(const HbsNodeDev *__restrict__ root,
                                                 const F *__restrict__ fac, size_t bstride,
                                                 double *__restrict__ hat, size_t hstride,
                                                 size_t hoff_x, size_t hoff_y, int trans) {
  __shared__ double v[kMaxN], out[kMaxN], red[WG / 64][kMaxN];
  const HbsNodeDev R = root[0];
  const int b = blockIdx.x;
  const double *in = hat + b * hstride + hoff_x;
  for (int i = threadIdx.x; i < R.n; i += WG) {
    v[i] = in[i];
    out[i] = 0.0;
  }
  __syncthreads();
  const F *D = fac + b * bstride + R.pD;
  if (trans)
    mv_cols(D, R.ldn, R.n, R.n, v, out, red);
  else
    mv_rows(D, R.ldn, R.n, R.n, v, out);
  __syncthreads();
  double *o = hat + b * hstride + hoff_y;
  for (int i = threadIdx.x; i < R.n; i += WG) o[i] = out[i];
}

// Down, internal level d: yh[b][d+1][children] = B' yh[b][d][t] + D xh[b][d+1][children]
// (B' = U, or V if trans; D or D^T).
template <typename F>
__global__ __launch_bounds__(WG) void k_hbs_down(const HbsNodeDev *__restrict__ nodes,
                                                 const F *__restrict__ fac, size_t bstride,
                                                 double *__restrict__ hat, size_t hstride,
                                                 size_t hoff_xc, size_t hoff_y, size_t hoff_yc,
                                                 int trans) {
  __shared__ double vy[kMaxN], vx[kMaxN], out[kMaxN], red[WG / 64][kMaxN];
  const HbsNodeDev N = nodes[blockIdx.x];
  const int b = blockIdx.y;
  double *hb = hat + b * hstride;
  for (int c = threadIdx.x; c < N.r; c += WG) vy[c] = hb[hoff_y + N.roff + c];
  for (int i = threadIdx.x; i < N.n; i += WG) {
    vx[i] = hb[hoff_xc + N.coff + i];
    out[i] = 0.0;
  }
  __syncthreads();
  const F *fb = fac + b * bstride;
  mv_rows(fb + (trans ? N.pV : N.pU), N.ldr, N.n, N.r, vy, out);
  __syncthreads();
  if (trans)
    mv_cols(fb + N.pD, N.ldn, N.n, N.n, vx, out, red);
  else
    mv_rows(fb + N.pD, N.ldn, N.n, N.n, vx, out);
  __syncthreads();
  for (int i = threadIdx.x; i < N.n; i += WG) hb[hoff_yc + N.coff + i] = out[i];
}

// out[i] = sum_c A[i][c] v[c] (i < rows, c < cols) by one wavefront: a
// group of lp lanes per row, eight entries per lane and load, the row's
// partial sums reduced by shuffles.
template <typename F>
__device__ __forceinline__ void wave_mv_rows(const F *A, int lda, int rows, int cols,
                                             const double *v, double *out) {
  const int lane = threadIdx.x & 63;
  const int nch = (cols + 7) >> 3;
  const int lp = pow2_ge(nch);
  const int g = lane / lp, l = lane % lp, G = 64 / lp;
  for (int i0 = 0; i0 < rows; i0 += G) {
    const int i = i0 + g;
    double t = 0.0;
    if (i < rows)
      for (int ch = l; ch < nch; ch += lp) {
        double a[8];
        load8(A + (size_t)i * lda + 8 * ch, a);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (8 * ch + e < cols) t += a[e] * v[8 * ch + e];
      }
    for (int off = lp >> 1; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (i < rows && l == 0) out[i] = t;
  }
}

// Leaves: for output interface jo (blockIdx.y + 1) and leaf t,
//   y_jo[perm] = x_jo[perm] - sum over its blocks (B' yh + D x_in[perm])
// (B' = U, or V if trans; D or D^T); without a basis (a single cluster) the
// leaf is the root and only D is applied.  Wavefront 2 q + h takes block q's
// basis product (h = 0) or dense product (h = 1) into its own LDS slice;
// the slices are summed after one barrier.  The first leaf's work-group also
// copies the padding entries (M .. ld - 1) of y_jo from x_jo.
template <typename F>
__global__ __launch_bounds__(WG) void k_hbs_leaf_out(
    const HbsNodeDev *__restrict__ nodes, const F *__restrict__ fac, size_t bstride,
    const int *__restrict__ perm, const double *__restrict__ x, double *__restrict__ y, int M,
    int ld, int n_ds, const double *__restrict__ hat, size_t hstride, size_t hoff_y,
    int has_basis, int trans) {
  static_assert(WG == 256, "four wavefronts: two products for each of two blocks");
  __shared__ double vin[4][kMaxN], part[4][kMaxN];
  const HbsNodeDev N = nodes[blockIdx.x];
  const int jo = blockIdx.y + 1;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // blocks writing to jo: non-transposed S_{jo,jo-1} (b = 2(jo-2)) and
  // S_{jo,jo+1} (b = 2(jo-1)+1); transposed S_{jo+1,jo} (b = 2(jo-1)) and
  // S_{jo-1,jo} (b = 2(jo-2)+1)
  int bl[2], nb = 0;
  if (!trans) {
    if (jo >= 2) bl[nb++] = 2 * (jo - 2);
    if (jo <= n_ds - 1) bl[nb++] = 2 * (jo - 1) + 1;
  } else {
    if (jo <= n_ds - 1) bl[nb++] = 2 * (jo - 1);
    if (jo >= 2) bl[nb++] = 2 * (jo - 2) + 1;
  }
  const int q = w >> 1, h = w & 1;
  const bool act = q < nb && (h == 1 || has_basis);
  int b = 0;
  if (act) {
    b = bl[q];
    if (h == 0) {
      for (int c = lane; c < N.r; c += 64) vin[w][c] = hat[b * hstride + hoff_y + N.roff + c];
    } else {
      const double *xin = x + (size_t)(blk_in(b, trans) - 1) * ld;
      for (int i = lane; i < N.n; i += 64) vin[w][i] = xin[perm ? perm[N.lo + i] : N.lo + i];
    }
  }
  __syncthreads();
  if (act) {
    const F *fb = fac + b * bstride;
    if (h == 0)
      wave_mv_rows(fb + (trans ? N.pV : N.pU), N.ldr, N.n, N.r, vin[w], part[w]);
    else if (trans)
      wave_mv_cols(fb + N.pD, N.ldn, N.n, N.n, vin[w], part[w]);
    else
      wave_mv_rows(fb + N.pD, N.ldn, N.n, N.n, vin[w], part[w]);
  }
  __syncthreads();
  const double *xo = x + (size_t)(jo - 1) * ld;
  double *yo = y + (size_t)(jo - 1) * ld;
  for (int i = threadIdx.x; i < N.n; i += WG) {
    double s = 0.0;
    for (int u = 0; u < 4; ++u)
      if ((u >> 1) < nb && ((u & 1) == 1 || has_basis)) s += part[u][i];
    const int p = perm ? perm[N.lo + i] : N.lo + i;
    yo[p] = xo[p] - s;
  }
  if (blockIdx.x == 0)
    for (int c = M + threadIdx.x; c < ld; c += WG) yo[c] = xo[c];
}

// Stored factors from the FP64 compression output: job (j, b) copies one
// matrix (rows x cols, contiguous rows at src) of block b to rows padded to
// ldd entries at dst, converted to F.  The padding is cleared beforehand.
struct HbsPack {
  long long src, dst;
  int rows, cols, ldd, pad_;
};
template <typename F>
__global__ void k_pack_hbs(const HbsPack *__restrict__ jobs, const double *__restrict__ src,
                           size_t sblock, F *__restrict__ dst, size_t dblock) {
  const HbsPack J = jobs[blockIdx.x];
  const double *s = src + blockIdx.y * sblock + J.src;
  F *d = dst + blockIdx.y * dblock + J.dst;
  const int tot = J.rows * J.cols;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int i = e / J.cols, c = e % J.cols;
    d[(size_t)i * J.ldd + c] = FIO<F>::put(s[e]);
  }
}
}  // namespace

// ------------------------------------------------------------- host side
namespace {

// Uniform-depth binary cluster tree (as the oracle's): a line of M points
// split at the midpoint, or (grid) the n x n interface grid, rectangles split
// at the midpoint of their longer side (y on ties).  Fills levels with the
// leaf ranges (lo, size) at the deepest level and the node counts above, and
// the permutation cluster order -> natural order.
void hbs_tree(int dim, int n, int M, int leaf, std::vector<std::vector<std::pair<int, int>>> &sz,
              std::vector<int> &perm) {
  sz.clear();
  perm.clear();
  if (dim == 2) {
    std::vector<std::pair<int, int>> lev = {{0, M}};  // (lo, hi)
    sz.push_back(lev);
    for (;;) {
      int mx = 0;
      for (auto &p : lev) mx = std::max(mx, p.second - p.first);
      if (mx <= leaf) break;
      std::vector<std::pair<int, int>> nx;
      for (auto &p : lev) {
        const int mid = p.first + (p.second - p.first + 1) / 2;
        nx.push_back({p.first, mid});
        nx.push_back({mid, p.second});
      }
      lev = nx;
      sz.push_back(lev);
    }
    for (int i = 0; i < M; ++i) perm.push_back(i);
    return;
  }
  struct R { int y0, y1, z0, z1; };
  std::vector<std::vector<R>> rl = {{{0, n, 0, n}}};
  for (;;) {
    int mx = 0;
    for (auto &q : rl.back()) mx = std::max(mx, (q.y1 - q.y0) * (q.z1 - q.z0));
    if (mx <= leaf) break;
    std::vector<R> nx;
    for (auto &q : rl.back()) {
      if (q.y1 - q.y0 >= q.z1 - q.z0) {
        const int ym = q.y0 + (q.y1 - q.y0 + 1) / 2;
        nx.push_back({q.y0, ym, q.z0, q.z1});
        nx.push_back({ym, q.y1, q.z0, q.z1});
      } else {
        const int zm = q.z0 + (q.z1 - q.z0 + 1) / 2;
        nx.push_back({q.y0, q.y1, q.z0, zm});
        nx.push_back({q.y0, q.y1, zm, q.z1});
      }
    }
    rl.push_back(nx);
  }
  for (auto &q : rl.back())
    for (int yy = q.y0; yy < q.y1; ++yy)
      for (int zz = q.z0; zz < q.z1; ++zz) perm.push_back(yy * n + zz);
  for (auto &lev : rl) {
    std::vector<std::pair<int, int>> v;
    int at = 0;
    for (auto &q : lev) {
      const int c = (q.y1 - q.y0) * (q.z1 - q.z0);
      v.push_back({at, at + c});
      at += c;
    }
    sz.push_back(v);
  }
}

}  // namespace

void hbs_free(ddst_op *op) {
  Hbs *H = op->hbs;
  if (!H) return;
  (void)hipDeviceSynchronize();
  if (H->d_perm) dev_free(H->d_perm);
  if (H->factors) dev_free(H->factors);
  if (H->nodes) dev_free(H->nodes);
  if (H->hat) dev_free(H->hat);
  delete H;
  op->hbs = nullptr;
}

bool hbs_ready(const ddst_op *op) { return op->hbs != nullptr; }

void hbs_info(const ddst_op *op, double *bytes, int *rank, double *t_sample_ms,
              double *t_compress_ms) {
  const Hbs *H = op->hbs;
  if (bytes) *bytes = H ? (double)H->bytes : 0.0;
  if (rank) *rank = H ? H->k : 0;
  if (t_sample_ms) *t_sample_ms = H ? H->t_sample_ms : 0.0;
  if (t_compress_ms) *t_compress_ms = H ? H->t_compress_ms : 0.0;
}

namespace {

template <typename T>
void sample_chains(ddst_op *op, const double *Om, const double *Ps, int s, int sp,
                   const int *d_perm, double *Ycl, double *Zcl, hipStream_t st) {
  const int m = op->m, ld = op->ld, M = op->M, nsl = op->n_slabs, nds = op->n_ds;
  const int ns = nsl - 2;  // slabs between two interfaces
  const size_t mb = op->mat_bytes, cb = (size_t)ld * sp * sizeof(T);
  auto G = [&](int slab, int k) -> const void * {
    return static_cast<const unsigned char *>(op->G) + ((size_t)slab * (m - 1) + (k - 1)) * mb;
  };
  auto Sinv = [&](int j) -> const void * {
    return static_cast<const unsigned char *>(op->Sinv) + (size_t)(j - 1) * mb;
  };
  auto Em = [&](int plane) { return op->Em + (size_t)plane * ld; };
  auto Ep = [&](int plane) { return op->Ep + (size_t)plane * ld; };
  // buffers: padded Om, Ps; W_j = Sigma_j^{-T} Ps; two ping-pong buffers per
  // chain (four chains per slab); the transfer samples of every block
  BMem pad(2 * cb), wbuf((size_t)nds * cb), chains((size_t)8 * ns * cb), ybuf((size_t)2 * ns * cb);
  T *OmT = pad.as<T>(), *PsT = OmT + (size_t)ld * sp;
  auto W = [&](int j) { return wbuf.as<T>() + (size_t)(j - 1) * ld * sp; };
  auto CH = [&](int slab, int chain, int pp) {  // chain: 0 aY, 1 bY, 2 aZ, 3 bZ
    return chains.as<T>() + ((size_t)((slab - 1) * 4 + chain) * 2 + pp) * ld * sp;
  };
  auto YO = [&](int b) { return ybuf.as<T>() + (size_t)b * ld * sp; };
  const size_t tot = (size_t)ld * sp;
  hipLaunchKernelGGL(k_pad_samples<T>, dim3(nblk1(tot)), dim3(256), 0, st, Om, M, s, ld, sp, OmT);
  hipLaunchKernelGGL(k_pad_samples<T>, dim3(nblk1(tot)), dim3(256), 0, st, Ps, M, s, ld, sp, PsT);
  // one table of all jobs, per launch a slice
  std::vector<GemmJob> all;
  std::vector<std::pair<size_t, int>> lyN(m), lyT(m);  // per step i: (first, count)
  for (int i = 1; i <= m - 1; ++i) {
    lyN[i].first = all.size();
    for (int sl = 1; sl <= ns; ++sl) {
      const int ka = i, kb = m - i;
      all.push_back({G(sl, ka), i == 1 ? OmT : CH(sl, 0, (i - 1) & 1), CH(sl, 0, i & 1),
                     Em(sl * m + ka)});
      all.push_back({G(sl, kb), i == 1 ? OmT : CH(sl, 1, (i - 1) & 1), CH(sl, 1, i & 1),
                     Ep(sl * m + kb)});
    }
    lyN[i].second = (int)(all.size() - lyN[i].first);
    lyT[i].first = all.size();
    for (int sl = 1; sl <= ns; ++sl) {
      const int ka = m - i, kb = i;
      all.push_back({G(sl, ka), i == 1 ? W(sl + 1) : CH(sl, 2, (i - 1) & 1), CH(sl, 2, i & 1),
                     i == 1 ? Em((sl + 1) * m) : Em(sl * m + ka + 1)});
      all.push_back({G(sl, kb), i == 1 ? W(sl) : CH(sl, 3, (i - 1) & 1), CH(sl, 3, i & 1),
                     i == 1 ? Ep(sl * m) : Ep(sl * m + kb - 1)});
    }
    lyT[i].second = (int)(all.size() - lyT[i].first);
  }
  const size_t wfirst = all.size();
  for (int j = 1; j <= nds; ++j) all.push_back({Sinv(j), PsT, W(j), nullptr});
  const size_t yfirst = all.size();
  const int last = (m - 1) & 1;
  for (int sl = 1; sl <= ns; ++sl) {
    all.push_back({Sinv(sl + 1), CH(sl, 0, last), YO(2 * (sl - 1)), Em((sl + 1) * m)});
    all.push_back({Sinv(sl), CH(sl, 1, last), YO(2 * (sl - 1) + 1), Ep(sl * m)});
  }
  BMem tab(all.size() * sizeof(GemmJob));
  BCHK(hipMemcpyAsync(tab.p, all.data(), all.size() * sizeof(GemmJob), hipMemcpyHostToDevice, st));
  const GemmJob *dj = tab.as<GemmJob>();
  launch_gemm_rect<T>(dj + wfirst, nds, ld, sp, M, s, 1, 1.0, 0.0, st);
  for (int i = 1; i <= m - 1; ++i) {
    launch_gemm_rect<T>(dj + lyN[i].first, lyN[i].second, ld, sp, M, s, 0, -1.0, 0.0, st);
    launch_gemm_rect<T>(dj + lyT[i].first, lyT[i].second, ld, sp, M, s, 1, -1.0, 0.0, st);
  }
  launch_gemm_rect<T>(dj + yfirst, 2 * ns, ld, sp, M, s, 0, -1.0, 0.0, st);
  // FP64 cluster-order samples; the Z chains end with a row scaling
  const size_t per = (size_t)M * s;
  for (int sl = 1; sl <= ns; ++sl)
    for (int t = 0; t < 2; ++t) {
      const int b = 2 * (sl - 1) + t;
      hipLaunchKernelGGL(k_gather_samples<T>, dim3(nblk1(per)), dim3(256), 0, st, YO(b), sp,
                         d_perm, (const double *)nullptr, M, s, Ycl + (size_t)b * per);
      const double *e = t == 0 ? Em(sl * m + 1) : Ep(sl * m + m - 1);
      hipLaunchKernelGGL(k_gather_samples<T>, dim3(nblk1(per)), dim3(256), 0, st,
                         CH(sl, 2 + t, last), sp, d_perm, e, M, s, Zcl + (size_t)b * per);
    }
  BCHK(hipGetLastError());
  BCHK(hipStreamSynchronize(st));  // keeps the buffers alive until done
}

}  // namespace

int hbs_sample_blocks(ddst_op *op, int ncols, const double *X, double *Y, double *Z,
                      hipStream_t st) {
  if (op->n_slabs < 3) return DDST_OK;  // no transfer blocks
  const int sp = (ncols + kTile - 1) / kTile * kTile;
  if (op->prec == DDST_FP32)
    sample_chains<float>(op, X, X, ncols, sp, nullptr, Y, Z, st);
  else
    sample_chains<double>(op, X, X, ncols, sp, nullptr, Y, Z, st);
  return DDST_OK;
}

// Sampled HBS compression of every transfer block; returns DDST_OK,
// DDST_EINVAL (with *msg) or DDST_EBREAKDOWN (a Gram matrix not positive).
int hbs_compress(ddst_op *op, int k, int q, int leaf, int dtype, const double *omega,
                 const double *psi, uint64_t seed, hipStream_t st, std::string *msg) {
  const int M = op->M, nds = op->n_ds, ns = op->n_slabs - 2;
  const int s = 3 * k + q;
  if (k < 1 || q < 2) {
    *msg = "need rank k >= 1 and oversampling q >= 2";
    return DDST_EINVAL;
  }
  if (s > kMaxS) {
    *msg = "3 k + q must be <= " + std::to_string(kMaxS);
    return DDST_EINVAL;
  }
  if (leaf < 1) leaf = 2 * k;
  std::vector<std::vector<std::pair<int, int>>> rng;
  std::vector<int> perm;
  const int n = op->n;
  hbs_tree(op->dim, n, M, leaf, rng, perm);
  const int L = (int)rng.size() - 1;
  // node sizes and ranks per level
  std::vector<std::vector<int>> nn(L + 1), rr(L + 1);
  for (auto &pr : rng[L]) nn[L].push_back(pr.second - pr.first);
  for (int d = L; d >= 0; --d) {
    if (d < L) {
      nn[d].clear();
      for (size_t t = 0; t < rng[d].size(); ++t) nn[d].push_back(rr[d + 1][2 * t] + rr[d + 1][2 * t + 1]);
    }
    rr[d].clear();
    for (int v : nn[d]) rr[d].push_back(d == 0 ? 0 : std::min(k, v));
    for (int v : nn[d]) {
      const int need = v + (d == 0 ? 0 : std::min(k, v));
      if (v > kMaxN || need > s) {
        *msg = "a cluster of " + std::to_string(v) + " points needs " + std::to_string(need) +
               " samples (s = 3 k + q = " + std::to_string(s) + ", node size <= " +
               std::to_string(kMaxN) + "): lower the leaf size";
        return DDST_EINVAL;
      }
    }
  }
  hbs_free(op);
  Hbs *H = new Hbs();
  op->hbs = H;
  try {
    H->k = k;
    H->s = s;
    H->sp = (s + kTile - 1) / kTile * kTile;
    H->leaf = leaf;
    H->depth = L;
    H->dtype = dtype;
    H->nblk = 2 * std::max(ns, 0);
    H->perm = perm;
    // node tables: factor offsets per block, hat offsets per level
    H->lv.assign(L + 1, {});
    size_t off = 0, poff = 0;
    H->nhat.assign(L + 1, 0);
    for (int d = L; d >= 1; --d) {
      int roff = 0, coff = 0;
      for (size_t t = 0; t < nn[d].size(); ++t) {
        HbsNodeDev N{};
        N.n = nn[d][t];
        N.r = rr[d][t];
        N.lo = d == L ? rng[L][t].first : 0;
        N.roff = roff;
        roff += N.r;
        N.coff = coff;
        if (d < L) coff += nn[d][t];  // children's entries at level d+1
        N.fU = (long long)off;
        off += (size_t)N.n * N.r;
        N.fV = (long long)off;
        off += (size_t)N.n * N.r;
        N.fD = (long long)off;
        off += (size_t)N.n * N.n;
        N.ldr = (N.r + 7) / 8 * 8;
        N.ldn = (N.n + 7) / 8 * 8;
        N.pU = (long long)poff;
        poff += (size_t)N.n * N.ldr;
        N.pV = (long long)poff;
        poff += (size_t)N.n * N.ldr;
        N.pD = (long long)poff;
        poff += (size_t)N.n * N.ldn;
        H->lv[d].push_back(N);
      }
      H->nhat[d] = roff;
    }
    {
      HbsNodeDev R{};
      R.n = nn[0][0];
      R.r = 0;
      R.lo = 0;
      H->root_off = off;
      R.fD = (long long)off;
      off += (size_t)R.n * R.n;
      R.ldn = (R.n + 7) / 8 * 8;
      R.pD = (long long)poff;
      poff += (size_t)R.n * R.ldn;
      H->lv[0].push_back(R);
    }
    H->block_elems = (off + 63) / 64 * 64;
    H->stored_elems = (poff + 63) / 64 * 64;
    // hat vector layout per block: x^ then y^ for every level 1..L
    H->hoff.assign(2 * (L + 1), 0);
    size_t h = 0;
    for (int d = 1; d <= L; ++d) {
      H->hoff[2 * d] = h;
      h += H->nhat[d];
      H->hoff[2 * d + 1] = h;
      h += H->nhat[d];
    }
    H->hat_per_block = std::max<size_t>((h + 31) / 32 * 32, 32);
    // device node tables
    std::vector<unsigned char> nodeblob;
    H->node_off.assign(L + 1, 0);
    for (int d = 0; d <= L; ++d) {
      H->node_off[d] = nodeblob.size();
      const size_t bytes = H->lv[d].size() * sizeof(HbsNodeDev);
      nodeblob.resize(nodeblob.size() + (bytes + 255) / 256 * 256);
      std::memcpy(nodeblob.data() + H->node_off[d], H->lv[d].data(), bytes);
    }
    if (dev_malloc(&H->nodes, nodeblob.size()) != hipSuccess) throw std::bad_alloc();
    BCHK(hipMemcpyAsync(H->nodes, nodeblob.data(), nodeblob.size(), hipMemcpyHostToDevice, st));
    const bool ident = op->dim == 2;
    if (!ident) {
      if (dev_malloc((void **)&H->d_perm, (size_t)M * sizeof(int)) != hipSuccess)
        throw std::bad_alloc();
      BCHK(hipMemcpyAsync(H->d_perm, perm.data(), (size_t)M * sizeof(int), hipMemcpyHostToDevice,
                          st));
    }
    if (H->nblk > 0 && dev_malloc((void **)&H->hat, (size_t)H->nblk * H->hat_per_block * 8) != hipSuccess)
      throw std::bad_alloc();
    const size_t esz = dtype == DDST_FACTOR_BF16 ? 2 : dtype == DDST_FACTOR_FP32 ? 4 : 8;
    H->bytes = (size_t)H->nblk * H->stored_elems * esz;
    if (H->nblk == 0) {
      BCHK(hipStreamSynchronize(st));
      return DDST_OK;
    }
    hipEvent_t e0, e1, e2;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    BCHK(hipEventCreate(&e2));
    BCHK(hipEventRecord(e0, st));
    // ---- probes (caller's, or Philox) and the samples
    const size_t per = (size_t)M * s;
    BMem probes(2 * per * 8);
    double *Om = probes.as<double>(), *Ps = Om + per;
    if (omega)
      BCHK(hipMemcpyAsync(Om, omega, per * 8, hipMemcpyDeviceToDevice, st));
    else
      launch_gaussian(Om, M, s, seed, 101u, st);
    if (psi)
      BCHK(hipMemcpyAsync(Ps, psi, per * 8, hipMemcpyDeviceToDevice, st));
    else
      launch_gaussian(Ps, M, s, seed, 102u, st);
    const int nb = H->nblk;
    BMem samples((size_t)2 * nb * per * 8);
    double *Ycl = samples.as<double>(), *Zcl = Ycl + (size_t)nb * per;
    if (op->prec == DDST_FP32)
      sample_chains<float>(op, Om, Ps, s, H->sp, H->d_perm, Ycl, Zcl, st);
    else
      sample_chains<double>(op, Om, Ps, s, H->sp, H->d_perm, Ycl, Zcl, st);
    BCHK(hipEventRecord(e1, st));
    // cluster-order probes of the leaves
    BMem probes_cl(2 * per * 8);
    double *Omc = probes_cl.as<double>(), *Psc = Omc + per;
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk1(per)), dim3(256), 0, st, Om, H->d_perm, M, s, Omc);
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk1(per)), dim3(256), 0, st, Ps, H->d_perm, M, s, Psc);
    // ---- compression, level by level
    BMem stage((size_t)nb * H->block_elems * 8);  // FP64 factors
    double *F64 = stage.as<double>();
    BMem flagm(sizeof(int));
    BCHK(hipMemsetAsync(flagm.p, 0, sizeof(int), st));
    // sketch rows of the level being processed (above the leaves): per
    // block, node rows stacked, four arrays
    std::unique_ptr<BMem> cur, nxt;
    for (int d = L; d >= 0; --d) {
      const auto &lev = H->lv[d];
      const int nnode = (int)lev.size();
      int rows = 0;
      for (auto &N : lev) rows += N.n;
      const size_t lvl_rows = (size_t)rows * s;  // one block's rows at this level
      // the parent level's arrays
      int prow = 0;
      if (d >= 1)
        for (auto &N : H->lv[d - 1]) prow += N.n;
      if (d >= 1) nxt.reset(new BMem((size_t)4 * nb * prow * s * 8));
      // per-job scratch: G[2], H[2] (n x n), W[2] (n x s), T (n x s + 2 n^2:
      // at least n^2 + r n and 2 r n + r^2 for the diagonal block)
      std::vector<HbsJob> jobs;
      std::vector<size_t> scr_off;
      size_t scr = 0;
      for (int b = 0; b < nb; ++b)
        for (int t = 0; t < nnode; ++t) {
          const HbsNodeDev &N = lev[t];
          scr_off.push_back(scr);
          scr += (size_t)6 * N.n * N.n + (size_t)3 * N.n * s;
        }
      BMem scratch(std::max<size_t>(scr, 1) * 8);
      double *S0 = scratch.as<double>();
      int rowoff = 0;
      std::vector<int> node_row(nnode);
      for (int t = 0; t < nnode; ++t) {
        node_row[t] = rowoff;
        rowoff += lev[t].n;
      }
      std::vector<int> prow_of(nnode, 0);
      if (d >= 1) {
        // child t of parent t/2: rows at the parent's start (+ the first child's rank)
        int at = 0;
        for (size_t pt = 0; pt < H->lv[d - 1].size(); ++pt) {
          prow_of[2 * pt] = at;
          prow_of[2 * pt + 1] = at + lev[2 * pt].r;
          at += H->lv[d - 1][pt].n;
        }
      }
      for (int b = 0; b < nb; ++b)
        for (int t = 0; t < nnode; ++t) {
          const HbsNodeDev &N = lev[t];
          HbsJob J{};
          J.n = N.n;
          J.r = N.r;
          if (d == L) {
            J.om = Omc + (size_t)N.lo * s;
            J.ps = Psc + (size_t)N.lo * s;
            J.y = Ycl + (size_t)b * per + (size_t)N.lo * s;
            J.z = Zcl + (size_t)b * per + (size_t)N.lo * s;
          } else {
            const double *base = cur->as<double>();
            const size_t o = ((size_t)b * rows + node_row[t]) * s;
            J.om = base + o;
            J.ps = base + (size_t)nb * lvl_rows + o;
            J.y = base + (size_t)2 * nb * lvl_rows + o;
            J.z = base + (size_t)3 * nb * lvl_rows + o;
          }
          double *w = S0 + scr_off[(size_t)b * nnode + t];
          J.G[0] = w;
          J.G[1] = w + (size_t)N.n * N.n;
          J.H[0] = w + (size_t)2 * N.n * N.n;
          J.H[1] = w + (size_t)3 * N.n * N.n;
          J.W[0] = w + (size_t)4 * N.n * N.n;
          J.W[1] = J.W[0] + (size_t)N.n * s;
          J.T = J.W[1] + (size_t)N.n * s;
          double *fb = F64 + (size_t)b * H->block_elems;
          if (d >= 1) {
            J.B[0] = fb + N.fU;
            J.B[1] = fb + N.fV;
            J.D = fb + N.fD;
            double *pb = nxt->as<double>();
            const size_t plr = (size_t)prow * s;
            const size_t o = ((size_t)b * prow + prow_of[t]) * s;
            J.out[0] = pb + o;
            J.out[1] = pb + (size_t)nb * plr + o;
            J.out[2] = pb + (size_t)2 * nb * plr + o;
            J.out[3] = pb + (size_t)3 * nb * plr + o;
          } else {
            J.H[0] = fb + H->root_off;  // D_root = Y Om^+ straight into the factors
          }
          jobs.push_back(J);
        }
      BMem jt(jobs.size() * sizeof(HbsJob));
      BCHK(hipMemcpyAsync(jt.p, jobs.data(), jobs.size() * sizeof(HbsJob), hipMemcpyHostToDevice, st));
      const HbsJob *dj = jt.as<HbsJob>();
      const unsigned nj = (unsigned)jobs.size();
      const unsigned sides = d == 0 ? 1 : 2;
      hipLaunchKernelGGL(k_hbs_gram, dim3(nj, sides), dim3(WG), 0, st, dj, s);
      hipLaunchKernelGGL(k_hbs_solve, dim3(nj, sides), dim3(WG), 0, st, dj, flagm.as<int>());
      if (d >= 1) {
        hipLaunchKernelGGL(k_hbs_resid, dim3(nj, 2), dim3(WG), 0, st, dj, s);
        hipLaunchKernelGGL(k_hbs_cpqr, dim3(nj, 2), dim3(WG), 0, st, dj, s);
        hipLaunchKernelGGL(k_hbs_diag, dim3(nj), dim3(WG), 0, st, dj);
        hipLaunchKernelGGL(k_hbs_reduce, dim3(nj, 2), dim3(WG), 0, st, dj, s);
      }
      BCHK(hipGetLastError());
      BCHK(hipStreamSynchronize(st));  // job tables and scratch of this level
      cur.swap(nxt);
      nxt.reset();
    }
    int bad = 0;
    BCHK(hipMemcpy(&bad, flagm.p, sizeof(int), hipMemcpyDeviceToHost));
    if (bad) {
      *msg = "a probe Gram matrix is not positive definite (degenerate samples)";
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      (void)hipEventDestroy(e2);
      hbs_free(op);
      return DDST_EBREAKDOWN;
    }
    // ---- pack
    if (dev_malloc(&H->factors, std::max<size_t>(H->bytes, 16)) != hipSuccess) throw std::bad_alloc();
    BCHK(hipMemsetAsync(H->factors, 0, H->bytes, st));
    {
      std::vector<HbsPack> pk;
      for (int d = 0; d <= L; ++d)
        for (const HbsNodeDev &N : H->lv[d]) {
          if (d >= 1) {
            pk.push_back({N.fU, N.pU, N.n, N.r, N.ldr, 0});
            pk.push_back({N.fV, N.pV, N.n, N.r, N.ldr, 0});
          }
          pk.push_back({N.fD, N.pD, N.n, N.n, N.ldn, 0});
        }
      BMem pt(pk.size() * sizeof(HbsPack));
      BCHK(hipMemcpyAsync(pt.p, pk.data(), pk.size() * sizeof(HbsPack), hipMemcpyHostToDevice,
                          st));
      const dim3 grid((unsigned)pk.size(), (unsigned)nb);
      const HbsPack *pj = pt.as<HbsPack>();
      const size_t sb = H->block_elems, db = H->stored_elems;
      if (dtype == DDST_FACTOR_BF16)
        hipLaunchKernelGGL(k_pack_hbs<unsigned short>, grid, dim3(256), 0, st, pj, F64, sb,
                           static_cast<unsigned short *>(H->factors), db);
      else if (dtype == DDST_FACTOR_FP32)
        hipLaunchKernelGGL(k_pack_hbs<float>, grid, dim3(256), 0, st, pj, F64, sb,
                           static_cast<float *>(H->factors), db);
      else
        hipLaunchKernelGGL(k_pack_hbs<double>, grid, dim3(256), 0, st, pj, F64, sb,
                           static_cast<double *>(H->factors), db);
      BCHK(hipGetLastError());
      BCHK(hipStreamSynchronize(st));  // the job table
    }
    BCHK(hipEventRecord(e2, st));
    BCHK(hipEventSynchronize(e2));
    float ms1 = 0, ms2 = 0;
    BCHK(hipEventElapsedTime(&ms1, e0, e1));
    BCHK(hipEventElapsedTime(&ms2, e1, e2));
    H->t_sample_ms = ms1;
    H->t_compress_ms = ms2;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    return DDST_OK;
  } catch (...) {
    hbs_free(op);
    throw;
  }
}

// y = S x (or S^T x) through the HBS form (padded interface vectors).
template <typename F>
void hbs_apply_t(const ddst_op *op, const double *x, double *y, int trans, hipStream_t st) {
  const Hbs *H = op->hbs;
  const F *fac = static_cast<const F *>(H->factors);
  const int L = H->depth, nb = H->nblk, ld = op->ld;
  auto nodes = [&](int d) {
    return reinterpret_cast<const HbsNodeDev *>(static_cast<const unsigned char *>(H->nodes) +
                                                H->node_off[d]);
  };
  const size_t bs = H->stored_elems, hs = H->hat_per_block;
  if (nb == 0) {
    BCHK(hipMemcpyAsync(y, x, (size_t)op->n_ds * ld * 8, hipMemcpyDeviceToDevice, st));
    return;
  }
  if (L >= 1) {
    const unsigned nl = (unsigned)H->lv[L].size();
    hipLaunchKernelGGL(k_hbs_up_leaf4<F>, dim3((nl + WG / 64 - 1) / (WG / 64), nb), dim3(WG), 0,
                       st, nodes(L), (int)nl, fac, bs, H->d_perm, x, ld, H->hat, hs,
                       H->hoff[2 * L], trans);
    for (int d = L - 1; d >= 1; --d)
      hipLaunchKernelGGL(k_hbs_up<F>, dim3((unsigned)H->lv[d].size(), nb), dim3(WG), 0, st,
                         nodes(d), fac, bs, H->hat, hs, H->hoff[2 * d], H->hoff[2 * (d + 1)],
                         trans);
    hipLaunchKernelGGL(k_hbs_root<F>, dim3(nb), dim3(WG), 0, st, nodes(0), fac, bs, H->hat, hs,
                       H->hoff[2], H->hoff[3], trans);
    for (int d = 1; d <= L - 1; ++d)
      hipLaunchKernelGGL(k_hbs_down<F>, dim3((unsigned)H->lv[d].size(), nb), dim3(WG), 0, st,
                         nodes(d), fac, bs, H->hat, hs, H->hoff[2 * (d + 1)], H->hoff[2 * d + 1],
                         H->hoff[2 * (d + 1) + 1], trans);
    hipLaunchKernelGGL(k_hbs_leaf_out<F>, dim3(nl, op->n_ds), dim3(WG), 0, st, nodes(L), fac, bs,
                       H->d_perm, x, y, op->M, ld, op->n_ds, H->hat, hs, H->hoff[2 * L + 1], 1,
                       trans);
  } else {
    // a single cluster: the root block is the whole transfer block
    hipLaunchKernelGGL(k_hbs_leaf_out<F>, dim3(1, op->n_ds), dim3(WG), 0, st, nodes(0), fac, bs,
                       H->d_perm, x, y, op->M, ld, op->n_ds, H->hat, hs, (size_t)0, 0, trans);
  }
}

int hbs_apply(const ddst_op *op, const double *x, double *y, int transpose, hipStream_t st) {
  if (!op->hbs) return DDST_ESTATE;
  prof_begin(KK_GEMV, st);
  switch (op->hbs->dtype) {
    case DDST_FACTOR_BF16: hbs_apply_t<unsigned short>(op, x, y, transpose, st); break;
    case DDST_FACTOR_FP32: hbs_apply_t<float>(op, x, y, transpose, st); break;
    default: hbs_apply_t<double>(op, x, y, transpose, st);
  }
  prof_end(KK_GEMV, st, (double)op->hbs->bytes);
  return DDST_OK;
}

}  // namespace ddst
