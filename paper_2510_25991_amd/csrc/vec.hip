// Memory-bound kernels of libddst: stencil set-up and FP64 residual, batched
// dense matrix-vector products (slab sweeps, interface blocks), interface
// right-hand sides, Krylov helpers and the cellwise gradient.
//
// The stencil follows the FD model problem: on every grid edge the
// coefficient is the mean of the 2^(dim-1) cells sharing the edge,
// convection uses centred differences, and boundary neighbours carry g.
#include <stdexcept>

#include "internal.h"

namespace ddst {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-wide sum of 256 threads; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double kappa_at(const double *kappa, int dim, int n, int c0, int c1,
                                           int c2) {
  if (!kappa) return 1.0;
  const size_t nc = (size_t)n + 1;
  if (dim == 2) return kappa[(size_t)c0 * nc + c1];
  return kappa[((size_t)c0 * nc + c1) * nc + c2];
}

// Mean coefficient of the edge from node p to p + e_axis (p 1-based).
__device__ double edge_coef(const double *kappa, int dim, int n, const int *p, int axis) {
  if (!kappa) return 1.0;
  int base[3] = {p[0] - 1, p[1] - 1, dim == 3 ? p[2] - 1 : 0};
  base[axis] = p[axis];  // cell index along the edge axis = node index of the lower end
  double s = 0.0;
  if (dim == 2) {
    const int o = 1 - axis;  // the other axis
    for (int t = 0; t < 2; ++t) {
      int c[2] = {base[0], base[1]};
      c[o] += t;
      s += kappa_at(kappa, 2, n, c[0], c[1], 0);
    }
    return 0.5 * s;
  }
  int oa = (axis == 0) ? 1 : 0, ob = (axis == 2) ? 1 : 2;
  for (int t = 0; t < 4; ++t) {
    int c[3] = {base[0], base[1], base[2]};
    c[oa] += t & 1;
    c[ob] += t >> 1;
    s += kappa_at(kappa, 3, n, c[0], c[1], c[2]);
  }
  return 0.25 * s;
}

__global__ void k_setup_coef(const double *__restrict__ kappa, const double *__restrict__ cz,
                             double b0, double b1, double b2, int dim, int n, double h,
                             double *__restrict__ coef) {
  const size_t N = (dim == 2) ? (size_t)n * n : (size_t)n * n * n;
  const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  int p[3];
  if (dim == 2) {
    p[0] = (int)(node / n) + 1;
    p[1] = (int)(node % n) + 1;
    p[2] = 0;
  } else {
    p[0] = (int)(node / ((size_t)n * n)) + 1;
    p[1] = (int)((node / n) % n) + 1;
    p[2] = (int)(node % n) + 1;
  }
  const double ih2 = 1.0 / (h * h), i2h = 0.5 / h;
  const double b[3] = {b0, b1, b2};
  double diag = cz ? cz[node] : 0.0;
  for (int a = 0; a < dim; ++a) {
    const double kp = edge_coef(kappa, dim, n, p, a) * ih2;
    int q[3] = {p[0], p[1], p[2]};
    q[a] -= 1;
    const double km = edge_coef(kappa, dim, n, q, a) * ih2;
    diag += kp + km;
    coef[(size_t)(1 + 2 * a) * N + node] = -km - b[a] * i2h;
    coef[(size_t)(2 + 2 * a) * N + node] = -kp + b[a] * i2h;
  }
  coef[node] = diag;
}

// Em[i][r] = coupling of plane i to plane i-1, Ep[i][r] = to plane i+1
// (rows 0 and n+1 and the padding stay zero).
__global__ void k_fill_couplings(const double *__restrict__ coef, int n, int M, int ld,
                                 size_t N, double *__restrict__ Em, double *__restrict__ Ep) {
  const int i = blockIdx.y;  // plane 0..n+1
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ld; r += gridDim.x * blockDim.x) {
    double em = 0.0, ep = 0.0;
    if (i >= 1 && i <= n && r < M) {
      const size_t node = (size_t)(i - 1) * M + r;
      em = coef[1 * N + node];
      ep = coef[2 * N + node];
    }
    Em[(size_t)i * ld + r] = em;
    Ep[(size_t)i * ld + r] = ep;
  }
}

// Residual r = f - A_full(x; g) (or f - A^T x), padded volume layout.
__global__ void k_residual(const double *__restrict__ coef, int dim, int n, int M, int ld,
                           const double *__restrict__ f, const double *__restrict__ g,
                           const double *__restrict__ x, double *__restrict__ r,
                           int transpose) {
  const size_t N = (size_t)M * n;
  const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const int i = (int)(node / M);  // 0-based plane
  const int ip = (int)(node % M);
  int p[3];
  p[0] = i + 1;
  if (dim == 2) {
    p[1] = ip + 1;
    p[2] = 0;
  } else {
    p[1] = ip / n + 1;
    p[2] = ip % n + 1;
  }
  const size_t nb = (size_t)n + 2;
  double acc = coef[node] * x[(size_t)i * ld + ip];
  for (int a = 0; a < dim; ++a) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int q[3] = {p[0], p[1], p[2]};
      q[a] += sgn;
      const bool inside = q[a] >= 1 && q[a] <= n;
      const int slot = (sgn < 0) ? 1 + 2 * a : 2 + 2 * a;
      if (inside) {
        const size_t qi = (size_t)(q[0] - 1);
        const size_t qip = (dim == 2) ? (size_t)(q[1] - 1)
                                      : (size_t)(q[1] - 1) * n + (size_t)(q[2] - 1);
        const size_t qnode = qi * M + qip;
        const double xv = x[qi * ld + qip];
        // A^T_{p,q} = A_{q,p}: the opposite slot of node q
        const int oslot = (sgn < 0) ? 2 + 2 * a : 1 + 2 * a;
        acc += (transpose ? coef[(size_t)oslot * N + qnode] : coef[(size_t)slot * N + node]) * xv;
      } else if (!transpose && g) {
        const size_t bidx = (dim == 2) ? (size_t)q[0] * nb + q[1]
                                       : ((size_t)q[0] * nb + q[1]) * nb + q[2];
        acc += coef[(size_t)slot * N + node] * g[bidx];
      }
    }
  }
  const double fv = f ? f[node] : 0.0;
  r[(size_t)i * ld + ip] = fv - acc;
}

__global__ void k_pad(const double *__restrict__ src, double *__restrict__ dst, int rows, int M,
                      int ld) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rows * ld) return;
  const size_t row = e / ld, c = e % ld;
  dst[e] = (c < (size_t)M) ? src[row * M + c] : 0.0;
}

__global__ void k_unpad(const double *__restrict__ src, double *__restrict__ dst, int rows,
                        int M, int ld) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rows * M) return;
  const size_t row = e / M, c = e % M;
  dst[e] = src[row * ld + c];
}

// rows per wavefront of the GEMV (8 FP32 rows would take all 256 registers:
// the conversions to FP64 are scheduled early)
template <typename T> constexpr int gemv_rpw() { return 4; }
constexpr int kGemvCh = 1024;

// four consecutive matrix entries as doubles (global-memory vector loads)
template <typename T>
__device__ __forceinline__ void ld4(const T *p, double *o) {
  constexpr int V = 16 / sizeof(T);
#pragma unroll
  for (int h = 0; h < 4 / V; ++h) {
    const typename V16<T>::type v = ld16(p + V * h);
#pragma unroll
    for (int e = 0; e < V; ++e) o[V * h + e] = (double)v[e];
  }
}

// out[r] = w[r] + alpha * (G[r,:] (x1 - e.*x2) + G2[r,:] x3); 4 R rows per block.
// HBM-bound: each wavefront owns R rows and, per chunk of
// kGemvCh columns, issues all its 16-byte loads of a matrix before using
// any (4 R per matrix and chunk in flight per wavefront; no branches between
// them: columns past the chunk re-read an in-bounds address and meet x = 0);
// the first matrix's loads are issued before x is staged in LDS, which they
// do not depend on.
template <typename T, int R>
__device__ __forceinline__ void gemv_rows_load(const T *M, size_t row0_off, int ld, int c0,
                                               int cn, int lane, T (&g)[R][kGemvCh / 256][4]) {
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int i = 0; i < kGemvCh / 256; ++i) {
      const int c = lane * 4 + 256 * i;
      const T *src = M + row0_off + (size_t)q * ld + c0 + (c < cn ? c : 0);
      constexpr int V = 16 / sizeof(T);
#pragma unroll
      for (int h = 0; h < 4 / V; ++h) {
        const typename V16<T>::type v = ld16(src + V * h);
#pragma unroll
        for (int e = 0; e < V; ++e) g[q][i][V * h + e] = v[e];
      }
    }
}
// x: kGemvCh doubles in LDS, zero past the chunk
template <typename T, int R>
__device__ __forceinline__ void gemv_rows_fma(const T (&g)[R][kGemvCh / 256][4],
                                              const double *x, int lane, double (&acc)[R]) {
#pragma unroll
  for (int i = 0; i < kGemvCh / 256; ++i) {
    const int c = lane * 4 + 256 * i;
    const double x0 = x[c], x1 = x[c + 1], x2 = x[c + 2], x3 = x[c + 3];
#pragma unroll
    for (int q = 0; q < R; ++q)
      acc[q] += (double)g[q][i][0] * x0 + (double)g[q][i][1] * x1 +
                (double)g[q][i][2] * x2 + (double)g[q][i][3] * x3;
  }
}

template <typename T>
__device__ __forceinline__ void gemv_n_body(const GemvJob *__restrict__ jobs, int ld,
                                            double alpha) {
  constexpr int R = gemv_rpw<T>();
  __shared__ double xs[kGemvCh];
  __shared__ double x3s[kGemvCh];
  const GemvJob J = jobs[blockIdx.y];
  const T *G = static_cast<const T *>(J.G);
  const T *G2 = static_cast<const T *>(J.G2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.x * (4 * R) + wave * R;
  const size_t ro = (size_t)row0 * ld;
  if (!G && !G2) {  // no matrix term (an end of a sweep): out = w
    if (lane < R) {
      const int r = row0 + lane;
      gp(J.out)[r] = J.w ? gp(J.w)[r] : 0.0;
    }
    return;
  }
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0;
  T g[R][kGemvCh / 256][4];
  for (int c0 = 0; c0 < ld; c0 += kGemvCh) {
    const int cn = min(kGemvCh, ld - c0);
    gemv_rows_load<T, R>(G ? G : G2, ro, ld, c0, cn, lane, g);
    if (c0 > 0) __syncthreads();  // the previous chunk's x is no longer read
    for (int c = threadIdx.x; c < kGemvCh; c += 256) {
      double v = 0.0, v3 = 0.0;
      if (c < cn) {
        v = J.x1 ? gp(J.x1)[c0 + c] : 0.0;
        if (J.e) v -= gp(J.e)[c0 + c] * gp(J.x2)[c0 + c];
        v3 = (G2 && J.x3) ? gp(J.x3)[c0 + c] : 0.0;
      }
      xs[c] = v;
      x3s[c] = v3;
    }
    __syncthreads();
    if (G) {
      gemv_rows_fma<T, R>(g, xs, lane, acc);
      if (G2) {
        // keep the second matrix's loads after the first one's products
        // (hoisting them doubles the live registers)
        asm volatile("" ::: "memory");
        gemv_rows_load<T, R>(G2, ro, ld, c0, cn, lane, g);
        gemv_rows_fma<T, R>(g, x3s, lane, acc);
      }
    } else {
      gemv_rows_fma<T, R>(g, x3s, lane, acc);
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) {
      const int r = row0 + q;
      gp(J.out)[r] = (J.w ? gp(J.w)[r] : 0.0) + alpha * s;
    }
  }
}

// FP32 matrices: capped at 3 wavefronts' registers per SIMD (138 VGPRs, no
// spills) for more loads in flight per CU; FP64 keeps the compiler's choice
// (a cap spills).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gemv_n_f32(
    const GemvJob *__restrict__ jobs, int ld, double alpha) {
  gemv_n_body<float>(jobs, ld, alpha);
}
__global__ __launch_bounds__(256) void k_gemv_n_f64(const GemvJob *__restrict__ jobs, int ld,
                                                    double alpha) {
  gemv_n_body<double>(jobs, ld, alpha);
}

// Several right-hand sides per launch, on the matrix cores: vector v of a job
// is the job's vector shifted by v * vs (x1, x2, x3, w and out; the matrices
// and e are shared), up to 16 per launch.  Y = Mat X is a product of the
// matrix rows with a 16-column block of vectors, done by the FP64
// 16 x 16 x 4 MFMA (matrix entries converted exactly to FP64, FP64
// accumulation, as in the one-vector kernel): each wavefront owns a strip
// of 16 rows; per 16-column step lane l loads four
// consecutive entries of row l % 16 (columns 4 (l / 16) + 0..3), which feed
// the A operand of four MFMAs, the i-th taking columns {4 q + i}; the B
// operand is the matching entries of the 16 vectors, staged column-major in
// LDS per chunk of columns (zero for vectors past nv); the next chunk's
// matrix entries are loaded while a chunk is used.  The FP64 output holds
// vector l % 16 of rows 4 r + l / 16 in register r.
typedef double f64x4v __attribute__((ext_vector_type(4)));
constexpr int kMvLd = 17;  // LDS row stride (doubles) of the staged block
// columns staged per chunk: a divisor of every leading dimension (a multiple
// of 128)
constexpr int kMvCh = 128;

template <typename T, int NS>
__device__ __forceinline__ void mv_load(const T *Mt, size_t row_off, int c0, int kq,
                                        T (&a)[NS][4]) {
  constexpr int V = 16 / sizeof(T);
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    const T *src = Mt + row_off + c0 + 16 * st + 4 * kq;
#pragma unroll
    for (int h = 0; h < 4 / V; ++h) {
      const typename V16<T>::type v = ld16(src + V * h);
#pragma unroll
      for (int e = 0; e < V; ++e) a[st][V * h + e] = v[e];
    }
  }
}

// W wavefronts (16-row strips) per work-group: 8 share each staged block of
// x over 128 rows (fewer staging loads per row, better from 8 vectors on),
// 4 give twice the work-groups (better for 2 to 4 vectors).
template <typename T, int W>
__global__ __launch_bounds__(64 * W) void k_gemv_mfma(const GemvJob *__restrict__ jobs, int ld,
                                                      double alpha, int nv, size_t vs) {
  constexpr int CH = kMvCh, NS = CH / 16, RB = 16 * W;
  __shared__ double xt[CH * kMvLd];
  const GemvJob J = jobs[blockIdx.y];
  const T *G = static_cast<const T *>(J.G);
  const T *G2 = static_cast<const T *>(J.G2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int rowb = blockIdx.x * RB;  // first row of the work-group
  const int roww = rowb + wave * 16;  // first row of this wavefront's strip
  if (!G && !G2) {  // no matrix term: out = w
    for (int e = threadIdx.x; e < RB * nv; e += 64 * W) {
      const size_t o = (size_t)(e / RB) * vs + rowb + e % RB;
      gp(J.out)[o] = J.w ? gp(J.w)[o] : 0.0;
    }
    return;
  }
  f64x4v acc = {0.0, 0.0, 0.0, 0.0};
  const size_t row_off = (size_t)(roww + m) * ld;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    const T *Mt = pass == 0 ? G : G2;
    if (!Mt) continue;
    const double *xa = pass == 0 ? J.x1 : J.x3;
    const double *xe = pass == 0 ? J.e : nullptr;
    T a[NS][4], an[NS][4];
    mv_load<T, NS>(Mt, row_off, 0, kq, a);
    for (int c0 = 0; c0 < ld; c0 += CH) {
      // the next chunk's matrix entries go out before this chunk is used
      if (c0 + CH < ld) mv_load<T, NS>(Mt, row_off, c0 + CH, kq, an);
      __syncthreads();  // the previous block of x is no longer read
      for (int idx = threadIdx.x; idx < 16 * CH; idx += 64 * W) {
        const int v = idx / CH, c = idx % CH;
        double x = 0.0;
        if (v < nv) {
          const size_t o = (size_t)v * vs + c0 + c;
          x = xa ? gp(xa)[o] : 0.0;
          if (xe) x -= gp(xe)[c0 + c] * gp(J.x2)[o];
        }
        xt[c * kMvLd + v] = x;
      }
      __syncthreads();
#pragma unroll
      for (int st = 0; st < NS; ++st)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
              (double)a[st][i], xt[(16 * st + 4 * kq + i) * kMvLd + m], acc, 0, 0, 0);
#pragma unroll
      for (int st = 0; st < NS; ++st)
#pragma unroll
        for (int i = 0; i < 4; ++i) a[st][i] = an[st][i];
    }
  }
  if (m < nv) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const size_t o = (size_t)m * vs + roww + 4 * r + kq;
      gp(J.out)[o] = (J.w ? gp(J.w)[o] : 0.0) + alpha * acc[r];
    }
  }
}

// Transposed product, partial sums over row chunks:
// part[(job*nchunk + chunk)*ld + c] = sum_{r in chunk} G[r,c] xe[r] + G2[r,c] x3[r]
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_t_part(const GemvJob *__restrict__ jobs, int ld,
                                                     int rows_per_chunk,
                                                     double *__restrict__ part) {
  extern __shared__ double sh[];
  double *xs = sh;
  double *x3s = sh + rows_per_chunk;
  const int chunk = blockIdx.x, job = blockIdx.y, nchunk = gridDim.x;
  const GemvJob J = jobs[job];
  const T *G = static_cast<const T *>(J.G);
  const T *G2 = static_cast<const T *>(J.G2);
  const int r0 = chunk * rows_per_chunk;
  for (int r = threadIdx.x; r < rows_per_chunk; r += 256) {
    double v = J.x1 ? gp(J.x1)[r0 + r] : 0.0;
    if (J.e) v -= gp(J.e)[r0 + r] * gp(J.x2)[r0 + r];
    xs[r] = v;
    x3s[r] = (G2 && J.x3) ? gp(J.x3)[r0 + r] : 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x * 4; c < ld; c += 1024) {
    double s[4] = {0, 0, 0, 0};
    for (int r = 0; r < rows_per_chunk; ++r) {
      double gv[4];
      const size_t o = (size_t)(r0 + r) * ld + c;
      if (G) {
        ld4<T>(G + o, gv);
        const double xv = xs[r];
        s[0] += gv[0] * xv; s[1] += gv[1] * xv; s[2] += gv[2] * xv; s[3] += gv[3] * xv;
      }
      if (G2) {
        ld4<T>(G2 + o, gv);
        const double xv = x3s[r];
        s[0] += gv[0] * xv; s[1] += gv[1] * xv; s[2] += gv[2] * xv; s[3] += gv[3] * xv;
      }
    }
    double *po = part + ((size_t)job * nchunk + chunk) * ld + c;
    po[0] = s[0]; po[1] = s[1]; po[2] = s[2]; po[3] = s[3];
  }
}

__global__ void k_gemv_t_reduce(const GemvJob *__restrict__ jobs, int ld, int nchunk,
                                const double *__restrict__ part, double alpha) {
  const int job = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ld) return;
  const GemvJob J = jobs[job];
  double s = 0.0;
  for (int k = 0; k < nchunk; ++k) s += part[((size_t)job * nchunk + k) * ld + c];
  gp(J.out)[c] = (J.w ? gp(J.w)[c] : 0.0) + alpha * s;
}

__global__ void k_interface_rhs(const double *__restrict__ vol, const double *__restrict__ Zl,
                                const double *__restrict__ Zr, const double *__restrict__ Ea,
                                const double *__restrict__ Eb, int n_ds, int m, int ld,
                                int a_off, int b_off, double *__restrict__ out) {
  const int j = blockIdx.y + 1;  // interface 1..n_ds
  const int pl = j * m;          // node plane (1-based)
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ld; r += gridDim.x * blockDim.x) {
    const double v = (vol ? vol[(size_t)(pl - 1) * ld + r] : 0.0) -
                     Ea[(size_t)(pl + a_off) * ld + r] * Zl[(size_t)(pl - 2) * ld + r] -
                     Eb[(size_t)(pl + b_off) * ld + r] * Zr[(size_t)pl * ld + r];
    out[(size_t)(j - 1) * ld + r] = v;
  }
}

__global__ void k_copy_planes(const double *__restrict__ src, int src_stride, int src_off,
                              double *__restrict__ dst, int dst_stride, int dst_off, int ld,
                              int M) {
  const int k = blockIdx.y;
  const double *s = src + (size_t)(src_off + (size_t)k * src_stride) * ld;
  double *d = dst + (size_t)(dst_off + (size_t)k * dst_stride) * ld;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < ld; r += gridDim.x * blockDim.x)
    d[r] = (r < M) ? s[r] : 0.0;
}

__global__ void k_axpy(double *__restrict__ y, const double *__restrict__ x, double a,
                       size_t len) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) y[e] += a * x[e];
}

__global__ void k_fill(double *__restrict__ y, double v, size_t len) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) y[e] = v;
}

// Dot products of w with nvec vectors (stride apart), two passes:
// part[chunk][i] = sum over a 256-element chunk (one wavefront per vector,
// the chunk of w staged in LDS), then out[i] = sum over chunks (fixed order,
// deterministic).  A null V means w itself (squared norm).
constexpr int kDotChunk = 256;
constexpr int kDotVecs = 8;  // basis vectors per wavefront and round

// Partial dot products of one kDotChunk chunk (in LDS, zero past the end)
// with V_0..V_{nvec-1} (V null: the chunk with itself), one wavefront per
// vector: part[chunk * nvec + i].
// Each wavefront takes kDotVecs vectors at a time with independent sums,
// their loads issued together (entries past the chunk re-read its last element
// and meet a zero of ws).
template <typename B>
__device__ __forceinline__ void chunk_dots(const B *__restrict__ V, size_t stride,
                                           int nvec, const double *ws, size_t base, int cn,
                                           double *__restrict__ part) {
  constexpr int E = kDotChunk / 64;  // entries per lane
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double wv[E];
#pragma unroll
  for (int t = 0; t < E; ++t) wv[t] = ws[lane + 64 * t];
  if (!V) {  // squared norm of the chunk (nvec == 1): the first wavefront
    if (wave == 0) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < E; ++t) s += wv[t] * wv[t];
      s = wave_sum(s);
      if (lane == 0) part[blockIdx.x] = s;
    }
    return;
  }
  for (int i0 = wave; i0 < nvec; i0 += 4 * kDotVecs) {
    double s[kDotVecs];
#pragma unroll
    for (int u = 0; u < kDotVecs; ++u) s[u] = 0.0;
#pragma unroll
    for (int u = 0; u < kDotVecs; ++u) {
      const int i = i0 + 4 * u;
      if (i < nvec) {
        const B *v = V + (size_t)i * stride + base;
#pragma unroll
        for (int t = 0; t < E; ++t) {
          const int e = lane + 64 * t;
          s[u] += (double)v[e < cn ? e : cn - 1] * wv[t];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kDotVecs; ++u) {
      const int i = i0 + 4 * u;
      const double r = wave_sum(s[u]);
      if (lane == 0 && i < nvec) part[(size_t)blockIdx.x * nvec + i] = r;
    }
  }
}

template <typename B>
__global__ __launch_bounds__(256) void k_multidot_part(const B *__restrict__ V, size_t stride,
                                                       int nvec, const double *__restrict__ w,
                                                       size_t len, double *__restrict__ part) {
  __shared__ double ws[kDotChunk];
  const size_t base = (size_t)blockIdx.x * kDotChunk;
  const int cn = (int)min((size_t)kDotChunk, len - base);
  for (int e = threadIdx.x; e < kDotChunk; e += 256) ws[e] = (e < cn) ? w[base + e] : 0.0;
  __syncthreads();
  chunk_dots(V, stride, nvec, ws, base, cn, part);
}

// One Gram-Schmidt update of a chunk, w += sign * V h, followed by the
// partial dot products of the updated chunk for the next pass (V2 = V,
// nvec2 = nvec) or its partial squared norm (V2 null, nvec2 = 1): the two
// kernels of the classical scheme that touch the same chunk, fused.
template <typename B>
__global__ __launch_bounds__(256) void k_mgs_update_dots(double *__restrict__ w,
                                                         const B *__restrict__ V,
                                                         size_t stride, int nvec,
                                                         const double *__restrict__ h,
                                                         double sign, size_t len,
                                                         const B *__restrict__ V2,
                                                         int nvec2, double *__restrict__ part) {
  __shared__ double ws[kDotChunk];
  const size_t base = (size_t)blockIdx.x * kDotChunk;
  const int cn = (int)min((size_t)kDotChunk, len - base);
  const int e = threadIdx.x;  // kDotChunk == blockDim.x
  double we = 0.0;
  if (e < cn) {
    // eight independent partial sums: eight basis-vector loads in flight
    const B *v = V + base + e;
    double t[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 8 <= nvec; i += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] += (double)v[(size_t)(i + u) * stride] * h[i + u];
    for (; i < nvec; ++i) t[0] += (double)v[(size_t)i * stride] * h[i];
    const double sum = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    we = w[base + e] + sign * sum;
    w[base + e] = we;
  }
  ws[e] = we;
  __syncthreads();
  chunk_dots(V2, stride, nvec2, ws, base, cn, part);
}

// Column j of H, staged in LDS cl[0..j+1] (cl[j+1] = hn, the subdiagonal
// entry), is rotated by the j previous Givens rotations (cs, sn staged in
// LDS), a new rotation zeroes its subdiagonal entry and is applied to g;
// writes column j of d.H, the rotation, g and res[2j], res[2j+1].  All 256
// threads of the work-group.  The rotations form the recurrence
//   a_0 = c_0,  a_{i+1} = -sn_i a_i + cs_i c_{i+1},  c_i <- cs_i a_i + sn_i c_{i+1}
// (c_j <- a_j before the new rotation): a first-order linear recurrence,
// evaluated as a parallel prefix of affine maps x -> m x + b (each thread
// composes the maps of a contiguous segment, the work-group scans the 256
// segment maps, then each thread replays its segment from its prefix), so
// the column costs O(j / 256 + log 256) steps instead of a serial chain of
// j rotations.
constexpr int kGivensLds = 2048;
__device__ __forceinline__ void givens_column_lds(double *cl, const double *cs,
                                                  const double *sn, int j, GmresDev d,
                                                  double beta, double hn) {
  __shared__ double sm[256], sb[256], co[kGivensLds + 1];
  __shared__ double aj;
  const int t = threadIdx.x;
  const int seg = (j + 255) / 256;
  const int i0 = min(t * seg, j), i1 = min(i0 + seg, j);
  double m = 1.0, b = 0.0;
  for (int i = i0; i < i1; ++i) {  // compose T_i after the segment so far
    const double mi = -sn[i], bi = cs[i] * cl[i + 1];
    b = mi * b + bi;
    m = mi * m;
  }
  sm[t] = m;
  sb[t] = b;
  __syncthreads();
  // inclusive scan over threads: P_t = S_t o ... o S_0
  for (int off = 1; off < 256; off <<= 1) {
    double pm = 1.0, pb = 0.0;
    const bool has = t >= off;
    if (has) {
      pm = sm[t - off];
      pb = sb[t - off];
    }
    __syncthreads();
    if (has) {  // (S_t o P_{t-off}): m = m_t pm, b = m_t pb + b_t
      const double mt = sm[t], bt = sb[t];
      sm[t] = mt * pm;
      sb[t] = mt * pb + bt;
    }
    __syncthreads();
  }
  // a at the start of this thread's segment: exclusive prefix applied to c_0
  double a = cl[0];
  if (t > 0) a = sm[t - 1] * cl[0] + sb[t - 1];
  for (int i = i0; i < i1; ++i) {
    const double bnext = cl[i + 1];
    co[i] = cs[i] * a + sn[i] * bnext;
    a = -sn[i] * a + cs[i] * bnext;
  }
  if (i1 == j && i0 < i1) aj = a;  // the thread that took the last step
  if (j == 0 && t == 0) aj = cl[0];
  __syncthreads();
  double *col = d.H + gmres_hoff(j);
  for (int i = t; i < j; i += 256) col[i] = co[i];
  if (t == 0) {
    const double av = aj;
    const double r = hypot(av, hn);
    const double ck = r > 0.0 ? av / r : 1.0;
    const double sk = r > 0.0 ? hn / r : 0.0;
    d.cs[j] = ck;
    d.sn[j] = sk;
    col[j] = r;
    col[j + 1] = 0.0;
    const double gk = j == 0 ? beta : d.g[j];
    d.g[j + 1] = -sk * gk;
    d.g[j] = ck * gk;
    d.res[2 * j] = fabs(d.g[j + 1]) / beta;
    d.res[2 * j + 1] = (hn > 0.0 && isfinite(hn)) ? 0.0 : 1.0;
  }
}

// The same for a column too long for LDS (j + 2 > kGivensLds): thread 0 runs
// the rotations serially on the column in global memory.
__device__ __forceinline__ void givens_column_global(double *col, int j, GmresDev d,
                                                     double beta, double hn) {
  if (threadIdx.x == 0) {
    col[j + 1] = hn;
    double a = col[0];
    for (int i = 0; i < j; ++i) {
      const double bnext = col[i + 1];
      col[i] = d.cs[i] * a + d.sn[i] * bnext;
      a = -d.sn[i] * a + d.cs[i] * bnext;
    }
    const double r = hypot(a, hn);
    const double ck = r > 0.0 ? a / r : 1.0;
    const double sk = r > 0.0 ? hn / r : 0.0;
    d.cs[j] = ck;
    d.sn[j] = sk;
    col[j] = r;
    col[j + 1] = 0.0;
    const double gk = j == 0 ? beta : d.g[j];
    d.g[j + 1] = -sk * gk;
    d.g[j] = ck * gk;
    d.res[2 * j] = fabs(d.g[j + 1]) / beta;
    d.res[2 * j + 1] = (hn > 0.0 && isfinite(hn)) ? 0.0 : 1.0;
  }
}

// Column k of H from the two classical Gram-Schmidt passes (hd[0..k] +
// hd[k+1..2k+1], new norm hn): kept unrotated in d.Hraw (for a later lagged
// step, which multiplies by H), then rotated.  All threads of one work-group.
__device__ __forceinline__ void gmres_givens_block(const double *__restrict__ hd, GmresDev d,
                                                   int k, double beta, double hn) {
  __shared__ double cl[kGivensLds + 2], cs[kGivensLds], sn[kGivensLds];
  for (int i = threadIdx.x; i <= k + 1; i += blockDim.x) {
    const double v = i <= k ? hd[i] + hd[k + 1 + i] : hn;
    d.Hraw[gmres_rix(i, k, d.maxit)] = v;
    if (k + 2 <= kGivensLds) {
      cl[i] = v;
      if (i < k) {
        cs[i] = d.cs[i];
        sn[i] = d.sn[i];
      }
    } else {
      d.H[gmres_hoff(k) + i] = v;
    }
  }
  __syncthreads();
  if (k + 2 <= kGivensLds)
    givens_column_lds(cl, cs, sn, k, d, beta, hn);
  else
    givens_column_global(d.H + gmres_hoff(k), k, d, beta, hn);
}

// Column j of H from d.Hraw (rows 0..j+1), rotated (the lagged steps).
__device__ __forceinline__ void gmres_givens_raw(GmresDev d, int j, double beta) {
  __shared__ double cl[kGivensLds + 2], cs[kGivensLds], sn[kGivensLds];
  const double hn = d.Hraw[gmres_rix(j + 1, j, d.maxit)];
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) {
    const double v = d.Hraw[gmres_rix(i, j, d.maxit)];
    if (j + 2 <= kGivensLds) {
      cl[i] = v;
      if (i < j) {
        cs[i] = d.cs[i];
        sn[i] = d.sn[i];
      }
    } else {
      d.H[gmres_hoff(j) + i] = v;
    }
  }
  __syncthreads();
  if (j + 2 <= kGivensLds)
    givens_column_lds(cl, cs, sn, j, d, beta, hn);
  else
    givens_column_global(d.H + gmres_hoff(j), j, d, beta, hn);
}

// Last kernel of Arnoldi step k: dst = src / sqrt(sum of the nchunk partial
// squared norms) (and its FP32 rounding in slot, if given), every
// work-group summing the partials in the same order; the first one stores
// the norm in hd and then applies the Givens rotations (column k of H from
// hd), concurrently with the others' scaling.
__global__ __launch_bounds__(256) void k_norm_scale_givens(const double *__restrict__ part,
                                                           int nchunk, double *__restrict__ hd,
                                                           const double *__restrict__ src,
                                                           double *__restrict__ dst,
                                                           float *__restrict__ slot, size_t len,
                                                           GmresDev gd, int k, double beta) {
  __shared__ double sh[1];
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += 64) s += part[c];
    s = wave_sum(s);
    if (threadIdx.x == 0) {
      const double d = sqrt(s);
      sh[0] = d;
      if (blockIdx.x == 0) hd[2 * (k + 1)] = d;
    }
  }
  __syncthreads();
  const double d = sh[0];
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) {
    const double v = (d > 0.0) ? src[e] / d : 0.0;
    dst[e] = v;
    if (slot) slot[e] = (float)v;
  }
  if (blockIdx.x == 0) gmres_givens_block(hd, gd, k, beta, d);
}

// ---- Arnoldi with lagged reorthogonalization (see launch_arnoldi_lagged) --

// Pass A: partial dot products of the m - 1 basis vectors Q (V, stride) and
// of the candidate u with u and with w (null: only those with u), per
// kLagChunk-element chunk: part[chunk][i] = V_i . u, part[chunk][m + i] =
// V_i . w (i < m - 1), part[chunk][m - 1] = u . u, part[chunk][2 m - 1] =
// u . w.  Work-group (chunk, g) takes the chunk of u and w (in LDS) and the
// kLagGroup basis vectors g kLagGroup ..: each wavefront 8 of them, four at
// a time with their loads issued together, 32 entries per lane and vector
// before one reduction per product; group 0 also forms the products of u.
constexpr int kLagChunk = 2048, kLagGroup = 32;
template <typename B>
__global__ __launch_bounds__(256) void k_lag_dots(const B *__restrict__ V, size_t stride, int m,
                                                  const double *__restrict__ u,
                                                  const double *__restrict__ w, size_t len,
                                                  double *__restrict__ part) {
  constexpr int E = kLagChunk / 64;  // entries per lane and vector
  __shared__ double us[kLagChunk], zs[kLagChunk];
  const size_t base = (size_t)blockIdx.x * kLagChunk;
  const int cn = (int)min((size_t)kLagChunk, len - base);
  for (int e = threadIdx.x; e < kLagChunk; e += 256) {
    us[e] = e < cn ? u[base + e] : 0.0;
    zs[e] = (w && e < cn) ? w[base + e] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double *pc = part + (size_t)blockIdx.x * 2 * m;
  if (blockIdx.y == 0 && wave == 0) {
    double su = 0.0, sz = 0.0;
    for (int t = 0; t < E; ++t) {
      const double x = us[lane + 64 * t];
      su += x * x;
      sz += x * zs[lane + 64 * t];
    }
    su = wave_sum(su);
    sz = wave_sum(sz);
    if (lane == 0) {
      pc[m - 1] = su;
      pc[2 * m - 1] = sz;
    }
  }
  const int nq = m - 1;
  const int i0 = blockIdx.y * kLagGroup + wave;
#pragma unroll 1
  for (int h = 0; h < kLagGroup / 4; h += 4) {
    // vectors i0 + 4 (h + q), q < 4
    double su[4] = {0.0, 0.0, 0.0, 0.0}, sz[4] = {0.0, 0.0, 0.0, 0.0};
    const B *v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = min(i0 + 4 * (h + q), max(nq - 1, 0));
      v[q] = V + (size_t)i * stride + base;
    }
    if (i0 + 4 * h < nq) {
#pragma unroll 4
      for (int t = 0; t < E; ++t) {
        const int e = lane + 64 * t;
        const int el = e < cn ? e : cn - 1;
        const double a = us[e], c = zs[e];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double x = (double)v[q][el];
          su[q] += x * a;
          sz[q] += x * c;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + 4 * (h + q);
      const double ru = wave_sum(su[q]), rz = wave_sum(sz[q]);
      if (lane == 0 && i < nq) {
        pc[i] = ru;
        pc[m + i] = rz;
      }
    }
  }
}

// nu = |u - Q a| = sqrt(|u|^2 - |a|^2) from the pass-A products (every
// thread of the work-group gets it).
__device__ __forceinline__ double lag_nu(const GmresDev &d, int k) {
  __shared__ double sh[4], snu;
  double t = 0.0;
  for (int i = threadIdx.x; i < k; i += 256) t += d.dA[i] * d.dA[i];
  t = block_sum(t, sh);
  if (threadIdx.x == 0) {
    const double nu2 = d.dA[k] - t;
    snu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
  }
  __syncthreads();
  return snu;
}

// d = H a over rows 0..k (one wavefront per row, four rows per work-group),
// with column k - 1 taken as finalized now (unless col_final: it is in
// Hraw already): prov + rho a above the diagonal, rho nu below it; work-group
// 0 stores that column in Hraw.
__global__ __launch_bounds__(256) void k_lag_hmul(GmresDev d, int k, int col_final) {
  const double nu = lag_nu(d, k);
  const double *a = d.dA;
  const double rho = d.sc[2];
  const bool fin = k >= 1 && !col_final;
  auto lastcol = [&](int i) { return i < k ? d.prov[i] + rho * a[i] : rho * nu; };
  if (blockIdx.x == 0 && fin)
    for (int i = threadIdx.x; i <= k; i += 256) d.Hraw[gmres_rix(i, k - 1, d.maxit)] = lastcol(i);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blockIdx.x * 4 + wave;
  if (r > k) return;
  const int j0 = r > 0 ? r - 1 : 0;
  const int jend = fin ? k - 1 : k;  // stored columns [j0, jend)
  const double *row = d.Hraw + gmres_roff(r, d.maxit) - j0;
  double acc = 0.0;
  for (int j = j0 + lane; j < jend; j += 64) acc += row[j] * a[j];
  acc = wave_sum(acc);
  if (lane == 0) d.dv[r] = acc + (fin ? lastcol(r) * a[k - 1] : 0.0);
}

// Coefficients of pass B (one work-group): with d = dv, b = Q^T w, gamma =
// u.w, the provisional column h_i = (b_i - d_i) / nu (i < k), h_k =
// ((gamma - a.b) / nu - d_k) / nu; e = d / nu + h; pass B forms
// z = w / nu - Q f - g u with f = e[0:k] - e_k a / nu, g = e_k / nu.
__global__ __launch_bounds__(256) void k_lag_coef(GmresDev d, int k) {
  __shared__ double sh[4], sek;
  const double nu = lag_nu(d, k);
  const int m = k + 1;
  const double *a = d.dA, *b = d.dA + m;
  double t = 0.0;
  for (int i = threadIdx.x; i < k; i += 256) t += a[i] * b[i];
  t = block_sum(t, sh);
  const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
  if (threadIdx.x == 0) {
    const double hk = ((b[k] - t) * inv - d.dv[k]) * inv;
    d.prov[k] = hk;
    sek = d.dv[k] * inv + hk;
    d.sc[0] = inv;
    d.sc[1] = sek * inv;
  }
  __syncthreads();
  const double ek = sek;
  for (int i = threadIdx.x; i < k; i += 256) {
    const double h = (b[i] - d.dv[i]) * inv;
    d.prov[i] = h;
    d.cf[i] = d.dv[i] * inv + h - ek * a[i] * inv;
  }
}

// Pass B, per 256-element chunk: q_k = (u - Q a) / nu into slot k of V, w =
// w / nu - Q f - g u, and the chunk's partial squared norm of the new w.
// u may be slot k itself (an FP64 basis): each element is read before it is
// overwritten, by the same thread.
template <typename B>
__global__ __launch_bounds__(256) void k_lag_update(B *V, size_t stride, int k, const double *u,
                                                    double *__restrict__ w, size_t len,
                                                    GmresDev d, double *__restrict__ part) {
  __shared__ double sh[4];
  const size_t e = (size_t)blockIdx.x * kDotChunk + threadIdx.x;
  double zn = 0.0;
  if (e < len) {
    const double *a = d.dA, *f = d.cf;
    const B *v = V + e;
    double ta[8] = {0, 0, 0, 0, 0, 0, 0, 0}, tf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = 0;
    for (; i + 8 <= k; i += 8)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double x = (double)v[(size_t)(i + q) * stride];
        ta[q] += x * a[i + q];
        tf[q] += x * f[i + q];
      }
    for (; i < k; ++i) {
      const double x = (double)v[(size_t)i * stride];
      ta[0] += x * a[i];
      tf[0] += x * f[i];
    }
    const double sa = ((ta[0] + ta[1]) + (ta[2] + ta[3])) + ((ta[4] + ta[5]) + (ta[6] + ta[7]));
    const double sf = ((tf[0] + tf[1]) + (tf[2] + tf[3])) + ((tf[4] + tf[5]) + (tf[6] + tf[7]));
    const double inv = d.sc[0], g = d.sc[1];
    const double ue = u[e];
    V[(size_t)k * stride + e] = (B)((ue - sa) * inv);
    zn = w[e] * inv - sf - g * ue;
    w[e] = zn;
  }
  const double s = block_sum(zn * zn, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// rho = |w| (every work-group sums the partials in the same order; the
// first stores it), vnext = w / rho, and work-group 0 rotates column
// givens_col of H (< 0: none) from Hraw, beside the others' scaling.
__global__ __launch_bounds__(256) void k_lag_norm_scale(const double *__restrict__ part, int nchunk,
                                                        const double *__restrict__ w,
                                                        double *__restrict__ vnext, size_t len,
                                                        GmresDev d, int givens_col, double beta) {
  __shared__ double sh[1];
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += 64) s += part[c];
    s = wave_sum(s);
    if (threadIdx.x == 0) {
      const double r = sqrt(s);
      sh[0] = r;
      if (blockIdx.x == 0 && len > 0) d.sc[2] = r;
    }
  }
  __syncthreads();
  const double r = sh[0];
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) vnext[e] = (r > 0.0) ? w[e] / r : 0.0;
  if (blockIdx.x == 0 && givens_col >= 0) gmres_givens_raw(d, givens_col, beta);
}

// One work-group per vector sums its partials (strided, then a tree).
__global__ __launch_bounds__(256) void k_multidot_reduce(const double *__restrict__ part,
                                                         int nchunk, int nvec,
                                                         double *__restrict__ out,
                                                         int take_sqrt) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) s += part[(size_t)c * nvec + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[i] = take_sqrt ? sqrt(s) : s;
}

template <typename B>
__global__ void k_mgs_update(double *__restrict__ w, const B *__restrict__ V, size_t stride,
                             int nvec, const double *__restrict__ h, double sign, size_t len) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int i = 0; i < nvec; ++i) s += (double)V[(size_t)i * stride + e] * h[i];
  w[e] += sign * s;
}

__global__ void k_to_float(float *__restrict__ dst, const double *__restrict__ src, size_t len) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) dst[e] = (float)src[e];
}

__global__ void k_scale_by_inv(double *__restrict__ dst, const double *__restrict__ src,
                               const double *__restrict__ nrm, size_t len) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) {
    const double d = nrm[0];
    dst[e] = (d > 0.0) ? src[e] / d : 0.0;
  }
}

// dL/dkappa on cells: -1/(2^(d-1) h^2) sum_edges (lam_p - lam_q)(u_p - u_q).
__global__ void k_cell_gradient(const double *__restrict__ u, const double *__restrict__ lam,
                                const double *__restrict__ g, int dim, int n, int M, int ld,
                                double h, double *__restrict__ grad) {
  const size_t nc = (size_t)n + 1;
  const size_t ncell = (dim == 2) ? nc * nc : nc * nc * nc;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= ncell) return;
  int c[3];
  if (dim == 2) {
    c[0] = (int)(cell / nc); c[1] = (int)(cell % nc); c[2] = 0;
  } else {
    c[0] = (int)(cell / (nc * nc)); c[1] = (int)((cell / nc) % nc); c[2] = (int)(cell % nc);
  }
  const size_t nb = (size_t)n + 2;
  // corner values of the cell: node c + o, o in {0,1}^dim
  double U[8], L[8];
  const int ncorner = 1 << dim;
  for (int o = 0; o < ncorner; ++o) {
    int q[3] = {c[0] + (o & 1), c[1] + ((o >> 1) & 1), dim == 3 ? c[2] + ((o >> 2) & 1) : 0};
    bool inside = true;
    for (int a = 0; a < dim; ++a) inside = inside && q[a] >= 1 && q[a] <= n;
    if (inside) {
      const size_t ip = (dim == 2) ? (size_t)(q[1] - 1) : (size_t)(q[1] - 1) * n + (q[2] - 1);
      U[o] = u[(size_t)(q[0] - 1) * M + ip];
      L[o] = lam[(size_t)(q[0] - 1) * ld + ip];
    } else {
      const size_t bidx = (dim == 2) ? (size_t)q[0] * nb + q[1]
                                     : ((size_t)q[0] * nb + q[1]) * nb + q[2];
      U[o] = g ? g[bidx] : 0.0;
      L[o] = 0.0;
    }
  }
  double s = 0.0;
  for (int o = 0; o < ncorner; ++o)
    for (int a = 0; a < dim; ++a)
      if (!((o >> a) & 1)) {
        const int o2 = o | (1 << a);
        s += (L[o] - L[o2]) * (U[o] - U[o2]);
      }
  grad[cell] = -s / ((double)(1 << (dim - 1)) * h * h);
}

__global__ void k_check_finite(const double *__restrict__ x, size_t len, double lo, int *bad) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < len) {
    const double v = x[e];
    if (!isfinite(v) || !(v > lo)) atomicOr(bad, 1);
  }
}

// Largest |x_e| into *out (bit pattern of a non-negative double, which
// orders like an unsigned integer; NaN entries are skipped).
__global__ void k_maxabs(const double *__restrict__ x, size_t len,
                         unsigned long long *__restrict__ out) {
  double v = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len;
       e += (size_t)gridDim.x * blockDim.x)
    v = fmax(v, fabs(x[e]));
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

inline unsigned nblk(size_t len, unsigned b = 256) { return (unsigned)((len + b - 1) / b); }

}  // namespace

void launch_setup_coef(const double *kappa, const double *c, const double *b, int dim, int n,
                       double h, double *coef, int *, hipStream_t s) {
  const size_t N = (dim == 2) ? (size_t)n * n : (size_t)n * n * n;
  hipLaunchKernelGGL(k_setup_coef, dim3(nblk(N)), dim3(256), 0, s, kappa, c, b[0], b[1], b[2],
                     dim, n, h, coef);
}

void launch_fill_couplings(const double *coef, int dim, int n, int M, int ld, double *Em,
                           double *Ep, hipStream_t s) {
  const size_t N = (size_t)M * n;
  hipLaunchKernelGGL(k_fill_couplings, dim3(nblk(ld), n + 2), dim3(256), 0, s, coef, n, M, ld,
                     N, Em, Ep);
  (void)dim;
}

void launch_residual(const double *coef, int dim, int n, int M, int ld, const double *f,
                     const double *g, const double *x, double *r, int transpose,
                     hipStream_t s) {
  const size_t N = (size_t)M * n;
  hipLaunchKernelGGL(k_residual, dim3(nblk(N)), dim3(256), 0, s, coef, dim, n, M, ld, f, g, x,
                     r, transpose);
}

void launch_pad(const double *src, double *dst, int rows, int M, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_pad, dim3(nblk((size_t)rows * ld)), dim3(256), 0, s, src, dst, rows, M,
                     ld);
}

void launch_unpad(const double *src, double *dst, int rows, int M, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_unpad, dim3(nblk((size_t)rows * M)), dim3(256), 0, s, src, dst, rows, M,
                     ld);
}

template <typename T>
void launch_gemv(const GemvJob *jobs, int njobs, int ld, int M, int transpose, double alpha,
                 double *partial, hipStream_t s) {
  (void)M;
  if (njobs <= 0) return;
  const ProfSpan ps = prof_open(KK_GEMV);
  if (!transpose) {
    auto kern = sizeof(T) == 4 ? k_gemv_n_f32 : k_gemv_n_f64;
    hipExtLaunchKernelGGL(kern, dim3(ld / (4 * gemv_rpw<T>()), njobs), dim3(256), 0, s, ps.a,
                          ps.b, 0, jobs, ld, alpha);
  } else {
    const int nchunk = (ld / kGemvChunk <= 64) ? ld / kGemvChunk : 64;
    const int rpc = ld / nchunk;
    hipExtLaunchKernelGGL(k_gemv_t_part<T>, dim3(nchunk, njobs), dim3(256),
                          2 * rpc * sizeof(double), s, ps.a, nullptr, 0, jobs, ld, rpc, partial);
    hipExtLaunchKernelGGL(k_gemv_t_reduce, dim3(nblk(ld), njobs), dim3(256), 0, s, nullptr, ps.b,
                          0, jobs, ld, nchunk, partial, alpha);
  }
  // matrix bytes dominate: one or two M x M matrices per job (upper bound 1)
  prof_close(ps, KK_GEMV, (double)njobs * M * M * sizeof(T));
}
template <typename T>
void launch_gemv_many(const GemvJob *jobs, int njobs, int ld, int M, double alpha, int nv,
                      size_t vs, double *partial, hipStream_t s) {
  if (nv <= 1) {
    launch_gemv<T>(jobs, njobs, ld, M, 0, alpha, partial, s);
    return;
  }
  if (njobs <= 0) return;
  // one launch takes up to 16 vectors (the most ddst_solve_many allows)
  if (nv > 16) throw std::invalid_argument("launch_gemv_many: more than 16 vectors");
  const ProfSpan ps = prof_open(KK_GEMV_MANY);
  // 64 or 128 rows per work-group (ld % 128 == 0: whole work-groups and chunks)
  if (nv <= 4)
    hipExtLaunchKernelGGL(k_gemv_mfma<T, 4>, dim3(ld / 64, njobs), dim3(256), 0, s, ps.a, ps.b,
                          0, jobs, ld, alpha, nv, vs);
  else
    hipExtLaunchKernelGGL(k_gemv_mfma<T, 8>, dim3(ld / 128, njobs), dim3(512), 0, s, ps.a, ps.b,
                          0, jobs, ld, alpha, nv, vs);
  // one M x M matrix per job (interface jobs read two: a lower bound)
  prof_close(ps, KK_GEMV_MANY, (double)njobs * M * M * sizeof(T));
}
template void launch_gemv_many<float>(const GemvJob *, int, int, int, double, int, size_t,
                                      double *, hipStream_t);
template void launch_gemv_many<double>(const GemvJob *, int, int, int, double, int, size_t,
                                       double *, hipStream_t);
template void launch_gemv<float>(const GemvJob *, int, int, int, int, double, double *,
                                 hipStream_t);
template void launch_gemv<double>(const GemvJob *, int, int, int, int, double, double *,
                                  hipStream_t);

void launch_interface_rhs(const double *vol, const double *Zl, const double *Zr,
                          const double *Ea, const double *Eb, int n_ds, int m, int ld,
                          int a_off, int b_off, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_interface_rhs, dim3(nblk(ld), n_ds), dim3(256), 0, s, vol, Zl, Zr, Ea,
                     Eb, n_ds, m, ld, a_off, b_off, out);
}

void launch_copy_planes(const double *src, int src_stride, int src_off, double *dst,
                        int dst_stride, int dst_off, int count, int ld, int M, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_copy_planes, dim3(nblk(ld), count), dim3(256), 0, s, src, src_stride,
                     src_off, dst, dst_stride, dst_off, ld, M);
}

void launch_axpy(double *y, const double *x, double a, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(nblk(len)), dim3(256), 0, s, y, x, a, len);
}

void launch_fill(double *y, double v, size_t len, hipStream_t s) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblk(len)), dim3(256), 0, s, y, v, len);
}

template <typename B>
void launch_mgs_update(double *w, const B *V, size_t stride, int nvec, const double *h,
                       double sign, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_update<B>, dim3(nblk(len)), dim3(256), 0, s, w, V, stride, nvec, h,
                     sign, len);
}
template void launch_mgs_update<double>(double *, const double *, size_t, int, const double *,
                                        double, size_t, hipStream_t);
template void launch_mgs_update<float>(double *, const float *, size_t, int, const double *,
                                       double, size_t, hipStream_t);

void launch_to_float(float *dst, const double *src, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_to_float, dim3(nblk(len)), dim3(256), 0, s, dst, src, len);
}

template <typename B>
void launch_arnoldi_step(const B *V, size_t stride, int k, double *w, size_t len, double *hd,
                         double *vnext, float *vslot, double *part, GmresDev gd, double beta,
                         hipStream_t s) {
  const int nvec = k + 1;
  const int nchunk = (int)((len + kDotChunk - 1) / kDotChunk);
  static_assert(kDotChunk == 256, "one element per thread in the fused update");
  // pass 1: h1 = V^T w
  hipLaunchKernelGGL(k_multidot_part<B>, dim3(nchunk), dim3(256), 0, s, V, stride, nvec,
                     (const double *)w, len, part);
  hipLaunchKernelGGL(k_multidot_reduce, dim3(nvec), dim3(256), 0, s, (const double *)part,
                     nchunk, nvec, hd, 0);
  // w -= V h1, then pass 2 partials
  hipLaunchKernelGGL(k_mgs_update_dots<B>, dim3(nchunk), dim3(256), 0, s, w, V, stride, nvec,
                     (const double *)hd, -1.0, len, V, nvec, part);
  hipLaunchKernelGGL(k_multidot_reduce, dim3(nvec), dim3(256), 0, s, (const double *)part,
                     nchunk, nvec, hd + nvec, 0);
  // w -= V h2, then partial squared norms; v_next = w / |w| and the rotations
  hipLaunchKernelGGL(k_mgs_update_dots<B>, dim3(nchunk), dim3(256), 0, s, w, V, stride, nvec,
                     (const double *)(hd + nvec), -1.0, len, (const B *)nullptr, 1, part);
  hipLaunchKernelGGL(k_norm_scale_givens, dim3(nblk(len)), dim3(256), 0, s,
                     (const double *)part, nchunk, hd, (const double *)w, vnext, vslot, len, gd,
                     k, beta);
}
template void launch_arnoldi_step<double>(const double *, size_t, int, double *, size_t,
                                          double *, double *, float *, double *, GmresDev,
                                          double, hipStream_t);
template void launch_arnoldi_step<float>(const float *, size_t, int, double *, size_t, double *,
                                         double *, float *, double *, GmresDev, double,
                                         hipStream_t);

template <typename B>
void launch_arnoldi_lagged(B *V, size_t stride, int k, const double *u, double *w,
                           double *unext, size_t len, double *part, GmresDev gd, double beta,
                           int col_final, int finalize_only, hipStream_t s) {
  const int m = k + 1;
  const int nchunk = (int)((len + kDotChunk - 1) / kDotChunk);
  static_assert(kDotChunk == 256, "one element per thread in pass B");
  const int nlchunk = (int)((len + kLagChunk - 1) / kLagChunk);
  const int ngroup = std::max((m - 1 + kLagGroup - 1) / kLagGroup, 1);
  hipLaunchKernelGGL(k_lag_dots<B>, dim3(nlchunk, ngroup), dim3(256), 0, s, (const B *)V, stride,
                     m, u, finalize_only ? (const double *)nullptr : (const double *)w, len, part);
  hipLaunchKernelGGL(k_multidot_reduce, dim3(2 * m), dim3(256), 0, s, (const double *)part,
                     nlchunk, 2 * m, gd.dA, 0);
  hipLaunchKernelGGL(k_lag_hmul, dim3((m + 3) / 4), dim3(256), 0, s, gd, k, col_final);
  const int gcol = (k >= 1 && !col_final) ? k - 1 : -1;
  if (finalize_only) {
    hipLaunchKernelGGL(k_lag_norm_scale, dim3(1), dim3(256), 0, s, (const double *)part, 0,
                       (const double *)nullptr, (double *)nullptr, (size_t)0, gd, gcol, beta);
    return;
  }
  hipLaunchKernelGGL(k_lag_coef, dim3(1), dim3(256), 0, s, gd, k);
  hipLaunchKernelGGL(k_lag_update<B>, dim3(nchunk), dim3(256), 0, s, V, stride, k, u, w, len, gd,
                     part);
  hipLaunchKernelGGL(k_lag_norm_scale, dim3(nblk(len)), dim3(256), 0, s, (const double *)part,
                     nchunk, (const double *)w, unext, len, gd, gcol, beta);
}
template void launch_arnoldi_lagged<double>(double *, size_t, int, const double *, double *,
                                            double *, size_t, double *, GmresDev, double, int,
                                            int, hipStream_t);
template void launch_arnoldi_lagged<float>(float *, size_t, int, const double *, double *,
                                           double *, size_t, double *, GmresDev, double, int,
                                           int, hipStream_t);

void launch_norm(const double *w, size_t len, double *out, double *part, hipStream_t s) {
  const int nchunk = (int)((len + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(k_multidot_part<double>, dim3(nchunk), dim3(256), 0, s,
                     (const double *)nullptr, (size_t)0, 1, w, len, part);
  hipLaunchKernelGGL(k_multidot_reduce, dim3(1), dim3(256), 0, s, part, nchunk, 1, out, 1);
}

namespace {
// Back substitution R y = g, column by column: y_j is fixed, then every
// thread removes its contribution from rows i < j.
__global__ __launch_bounds__(256) void k_gmres_backsub(GmresDev d, int k) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) d.y[i] = d.g[i];
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double *col = d.H + gmres_hoff(j);
    const double yj = col[j] != 0.0 ? d.y[j] / col[j] : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) d.y[j] = yj;
    for (int i = threadIdx.x; i < j; i += blockDim.x) d.y[i] -= col[i] * yj;
    __syncthreads();
  }
}
}  // namespace


template <typename B>
void launch_gmres_solution(GmresDev d, int k, double *x, const B *V, size_t len, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_gmres_backsub, dim3(1), dim3(256), 0, s, d, k);
  launch_mgs_update<B>(x, V, len, k, d.y, 1.0, len, s);
}
template void launch_gmres_solution<double>(GmresDev, int, double *, const double *, size_t,
                                            hipStream_t);
template void launch_gmres_solution<float>(GmresDev, int, double *, const float *, size_t,
                                           hipStream_t);

void launch_scale_by_inv(double *dst, const double *src, const double *nrm, size_t len,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by_inv, dim3(nblk(len)), dim3(256), 0, s, dst, src, nrm, len);
}

void launch_cell_gradient(const double *u, const double *lam, const double *g, int dim, int n,
                          int M, int ld, double h, double *grad, hipStream_t s) {
  const size_t nc = (size_t)n + 1;
  const size_t ncell = (dim == 2) ? nc * nc : nc * nc * nc;
  hipLaunchKernelGGL(k_cell_gradient, dim3(nblk(ncell)), dim3(256), 0, s, u, lam, g, dim, n, M,
                     ld, h, grad);
}

void launch_maxabs(const double *x, size_t len, unsigned long long *out, hipStream_t s) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_maxabs, dim3(std::min<unsigned>(nblk(len), 1024)), dim3(256), 0, s, x, len,
                     out);
}

void launch_check_finite(const double *x, size_t len, double lo, int *bad, hipStream_t s) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_check_finite, dim3(nblk(len)), dim3(256), 0, s, x, len, lo, bad);
}

}  // namespace ddst
