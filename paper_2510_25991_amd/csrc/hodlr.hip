// Compressed form of the transfer blocks: weak-admissibility hierarchical
// low-rank (HODLR) representation on a cluster tree shared by source and
// target interface (the rank-structured format of the paper's Section 2.4;
// every interaction between two distinct children of a tree node is low
// rank, leaf diagonal blocks stay dense).
//
// Compression of one admissible block B (m x n), batched over all blocks of
// one tree level of every transfer block:
//   1. Omega (n x s) Gaussian, s = rank cap + oversampling (Philox-4x32-10
//      counter generator + Box-Muller), Y = B Omega                 (GEMM)
//   2. Householder QR of Y, explicit Q (m x s)                     (FP64)
//   3. X = B^T Q (n x s), so that B ~ Q X^T                         (GEMM)
//   4. Householder QR X = Q2 R (R s x s), one-sided Jacobi on the columns
//      of R: R V = Rt with orthogonal columns, sigma_k = |Rt_k|, and
//      Xt = X V = Q2 Rt (the rotations run on s rows instead of n)
//   5. keep sigma_k > tol * ||S_{j,j'}||_2 (norm by power iteration):
//      U = Q V_sel (m x r), Vt = Xt_sel^T (r x n), packed in BF16/FP32/FP64.
// Apply: one work-group per (interface, row cluster) at each level sums all
// contributions of that cluster (both transfer blocks, all siblings), so no
// two work-groups write the same output entries.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <tuple>
#include <type_traits>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"

namespace ddst {

// ---------------------------------------------------------------- host data
struct HBlock {
  int smat;        // transfer matrix index: 2*(j-1) + 0 for S_{j,j-1}, +1 for S_{j,j+1}
  int r0, r1;      // row range (cluster-ordered indices)
  int c0, c1;      // column range
  int level;       // tree level of the parent node (0 = root) ; leaves: -1
  int rank;        // -1 for a dense leaf
  size_t off_u;    // element offset of U (m x rank, row-major) or of the leaf (m x n)
  size_t off_v;    // element offset of Vt (rank x n, row-major)
};

struct Hodlr {
  int tree = 0, leaf = 0, dtype = 0, nlev = 0;
  std::vector<int> perm;     // cluster order -> natural interface index
  int *d_perm = nullptr;     // device copy (null for the identity)
  void *factors = nullptr;   // packed factor storage
  size_t bytes = 0;
  std::vector<HBlock> blocks;
  int max_rank = 0, min_rank = 1 << 30;
  // apply job tables (device), per direction and stage
  void *jobs = nullptr;
  std::vector<size_t> off_lr[2];  // per level offset of its LrJob list
  std::vector<int> n_lr[2];
  size_t off_leaf[2] = {0, 0};
  int n_leaf[2] = {0, 0};
  size_t off_con = 0;        // byte offset of the Contrib table in `jobs`
  // fused product (k_hodlr_apply_fused): one job per (interface, leaf
  // cluster) holding every contribution to its rows, per direction
  void *fjobs = nullptr;
  size_t foff_con = 0;       // byte offset of the FContrib table in `fjobs`
  size_t foff[2] = {0, 0};
  int fn[2] = {0, 0};
  double *pbuf = nullptr;    // 2 * n_ds * ld doubles: permuted x and y
  double tol_used = 0;       // truncation tolerance after the precision floor
};

// One output cluster of one interface at one level (or a leaf): the
// contributions are listed in the Contrib table [first, first+count).
struct LrJob {
  int out_iface;   // interface whose output rows are updated (0-based)
  int r0, r1;      // output rows (cluster order)
  int first, count;
};
struct Contrib {
  int in_iface;    // interface the input is read from (0-based)
  int c0, c1;      // input columns (cluster order)
  int rank;        // -1 dense
  long long off_u, off_v;
  int trans;       // apply the transpose of the stored block
  int pad_;
};
// A contribution to the rows [r0, r1) of a leaf cluster: a dense leaf
// (rank -1, rows x rows, row stride lds), or the rows roff .. roff + (r1 - r0)
// of a low-rank block whose output side has rfull rows (U: rfull x rank
// row-major, V^T: rank x n row-major; transposed: U^T x, then V^T rows).
struct FContrib {
  int in_iface, c0, c1, rank;
  long long off_u, off_v;
  int trans, roff, rfull, lds;
};

namespace {

// ----------------------------------------------------------- RNG (Philox)
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), then Box-Muller.
__device__ __forceinline__ void philox_round(unsigned (&c)[4], const unsigned (&k)[2]) {
  const unsigned long long p0 = (unsigned long long)0xD2511F53u * c[0];
  const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c[2];
  const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
  const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
  const unsigned n0 = hi1 ^ c[1] ^ k[0];
  const unsigned n1 = lo1;
  const unsigned n2 = hi0 ^ c[3] ^ k[1];
  const unsigned n3 = lo0;
  c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

__device__ void philox4x32_10(unsigned (&c)[4], unsigned k0, unsigned k1) {
  unsigned k[2] = {k0, k1};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
}

// Omega[i][k] (n x s, row-major) ~ N(0,1), counter = (i, k, level, 0).
__global__ void k_gaussian(double *__restrict__ om, int n, int s, unsigned long long seed,
                           int level) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * s) return;
  unsigned c[4] = {(unsigned)(e / s), (unsigned)(e % s), (unsigned)level, 0u};
  philox4x32_10(c, (unsigned)seed, (unsigned)(seed >> 32));
  const double u1 = ((double)c[0] + 1.0) * 2.3283064365386963e-10;  // (0, 1]
  const double u2 = (double)c[1] * 2.3283064365386963e-10;          // [0, 1)
  om[e] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// ------------------------------------------------------- batched block GEMM
// C (m x s, column-major, FP64) = op(B) * W with
//   trans == 0: op(B) = B       (m x n),  W: Omega, row-major n x s
//   trans == 1: op(B) = B^T     (m = n_B), W: Q, column-major n_B x s
// B is the (r0.., c0..) sub-block of a transfer matrix (ld, type T); with a
// permutation the row / column indices are mapped through perm.
struct BlockGemmJob {
  const void *S;
  int r0, c0, m, n;   // block origin and size in cluster order (m rows, n cols of B)
  double *C;          // output
  const double *W;    // Omega (shared) or this block's Q
};

// Work-group tile: TM rows of op(B) x SC columns (SC >= s), k in steps of
// GK (8 or 16); thread (tr, tc) accumulates rows 4 tr .. 4 tr + 3 and columns
// 8 tc .. 8 tc + 7 (32 FP64 sums), reading four op(B) and eight W values
// from LDS per k (16-byte reads).  Global reads are contiguous along S's
// rows (trans 0: along k; trans 1: along the output rows) and along W's
// contiguous index; a tile is staged through registers while the previous
// one is multiplied.
template <typename T, int SC>
__global__ __launch_bounds__(256) void k_block_gemm(const BlockGemmJob *__restrict__ jobs,
                                                    const int *__restrict__ perm, int ld, int s,
                                                    int trans) {
  constexpr int GK = SC == 32 ? 8 : 16;  // the 256-row tile: 8 staged values per thread
  constexpr int NTC = SC / 8, NTR = 256 / NTC, TM = 4 * NTR;
  constexpr int BP = TM + 2, WP = SC + 2;  // LDS rows (16-byte aligned)
  constexpr int NB = TM * GK / 256, NW = (GK * SC + 255) / 256;
  __shared__ __align__(16) double Bs[GK][BP];
  __shared__ __align__(16) double Ws[GK][WP];
  const BlockGemmJob J = jobs[blockIdx.y];
  const T *S = static_cast<const T *>(J.S);
  const int mrows = trans ? J.n : J.m;  // rows of op(B)
  const int kdim = trans ? J.m : J.n;
  const int row0 = blockIdx.x * TM;
  if (row0 >= mrows) return;
  const int tid = threadIdx.x;
  const int tr = tid % NTR, tc = tid / NTR;
  double rb[NB], rw[NW];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      // trans 0: k fastest (along a row of S); trans 1: the output row fastest
      const int kk = trans ? e / TM : e % GK, ii = trans ? e % TM : e / GK;
      const int i = row0 + ii, k = k0 + kk;
      double v = 0.0;
      if (i < mrows && k < kdim) {
        const int br = trans ? k : i, bc = trans ? i : k;  // entry B[br][bc]
        int gr = J.r0 + br, gc = J.c0 + bc;
        if (perm) {
          gr = perm[gr];
          gc = perm[gc];
        }
        v = (double)S[(size_t)gr * ld + gc];
      }
      rb[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const int e = tid + 256 * q;
      double v = 0.0;
      if (e < GK * SC) {
        // Omega row-major (n x s): q fastest; Q column-major (kdim x s): k fastest
        const int kk = trans ? e % GK : e / SC, c = trans ? e / GK : e % SC;
        const int k = k0 + kk;
        if (k < kdim && c < s) v = trans ? J.W[(size_t)c * kdim + k] : J.W[(size_t)k * s + c];
      }
      rw[q] = v;
    }
  };
  double acc[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[a][c] = 0.0;
  load(0);
  for (int k0 = 0; k0 < kdim; k0 += GK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      const int kk = trans ? e / TM : e % GK, ii = trans ? e % TM : e / GK;
      Bs[kk][ii] = rb[q];
    }
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const int e = tid + 256 * q;
      if (e < GK * SC) {
        const int kk = trans ? e % GK : e / SC, c = trans ? e / GK : e % SC;
        Ws[kk][c] = rw[q];
      }
    }
    __syncthreads();
    if (k0 + GK < kdim) load(k0 + GK);
#pragma unroll 4
    for (int kk = 0; kk < GK; ++kk) {
      typedef double d2 __attribute__((ext_vector_type(2)));
      const d2 b01 = *reinterpret_cast<const d2 *>(&Bs[kk][4 * tr]);
      const d2 b23 = *reinterpret_cast<const d2 *>(&Bs[kk][4 * tr + 2]);
      const double bv[4] = {b01[0], b01[1], b23[0], b23[1]};
      double wv[8];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const d2 w2 = *reinterpret_cast<const d2 *>(&Ws[kk][8 * tc + 2 * c]);
        wv[2 * c] = w2[0];
        wv[2 * c + 1] = w2[1];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[a][c] += bv[a] * wv[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int q = 8 * tc + c;
    if (q >= s) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = row0 + 4 * tr + a;
      if (i < mrows) J.C[(size_t)q * mrows + i] = acc[a][c];
    }
  }
}
template <typename T>
void launch_block_gemm(const BlockGemmJob *jobs, int nbk, int rows_max, const int *perm, int ld,
                       int s, int trans, hipStream_t st) {
  // tile widths 32, 64, 128 columns: 256, 128, 64 rows
  if (s <= 32)
    hipLaunchKernelGGL((k_block_gemm<T, 32>), dim3((rows_max + 255) / 256, nbk), dim3(256), 0, st,
                       jobs, perm, ld, s, trans);
  else if (s <= 64)
    hipLaunchKernelGGL((k_block_gemm<T, 64>), dim3((rows_max + 127) / 128, nbk), dim3(256), 0, st,
                       jobs, perm, ld, s, trans);
  else
    hipLaunchKernelGGL((k_block_gemm<T, 128>), dim3((rows_max + 63) / 64, nbk), dim3(256), 0, st,
                       jobs, perm, ld, s, trans);
}

// --------------------------------------------------- Householder QR + form Q
// In place on A (m x s, column-major): on exit A holds the explicit Q.
// One work-group per block; tau in LDS.
__device__ double block_reduce_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  return s;
}

struct QrJob {
  double *A;  // m x s column-major
  int m;
  double *R;  // optional: receives R (s x s, column-major, zero below the diagonal)
  double *Qs; // m x s scratch (Q is formed here, then copied over A)
};

__device__ __forceinline__ double qr_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;  // lane 0 holds the sum
}

// Blocked Householder QR, one work-group of kQrThreads per block.  Panels of
// kQb columns are factored column by column (each reflector applied to the
// panel's later columns only); the panel's reflectors H_j = I - tau_j v_j
// v_j^T (v_j: 1 at row j, stored below the diagonal of A) then act on the
// trailing columns together as H_{j0+b-1} ... H_{j0} = I - V T^T V^T (compact
// WY form: V the panel's reflectors, T upper triangular from their Gram
// matrix and tau), in two passes over the trailing columns: d_c = V^T a_c
// (a wavefront per trailing column group, each lane holding the panel's
// entries of one row of a 64-row chunk), then a_c -= V (T^T d_c) (a thread
// per row, its kQb reflector entries in registers).  The trailing columns are
// streamed twice per panel instead of three times per column.  Q = H_0 ...
// H_{k-1} [I; 0] is formed the same way in Qs, panels in reverse order
// (I - V T V^T on the columns from the panel's first on), and copied over A.
constexpr int kQrThreads = 1024;
constexpr int kQrWaves = kQrThreads / 64;
constexpr int kQb = 8;
constexpr int kQrMaxS = 128;
static_assert(kQrMaxS % kQb == 0, "whole panels");

// v_j's entry in row i (j < m): 1 on the diagonal, A below it, 0 above
__device__ __forceinline__ double qr_vent(const double *A, int m, int j, int i) {
  return i > j ? A[(size_t)j * m + i] : (i == j ? 1.0 : 0.0);
}

// X[:, c] -= V_p (M d_c) for the columns c0 <= c < s of X (m x s, rows >=
// j0 only; V_p: the reflectors j0 .. j0 + jb - 1 stored in A), with d_c =
// V_p^T X[:, c] and M = T^T (apply H_{j0+jb-1} ... H_{j0}) or T (apply
// H_{j0} ... H_{j0+jb-1}).  All threads of the work-group; ends with a
// barrier.  dl: kQb x kQrMaxS doubles of LDS.
template <bool TRANS>
__device__ void qr_apply_panel(const double *A, double *X, int m, int s, int j0, int jb, int c0,
                               const double (*T)[kQb], double (*dl)[kQrMaxS]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nc = s - c0;
  // pass 1: wavefront w takes the columns c0 + w, c0 + w + kQrWaves, ...,
  // four at a time (register budget of 1024-thread work-groups)
  constexpr int CPW = kQrMaxS / kQrWaves;  // columns per wavefront, at most
  constexpr int CH = 4;
  for (int u0 = 0; u0 < CPW; u0 += CH) {
    if (c0 + wave + kQrWaves * u0 >= s) break;  // wave-uniform
    double t[CH][kQb];
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
      for (int p = 0; p < kQb; ++p) t[u][p] = 0.0;
    for (int i0 = j0; i0 < m; i0 += 64) {
      const int i = i0 + lane;
      double v[kQb];
#pragma unroll
      for (int p = 0; p < kQb; ++p) v[p] = (p < jb && i < m) ? qr_vent(A, m, j0 + p, i) : 0.0;
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int c = c0 + wave + kQrWaves * (u0 + u);
        if (c < s) {
          const double x = i < m ? X[(size_t)c * m + i] : 0.0;
#pragma unroll
          for (int p = 0; p < kQb; ++p) t[u][p] += v[p] * x;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int c = c0 + wave + kQrWaves * (u0 + u);
#pragma unroll
      for (int p = 0; p < kQb; ++p) {
        const double r = qr_wave_sum(t[u][p]);
        if (lane == 0 && c < s && p < jb) dl[p][c] = r;
      }
    }
  }
  __syncthreads();
  // w_c = M d_c, in place (a thread per column)
  for (int c = c0 + threadIdx.x; c < s; c += kQrThreads) {
    double w[kQb];
#pragma unroll
    for (int q = 0; q < kQb; ++q) {
      double acc = 0.0;
      if (q < jb)
        for (int p = 0; p < jb; ++p) acc += (TRANS ? T[p][q] : T[q][p]) * dl[p][c];
      w[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < kQb; ++q)
      if (q < jb) dl[q][c] = w[q];
  }
  __syncthreads();
  // pass 2: X[i][c] -= sum_p v_p[i] w_c[p], a thread per row
  if (nc > 0)
    for (int i = j0 + threadIdx.x; i < m; i += kQrThreads) {
      double v[kQb];
#pragma unroll
      for (int p = 0; p < kQb; ++p) v[p] = p < jb ? qr_vent(A, m, j0 + p, i) : 0.0;
      for (int c = c0; c < s; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int p = 0; p < kQb; ++p) acc += v[p] * dl[p][c];
        X[(size_t)c * m + i] -= acc;
      }
    }
  __syncthreads();
}

__global__ __launch_bounds__(kQrThreads) void k_householder_q(const QrJob *__restrict__ jobs,
                                                              int s) {
  __shared__ double tau[kQrMaxS];
  __shared__ double sh[kQrWaves];
  __shared__ double dots[kQrMaxS];
  __shared__ double G[kQb][kQb];
  __shared__ double Tm[kQrMaxS / kQb][kQb][kQb];  // T of every panel
  __shared__ double dl[kQb][kQrMaxS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const QrJob J = jobs[blockIdx.x];
  double *A = J.A;
  const int m = J.m;
  const int kmax = min(s, m);
  for (int j0 = 0; j0 < kmax; j0 += kQb) {
    const int jb = min(kQb, kmax - j0);
    // the panel, column by column
    for (int j = j0; j < j0 + jb; ++j) {
      double *a = A + (size_t)j * m;
      double part = 0.0;
      for (int i = j + 1 + threadIdx.x; i < m; i += kQrThreads) part += a[i] * a[i];
      const double sig = block_reduce_sum(part, sh);
      const double x0 = a[j];
      double beta, t, scale;
      if (sig == 0.0) {
        t = 0.0;
        beta = x0;
        scale = 0.0;
      } else {
        const double mu = sqrt(x0 * x0 + sig);
        beta = (x0 <= 0.0) ? mu : -mu;  // beta = -sign(x0) |x|
        const double v0 = x0 - beta;
        t = (beta - x0) / beta;
        scale = 1.0 / v0;
      }
      __syncthreads();
      for (int i = j + 1 + threadIdx.x; i < m; i += kQrThreads) a[i] *= scale;  // v (v_0 = 1)
      if (threadIdx.x == 0) {
        a[j] = beta;
        tau[j] = t;
      }
      __syncthreads();
      // H_j on the panel's later columns: a wavefront per column for the dots
      for (int c = j + 1 + wave; c < j0 + jb; c += kQrWaves) {
        const double *ac = A + (size_t)c * m;
        double p2 = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) p2 += a[i] * ac[i];
        p2 = qr_wave_sum(p2);
        if (lane == 0) dots[c] = p2 + ac[j];
      }
      __syncthreads();
      for (int c = j + 1; c < j0 + jb; ++c) {
        double *ac = A + (size_t)c * m;
        const double w = t * dots[c];
        for (int i = j + 1 + threadIdx.x; i < m; i += kQrThreads) ac[i] -= w * a[i];
        if (threadIdx.x == 0) ac[j] -= w;
      }
      __syncthreads();
    }
    // Gram of the panel's reflectors, G[p][q] = v_p . v_q (p < q): v_q is 1
    // in row j0 + q and zero above it
    for (int pq = wave; pq < jb * jb; pq += kQrWaves) {
      const int p = pq / jb, q = pq % jb;
      if (p >= q) continue;
      const double *ap = A + (size_t)(j0 + p) * m, *aq = A + (size_t)(j0 + q) * m;
      double g = 0.0;
      for (int i = j0 + q + 1 + lane; i < m; i += 64) g += ap[i] * aq[i];
      g = qr_wave_sum(g);
      if (lane == 0) G[p][q] = g + ap[j0 + q];
    }
    __syncthreads();
    // T: T[q][q] = tau_q, T[0:q][q] = -tau_q T[0:q][0:q] G[0:q][q], zero below
    double (*T)[kQb] = Tm[j0 / kQb];
    if (threadIdx.x == 0) {
      for (int q = 0; q < kQb; ++q) {
        const double tq = q < jb ? tau[j0 + q] : 0.0;
        for (int p = 0; p < q; ++p) {
          double acc = 0.0;
          for (int r = p; r < q; ++r) acc += T[p][r] * G[r][q];
          T[p][q] = q < jb ? -tq * acc : 0.0;
        }
        T[q][q] = tq;
        for (int p = q + 1; p < kQb; ++p) T[p][q] = 0.0;
      }
    }
    __syncthreads();
    if (j0 + jb < s) qr_apply_panel<true>(A, A, m, s, j0, jb, j0 + jb, T, dl);
  }
  if (J.R) {  // R: the upper triangle left by the elimination
    for (int e = threadIdx.x; e < s * s; e += kQrThreads) {
      const int i = e % s, c = e / s;
      J.R[e] = (i <= c && i < kmax) ? A[(size_t)c * m + i] : 0.0;
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{k-1} [I; 0] in Qs (columns beyond min(s, m), when m < s: 0)
  double *Q = J.Qs;
  for (size_t e = threadIdx.x; e < (size_t)m * s; e += kQrThreads) {
    const int c = (int)(e / m), i = (int)(e % m);
    Q[e] = (i == c && c < kmax) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int np = (kmax + kQb - 1) / kQb;
  for (int pn = np - 1; pn >= 0; --pn) {
    const int j0 = pn * kQb, jb = min(kQb, kmax - j0);
    qr_apply_panel<false>(A, Q, m, s, j0, jb, j0, Tm[pn], dl);
  }
  for (size_t e = threadIdx.x; e < (size_t)m * s; e += kQrThreads) A[e] = Q[e];
}

// -------------------------------------------------- one-sided Jacobi SVD
// X (n x s, column-major, n <= SMAX, s <= SMAX, s even) -> X V with
// mutually orthogonal columns; V (s x s, column-major) accumulates the
// rotations, and sigma_k = |(X V)_k| is written for every column.
// Round-robin pair ordering (player 0 fixed, the others rotating), 256 / (s/2)
// threads per pair; stops when a sweep performs no rotation.
struct JacJob {
  double *X;
  double *V;
  int n;
};

// The columns being rotated (the s x s R factor of the sample block) live in
// LDS, and so do the rotations when they fit beside them (SMAX <= 64: two
// 32 KB arrays, so several blocks share a CU); at SMAX = 128 V stays in
// global memory.
template <int SMAX>
__global__ __launch_bounds__(256) void k_jacobi(const JacJob *__restrict__ jobs, int s,
                                                int max_sweeps, double *__restrict__ sigma) {
  constexpr bool VL = SMAX <= 64;
  constexpr int TPP = 256 / (SMAX / 2);  // threads per pair
  __shared__ int rotated;
  __shared__ double X[SMAX * SMAX];
  __shared__ double Vl[VL ? SMAX * SMAX : 1];
  const JacJob J = jobs[blockIdx.x];
  const int n = J.n;
  double *V = VL ? Vl : J.V;
  for (int e = threadIdx.x; e < s * s; e += 256) V[e] = (e / s == e % s) ? 1.0 : 0.0;
  for (int e = threadIdx.x; e < n * s; e += 256) X[e] = J.X[e];
  __syncthreads();
  const int grp = threadIdx.x / TPP, sub = threadIdx.x % TPP;
  const int npairs = s / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < s - 1; ++round) {
      if (grp < npairs) {
        auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + round) % (s - 1); };
        int p = pos(grp), q = pos(s - 1 - grp);
        if (p > q) { const int t = p; p = q; q = t; }
        double *xp = X + (size_t)p * n, *xq = X + (size_t)q * n;
        double a = 0, b = 0, g = 0;
        for (int i = sub; i < n; i += TPP) {
          const double u = xp[i], v = xq[i];
          a += u * u; b += v * v; g += u * v;
        }
        // combine the partial sums of the pair's TPP consecutive lanes
#pragma unroll
        for (int off = 1; off < TPP; off <<= 1) {
          a += __shfl_xor(a, off, 64);
          b += __shfl_xor(b, off, 64);
          g += __shfl_xor(g, off, 64);
        }
        if (g != 0.0 && fabs(g) > 1e-15 * sqrt(a * b)) {
          const double zeta = (b - a) / (2.0 * g);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          for (int i = sub; i < n; i += TPP) {
            const double u = xp[i], v = xq[i];
            xp[i] = c * u - sn * v;
            xq[i] = sn * u + c * v;
          }
          double *vp = V + (size_t)p * s, *vq = V + (size_t)q * s;
          for (int i = sub; i < s; i += TPP) {
            const double u = vp[i], v = vq[i];
            vp[i] = c * u - sn * v;
            vq[i] = sn * u + c * v;
          }
          if (sub == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * s; e += 256) J.X[e] = X[e];
  if (VL)
    for (int e = threadIdx.x; e < s * s; e += 256) J.V[e] = V[e];
  for (int k = threadIdx.x; k < s; k += 256) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += X[(size_t)k * n + i] * X[(size_t)k * n + i];
    sigma[(size_t)blockIdx.x * s + k] = sqrt(t);
  }
}

// --------------------------------------------------- batched dense product
// C (m x s) = A (m x s) B (s x s), all column-major FP64 (the orthogonalised
// sample block Q R' after the Jacobi rotations of R).
struct DenseGemmJob {
  const double *A, *B;
  double *C;
  int m;
};

__global__ __launch_bounds__(256) void k_dense_gemm(const DenseGemmJob *__restrict__ jobs,
                                                    int s) {
  constexpr int TM = 64, TK = 32;
  __shared__ double As[TK][TM + 1];  // A tile, k-major
  __shared__ double Bs[TK][129];     // B rows k0.., s <= 128 columns
  const DenseGemmJob J = jobs[blockIdx.y];
  const int row0 = blockIdx.x * TM;
  if (row0 >= J.m) return;
  const int tid = threadIdx.x, tr = tid & 63, tc = tid >> 6;
  double acc[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < s; k0 += TK) {
    __syncthreads();
    for (int e = tid; e < TK * TM; e += 256) {
      const int kk = e / TM, ii = e % TM, i = row0 + ii, k = k0 + kk;
      As[kk][ii] = (i < J.m && k < s) ? J.A[(size_t)k * J.m + i] : 0.0;
    }
    for (int e = tid; e < TK * s; e += 256) {
      const int kk = e / s, q = e % s, k = k0 + kk;
      Bs[kk][q] = (k < s) ? J.B[(size_t)q * s + k] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < TK; ++kk) {
      const double a = As[kk][tr];
#pragma unroll
      for (int q = 0; q < 32; ++q)
        if (tc + 4 * q < s) acc[q] += a * Bs[kk][tc + 4 * q];
    }
  }
  const int i = row0 + tr;
  if (i < J.m)
#pragma unroll
    for (int q = 0; q < 32; ++q)
      if (tc + 4 * q < s) J.C[(size_t)(tc + 4 * q) * J.m + i] = acc[q];
}

// ----------------------------------------------------------------- packing
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  const unsigned lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

template <typename F> struct FactorIO;
template <> struct FactorIO<unsigned short> {
  static __device__ __forceinline__ unsigned short put(double v) { return f32_to_bf16((float)v); }
  static __device__ __forceinline__ float get(unsigned short v) { return bf16_to_f32(v); }
};
template <> struct FactorIO<float> {
  static __device__ __forceinline__ float put(double v) { return (float)v; }
  static __device__ __forceinline__ float get(float v) { return v; }
};
template <> struct FactorIO<double> {
  static __device__ __forceinline__ double put(double v) { return v; }
  static __device__ __forceinline__ double get(double v) { return v; }
};

struct PackJob {
  const double *Q;    // m x s col-major
  const double *X;    // n x s col-major (rotated)
  const double *V;    // s x s col-major
  const int *sel;     // selected columns (rank entries)
  int m, n, rank;
  long long off_u, off_v;
};

// U = Q V_sel (m x rank, row-major), Vt = X_sel^T (rank x n, row-major)
template <typename F>
__global__ __launch_bounds__(256) void k_pack(const PackJob *__restrict__ jobs, int s,
                                              F *__restrict__ store) {
  const PackJob J = jobs[blockIdx.y];
  const size_t tot_u = (size_t)J.m * J.rank, tot_v = (size_t)J.rank * J.n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot_u + tot_v;
       e += (size_t)gridDim.x * blockDim.x) {
    if (e < tot_u) {
      // U[i][k] = (Q V)[i][sel[k]]: consecutive threads take consecutive rows
      // of Q (column-major) for the same column of V
      const int k = (int)(e / J.m), i = (int)(e % J.m);
      const double *vk = J.V + (size_t)J.sel[k] * s;
      double v = 0.0;
      for (int q = 0; q < s; ++q) v += J.Q[(size_t)q * J.m + i] * vk[q];
      store[J.off_u + (size_t)i * J.rank + k] = FactorIO<F>::put(v);
    } else {
      const size_t f = e - tot_u;
      const int k = (int)(f / J.n), c = (int)(f % J.n);
      store[J.off_v + f] = FactorIO<F>::put(J.X[(size_t)J.sel[k] * J.n + c]);
    }
  }
}

struct LeafJob {
  const void *S;
  int r0, n, lds;  // lds: row stride in the store (n rounded up to 8; padding zero)
  long long off;
};

template <typename T, typename F>
__global__ void k_pack_leaf(const LeafJob *__restrict__ jobs, const int *__restrict__ perm,
                            int ld, F *__restrict__ store) {
  const LeafJob J = jobs[blockIdx.y];
  const T *S = static_cast<const T *>(J.S);
  const size_t tot = (size_t)J.n * J.lds;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / J.lds), c = (int)(e % J.lds);
    double v = 0.0;
    if (c < J.n) {
      int gr = J.r0 + r, gc = J.r0 + c;
      if (perm) { gr = perm[gr]; gc = perm[gc]; }
      v = (double)S[(size_t)gr * ld + gc];
    }
    store[J.off + e] = FactorIO<F>::put(v);
  }
}

// ------------------------------------------------------------------- apply
// Eight consecutive factors (16-byte aligned) as accumulation values.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename F, typename Acc>
__device__ __forceinline__ void load8f(const F *p, Acc (&v)[8]) {
  if constexpr (sizeof(F) == 2) {
    const u32x4 q = *reinterpret_cast<const __attribute__((address_space(1))) u32x4 *>(gp(p));
    const unsigned w[4] = {q[0], q[1], q[2], q[3]};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[2 * e] = (Acc)__uint_as_float(w[e] << 16);
      v[2 * e + 1] = (Acc)__uint_as_float(w[e] & 0xffff0000u);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (Acc)FactorIO<F>::get(p[e]);
  }
}

// y = x - S x (or x - S^T x) over the rows of one leaf cluster of one
// interface per work-group, in one launch: the identity part, the dense
// leaves of both neighbouring transfer blocks, and at every tree level the
// low-rank blocks whose row cluster contains these rows (their t = V^T x
// formed by each leaf work-group again: a few thousand entries).  Rows of a
// work-group are disjoint from every other's, so there are no write races;
// the last cluster of an interface also copies the padding (rows >= M).
template <typename F>
__global__ __launch_bounds__(256) void k_hodlr_apply_fused(const LrJob *__restrict__ jobs,
                                                           const FContrib *__restrict__ con,
                                                           const F *__restrict__ store,
                                                           const double *__restrict__ x,
                                                           double *__restrict__ y, int ld, int M) {
  using Acc = typename std::conditional<std::is_same<F, double>::value, double, float>::type;
  __shared__ Acc t[128];
  __shared__ Acc xs[128];
  const LrJob J = jobs[blockIdx.x];
  const int rows = J.r1 - J.r0;
  const double *xo = x + (size_t)J.out_iface * ld;
  double *yo = y + (size_t)J.out_iface * ld + J.r0;
  for (int r = threadIdx.x; r < rows; r += 256) yo[r] = xo[J.r0 + r];
  if (J.r1 == M)
    for (int r = M + threadIdx.x; r < ld; r += 256) y[(size_t)J.out_iface * ld + r] = xo[r];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int ci = 0; ci < J.count; ++ci) {
    const FContrib C = con[J.first + ci];
    const double *xin = x + (size_t)C.in_iface * ld + C.c0;
    const int ncol = C.c1 - C.c0;
    if (C.rank < 0) {  // dense square leaf, row stride lds (padding zero)
      const F *Lf = store + C.off_u;
      if (!C.trans) {
        // 16 lanes per row with 8 columns each (one 16-byte load of BF16),
        // four rows per wavefront at a time; x staged per 128 columns
        const int sub = lane >> 4, l16 = lane & 15;
        for (int cb = 0; cb < ncol; cb += 128) {
          const int cw = min(128, ncol - cb);
          __syncthreads();
          for (int c = threadIdx.x; c < 128; c += 256) xs[c] = c < cw ? (Acc)xin[cb + c] : Acc(0);
          __syncthreads();
          for (int r0 = 4 * wave; r0 < rows; r0 += 16) {
            const int r = r0 + sub;
            Acc acc = 0;
            if (r < rows && 8 * l16 < cw) {
              Acc v[8];
              load8f<F, Acc>(Lf + (size_t)r * C.lds + cb + 8 * l16, v);
#pragma unroll
              for (int e = 0; e < 8; ++e) acc += v[e] * xs[8 * l16 + e];
            }
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) acc += __shfl_down(acc, off, 16);
            if (l16 == 0 && r < rows) yo[r] -= (double)acc;
          }
        }
      } else {
        // one thread per row: column c of the leaf is contiguous over rows
        for (int r = threadIdx.x; r < rows; r += 256) {
          Acc acc = 0;
          for (int c = 0; c < ncol; ++c)
            acc += (Acc)FactorIO<F>::get(Lf[(size_t)c * C.lds + r]) * (Acc)xin[c];
          yo[r] -= (double)acc;
        }
      }
      __syncthreads();
      continue;
    }
    const int rk = C.rank;
    // t = V^T x (or U^T x for the transpose): one wavefront per entry of t
    for (int k = wave; k < rk; k += 4) {
      Acc acc = 0;
      if (!C.trans) {
        const F *v = store + C.off_v + (size_t)k * ncol;
        for (int c = lane; c < ncol; c += 64) acc += (Acc)FactorIO<F>::get(v[c]) * (Acc)xin[c];
      } else {
        const F *u = store + C.off_u;
        for (int c = lane; c < ncol; c += 64)
          acc += (Acc)FactorIO<F>::get(u[(size_t)c * rk + k]) * (Acc)xin[c];
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
      if (lane == 0) t[k] = acc;
    }
    __syncthreads();
    // rows roff .. roff + rows of the block's output side
    for (int r = threadIdx.x; r < rows; r += 256) {
      Acc acc = 0;
      const int rr = C.roff + r;
      if (!C.trans) {
        const F *u = store + C.off_u + (size_t)rr * rk;
        for (int k = 0; k < rk; ++k) acc += (Acc)FactorIO<F>::get(u[k]) * t[k];
      } else {
        const F *v = store + C.off_v;
        for (int k = 0; k < rk; ++k)
          acc += (Acc)FactorIO<F>::get(v[(size_t)k * C.rfull + rr]) * t[k];
      }
      yo[r] -= (double)acc;
    }
    __syncthreads();
  }
}

// Gather to cluster order (inverse = 0: dst[i] = src[perm[i]]) or scatter
// back (inverse = 1: dst[perm[i]] = src[i]); padding entries are zero.
__global__ void k_permute(const double *__restrict__ src, double *__restrict__ dst,
                          const int *__restrict__ perm, int M, int ld, int inverse) {
  const int j = blockIdx.y;
  const double *sj = src + (size_t)j * ld;
  double *dj = dst + (size_t)j * ld;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ld; i += gridDim.x * blockDim.x) {
    if (i >= M) {
      dj[i] = 0.0;
    } else if (inverse) {
      dj[perm[i]] = sj[i];
    } else {
      dj[i] = sj[perm[i]];
    }
  }
}

__global__ void k_copy_d(const double *__restrict__ s, double *__restrict__ d, size_t n) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] = s[e];
}

inline unsigned nb(size_t n, unsigned b = 256) { return (unsigned)((n + b - 1) / b); }
inline size_t pad8(size_t n) { return (n + 7) & ~size_t(7); }

// ----------------------------------------------------------- host helpers
struct HipErr : std::runtime_error {
  using std::runtime_error::runtime_error;
};
#define HCHK(x)                                                                        \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) throw HipErr(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct DMem {
  void *p = nullptr;
  explicit DMem(size_t b) {
    if (b && dev_malloc(&p, b) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
  }
  ~DMem() {
    if (p) dev_free(p);
  }
  template <typename X>
  X *as() const { return static_cast<X *>(p); }
};

template <typename J>
void *upload(const std::vector<J> &v, hipStream_t s, std::vector<DMem *> &keep) {
  DMem *m = new DMem(std::max<size_t>(v.size(), 1) * sizeof(J));
  keep.push_back(m);
  if (!v.empty()) HCHK(hipMemcpyAsync(m->p, v.data(), v.size() * sizeof(J), hipMemcpyHostToDevice, s));
  return m->p;
}

struct Node {
  int lo, hi;                 // cluster-order range
  std::vector<int> kids;      // indices into the node list
  int level;
};

// Build the cluster tree; perm maps cluster order to natural order.
void build_tree(int dim, int n, int M, int tree, int leaf, std::vector<Node> &nodes,
                std::vector<int> &perm) {
  nodes.clear();
  perm.clear();
  if (tree == DDST_TREE_BINARY || dim == 2) {
    perm.resize(M);
    std::iota(perm.begin(), perm.end(), 0);
    std::vector<int> stack;
    nodes.push_back({0, M, {}, 0});
    stack.push_back(0);
    while (!stack.empty()) {
      const int id = stack.back();
      stack.pop_back();
      const int lo = nodes[id].lo, hi = nodes[id].hi;
      if (hi - lo <= leaf) continue;
      const int mid = lo + (hi - lo + 1) / 2;
      for (auto r : {std::make_pair(lo, mid), std::make_pair(mid, hi)}) {
        nodes.push_back({r.first, r.second, {}, nodes[id].level + 1});
        nodes[id].kids.push_back((int)nodes.size() - 1);
        stack.push_back((int)nodes.size() - 1);
      }
    }
    return;
  }
  // quadtree over the n x n interface grid (natural index y*n + z)
  // first pass: build the tree of rectangles, assign ranges by DFS order
  struct RNode { int y0, y1, z0, z1, level; std::vector<int> kids; };
  std::vector<RNode> rn;
  rn.push_back({0, n, 0, n, 0, {}});
  std::vector<int> st = {0};
  while (!st.empty()) {
    const int id = st.back();
    st.pop_back();
    const RNode r = rn[id];
    const int size = (r.y1 - r.y0) * (r.z1 - r.z0);
    if (size <= leaf || (r.y1 - r.y0 < 2 && r.z1 - r.z0 < 2)) continue;
    const int ym = r.y0 + (r.y1 - r.y0 + 1) / 2, zm = r.z0 + (r.z1 - r.z0 + 1) / 2;
    const int ys[3] = {r.y0, ym, r.y1}, zs[3] = {r.z0, zm, r.z1};
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        if (ys[a + 1] > ys[a] && zs[b + 1] > zs[b]) {
          rn.push_back({ys[a], ys[a + 1], zs[b], zs[b + 1], r.level + 1, {}});
          rn[id].kids.push_back((int)rn.size() - 1);
          st.push_back((int)rn.size() - 1);
        }
  }
  // depth-first numbering: leaves in DFS order give the permutation
  nodes.resize(rn.size());
  std::function<void(int)> visit = [&](int id) {
    Node nd;
    nd.level = rn[id].level;
    nd.lo = (int)perm.size();
    if (rn[id].kids.empty()) {
      for (int y = rn[id].y0; y < rn[id].y1; ++y)
        for (int z = rn[id].z0; z < rn[id].z1; ++z) perm.push_back(y * n + z);
    } else {
      for (int k : rn[id].kids) visit(k);
    }
    nd.hi = (int)perm.size();
    nd.kids = rn[id].kids;
    nodes[id] = nd;
  };
  visit(0);
}

template <typename T, typename F>
int compress_impl(ddst_op *op, const ddst_compress_opts_t &o, hipStream_t st, int *overflow) {
  Hodlr *H = new Hodlr();
  std::vector<DMem *> keep;
  auto cleanup = [&]() {
    for (DMem *m : keep) delete m;
    keep.clear();
  };
  auto drop = [&]() {
    if (H->d_perm) dev_free(H->d_perm);
    if (H->factors) dev_free(H->factors);
    if (H->jobs) dev_free(H->jobs);
    if (H->fjobs) dev_free(H->fjobs);
    if (H->pbuf) dev_free(H->pbuf);
    delete H;
  };
  try {
    H->tree = o.tree;
    H->leaf = o.leaf;
    H->dtype = o.factor_dtype;
    // An FP32-built transfer block resolves singular values only down to a
    // few units of eps32 times its norm; below that the tail is rounding
    // noise, so the FP32 path truncates no lower than 1e-6.
    H->tol_used = (op->prec == DDST_FP32) ? std::max(o.tol, 1e-6) : o.tol;
    std::vector<Node> nodes;
    build_tree(op->dim, op->n, op->M, o.tree, o.leaf, nodes, H->perm);
    bool identity = true;
    for (int i = 0; i < op->M; ++i) identity = identity && H->perm[i] == i;
    const int *d_perm = nullptr;
    if (!identity) {
      HCHK(dev_malloc(reinterpret_cast<void **>(&H->d_perm), op->M * sizeof(int)));
      HCHK(hipMemcpyAsync(H->d_perm, H->perm.data(), op->M * sizeof(int), hipMemcpyHostToDevice,
                          st));
      HCHK(dev_malloc(reinterpret_cast<void **>(&H->pbuf),
                      (size_t)2 * op->n_ds * op->ld * sizeof(double)));
      d_perm = H->d_perm;
    }
    // transfer matrices that exist
    std::vector<int> mats;
    for (int j = 1; j <= op->n_ds; ++j) {
      if (j >= 2) mats.push_back(2 * (j - 1));
      if (j <= op->n_ds - 1) mats.push_back(2 * (j - 1) + 1);
    }
    const int nmat = (int)mats.size();
    auto Sptr = [&](int sm) {
      return static_cast<const void *>(static_cast<unsigned char *>(op->S) +
                                       (size_t)sm * op->mat_bytes);
    };
    // ---- ||S||_2 of every transfer matrix: power iteration on S^T S
    std::vector<double> snorm(2 * op->n_ds, 0.0);
    if (nmat > 0) {
      DMem vec((size_t)2 * nmat * op->ld * sizeof(double));
      double *v0 = static_cast<double *>(vec.p), *v1 = v0 + (size_t)nmat * op->ld;
      std::vector<double> h((size_t)nmat * op->ld, 0.0);
      for (int b = 0; b < nmat; ++b)
        for (int i = 0; i < op->M; ++i) h[(size_t)b * op->ld + i] = 1.0 + 0.37 * std::sin(1.7 * i + b);
      std::vector<GemvJob> fw, bw;
      for (int b = 0; b < nmat; ++b) {
        GemvJob g{};
        g.G = Sptr(mats[b]);
        g.x1 = v0 + (size_t)b * op->ld;
        g.out = v1 + (size_t)b * op->ld;
        fw.push_back(g);
        GemvJob q{};
        q.G = Sptr(mats[b]);
        q.x1 = v1 + (size_t)b * op->ld;
        q.out = v0 + (size_t)b * op->ld;
        bw.push_back(q);
      }
      const GemvJob *dfw = static_cast<const GemvJob *>(upload(fw, st, keep));
      const GemvJob *dbw = static_cast<const GemvJob *>(upload(bw, st, keep));
      const int nchunk = std::min(op->ld / kGemvChunk, 64);
      DMem part((size_t)nmat * nchunk * op->ld * sizeof(double));
      for (int it = 0; it < 8; ++it) {
        HCHK(hipMemcpyAsync(v0, h.data(), h.size() * 8, hipMemcpyHostToDevice, st));
        launch_gemv<T>(dfw, nmat, op->ld, op->M, 0, 1.0, static_cast<double *>(part.p), st);
        launch_gemv<T>(dbw, nmat, op->ld, op->M, 1, 1.0, static_cast<double *>(part.p), st);
        HCHK(hipMemcpyAsync(h.data(), v0, h.size() * 8, hipMemcpyDeviceToHost, st));
        HCHK(hipStreamSynchronize(st));
        for (int b = 0; b < nmat; ++b) {
          double ss = 0;
          for (int i = 0; i < op->M; ++i) ss += h[(size_t)b * op->ld + i] * h[(size_t)b * op->ld + i];
          const double nv = std::sqrt(ss);  // = sigma_max^2 for a converged unit vector
          snorm[mats[b]] = std::sqrt(nv);
          for (int i = 0; i < op->M; ++i) h[(size_t)b * op->ld + i] /= (nv > 0 ? nv : 1.0);
        }
      }
    }
    // ---- admissible pairs per tree level, and the leaves
    std::vector<std::vector<std::pair<int, int>>> lev;
    std::vector<int> leaves;
    for (size_t id = 0; id < nodes.size(); ++id) {
      const Node &nd = nodes[id];
      if (nd.kids.empty()) {
        leaves.push_back((int)id);
        continue;
      }
      if ((int)lev.size() <= nd.level) lev.resize(nd.level + 1);
      for (int a : nd.kids)
        for (int b : nd.kids)
          if (a != b) lev[nd.level].push_back({a, b});
    }
    H->nlev = (int)lev.size();
    const int s_cap = std::min(o.max_rank + o.oversample, 128);
    size_t store_elems = 0;
    for (int m : mats)
      for (int lf : leaves) {
        HBlock b{};
        b.smat = m;
        b.r0 = nodes[lf].lo;
        b.r1 = nodes[lf].hi;
        b.c0 = b.r0;
        b.c1 = b.r1;
        b.level = -1;
        b.rank = -1;
        b.off_u = store_elems;
        // rows padded to a multiple of 8 entries (16-byte factor loads)
        store_elems += (size_t)(b.r1 - b.r0) * pad8(b.r1 - b.r0);
        H->blocks.push_back(b);
      }
    // ---- compress level by level (FP64 staging kept until packing)
    struct LevelData {
      DMem *Y = nullptr, *X = nullptr, *V = nullptr, *sig = nullptr, *sel = nullptr;
      DMem *R = nullptr, *XR = nullptr;  // R of X = Q2 R, and X rotated (Q2 R J)
      int s = 0;
      std::vector<HBlock> blocks;
      std::vector<char> kept;  // block accepted at this sample count
      std::vector<size_t> offY, offX;
      std::vector<int> selofs;
    };
    std::vector<LevelData> levels;
    int worst = 0;
    // Adaptive sample counts.  Every admissible block is first sampled with
    // kSampleStart Gaussian columns (or all of them, when its smaller side
    // is shorter); a block whose numerical rank comes within `oversample` of
    // its sample count is sampled again with twice as many, up to
    // min(rank cap + oversample, smaller side).  Blocks of one tree level
    // and one sample count are compressed together (one group); most blocks
    // of the workloads here are accepted at the first count, so the QR and
    // the Jacobi sweeps (whose cost grows like s^2 and s^3) run on s = 32.
    constexpr int kSampleStart = 32;
    struct Group {
      int L, s;
      std::vector<HBlock> blocks;
    };
    auto full_count = [&](const HBlock &b) {  // largest useful sample count
      int sb = std::min(s_cap, std::min(b.r1 - b.r0, b.c1 - b.c0));
      sb -= sb & 1;
      return std::max(sb, 2);
    };
    std::vector<Group> groups;
    auto add_block = [&](const HBlock &b, int sb) {
      for (Group &g : groups)
        if (g.L == b.level && g.s == sb) {
          g.blocks.push_back(b);
          return;
        }
      groups.push_back({b.level, sb, {b}});
    };
    for (size_t L = 0; L < lev.size(); ++L)
      for (int mi = 0; mi < nmat; ++mi)
        for (auto &pr : lev[L]) {
          HBlock b{};
          b.smat = mats[mi];
          b.r0 = nodes[pr.first].lo;
          b.r1 = nodes[pr.first].hi;
          b.c0 = nodes[pr.second].lo;
          b.c1 = nodes[pr.second].hi;
          b.level = (int)L;
          add_block(b, std::min(full_count(b), kSampleStart));
        }
    // groups appended while this loop runs (blocks sampled again) are
    // processed by it too; a group is never revisited once processed
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      if (nmat == 0) continue;
      const int L = groups[gi].L;
      const int s = groups[gi].s;
      LevelData D;
      D.s = s;
      D.blocks = groups[gi].blocks;
      int mmax = 0, nmax = 0;
      size_t totY = 0, totX = 0;
      for (const HBlock &b : D.blocks) {
        mmax = std::max(mmax, b.r1 - b.r0);
        nmax = std::max(nmax, b.c1 - b.c0);
        D.offY.push_back(totY);
        D.offX.push_back(totX);
        totY += (size_t)(b.r1 - b.r0) * s;
        totX += (size_t)(b.c1 - b.c0) * s;
      }
      const int nbk = (int)D.blocks.size();
      D.Y = new DMem(totY * 8); keep.push_back(D.Y);
      D.X = new DMem(totX * 8); keep.push_back(D.X);
      D.V = new DMem((size_t)nbk * s * s * 8); keep.push_back(D.V);
      D.R = new DMem((size_t)nbk * s * s * 8); keep.push_back(D.R);
      D.XR = new DMem(totX * 8); keep.push_back(D.XR);
      D.sig = new DMem((size_t)nbk * s * 8); keep.push_back(D.sig);
      DMem om((size_t)nmax * s * 8);
      DMem qsm(std::max(totY, totX) * 8);  // Q of each QR is formed here (one QR at a time)
      double *qs = static_cast<double *>(qsm.p);
      hipLaunchKernelGGL(k_gaussian, dim3(nb((size_t)nmax * s)), dim3(256), 0, st,
                         static_cast<double *>(om.p), nmax, s, (unsigned long long)o.seed, (int)L);
      std::vector<BlockGemmJob> gy, gx;
      std::vector<QrJob> qr, qx;
      std::vector<JacJob> jac;
      std::vector<DenseGemmJob> rot;
      for (int b = 0; b < nbk; ++b) {
        const HBlock &hb = D.blocks[b];
        const int m = hb.r1 - hb.r0, n = hb.c1 - hb.c0;
        double *Yb = static_cast<double *>(D.Y->p) + D.offY[b];
        double *Xb = static_cast<double *>(D.X->p) + D.offX[b];
        double *Rb = static_cast<double *>(D.R->p) + (size_t)b * s * s;
        gy.push_back({Sptr(hb.smat), hb.r0, hb.c0, m, n, Yb, static_cast<double *>(om.p)});
        gx.push_back({Sptr(hb.smat), hb.r0, hb.c0, m, n, Xb, Yb});
        qr.push_back({Yb, m, nullptr, qs + D.offY[b]});
        // X = Q2 R: the Jacobi rotations run on the s x s R instead of the
        // n x s X (same singular values and rotations), then X J = Q2 (R J)
        qx.push_back({Xb, n, Rb, qs + D.offX[b]});
        jac.push_back({Rb, static_cast<double *>(D.V->p) + (size_t)b * s * s, s});
        rot.push_back({Xb, Rb, static_cast<double *>(D.XR->p) + D.offX[b], n});
      }
      const BlockGemmJob *dgy = static_cast<const BlockGemmJob *>(upload(gy, st, keep));
      const BlockGemmJob *dgx = static_cast<const BlockGemmJob *>(upload(gx, st, keep));
      const QrJob *dqr = static_cast<const QrJob *>(upload(qr, st, keep));
      const JacJob *djac = static_cast<const JacJob *>(upload(jac, st, keep));
      const QrJob *dqx = static_cast<const QrJob *>(upload(qx, st, keep));
      const DenseGemmJob *drot = static_cast<const DenseGemmJob *>(upload(rot, st, keep));
      launch_block_gemm<T>(dgy, nbk, mmax, d_perm, op->ld, s, 0, st);
      if (s > kQrMaxS) throw std::logic_error("sample count above the QR kernel's column limit");
      hipLaunchKernelGGL(k_householder_q, dim3(nbk), dim3(kQrThreads), 0, st, dqr, s);
      launch_block_gemm<T>(dgx, nbk, nmax, d_perm, op->ld, s, 1, st);
      hipLaunchKernelGGL(k_householder_q, dim3(nbk), dim3(kQrThreads), 0, st, dqx, s);
      double *dsig = static_cast<double *>(D.sig->p);
      if (s <= 32)
        hipLaunchKernelGGL(k_jacobi<32>, dim3(nbk), dim3(256), 0, st, djac, s, 30, dsig);
      else if (s <= 64)
        hipLaunchKernelGGL(k_jacobi<64>, dim3(nbk), dim3(256), 0, st, djac, s, 30, dsig);
      else
        hipLaunchKernelGGL(k_jacobi<128>, dim3(nbk), dim3(256), 0, st, djac, s, 30, dsig);
      hipLaunchKernelGGL(k_dense_gemm, dim3((nmax + 63) / 64, nbk), dim3(256), 0, st, drot, s);
      HCHK(hipGetLastError());
      std::vector<double> sig((size_t)nbk * s);
      HCHK(hipMemcpyAsync(sig.data(), D.sig->p, sig.size() * 8, hipMemcpyDeviceToHost, st));
      HCHK(hipStreamSynchronize(st));
      std::vector<int> selall;
      std::vector<HBlock> again;
      D.kept.assign(nbk, 0);
      for (int b = 0; b < nbk; ++b) {
        HBlock &hb = D.blocks[b];
        const double thr = H->tol_used * snorm[hb.smat];
        std::vector<std::pair<double, int>> sv;
        for (int k = 0; k < s; ++k) sv.push_back({sig[(size_t)b * s + k], k});
        std::sort(sv.begin(), sv.end(),
                  [](const std::pair<double, int> &a, const std::pair<double, int> &c) {
                    return a.first > c.first;
                  });
        int r = 0;
        while (r < s && sv[r].first > thr) ++r;
        // The sample count bounds the rank that can be certified: a block
        // sampled with fewer columns than its smaller side whose rank comes
        // within `oversample` of s may have more singular values above the
        // threshold than the samples show.  It is sampled again with twice
        // the count while that stays below min(cap, smaller side); at that
        // limit (the rank cap) it is a rank overflow.  A block with s equal
        // to its smaller side is sampled completely.
        const bool undersampled = s < std::min(hb.r1 - hb.r0, hb.c1 - hb.c0);
        if (undersampled && r > s - o.oversample) {
          const int sf = full_count(hb);
          if (s < sf) {
            again.push_back(hb);
            D.selofs.push_back(0);
            continue;
          }
          worst = std::max(worst, r);
        }
        D.kept[b] = 1;
        hb.rank = r;
        hb.off_u = store_elems;
        store_elems += pad8((size_t)(hb.r1 - hb.r0) * r);
        hb.off_v = store_elems;
        store_elems += pad8((size_t)r * (hb.c1 - hb.c0));
        D.selofs.push_back((int)selall.size());
        for (int k = 0; k < r; ++k) selall.push_back(sv[k].second);
        H->max_rank = std::max(H->max_rank, r);
        H->min_rank = std::min(H->min_rank, r);
      }
      D.sel = new DMem(std::max<size_t>(selall.size(), 1) * sizeof(int));
      keep.push_back(D.sel);
      if (!selall.empty())
        HCHK(hipMemcpyAsync(D.sel->p, selall.data(), selall.size() * sizeof(int),
                            hipMemcpyHostToDevice, st));
      HCHK(hipStreamSynchronize(st));
      levels.push_back(std::move(D));
      for (const HBlock &hb : again) {
        const int s2 = std::min(full_count(hb), 2 * s);
        bool found = false;
        for (size_t g2 = gi + 1; g2 < groups.size() && !found; ++g2)
          if (groups[g2].L == L && groups[g2].s == s2) {
            groups[g2].blocks.push_back(hb);
            found = true;
          }
        if (!found) groups.push_back({L, s2, {hb}});
      }
    }
    if (worst > 0) {
      cleanup();
      drop();
      *overflow = worst;
      return DDST_ERANK;
    }
    // ---- pack factors
    H->bytes = store_elems * sizeof(F);
    HCHK(dev_malloc(&H->factors, std::max<size_t>(H->bytes, 16)));
    F *store = static_cast<F *>(H->factors);
    std::vector<LeafJob> lj;
    for (const HBlock &b : H->blocks)
      if (b.rank < 0)
        lj.push_back({Sptr(b.smat), b.r0, b.r1 - b.r0, (int)pad8(b.r1 - b.r0), (long long)b.off_u});
    if (!lj.empty()) {
      const LeafJob *d = static_cast<const LeafJob *>(upload(lj, st, keep));
      hipLaunchKernelGGL((k_pack_leaf<T, F>), dim3(64, (unsigned)lj.size()), dim3(256), 0, st,
                         d, d_perm, op->ld, store);
    }
    for (LevelData &D : levels) {
      const int nbk = (int)D.blocks.size();
      std::vector<PackJob> pj;
      for (int b = 0; b < nbk; ++b) {
        if (!D.kept[b]) continue;  // sampled again with more columns
        const HBlock &hb = D.blocks[b];
        pj.push_back({static_cast<double *>(D.Y->p) + D.offY[b], static_cast<double *>(D.XR->p) + D.offX[b],
                      static_cast<double *>(D.V->p) + (size_t)b * D.s * D.s, static_cast<int *>(D.sel->p) + D.selofs[b],
                      hb.r1 - hb.r0, hb.c1 - hb.c0, hb.rank, (long long)hb.off_u,
                      (long long)hb.off_v});
        H->blocks.push_back(hb);
      }
      if (pj.empty()) continue;
      size_t most = 1;  // entries of the largest job: one per thread
      for (const PackJob &j : pj)
        most = std::max(most, (size_t)j.m * j.rank + (size_t)j.rank * j.n);
      const unsigned gx = (unsigned)std::min<size_t>((most + 255) / 256, 4096);
      const PackJob *d = static_cast<const PackJob *>(upload(pj, st, keep));
      hipLaunchKernelGGL(k_pack<F>, dim3(gx, (unsigned)pj.size()), dim3(256), 0, st, d, D.s,
                         store);
    }
    HCHK(hipGetLastError());
    HCHK(hipStreamSynchronize(st));
    // ---- apply tables.  Transfer matrix sm = 2j (S_{j+1,j}, 0-based j here
    // means output interface sm/2 reading interface sm/2 - 1) or 2j+1
    // (reading sm/2 + 1).  For S^T, (S^T)_{a,b} = S_{b,a}^T: the block of
    // matrix sm is applied transposed from its output interface to its input.
    std::vector<LrJob> jobs;
    std::vector<Contrib> con;
    auto in_iface = [](int sm) { return (sm & 1) ? (sm >> 1) + 1 : (sm >> 1) - 1; };
    auto out_iface = [](int sm) { return sm >> 1; };
    for (int dir = 0; dir < 2; ++dir) {
      H->off_lr[dir].assign(H->nlev, 0);
      H->n_lr[dir].assign(H->nlev, 0);
      for (int L = -1; L < H->nlev; ++L) {
        std::vector<std::tuple<int, int, int, int>> keys;  // out iface, r0, r1, block
        for (size_t bi = 0; bi < H->blocks.size(); ++bi) {
          const HBlock &b = H->blocks[bi];
          if (b.level != L) continue;
          const int oi = dir ? in_iface(b.smat) : out_iface(b.smat);
          keys.push_back({oi, dir ? b.c0 : b.r0, dir ? b.c1 : b.r1, (int)bi});
        }
        std::sort(keys.begin(), keys.end());
        const size_t first_job = jobs.size();
        for (size_t k = 0; k < keys.size();) {
          size_t e = k;
          while (e < keys.size() && std::get<0>(keys[e]) == std::get<0>(keys[k]) &&
                 std::get<1>(keys[e]) == std::get<1>(keys[k]))
            ++e;
          LrJob jb{std::get<0>(keys[k]), std::get<1>(keys[k]), std::get<2>(keys[k]),
                   (int)con.size(), (int)(e - k)};
          for (size_t q = k; q < e; ++q) {
            const HBlock &b = H->blocks[std::get<3>(keys[q])];
            Contrib c{};
            c.in_iface = dir ? out_iface(b.smat) : in_iface(b.smat);
            c.c0 = dir ? b.r0 : b.c0;
            c.c1 = dir ? b.r1 : b.c1;
            c.rank = b.rank;
            c.off_u = (long long)b.off_u;
            c.off_v = (long long)b.off_v;
            c.trans = dir;
            con.push_back(c);
          }
          jobs.push_back(jb);
          k = e;
        }
        if (L < 0) {
          H->off_leaf[dir] = first_job;
          H->n_leaf[dir] = (int)(jobs.size() - first_job);
        } else {
          H->off_lr[dir][L] = first_job;
          H->n_lr[dir][L] = (int)(jobs.size() - first_job);
        }
      }
    }
    const size_t bytes_jobs = jobs.size() * sizeof(LrJob);
    H->off_con = (bytes_jobs + 255) & ~size_t(255);
    HCHK(dev_malloc(&H->jobs, H->off_con + std::max<size_t>(con.size(), 1) * sizeof(Contrib)));
    if (!jobs.empty())
      HCHK(hipMemcpyAsync(H->jobs, jobs.data(), bytes_jobs, hipMemcpyHostToDevice, st));
    if (!con.empty())
      HCHK(hipMemcpyAsync(static_cast<unsigned char *>(H->jobs) + H->off_con, con.data(),
                          con.size() * sizeof(Contrib), hipMemcpyHostToDevice, st));
    // ---- fused tables: every leaf job takes its own dense contributions and,
    // at each level, those of the job whose row cluster contains its rows
    // (their low-rank rows restricted to the leaf's)
    std::vector<LrJob> fj;
    std::vector<FContrib> fc;
    for (int dir = 0; dir < 2; ++dir) {
      H->foff[dir] = fj.size();
      for (int li = 0; li < H->n_leaf[dir]; ++li) {
        const LrJob &lf = jobs[H->off_leaf[dir] + li];
        LrJob f{lf.out_iface, lf.r0, lf.r1, (int)fc.size(), 0};
        auto add = [&](const LrJob &src, int roff, int rfull) {
          for (int q = 0; q < src.count; ++q) {
            const Contrib &c = con[src.first + q];
            FContrib x{};
            x.in_iface = c.in_iface;
            x.c0 = c.c0;
            x.c1 = c.c1;
            x.rank = c.rank;
            x.off_u = c.off_u;
            x.off_v = c.off_v;
            x.trans = c.trans;
            x.roff = roff;
            x.rfull = rfull;
            x.lds = (int)pad8(c.c1 - c.c0);
            fc.push_back(x);
          }
        };
        add(lf, 0, lf.r1 - lf.r0);
        for (int L = 0; L < H->nlev; ++L)
          for (int q = 0; q < H->n_lr[dir][L]; ++q) {
            const LrJob &lj = jobs[H->off_lr[dir][L] + q];
            if (lj.out_iface == lf.out_iface && lj.r0 <= lf.r0 && lf.r1 <= lj.r1)
              add(lj, lf.r0 - lj.r0, lj.r1 - lj.r0);
          }
        f.count = (int)fc.size() - f.first;
        fj.push_back(f);
      }
      H->fn[dir] = (int)(fj.size() - H->foff[dir]);
    }
    const size_t bytes_fj = fj.size() * sizeof(LrJob);
    H->foff_con = (bytes_fj + 255) & ~size_t(255);
    HCHK(dev_malloc(&H->fjobs, H->foff_con + std::max<size_t>(fc.size(), 1) * sizeof(FContrib)));
    if (!fj.empty())
      HCHK(hipMemcpyAsync(H->fjobs, fj.data(), bytes_fj, hipMemcpyHostToDevice, st));
    if (!fc.empty())
      HCHK(hipMemcpyAsync(static_cast<unsigned char *>(H->fjobs) + H->foff_con, fc.data(),
                          fc.size() * sizeof(FContrib), hipMemcpyHostToDevice, st));
    HCHK(hipStreamSynchronize(st));
    cleanup();
    if (H->min_rank > H->max_rank) H->min_rank = 0;
    hodlr_free(op);
    op->hodlr = H;
    return DDST_OK;
  } catch (...) {
    cleanup();
    drop();
    throw;
  }
}

}  // namespace

void hodlr_free(ddst_op *op) {
  if (!op || !op->hodlr) return;
  Hodlr *H = op->hodlr;
  if (H->d_perm) dev_free(H->d_perm);
  if (H->factors) dev_free(H->factors);
  if (H->jobs) dev_free(H->jobs);
  if (H->fjobs) dev_free(H->fjobs);
  if (H->pbuf) dev_free(H->pbuf);
  delete H;
  op->hodlr = nullptr;
}

bool hodlr_ready(const ddst_op *op) { return op && op->hodlr != nullptr; }

void hodlr_info(const ddst_op *op, double *bytes, int *max_rank, int *min_rank) {
  const Hodlr *H = op ? op->hodlr : nullptr;
  if (bytes) *bytes = H ? (double)H->bytes : 0.0;
  if (max_rank) *max_rank = H ? H->max_rank : 0;
  if (min_rank) *min_rank = H ? H->min_rank : 0;
}

int hodlr_compress(ddst_op *op, const ddst_compress_opts_t &o, hipStream_t s, int *overflow) {
  if (op->prec == DDST_FP32) {
    switch (o.factor_dtype) {
      case DDST_FACTOR_BF16: return compress_impl<float, unsigned short>(op, o, s, overflow);
      case DDST_FACTOR_FP32: return compress_impl<float, float>(op, o, s, overflow);
      default: return compress_impl<float, double>(op, o, s, overflow);
    }
  }
  switch (o.factor_dtype) {
    case DDST_FACTOR_BF16: return compress_impl<double, unsigned short>(op, o, s, overflow);
    case DDST_FACTOR_FP32: return compress_impl<double, float>(op, o, s, overflow);
    default: return compress_impl<double, double>(op, o, s, overflow);
  }
}

// y = S x (transpose 0) or S^T x (1) for padded interface vectors x, y
// (distinct buffers), through the compressed blocks.
void launch_gaussian(double *out, int rows, int s, uint64_t seed, unsigned stream_id,
                     hipStream_t st) {
  const size_t n = (size_t)rows * s;
  if (n == 0) return;
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, rows, s,
                     (unsigned long long)seed, (int)stream_id);
}

int hodlr_apply_jobs(const ddst_op *op, const double *x, double *y, int transpose,
                     hipStream_t s) {
  Hodlr *H = op->hodlr;
  if (!H) return DDST_ESTATE;
  const int dir = transpose ? 1 : 0;
  const size_t len = (size_t)op->n_ds * op->ld;
  const bool perm = H->d_perm != nullptr;
  double *xp = perm ? H->pbuf : nullptr;
  double *yp = perm ? H->pbuf + len : y;
  if (perm)
    hipLaunchKernelGGL(k_permute, dim3(nb(op->ld), op->n_ds), dim3(256), 0, s, x, xp, H->d_perm,
                       op->M, op->ld, 0);
  const double *xi = perm ? xp : x;
  const int nj = H->fn[dir];
  prof_begin(KK_GEMV, s);
  if (nj == 0) {  // one interface: no transfer blocks, S = I
    hipLaunchKernelGGL(k_copy_d, dim3(nb(len)), dim3(256), 0, s, xi, yp, len);
  } else {
    const LrJob *fj = static_cast<const LrJob *>(H->fjobs) + H->foff[dir];
    const FContrib *fc = reinterpret_cast<const FContrib *>(
        static_cast<const unsigned char *>(H->fjobs) + H->foff_con);
    switch (H->dtype) {
      case DDST_FACTOR_BF16:
        hipLaunchKernelGGL(k_hodlr_apply_fused<unsigned short>, dim3(nj), dim3(256), 0, s, fj, fc,
                           static_cast<const unsigned short *>(H->factors), xi, yp, op->ld,
                           op->M);
        break;
      case DDST_FACTOR_FP32:
        hipLaunchKernelGGL(k_hodlr_apply_fused<float>, dim3(nj), dim3(256), 0, s, fj, fc,
                           static_cast<const float *>(H->factors), xi, yp, op->ld, op->M);
        break;
      default:
        hipLaunchKernelGGL(k_hodlr_apply_fused<double>, dim3(nj), dim3(256), 0, s, fj, fc,
                           static_cast<const double *>(H->factors), xi, yp, op->ld, op->M);
    }
  }
  prof_end(KK_GEMV, s, (double)H->bytes);
  if (perm)
    hipLaunchKernelGGL(k_permute, dim3(nb(op->ld), op->n_ds), dim3(256), 0, s, yp, y, H->d_perm,
                       op->M, op->ld, 1);
  return hipGetLastError() == hipSuccess ? DDST_OK : DDST_EHIP;
}

}  // namespace ddst
