// Dense batched kernels of the transfer-block build (CDNA4 / gfx950).
//
// * k_assemble   : plane blocks D_k = A_plane - diag(r) G diag(c) [- ...]
//                  (the Schur complement recursion of block-tridiagonal
//                  elimination across the thin slab direction);
// * gj_invert    : in-place blocked Gauss-Jordan inversion without pivoting,
//                  kNB-wide pivot blocks; each step is a rank-kNB update done
//                  on the matrix cores (MFMA 16x16x4, FP32 or FP64);
// * k_gemm       : batched C = alpha A diag(s) B + beta C on the matrix cores
//                  (transfer chains Y_k = -G_k E Y_{k-1} and S = Sigma^{-1} R);
// * k_scale_cols : C = alpha A diag(s) (first link of a transfer chain).
//
// All matrices are ld x ld row-major, ld a multiple of 128, padded with the
// identity, so no kernel tests edges.  Work-group tiles are 128 x 128 with 4
// wavefronts of 64 lanes, each owning a 64 x 64 sub-tile (4 x 4 MFMA tiles).
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace ddst {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct AccT;
template <> struct AccT<float> { using type = f32x4; };
template <> struct AccT<double> { using type = f64x4; };

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int BK = 16;           // k-depth of one LDS stage
constexpr int LW = kTile + 16;   // LDS row width (padding spreads banks)

template <typename T>
__device__ __forceinline__ void ld8(const T *p, T *r) {
  constexpr int V = 16 / sizeof(T);
#pragma unroll
  for (int i = 0; i < 8 / V; ++i) {
    const typename V16<T>::type v = ld16(p + V * i);
#pragma unroll
    for (int e = 0; e < V; ++e) r[V * i + e] = v[e];
  }
}

// N consecutive elements (N * sizeof(T) a multiple of 16, p 16-byte aligned)
// with 16-byte loads.
template <int N, typename T>
__device__ __forceinline__ void ld16n(const T *p, T *r) {
  constexpr int V = 16 / sizeof(T);
  static_assert(N % V == 0, "whole 16-byte vectors");
#pragma unroll
  for (int i = 0; i < N / V; ++i) {
    const typename V16<T>::type v = ld16(p + V * i);
#pragma unroll
    for (int e = 0; e < V; ++e) r[V * i + e] = v[e];
  }
}

// Map the linear work-group id so that consecutive logical tiles land on
// the same XCD (work-groups are dispatched round-robin over the 8 XCDs):
// tiles of one batch entry then share one L2.  XCD x receives ids x, x + 8,
// ...; it is given the contiguous logical range starting at
// x q + min(x, rem) (total = 8 q + rem), a bijection for any total.
__device__ __forceinline__ int xcd_remap(int lin, int total) {
  const int x = lin & 7, k = lin >> 3, q = total >> 3, rem = total & 7;
  return x * q + (x < rem ? x : rem) + k;
}

template <typename T>
struct Tile {
  typename AccT<T>::type v[4][4];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[i][j][r] = T(0);
  }
};

// FP32 products on the BF16 matrix cores.  Every FP32 operand is split
// into three BF16 parts, x = x1 + x2 + x3 (x1 = bf16(x), x2 = bf16(x - x1),
// x3 = bf16(x - x1 - x2); each difference is exact in FP32 and the three
// parts carry the 24-bit significand), and a b is formed from the six
// products whose parts carry weight down to 2^-24 relative (a1 b1, a1 b2,
// a2 b1, a1 b3, a2 b2, a3 b1; the three dropped ones are below 2^-27),
// each exact in the FP32 accumulators of v_mfma_f32_16x16x32_bf16, added
// smallest first.  The result has the accuracy of an FP32 product; the
// BF16 matrix cores do the six products in 6 x 16 cycles per 16 x 16 x 32
// tile against 8 x 32 for the FP32 instruction (dense peaks 2.5 PFLOP/s
// BF16 and 157.3 TFLOP/s FP32).  FP32 operands are staged 32 deep.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
struct Split3 {
  bf16x8 h, m, l;
};
// Parts of eight FP32 values (x[j] = h[j] + m[j] + l[j] to 2^-26 relative).
// Pairs are rounded together (one packed conversion gives two BF16 values
// in one register); the FP32 value of a part is its BF16 bits moved to the
// upper half (a shift for the low element, a mask for the high one), so a
// pair costs three conversions, two shifts, two masks and four
// subtractions.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned cvt_pk(float a, float b) {
  const f32x2 v = {a, b};
  const bf16x2 p = __builtin_convertvector(v, bf16x2);
  return __builtin_bit_cast(unsigned, p);
}
__device__ __forceinline__ float lo_f(unsigned p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float hi_f(unsigned p) { return __uint_as_float(p & 0xffff0000u); }
__device__ __forceinline__ void split8(const float (&x)[8], Split3 &s) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 h, m, l;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float x0 = x[2 * j], x1 = x[2 * j + 1];
    const unsigned hp = cvt_pk(x0, x1);
    const float r0 = x0 - lo_f(hp), r1 = x1 - hi_f(hp);
    const unsigned mp = cvt_pk(r0, r1);
    const float q0 = r0 - lo_f(mp), q1 = r1 - hi_f(mp);
    h[j] = hp;
    m[j] = mp;
    l[j] = cvt_pk(q0, q1);
  }
  s.h = __builtin_bit_cast(bf16x8, h);
  s.m = __builtin_bit_cast(bf16x8, m);
  s.l = __builtin_bit_cast(bf16x8, l);
}
__device__ __forceinline__ f32x4 mfma_x6(const Split3 &a, const Split3 &b, f32x4 c) {
  c = mfma_bf16(a.l, b.h, c);
  c = mfma_bf16(a.m, b.m, c);
  c = mfma_bf16(a.h, b.l, c);
  c = mfma_bf16(a.m, b.h, c);
  c = mfma_bf16(a.h, b.m, c);
  return mfma_bf16(a.h, b.h, c);
}

// LDS of one tile product: FP64 operands staged 16 deep ([16][LW] each);
// FP32 operands as their three BF16 parts, 32 deep, in fragment order
// ([part][row or column][k], k contiguous, rows padded to 40 entries).
constexpr int XK = 2 * BK;       // 32: k per stage of the split products
constexpr int XKP = XK + 8;      // padded row of one BF16 part
template <typename T> struct MmaLds {
  static constexpr int bytes = 2 * BK * LW * (int)sizeof(T);
};
template <> struct MmaLds<float> {
  static constexpr int bytes = 2 * 3 * kTile * XKP * 2;
};

// acc += (NEG_A ? -A : A)[0:128, 0:K] * diag(bscale[0:K]) * B[0:K, 0:128]
// with FP32 operands on the BF16 matrix cores (split products above);
// layouts and arguments as mma_tile.  Each stage loads 32 k of both
// operands (a thread holds 16 values of one row of A and of one column of
// B), splits them once and stores the three parts in fragment order, so the
// product loop reads whole 8-element fragments (16 bytes) from LDS.
template <bool NEG_A, bool TA>
__device__ __forceinline__ void mma_tile_x6(const float *__restrict__ A, int lda,
                                            const float *__restrict__ B, int ldb,
                                            const double *__restrict__ bscale, int K,
                                            unsigned char *smem, Tile<float> &acc) {
  typedef __bf16 Part[kTile][XKP];
  Part *Ap = reinterpret_cast<Part *>(smem);         // Ap[part][row][k]
  Part *Bp = Ap + 3;                                 // Bp[part][col][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int rr = tid & (kTile - 1), kh = (tid >> 7) * 16;  // row / column, k half
  float ra[16], rb[16];
  auto load = [&](int k0) {
    if (TA) {
#pragma unroll
      for (int e = 0; e < 16; ++e) ra[e] = gp(A)[(size_t)(k0 + kh + e) * lda + rr];
    } else {
      ld8(A + (size_t)rr * lda + k0 + kh, ra);
      ld8(A + (size_t)rr * lda + k0 + kh + 8, ra + 8);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) rb[e] = gp(B)[(size_t)(k0 + kh + e) * ldb + rr];
    if (bscale) {
#pragma unroll
      for (int e = 0; e < 16; ++e) rb[e] *= (float)gp(bscale)[k0 + kh + e];
    }
  };
  auto store = [&](Part *P, const float (&x)[16], bool neg) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = neg ? -x[8 * hh + e] : x[8 * hh + e];
      Split3 sp;
      split8(v, sp);
      *reinterpret_cast<bf16x8 *>(&P[0][rr][kh + 8 * hh]) = sp.h;
      *reinterpret_cast<bf16x8 *>(&P[1][rr][kh + 8 * hh]) = sp.m;
      *reinterpret_cast<bf16x8 *>(&P[2][rr][kh + 8 * hh]) = sp.l;
    }
  };
  load(0);
  const int g = lane >> 4, c = lane & 15;
  for (int k0 = 0; k0 < K; k0 += XK) {
    __syncthreads();
    store(Ap, ra, NEG_A);
    store(Bp, rb, false);
    __syncthreads();
    if (k0 + XK < K) load(k0 + XK);
    // lane l holds row / column l % 16 of its tile and k = 8 (l / 16) + 0..7
    Split3 bs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wn + j * 16 + c;
      bs[j].h = *reinterpret_cast<const bf16x8 *>(&Bp[0][col][8 * g]);
      bs[j].m = *reinterpret_cast<const bf16x8 *>(&Bp[1][col][8 * g]);
      bs[j].l = *reinterpret_cast<const bf16x8 *>(&Bp[2][col][8 * g]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm + i * 16 + c;
      Split3 as;
      as.h = *reinterpret_cast<const bf16x8 *>(&Ap[0][row][8 * g]);
      as.m = *reinterpret_cast<const bf16x8 *>(&Ap[1][row][8 * g]);
      as.l = *reinterpret_cast<const bf16x8 *>(&Ap[2][row][8 * g]);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc.v[i][j] = mfma_x6(as, bs[j], acc.v[i][j]);
    }
  }
}

// acc += (NEG_A ? -A : A)[0:128, 0:K] * diag(bscale[0:K]) * B[0:K, 0:128]
// A row-major with leading dim lda (points at the tile's first row),
// B row-major with leading dim ldb (points at the tile's first column).
// TA: the operand is the transpose of a row-major matrix G, A[i][k] =
// G[k][i]; A then points at G's column of the tile's first row.
// FP32 operands go to mma_tile_x6 (BF16 matrix cores, 32-deep stages of
// stages), FP64 ones to the FP64 matrix cores (16 deep).
template <typename T, bool NEG_A = false, bool TA = false>
__device__ __forceinline__ void mma_tile(const T *__restrict__ A, int lda,
                                         const T *__restrict__ B, int ldb,
                                         const double *__restrict__ bscale, int K,
                                         T (*As)[LW], T (*Bs)[LW], Tile<T> &acc) {
  if constexpr (std::is_same<T, float>::value) {
    // As is the start of an MmaLds<float>::bytes buffer
    mma_tile_x6<NEG_A, TA>(A, lda, B, ldb, bscale, K, reinterpret_cast<unsigned char *>(As), acc);
    return;
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int ar = tid >> 1, ak = (tid & 1) * 8;    // A tile: 128 rows x 16
  const int br = tid >> 4, bc = (tid & 15) * 8;   // B tile: 16 rows x 128
  T ra[8], rb[8];
  auto load = [&](int k0) {
    if (TA)
      ld8(A + (size_t)(k0 + br) * lda + bc, ra);
    else
      ld8(A + (size_t)ar * lda + k0 + ak, ra);
    ld8(B + (size_t)(k0 + br) * ldb + bc, rb);
    if (bscale) {
      const T s = (T)gp(bscale)[k0 + br];
#pragma unroll
      for (int q = 0; q < 8; ++q) rb[q] *= s;
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    if (TA) {
#pragma unroll
      for (int q = 0; q < 8; ++q) As[br][bc + q] = NEG_A ? -ra[q] : ra[q];
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) As[ak + q][ar] = NEG_A ? -ra[q] : ra[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) Bs[br][bc + q] = rb[q];
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[4], b[4];
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kr][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc.v[i][j] = mfma16(a[i], b[j], acc.v[i][j]);
    }
  }
}

// Row / column of accumulator element (i, j, r) inside the 128 x 128 tile.
// Lane l holds column l % 16 of each 16 x 16 MFMA output; the row of
// register r is 4*(l/16) + r for the FP32 instruction and 4*r + l/16 for
// the FP64 one (measured on gfx950 with identity operands).
template <typename T>
__device__ __forceinline__ int acc_row(int i, int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int in16 = sizeof(T) == 4 ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4);
  return (wave >> 1) * 64 + i * 16 + in16;
}
__device__ __forceinline__ int acc_col(int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 64 + j * 16 + (lane & 15);
}

// FP64: at least two wavefronts per SIMD, as for the update
template <typename T>
__global__ __launch_bounds__(256, 2) void k_gemm(
    const GemmJob *__restrict__ jobs, int ld, int tiles_per_mat, T alpha, T beta) {
  __shared__ __align__(16) unsigned char smem[MmaLds<T>::bytes];
  T (*As)[LW] = reinterpret_cast<T (*)[LW]>(smem);
  T (*Bs)[LW] = As + BK;
  const int total = gridDim.x;
  const int lin = xcd_remap(blockIdx.x, total);
  const int b = lin / tiles_per_mat;
  const int t = lin % tiles_per_mat;
  const int nt = ld / kTile;
  const int bm = (t / nt) * kTile, bn = (t % nt) * kTile;
  const GemmJob J = jobs[b];
  const T *A = static_cast<const T *>(J.A);
  const T *B = static_cast<const T *>(J.B);
  auto *C = gp(static_cast<T *>(J.C));
  Tile<T> acc;
  acc.zero();
  mma_tile<T>(A + (size_t)bm * ld, ld, B + bn, ld, J.bscale, ld, As, Bs, acc);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t idx = (size_t)(bm + acc_row<T>(i, r)) * ld + bn + acc_col(j);
        T v = alpha * acc.v[i][j][r];
        if (beta != T(0)) v += beta * C[idx];
        C[idx] = v;
      }
}

// Broadcast lane src (wave-uniform) of a double to the whole wavefront.
__device__ __forceinline__ double bcast_lane(double x, int src) {
  const long long u = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Broadcast lane k (a compile-time constant after unrolling) of each
// 16-lane row to the whole row: DPP row_newbcast (gfx90a and later).
__device__ __forceinline__ int dpp_row_bcast(int x, int k) {
  switch (k) {
#define DDST_BC(K) \
  case K: return __builtin_amdgcn_update_dpp(0, x, 0x150 + K, 0xF, 0xF, false);
    DDST_BC(0) DDST_BC(1) DDST_BC(2) DDST_BC(3) DDST_BC(4) DDST_BC(5) DDST_BC(6) DDST_BC(7)
    DDST_BC(8) DDST_BC(9) DDST_BC(10) DDST_BC(11) DDST_BC(12) DDST_BC(13) DDST_BC(14)
    DDST_BC(15)
#undef DDST_BC
  }
  return 0;
}
__device__ __forceinline__ double row_bcast(double x, int k) {
  const long long u = __double_as_longlong(x);
  const unsigned lo = (unsigned)dpp_row_bcast((int)u, k);
  const unsigned hi = (unsigned)dpp_row_bcast((int)(u >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// In-place Gauss-Jordan inversion, without pivoting, of a 16 x 16 FP64 block
// held by one wavefront: lane l holds row l % 16, columns l / 16 + 4c in
// v[c].  That is the A-operand layout of four chained 16x16x4 FP64 MFMAs
// (v[c] feeds k = 4c + l / 16), so the inverse multiplies without a
// reshuffle.  Returns false if a pivot is not finite, or not positive
// unless ANY_SIGN (indefinite, nonsingular blocks).
template <bool ANY_SIGN>
__device__ __forceinline__ bool leaf_invert16(double (&v)[4]) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, g = l >> 4;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int kg = k & 3, kc = k >> 2;  // column k: lanes with g == kg, v[kc]
    const double colk = __shfl(v[kc], kg * 16 + i);  // P[i][k]
    double prow[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) prow[c] = row_bcast(v[c], k);  // P[k][g + 4c]
    const double piv = bcast_lane(v[kc], kg * 16 + k);
    ok = ok && isfinite(piv) && (ANY_SIGN ? piv != 0.0 : piv > 0.0);
    const double inv = 1.0 / piv;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const bool isk = (g == kg) && (c == kc);
      const double rk = isk ? inv : prow[c] * inv;  // new pivot row
      // other rows: P[i][j] - P[i][k] rk[j]; column k itself -P[i][k] / piv
      const double other = fma(-colk, rk, isk ? 0.0 : v[c]);
      v[c] = (i == k) ? rk : other;
    }
  }
  return ok;
}

// One Gauss-Jordan step, pivot part: one work-group (4 wavefronts) per
// matrix inverts the kNB x kNB (128 x 128) pivot block P = D[p, p] in FP64,
// without pivoting, and writes P^{-1} (row-major, rounded to T) to Pinv[b],
// the operand of the panel product.  FP64 throughout: the transfer blocks
// inherit the error of these inverses amplified by the conditioning of the
// interface Schur block.
//
// The block stays in registers for the whole inversion, as 16 x 16 tiles in
// the FP64 MFMA output layout: wave w owns column tiles 2w and 2w + 1 of all
// eight row tiles.  It is inverted by blocked Gauss-Jordan with 16-wide
// leaves.  Sub-step q: the row block q and the column block q go to LDS
// (double-buffered, one barrier per sub-step); every wave inverts the leaf
// P_qq itself (the same arithmetic in each wave, so no second barrier), forms
// R_J = P_qq^{-1} P_qJ for its column tiles and applies the rank-16 update
// to them on the matrix cores, with the tiles as accumulators:
//   row tile q:        T_qJ = R_J                   (R_q = P_qq^{-1})
//   column tile q:     T_Iq = -P_Iq P_qq^{-1}       (formed from zero)
//   others:            T_IJ = T_IJ - P_Iq R_J
// The MFMA output layout of R_J (row 4r + l / 16 in register r) is the
// B-operand layout of the update's k-step r, and the leaf layout is the
// A-operand layout, so no data moves between the two.  The sub-step loop is
// unrolled so that every tile index is static, and no vector ALU operation
// touches a tile.  The register cap keeps the whole work-group within about
// 190 registers per SIMD lane, so it can be placed on a CU next to the
// update and GEMM work-groups that run concurrently on other streams (a
// larger footprint waits for a CU to drain).
constexpr int kLeaf = 16;
constexpr int kCqS = 20;        // LDS row stride of the column block (doubles)
constexpr int kRqS = kNB + 16;  // LDS row stride of the row block (doubles)
static_assert(kNB == 128, "the register layout below assumes 128-wide pivots");

template <typename T, bool ANY_SIGN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_num_vgpr(96))) void k_gj_pivot(void *const *__restrict__ mats,
                                                  T *__restrict__ Pinv,
                                                  const T *__restrict__ Rprev,
                                                  const T *__restrict__ Cprev, int ld, int p,
                                                  int M, int *__restrict__ flag) {
  constexpr int kCqN = 2 * kNB * kCqS, kRqN = 2 * kLeaf * kRqS;
  __shared__ double lds[kCqN + kRqN];
  double (*Cq)[kNB][kCqS] = reinterpret_cast<double (*)[kNB][kCqS]>(lds);
  double (*Rq)[kLeaf][kRqS] = reinterpret_cast<double (*)[kLeaf][kRqS]>(lds + kCqN);
  const int b = blockIdx.x, l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = l >> 4, lc = l & 15;
  const auto *D = gp(static_cast<const T *>(mats[b]) + (size_t)p * kNB * ld + p * kNB);
  f64x4 t[8][2];  // t[I][jj][r] = P[16 I + 4 r + lr][16 (2 w + jj) + lc]
  auto load_block = [&]() {
#pragma unroll
    for (int I = 0; I < 8; ++I)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          t[I][jj][r] = (double)D[(size_t)(16 * I + 4 * r + lr) * ld + 16 * (2 * w + jj) + lc];
  };
  if (Rprev) {
    // The previous step's update of this block, P = D - Cprev[p] Rprev[:, p].
    // FP32: the arithmetic of the update kernel (products accumulated over k
    // in order from zero, subtracted once in FP32), so the block equals what
    // that kernel would have written; the A rows are fed permuted (row
    // 4 (i % 4) + i / 4 at position i) so that the accumulators come out in
    // the FP64 layout of t.  FP64: accumulated into the block itself (a
    // second set of FP64 accumulators would not fit next to it).  Operands
    // are staged through LDS in KS-deep slices.
    constexpr int KS = sizeof(T) == 4 ? 32 : 16;
    static_assert(2 * KS * LW * sizeof(T) <= sizeof(lds), "operand slices fit the LDS");
    T (*As)[LW] = reinterpret_cast<T (*)[LW]>(lds);
    T (*Bs)[LW] = reinterpret_cast<T (*)[LW]>(reinterpret_cast<T *>(lds) + KS * LW);
    const T *A = Cprev + (size_t)b * ld * kNB + (size_t)p * kNB * kNB;  // rows p, kNB wide
    const T *B = Rprev + (size_t)b * kNB * ld + p * kNB;               // kNB rows, cols p
    const int tid = threadIdx.x;
    constexpr int AE = kNB * KS / 256;  // A elements per thread (128 rows x KS)
    constexpr int BE = KS * kNB / 256;  // B elements per thread (KS rows x 128)
    const int ar = tid / (KS / AE), ak = (tid % (KS / AE)) * AE;
    const int bk = tid / (kNB / BE), bc = (tid % (kNB / BE)) * BE;
    const int arow = sizeof(T) == 4 ? 4 * (lc & 3) + (lc >> 2) : lc;
    auto product = [&](auto &C, T sign) {
      for (int k0 = 0; k0 < kNB; k0 += KS) {
        T ra[AE], rb[BE];
        ld16n<AE>(A + (size_t)ar * kNB + k0 + ak, ra);
        ld16n<BE>(B + (size_t)(k0 + bk) * ld + bc, rb);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < AE; ++e) As[ak + e][ar] = sign * ra[e];
#pragma unroll
        for (int e = 0; e < BE; ++e) Bs[bk][bc + e] = rb[e];
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KS; kk += 4) {
          T bv[2];
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) bv[jj] = Bs[kk + lr][16 * (2 * w + jj) + lc];
#pragma unroll
          for (int I = 0; I < 8; ++I) {
            const T av = As[kk + lr][16 * I + arow];
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) C[I][jj] = mfma16(av, bv[jj], C[I][jj]);
          }
        }
      }
      __syncthreads();  // the slices alias the blocks used below
    };
    if constexpr (sizeof(T) == 4) {
      f32x4 acc[8][2];
#pragma unroll
      for (int I = 0; I < 8; ++I)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[I][jj][r] = 0.f;
      product(acc, 1.f);
#pragma unroll
      for (int I = 0; I < 8; ++I)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float d = D[(size_t)(16 * I + 4 * r + lr) * ld + 16 * (2 * w + jj) + lc];
            t[I][jj][r] = (double)(d - acc[I][jj][r]);
          }
    } else {
      load_block();
      product(t, -1.0);
    }
  } else {
    load_block();
  }
  bool ok = true;
#pragma unroll
  for (int q = 0; q < kNB / kLeaf; ++q) {
    const int buf = q & 1, qj = q & 1;
    const bool owner = w == (q >> 1);  // this wave holds column tile q (as jj = qj)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) Rq[buf][4 * r + lr][16 * (2 * w + jj) + lc] = t[q][jj][r];
    if (owner) {
#pragma unroll
      for (int I = 0; I < 8; ++I)
#pragma unroll
        for (int r = 0; r < 4; ++r) Cq[buf][16 * I + 4 * r + lr][lc] = t[I][qj][r];
    }
    __syncthreads();
    double v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = Rq[buf][lc][16 * q + lr + 4 * c];
    ok = leaf_invert16<ANY_SIGN>(v) && ok;
    f64x4 R[2];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const bool pc = owner && jj == qj;
#pragma unroll
      for (int r = 0; r < 4; ++r) R[jj][r] = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double id = 4 * s + lr == lc ? 1.0 : 0.0;
        const double bs = pc ? id : Rq[buf][4 * s + lr][16 * (2 * w + jj) + lc];
        R[jj] = mfma16(v[s], bs, R[jj]);
      }
    }
#pragma unroll
    for (int I = 0; I < 8; ++I) {
      if (I == q) continue;
      double a[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) a[s] = -Cq[buf][16 * I + lc][4 * s + lr];
#pragma unroll
      for (int s = 0; s < 4; ++s) t[I][1 - qj] = mfma16(a[s], R[1 - qj][s], t[I][1 - qj]);
      if (owner) {  // pivot-column tile, formed from zero
        f64x4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) z = mfma16(a[s], R[qj][s], z);
        t[I][qj] = z;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) t[I][qj] = mfma16(a[s], R[qj][s], t[I][qj]);
      }
    }
    t[q][0] = R[0];
    t[q][1] = R[1];
  }
  if (!ok && threadIdx.x == 0) atomicOr(flag, 1);
  T *out = Pinv + (size_t)b * kNB * kNB;
  // largest |entry| of the inverse outside the identity padding (rows and
  // columns >= M), for the pivot growth
  double amax = 0.0;
  const int lim = M - p * kNB;  // local rows / columns below M
#pragma unroll
  for (int I = 0; I < 8; ++I)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * I + 4 * r + lr, col = 16 * (2 * w + jj) + lc;
        out[row * kNB + col] = (T)t[I][jj][r];
        if (row < lim && col < lim) amax = fmax(amax, fabs(t[I][jj][r]));
      }
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  if (l == 0)
    atomicMax(reinterpret_cast<unsigned long long *>(flag) + 1,
              (unsigned long long)__double_as_longlong(amax));
}

// One Gauss-Jordan step, panel part.  Work-group (jt, b), 4 wavefronts,
// for the 128 columns j0 = 128 jt:
//  * R[:, j0..j0+127] = P^{-1} D[p, j0..j0+127], a 128 x 128 x 128 product
//    on the matrix cores through the LDS-staged tile routine (R = P^{-1}
//    itself on the pivot block);
//  * Cbuf[j0..j0+127, :] = D[j0..j0+127, p] (copy of the old pivot columns)
//    when copy_c is set; after the first step the update that produced
//    column block p writes this copy itself.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_gj_panel(void *const *__restrict__ mats,
                                                  const T *__restrict__ Pinv,
                                                  T *__restrict__ Rbuf, T *__restrict__ Cbuf,
                                                  int ld, int p, int copy_c) {
  __shared__ __align__(16) unsigned char smem[MmaLds<T>::bytes];
  T (*As)[LW] = reinterpret_cast<T (*)[LW]>(smem);
  T (*Bs)[LW] = As + BK;
  const int b = blockIdx.y, jt = blockIdx.x, tid = threadIdx.x;
  const T *D = static_cast<const T *>(mats[b]);
  T *R = Rbuf + (size_t)b * kNB * ld;
  T *Cb = Cbuf + (size_t)b * ld * kNB;
  const T *Pi = Pinv + (size_t)b * kNB * kNB;
  const int p0 = p * kNB, j0 = jt * kTile;
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte access
  for (int e = tid * V; copy_c && e < kTile * kNB; e += 256 * V) {
    const int r = e / kNB, c = e % kNB;
    st16(Cb + (size_t)(j0 + r) * kNB + c, ld16(D + (size_t)(j0 + r) * ld + p0 + c));
  }
  if (jt == p) {
    for (int e = tid * V; e < kNB * kTile; e += 256 * V) {
      const int r = e / kTile, c = e % kTile;
      st16(R + (size_t)r * ld + j0 + c, ld16(Pi + r * kNB + c));
    }
    return;
  }
  Tile<T> acc;
  acc.zero();
  mma_tile<T>(Pi, kNB, D + (size_t)p0 * ld + j0, ld, nullptr, kNB, As, Bs, acc);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        R[(size_t)acc_row<T>(i, r) * ld + j0 + acc_col(j)] = acc.v[i][j][r];
}

// (i, j) of the t-th tile of a lower triangle of tiles, in row order
__device__ __forceinline__ void tri_index(int t, int &i, int &j) {
  int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (r > 0 && r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  i = r;
  j = t - r * (r + 1) / 2;
}

// Transposed copy of a 128 x 128 tile through LDS, 32 source rows at a
// time: dst[r][c] = sg * src[c][r] (src row-major with leading dim lds_,
// dst with leading dim ldd).  X: 32 x (kTile + 1) elements of LDS.
template <typename T>
__device__ __forceinline__ void tile_transpose(const T *__restrict__ src, int lds_,
                                               T *__restrict__ dst, int ldd, T sg,
                                               T (*X)[kTile + 1]) {
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < kTile; c0 += 32) {
    __syncthreads();
    for (int e = tid; e < 32 * kTile; e += 256) {
      const int rr = e / kTile, cc = e % kTile;
      X[rr][cc] = gp(src)[(size_t)(c0 + rr) * lds_ + cc];
    }
    __syncthreads();
    for (int e = tid; e < kTile * 32; e += 256) {
      const int r = e / 32, cc = e % 32;
      gp(dst)[(size_t)r * ldd + c0 + cc] = sg * X[cc][r];
    }
  }
  __syncthreads();
}

// One step of the symmetric elimination, panel part (the general update's
// layout; see k_gj_update).  Work-group (it, b) takes row block i = it:
//  * i == p: Rbuf[:, p] = P^{-1};
//  * otherwise C_i = D[i, p] (i > p) or -D[p, i]^T (i < p), read from the
//    lower triangle, is copied to Cbuf rows i (the operand of the update,
//    which overwrites column and row block p), and W_i = C_i P^{-1} is
//    formed on the matrix cores and written transposed to Rbuf[:, i].
template <typename T>
__global__ __launch_bounds__(256, 2) void k_gj_panel_sym(void *const *__restrict__ mats,
                                                      const T *__restrict__ Pinv,
                                                      T *__restrict__ Rbuf, T *__restrict__ Cbuf,
                                                      int ld, int p) {
  __shared__ __align__(16) unsigned char smem[MmaLds<T>::bytes];
  static_assert(32 * (kTile + 1) * sizeof(T) <= MmaLds<T>::bytes, "transpose chunk fits");
  T (*As)[LW] = reinterpret_cast<T (*)[LW]>(smem);
  T (*Bs)[LW] = As + BK;
  const int b = blockIdx.y, it = blockIdx.x, tid = threadIdx.x;
  const T *D = static_cast<const T *>(mats[b]);
  T *R = Rbuf + (size_t)b * kNB * ld;
  T *Cb = Cbuf + (size_t)b * ld * kNB;
  const T *Pi = Pinv + (size_t)b * kNB * kNB;
  const int p0 = p * kNB, i0 = it * kTile;
  constexpr int V = 16 / sizeof(T);
  if (it == p) {
    for (int e = tid * V; e < kNB * kTile; e += 256 * V) {
      const int r = e / kTile, c = e % kTile;
      st16(R + (size_t)r * ld + p0 + c, ld16(Pi + r * kNB + c));
    }
    return;
  }
  Tile<T> acc;
  acc.zero();
  if (it > p)
    mma_tile<T>(D + (size_t)i0 * ld + p0, ld, Pi, kNB, nullptr, kNB, As, Bs, acc);
  else
    mma_tile<T, true, true>(D + (size_t)p0 * ld + i0, ld, Pi, kNB, nullptr, kNB, As, Bs, acc);
  // Rbuf[c][i0 + r] = W_i[r][c]
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        R[(size_t)acc_col(j) * ld + i0 + acc_row<T>(i, r)] = acc.v[i][j][r];
  if (it > p) {
    for (int e = tid * V; e < kTile * kNB; e += 256 * V) {
      const int r = e / kNB, c = e % kNB;
      st16(Cb + (size_t)(i0 + r) * kNB + c, ld16(D + (size_t)(i0 + r) * ld + p0 + c));
    }
  } else {
    __syncthreads();  // the product's LDS is reused
    tile_transpose<T>(D + (size_t)p0 * ld + i0, ld, Cb + (size_t)i0 * kNB, kNB, T(-1),
                      reinterpret_cast<T (*)[kTile + 1]>(smem));
  }
}

// Diagonal tiles made exactly symmetric from their lower triangle, before a
// symmetric elimination: work-group (t, b) mirrors tile (t, t) of matrix b.
// The elimination reads only lower tiles and assumes symmetry; an input whose
// diagonal tiles carry rounding asymmetry (the previous plane's inverse
// after the Schur update) is then inverted inconsistently, and along a sweep
// of an indefinite problem that error grows geometrically with the planes.
template <typename T>
__global__ __launch_bounds__(256) void k_sym_diag(void *const *__restrict__ mats, int ld) {
  __shared__ T X[32][kTile + 1];
  T *D = static_cast<T *>(mats[blockIdx.y]) + (size_t)blockIdx.x * kTile * (ld + 1);
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < kTile; c0 += 32) {
    __syncthreads();
    for (int e = tid; e < 32 * kTile; e += 256) {
      const int rr = e / kTile, cc = e % kTile;
      X[rr][cc] = gp(D)[(size_t)(c0 + rr) * ld + cc];
    }
    __syncthreads();
    // rows of later chunks are not written (r < c0 + cc <= c0 + 31)
    for (int e = tid; e < kTile * 32; e += 256) {
      const int r = e / 32, cc = e % 32;
      if (c0 + cc > r) gp(D)[(size_t)r * ld + c0 + cc] = X[cc][r];
    }
  }
}

// Upper triangle of every matrix from its lower triangle (the inverse left
// by the symmetric elimination is symmetric): work-group (t, b) copies the
// transpose of the t-th tile strictly below the diagonal to its mirror.
template <typename T>
__global__ __launch_bounds__(256) void k_mirror_lower(void *const *__restrict__ mats, int ld) {
  __shared__ T X[32][kTile + 1];
  T *D = static_cast<T *>(mats[blockIdx.y]);
  int ti, tj;
  tri_index(blockIdx.x, ti, tj);
  ti += 1;  // strictly lower: the t-th tile of the triangle of nt - 1 rows, shifted
  tile_transpose<T>(D + (size_t)ti * kTile * ld + tj * kTile, ld,
                    D + (size_t)tj * kTile * ld + ti * kTile, ld, T(1), X);
}

// One Gauss-Jordan step, update part (Cbuf = old column p, R = P^{-1} D[p,:]):
//   pivot rows               D[p, :] = R             (P^{-1} on the block p)
//   other rows, column p     D[i, p] = -D[i, p] P^{-1}
//   other rows, other cols   D[i, j] -= D[i, p] P^{-1} D[p, j]
// The 128 x 128 tile of D is read and written with 16-byte accesses, each
// wavefront covering whole rows (VEC elements per lane).  It is read after
// the product, half a tile at a time, and the MFMA accumulators are
// exchanged into its row layout through LDS (64 rows, the two wavefronts
// holding them write, all four read; the operand stages live in the same
// buffer).  Keeping D out of registers during the product and the LDS
// buffer at 34 KB lets four work-groups share a CU (FP32), whose products
// hide each other's D latency.  With Cnext, tiles of column block p + 1 are
// also written to the next step's column panel.  The product is formed from
// zero and subtracted once, keeping the rounding at the scale of the update
// rather than of D; the pivot column is written as -acc rather than
// D - (D + D P^{-1}), which would add O(1) to O(|P^{-1}|) entries.
template <typename T> struct UpdGeom;
template <> struct UpdGeom<float> {
  static constexpr int VEC = 4;     // floats per 16-byte access
  static constexpr int RPI = 8;     // rows covered by one pass of 256 threads
  static constexpr int NQ = 16;     // passes per tile (128 / RPI)
};
template <> struct UpdGeom<double> {
  static constexpr int VEC = 2;
  static constexpr int RPI = 4;
  static constexpr int NQ = 32;
};

// Tile subsets of one update (q = p + 1, the next pivot block): all tiles
// (last step); the row and column blocks of q without the tile (q, q)
// (whose update the next pivot kernel does itself); everything outside
// them.
enum { kSelAll = 0, kSelCross = 1, kSelRest = 2 };
__host__ __device__ inline int sel_tiles(int sel, int nt) {
  return sel == kSelAll ? nt * nt : sel == kSelCross ? 2 * nt - 2 : (nt - 1) * (nt - 1);
}
__device__ __forceinline__ void sel_tile(int sel, int nt, int q, int t, int &tr, int &tc) {
  if (sel == kSelAll) {
    tr = t / nt;
    tc = t % nt;
  } else if (sel == kSelCross) {  // row block q, then column block q, both without (q, q)
    if (t < nt - 1) {
      tr = q;
      tc = t + (t >= q);
    } else {
      const int u = t - (nt - 1);
      tr = u + (u >= q);
      tc = q;
    }
  } else {  // everything outside row and column block q
    tr = t / (nt - 1);
    tc = t % (nt - 1);
    tr += tr >= q;
    tc += tc >= q;
  }
}

// Tile subsets of the symmetric elimination, which updates only the lower
// triangle of tiles (tr >= tc): all of them (last step); row block q left of
// (q, q) and column block q below it; everything outside row and column
// block q.
__host__ __device__ inline int sel_tiles_sym(int sel, int nt) {
  return sel == kSelAll ? nt * (nt + 1) / 2 : sel == kSelCross ? nt - 1 : (nt - 1) * nt / 2;
}
__device__ __forceinline__ void sel_tile_sym(int sel, int nt, int q, int t, int &tr, int &tc) {
  if (sel == kSelAll) {
    tri_index(t, tr, tc);
  } else if (sel == kSelCross) {  // (q, 0..q-1), then (q+1..nt-1, q)
    if (t < q) {
      tr = q;
      tc = t;
    } else {
      tr = t + 1;
      tc = q;
    }
  } else {  // the lower triangle of the nt - 1 blocks other than q
    tri_index(t, tr, tc);
    tr += tr >= q;
    tc += tc >= q;
  }
}

// FP64: at least two wavefronts per SIMD (its accumulators would otherwise
// take the register file of two)
//
// SYM: the symmetric elimination (a symmetric matrix, Gauss-Jordan without
// pivoting in block order).  After the steps 0..p-1 the matrix is
//   [ A_SS^{-1}              A_SS^{-1} A_SN          ]
//   [ -A_NS A_SS^{-1}        A_NN - A_NS A_SS^{-1} A_SN ]
// (S the eliminated blocks, N the others): its SS and NN parts are
// symmetric and NS = -(SN)^T, so the lower triangle of tiles determines it.
// With C_i the current column block p (C_i = D[i, p] for i > p, -D[p, i]^T
// for i < p) and W_i = C_i P^{-1}, a step is, on lower tiles only:
//   D[i, j] -= s_j C_i W_j^T  (s_j = +1 for j > p, -1 for j < p)
//   D[i, p] = -W_i (i > p),  D[p, j] = -W_j^T (j < p),  D[p, p] = P^{-1}
// Rbuf holds W^T (kNB x ld, W_p^T taken as P^{-1}), so every product is the
// one of the general update, only its sign and the pivot-row copy differ.
template <typename T, bool SYM>
__global__ __launch_bounds__(256, 2) void k_gj_update(
    void *const *__restrict__ mats,
                                                   const T *__restrict__ Rbuf,
                                                   const T *__restrict__ Cbuf,
                                                   T *__restrict__ Cnext, int ld, int p,
                                                   int sel) {
  using G = UpdGeom<T>;
  constexpr int XW = kTile + 4;  // exchange row width
  constexpr int HR = kTile / 2;  // rows per exchange half
  // the staging buffers of the product live inside the exchange buffer
  constexpr int LDSN = HR * XW * (int)sizeof(T) > MmaLds<T>::bytes ? HR * XW * (int)sizeof(T)
                                                                    : MmaLds<T>::bytes;
  __shared__ __align__(16) unsigned char smem[LDSN];
  T *lds = reinterpret_cast<T *>(smem);
  T (*As)[LW] = reinterpret_cast<T (*)[LW]>(lds);
  T (*Bs)[LW] = As + BK;
  T (*Xs)[XW] = reinterpret_cast<T (*)[XW]>(lds);
  const int nt = ld / kTile;
  const int tiles_per_mat = SYM ? sel_tiles_sym(sel, nt) : sel_tiles(sel, nt);
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int b = lin / tiles_per_mat;
  int tr, tc;
  if (SYM)
    sel_tile_sym(sel, nt, p + 1, lin % tiles_per_mat, tr, tc);
  else
    sel_tile(sel, nt, p + 1, lin % tiles_per_mat, tr, tc);
  const int bm = tr * kTile, bn = tc * kTile;
  T *D = static_cast<T *>(mats[b]);
  const T *R = Rbuf + (size_t)b * kNB * ld;
  const T *Cb = Cbuf + (size_t)b * ld * kNB;
  const int p0 = p * kNB;
  const int tid = threadIdx.x;
  constexpr int LPR = kTile / G::VEC;           // lanes per row
  const int trow = tid / LPR, tcol = (tid % LPR) * G::VEC;
  using VT = typename V16<T>::type;
  // tiles of column block p + 1 also go to the next step's column panel
  T *Cn = (!SYM && Cnext && bn == p0 + kNB) ? Cnext + (size_t)b * ld * kNB : nullptr;
  if (bm == p0) {  // pivot rows: D[p, :] = R (SYM: -W^T left of the pivot), no product
    const T sg = (SYM && bn < p0) ? T(-1) : T(1);
#pragma unroll
    for (int q = 0; q < G::NQ; ++q) {
      const int row = bm + q * G::RPI + trow;
      VT v = ld16(R + (size_t)(row - p0) * ld + bn + tcol);
#pragma unroll
      for (int e = 0; e < G::VEC; ++e) v[e] *= sg;
      st16(D + (size_t)row * ld + bn + tcol, v);
      if (Cn) st16(Cn + (size_t)row * kNB + tcol, v);
    }
    return;
  }
  Tile<T> acc;
  acc.zero();
  mma_tile<T>(Cb + (size_t)bm * kNB, kNB, R + bn, ld, nullptr, kNB, As, Bs, acc);
  const bool pivcols = (bn + tcol >= p0) && (bn + tcol < p0 + kNB);
  const bool plus = SYM && bn < p0;  // s_j = -1: the product is added
  const int wave = tid >> 6;
  constexpr int NH = G::NQ / 2;  // row passes per half
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    VT dv[NH];
#pragma unroll
    for (int q = 0; q < NH; ++q)
      dv[q] = ld16(D + (size_t)(bm + h * HR + q * G::RPI + trow) * ld + bn + tcol);
    __syncthreads();
    if ((wave >> 1) == h) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Xs[acc_row<T>(i, r) - h * HR][acc_col(j)] = acc.v[i][j][r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      const int lrow = q * G::RPI + trow;
      VT v;
#pragma unroll
      for (int e = 0; e < G::VEC; ++e)
        v[e] = (pivcols ? T(0) : dv[q][e]) + (plus ? Xs[lrow][tcol + e] : -Xs[lrow][tcol + e]);
      st16(D + (size_t)(bm + h * HR + lrow) * ld + bn + tcol, v);
      if (Cn) st16(Cn + (size_t)(bm + h * HR + lrow) * kNB + tcol, v);
    }
  }
}

// D = A_plane - diag(r1) G1 diag(c1) - diag(r2) G2 diag(c2).  Streams G
// and D once (HBM-bound): work-group (x, b) covers kAsmRows rows of job b,
// each thread V consecutive columns with 16-byte loads and stores; the
// column scales are read once per thread and reused over the rows.
constexpr int kAsmRows = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_assemble(const AsmJob *__restrict__ jobs,
                                                  const double *__restrict__ coef, int n,
                                                  int dim, int M, int ld) {
  constexpr int V = 16 / sizeof(T);
  using VT = typename V16<T>::type;
  const AsmJob J = jobs[blockIdx.y];
  const size_t N = (size_t)M * n;
  const T *G1 = static_cast<const T *>(J.G1);
  const T *G2 = static_cast<const T *>(J.G2);
  for (int c0 = threadIdx.x * V; c0 < ld; c0 += 256 * V) {
    double sc1[V], sc2[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const bool in = c0 + e < M;
      sc1[e] = (G1 && in) ? gp(J.c1)[c0 + e] : 0.0;
      sc2[e] = (G2 && in) ? gp(J.c2)[c0 + e] : 0.0;
    }
#pragma unroll
    for (int rr = 0; rr < kAsmRows; ++rr) {
      const int r = blockIdx.x * kAsmRows + rr;
      T out[V];
      if (r >= M) {
#pragma unroll
        for (int e = 0; e < V; ++e) out[e] = (c0 + e == r) ? T(1) : T(0);
      } else {
        VT g1 = {}, g2 = {};
        if (G1) g1 = ld16(G1 + (size_t)r * ld + c0);
        if (G2) g2 = ld16(G2 + (size_t)r * ld + c0);
        const double s1 = G1 ? gp(J.r1)[r] : 0.0;
        const double s2 = G2 ? gp(J.r2)[r] : 0.0;
        double v[V];
#pragma unroll
        for (int e = 0; e < V; ++e)
          v[e] = c0 + e < M ? -s1 * (double)g1[e] * sc1[e] - s2 * (double)g2[e] * sc2[e] : 0.0;
        // in-plane stencil entries of row r (boundary neighbours are not in A_plane)
        const size_t node = (size_t)(J.plane - 1) * M + r;
        auto add = [&](int col, double val) {
          if (col >= c0 && col < c0 + V) {
#pragma unroll
            for (int e = 0; e < V; ++e)
              if (c0 + e == col) v[e] += val;
          }
        };
        add(r, coef[node]);
        if (dim == 2) {
          if (r >= 1) add(r - 1, coef[3 * N + node]);
          if (r <= n - 2) add(r + 1, coef[4 * N + node]);
        } else {
          const int y = r / n, z = r % n;
          if (y >= 1) add(r - n, coef[3 * N + node]);
          if (y <= n - 2) add(r + n, coef[4 * N + node]);
          if (z >= 1) add(r - 1, coef[5 * N + node]);
          if (z <= n - 2) add(r + 1, coef[6 * N + node]);
        }
#pragma unroll
        for (int e = 0; e < V; ++e) out[e] = (T)v[e];
      }
      VT o;
#pragma unroll
      for (int e = 0; e < V; ++e) o[e] = out[e];
      st16(static_cast<T *>(J.D) + (size_t)r * ld + c0, o);
    }
  }
}

// C = alpha * A * diag(s), one block per row.
// Products of the sampling chains: C (ld x ldc) = alpha op(A) diag(bscale) B
// + beta C with A ld x ld (op(A) = A, or A^T when TRANS), B and C ld x ldc
// (ldc a multiple of 128), all row-major; 128 x 128 output tiles as k_gemm.
template <typename T, bool TRANS>
__global__ __launch_bounds__(256, 2) void k_gemm_rect(
    const GemmJob *__restrict__ jobs, int ld, int ldc, int tiles_per_job, T alpha, T beta) {
  __shared__ __align__(16) unsigned char smem[MmaLds<T>::bytes];
  T (*As)[LW] = reinterpret_cast<T (*)[LW]>(smem);
  T (*Bs)[LW] = As + BK;
  const int total = gridDim.x;
  const int lin = xcd_remap(blockIdx.x, total);
  const int b = lin / tiles_per_job;
  const int t = lin % tiles_per_job;
  const int ntc = ldc / kTile;
  const int bm = (t / ntc) * kTile, bn = (t % ntc) * kTile;
  const GemmJob J = jobs[b];
  const T *A = static_cast<const T *>(J.A);
  const T *B = static_cast<const T *>(J.B);
  auto *C = gp(static_cast<T *>(J.C));
  Tile<T> acc;
  acc.zero();
  if (TRANS)
    mma_tile<T, false, true>(A + bm, ld, B + bn, ldc, J.bscale, ld, As, Bs, acc);
  else
    mma_tile<T>(A + (size_t)bm * ld, ld, B + bn, ldc, J.bscale, ld, As, Bs, acc);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t idx = (size_t)(bm + acc_row<T>(i, r)) * ldc + bn + acc_col(j);
        T v = alpha * acc.v[i][j][r];
        if (beta != T(0)) v += beta * C[idx];
        C[idx] = v;
      }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale_cols(const GemmJob *__restrict__ jobs, int ld,
                                                    T alpha) {
  const GemmJob J = jobs[blockIdx.y];
  const int r = blockIdx.x;
  const auto *A = gp(static_cast<const T *>(J.A) + (size_t)r * ld);
  auto *C = gp(static_cast<T *>(J.C) + (size_t)r * ld);
  for (int c = threadIdx.x; c < ld; c += blockDim.x)
    C[c] = alpha * A[c] * (T)gp(J.bscale)[c];
}

}  // namespace

template <typename T>
void launch_assemble(const AsmJob *jobs, int njobs, const double *coef, int n, int dim,
                     int M, int ld, hipStream_t s) {
  if (njobs <= 0) return;
  const ProfSpan ps = prof_open(KK_ASSEMBLE);
  hipExtLaunchKernelGGL(k_assemble<T>, dim3(ld / kAsmRows, njobs), dim3(256), 0, s, ps.a, ps.b,
                        0, jobs, coef, n, dim, M, ld);
  // reads G (and up to one more) and writes D: 2 M^2 elements per job
  prof_close(ps, KK_ASSEMBLE, 2.0 * njobs * (double)M * M * sizeof(T));
}

template <typename T>
void launch_scale_cols(const GemmJob *jobs, int njobs, int ld, double alpha, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_scale_cols<T>, dim3(ld, njobs), dim3(256), 0, s, jobs, ld, (T)alpha);
}

template <typename T>
void launch_gemm(const GemmJob *jobs, int njobs, int ld, int M, double alpha, double beta,
                 hipStream_t s) {
  if (njobs <= 0) return;
  const int tpm = (ld / kTile) * (ld / kTile);
  const ProfSpan ps = prof_open(KK_GEMM);
  hipExtLaunchKernelGGL(k_gemm<T>, dim3(tpm * njobs), dim3(256), 0, s, ps.a, ps.b, 0, jobs, ld,
                        tpm, (T)alpha, (T)beta);
  prof_close(ps, KK_GEMM, 2.0 * njobs * (double)M * M * M);
}

template <typename T>
void launch_gemm_rect(const GemmJob *jobs, int njobs, int ld, int ldc, int M, int ncols,
                      int trans, double alpha, double beta, hipStream_t s) {
  if (njobs <= 0) return;
  const int tpj = (ld / kTile) * (ldc / kTile);
  const ProfSpan ps = prof_open(KK_GEMM);
  hipExtLaunchKernelGGL(trans ? k_gemm_rect<T, true> : k_gemm_rect<T, false>, dim3(tpj * njobs),
                        dim3(256), 0, s, ps.a, ps.b, 0, jobs, ld, ldc, tpj, (T)alpha, (T)beta);
  prof_close(ps, KK_GEMM, 2.0 * njobs * (double)M * M * ncols);
}

hipError_t GjStreams::create() {
  hipError_t e = hipStreamCreateWithFlags(&h, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
  for (hipEvent_t *ev : {&panel, &rest[0], &rest[1], &cross[0], &cross[1]})
    if (e == hipSuccess)
      e = hipEventCreateWithFlags(ev, hipEventDisableTiming | hipEventDisableSystemFence);
  return e;
}

GjStreams::~GjStreams() {
  for (hipStream_t st : {h, x})
    if (st) (void)hipStreamSynchronize(st);
  for (hipEvent_t ev : {panel, rest[0], rest[1], cross[0], cross[1]})
    if (ev) (void)hipEventDestroy(ev);
  for (hipStream_t st : {h, x})
    if (st) (void)hipStreamDestroy(st);
}

// Schedule of one inversion (q = p + 1; buffers of step p: R, Cbuf index
// p & 1; Ux(p) = the tiles of row and column block q except (q, q), Ur(p) =
// all tiles outside them):
//   s   : pivot(0) panel(0) | pivot(1) . panel(1) | pivot(2) . panel(2) ...
//   gs.x:                     Ux(0)                 Ux(1)
//   gs.h:                     Ur(0)                 Ur(1) ...
// pivot(q) first applies step p's update to the block (q, q) itself, so the
// next pivot is inverted while the other tiles are updated; Ux(p), which
// the panel of step q needs, runs beside the larger Ur(p) rather than before
// it.  Ux(p) also writes column block q to the column panel of step q.
// Dependencies: Ux(p) and Ur(p) wait for panel(p); Ux(p) and pivot(q) wait
// for Ur(p - 1) (which last wrote their tiles and read the buffers that
// Ux(p) and panel(q) overwrite); Ur(p) waits for Ux(p - 1) (same reason);
// panel(q) waits for Ux(p).  The last step updates all tiles on s.
//
// sym: the matrices are symmetric; the updates touch only the lower
// triangle of tiles (about half the work, see k_gj_update), the panel
// kernel forms C and W^T from it, and one last launch mirrors the lower
// triangle of the (symmetric) inverse into the upper one.  The pivot
// kernel is the same: W_q^T is the block q of its R operand.
template <typename T>
hipError_t gj_invert(void *const *mats, int nmat, int ld, int M, void *work, int *flag,
                     int any_sign, int sym, GjStreams &gs, hipStream_t s) {
  if (nmat <= 0) return hipSuccess;
  static_assert(kNB == kTile, "one pivot block per tile row");
  const int nt = ld / kTile;
  const size_t pan = (size_t)nmat * kNB * ld;
  T *w = static_cast<T *>(work);
  T *Rb[2] = {w, w + 2 * pan}, *Cb[2] = {w + pan, w + 3 * pan};
  T *PinvT = w + 4 * pan;  // nmat kNB x kNB inverses, rounded to T
  // blocks that hold only identity padding need no elimination step
  const int nreal = (M + kNB - 1) / kNB;
  // algorithmic flops of one step: rank-kNB update of the M - kNB other rows
  const double step_flops = 2.0 * nmat * (double)kNB * M * std::max(M - kNB, 0);
  const double mfma_tiles = (double)nt * (nt - 1);  // tiles off the pivot rows
  // Each launch signals its completion through the profiler's stop event
  // when its class is timed, else through `done` (attached either way).
  auto pivot = [&](int p) {
    const ProfSpan ps = prof_open(KK_GJ_PANEL);
    const T *Rp = p >= 1 ? Rb[(p - 1) & 1] : nullptr;
    const T *Cp = p >= 1 ? Cb[(p - 1) & 1] : nullptr;
    hipExtLaunchKernelGGL(any_sign ? k_gj_pivot<T, true> : k_gj_pivot<T, false>, dim3(nmat),
                          dim3(256), 0, s, ps.a, ps.b, 0, mats, PinvT, Rp, Cp, ld, p, M, flag);
    prof_close(ps, KK_GJ_PANEL, (p >= 1 ? 4.0 : 2.0) * nmat * (double)kNB * kNB * kNB);
  };
  auto panel = [&](int p, hipEvent_t done) {
    const ProfSpan ps = prof_open(KK_GJ_PANEL);
    if (sym)
      hipExtLaunchKernelGGL(k_gj_panel_sym<T>, dim3(nt, nmat), dim3(256), 0, s, ps.a,
                            ps.b ? ps.b : done, 0, mats, PinvT, Rb[p & 1], Cb[p & 1], ld, p);
    else
      hipExtLaunchKernelGGL(k_gj_panel<T>, dim3(nt, nmat), dim3(256), 0, s, ps.a,
                            ps.b ? ps.b : done, 0, mats, PinvT, Rb[p & 1], Cb[p & 1], ld, p,
                            p == 0 ? 1 : 0);
    prof_close(ps, KK_GJ_PANEL, 2.0 * nmat * (double)kNB * kNB * std::max(M - kNB, 0));
    return ps.b ? ps.b : done;
  };
  auto update = [&](int p, int sel, hipStream_t st, hipEvent_t done) {
    const int ntiles = sym ? sel_tiles_sym(sel, nt) : sel_tiles(sel, nt);
    // tiles that take a product (the pivot-row tiles are copies; the
    // symmetric sets hold p + 1 of them outside the cross set)
    const double tiles = sym ? (sel == kSelCross ? nt - 1.0 : ntiles - (p + 1.0))
                         : sel == kSelAll   ? mfma_tiles
                         : sel == kSelCross ? 2.0 * nt - 3
                                            : (nt - 1.0) * (nt - 2);
    T *Cn = (!sym && sel == kSelCross) ? Cb[(p + 1) & 1] : nullptr;
    const ProfSpan ps = prof_open(KK_GJ_UPDATE);
    hipExtLaunchKernelGGL(sym ? k_gj_update<T, true> : k_gj_update<T, false>,
                          dim3(ntiles * nmat), dim3(256), 0, st, ps.a, ps.b ? ps.b : done, 0,
                          mats, Rb[p & 1], Cb[p & 1], Cn, ld, p, sel);
    prof_close(ps, KK_GJ_UPDATE, mfma_tiles > 0 ? step_flops * tiles / mfma_tiles : 0.0);
    return ps.b ? ps.b : done;
  };
  hipError_t e = hipSuccess;
#define GJCHK(call)                           \
  do {                                        \
    if ((e = (call)) != hipSuccess) return e; \
  } while (0)
  if (sym && nreal > 0)
    hipLaunchKernelGGL(k_sym_diag<T>, dim3(nreal, nmat), dim3(256), 0, s, mats, ld);
  pivot(0);
  hipEvent_t ev_panel = panel(0, gs.panel);
  hipEvent_t ev_rest[2] = {nullptr, nullptr}, ev_cross[2] = {nullptr, nullptr};
  for (int p = 0; p < nreal; ++p) {
    if (p + 1 < nreal) {
      GJCHK(hipStreamWaitEvent(gs.x, ev_panel, 0));
      if (p >= 1) GJCHK(hipStreamWaitEvent(gs.x, ev_rest[(p - 1) & 1], 0));
      ev_cross[p & 1] = update(p, kSelCross, gs.x, gs.cross[p & 1]);
      GJCHK(hipStreamWaitEvent(gs.h, ev_panel, 0));
      if (p >= 1) GJCHK(hipStreamWaitEvent(gs.h, ev_cross[(p - 1) & 1], 0));
      ev_rest[p & 1] = update(p, kSelRest, gs.h, gs.rest[p & 1]);
      if (p >= 1) GJCHK(hipStreamWaitEvent(s, ev_rest[(p - 1) & 1], 0));
      pivot(p + 1);
      GJCHK(hipStreamWaitEvent(s, ev_cross[p & 1], 0));
      ev_panel = panel(p + 1, gs.panel);
    } else {
      if (p >= 1) GJCHK(hipStreamWaitEvent(s, ev_rest[(p - 1) & 1], 0));
      update(p, kSelAll, s, nullptr);
    }
  }
  if (sym && nt > 1)
    hipLaunchKernelGGL(k_mirror_lower<T>, dim3(nt * (nt - 1) / 2, nmat), dim3(256), 0, s, mats,
                       ld);
#undef GJCHK
  return hipGetLastError();
}

#define DDST_INST(T)                                                                      \
  template void launch_assemble<T>(const AsmJob *, int, const double *, int, int, int, int, \
                                   hipStream_t);                                           \
  template void launch_scale_cols<T>(const GemmJob *, int, int, double, hipStream_t);       \
  template void launch_gemm<T>(const GemmJob *, int, int, int, double, double, hipStream_t); \
  template void launch_gemm_rect<T>(const GemmJob *, int, int, int, int, int, int, double,     \
                                    double, hipStream_t);                                      \
  template hipError_t gj_invert<T>(void *const *, int, int, int, void *, int *, int, int,   \
                                   GjStreams &, hipStream_t);
DDST_INST(float)
DDST_INST(double)
#undef DDST_INST

}  // namespace ddst

namespace ddst {
namespace {
template <typename T>
__global__ void k_extract(const T *__restrict__ src, int M, int ld, double *__restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)M * M) return;
  const size_t r = e / M, c = e % M;
  dst[e] = (double)src[r * ld + c];
}
}  // namespace

void launch_extract_block(const void *src, int prec, int M, int ld, double *dst,
                          hipStream_t s) {
  const size_t len = (size_t)M * M;
  const unsigned nb = (unsigned)((len + 255) / 256);
  if (prec == DDST_FP32)
    hipLaunchKernelGGL(k_extract<float>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float *>(src), M, ld, dst);
  else
    hipLaunchKernelGGL(k_extract<double>, dim3(nb), dim3(256), 0, s,
                       static_cast<const double *>(src), M, ld, dst);
}
}  // namespace ddst
