// GAP energy and its adjoint on the matrix cores (Sec. IV.A: e_i = sum_s alpha_s
// k(i, s) with the dot-product SOAP kernel k = (q_i . q_s)^zeta of Sec. I).
//
//   scores:  S = Q Q_s^T  (N x M, contraction over the descriptor length K), then
//            e_i = sum_s alpha_s S_is^zeta, alpha_bar_s = sum_i S_is^zeta and
//            G_is = zeta alpha_s S_is^(zeta-1), stored in the operand precision;
//   qbar:    Qbar = G Q_s (N x K, contraction over the M sparse points).
//
// The FP64 inputs are first converted once into zero-padded operand buffers
// (Q: N x Kp, Q_s: Mp x Kp, Q_s^T: Kp x Mp; both contraction dimensions padded
// to the K-tile), so the GEMM loop has no tail branches and loads 16 bytes per
// lane.  Each 256-thread workgroup owns one BM x BN output tile split 2 x 2
// over its four wavefronts; each K-tile is prefetched into registers while the
// previous one is multiplied from LDS.  Precision policies:
//   FP64    v_mfma_f64_16x16x4_f64, FP64 accumulation, 64 x 64 tiles
//   F32     v_mfma_f32_16x16x4_f32, FP32 accumulation, 64 x 64 tiles
//   BF16    v_mfma_f32_16x16x32_bf16, FP32 accumulation, 128 x 128 tiles; the
//           scores pass with 128-wide K-tiles, the Qbar pass with 64-wide ones
//           double-buffered in LDS (the next K-tile is stored while the current
//           one is multiplied: one barrier per K-tile) in rows of 128 bytes whose
//           16-byte pieces are permuted by row % 8 (XOR), so that the 16-byte
//           operand reads of eight consecutive rows hit distinct banks
//   BF16X3  a = a_hi + a_lo in BF16, a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// Row / column sums of the epilogue go to per-tile partial arrays that are
// added in a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gap.h"

namespace soap {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));  // 16-byte move

// kSwizzled: double-buffered K-tiles of 128-byte rows, 16-byte pieces XOR-permuted
// by row % 8 (needs KT * sizeof(T) = 128); otherwise one buffer, rows padded by 16 bytes
struct PF64 {
  using T = double;
  using Acc = d4;
  static constexpr int BM = 64, BN = 64, KT = 32;
  static constexpr bool kSplit = false;
  static constexpr bool kRowsInterleaved = true;  // D[l/16 + 4r][l%16]
  static constexpr bool kSwizzled = false;
};
struct PF32 {
  using T = float;
  using Acc = f4;
  static constexpr int BM = 64, BN = 64, KT = 32;
  static constexpr bool kSplit = false;
  static constexpr bool kRowsInterleaved = false;  // D[4(l/16) + r][l%16]
  static constexpr bool kSwizzled = false;
};
struct PBF16 {
  using T = __bf16;
  using Acc = f4;
  static constexpr int BM = 128, BN = 128, KT = 128;
  static constexpr bool kSplit = false;
  static constexpr bool kRowsInterleaved = false;
  static constexpr bool kSwizzled = false;
};
// the alternative BF16 scores tile (tile shape 1): 64-wide K-tiles, double-buffered
struct PBF16D : PBF16 {
  static constexpr int KT = 64;
  static constexpr bool kSwizzled = true;
};
struct PBF16X3 {
  using T = __bf16;
  using Acc = f4;
  static constexpr int BM = 128, BN = 128, KT = 32;
  static constexpr bool kSplit = true;
  static constexpr bool kRowsInterleaved = false;
  static constexpr bool kSwizzled = false;
};
// the Qbar pass (N x K output, K ~ 300) in 64 x 64 tiles, so that it fills the chip
template <typename P>
struct QbarTile : P {
  static constexpr int BM = 64, BN = 64;
};
// BF16 Qbar: the contraction runs over all sparse points (Mp ~ 2000) in 128 x 128
// tiles, double-buffered 64-wide K-tiles (the scores pass, with its heavier
// epilogue, keeps one buffer of 128-wide K-tiles: measured faster there)
template <>
struct QbarTile<PBF16> : PBF16 {
  static constexpr int KT = 64;
  static constexpr bool kSwizzled = true;
};
// the alternative BF16 Qbar tile (tile shape 1): 64 x 64, one buffer of 128-wide K-tiles
struct QbarSmallBF16 : PBF16 {
  static constexpr int BM = 64, BN = 64, KT = 128;
  static constexpr bool kSwizzled = false;
};
template <>
struct QbarTile<PF64> : PF64 {};
template <>
struct QbarTile<PF32> : PF32 {};

constexpr int kPad = 128;  // contraction dims are padded to a multiple of this (>= every KT)

inline int padded(int x) { return (x + kPad - 1) / kPad * kPad; }

template <typename T>
__device__ inline T cvt(double x) {
  return (T)x;
}
template <>
__device__ inline __bf16 cvt<__bf16>(double x) {
  return (__bf16)(float)x;
}
__device__ inline __bf16 cvt_lo(double x, __bf16 hi) { return (__bf16)(float)(x - (double)(float)hi); }
template <typename T>
__device__ inline T cvt_lo_any(double x, T hi) {
  if constexpr (sizeof(T) == 2) return cvt_lo(x, hi);
  else return (T)0;
}

// dst (rows_p x cols_p, pitch cols_p) = src (rows x cols) converted, zero padded;
// transpose: dst[c][r] = src[r][c]
template <typename T, bool SPLIT, bool TRANSPOSE>
__global__ void k_convert(int rows, int cols, int rows_p, int cols_p, const double* __restrict__ src,
                          T* __restrict__ dst, T* __restrict__ dst_lo) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows_p * cols_p) return;
  const int r = (int)(e / cols_p), c = (int)(e % cols_p);
  double x;
  if (TRANSPOSE) x = (c < rows && r < cols) ? src[(size_t)c * cols + r] : 0.0;
  else x = (r < rows && c < cols) ? src[(size_t)r * cols + c] : 0.0;
  const T h = cvt<T>(x);
  dst[e] = h;
  if (SPLIT) dst_lo[e] = cvt_lo_any<T>(x, h);
}

// the three operand conversions of one GAP call in one launch: Q (N x Kp), Q_s
// (Mp x Kp) and Q_s^T (Kp x Mp), zero padded
// I: the element index type, int when N Kp + 2 Mp Kp fits (its divisions are
// much cheaper than 64-bit ones), else long long
template <typename T, bool SPLIT, typename I>
__global__ void k_convert3(int N, int M, int K, int Kp, int Mp, I e0, const double* __restrict__ Q,
                           const double* __restrict__ Qs, T* __restrict__ qc, T* __restrict__ qc_lo,
                           T* __restrict__ qsc, T* __restrict__ qsc_lo, T* __restrict__ qst, T* __restrict__ qst_lo) {
  I e = e0 + (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;  // e0 = N Kp when Q is already converted
  const I n1 = (I)N * Kp, n2 = (I)Mp * Kp;
  double x;
  T* dst;
  T* dlo;
  if (e < n1) {
    const int r = (int)(e / Kp), c = (int)(e - (I)r * Kp);
    x = c < K ? Q[(size_t)r * K + c] : 0.0;
    dst = qc;
    dlo = qc_lo;
  } else if ((e -= n1) < n2) {
    const int r = (int)(e / Kp), c = (int)(e - (I)r * Kp);
    x = (r < M && c < K) ? Qs[(size_t)r * K + c] : 0.0;
    dst = qsc;
    dlo = qsc_lo;
  } else if ((e -= n2) < n2) {
    const int r = (int)(e / Mp), c = (int)(e - (I)r * Mp);  // dst[r][c] = Qs[c][r]
    x = (c < M && r < K) ? Qs[(size_t)c * K + r] : 0.0;
    dst = qst;
    dlo = qst_lo;
  } else {
    return;
  }
  const T h = cvt<T>(x);
  dst[e] = h;
  if (SPLIT) dlo[e] = cvt_lo_any<T>(x, h);
}

template <typename P>
struct Smem {
  static constexpr int EPV = 16 / sizeof(typename P::T);  // elements per 16-byte vector
  static constexpr bool SW = P::kSwizzled;
  static_assert(!SW || (P::KT * sizeof(typename P::T) == 128 && !P::kSplit), "swizzled rows are 128 bytes");
  static constexpr int PITCH = SW ? P::KT : P::KT + EPV;  // row pitch in elements (16-byte multiple)
  static constexpr int NB = SW ? 2 : 1;                   // K-tile buffers
  alignas(16) typename P::T a[NB * P::BM * PITCH];
  alignas(16) typename P::T b[NB * P::BN * PITCH];
  alignas(16) typename P::T a_lo[P::kSplit ? P::BM * PITCH : 1];
  alignas(16) typename P::T b_lo[P::kSplit ? P::BN * PITCH : 1];
  // element offset of (row r, column c) of a K-tile, c a multiple of EPV
  __device__ static inline int off(int r, int c) {
    if constexpr (SW) return r * PITCH + (((c / EPV) ^ (r & 7)) * EPV);
    else return r * PITCH + c;
  }
};

// Register staging of one K-tile of a (rows x KT) block: 16-byte vectors
template <typename P, int ROWS>
struct Stage {
  static constexpr int EPV = 16 / sizeof(typename P::T);
  static constexpr int VPR = P::KT / EPV;         // vectors per row
  static constexpr int NV = ROWS * VPR / 256;     // vectors per thread
  u4 v[NV];
  __device__ inline void load(const typename P::T* __restrict__ g, int ld, int row0, int nrows, int k0, int tid) {
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int idx = tid + 256 * t, r = idx / VPR, c = (idx % VPR) * EPV;
      const int gr = row0 + r;
      if (gr < nrows) v[t] = *(const u4*)(g + (size_t)gr * ld + k0 + c);
      else v[t] = u4{0u, 0u, 0u, 0u};
    }
  }
  __device__ inline void store(typename P::T* s, int tid) const {
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int idx = tid + 256 * t, r = idx / VPR, c = (idx % VPR) * EPV;
      *(u4*)(s + Smem<P>::off(r, c)) = v[t];
    }
  }
};

template <typename P>
struct Frag {
  static constexpr int TM = P::BM / 32, TN = P::BN / 32;  // 16 x 16 tiles per wave
};

// acc[x][y] += A(wave rows x) B(wave cols y)^T over the K-tile in LDS (buffer buf)
template <typename P>
__device__ inline void mma_ktile(const Smem<P>& sm, int buf, int wm, int wn, int lane,
                                 typename P::Acc (&acc)[Frag<P>::TM][Frag<P>::TN]) {
  constexpr int PITCH = Smem<P>::PITCH, TM = Frag<P>::TM, TN = Frag<P>::TN;
  using Sm = Smem<P>;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ra = wm * (P::BM / 2), rb = wn * (P::BN / 2);
  if constexpr (sizeof(typename P::T) >= 4) {
#pragma unroll
    for (int ks = 0; ks < P::KT; ks += 4) {
      typename P::T a[TM], b[TN];
#pragma unroll
      for (int x = 0; x < TM; ++x) a[x] = sm.a[(ra + x * 16 + r16) * PITCH + ks + kq];
#pragma unroll
      for (int y = 0; y < TN; ++y) b[y] = sm.b[(rb + y * 16 + r16) * PITCH + ks + kq];
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y) {
          if constexpr (sizeof(typename P::T) == 8)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
          else
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
  } else {
    const typename P::T* sa = sm.a + buf * P::BM * PITCH;
    const typename P::T* sb = sm.b + buf * P::BN * PITCH;
#pragma unroll
    for (int ks = 0; ks < P::KT; ks += 32) {
      b8 a[TM], b[TN], al[TM], bl[TN];
#pragma unroll
      for (int x = 0; x < TM; ++x) {
        a[x] = *(const b8*)&sa[Sm::off(ra + x * 16 + r16, ks + 8 * kq)];
        if constexpr (P::kSplit) al[x] = *(const b8*)&sm.a_lo[Sm::off(ra + x * 16 + r16, ks + 8 * kq)];
      }
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        b[y] = *(const b8*)&sb[Sm::off(rb + y * 16 + r16, ks + 8 * kq)];
        if constexpr (P::kSplit) bl[y] = *(const b8*)&sm.b_lo[Sm::off(rb + y * 16 + r16, ks + 8 * kq)];
      }
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y) {
          if constexpr (P::kSplit) {
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], b[y], acc[x][y], 0, 0, 0);
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], bl[y], acc[x][y], 0, 0, 0);
          }
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
  }
}

// C tile = A[row0.., :kdim] B[col0.., :kdim]^T into acc; A rows beyond arows and
// B rows beyond brows read as zero.  kdim is a multiple of KT.
template <typename P>
__device__ inline void gemm_tile(Smem<P>& sm, const typename P::T* __restrict__ A, const typename P::T* __restrict__ A_lo,
                                 int lda, int arows, const typename P::T* __restrict__ B,
                                 const typename P::T* __restrict__ B_lo, int ldb, int brows, int kdim, int row0,
                                 int col0, typename P::Acc (&acc)[Frag<P>::TM][Frag<P>::TN]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
  Stage<P, P::BM> sa, sal;
  Stage<P, P::BN> sb, sbl;
  sa.load(A, lda, row0, arows, 0, tid);
  sb.load(B, ldb, col0, brows, 0, tid);
  if constexpr (P::kSplit) {
    sal.load(A_lo, lda, row0, arows, 0, tid);
    sbl.load(B_lo, ldb, col0, brows, 0, tid);
  }
  if constexpr (Smem<P>::SW) {
    // double buffer: K-tile t is multiplied from buffer t % 2 while tile t + 1,
    // already in registers, is stored into the other one; the barrier that ends
    // step t also guarantees that no wave still reads the buffer step t + 1 fills
    constexpr int AB = P::BM * Smem<P>::PITCH, BB = P::BN * Smem<P>::PITCH;
    sa.store(sm.a, tid);
    sb.store(sm.b, tid);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < kdim; k0 += P::KT) {
      const bool more = k0 + P::KT < kdim;
      if (more) {
        sa.load(A, lda, row0, arows, k0 + P::KT, tid);
        sb.load(B, ldb, col0, brows, k0 + P::KT, tid);
      }
      mma_ktile<P>(sm, buf, wm, wn, lane, acc);
      if (more) {
        sa.store(sm.a + (buf ^ 1) * AB, tid);
        sb.store(sm.b + (buf ^ 1) * BB, tid);
      }
      __syncthreads();
      buf ^= 1;
    }
  } else {
    for (int k0 = 0; k0 < kdim; k0 += P::KT) {
      sa.store(sm.a, tid);
      sb.store(sm.b, tid);
      if constexpr (P::kSplit) {
        sal.store(sm.a_lo, tid);
        sbl.store(sm.b_lo, tid);
      }
      __syncthreads();
      if (k0 + P::KT < kdim) {  // prefetch the next K-tile while this one is multiplied
        sa.load(A, lda, row0, arows, k0 + P::KT, tid);
        sb.load(B, ldb, col0, brows, k0 + P::KT, tid);
        if constexpr (P::kSplit) {
          sal.load(A_lo, lda, row0, arows, k0 + P::KT, tid);
          sbl.load(B_lo, ldb, col0, brows, k0 + P::KT, tid);
        }
      }
      mma_ktile<P>(sm, 0, wm, wn, lane, acc);
      __syncthreads();
    }
  }
}

// (column tile, row tile) of this workgroup.  Workgroups are handed to the eight
// XCDs round-robin by linear index; tiles are numbered so that each XCD takes
// one rectangle of the tile grid (the grid cut into xr x xc rectangles, xr xc =
// 8), which its L2 serves: every row and column operand tile is then fetched
// from HBM by one or a few XCDs instead of by all eight.
__device__ inline void xcd_tile(int& tc, int& tr, int xr, int xc) {
  const int nc = gridDim.x, nr = gridDim.y;
  const int b = blockIdx.y * nc + blockIdx.x;
  if (nr % xr == 0 && nc % xc == 0) {
    const int x = b % 8, slot = b / 8, cc = nc / xc;
    tr = (x / xc) * (nr / xr) + slot / cc;
    tc = (x % xc) * cc + slot % cc;
  } else {
    tc = b % nc;
    tr = b / nc;
  }
}

// row of element r of acc[x][.] within the wave's block
template <typename P>
__device__ inline int acc_row(int x, int r, int lane) {
  return x * 16 + (P::kRowsInterleaved ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
}

__device__ inline double ipow(double x, int e) {
  double r = 1.0;
  for (int t = 0; t < e; ++t) r *= x;
  return r;
}

// S = Q Q_s^T tile with the zeta epilogue: G (N x Mp) in the operand precision
// (zero for padding columns), e_part[col_tile][i], ab_part[row_tile][s]
template <typename P>
__global__ __launch_bounds__(256) void k_scores(int N, int M, int Mp, int Kp, const typename P::T* __restrict__ Qc,
                                                const typename P::T* __restrict__ Qc_lo,
                                                const typename P::T* __restrict__ Qsc,
                                                const typename P::T* __restrict__ Qsc_lo,
                                                const double* __restrict__ alpha, int zeta,
                                                typename P::T* __restrict__ G, typename P::T* __restrict__ G_lo,
                                                double* __restrict__ e_part, double* __restrict__ ab_part) {
  using T = typename P::T;
  constexpr int TM = Frag<P>::TM, TN = Frag<P>::TN;
  extern __shared__ __align__(16) char dsm[];  // the operand tiles, sizeof(Smem<P>)
  Smem<P>& sm = *reinterpret_cast<Smem<P>*>(dsm);
  __shared__ double rowsum[2][P::BM];
  __shared__ double colsum[2][P::BN];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
  int tc, tr;
  xcd_tile(tc, tr, 4, 2);  // both operands are reused across the grid
  const int i0 = tr * P::BM, s0 = tc * P::BN;
  typename P::Acc acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = typename P::Acc{};
  gemm_tile<P>(sm, Qc, Qc_lo, Kp, N, Qsc, Qsc_lo, Kp, Mp, Kp, i0, s0, acc);
  // G goes through LDS (the operand tiles are no longer needed) and out as
  // whole 16-byte row pieces; the BF16X3 low part takes a second pass
  constexpr int EPV = 16 / sizeof(T), GP = P::BN + EPV, VPR = P::BN / EPV;
  static_assert(sizeof(T) * P::BM * GP <= sizeof(Smem<P>), "G tile must fit in the operand LDS");
  T* gt = reinterpret_cast<T*>(&sm);
  // 16-bit operands: the zeta power and the tile's row and column sums (at most
  // BN and BM terms, added in FP64 across tiles) in FP32, whose rounding is far
  // below that of the operands; otherwise in FP64
  using E = typename std::conditional<sizeof(T) == 2, float, double>::type;
  E rows[TM][4] = {}, cols[TN] = {};
  // the weights of this lane's columns, read once; a padding column (gs >= M)
  // has weight 0, and its scores, like those of padding rows, are exactly 0
  // (zero operand rows), so the tile needs no per-element bounds test: padding
  // contributes nothing to the sums, and its G entries are 0 or never stored
  E al_y[TN];
#pragma unroll
  for (int y = 0; y < TN; ++y) {
    const int gs = s0 + wn * (P::BN / 2) + y * 16 + (lane & 15);
    al_y[y] = gs < M ? (E)alpha[gs] : (E)0;
  }
  // s^(zeta - 1) of every element, the running product 1, s, s s, (s s) s, ...:
  // with one pass, one loop over the power for all of the lane's elements at
  // once; the split mode, whose two passes would keep them all live, forms it
  // per element in each pass
  E pw[TM][TN][4];
  if constexpr (!P::kSplit) {
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) pw[x][y][r] = (E)1;
    for (int t = 1; t < zeta; ++t) {
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) pw[x][y][r] *= (E)acc[x][y][r];
    }
  }
#pragma unroll
  for (int pass = 0; pass < (P::kSplit ? 2 : 1); ++pass) {
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int lr = wm * (P::BM / 2) + acc_row<P>(x, r, lane);
          const int lc = wn * (P::BN / 2) + y * 16 + (lane & 15);
          const E sv = (E)acc[x][y][r];
          E sz1;
          if constexpr (P::kSplit) {
            sz1 = (E)1;
            for (int t = 1; t < zeta; ++t) sz1 *= sv;
          } else {
            sz1 = pw[x][y][r];
          }
          const E al = al_y[y];
          const E g = (E)zeta * al * sz1;
          if (pass == 0) {
            const E kv = sz1 * sv;
            rows[x][r] = fma(al, kv, rows[x][r]);
            cols[y] += kv;
          }
          const T gh = cvt<T>((double)g);
          gt[lr * GP + lc] = pass == 0 ? gh : cvt_lo_any<T>((double)g, gh);
        }
    __syncthreads();
    T* __restrict__ dst = pass == 0 ? G : G_lo;
    for (int u = tid; u < P::BM * VPR; u += 256) {
      const int lr = u / VPR, c = (u % VPR) * EPV, gi = i0 + lr;
      if (gi < N) *(u4*)(dst + (size_t)gi * Mp + s0 + c) = *(const u4*)(gt + lr * GP + c);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      E v = rows[x][r];
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
      if ((lane & 15) == 0) rowsum[wn][wm * (P::BM / 2) + acc_row<P>(x, r, lane)] = (double)v;
    }
#pragma unroll
  for (int y = 0; y < TN; ++y) {
    E v = cols[y];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < 16) colsum[wm][wn * (P::BN / 2) + y * 16 + lane] = (double)v;
  }
  __syncthreads();
  for (int t = tid; t < P::BM + P::BN; t += 256) {
    if (t < P::BM) {
      const int gi = i0 + t;
      if (gi < N) e_part[(size_t)tc * N + gi] = rowsum[0][t] + rowsum[1][t];
    } else {
      const int c = t - P::BM, gs = s0 + c;
      if (gs < M) ab_part[(size_t)tr * M + gs] = colsum[0][c] + colsum[1][c];
    }
  }
}

// e[i] = sum_t e_part[t][i] (t < nte) and, if ab, ab[j] = sum_t ab_part[t][j] (t < nta),
// each in a fixed order; the loads of eight terms are issued together
__device__ inline double ordered_sum(const double* __restrict__ part, int n, int nt, int j) {
  double s = 0.0;
  int t = 0;
  for (; t + 8 <= nt; t += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(t + u) * n + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; t < nt; ++t) s += part[(size_t)t * n + j];
  return s;
}

// Qbar tile = G (N x Mp) Q_s^T-converted (Kp x Mp)^T, written for descriptor columns < K
// OT: the storage type of Qbar (double, or float for the FP32 accumulators)
template <typename P, typename OT>
__global__ __launch_bounds__(256) void k_qbar(int N, int K, int Mp, int Kp, int kslice,
                                              const typename P::T* __restrict__ G,
                                              const typename P::T* __restrict__ G_lo,
                                              const typename P::T* __restrict__ QsT,
                                              const typename P::T* __restrict__ QsT_lo, OT* __restrict__ Qbar,
                                              int M, int nte, const double* __restrict__ e_part,
                                              double* __restrict__ e, int nta, const double* __restrict__ ab_part,
                                              double* __restrict__ ab) {
  constexpr int TM = Frag<P>::TM, TN = Frag<P>::TN;
  extern __shared__ __align__(16) char dsm[];  // the operand tiles, sizeof(Smem<P>)
  Smem<P>& sm = *reinterpret_cast<Smem<P>*>(dsm);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
  int tc, tr;
  xcd_tile(tc, tr, 8, 1);  // few column tiles: an XCD takes whole rows of tiles
  const int i0 = tr * P::BM, c0 = tc * P::BN;
  typename P::Acc acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = typename P::Acc{};
  // slice z of the contraction over the sparse points: points z kslice ..
  // (z + 1) kslice - 1, into its own N x K part of Qbar
  const int z = blockIdx.z, k0 = z * kslice;
  gemm_tile<P>(sm, G + k0, G_lo + k0, Mp, N, QsT + k0, QsT_lo + k0, Mp, Kp, kslice, i0, c0, acc);
  OT* __restrict__ Qz = Qbar + (size_t)z * N * K;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wm * (P::BM / 2) + acc_row<P>(x, r, lane);
        const int gc = c0 + wn * (P::BN / 2) + y * 16 + (lane & 15);
        if (gi < N && gc < K) Qz[(size_t)gi * K + gc] = (OT)acc[x][y][r];
      }
  // the scores pass's per-tile partial sums, finished here (e non-null) by the
  // first slice: each workgroup takes one part of the N + M outputs, each
  // output a fixed-order sum
  if (e && z == 0) {
    const int nb = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
    const int per = (N + M + nb - 1) / nb, j1 = min((b + 1) * per, N + M);
    for (int j = b * per + tid; j < j1; j += 256) {
      if (j < N) e[j] = ordered_sum(e_part, N, nte, j);
      else if (ab) ab[j - N] = ordered_sum(ab_part, M, nta, j - N);
    }
  }
}

__global__ void k_sum_parts2(int N, int nte, const double* __restrict__ e_part, double* __restrict__ e, int M, int nta,
                             const double* __restrict__ ab_part, double* __restrict__ ab) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) e[j] = ordered_sum(e_part, N, nte, j);
  else if (ab && j < N + M) ab[j - N] = ordered_sum(ab_part, M, nta, j - N);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- fused pass
// Scores, zeta epilogue and Qbar in one kernel for the 16- and 32-bit operand
// modes when the padded descriptor fits in LDS (K <= kFusedK).  Workgroup
// (rb, sp) keeps rows [rb BM, rb BM + BM) of Q converted in LDS and walks the
// sparse points of slice sp in chunks of BN:
//   S = Q_blk Q_s,c^T                 (MFMA, contraction over K)
//   e_i += alpha_s S^zeta,  column sums of S^zeta -> ab_part[rb][s],
//   G = zeta alpha_s S^(zeta-1)        (registers -> LDS, operand precision)
//   Qbar_blk += G Q_s,c                (MFMA, contraction over the chunk)
// so G never goes to HBM.  Slices are combined by k_gap_reduce in a fixed order.
constexpr int kFusedK = 352;  // padded descriptor length limit (multiple of 32)
constexpr int kFusedTNq = 6;  // Qbar column tiles per wavefront: 4 x 6 x 16 = 384 >= kFusedK

struct FB16 {
  using T = __bf16;
  using Acc = f4;
  static constexpr int BM = 64, BN = 64, KSTEP = 32;
  static constexpr bool kSplit = false;
};
struct FB16X3 {
  using T = __bf16;
  using Acc = f4;
  static constexpr int BM = 32, BN = 32, KSTEP = 32;
  static constexpr bool kSplit = true;
};
struct FF32 {
  using T = float;
  using Acc = f4;
  static constexpr int BM = 32, BN = 32, KSTEP = 4;
  static constexpr bool kSplit = false;
};

template <typename F>
struct FusedSmem {
  using T = typename F::T;
  static constexpr int EPV = 16 / sizeof(T);
  static constexpr int PQ = kFusedK + EPV;  // row pitch over the descriptor
  static constexpr int PS = F::BN + EPV;    // row pitch over the sparse points of a chunk
  static constexpr int NL = F::kSplit ? 1 : 0;
  alignas(16) T q[F::BM * PQ];
  alignas(16) T q_lo[NL ? F::BM * PQ : 1];
  alignas(16) T qs[F::BN * PQ];
  alignas(16) T qs_lo[NL ? F::BN * PQ : 1];
  alignas(16) T qst[kFusedK * PS];
  alignas(16) T qst_lo[NL ? kFusedK * PS : 1];
  alignas(16) T g[F::BM * PS];
  alignas(16) T g_lo[NL ? F::BM * PS : 1];
  double colsum[2][F::BN];
  double rowsum[2][F::BM];
  double alpha[F::BN];
};

// acc[x][y] += A[a0 + 16x .., k0 ..) B^T[b0 + 16y .., k0 ..)^T: one MFMA k-step from LDS;
// tiles y with b0 + 16y >= bcap are skipped (uniform per wavefront)
template <typename F, int TM, int TN>
__device__ inline void fused_step(const typename F::T* A, const typename F::T* A_lo, int pa, int a0,
                                  const typename F::T* B, const typename F::T* B_lo, int pb, int b0, int bcap,
                                  int k0, int lane, typename F::Acc (&acc)[TM][TN]) {
  const int r16 = lane & 15, kq = lane >> 4;
  if constexpr (sizeof(typename F::T) == 4) {
    float a[TM], b[TN];
#pragma unroll
    for (int x = 0; x < TM; ++x) a[x] = A[(a0 + 16 * x + r16) * pa + k0 + kq];
#pragma unroll
    for (int y = 0; y < TN; ++y) b[y] = (b0 + 16 * y < bcap) ? B[(b0 + 16 * y + r16) * pb + k0 + kq] : 0.0f;
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y)
        if (b0 + 16 * y < bcap) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
  } else {
    b8 a[TM], al[TM], b[TN], bl[TN];
#pragma unroll
    for (int x = 0; x < TM; ++x) {
      a[x] = *(const b8*)&A[(a0 + 16 * x + r16) * pa + k0 + 8 * kq];
      if constexpr (F::kSplit) al[x] = *(const b8*)&A_lo[(a0 + 16 * x + r16) * pa + k0 + 8 * kq];
    }
#pragma unroll
    for (int y = 0; y < TN; ++y) {
      if (b0 + 16 * y < bcap) {
        b[y] = *(const b8*)&B[(b0 + 16 * y + r16) * pb + k0 + 8 * kq];
        if constexpr (F::kSplit) bl[y] = *(const b8*)&B_lo[(b0 + 16 * y + r16) * pb + k0 + 8 * kq];
      }
    }
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y)
        if (b0 + 16 * y < bcap) {
          if constexpr (F::kSplit) {
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], b[y], acc[x][y], 0, 0, 0);
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], bl[y], acc[x][y], 0, 0, 0);
          }
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
        }
  }
}

// A rows x cols tile of T (row pitch ld in HBM, lp in LDS) held in registers as
// 16-byte vectors, NV per thread at most (rows * cols <= 256 * NV * 16 / sizeof(T)):
// load() issues every global read before any is used, store() writes LDS.
template <typename T, int NV>
struct RegTile {
  u4 v[NV];
  __device__ inline void load(const T* __restrict__ g, int ld, int rows, int cols, int tid) {
    constexpr int EPV = 16 / sizeof(T);
    const int vpr = cols / EPV;
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int x = tid + 256 * t, r = x / vpr, c = (x - r * vpr) * EPV;
      if (r < rows) v[t] = *(const u4*)(g + (size_t)r * ld + c);
    }
  }
  __device__ inline void store(T* s, int lp, int rows, int cols, int tid) const {
    constexpr int EPV = 16 / sizeof(T);
    const int vpr = cols / EPV;
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int x = tid + 256 * t, r = x / vpr, c = (x - r * vpr) * EPV;
      if (r < rows) *(u4*)(s + r * lp + c) = v[t];
    }
  }
};

template <typename F, typename OT>
__global__ __launch_bounds__(256) void k_gap_fused(int N, int M, int K, int Kf, int Mp, int chunks_per_slice,
                                                   const double* __restrict__ Q,
                                                   const typename F::T* __restrict__ QsC,
                                                   const typename F::T* __restrict__ QsC_lo,
                                                   const typename F::T* __restrict__ QsT,
                                                   const typename F::T* __restrict__ QsT_lo,
                                                   const double* __restrict__ alpha, int zeta,
                                                   double* __restrict__ e_out, float* __restrict__ qbar_part,
                                                   OT* __restrict__ qbar_out, double* __restrict__ ab_part) {
  using T = typename F::T;
  using Sm = FusedSmem<F>;
  constexpr int BM = F::BM, BN = F::BN, TMs = BM / 32, TNs = BN / 32, TMq = BM / 16;
  extern __shared__ __align__(16) unsigned char fused_raw[];
  Sm& sm = *reinterpret_cast<Sm*>(fused_raw);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
  const int rb = blockIdx.x, sp = blockIdx.y, nsp = gridDim.y;
  const int i0 = rb * BM;
  const int Kq = (K + 15) / 16 * 16;
  // Q rows of this block, converted and zero padded to Kf (loads batched eight deep)
  for (int t0 = tid; t0 < BM * Kf; t0 += 256 * 8) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + 256 * u, r = t / Kf, k = t - r * Kf;
      x[u] = (t < BM * Kf && i0 + r < N && k < K) ? Q[(size_t)(i0 + r) * K + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + 256 * u, r = t / Kf, k = t - r * Kf;
      if (t < BM * Kf) {
        const T h = cvt<T>(x[u]);
        sm.q[r * Sm::PQ + k] = h;
        if constexpr (F::kSplit) sm.q_lo[r * Sm::PQ + k] = cvt_lo_any<T>(x[u], h);
      }
    }
  }
  typename F::Acc aq[TMq][kFusedTNq];
#pragma unroll
  for (int x = 0; x < TMq; ++x)
#pragma unroll
    for (int y = 0; y < kFusedTNq; ++y) aq[x][y] = typename F::Acc{};
  double rows[TMs][4] = {};
  const int c_begin = sp * chunks_per_slice;
  const int c_end = min(c_begin + chunks_per_slice, Mp / BN);
  // the next chunk's Q_s rows and Q_s^T columns are loaded into registers while
  // the current chunk is multiplied
  constexpr int EPV = 16 / sizeof(T);
  constexpr int NV = (BN * kFusedK / EPV + 255) / 256;
  RegTile<T, NV> rq, rt, rq_lo, rt_lo;
  double ra = 0.0;
  auto fetch = [&](int c) {
    const int s0 = c * BN;
    rq.load(QsC + (size_t)s0 * Kf, Kf, BN, Kf, tid);
    rt.load(QsT + s0, Mp, Kf, BN, tid);
    if constexpr (F::kSplit) {
      rq_lo.load(QsC_lo + (size_t)s0 * Kf, Kf, BN, Kf, tid);
      rt_lo.load(QsT_lo + s0, Mp, Kf, BN, tid);
    }
    ra = (tid < BN && s0 + tid < M) ? alpha[s0 + tid] : 0.0;
  };
  if (c_begin < c_end) fetch(c_begin);
  for (int c = c_begin; c < c_end; ++c) {
    const int s0 = c * BN;
    __syncthreads();  // the previous chunk is done with qs, qst, g and alpha
    rq.store(sm.qs, Sm::PQ, BN, Kf, tid);
    rt.store(sm.qst, Sm::PS, Kf, BN, tid);
    if constexpr (F::kSplit) {
      rq_lo.store(sm.qs_lo, Sm::PQ, BN, Kf, tid);
      rt_lo.store(sm.qst_lo, Sm::PS, Kf, BN, tid);
    }
    if (tid < BN) sm.alpha[tid] = ra;
    __syncthreads();
    if (c + 1 < c_end) fetch(c + 1);
    // S = Q_blk Q_s,c^T: wave (wm, wn) owns rows wm BM/2 .., sparse points wn BN/2 ..
    typename F::Acc as[TMs][TNs];
#pragma unroll
    for (int x = 0; x < TMs; ++x)
#pragma unroll
      for (int y = 0; y < TNs; ++y) as[x][y] = typename F::Acc{};
    for (int k0 = 0; k0 < Kf; k0 += F::KSTEP)
      fused_step<F, TMs, TNs>(sm.q, sm.q_lo, Sm::PQ, wm * (BM / 2), sm.qs, sm.qs_lo, Sm::PQ, wn * (BN / 2), BN, k0,
                              lane, as);
    // zeta epilogue: G to LDS, row sums in registers, column sums per chunk
    double cols[TNs] = {};
#pragma unroll
    for (int x = 0; x < TMs; ++x)
#pragma unroll
      for (int y = 0; y < TNs; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wm * (BM / 2) + 16 * x + 4 * (lane >> 4) + r;
          const int col = wn * (BN / 2) + 16 * y + (lane & 15);
          double gv = 0.0;
          if (s0 + col < M) {
            const double sv = (double)as[x][y][r];
            const double sz1 = ipow(sv, zeta - 1);
            const double kv = sz1 * sv;
            const double al = sm.alpha[col];
            gv = (double)zeta * al * sz1;
            if (i0 + row < N) {
              rows[x][r] = fma(al, kv, rows[x][r]);
              cols[y] += kv;
            }
          }
          const T gh = cvt<T>(gv);
          sm.g[row * Sm::PS + col] = gh;
          if constexpr (F::kSplit) sm.g_lo[row * Sm::PS + col] = cvt_lo_any<T>(gv, gh);
        }
#pragma unroll
    for (int y = 0; y < TNs; ++y) {
      double v = cols[y];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (lane < 16) sm.colsum[wm][wn * (BN / 2) + 16 * y + lane] = v;
    }
    __syncthreads();
    if (tid < BN && s0 + tid < M) ab_part[(size_t)rb * M + s0 + tid] = sm.colsum[0][tid] + sm.colsum[1][tid];
    // Qbar_blk += G Q_s,c: wave wv owns descriptor columns 96 wv ..
    for (int k0 = 0; k0 < BN; k0 += F::KSTEP)
      fused_step<F, TMq, kFusedTNq>(sm.g, sm.g_lo, Sm::PS, 0, sm.qst, sm.qst_lo, Sm::PS, wv * 16 * kFusedTNq, Kq, k0,
                                    lane, aq);
  }
  // e: rows summed over the 16 lanes of a column group and the two wn waves
#pragma unroll
  for (int x = 0; x < TMs; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = rows[x][r];
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
      if ((lane & 15) == 0) sm.rowsum[wn][wm * (BM / 2) + 16 * x + 4 * (lane >> 4) + r] = v;
    }
  __syncthreads();
  if (tid < BM && i0 + tid < N) {
    const double v = sm.rowsum[0][tid] + sm.rowsum[1][tid];
    e_out[(size_t)sp * N + i0 + tid] = v;
  }
#pragma unroll
  for (int x = 0; x < TMq; ++x)
#pragma unroll
    for (int y = 0; y < kFusedTNq; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * x + 4 * (lane >> 4) + r;
        const int col = wv * 16 * kFusedTNq + 16 * y + (lane & 15);
        if (i0 + row < N && col < K) {
          if (nsp == 1) qbar_out[(size_t)(i0 + row) * K + col] = (OT)aq[x][y][r];
          else qbar_part[((size_t)sp * N + i0 + row) * K + col] = aq[x][y][r];
        }
      }
}

// e[i] = sum_sp e_part[sp][i]; Qbar = sum_sp qbar_part[sp] (when nsp > 1); ab[s] = sum_rb ab_part[rb][s],
// all in a fixed order
template <typename OT>
__global__ void k_gap_reduce(int N, int K, int M, int nsp, int nrb, const double* __restrict__ e_part,
                             const float* __restrict__ qbar_part, const double* __restrict__ ab_part,
                             double* __restrict__ e, OT* __restrict__ qbar, double* __restrict__ ab) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nq = nsp > 1 ? (long long)N * K : 0;
  if (t < nq) {
    double v = 0.0;
    for (int s = 0; s < nsp; ++s) v += (double)qbar_part[(size_t)s * N * K + t];
    qbar[t] = (OT)v;
  } else if (t < nq + N) {
    const int i = (int)(t - nq);
    double v = 0.0;
    for (int s = 0; s < nsp; ++s) v += e_part[(size_t)s * N + i];
    e[i] = v;
  } else if (t < nq + N + M && ab) {
    const int j = (int)(t - nq - N);
    double v = 0.0;
    for (int r = 0; r < nrb; ++r) v += ab_part[(size_t)r * M + j];
    ab[j] = v;
  }
}

struct FusedLayout {
  size_t qsc, qsc_lo, qst, qst_lo, e_part, qbar_part, ab_part, total;
  int Kf, Mp, nrb, nsp, cps;
};

template <typename F>
FusedLayout fused_layout(int N, int M, int K, int target) {
  FusedLayout L{};
  const size_t es = sizeof(typename F::T);
  L.Kf = (K + 31) / 32 * 32;
  L.Mp = padded(M);
  L.nrb = (N + F::BM - 1) / F::BM;
  const int nchunks = L.Mp / F::BN;
  L.nsp = std::min(nchunks, std::max(1, (target + L.nrb - 1) / L.nrb));
  L.cps = (nchunks + L.nsp - 1) / L.nsp;
  L.nsp = (nchunks + L.cps - 1) / L.cps;
  const size_t nlo = F::kSplit ? 1 : 0;
  size_t o = 0;
  L.qsc = o;
  o += align256(es * L.Mp * L.Kf);
  L.qsc_lo = o;
  o += align256(es * L.Mp * L.Kf * nlo);
  L.qst = o;
  o += align256(es * L.Kf * L.Mp);
  L.qst_lo = o;
  o += align256(es * L.Kf * L.Mp * nlo);
  L.e_part = o;
  o += align256(sizeof(double) * (size_t)L.nsp * N);
  L.qbar_part = o;
  o += align256(L.nsp > 1 ? sizeof(float) * (size_t)L.nsp * N * K : 0);
  L.ab_part = o;
  o += align256(sizeof(double) * (size_t)L.nrb * M);
  L.total = o;
  return L;
}

template <typename F, typename OT>
hipError_t fused_impl(int N, int M, int K, const double* Q, const double* Qs, const double* alpha, int zeta, double* e,
                      double* alpha_bar, OT* Qbar, void* work, int target, hipStream_t st) {
  using T = typename F::T;
  const FusedLayout L = fused_layout<F>(N, M, K, target);
  char* w = (char*)work;
  T *qsc = (T*)(w + L.qsc), *qsc_lo = (T*)(w + L.qsc_lo), *qst = (T*)(w + L.qst), *qst_lo = (T*)(w + L.qst_lo);
  double *e_part = (double*)(w + L.e_part), *ab_part = (double*)(w + L.ab_part);
  float* qbar_part = (float*)(w + L.qbar_part);
  auto blocks = [](long long n) { return dim3((unsigned)((n + 255) / 256)); };
  hipLaunchKernelGGL((k_convert<T, F::kSplit, false>), blocks((long long)L.Mp * L.Kf), dim3(256), 0, st, M, K, L.Mp,
                     L.Kf, Qs, qsc, qsc_lo);
  hipLaunchKernelGGL((k_convert<T, F::kSplit, true>), blocks((long long)L.Kf * L.Mp), dim3(256), 0, st, M, K, L.Kf,
                     L.Mp, Qs, qst, qst_lo);
  hipLaunchKernelGGL((k_gap_fused<F, OT>), dim3(L.nrb, L.nsp), dim3(256), sizeof(FusedSmem<F>), st, N, M, K, L.Kf, L.Mp,
                     L.cps, Q, qsc, qsc_lo, qst, qst_lo, alpha, zeta, e_part, qbar_part, Qbar, ab_part);
  const long long nred = (L.nsp > 1 ? (long long)N * K : 0) + N + M;
  hipLaunchKernelGGL(k_gap_reduce<OT>, blocks(nred), dim3(256), 0, st, N, K, M, L.nsp, L.nrb, e_part, qbar_part,
                     ab_part, e, Qbar, alpha_bar);
  return hipGetLastError();
}

// ---------------------------------------------------------------- workspace
// [Qc | Qc_lo | Qsc | Qsc_lo | QsT | QsT_lo | G | G_lo | e_part | ab_part], 256-byte aligned pieces
struct Layout {
  size_t qc, qc_lo, qsc, qsc_lo, qst, qst_lo, g, g_lo, e_part, ab_part, total;
};


template <typename P>
Layout layout(int N, int M, int K) {
  const size_t es = sizeof(typename P::T);
  const size_t Kp = padded(K), Mp = padded(M);
  const size_t nlo = P::kSplit ? 1 : 0;
  const size_t nst = (Mp + P::BN - 1) / P::BN, nit = (N + P::BM - 1) / P::BM;
  Layout L{};
  size_t o = 0;
  L.qc = o;
  o += align256(es * N * Kp);
  L.qc_lo = o;
  o += align256(es * N * Kp * nlo);
  L.qsc = o;
  o += align256(es * Mp * Kp);
  L.qsc_lo = o;
  o += align256(es * Mp * Kp * nlo);
  L.qst = o;
  o += align256(es * Kp * Mp);
  L.qst_lo = o;
  o += align256(es * Kp * Mp * nlo);
  L.g = o;
  o += align256(es * N * Mp);
  L.g_lo = o;
  o += align256(es * N * Mp * nlo);
  L.e_part = o;
  o += align256(sizeof(double) * nst * N);
  L.ab_part = o;
  o += align256(sizeof(double) * nit * M);
  L.total = o;
  return L;
}

template <typename P>
hipError_t scores_impl(int N, int M, int K, const double* Q, const double* Qs, const double* alpha, int zeta,
                       double* e, double* alpha_bar, bool sums, bool q_ready, void* work, hipStream_t st) {
  using T = typename P::T;
  const Layout L = layout<P>(N, M, K);
  char* w = (char*)work;
  const int Kp = padded(K), Mp = padded(M);
  T *qc = (T*)(w + L.qc), *qc_lo = (T*)(w + L.qc_lo), *qsc = (T*)(w + L.qsc), *qsc_lo = (T*)(w + L.qsc_lo);
  T *qst = (T*)(w + L.qst), *qst_lo = (T*)(w + L.qst_lo), *G = (T*)(w + L.g), *G_lo = (T*)(w + L.g_lo);
  double *e_part = (double*)(w + L.e_part), *ab_part = (double*)(w + L.ab_part);
  auto blocks = [](long long n) { return dim3((unsigned)((n + 255) / 256)); };
  const long long nconv = (long long)N * Kp + 2LL * Mp * Kp, e0 = q_ready ? (long long)N * Kp : 0;
  if (nconv < 2147483647LL - 256)
    hipLaunchKernelGGL((k_convert3<T, P::kSplit, int>), blocks(nconv - e0), dim3(256), 0, st, N, M, K, Kp, Mp, (int)e0,
                       Q, Qs, qc, qc_lo, qsc, qsc_lo, qst, qst_lo);
  else
    hipLaunchKernelGGL((k_convert3<T, P::kSplit, long long>), blocks(nconv - e0), dim3(256), 0, st, N, M, K, Kp, Mp,
                       e0, Q, Qs, qc, qc_lo, qsc, qsc_lo, qst, qst_lo);
  const int nst = (Mp + P::BN - 1) / P::BN, nit = (N + P::BM - 1) / P::BM;
  static bool attr = false;  // operand tiles above 64 KB of LDS need the opt-in
  if (!attr && sizeof(Smem<P>) > 65536) {
    const hipError_t a = hipFuncSetAttribute((const void*)k_scores<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)sizeof(Smem<P>));
    if (a != hipSuccess) return a;
  }
  attr = true;
  hipLaunchKernelGGL(k_scores<P>, dim3(nst, nit), dim3(256), sizeof(Smem<P>), st, N, M, Mp, Kp, qc, qc_lo, qsc,
                     qsc_lo, alpha, zeta, G, G_lo, e_part, ab_part);
  if (sums)
    hipLaunchKernelGGL(k_sum_parts2, dim3((N + M + 255) / 256), dim3(256), 0, st, N, nst, e_part, e, M, nit, ab_part,
                       alpha_bar);
  return hipGetLastError();
}

// P: the scores pass's policy (its tile counts index the partial sums), Q: the
// Qbar pass's tile
template <typename P, typename Q = QbarTile<P>>
hipError_t qbar_impl(int N, int M, int K, void* Qbar, bool f32, double* e, double* alpha_bar, const void* work,
                     int slices, hipStream_t st) {
  using T = typename P::T;
  const Layout L = layout<P>(N, M, K);
  const char* w = (const char*)work;
  const int Kp = padded(K), Mp = padded(M);
  const T *qst = (const T*)(w + L.qst), *qst_lo = (const T*)(w + L.qst_lo);
  const T *G = (const T*)(w + L.g), *G_lo = (const T*)(w + L.g_lo);
  const int nit = (N + Q::BM - 1) / Q::BM, nct = (Kp + Q::BN - 1) / Q::BN;
  const double* e_part = (const double*)(w + L.e_part);
  const double* ab_part = (const double*)(w + L.ab_part);
  const int nst = Mp / P::BN, nsi = (N + P::BM - 1) / P::BM;  // the scores pass's tile counts
  if (slices < 1 || Mp % (slices * Q::KT) != 0) return hipErrorInvalidValue;
  auto run = [&]<typename OT>() {
    static bool attr = false;  // operand tiles above 64 KB of LDS need the opt-in
    if (!attr && sizeof(Smem<Q>) > 65536) {
      const hipError_t a = hipFuncSetAttribute((const void*)k_qbar<Q, OT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)sizeof(Smem<Q>));
      if (a != hipSuccess) return a;
    }
    attr = true;
    hipLaunchKernelGGL((k_qbar<Q, OT>), dim3(nct, nit, slices), dim3(256), sizeof(Smem<Q>), st, N, K, Mp, Kp,
                       Mp / slices, G, G_lo, qst, qst_lo, static_cast<OT*>(Qbar), M, nst, e_part, e, nsi, ab_part,
                       alpha_bar);
    return hipGetLastError();
  };
  if constexpr (sizeof(T) == 8) {  // FP64 operands accumulate in FP64
    if (f32) return hipErrorInvalidValue;
    return run.template operator()<double>();
  } else {
    return f32 ? run.template operator()<float>() : run.template operator()<double>();
  }
}

}  // namespace

size_t gap_workspace_bytes(int N, int M, int K, int prec) {
  switch (prec) {
    case 0: return layout<PF64>(N, M, K).total;
    case 1: return layout<PF32>(N, M, K).total;
    case 2: return layout<PBF16>(N, M, K).total;
    default: return layout<PBF16X3>(N, M, K).total;
  }
}

hipError_t launch_gap_scores(int prec, int N, int M, int K, const double* Q, const double* Qs, const double* alpha,
                             int zeta, double* e, double* alpha_bar, bool sums, bool q_ready, void* work, int tile,
                             hipStream_t st) {
  if (N == 0) return hipSuccess;
  if (q_ready && !gap_q_operand(prec, N, M, K, work)) return hipErrorInvalidValue;
  switch (prec) {
    case 0: return scores_impl<PF64>(N, M, K, Q, Qs, alpha, zeta, e, alpha_bar, sums, q_ready, work, st);
    case 1: return scores_impl<PF32>(N, M, K, Q, Qs, alpha, zeta, e, alpha_bar, sums, q_ready, work, st);
    case 2:
      if (tile == 1)
        return scores_impl<PBF16D>(N, M, K, Q, Qs, alpha, zeta, e, alpha_bar, sums, q_ready, work, st);
      return scores_impl<PBF16>(N, M, K, Q, Qs, alpha, zeta, e, alpha_bar, sums, q_ready, work, st);
    default: return scores_impl<PBF16X3>(N, M, K, Q, Qs, alpha, zeta, e, alpha_bar, sums, q_ready, work, st);
  }
}

void* gap_q_operand(int prec, int N, int M, int K, void* work) {
  if (prec != 2 || !work) return nullptr;
  return static_cast<char*>(work) + layout<PBF16>(N, M, K).qc;
}

int gap_q_pitch(int K) { return padded(K); }

bool gap_fused_supported(int K, int prec) { return prec != 0 && (K + 31) / 32 * 32 <= kFusedK; }

size_t gap_fused_workspace_bytes(int N, int M, int K, int prec, int target) {
  switch (prec) {
    case 1: return fused_layout<FF32>(N, M, K, target).total;
    case 2: return fused_layout<FB16>(N, M, K, target).total;
    default: return fused_layout<FB16X3>(N, M, K, target).total;
  }
}

hipError_t launch_gap_fused(int prec, int N, int M, int K, const double* Q, const double* Qs, const double* alpha,
                            int zeta, double* e, double* alpha_bar, void* Qbar, bool f32, void* work, int target,
                            hipStream_t st) {
  if (N == 0) return hipSuccess;
  static bool attr_set[4][2] = {};
  auto run = [&]<typename F>() {
    auto go = [&]<typename OT>() {
      if (!attr_set[prec][sizeof(OT) == 4]) {  // opt in to more than 64 KB of LDS per workgroup
        hipError_t a = hipFuncSetAttribute((const void*)k_gap_fused<F, OT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(FusedSmem<F>));
        if (a != hipSuccess) return a;
        attr_set[prec][sizeof(OT) == 4] = true;
      }
      return fused_impl<F, OT>(N, M, K, Q, Qs, alpha, zeta, e, alpha_bar, static_cast<OT*>(Qbar), work, target, st);
    };
    return f32 ? go.template operator()<float>() : go.template operator()<double>();
  };
  switch (prec) {
    case 1: return run.template operator()<FF32>();
    case 2: return run.template operator()<FB16>();
    default: return run.template operator()<FB16X3>();
  }
}

int gap_qbar_slices(int N, int M, int K, int prec, int tile) {
  const int Mp = padded(M);
  int kt, bm, bn;
  switch (prec) {
    case 0: kt = QbarTile<PF64>::KT, bm = QbarTile<PF64>::BM, bn = QbarTile<PF64>::BN; break;
    case 1: kt = QbarTile<PF32>::KT, bm = QbarTile<PF32>::BM, bn = QbarTile<PF32>::BN; break;
    case 2:
      if (tile == 1) kt = QbarSmallBF16::KT, bm = QbarSmallBF16::BM, bn = QbarSmallBF16::BN;
      else kt = QbarTile<PBF16>::KT, bm = QbarTile<PBF16>::BM, bn = QbarTile<PBF16>::BN;
      break;
    default: kt = QbarTile<PBF16X3>::KT, bm = QbarTile<PBF16X3>::BM, bn = QbarTile<PBF16X3>::BN; break;
  }
  // one slice already has eight workgroups per CU: a second would only add a
  // second N x K part to write here and to read in the adjoint (262,144 atoms,
  // n = l = 10: Qbar 2.17 -> 1.98 ms, adjoint 5.12 -> 5.03 ms with one slice)
  const long long grid = (long long)((N + bm - 1) / bm) * ((K + bn - 1) / bn);
  if (grid >= 2048) return 1;
  // two slices once each keeps at least four K-steps
  return (Mp % (2 * kt) == 0 && Mp / 2 >= 4 * kt) ? 2 : 1;
}

hipError_t launch_gap_qbar(int prec, int N, int M, int K, void* Qbar, bool f32, double* e, double* alpha_bar,
                           const void* work, int slices, int tile, hipStream_t st) {
  if (N == 0) return hipSuccess;
  switch (prec) {
    case 0: return qbar_impl<PF64>(N, M, K, Qbar, f32, e, alpha_bar, work, slices, st);
    case 1: return qbar_impl<PF32>(N, M, K, Qbar, f32, e, alpha_bar, work, slices, st);
    case 2:
      // both scores tiles are 128 x 128, so the partial sums are indexed alike
      static_assert(PBF16::BM == PBF16D::BM && PBF16::BN == PBF16D::BN, "scores tiles of one shape");
      if (tile == 1) return qbar_impl<PBF16, QbarSmallBF16>(N, M, K, Qbar, f32, e, alpha_bar, work, slices, st);
      return qbar_impl<PBF16>(N, M, K, Qbar, f32, e, alpha_bar, work, slices, st);
    default: return qbar_impl<PBF16X3>(N, M, K, Qbar, f32, e, alpha_bar, work, slices, st);
  }
}

}  // namespace soap
