// Descriptor forward and adjoint kernels (FP64 VALU).
//
// k_pair_prep, per neighbour pair i -> j (d = r_j + T - r_i, r = |d|,
// u = d / r): everything of Eq. (08) that depends on the pair alone, written as
// the pair's fields in HBM (blocks of 64 pairs, field-major, so every store and
// every per-lane load of a field is one contiguous run) that the forward and the
// adjoint kernels share:
//   B_k = 4 pi A b_k          radial overlaps, Eqs. (02), (04), (19), (06), Eq. (15)
//   w_l e_l                   ilexp, Sec. III.C
//   u_z, u_x, u_y             the direction (the real harmonics' arguments)
// and, for forces, dB_k/dr, d(w_l e_l)/dr and 1/r.  The azimuthal powers
// (u_x + i u_y)^m are formed from u_x, u_y by the kernels that use them.
//
// k_descriptor, one 64-lane wavefront per centre atom.  Its neighbours of one
// species are compacted with a wave ballot and their fields staged in LDS, 32
// at a time.  Each lane owns one (l, m) record (l_max = 8, 12: both real
// harmonics) or whole columns lm of c (l_max = 6, 10, where that fills the lanes
// better) and takes the neighbours one after the other: it evaluates
// Qbar_lm(u_z) as a short polynomial and accumulates its harmonics times every
// B_k in registers:
//   c_{k,lm} += B_k w_l e_l Y_lm                                    (Eq. (08))
// so no cross-lane sum is needed; the central atom joins l = 0 and c goes to
// HBM.  The power spectrum p_{ab l} = sum_m c_{a,lm} c_{b,lm}
// (the real form of Eq. (09)), packed a <= b then l with sqrt(2) off the
// diagonal, and q = p / |p| follow from c staged in LDS.
//
// Adjoint: each wave of k_pair_adjoint first forms, for its atom, vbar =
// (qbar - q (q.qbar)) / |p| and cbar = M c
// (M_aa = 2 vbar_aal, M_ab = sqrt(2) vbar_abl), the derivative of the power
// spectrum and of the normalisation.  k_pair_adjoint then takes the pairs in
// rounds of up to 64, one pair per lane, or R = 2, 4, 8 lanes per pair in a round
// with fewer pairs left (each lane a share of the degrees l): a lane reads its
// pair's fields and runs over its records (l, m), with the cbar of the
// neighbour's species and the record table read from LDS:
//   U_lm = sum_k cbar_{k,lm} dB_k/dr,  V_lm = sum_k cbar_{k,lm} B_k,
//   dE/dd = sum_lm [(U_lm a_lm + V_lm da_lm/dr) u + V_lm w_l e_l (I - u u^T) grad_u Y_lm / r]
// with a_lm = w_l e_l Y_lm, summed in the lane's registers.  Forces are gathered
// per atom through the reverse-pair index: no atomics, so FP64 results are
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pair_kernels.h"
#include "soap_device.h"

namespace soap {

namespace {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Keeps a batch of loads in flight together: the empty statement takes every
// value in a register, so the compiler cannot move a load down into the
// conditional code that consumes it, where each load would wait for its own
// memory round trip.  It reads and writes nothing.
template <int B, typename T>
__device__ __forceinline__ void hold_batch(T (&v)[B]) {
#pragma unroll
  for (int u = 0; u < B; ++u) asm volatile("" : "+v"(v[u]));
}

// packed index of the unordered channel pair a <= b ("for a, for b >= a")
__device__ inline int ab_index(int a, int b, int nch) { return a * nch - a * (a - 1) / 2 + (b - a); }

__device__ inline void ab_decode(int ab, int nch, int& a, int& b) {
  a = 0;
  while (ab >= nch - a) {
    ab -= nch - a;
    ++a;
  }
  b = a + ab;
}

__device__ inline int isqrt_small(int v) {
  int l = 0;
  while ((l + 1) * (l + 1) <= v) ++l;
  return l;
}

constexpr int even(int w) { return w + (w & 1); }
template <int NMAX, int LMAX>
struct Shape {
  static constexpr int NREC = (LMAX + 1) * (LMAX + 2) / 2;
  static constexpr int E2 = (NREC + 63) / 64;  // records per lane of the forward kernel
  static constexpr int NC = LMAX / 2 + 1;  // polynomial terms in u_z^2
  // pair row, forward part: B_k | w_l e_l | u_z u_x u_y
  static constexpr int FB = 0, FW = NMAX, FU = FW + LMAX + 1, FX = FU + 1, FY = FU + 2;
  static constexpr int FR = even(FY + 1);
  // derivative part: dB_k/dr | d(w_l e_l)/dr | 1/r
  static constexpr int XD = 0, XW = NMAX, XI = XW + LMAX + 1;
  static constexpr int XR = even(XI + 1);
  // HBM: blocks of 64 pairs, field-major inside a block (field f of pair p at
  // (p / 64) * ROW * 64 + f * 64 + p % 64)
  static constexpr int ROW = FR + XR;  // doubles per pair
  // forward kernel: CH pairs staged in LDS rows of FRP doubles: the azimuthal
  // powers (u_x + i u_y)^m, m = 0..LMAX (LZ doubles, formed there from u_x, u_y),
  // then the forward part of the pair row.  FRP is even, for 16-byte reads, and
  // 2 mod 4, so that the staging writes spread over the banks
  static constexpr int LZ = 2 * (LMAX + 1);
  static constexpr int CH = 32, FRP = (LZ + FR) | 2;
  // forward lanes: one (l, m) record (both real harmonics) per lane slot, or one
  // column lm of c per lane slot where that fills the 64 lanes better: l_max = 6
  // has 28 records but 49 columns (one pass either way), l_max = 10 66 records
  // (two passes, the second with 2 live lanes) but 121 columns (two passes)
  static constexpr bool COLS = LMAX == 6 || LMAX == 10;
  static constexpr int EC = ((LMAX + 1) * (LMAX + 1) + 63) / 64;  // columns per lane
};

// columns lane + 64 e (e < EC) of a whole wave: lm = l^2 + l + m', the cos part of
// record (l, |m'|) for m' >= 0 and its sin part for m' < 0; the record's
// polynomial from the tables (records m outer, l = m..L inner); columns past
// (L + 1)^2: zero polynomial and the sink column
template <int EC, int NC>
struct LaneColumns {
  double cf[EC][NC];
  int l[EC], m[EC], par[EC], sn[EC], lm[EC];
};

// the columns lm = l^2 + l + m' of l_max = LMAX in the order of the degree
// (l - |m'|) / 2 of their polynomial in u_z^2, highest first, so that the lane
// slots 64.. of a wave (the second column of every lane) need fewer Horner steps;
// terms[e]: the polynomial terms that slots 64 e .. 64 e + 63 need
constexpr int column_degree(int lm) {
  int l = 0;
  while ((l + 1) * (l + 1) <= lm) ++l;
  const int ms = lm - l * l - l;
  return (l - (ms < 0 ? -ms : ms)) >> 1;
}

template <int LMAX>
struct ColumnOrder {
  static constexpr int NCOL = (LMAX + 1) * (LMAX + 1), NG = (NCOL + 63) / 64;
  short lm[NCOL];
  int terms[NG];
  constexpr ColumnOrder() : lm(), terms() {
    int k = 0;
    for (int d = LMAX / 2; d >= 0; --d)
      for (int c = 0; c < NCOL; ++c)
        if (column_degree(c) == d) lm[k++] = (short)c;
    for (int g = 0; g < NG; ++g) terms[g] = column_degree(lm[64 * g]) + 1;
  }
};

template <int LMAX>
__device__ constexpr ColumnOrder<LMAX> kColumnOrder{};

template <int LMAX, int EC, int NC>
__device__ inline void lane_columns(const DevTables* __restrict__ T, int lane, int L, int LL, LaneColumns<EC, NC>& C) {
  constexpr int NCOL = (LMAX + 1) * (LMAX + 1);
#pragma unroll
  for (int e = 0; e < EC; ++e) {
    const int sl = lane + 64 * e;
    const int j = sl < NCOL ? kColumnOrder<LMAX>.lm[sl] : NCOL;
    const bool ok = j < LL;
    int l = 0;
    while (ok && (l + 1) * (l + 1) <= j) ++l;
    const int ms = ok ? j - l * l - l : 0, m = ms < 0 ? -ms : ms;
    const int rec = m * (L + 1) - m * (m - 1) / 2 + (l - m);
    const int jj = rec % kRecLanes, slot = rec / kRecLanes;
    C.l[e] = l;
    C.m[e] = m;
    C.par[e] = ok ? (T->rec_lmp[jj][slot] >> 16) : 0;
    C.sn[e] = ms < 0 ? 1 : 0;
    C.lm[e] = ok ? j : LL;
#pragma unroll
    for (int x = 0; x < NC; ++x) C.cf[e][x] = ok ? T->rec_coef[jj][slot][x] : 0.0;
  }
}

// records lane + 64 e (e < E2) of a whole wave, read straight from the tables;
// records past NREC: zero polynomial, sink columns
template <int E2, int NC>
struct LaneRecords {
  double cf[E2][NC];
  int l[E2], m[E2], par[E2], lmc[E2], lms[E2];
};

template <int E2, int NC>
__device__ inline void lane_records(const DevTables* __restrict__ T, int lane, int nrec, int LL,
                                    LaneRecords<E2, NC>& R) {
#pragma unroll
  for (int e = 0; e < E2; ++e) {
    const int r = lane + 64 * e;
    const bool ok = r < nrec;
    const int jj = ok ? r % kRecLanes : 0, slot = ok ? r / kRecLanes : 0;
    const int info = ok ? T->rec_lmp[jj][slot] : 0;
    R.l[e] = info & 255;
    R.m[e] = (info >> 8) & 255;
    R.par[e] = info >> 16;
    const int lc = ok ? T->rec_lm[jj][slot][0] : -1, ls = ok ? T->rec_lm[jj][slot][1] : -1;
    R.lmc[e] = lc < 0 ? LL : lc;
    R.lms[e] = ls < 0 ? LL : ls;
#pragma unroll
    for (int x = 0; x < NC; ++x) R.cf[e][x] = ok ? T->rec_coef[jj][slot][x] : 0.0;
  }
}

// (c_r + i c_i) <- (c_r + i c_i)(u_x + i u_y) with explicit FMAs, so that every
// kernel forming the powers (u_x + i u_y)^m gets the same bits
__device__ inline void azimuthal_step(double& cr, double& ci, double ux, double uy) {
  const double nr = fma(cr, ux, -(ci * uy));
  ci = fma(cr, uy, ci * ux);
  cr = nr;
}

// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8), each
// with its own L2.  The per-atom kernels number their atoms XCD by XCD (workgroup
// b takes atom (b mod 8) per + b / 8 with per = ceil(n / 8)), so that atoms next
// to each other, whose pair ranges share the cache lines at their ends, meet in
// one L2; the grid is 8 per workgroups, and those past n do nothing.
__host__ __device__ inline int xcd_per(int n) { return (n + 7) >> 3; }
__device__ inline int xcd_item(int b, int n) { return (b & 7) * xcd_per(n) + (b >> 3); }

// Two launches per list: PART 1 writes the radial fields (B_k, dB_k/dr) and the
// central atom's factors, PART 2 the angular ones (w_l e_l, its derivative, u
// and 1/r; the azimuthal powers are formed where they are used, which costs less
// than moving them through HBM).  Each pair's serial FP64 chain is split in two,
// each half runs with the registers it needs (the double-double radial stage
// needs about twice those of the angular one), and the two are timed apart.
// DD: the radial stage in double-double arithmetic (radial<..., true>)
// RT: the storage type of the pair fields (double, or float in the mixed modes,
// where the arithmetic stays FP64 and only the stored values are rounded)
template <int NMAX, int LMAX, bool DERIV, bool DD, int PART, typename RT>
__global__ __launch_bounds__(256) void k_pair_prep(DevParams P, const DevTables* __restrict__ T, int bound,
                                                     const int* __restrict__ count, const double* __restrict__ dx,
                                                     const double* __restrict__ dy, const double* __restrict__ dz,
                                                     RT* __restrict__ rows, double* __restrict__ bc) {
  using S = Shape<NMAX, LMAX>;
  __shared__ PairTab<NMAX, LMAX> tab;
  // pairs 0..n_pairs: the bound, or the device-side count cut at the bound
  const int n_pairs = count ? min(bound, max(*count, 0)) : bound;
  const int pblock = blockIdx.x;
  constexpr bool angular = PART == 2;
  if (pblock > 0 && (int)(pblock * blockDim.x) >= n_pairs) return;  // block 0 also writes bc
  const int p = pblock * blockDim.x + threadIdx.x;
  double x = 0.0, y = 0.0, z = 0.0;
  if (p < n_pairs) {  // in flight while the tables are staged
    x = dx[p];
    y = dy[p];
    z = dz[p];
  }
  stage_pair_tables<NMAX, LMAX>(T, tab, threadIdx.x, blockDim.x);
  __syncthreads();
  if (!angular && blockIdx.x == 0 && threadIdx.x == 0) {
    // central atom: a Gaussian at r = 0, where e_0 = 1, e_{l>0} = 0, Y_00 = 1 / sqrt(4 pi)
    double B[NMAX], dB[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) B[k] = dB[k] = 0.0;
    radial<NMAX, false, DD>(P, tab, 0.0, B, dB);
#pragma unroll
    for (int k = 0; k < NMAX; ++k) bc[k] = P.cw * B[k] * tab.lw[0] * 0.28209479177387814;
  }
  if (p >= n_pairs) return;
  const double r = sqrt(x * x + y * y + z * z);
  // field f of this pair: one coalesced 512-byte segment per field for each 64 pairs
  RT* __restrict__ row = rows + (size_t)(p >> 6) * (S::ROW * 64) + (p & 63);
  auto st = [&](int f, double v) { row[f * 64] = (RT)v; };
  if (!angular) {
    double B[NMAX], dB[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) B[k] = dB[k] = 0.0;  // channels k >= n_max stay zero
    radial<NMAX, DERIV, DD>(P, tab, r, B, dB);
    if (!(r < P.rc)) {  // a pair of a list built with a skin beyond r_cut: no density, no gradient
#pragma unroll
      for (int k = 0; k < NMAX; ++k) B[k] = dB[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < NMAX; ++k) st(S::FB + k, B[k]);
    if (DERIV) {
#pragma unroll
      for (int k = 0; k < NMAX; ++k) st(S::FR + S::XD + k, dB[k]);
    }
    return;
  }
  const double ir = 1.0 / r;
  const double sp = P.s0p + P.ap * r;
  const double zz = r * r / (sp * sp);
  constexpr int LE = DERIV ? LMAX + 1 : LMAX;
  double e[LE + 1];
#pragma unroll
  for (int l = 0; l <= LE; ++l) e[l] = 0.0;
  ilexp<LE>(zz, P.l + (DERIV ? 1 : 0), tab.rec[DERIV ? 2 : 1], tab.rec[DERIV ? 1 : 0], tab.idf, e);
  const double izz = 1.0 / zz;
  const double dzdr = 2.0 * r / (sp * sp) - 2.0 * r * r * P.ap / (sp * sp * sp);
  const double ux = x * ir, uy = y * ir, uz = z * ir;
#pragma unroll
  for (int l = 0; l <= LMAX; ++l) st(S::FW + l, tab.lw[l] * e[l]);
  st(S::FU, uz);
  st(S::FX, ux);
  st(S::FY, uy);
  if (DERIV) {
    // d e_l / dz = e_{l+1} + (l/z - 1) e_l
#pragma unroll
    for (int l = 0; l <= LMAX; ++l)
      st(S::FR + S::XW + l, tab.lw[l] * (e[l + 1] + ((double)l * izz - 1.0) * e[l]) * dzdr);
    st(S::FR + S::XI, ir);
  }
}

// two consecutive FP64 values to or from storage of type double or float (the
// mixed modes store the pair fields, c and qbar of the energy and force path in
// FP32; the arithmetic stays FP64)
__device__ __forceinline__ void store_pair(double* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }
__device__ __forceinline__ void store_pair(float* p, double2 v) {
  *reinterpret_cast<float2*>(p) = float2{(float)v.x, (float)v.y};
}
__device__ __forceinline__ double2 load_pair(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ double2 load_pair(const float* p) {
  const float2 f = *reinterpret_cast<const float2*>(p);
  return double2{(double)f.x, (double)f.y};
}

// fields 0..WIDTH-1 of the compacted pairs idx[0..cnt) copied into LDS rows,
// dst[t * STRIDE + f]; for consecutive pairs each field is one or two
// contiguous runs in HBM.  BATCH loads per lane are issued before the first is
// stored, so the wave waits for memory ceil(WIDTH CH / (64 BATCH)) times instead
// of once per load; out-of-range slots read the first field of the first block.
template <int WIDTH, int ROW, int CH, int STRIDE, int BATCH, typename RT>
__device__ inline void stage_fields(const RT* __restrict__ rows, const int* idx, int cnt,
                                    double* __restrict__ dst, int lane) {
  constexpr int ITER = (WIDTH * CH + 63) / 64;
#pragma unroll 1
  for (int k0 = 0; k0 < ITER; k0 += BATCH) {
    double v[BATCH];
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int u = lane + 64 * (k0 + k);
      const int f = u / CH, t = u % CH;
      const bool ok = k0 + k < ITER && u < WIDTH * CH && t < cnt;
      const int p = ok ? idx[t] : 0;
      v[k] = (double)rows[ok ? (size_t)(p >> 6) * (ROW * 64) + f * 64 + (p & 63) : 0];
    }
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int u = lane + 64 * (k0 + k);
      const int f = u / CH, t = u % CH;
      if (k0 + k < ITER && u < WIDTH * CH && t < cnt) dst[t * STRIDE + f] = v[k];
    }
  }
}

// The power spectrum P_l = C_l C_l^T of one atom (C_l: n_ch x (2l + 1), the
// real form of Eq. (09)) on the matrix cores: BF16 operands, FP32 accumulation,
// one v_mfma_f32_16x16x32_bf16 per 16 x 16 tile of channel pairs and per l
// (2l + 1 <= 25 fits one 32-deep step).  c is read from csh in its layout
// [species][lm][k]; the packed entries a <= b (sqrt(2) off the diagonal) go to
// pv[ab L1 + l].  Operand lane layout: lane j holds row j % 16 and contraction
// positions 8 (j / 16) .. 8 (j / 16) + 7; result lane j holds rows
// 4 (j / 16) .. + 3 of column j % 16.  Returns this lane's sum of squares.  CT:
// the type c is staged in (double, or float where c was stored in FP32).
template <int NMAX, typename CT>
__device__ __forceinline__ double power_spectrum_mfma(const DevParams& P, const CT* csh, double* pv, int lane) {
  const int n = P.n, nch = P.nch, L1 = P.l + 1, LLP = P.LL + 1;
  const int r16 = lane & 15, kq = lane >> 4, T = (nch + 15) / 16;
  // operand: channel row a, positions m' = 8 kq + j of degree l
  auto operand = [&](int a, int l) {
    bf16x8 v;
    const int sa = a / n, ka = a - sa * n;
    const CT* c = csh + ((size_t)sa * LLP + l * l) * NMAX + ka;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int m = 8 * kq + j;
      v[j] = (__bf16)(float)((a < nch && m <= 2 * l) ? (double)c[m * NMAX] : 0.0);
    }
    return v;
  };
  double ss = 0.0;
  for (int ta = 0; ta < T; ++ta)
    for (int tb = ta; tb < T; ++tb)
      for (int l = 0; l < L1; ++l) {
        const bf16x8 A = operand(16 * ta + r16, l);
        const bf16x8 B = tb == ta ? A : operand(16 * tb + r16, l);
        const f32x4 D = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        const int b = 16 * tb + r16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 16 * ta + 4 * kq + r;
          if (a < nch && b < nch && a <= b) {
            const double v = (double)D[r] * (a != b ? kSqrt2 : 1.0);
            pv[ab_index(a, b, nch) * L1 + l] = v;
            ss = fma(v, v, ss);
          }
        }
      }
  return ss;
}

// the forward keeps the power spectrum in LDS when c and p of one atom together
// stay within the row staging area or within 16 KB (not at n_max = 10)
template <int NMAX, int LMAX>
__host__ __device__ inline bool fwd_p_in_lds(const DevParams& P) {
  using S = Shape<NMAX, LMAX>;
  const int need = P.ns * NMAX * (P.LL + 1) + P.K;
  // at n_max = 10, which runs 3 waves per SIMD, LDS beyond the staging area
  // would cost a wave: p goes to the q row there
  return need <= S::CH * S::FRP || (NMAX != 10 && need * (int)sizeof(double) <= 16384);
}

// the FP32 staging of c in the forward's epilogue (FP32 storage assumed): several
// species, the matrix-core power spectrum, and p in the q row
template <int NMAX, int LMAX>
__host__ __device__ inline bool fwd_c32(const DevParams& P) {
  return P.ps_mfma && P.ns > 1 && !fwd_p_in_lds<NMAX, LMAX>(P);
}

// Registers: 4 waves per SIMD up to n_max = 8, 3 at n_max = 10 (155 VGPRs; with
// p out of LDS, 12 waves per CU fit), 2 at n_max = 12
template <int NMAX, int LMAX, typename ST>
__global__ __launch_bounds__(64, NMAX <= 8 ? 4 : (NMAX == 10 ? 3 : 2)) void k_descriptor(DevParams P, const DevTables* __restrict__ T,
                                                                     int n_atoms, const int* __restrict__ offsets,
                                                                     int bound, const int* __restrict__ nj,
                                                                     const int* __restrict__ species,
                                                                     const ST* __restrict__ rows,
                                                                     const double* __restrict__ bc_in,
                                                                     ST* __restrict__ c_out,
                                                                     double* __restrict__ q_out, int q_pitch,
                                                                     double* __restrict__ pnorm_out,
                                                                     __bf16* __restrict__ qc, int qc_pitch) {
  using S = Shape<NMAX, LMAX>;
  constexpr int E2 = S::E2, NC = S::NC, CH = S::CH, FRP = S::FRP;
  extern __shared__ __align__(16) double dyn[];
  __shared__ int idx[CH];

  const int i = xcd_item(blockIdx.x, n_atoms);
  if (i >= n_atoms) return;
  const int lane = threadIdx.x;
  const int n = P.n, LL = P.LL, LLP = LL + 1, nch = P.nch;
  const int p0 = min(offsets[i], bound), p1 = min(offsets[i + 1], bound);  // pairs below the bound only
  const int si = P.ns == 1 ? 0 : species[i];
  ST* __restrict__ ci_out = c_out + (size_t)i * P.ns * NMAX * LLP;
  constexpr bool COLS = S::COLS;
  constexpr int EC = S::EC;
  // record mode: acc[e][part][k]; column mode: acc[e][0][k] (EC columns)
  constexpr int NE = COLS ? EC : E2, NP = COLS ? 1 : 2;
  LaneRecords<COLS ? 1 : E2, NC> R;
  LaneColumns<COLS ? EC : 1, NC> C;
  if constexpr (COLS) lane_columns<LMAX, EC, NC>(T, lane, P.l, LL, C);
  else lane_records<E2, NC>(T, lane, S::NREC, LL, R);

  for (int s = 0; s < P.ns; ++s) {
    double acc[NE][NP][NMAX];
#pragma unroll
    for (int e = 0; e < NE; ++e)
#pragma unroll
      for (int h = 0; h < NP; ++h)
#pragma unroll
        for (int k = 0; k < NMAX; ++k) acc[e][h][k] = 0.0;
    for (int w0 = p0; w0 < p1; w0 += CH) {
      const int pp = w0 + lane;
      const bool take = lane < CH && pp < p1 && (P.ns == 1 || species[nj[pp]] == s);
      const unsigned long long mask = __ballot(take);
      __syncthreads();  // the previous chunk is done with idx and the rows
      if (take) idx[__popcll(mask & ((1ull << lane) - 1ull))] = pp;
      const int cnt = __popcll(mask);
      __syncthreads();
      stage_fields<S::FR, S::ROW, CH, FRP, 6, ST>(rows, idx, cnt, dyn + S::LZ, lane);
      __syncthreads();
      if (lane < cnt) {  // the azimuthal powers of staged pair `lane`
        double* __restrict__ zt = dyn + lane * FRP;
        const double ux = zt[S::LZ + S::FX], uy = zt[S::LZ + S::FY];
        double cr = 1.0, ci = 0.0;
#pragma unroll
        for (int m = 0; m <= LMAX; ++m) {
          zt[2 * m] = cr;
          zt[2 * m + 1] = ci;
          azimuthal_step(cr, ci, ux, uy);
        }
      }
      __syncthreads();
#pragma unroll 2
      for (int t = 0; t < cnt; ++t) {
        const double* __restrict__ zt = dyn + t * FRP;  // (u_x + i u_y)^m at 2m, 2m + 1
        const double* __restrict__ rt = zt + S::LZ;     // the forward fields
        auto row = [&](int f) { return rt[f]; };
        double b[NMAX];
#pragma unroll
        for (int k = 0; k < NMAX; k += 2) {
          const double2 v = *reinterpret_cast<const double2*>(rt + S::FB + k);
          b[k] = v.x;
          b[k + 1] = v.y;
        }
        const double uz = row(S::FU), x2 = uz * uz;
        if constexpr (COLS) {
          // the same products as the record mode (a column is one of its two parts)
#pragma unroll
          for (int e = 0; e < EC; ++e) {
            // the higher coefficients of this group's columns are zero (the same
            // bits as running over all NC terms); e is unrolled, so NT is a constant
            constexpr ColumnOrder<LMAX> order{};
            const int NT = e == 0 ? order.terms[0] : order.terms[ColumnOrder<LMAX>::NG - 1];
            double Rv = C.cf[e][NT - 1];
#pragma unroll
            for (int t2 = NT - 2; t2 >= 0; --t2) Rv = fma(Rv, x2, C.cf[e][t2]);
            const double Q = C.par[e] ? uz * Rv : Rv;
            const double a = row(S::FW + C.l[e]) * Q;
            const double a0 = a * zt[2 * C.m[e] + C.sn[e]];
#pragma unroll
            for (int k = 0; k < NMAX; ++k) acc[e][0][k] = fma(a0, b[k], acc[e][0][k]);
          }
        } else {
#pragma unroll
          for (int e = 0; e < E2; ++e) {
            double Rv = R.cf[e][NC - 1];
#pragma unroll
            for (int t2 = NC - 2; t2 >= 0; --t2) Rv = fma(Rv, x2, R.cf[e][t2]);
            const double Q = R.par[e] ? uz * Rv : Rv;
            const double a = row(S::FW + R.l[e]) * Q;
            const double a0 = a * zt[2 * R.m[e]], a1 = a * zt[2 * R.m[e] + 1];
#pragma unroll
            for (int k = 0; k < NMAX; ++k) {
              acc[e][0][k] = fma(a0, b[k], acc[e][0][k]);
              acc[e][NP - 1][k] = fma(a1, b[k], acc[e][NP - 1][k]);
            }
          }
        }
      }
    }
    // c of species s: LL + 1 columns lm (the last one a sink, left zero) of NMAX
    // channels; with one species it also goes to LDS, where the power spectrum
    // reads it, once the wave is done with the staged rows
    ST* __restrict__ cs = ci_out + (size_t)s * LLP * NMAX;
    const bool c_lds = P.ns == 1;
    if (c_lds) __syncthreads();
    if constexpr (COLS) {
#pragma unroll
      for (int e = 0; e < EC; ++e) {
        if (C.lm[e] == LL) continue;
        const bool central = C.lm[e] == 0 && s == si;
        ST* __restrict__ dc = cs + C.lm[e] * NMAX;
#pragma unroll
        for (int k = 0; k < NMAX; k += 2) {
          const double2 v{acc[e][0][k] + (central ? bc_in[k] : 0.0),
                          acc[e][0][k + 1] + (central ? bc_in[k + 1] : 0.0)};
          store_pair(dc + k, v);
          if (c_lds) *reinterpret_cast<double2*>(dyn + C.lm[e] * NMAX + k) = v;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < (COLS ? 0 : E2); ++e) {
      if (lane + 64 * e >= S::NREC || R.lmc[e] == LL) continue;
      const bool central = R.lmc[e] == 0 && s == si;
      ST* __restrict__ dc = cs + R.lmc[e] * NMAX;
#pragma unroll
      for (int k = 0; k < NMAX; k += 2) {
        const double2 v{acc[e][0][k] + (central ? bc_in[k] : 0.0), acc[e][0][k + 1] + (central ? bc_in[k + 1] : 0.0)};
        store_pair(dc + k, v);
        if (c_lds) *reinterpret_cast<double2*>(dyn + R.lmc[e] * NMAX + k) = v;
      }
      if (R.lms[e] != LL) {
        ST* __restrict__ ds = cs + R.lms[e] * NMAX;
#pragma unroll
        for (int k = 0; k < NMAX; k += 2) {
          const double2 v{acc[e][NP - 1][k], acc[e][NP - 1][k + 1]};
          store_pair(ds + k, v);
          if (c_lds) *reinterpret_cast<double2*>(dyn + R.lms[e] * NMAX + k) = v;
        }
      }
    }
    if (lane < NMAX) {
      cs[LL * NMAX + lane] = (ST)0;
      if (c_lds) dyn[LL * NMAX + lane] = 0.0;
    }
  }
  __threadfence_block();
  __syncthreads();
  // power spectrum from c staged in LDS in its HBM layout [species][lm][k]: lane per
  // channel pair (a, b), a <= b, all l.  p is kept in LDS when it fits
  // (fwd_p_in_lds); otherwise it stays in registers (one channel pair per lane) or
  // goes straight to the q row and is rescaled there, so that several species do
  // not cut the number of wavefronts per CU.  With several species, FP32 storage and the matrix-core power spectrum, c is
  // staged in FP32, the precision it was stored in (its BF16 operands are the
  // same), which halves the LDS the wave holds (fwd_c32)
  const int per_atom = P.ns * NMAX * LLP;
  double* csh = dyn;
  double* __restrict__ qi = q_out + (size_t)i * q_pitch;
  double* __restrict__ pv = fwd_p_in_lds<NMAX, LMAX>(P) ? dyn + per_atom : qi;
  const bool c32 = sizeof(ST) == 4 && fwd_c32<NMAX, LMAX>(P);
  if (P.ns > 1) {
    if (c32) {
      for (int t = lane; t < per_atom / 2; t += 64)
        reinterpret_cast<float2*>(dyn)[t] = reinterpret_cast<const float2*>(ci_out)[t];
    } else {
      for (int t = lane; t < per_atom / 2; t += 64)
        reinterpret_cast<double2*>(csh)[t] = load_pair(ci_out + 2 * t);
    }
    __syncthreads();
  }
  const int L1 = P.l + 1, nab = nch * (nch + 1) / 2;
  // p in the q row with at most one channel pair per lane (VALU power spectrum):
  // the lane keeps its entries in registers and writes q once, already scaled
  const bool hold = !P.ps_mfma && pv == qi && nab <= 64;
  double pr[LMAX + 1];
  double ss = 0.0;
  if (P.ps_mfma) {
    if constexpr (sizeof(ST) == 4)
      ss = c32 ? power_spectrum_mfma<NMAX>(P, reinterpret_cast<const float*>(dyn), pv, lane)
               : power_spectrum_mfma<NMAX>(P, csh, pv, lane);
    else
      ss = power_spectrum_mfma<NMAX>(P, csh, pv, lane);
  }
  for (int ab = P.ps_mfma ? nab : lane; ab < nab; ab += 64) {
    int a, b;
    ab_decode(ab, nch, a, b);
    const int sa = a / n, sb = b / n;
    const double* ca = csh + sa * LLP * NMAX + (a - sa * n);
    const double* cb = csh + sb * LLP * NMAX + (b - sb * n);
    const double scale = a != b ? kSqrt2 : 1.0;
    // unrolled over l and m, so that the LDS reads of each l are issued together
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
      if (l < L1) {
        double v = 0.0;
#pragma unroll
        for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm) v = fma(ca[lm * NMAX], cb[lm * NMAX], v);
        v *= scale;
        if (hold) pr[l] = v;
        else pv[ab * L1 + l] = v;
        ss = fma(v, v, ss);
      }
    }
  }
  ss = wave_sum(ss);
  const double nrm = sqrt(ss);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  // qc: the bf16 operand row of the GAP contraction, the same rounding of the
  // same q values as a separate conversion pass would apply
  __bf16* __restrict__ qci = qc ? qc + (size_t)i * qc_pitch : nullptr;
  if (pv != qi) {  // p in LDS: every lane writes a contiguous part of q
    __syncthreads();
    for (int k = lane; k < q_pitch; k += 64) qi[k] = k < P.K ? pv[k] * inv : 0.0;
    if (qci)
      for (int k = lane; k < qc_pitch; k += 64) qci[k] = (__bf16)(float)(k < P.K ? pv[k] * inv : 0.0);
  } else {
    if (hold) {
      if (lane < nab) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l)
          if (l < L1) {
            const double x = pr[l] * inv;
            qi[lane * L1 + l] = x;
            if (qci) qci[lane * L1 + l] = (__bf16)(float)x;
          }
      }
    } else {
      // p in the q row, written by other lanes (the matrix-core layout) or several
      // channel pairs per lane: once those stores are visible to the wave, every
      // lane rescales a strided part, sixteen loads in flight at a time (a loop
      // with one load per entry waits one memory round trip per entry)
      constexpr int B = 16;
      __threadfence_block();
      __syncthreads();
      for (int k0 = 0; k0 < P.K; k0 += 64 * B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int k = k0 + lane + 64 * u;
          v[u] = k < P.K ? qi[k] : 0.0;
        }
        hold_batch(v);
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int k = k0 + lane + 64 * u;
          if (k < P.K) {
            const double x = v[u] * inv;
            qi[k] = x;
            if (qci) qci[k] = (__bf16)(float)x;
          }
        }
      }
    }
    for (int k = P.K + lane; k < q_pitch; k += 64) qi[k] = 0.0;
    if (qci)
      for (int k = P.K + lane; k < qc_pitch; k += 64) qci[k] = (__bf16)0.0f;
  }
  if (lane == 0 && pnorm_out) pnorm_out[i] = nrm;
}

// cbar = M(l) c in place for every column lm < LL of one species' cb, one
// column per lane: M_ab(l) = 2 vbar_aal (a = b), sqrt(2) vbar_abl (a != b),
// vbar packed a <= b then l (stored as VT: double, or float in the mixed modes)
template <int NMAX, int LMAX, bool FULL, typename VT>
__device__ __forceinline__ void transform_columns_t(int n, int nch, int LL, int L1, double* cb, const VT* vb,
                                                    int lane) {
  // FULL: n_max and l_max fill the compiled bucket, so every vbar index is a
  // compile-time offset from the column's l (no index arithmetic per entry)
  const int n_ = FULL ? NMAX : n, nch_ = FULL ? NMAX : nch, L1_ = FULL ? LMAX + 1 : L1;
  for (int lm = lane; lm < LL; lm += 64) {
    const int l = isqrt_small(lm);
    double* col = cb + (size_t)lm * NMAX;
    const VT* __restrict__ vl = vb + l;
    double cv[NMAX];
#pragma unroll
    for (int kb = 0; kb < NMAX; kb += 2) {
      const double2 v = *reinterpret_cast<const double2*>(col + kb);
      cv[kb] = v.x;
      cv[kb + 1] = v.y;
    }
    // each vbar entry of the symmetric M(l) is read once; every acc[k] still
    // takes its terms in the order kb = 0, 1, ...
    double acc[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) acc[k] = 0.0;
#pragma unroll
    for (int a = 0; a < NMAX; ++a)
#pragma unroll
      for (int b = a; b < NMAX; ++b)
        if (b < n_) {
          const double v = (double)vl[(a * nch_ - a * (a - 1) / 2 + (b - a)) * L1_];
          if (a == b) {
            acc[a] = fma(2.0 * v, cv[a], acc[a]);
          } else {
            const double w = kSqrt2 * v;
            acc[a] = fma(w, cv[b], acc[a]);
            acc[b] = fma(w, cv[a], acc[b]);
          }
        }
#pragma unroll
    for (int k = 0; k < NMAX; k += 2) *reinterpret_cast<double2*>(col + k) = double2{acc[k], acc[k + 1]};
  }
}

template <int NMAX, int LMAX, typename VT>
__device__ __forceinline__ void transform_columns(int n, int nch, int LL, int L1, double* cb, const VT* vb,
                                                  int lane) {
  if (n == NMAX && L1 == LMAX + 1) transform_columns_t<NMAX, LMAX, true>(n, nch, LL, L1, cb, vb, lane);
  else transform_columns_t<NMAX, LMAX, false>(n, nch, LL, L1, cb, vb, lane);
}

// The same transform in place for several species: task (column lm, output
// species sa) takes the column's c of every species from cb and forms the n_max
// rows of species sa.  A pass holds whole columns (64 / ns of them), so every
// read of a column precedes the writes to it (one wavefront: its LDS operations
// complete in order).  abx[a][b] = (packed index of {a, b}) * (l_max + 1).  Each
// output takes its terms in the order (sb, kb).
template <int NMAX, typename VT>
__device__ __forceinline__ void transform_columns_species(int n, int ns, int nch, int LL, int L1, int cbs, double* cb,
                                                 const VT* vb, const int* abx, int lane) {
  const int cpp = 64 / ns;  // columns per pass
  const int lmo = lane / ns, sa = lane - lmo * ns;
  for (int c0 = 0; c0 < LL; c0 += cpp) {
    const int lm = c0 + lmo;
    const bool live = lmo < cpp && lm < LL;
    double acc[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) acc[k] = 0.0;
    if (live) {
      const int l = isqrt_small(lm);
      for (int sb = 0; sb < ns; ++sb) {
        const double* col = cb + (size_t)sb * cbs + lm * NMAX;
        double cv[NMAX];
#pragma unroll
        for (int kb = 0; kb < NMAX; kb += 2) {
          const double2 v = *reinterpret_cast<const double2*>(col + kb);
          cv[kb] = v.x;
          cv[kb + 1] = v.y;
        }
#pragma unroll
        for (int ka = 0; ka < NMAX; ++ka) {
          const int a = sa * n + ka;
          if (ka < n) {
            const int* __restrict__ row = abx + a * nch + sb * n;
#pragma unroll
            for (int kb = 0; kb < NMAX; ++kb)
              if (kb < n) acc[ka] = fma((sb * n + kb == a ? 2.0 : kSqrt2) * (double)vb[row[kb] + l], cv[kb], acc[ka]);
          }
        }
      }
    }
    if (live) {
      double* dst = cb + (size_t)sa * cbs + lm * NMAX;
#pragma unroll
      for (int k = 0; k < NMAX; k += 2) *reinterpret_cast<double2*>(dst + k) = double2{acc[k], acc[k + 1]};
    }
  }
}

// cbar_l = M(l) C_l for every l (M(l)_aa = 2 vbar_aal, M(l)_ab = sqrt(2) vbar_abl,
// vbar packed a <= b then l) on the matrix cores: BF16 operands, FP32
// accumulation, v_mfma_f32_16x16x32_bf16 over 16 channel rows x 16 columns m'
// of degree l, contracted over the channels b in steps of 32.  c comes from
// csrc ([species][lm][k], species cbs doubles apart; it may be cb itself: every
// tile of an l is formed in registers before any of them is written); the result
// goes to cb in the same layout.  Entries outside the channels and columns (the sink column, channels
// k >= n_max) are left as they are.  n_ch <= 48.  vb: vbar as double or float, or
// as the BF16 operand entries themselves (VT = __bf16: the factor 2 or sqrt(2)
// already applied, see form_cbar).
template <int NMAX, typename CT, typename VT>
__device__ __forceinline__ void cbar_mfma(const DevParams& P, int cbs, const CT* csrc, CT* cb, const VT* vb,
                                          int lane) {
  const int n = P.n, nch = P.nch, L1 = P.l + 1;
  const int r16 = lane & 15, kq = lane >> 4;
  const int TA = (nch + 15) / 16, TK = (nch + 31) / 32;
  for (int l = 0; l < L1; ++l) {
    const int w = 2 * l + 1, TM = (w + 15) / 16;
    f32x4 D[3][2];
#pragma unroll
    for (int ta = 0; ta < 3; ++ta)
#pragma unroll
      for (int tm = 0; tm < 2; ++tm) D[ta][tm] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int tk = 0; tk < TK; ++tk) {
      bf16x8 Bm[2];
#pragma unroll
      for (int tm = 0; tm < 2; ++tm) {
        const int m = 16 * tm + r16;  // column of C_l
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int b = 32 * tk + 8 * kq + j, sb = b / n;
          Bm[tm][j] = (__bf16)(float)((tm < TM && b < nch && m < w)
                                          ? csrc[(size_t)sb * cbs + (l * l + m) * NMAX + (b - sb * n)]
                                          : 0.0);
        }
      }
#pragma unroll
      for (int ta = 0; ta < 3; ++ta) {
        if (ta >= TA) break;
        const int a = 16 * ta + r16;
        bf16x8 A;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int b = 32 * tk + 8 * kq + j;
          if constexpr (std::is_same_v<VT, __bf16>) {
            A[j] = (a < nch && b < nch) ? vb[ab_index(a < b ? a : b, a < b ? b : a, nch) * L1 + l] : (__bf16)0.0f;
          } else {
            double v = 0.0;
            if (a < nch && b < nch)
              v = (a == b ? 2.0 : kSqrt2) * (double)vb[ab_index(a < b ? a : b, a < b ? b : a, nch) * L1 + l];
            A[j] = (__bf16)(float)v;
          }
        }
#pragma unroll
        for (int tm = 0; tm < 2; ++tm)
          if (tm < TM) D[ta][tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bm[tm], D[ta][tm], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ta = 0; ta < 3; ++ta)
#pragma unroll
      for (int tm = 0; tm < 2; ++tm) {
        const int m = 16 * tm + r16;
        if (ta >= TA || tm >= TM || m >= w) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 16 * ta + 4 * kq + r;
          if (a < nch) {
            const int sa = a / n;
            cb[(size_t)sa * cbs + (l * l + m) * NMAX + (a - sa * n)] = (CT)D[ta][tm][r];
          }
        }
      }
  }
}

// vbar = (qbar - q (q . qbar)) / |p| and cbar_{a,lm} = sum_b M_ab(l) c_{b,lm} of atom
// i (qbar = qbar + qbar2 when qbar2 is not null, in that order), written into cb
// (LDS) in the padded layout of c ([species][lm < LL + 1][k < NMAX], species cbs
// doubles apart) with zeros in the sink column lm = LL and in the channels
// k >= n_max.  vb: K entries of LDS scratch (VT); abx: n_ch^2 ints of LDS
// scratch (several species, VALU transform only).  Ends with a block barrier.
// The atom's c (every species) is first copied into cb and transformed there in
// place: a column of cbar needs only the same column of c.  With one species and
// NMAX <= 8 every global read (c, q, qbar, qbar2, |p|) is issued at once and q,
// qbar stay in registers from the dot product to vbar; otherwise the reads go
// sixteen per lane at a time.  VT = __bf16 (matrix-core transform, several
// species): vb holds the BF16 operands of cbar_mfma, vbar rounded to FP32 as in
// the FP32 layout, times 2 (a = b) or sqrt(2), rounded to BF16; the same
// operands as the FP32 layout gives, in half its LDS.
template <int NMAX, int LMAX, typename ST, typename VT, typename CT>
__device__ __forceinline__ void form_cbar(const DevParams& P, int i, const ST* __restrict__ c,
                                 const double* __restrict__ q, int q_pitch, const double* __restrict__ pnorm,
                                 const ST* __restrict__ qbar, const ST* __restrict__ qbar2, int qbar_pitch,
                                 int cbs, CT* cb, VT* vb, int* abx, int lane) {
  constexpr int B = 16;  // loads per lane in flight
  const int n = P.n, ns = P.ns, nch = P.nch, LL = P.LL, LLP = LL + 1, K = P.K, L1 = P.l + 1;
  const ST* __restrict__ csh = c + (size_t)i * ns * NMAX * LLP;  // c of atom i, [species][lm][k]
  const double* qi = q + (size_t)i * q_pitch;
  const ST* qb = qbar + (size_t)i * qbar_pitch;
  const ST* qb2 = qbar2 ? qbar2 + (size_t)i * qbar_pitch : nullptr;  // a second part of qbar, added
  constexpr bool VB16 = std::is_same_v<VT, __bf16>;
  static_assert(VB16 || std::is_same_v<CT, double>, "FP32 cbar comes from the matrix-core transform only");
  if constexpr (NMAX <= 8 && !VB16) {
    constexpr int KPL = (NMAX * (NMAX + 1) / 2 * (LMAX + 1) + 63) / 64;   // K per lane, one species
    constexpr int CPL = (NMAX * ((LMAX + 1) * (LMAX + 1) + 1) + 63) / 64;  // c per lane
    const int nc = NMAX * LLP;
    if (ns == 1 && K <= 64 * KPL && nc <= 64 * CPL) {
      double cv[CPL], a[KPL], g[KPL], g2[KPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) cv[u] = csh[min(lane + 64 * u, nc - 1)];
#pragma unroll
      for (int u = 0; u < KPL; ++u) {
        const int k = min(lane + 64 * u, K - 1);
        a[u] = qi[k];
        g[u] = qb[k];
      }
      if (qb2) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) g2[u] = qb2[min(lane + 64 * u, K - 1)];
      }
      const double nrm = pnorm[i];
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (lane + 64 * u < nc) cb[lane + 64 * u] = cv[u];
      if (qb2) {
#pragma unroll
        for (int u = 0; u < KPL; ++u) g[u] += g2[u];
      }
      // the same terms in the same order as the batched loop below
      double dot = 0.0;
#pragma unroll
      for (int u = 0; u < KPL; ++u)
        if (lane + 64 * u < K) dot = fma(a[u], g[u], dot);
      dot = wave_sum(dot);
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
#pragma unroll
      for (int u = 0; u < KPL; ++u)
        if (lane + 64 * u < K) vb[lane + 64 * u] = (VT)((g[u] - a[u] * dot) * inv);
      __syncthreads();
      if (P.ps_mfma) cbar_mfma<NMAX>(P, cbs, cb, cb, vb, lane);
      else transform_columns<NMAX, LMAX>(n, nch, LL, L1, cb, vb, lane);
      __syncthreads();
      return;
    }
  }
  {
    // the atom's c, every species, into cb (transformed there in place below)
    const int nc = ns * cbs;
    for (int t0 = 0; t0 < nc; t0 += 64 * B) {
      double v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) v[u] = csh[min(t0 + lane + 64 * u, nc - 1)];
      hold_batch(v);
#pragma unroll
      for (int u = 0; u < B; ++u)
        if (t0 + lane + 64 * u < nc) cb[t0 + lane + 64 * u] = (CT)v[u];
    }
  }
  if constexpr (VB16) {
    // dot = q . qbar; then q and qbar read again (now from the caches) for vbar
    double dot = 0.0;
    for (int k0 = 0; k0 < K; k0 += 64 * B) {
      double a[B], g[B], g2[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int k = min(k0 + lane + 64 * u, K - 1);
        a[u] = qi[k];
        g[u] = qb[k];
      }
      if (qb2) {  // a branch of its own, not one per entry: the loads stay together
#pragma unroll
        for (int u = 0; u < B; ++u) g2[u] = qb2[min(k0 + lane + 64 * u, K - 1)];
        hold_batch(g2);
#pragma unroll
        for (int u = 0; u < B; ++u) g[u] += g2[u];
      }
      hold_batch(a);
      hold_batch(g);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (k0 + lane + 64 * u < K) dot = fma(a[u], g[u], dot);
      }
    }
    dot = wave_sum(dot);
    const double nrm = pnorm[i];
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    // k = (packed pair {a, b}) (l_max + 1) + l, pairs a <= b in rows a: row a
    // spans [rbeg, rend) and its first l_max + 1 entries are the diagonal a = b
    int ra = 0, rbeg = 0, rend = nch * L1;
    for (int k0 = 0; k0 < K; k0 += 64 * B) {
      double a[B], g[B], g2[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int k = min(k0 + lane + 64 * u, K - 1);
        a[u] = qi[k];
        g[u] = qb[k];
      }
      if (qb2) {  // a branch of its own, not one per entry: the loads stay together
#pragma unroll
        for (int u = 0; u < B; ++u) g2[u] = qb2[min(k0 + lane + 64 * u, K - 1)];
        hold_batch(g2);
#pragma unroll
        for (int u = 0; u < B; ++u) g[u] += g2[u];
      }
      hold_batch(a);
      hold_batch(g);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int k = k0 + lane + 64 * u;
        if (k < K) {
          const float v = (float)(((double)(float)g[u] - a[u] * dot) * inv);
          while (k >= rend) {
            ++ra;
            rbeg = rend;
            rend += (nch - ra) * L1;
          }
          vb[k] = (__bf16)(float)((k < rbeg + L1 ? 2.0 : kSqrt2) * (double)v);
        }
      }
    }
    __syncthreads();
    cbar_mfma<NMAX>(P, cbs, cb, cb, vb, lane);
    __syncthreads();
  } else {
    // dot = q . qbar, with qbar kept in vb; then vbar in place, q read again (now
    // from the caches).  Each lane reads back only the entries it wrote.
    double dot = 0.0;
    for (int k0 = 0; k0 < K; k0 += 64 * B) {
      double a[B], g[B], g2[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int k = min(k0 + lane + 64 * u, K - 1);
        a[u] = qi[k];
        g[u] = qb[k];
      }
      if (qb2) {  // a branch of its own, not one per entry: the loads stay together
#pragma unroll
        for (int u = 0; u < B; ++u) g2[u] = qb2[min(k0 + lane + 64 * u, K - 1)];
        hold_batch(g2);
#pragma unroll
        for (int u = 0; u < B; ++u) g[u] += g2[u];
      }
      hold_batch(a);
      hold_batch(g);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (k0 + lane + 64 * u < K) {
          dot = fma(a[u], g[u], dot);
          vb[k0 + lane + 64 * u] = (VT)g[u];
        }
      }
    }
    dot = wave_sum(dot);
    const double nrm = pnorm[i];
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int k0 = 0; k0 < K; k0 += 64 * B) {
      double a[B];
#pragma unroll
      for (int u = 0; u < B; ++u) a[u] = qi[min(k0 + lane + 64 * u, K - 1)];
      hold_batch(a);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int k = k0 + lane + 64 * u;
        if (k < K) vb[k] = (VT)(((double)vb[k] - a[u] * dot) * inv);
      }
    }
    // abx[a][b] = (packed index of the pair {a, b}) * (l_max + 1), the row of vbar
    for (int r = lane; r < (ns > 1 && !P.ps_mfma ? nch * nch : 0); r += 64) {
      const int a = r / nch, b = r - a * nch;
      abx[r] = ab_index(a < b ? a : b, a < b ? b : a, nch) * L1;
    }
    __syncthreads();
    // c of every species is in cb; the sink column and the channels k >= n_max are
    // zero there and stay so
    if (P.ps_mfma) cbar_mfma<NMAX>(P, cbs, cb, cb, vb, lane);
    else if (ns == 1) transform_columns<NMAX, LMAX>(n, nch, LL, L1, cb, vb, lane);
    else transform_columns_species<NMAX>(n, ns, nch, LL, L1, cbs, cb, vb, abx, lane);
    __syncthreads();
  }
}

// LDS of the adjoint: the atom's cbar for every species ([species][lm][k], in
// FP64, or in FP32 where the matrix-core transform forms it: C32), then
// a region that first holds vbar (K values: FP64, or FP32 in the mixed modes
// where that lets more wavefronts share a CU, see launch_pair_adjoint) and then
// the record coefficients [r][NC] and (parity, cos column, sin column) [r][4],
// then the channel-pair index table of form_cbar (n_ch^2 ints, where the VALU
// transform of several species needs it)
template <int NMAX, int LMAX>
struct AdjLds {
  static constexpr int NC = Shape<NMAX, LMAX>::NC;
  __host__ __device__ static int cb_stride(int LL) { return (LL + 1) * NMAX; }
  // the cbar region in doubles (c32: FP32 entries)
  __host__ __device__ static int cb_doubles(int ns, int LL, bool c32) {
    const int e = ns * cb_stride(LL);
    return c32 ? (e + 1) / 2 : e;
  }
  __host__ __device__ static int vbar_doubles(int K, int es) { return (K * es + 7) / 8; }
  // es: bytes per vbar entry (8, 4 or 2); c32: cbar in FP32
  static size_t bytes(const DevParams& P, int es, bool c32) {
    const size_t nrec = (size_t)(P.l + 1) * (P.l + 2) / 2, rec = nrec * NC + 2 * nrec;
    const size_t nv = (size_t)vbar_doubles(P.K, es);
    const size_t nabx = P.ns > 1 && !P.ps_mfma ? (size_t)P.nch * P.nch : 0;
    return sizeof(double) * (cb_doubles(P.ns, P.LL, c32) + (rec > nv ? rec : nv)) + sizeof(int) * nabx;
  }
};

// the pair's contraction with the cbar of one species over the records (l, m) of
// the degrees l set in deg (l outer, ascending, m inner): S_r, S_x, S_y, S_z of
// the gradient (partial sums when deg holds only some degrees)
template <int NMAX, int LMAX, typename CT, typename FieldFn>
__device__ __forceinline__ void adjoint_records(int L, unsigned deg, const CT* __restrict__ cb,
                                       const double* __restrict__ rc,
                                       const int* __restrict__ ri, FieldFn F, const double (&b)[NMAX],
                                       const double (&db)[NMAX], double uz, double ux, double uy, double& sr,
                                       double& sx, double& sy, double& sz) {
  using S = Shape<NMAX, LMAX>;
  constexpr int NC = S::NC;
  const double x2 = uz * uz;
  for (unsigned dm = deg; dm; dm &= dm - 1) {
    const int l = __builtin_ctz(dm);
    const double we = F(S::FW + l), wd = F(S::FR + S::XW + l);
    // Qbar_lm = x^par R(x^2): Horner over all NC table terms, unrolled (the
    // coefficients above degree (l - m) / 2 are zero, so the steps before the top
    // non-zero one leave Rv = Rd = 0: the same bits as starting there)
    auto qbar = [&](int r, double& Q, double& Qd) {
      const double* __restrict__ cf = rc + r * NC;
      const int par = ri[4 * r];
      double Rv = cf[NC - 1], Rd = 0.0;
#pragma unroll
      for (int t2 = NC - 2; t2 >= 0; --t2) {
        Rd = fma(Rd, x2, Rv);
        Rv = fma(Rv, x2, cf[t2]);
      }
      Q = par ? uz * Rv : Rv;
      Qd = par ? fma(2.0 * x2, Rd, Rv) : 2.0 * uz * Rd;
    };
    {
      // m = 0 (record r = l): only the cos column (the sin column is the sink, all
      // zeros), no azimuthal factor and no contribution to S_x, S_y
      double Q, Qd;
      qbar(l, Q, Qd);
      const CT* __restrict__ c0 = cb + ri[4 * l + 1] * NMAX;
      double U0 = 0.0, V0 = 0.0;
#pragma unroll
      for (int k = 0; k < NMAX; ++k) {
        U0 = fma((double)c0[k], db[k], U0);
        V0 = fma((double)c0[k], b[k], V0);
      }
      sr = fma(Q, fma(U0, we, V0 * wd), sr);
      sz = fma(Qd, V0 * we, sz);
    }
    // (u_x + i u_y)^m and ^(m-1) by the recurrence of the per-pair kernel (the same bits)
    double zr = 1.0, zi = 0.0, zr1 = 1.0, zi1 = 0.0;
#pragma unroll 2
    for (int m = 1; m <= l; ++m) {
      // the record of (l, m) in the tables: m outer, l = m..L inner
      const int r = m * (L + 1) - m * (m - 1) / 2 + (l - m);
      const int lc = ri[4 * r + 1], ls = ri[4 * r + 2];
      double Q, Qd;
      qbar(r, Q, Qd);
      zr1 = zr;
      zi1 = zi;
      azimuthal_step(zr, zi, ux, uy);
      const CT* __restrict__ c0 = cb + lc * NMAX;
      const CT* __restrict__ c1 = cb + ls * NMAX;
      double U0 = 0.0, V0 = 0.0, U1 = 0.0, V1 = 0.0;
#pragma unroll
      for (int k = 0; k < NMAX; ++k) {
        U0 = fma((double)c0[k], db[k], U0);
        V0 = fma((double)c0[k], b[k], V0);
        U1 = fma((double)c1[k], db[k], U1);
        V1 = fma((double)c1[k], b[k], V1);
      }
      const double fm = (double)m;
      sr = fma(Q, fma(fma(U0, we, V0 * wd), zr, fma(U1, we, V1 * wd) * zi), sr);
      const double W0 = V0 * we, W1 = V1 * we;
      const double qm = Q * fm;
      sx = fma(qm, fma(W0, zr1, W1 * zi1), sx);
      sy = fma(qm, fma(W1, zr1, -W0 * zi1), sy);
      sz = fma(Qd, fma(W0, zr, W1 * zi), sz);
    }
  }
}

// whole rounds of the adjoint take the compile-time record loop up to l_max = 10
// (66 records); l_max = 12 (91 records) would not fit the instruction cache
template <int NMAX, int LMAX>
constexpr bool kFullRecords = LMAX <= 10;

// adjoint_records for a whole round of one pair per lane with l_max equal to the
// compiled bucket: the same sums in the same order, with every loop bound and
// index fixed at compile time (record (l, m) at m (l_max + 1) - m (m - 1) / 2 +
// l - m, c columns l^2 + l + m and l^2 + l - m, parity (l - m) mod 2), so the
// Horner steps, the table and cbar reads and the parity selects need no runtime
// index arithmetic, loop control or branches
template <int NMAX, int LMAX, typename CT, typename FieldFn>
__device__ __forceinline__ void adjoint_records_full(const CT* __restrict__ cb, const double* __restrict__ rc,
                                                     FieldFn F, const double (&b)[NMAX], const double (&db)[NMAX],
                                                     double uz, double ux, double uy, double& sr, double& sx,
                                                     double& sy, double& sz) {
  using S = Shape<NMAX, LMAX>;
  constexpr int NC = S::NC;
  const double x2 = uz * uz;
#pragma unroll
  for (int l = 0; l <= LMAX; ++l) {
    const double we = F(S::FW + l), wd = F(S::FR + S::XW + l);
    double zr = 1.0, zi = 0.0, zr1 = 1.0, zi1 = 0.0;
#pragma unroll
    for (int m = 0; m <= l; ++m) {
      const int r = m * (LMAX + 1) - m * (m - 1) / 2 + (l - m), d = (l - m) >> 1;
      const bool par = (l - m) & 1;
      const double* __restrict__ cf = rc + r * NC;
      double Rv = cf[d], Rd = 0.0;
#pragma unroll
      for (int t2 = d - 1; t2 >= 0; --t2) {
        Rd = fma(Rd, x2, Rv);
        Rv = fma(Rv, x2, cf[t2]);
      }
      const double Q = par ? uz * Rv : Rv;
      const double Qd = par ? fma(2.0 * x2, Rd, Rv) : 2.0 * uz * Rd;
      const CT* __restrict__ c0 = cb + (l * l + l + m) * NMAX;
      if (m == 0) {
        double U0 = 0.0, V0 = 0.0;
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
          U0 = fma((double)c0[k], db[k], U0);
          V0 = fma((double)c0[k], b[k], V0);
        }
        sr = fma(Q, fma(U0, we, V0 * wd), sr);
        sz = fma(Qd, V0 * we, sz);
        continue;
      }
      zr1 = zr;
      zi1 = zi;
      azimuthal_step(zr, zi, ux, uy);
      const CT* __restrict__ c1 = cb + (l * l + l - m) * NMAX;
      double U0 = 0.0, V0 = 0.0, U1 = 0.0, V1 = 0.0;
#pragma unroll
      for (int k = 0; k < NMAX; ++k) {
        U0 = fma((double)c0[k], db[k], U0);
        V0 = fma((double)c0[k], b[k], V0);
        U1 = fma((double)c1[k], db[k], U1);
        V1 = fma((double)c1[k], b[k], V1);
      }
      const double fm = (double)m;
      sr = fma(Q, fma(fma(U0, we, V0 * wd), zr, fma(U1, we, V1 * wd) * zi), sr);
      const double W0 = V0 * we, W1 = V1 * we;
      const double qm = Q * fm;
      sx = fma(qm, fma(W0, zr1, W1 * zi1), sx);
      sy = fma(qm, fma(W1, zr1, -W0 * zi1), sy);
      sz = fma(Qd, fma(W0, zr, W1 * zi), sz);
    }
  }
}

// One wave per centre atom, in rounds of up to 64 pairs: a full round takes one
// pair per lane; a round with fewer pairs left (the tail of a long list, or a
// short list) gives each pair R = 2, 4 or 8 lanes, lane sub of a pair taking the
// records with l = sub, sub + R, ..., and the R partial sums are added by a fixed
// butterfly.  Each lane reads its pair's fields (coalesced across the pairs),
// contracts them with the cbar of the neighbour's species over its records and
// the pair gradient g = dE/dd follows from the sums.  The wave first forms the
// atom's cbar in LDS (form_cbar), then stages the record table; both are read
// as broadcasts.  Registers: up to 168 per lane (3 waves per SIMD) in the buckets
// up to n_max = 8, where the compile-time record loop spills at 128; the larger
// buckets need up to 256 (2 waves per SIMD).
template <int NMAX, int LMAX, typename ST, bool C32>
__global__ __launch_bounds__(64, NMAX <= 8 ? 3 : 2) void k_pair_adjoint(DevParams P, const DevTables* __restrict__ T,
                                                                       int n_atoms, const int* __restrict__ offsets,
                                                                       int bound, const int* __restrict__ nj,
                                                                       const int* __restrict__ species,
                                                                       const ST* __restrict__ rows,
                                                                       const ST* __restrict__ c,
                                                                       const double* __restrict__ q, int q_pitch,
                                                                       const double* __restrict__ pnorm,
                                                                       const ST* __restrict__ qbar,
                                                                       const ST* __restrict__ qbar2,
                                                                       int qbar_pitch, double* __restrict__ gx,
                                                                       double* __restrict__ gy,
                                                                       double* __restrict__ gz, int gstride, int vbar_f32) {
  using S = Shape<NMAX, LMAX>;
  constexpr int NC = S::NC;
  extern __shared__ __align__(16) double dyn[];
  const int i = xcd_item(blockIdx.x, n_atoms);
  if (i >= n_atoms) return;
  const int lane = threadIdx.x;
  const int LLP = P.LL + 1, L = P.l, nrec = (L + 1) * (L + 2) / 2;
  const int p0 = min(offsets[i], bound), p1 = min(offsets[i + 1], bound);  // pairs below the bound only
  if (p0 >= p1) return;
  // cbar in FP32 (C32: the mixed modes' matrix-core transform, several species,
  // whose FP32 results it holds exactly) or FP64
  using CT = std::conditional_t<C32, float, double>;
  const int cbs = AdjLds<NMAX, LMAX>::cb_stride(P.LL);
  CT* cb = reinterpret_cast<CT*>(dyn);
  double* rc = dyn + AdjLds<NMAX, LMAX>::cb_doubles(P.ns, P.LL, C32);
  int* ri = reinterpret_cast<int*>(rc + nrec * NC);
  {
    // the record table; its global reads are issued before form_cbar, its
    // stores follow it (vbar lives in the record region until then)
    constexpr int RPL = (S::NREC * NC + 63) / 64;
    double v[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int u = min(lane + 64 * k, nrec * NC - 1), r = u / NC, t = u - r * NC;
      v[k] = T->rec_coef[r % kRecLanes][r / kRecLanes][t];
    }
    constexpr int IPL = (S::NREC + 63) / 64;
    int lmp[IPL], lc[IPL], ls[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int r = min(lane + 64 * k, nrec - 1), jj = r % kRecLanes, slot = r / kRecLanes;
      lmp[k] = T->rec_lmp[jj][slot];
      lc[k] = T->rec_lm[jj][slot][0];
      ls[k] = T->rec_lm[jj][slot][1];
    }
    // bytes per vbar entry: BF16 operands with C32, FP32 with vbar_f32 (the mixed
    // modes only), FP64 otherwise
    const int es = C32 ? 2 : (sizeof(ST) == 4 && vbar_f32 ? 4 : 8);
    const int nrec_d = nrec * NC + 2 * nrec, nv_d = AdjLds<NMAX, LMAX>::vbar_doubles(P.K, es);
    int* abx = reinterpret_cast<int*>(rc + (nrec_d > nv_d ? nrec_d : nv_d));
    if constexpr (C32) {
      form_cbar<NMAX, LMAX, ST, __bf16, float>(P, i, c, q, q_pitch, pnorm, qbar, qbar2, qbar_pitch, cbs, cb,
                                               reinterpret_cast<__bf16*>(rc), abx, lane);
    } else if (es == 4) {
      form_cbar<NMAX, LMAX, ST, float, double>(P, i, c, q, q_pitch, pnorm, qbar, qbar2, qbar_pitch, cbs, cb,
                                               reinterpret_cast<float*>(rc), abx, lane);
    } else {
      form_cbar<NMAX, LMAX, ST, double, double>(P, i, c, q, q_pitch, pnorm, qbar, qbar2, qbar_pitch, cbs, cb, rc,
                                                abx, lane);
    }
#pragma unroll
    for (int k = 0; k < RPL; ++k)
      if (lane + 64 * k < nrec * NC) rc[lane + 64 * k] = v[k];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int r = lane + 64 * k;
      if (r < nrec) {
        ri[4 * r] = lmp[k] >> 16;
        ri[4 * r + 1] = lc[k];
        ri[4 * r + 2] = ls[k] < 0 ? P.LL : ls[k];
      }
    }
  }
  __syncthreads();
  for (int pb = p0; pb < p1;) {
    const int left = p1 - pb;
    const int lgR = left > 32 ? 0 : (left > 16 ? 1 : (left > 8 ? 2 : 3)), R = 1 << lgR;
    const int sub = lane & (R - 1), p = pb + (lane >> lgR);
    pb += 64 >> lgR;
    const bool live = p < p1;
    const int pq = live ? p : p0;  // idle lanes read a valid row
    const ST* __restrict__ row = rows + (size_t)(pq >> 6) * (S::ROW * 64) + (pq & 63);
    auto F = [&](int f) { return (double)row[f * 64]; };
    double b[NMAX], db[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      b[k] = F(S::FB + k);
      db[k] = F(S::FR + S::XD + k);
    }
    const double uz = F(S::FU), ux = F(S::FX), uy = F(S::FY);
    double sr = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    bool on = live;
    int sj = 0;
    if (P.ns > 1) {
      // a neighbour label outside 0..n_species-1 contributes nothing
      sj = species[nj[pq]];
      on = on && sj >= 0 && sj < P.ns;
      sj = on ? sj : 0;
    }
    const CT* __restrict__ cbj = cb + (size_t)sj * cbs;
    if (kFullRecords<NMAX, LMAX> && R == 1 && L == LMAX)
      adjoint_records_full<NMAX, LMAX>(cbj, rc, F, b, db, uz, ux, uy, sr, sx, sy, sz);
    else
      adjoint_records<NMAX, LMAX>(L, R == 1 ? (2u << L) - 1u : (unsigned)P.tail_deg[lgR - 1][sub], cbj, rc, ri, F,
                                  b, db, uz, ux, uy, sr, sx, sy, sz);
    for (int o = 1; o < R; o <<= 1) {
      sr += __shfl_xor(sr, o, 64);
      sx += __shfl_xor(sx, o, 64);
      sy += __shfl_xor(sy, o, 64);
      sz += __shfl_xor(sz, o, 64);
    }
    if (live && sub == 0) {
      const double ir = F(S::FR + S::XI);
      // d u / d d = (I - u u^T) / r
      const double ut = ux * sx + uy * sy + uz * sz;
      const double g0 = on ? sr * ux + (sx - ux * ut) * ir : 0.0;
      const double g1 = on ? sr * uy + (sy - uy * ut) * ir : 0.0;
      const double g2 = on ? sr * uz + (sz - uz * ut) * ir : 0.0;
      if (gstride == 4) {  // one 32-byte record (x, y, z, 0) per pair
        *reinterpret_cast<dvec4*>(gx + 4 * (size_t)p) = dvec4{g0, g1, g2, 0.0};
      } else {
        gx[p] = g0;
        gy[p] = g1;
        gz[p] = g2;
      }
    }
  }
}

// F_k = sum over k's pairs q of (g_q - g_rev(q)) (= -dE/dr_k); mode 1 adds -F_k into
// pos_grad.  The pair gradients are (x, y, z, 0) records, so a pair and its reverse
// pair cost one 32-byte read each.  One wavefront per atom, one pair per lane (an
// atom's list is usually shorter than 64, so its reverse indices and both
// gradients are read in one round); the lane sums are combined by a fixed
// butterfly, so the result is the same on every run.
__global__ __launch_bounds__(256) void k_force_gather(int n_atoms, const int* __restrict__ offsets, int bound,
                                                      const int* __restrict__ rev, const dvec4* __restrict__ g,
                                                      double* __restrict__ out, int accumulate_grad) {
  const int k = xcd_item(blockIdx.x, (n_atoms + 3) / 4) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n_atoms) return;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const int q1 = min(offsets[k + 1], bound);
  for (int q = min(offsets[k], bound) + lane; q < q1; q += 64) {
    const dvec4 a = g[q], b = g[rev[q]];
    fx += a.x - b.x;
    fy += a.y - b.y;
    fz += a.z - b.z;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    fx += __shfl_xor(fx, o, 64);
    fy += __shfl_xor(fy, o, 64);
    fz += __shfl_xor(fz, o, 64);
  }
  if (lane == 0) {
    if (accumulate_grad) {
      out[3 * k] -= fx;
      out[3 * k + 1] -= fy;
      out[3 * k + 2] -= fz;
    } else {
      out[3 * k] = fx;
      out[3 * k + 1] = fy;
      out[3 * k + 2] = fz;
    }
  }
}

__global__ void k_fill(double* __restrict__ p, long long n, double v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// compile-time (n_max, l_max) buckets: the kernels handle any n <= NMAX, l <= LMAX
struct Bucket {
  int n, l;
};
Bucket bucket_of(int n, int l) {
  if (n <= 6 && l <= 6) return {6, 6};
  if (n <= 8 && l <= 6) return {8, 6};
  if (n <= 8 && l <= 8) return {8, 8};
  if (n <= 10 && l <= 10) return {10, 10};
  return {12, 12};
}

template <typename F>
hipError_t dispatch(int n, int l, F&& f) {
  const Bucket b = bucket_of(n, l);
  if (b.n == 6) return f.template operator()<6, 6>();
  if (b.n == 8 && b.l == 6) return f.template operator()<8, 6>();
  if (b.n == 8) return f.template operator()<8, 8>();
  if (b.n == 10) return f.template operator()<10, 10>();
  return f.template operator()<12, 12>();
}

template <typename F>
size_t dispatch_size(int n, int l, F&& f) {
  const Bucket b = bucket_of(n, l);
  if (b.n == 6) return f.template operator()<6, 6>();
  if (b.n == 8 && b.l == 6) return f.template operator()<8, 6>();
  if (b.n == 8) return f.template operator()<8, 8>();
  if (b.n == 10) return f.template operator()<10, 10>();
  return f.template operator()<12, 12>();
}

// store_f32: c stored (and, with fwd_c32, staged) in FP32
size_t fwd_dyn_bytes(const DevParams& P, bool store_f32) {
  return dispatch_size(P.n, P.l, [&]<int N, int LM>() -> size_t {
    using S = Shape<N, LM>;
    const size_t nc = (size_t)P.ns * N * (P.LL + 1);
    const size_t rows = (size_t)S::CH * S::FRP,
                 epi = store_f32 && fwd_c32<N, LM>(P) ? (nc + 1) / 2
                                                      : nc + (fwd_p_in_lds<N, LM>(P) ? (size_t)P.K : 0);
    return sizeof(double) * (rows > epi ? rows : epi);
  });
}
size_t adj_dyn_bytes(const DevParams& P, int es, bool c32) {
  return dispatch_size(P.n, P.l, [&]<int N, int LM>() -> size_t { return AdjLds<N, LM>::bytes(P, es, c32); });
}

}  // namespace

size_t c_doubles_per_atom(const DevParams& P) {
  return dispatch_size(P.n, P.l, [&]<int N, int LM>() -> size_t { return (size_t)P.ns * N * (P.LL + 1); });
}
size_t pair_row_doubles(const DevParams& P) {
  return dispatch_size(P.n, P.l, [&]<int N, int LM>() -> size_t { return (size_t)Shape<N, LM>::ROW; });
}
size_t pair_rows_bytes(const DevParams& P, long long n_pairs, bool f32) {
  const size_t blocks = (size_t)((n_pairs + 63) / 64);
  return (f32 ? sizeof(float) : sizeof(double)) * (blocks > 0 ? blocks : 1) * 64 * pair_row_doubles(P);
}

size_t descriptor_lds_bytes(const DevParams& P) {
  return fwd_dyn_bytes(P, false) + 64 * sizeof(int);  // the larger (FP64) layout
}
size_t adjoint_lds_bytes(const DevParams& P) { return adj_dyn_bytes(P, 8, false); }  // the largest (FP64) layout

hipError_t launch_pair_prep(const DevParams& P, const DevTables* T, long long n_pairs, const int* count,
                            const double* dx, const double* dy, const double* dz, void* rows_v, bool rows_f32,
                            bool deriv, double* bc, int block, int part, hipStream_t st) {
  if (block != 64 && block != 128) block = 256;
  if (part != 1 && part != 2) return hipErrorInvalidValue;
  if (rows_f32 && P.radial_dd) return hipErrorInvalidValue;  // FP32 rows only with the FP64 radial stage
  // one workgroup per block of pairs; block 0 of the radial launch also writes bc
  const int blocks = (int)((n_pairs + block - 1) / block) + (n_pairs == 0 ? 1 : 0);
  auto f = [&]<int N, int LM>() {
    const int np = (int)n_pairs;
    const dim3 g(blocks), b(block);
    if (rows_f32) {
      float* rf = static_cast<float*>(rows_v);
      if (part == 2 && deriv)
        hipLaunchKernelGGL((k_pair_prep<N, LM, true, false, 2, float>), g, b, 0, st, P, T, np, count, dx, dy, dz, rf, bc);
      else if (part == 2)
        hipLaunchKernelGGL((k_pair_prep<N, LM, false, false, 2, float>), g, b, 0, st, P, T, np, count, dx, dy, dz, rf, bc);
      else if (deriv)
        hipLaunchKernelGGL((k_pair_prep<N, LM, true, false, 1, float>), g, b, 0, st, P, T, np, count, dx, dy, dz, rf, bc);
      else
        hipLaunchKernelGGL((k_pair_prep<N, LM, false, false, 1, float>), g, b, 0, st, P, T, np, count, dx, dy, dz, rf, bc);
      return hipGetLastError();
    }
    double* rows = static_cast<double*>(rows_v);
    if (part == 2) {
      if (deriv)
        hipLaunchKernelGGL((k_pair_prep<N, LM, true, false, 2, double>), g, b, 0, st, P, T, np, count, dx, dy, dz, rows, bc);
      else
        hipLaunchKernelGGL((k_pair_prep<N, LM, false, false, 2, double>), g, b, 0, st, P, T, np, count, dx, dy, dz, rows, bc);
    } else if (deriv && P.radial_dd) {
      hipLaunchKernelGGL((k_pair_prep<N, LM, true, true, 1, double>), g, b, 0, st, P, T, np, count, dx, dy, dz, rows, bc);
    } else if (deriv) {
      hipLaunchKernelGGL((k_pair_prep<N, LM, true, false, 1, double>), g, b, 0, st, P, T, np, count, dx, dy, dz, rows, bc);
    } else if (P.radial_dd) {
      hipLaunchKernelGGL((k_pair_prep<N, LM, false, true, 1, double>), g, b, 0, st, P, T, np, count, dx, dy, dz, rows, bc);
    } else {
      hipLaunchKernelGGL((k_pair_prep<N, LM, false, false, 1, double>), g, b, 0, st, P, T, np, count, dx, dy, dz, rows, bc);
    }
    return hipGetLastError();
  };
  return dispatch(P.n, P.l, f);
}

hipError_t launch_descriptor(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, int bound,
                             const int* nj,
                             const int* species, const void* rows, bool store_f32, const double* bc, void* c,
                             double* q, int q_pitch, double* pnorm, void* qc, int qc_pitch, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  if (qc && qc_pitch < P.K) return hipErrorInvalidValue;
  const size_t dyn = fwd_dyn_bytes(P, store_f32);
  auto f = [&]<int N, int LM>() {
    if (store_f32)
      hipLaunchKernelGGL((k_descriptor<N, LM, float>), dim3(8 * xcd_per(n_atoms)), dim3(64), dyn, st, P, T, n_atoms,
                         offsets, bound, nj, species, static_cast<const float*>(rows), bc, static_cast<float*>(c), q,
                         q_pitch, pnorm, static_cast<__bf16*>(qc), qc_pitch);
    else
      hipLaunchKernelGGL((k_descriptor<N, LM, double>), dim3(8 * xcd_per(n_atoms)), dim3(64), dyn, st, P, T, n_atoms,
                         offsets, bound, nj, species, static_cast<const double*>(rows), bc, static_cast<double*>(c),
                         q, q_pitch, pnorm, static_cast<__bf16*>(qc), qc_pitch);
    return hipGetLastError();
  };
  return dispatch(P.n, P.l, f);
}

hipError_t launch_pair_adjoint(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, int bound,
                               const int* nj, const int* species, const void* rows, bool store_f32, const void* c,
                               const double* q, int q_pitch, const double* pnorm, const void* qbar,
                               const void* qbar2, int qbar_pitch, double* gx, double* gy, double* gz,
                               int gstride, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  if (gstride != 1 && gstride != 4) return hipErrorInvalidValue;
  // vbar in FP32 when the FP64 layout leaves a CU (160 KB of LDS) one wavefront
  // per SIMD and the FP32 one fits more (three species at K = 2700: 39.6 -> 28.8
  // KB, 4 -> 5 wavefronts per CU, adjoint 1.72 -> 1.49 ms); elsewhere the
  // conversions cost more than the extra wavefronts gain.  The matrix-core
  // transform of several species (C32) keeps cbar in FP32 and its BF16 operands
  // instead of vbar, with no channel-pair table (three species at K = 2700:
  // 28.8 -> 13.3 KB)
  const size_t b64 = adj_dyn_bytes(P, 8, false), b32 = adj_dyn_bytes(P, 4, false), lds_cu = 160 * 1024;
  const bool c32 = store_f32 && P.ps_mfma && P.ns > 1;
  const bool vbar_f32 = !c32 && store_f32 && lds_cu / b64 <= 4 && lds_cu / b32 > lds_cu / b64;
  const size_t dyn = c32 ? adj_dyn_bytes(P, 2, true) : (vbar_f32 ? b32 : b64);
  auto f = [&]<int N, int LM>() {
    if (c32)
      hipLaunchKernelGGL((k_pair_adjoint<N, LM, float, true>), dim3(8 * xcd_per(n_atoms)), dim3(64), dyn, st, P, T,
                         n_atoms, offsets, bound, nj, species, static_cast<const float*>(rows),
                         static_cast<const float*>(c), q, q_pitch, pnorm, static_cast<const float*>(qbar),
                         static_cast<const float*>(qbar2), qbar_pitch, gx, gy, gz, gstride, 0);
    else if (store_f32)
      hipLaunchKernelGGL((k_pair_adjoint<N, LM, float, false>), dim3(8 * xcd_per(n_atoms)), dim3(64), dyn, st, P, T,
                         n_atoms, offsets, bound, nj, species, static_cast<const float*>(rows),
                         static_cast<const float*>(c), q, q_pitch, pnorm, static_cast<const float*>(qbar),
                         static_cast<const float*>(qbar2), qbar_pitch, gx, gy, gz, gstride, vbar_f32 ? 1 : 0);
    else
      hipLaunchKernelGGL((k_pair_adjoint<N, LM, double, false>), dim3(8 * xcd_per(n_atoms)), dim3(64), dyn, st, P, T,
                         n_atoms, offsets, bound, nj, species, static_cast<const double*>(rows),
                         static_cast<const double*>(c), q, q_pitch, pnorm, static_cast<const double*>(qbar),
                         static_cast<const double*>(qbar2), qbar_pitch, gx, gy, gz, gstride, 0);
    return hipGetLastError();
  };
  return dispatch(P.n, P.l, f);
}

// qbar (n_rows x K) set to the unit vector e_kset on every row; column kclear
// (a previous kset) is cleared, or, with kclear < 0, the whole matrix
__global__ void k_unit_rows(int n_rows, int K, int kset, int kclear, double* __restrict__ qbar) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (kclear < 0) {
    if (t < (long long)n_rows * K) qbar[t] = (int)(t % K) == kset ? 1.0 : 0.0;
  } else if (t < n_rows) {
    qbar[t * K + kclear] = 0.0;
    qbar[t * K + kset] = 1.0;
  }
}

hipError_t launch_unit_rows(int n_rows, int K, int kset, int kclear, double* qbar, hipStream_t st) {
  const long long n = kclear < 0 ? (long long)n_rows * K : n_rows;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n_rows, K, kset, kclear, qbar);
  return hipGetLastError();
}

hipError_t launch_force_gather(int n_atoms, const int* offsets, int bound, const int* rev, const double* g,
                               double* out, bool accumulate_grad, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_force_gather, dim3(8 * xcd_per((n_atoms + 3) / 4)), dim3(256), 0, st, n_atoms, offsets, bound, rev,
                     reinterpret_cast<const dvec4*>(g), out, accumulate_grad ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

void build_angular_tables(const DevParams& P, DevTables& T) {
  // ilexp series factors for the two top orders
  for (int o = 0; o < 3; ++o) {
    const int l = P.l - 1 + o;
    for (int k = 0; k < kIlexpTerms; ++k) T.ilx_rec[o][k] = 1.0 / ((double)(k + 1) * (double)(2 * l + 2 * k + 3));
  }
  double df = 1.0;  // (2l+1)!!
  for (int l = 0; l < kMaxL + 3; ++l) {
    if (l > 0) df *= (double)(2 * l + 1);
    T.ilx_idf[l] = 1.0 / df;
  }
  // Qbar_lm polynomials in extended precision from the three-term recursion
  //   Qbar_mm = sqrt(2)^(m>0) (4 pi)^(-1/2) prod_{k<=m} sqrt((2k+1)/(2k)),
  //   Qbar_lm = a_lm x Qbar_{l-1,m} - b_lm Qbar_{l-2,m},
  //   a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)(2l+1)/((2l-3)(l^2-m^2)))
  for (int jj = 0; jj < kRecLanes; ++jj)
    for (int e = 0; e < kMaxRec; ++e) {
      for (int t = 0; t < kPolyTerms; ++t) T.rec_coef[jj][e][t] = 0.0;
      T.rec_lmp[jj][e] = 0;
      T.rec_lm[jj][e][0] = T.rec_lm[jj][e][1] = -1;
    }
  int rec = 0;
  long double qmm = 0.28209479177387814347403972578038629L;  // (4 pi)^(-1/2)
  for (int m = 0; m <= P.l; ++m) {
    if (m > 0) qmm *= std::sqrt((2.0L * m + 1.0L) / (2.0L * m));
    const long double seed = m > 0 ? qmm * 1.41421356237309504880168872420969808L : qmm;
    long double q2[kMaxL + 2] = {}, q1[kMaxL + 2] = {}, qc[kMaxL + 2] = {};  // coefficients of x^d
    for (int l = m; l <= P.l; ++l) {
      for (int d = 0; d <= kMaxL + 1; ++d) qc[d] = 0.0L;
      if (l == m) {
        qc[0] = seed;
      } else {
        const long double l2m2 = (long double)(l * l - m * m);
        const long double a = std::sqrt((4.0L * l * l - 1.0L) / l2m2);
        const long double num = (long double)((l - 1) * (l - 1) - m * m) * (2.0L * l + 1.0L);
        const long double b = num == 0.0L ? 0.0L : std::sqrt(num / ((2.0L * l - 3.0L) * l2m2));
        for (int d = 0; d <= kMaxL; ++d) qc[d + 1] += a * q1[d];
        for (int d = 0; d <= kMaxL + 1; ++d) qc[d] -= b * q2[d];
      }
      const int par = (l - m) & 1, jj = rec % kRecLanes, e = rec / kRecLanes;
      for (int t = 0; 2 * t + par <= l - m; ++t) T.rec_coef[jj][e][t] = (double)qc[2 * t + par];
      T.rec_lmp[jj][e] = l | (m << 8) | (par << 16);
      T.rec_lm[jj][e][0] = (short)(l * l + l + m);
      T.rec_lm[jj][e][1] = (short)(m > 0 ? l * l + l - m : -1);
      ++rec;
      for (int d = 0; d <= kMaxL + 1; ++d) {
        q2[d] = q1[d];
        q1[d] = qc[d];
      }
    }
  }
}

}  // namespace soap
