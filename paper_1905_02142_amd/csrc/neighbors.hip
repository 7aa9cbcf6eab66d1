// Neighbour list inside the cutoff sphere (Sec. I): every (i, j, T) with
// 0 < |r_j + T - r_i| < r_cut, T a lattice translation of i's structure.
//
// Cell list per structure in fractional coordinates.  Along a periodic axis the
// cell is cut into nbin = max(1, floor(w / r_cut)) slabs (w = width perpendicular
// to the two other lattice vectors); a centre scans R = ceil(r_cut nbin / w) slabs
// either side.  When 2R + 1 > nbin the same slab is visited with different
// lattice shifts, which enumerates every periodic image exactly once, so boxes
// narrower than 2 r_cut work unchanged.  Non-periodic axes use one slab.
//
// Order: each centre's pairs follow the fixed slab-offset loop and, within a
// bin, ascending atom index, so the list is identical on every run.  That order
// also places every reverse pair without a search: if centre i meets j at slab
// offset o with bin shift g, centre j meets i at offset -o with shift -g, after
// its hits of the offsets before -o (recorded per centre and offset by the count
// pass) and after the atoms of i's bin with a smaller index that j also reaches.
#include <hip/hip_runtime.h>

#include <hip/hip_runtime.h>

#include <cstdint>

#include "neighbors.h"

namespace soap {

namespace {

__device__ inline int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

__device__ inline int find_structure(const int* __restrict__ so, int ns, int a) {
  int lo = 0, hi = ns;  // so[lo] <= a < so[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (so[mid] <= a) lo = mid;
    else hi = mid;
  }
  return lo;
}

// bin (global bin index) of a position in structure M and the lattice wrap that
// brings it into its cell
__device__ inline void locate_pos(const StructMeta& M, double p0, double p1, double p2, int* __restrict__ err,
                                  int& bin_out, int& wrap_out) {
  double p[3] = {p0, p1, p2};
  if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) {
    atomicOr(err, kErrNonFinite);
    p[0] = p[1] = p[2] = 0.0;
  }
  int b[3], w[3];
  for (int x = 0; x < 3; ++x) {
    double f = p[0] * M.inv[0 * 3 + x] + p[1] * M.inv[1 * 3 + x] + p[2] * M.inv[2 * 3 + x];
    if (M.pbc[x]) {
      double fw = floor(f);
      f -= fw;
      int wi = (int)fw;
      if (f >= 1.0) {
        f -= 1.0;
        wi += 1;
      }
      if (wi < -kWrapMax || wi > kWrapMax) {
        atomicOr(err, kErrFarOutside);
        wi = 0;
      }
      w[x] = wi;
      int bx = (int)(f * M.nbin[x]);
      b[x] = bx < M.nbin[x] ? (bx < 0 ? 0 : bx) : M.nbin[x] - 1;
    } else {
      w[x] = 0;
      b[x] = 0;
    }
  }
  bin_out = M.bin0 + (b[2] * M.nbin[1] + b[1]) * M.nbin[0] + b[0];
  wrap_out = pack_img(w[0], w[1], w[2]);
}

// the same for atom a of the batch
__device__ inline void locate_atom(int a, const double* __restrict__ pos, const StructMeta* __restrict__ meta,
                                   const int* __restrict__ so, int n_struct, int* __restrict__ err, int& bin_out,
                                   int& wrap_out) {
  locate_pos(meta[find_structure(so, n_struct, a)], pos[3 * a], pos[3 * a + 1], pos[3 * a + 2], err, bin_out,
             wrap_out);
}

__global__ void k_bin_atoms(int n_atoms, const double* __restrict__ pos, const StructMeta* __restrict__ meta,
                            const int* __restrict__ so, int n_struct, int* __restrict__ atom_bin,
                            int* __restrict__ atom_wrap, int* __restrict__ bin_count, int* __restrict__ err) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_atoms) return;
  int bin, wrap;
  locate_atom(a, pos, meta, so, n_struct, err, bin, wrap);
  atom_bin[a] = bin;
  atom_wrap[a] = wrap;
  atomicAdd(&bin_count[bin], 1);
}

// the bins of up to PER atoms per thread (t + k * kSmallBinThreads) of one
// structure's geometry M, counted into the LDS bin counters; mybin[k] stays -1
// for k beyond the atoms; the positions of the first four (k < 4) are kept in
// kx, ky, kz
template <int PER>
__device__ inline void bin_block(int n_atoms, const double* __restrict__ pos, const StructMeta& M, int t,
                                 int* __restrict__ atom_bin, int* __restrict__ atom_wrap, int* __restrict__ cnt,
                                 int* __restrict__ err, int (&mybin)[PER], int (&mywrap)[PER], double (&kx)[4],
                                 double (&ky)[4], double (&kz)[4]) {
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += 4) {
    if (k0 * kSmallBinThreads >= n_atoms) break;  // the same for every thread
    // four positions requested before any is used; out-of-range atoms read the last one
    double px[4], py[4], pz[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = min(t + (k0 + k) * kSmallBinThreads, n_atoms - 1);
      px[k] = pos[3 * a];
      py[k] = pos[3 * a + 1];
      pz[k] = pos[3 * a + 2];
    }
    if (k0 == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        kx[k] = px[k];
        ky[k] = py[k];
        kz[k] = pz[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = t + (k0 + k) * kSmallBinThreads;
      if (a < n_atoms) {
        locate_pos(M, px[k], py[k], pz[k], err, mybin[k0 + k], mywrap[k0 + k]);
        atom_bin[a] = mybin[k0 + k];
        atom_wrap[a] = mywrap[k0 + k];
        atomicAdd(&cnt[mybin[k0 + k]], 1);
      }
    }
  }
}

// The whole cell list of a small system in one workgroup: error word cleared,
// atoms binned, bin counts scanned into bin_start, atoms placed by LDS cursors
// and then ranked by index inside each bin; the same result as k_init_build ..
// k_rank_bins in five launches.  Each thread keeps its atoms' bins in
// registers; counts, starts and the unsorted bin contents live in LDS
// (4 (n_atoms + 2 n_bins) bytes of dynamic LDS).
__global__ __launch_bounds__(kSmallBinThreads) void k_bin_small(int n_atoms, const double* __restrict__ pos,
                                                                const StructMeta* __restrict__ meta,
                                                                const int* __restrict__ so, int n_struct, int n_bins,
                                                                int* __restrict__ atom_bin, int* __restrict__ atom_wrap,
                                                                int* __restrict__ bin_start, Cand* __restrict__ cand,
                                                                int* __restrict__ err) {
  constexpr int PER = kSmallAtoms / kSmallBinThreads;  // atoms per thread at most
  extern __shared__ int lds[];
  int* cnt = lds;               // n_bins: counts, then cursors
  int* start = lds + n_bins;    // n_bins
  int* unsorted = lds + 2 * n_bins;  // n_atoms
  const int t = threadIdx.x;
  for (int b = t; b < n_bins; b += kSmallBinThreads) cnt[b] = 0;
  if (t < 4) err[t] = 0;
  __syncthreads();
  int mybin[PER], mywrap[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) mybin[k] = mywrap[k] = -1;
  double kx[4], ky[4], kz[4];  // the positions of the thread's first four atoms, one structure only
  const bool kept = n_struct == 1;
  if (kept) {
    // one structure: its geometry sits in scalar registers for every atom
    const StructMeta M = meta[0];
    bin_block<PER>(n_atoms, pos, M, t, atom_bin, atom_wrap, cnt, err, mybin, mywrap, kx, ky, kz);
  } else {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int a = t + k * kSmallBinThreads;
      if (a < n_atoms) {
        locate_atom(a, pos, meta, so, n_struct, err, mybin[k], mywrap[k]);
        atom_bin[a] = mybin[k];
        atom_wrap[a] = mywrap[k];
        atomicAdd(&cnt[mybin[k]], 1);
      }
    }
  }
  __syncthreads();
  // exclusive scan of the bin counts: thread t owns bins t*per .. t*per+per-1;
  // a scan inside each wavefront, then over the wavefront totals
  __shared__ int wsum[kSmallBinThreads / 64];
  const int per = (n_bins + kSmallBinThreads - 1) / kSmallBinThreads;
  int sum = 0;
  for (int k = 0; k < per; ++k) {
    const int b = t * per + k;
    if (b < n_bins) sum += cnt[b];
  }
  const int lane = t & 63, w = t >> 6;
  int incl = sum;
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(incl, d, 64);
    if (lane >= d) incl += v;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int run = incl - sum, total = 0;
  for (int k = 0; k < kSmallBinThreads / 64; ++k) {
    const int v = wsum[k];
    run += k < w ? v : 0;
    total += v;
  }
  for (int k = 0; k < per; ++k) {
    const int b = t * per + k;
    if (b < n_bins) {
      const int c = cnt[b];
      bin_start[b] = run;
      start[b] = run;
      cnt[b] = run;  // from here on the placement cursor
      run += c;
    }
  }
  if (t == 0) bin_start[n_bins] = total;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (mybin[k] >= 0) unsorted[atomicAdd(&cnt[mybin[k]], 1)] = t + k * kSmallBinThreads;
  __syncthreads();
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += 4) {
    if (k0 * kSmallBinThreads >= n_atoms) break;
    double px[4], py[4], pz[4];
    if (k0 == 0 && kept) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        px[k] = kx[k];
        py[k] = ky[k];
        pz[k] = kz[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int a = min(t + (k0 + k) * kSmallBinThreads, n_atoms - 1);
        px[k] = pos[3 * a];
        py[k] = pos[3 * a + 1];
        pz[k] = pos[3 * a + 2];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (mybin[k0 + k] >= 0) {
        const int a = t + (k0 + k) * kSmallBinThreads;
        const int s0 = start[mybin[k0 + k]], e0 = cnt[mybin[k0 + k]];  // the cursor ends at the bin's end
        int rank = 0;
        for (int q = s0; q < e0; ++q) rank += unsorted[q] < a;
        Cand c;
        c.x = px[k];
        c.y = py[k];
        c.z = pz[k];
        c.j = a;
        c.wrap = mywrap[k0 + k];
        cand[s0 + rank] = c;
      }
    }
  }
}

__global__ void k_fill_bins(int n_atoms, const int* __restrict__ atom_bin, const int* __restrict__ bin_start,
                            int* __restrict__ bin_cursor, int* __restrict__ unsorted) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_atoms) return;
  int bin = atom_bin[a];
  int slot = atomicAdd(&bin_cursor[bin], 1);
  unsorted[bin_start[bin] + slot] = a;
}

// place atom a at its rank (by index) among the atoms of its bin; `unsorted`
// holds each bin's atoms in the arbitrary order the atomics produced
__global__ void k_rank_bins(int n_atoms, const double* __restrict__ pos, const int* __restrict__ atom_bin,
                            const int* __restrict__ atom_wrap, const int* __restrict__ bin_start,
                            const int* __restrict__ unsorted, Cand* __restrict__ cand) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_atoms) return;
  const int bin = atom_bin[a];
  const int s = bin_start[bin], e = bin_start[bin + 1];
  int rank = 0;
  for (int t = s; t < e; ++t) rank += unsorted[t] < a;
  Cand c;
  c.x = pos[3 * a];
  c.y = pos[3 * a + 1];
  c.z = pos[3 * a + 2];
  c.j = a;
  c.wrap = atom_wrap[a];
  cand[s + rank] = c;
}

// bits lo..hi-1 of a 64-bit mask (0 <= lo <= hi <= 64)
__device__ inline unsigned long long bit_range(int lo, int hi) {
  const unsigned long long below_hi = hi >= 64 ? ~0ull : (1ull << hi) - 1ull;
  const unsigned long long below_lo = lo >= 64 ? ~0ull : (1ull << lo) - 1ull;
  return below_hi & ~below_lo;
}

// One wavefront per centre atom.  The (2R+1)^3 slab offsets are taken 64 at a
// time: lane b describes offset b (bin, lattice shift, atom count), a wave scan
// turns the counts into a flat candidate range, and the lanes then sweep the
// candidates 64 at a time.  Hits are compacted with a ballot, so the pair order
// (offset order, then ascending atom index within a bin) is fixed.
//
// Count pass: count[i], and opre[m(i)][o] = the hits of i before offset o, where
// m(i) is i's slot in the cell list (bin order, so that the centres near each
// other, which the fill pass looks up together, have neighbouring rows).
// Fill pass: the pairs, and rev of each.  For the pair (i -> j, T) found at
// offset o with bin shift g, centre j meets i's bin at offset n_off - 1 - o
// with shift -g; among that bin's atoms (ascending index) the ones before i that
// j reaches precede (j -> i, -T) in j's list, so
//   rev = offsets[j] + opre[m(j)][n_off - 1 - o] + #{a in bin(i), a < i, j reaches a},
// where "j reaches a" is evaluated with exactly the arithmetic of j's own scan.
template <bool FILL>
__global__ __launch_bounds__(256) void k_pairs(int n_atoms, const double* __restrict__ pos,
                                               const StructMeta* __restrict__ meta, const int* __restrict__ so,
                                               int n_struct, double rc2, const int* __restrict__ atom_bin,
                                               const int* __restrict__ atom_wrap, const int* __restrict__ bin_start,
                                               const Cand* __restrict__ cand, int* __restrict__ count,
                                               int* __restrict__ opre, const int* __restrict__ offsets,
                                               long long capacity, int* __restrict__ nj, int* __restrict__ nimg,
                                               int* __restrict__ ncenter, double* __restrict__ ndx,
                                               double* __restrict__ ndy, double* __restrict__ ndz,
                                               int* __restrict__ nrev, int* __restrict__ err) {
  __shared__ int s_pref[4][65];   // inclusive scan of candidate counts
  __shared__ int s_start[4][64];  // first cand slot of each offset
  __shared__ int s_shift[4][64];  // lattice shift of each offset (packed)
  __shared__ int s_own[4][64];    // the offset whose first candidate is slot c - c0 of a chunk
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // centres are taken in cell-list order: wavefront mc takes the atom in slot mc,
  // so neighbouring wavefronts scan neighbouring bins (their candidate records and
  // hit prefixes meet in the caches).  The centre is uniform over the wavefront:
  // its data and its structure's geometry are read once into scalar registers
  const int mc = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
  if (mc >= n_atoms) return;
  const int i = __builtin_amdgcn_readfirstlane(cand[mc].j);
  const StructMeta& M = meta[n_struct == 1 ? 0 : find_structure(so, n_struct, i)];
  double cell[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) cell[k] = M.cell[k];
  const int nb0 = M.nbin[0], nb1 = M.nbin[1], nb2 = M.nbin[2];
  const int R0 = M.R[0], R1 = M.R[1], R2 = M.R[2];
  const int p0 = M.pbc[0], p1 = M.pbc[1], p2 = M.pbc[2];
  const int bin0 = M.bin0;
  const double pix = pos[3 * i], piy = pos[3 * i + 1], piz = pos[3 * i + 2];
  const int bi = atom_bin[i];
  const int local = bi - bin0;
  const int b0 = local % nb0, b1 = (local / nb0) % nb1, b2 = local / (nb0 * nb1);
  int wi[3];
  unpack_img(atom_wrap[i], wi);
  const int n0 = 2 * R0 + 1, n1 = 2 * R1 + 1, n2 = 2 * R2 + 1;
  const int n_off = n0 * n1 * n2;
  // the hit prefixes of the centre in slot m of this structure (whose slots
  // start at bin_start[bin0]): opre + obase + (m - bin_start[bin0]) n_off
  int* const opre_s = opre + (M.obase - (long long)bin_start[bin0] * n_off);
  long long out = FILL ? offsets[i] : 0;
  // fill: the slots of i's bin holding atoms with a smaller index than i (a bin
  // holds its atoms in index order, i at slot mc)
  const int m0 = FILL ? bin_start[bi] : 0;
  const int m1 = FILL ? mc : 0;
  int cnt = 0;
  // offset o = x + n0 (y + n1 z): below 2^21 offsets the quotients come exactly
  // from float reciprocals ((o + 0.5) / d lies at least 0.5 / d from an integer,
  // far beyond the float rounding of o / d); beyond, integer division
  const bool fdiv = n_off < (1 << 21);
  const float i0f = 1.0f / (float)n0, i01f = 1.0f / (float)(n0 * n1);
  // a bin shift of at most one cell count (R <= nbin) wraps at most once
  const bool w0 = R0 <= nb0, w1 = R1 <= nb1, w2 = R2 <= nb2;
  auto wrap = [](int u, int nb, bool once) { return once ? (u < 0 ? -1 : (u >= nb ? 1 : 0)) : floordiv(u, nb); };
  for (int g0 = 0; g0 < n_off; g0 += 64) {
    const int o = g0 + lane;
    int len = 0, start = 0, shift = 0;
    if (o < n_off) {
      int qx, qy, qz;
      if (fdiv) {
        qz = (int)(((float)o + 0.5f) * i01f);
        const int r = o - qz * n0 * n1;
        qy = (int)(((float)r + 0.5f) * i0f);
        qx = r - qy * n0;
      } else {
        qx = o % n0;
        qy = (o / n0) % n1;
        qz = o / (n0 * n1);
      }
      const int ox = qx - R0, oy = qy - R1, oz = qz - R2;
      const int ux = b0 + ox, uy = b1 + oy, uz = b2 + oz;
      const int gx = p0 ? wrap(ux, nb0, w0) : 0;
      const int gy = p1 ? wrap(uy, nb1, w1) : 0;
      const int gz = p2 ? wrap(uz, nb2, w2) : 0;
      const int cx = ux - gx * nb0, cy = uy - gy * nb1, cz = uz - gz * nb2;
      const int bin = bin0 + (cz * nb1 + cy) * nb0 + cx;
      start = bin_start[bin];
      len = bin_start[bin + 1] - start;
      shift = pack_img(gx, gy, gz);
    }
    // inclusive wave scan of len
    int incl = len;
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d, 64);
      if (lane >= d) incl += v;
    }
    const int excl = incl - len;
    s_pref[wv][lane + 1] = incl;
    if (lane == 0) s_pref[wv][0] = 0;
    s_start[wv][lane] = start;
    s_shift[wv][lane] = shift;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): LDS writes visible to the wave
    const int total = __shfl(incl, 63, 64);
    int my_hits = 0;  // count pass: hits of offset o (this lane's)
    int carry = -1;   // the offset of candidate c0 - 1
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int c = c0 + lane;
      // the offset of candidate c, the largest b with s_pref[b] <= c: each
      // non-empty offset marks its first candidate, and a running maximum over
      // the chunk (from the chunk before) fills the rest
      s_own[wv][lane] = -1;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);
      if (len > 0 && excl >= c0 && excl < c0 + 64) s_own[wv][excl - c0] = lane;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);
      int own = s_own[wv][lane];
      for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(own, d, 64);
        if (lane >= d) own = max(own, v);
      }
      own = max(own, carry);
      carry = __shfl(own, 63, 64);
      bool hit = false;
      int lo = 0, j = 0, mj = 0, T0 = 0, T1 = 0, T2 = 0;
      Cand a;
      a.x = a.y = a.z = 0.0;
      a.j = a.wrap = 0;
      double ddx = 0.0, ddy = 0.0, ddz = 0.0;
      if (c < total) {
        lo = own;                                      // s_pref[lo] <= c < s_pref[lo + 1]
        mj = s_start[wv][lo] + (c - s_pref[wv][lo]);  // j's slot
        a = cand[mj];
        j = a.j;
        int gsh[3], wj[3];
        unpack_img(s_shift[wv][lo], gsh);
        unpack_img(a.wrap, wj);
        T0 = gsh[0] - wj[0] + wi[0];
        T1 = gsh[1] - wj[1] + wi[1];
        T2 = gsh[2] - wj[2] + wi[2];
        if (!(j == i && T0 == 0 && T1 == 0 && T2 == 0)) {
          // d = (r_j - r_i) + T cell, the same operation order for a pair and its reverse
          double tx, ty, tz;
          lattice_shift(T0, T1, T2, cell, tx, ty, tz);
          ddx = (a.x - pix) + tx;
          ddy = (a.y - piy) + ty;
          ddz = (a.z - piz) + tz;
          const double r2 = __fma_rn(ddz, ddz, __fma_rn(ddy, ddy, ddx * ddx));
          hit = r2 < rc2;
          if (hit && r2 < 1e-16) atomicOr(err, kErrCoincident);
        }
      }
      const unsigned long long mask = __ballot(hit);
      if (!FILL) {
        // this lane's offset owns candidates excl..incl-1
        const int lo_b = min(max(excl - c0, 0), 64), hi_b = min(max(incl - c0, 0), 64);
        my_hits += __popcll(mask & bit_range(lo_b, hi_b));
      }
      if (FILL && hit) {
        const long long q = out + __popcll(mask & ((1ull << lane) - 1ull));
        if (q < capacity) {
          // the reverse pair: j's hits before the opposite offset, then the
          // atoms of i's bin below i that j reaches with the shift -g
          int gsh[3];
          unpack_img(s_shift[wv][lo], gsh);
          int wj[3];
          unpack_img(a.wrap, wj);
          int rank = 0;
          for (int m = m0; m < m1; ++m) {
            const Cand b = cand[m];
            int wb[3];
            unpack_img(b.wrap, wb);
            const int U0 = -gsh[0] - wb[0] + wj[0], U1 = -gsh[1] - wb[1] + wj[1], U2 = -gsh[2] - wb[2] + wj[2];
            if (!(b.j == j && U0 == 0 && U1 == 0 && U2 == 0)) {
              double ux, uy, uz;
              lattice_shift(U0, U1, U2, cell, ux, uy, uz);
              const double ex = (b.x - a.x) + ux, ey = (b.y - a.y) + uy, ez = (b.z - a.z) + uz;
              rank += __fma_rn(ez, ez, __fma_rn(ey, ey, ex * ex)) < rc2;
            }
          }
          const long long rq = (long long)offsets[j] + opre_s[(long long)mj * n_off + (n_off - 1 - (g0 + lo))] + rank;
          nj[q] = j;
          nimg[q] = pack_img(T0, T1, T2);
          ncenter[q] = i;
          nrev[q] = rq < capacity ? (int)rq : (int)q;  // an overflowed list holds no valid reverse
          ndx[q] = ddx;
          ndy[q] = ddy;
          ndz[q] = ddz;
        }
      }
      out += __popcll(mask);
      cnt += __popcll(mask);
    }
    if (!FILL) {
      // hits before each offset of this group: the centre's running count plus a wave scan
      int h = my_hits;
      for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(h, d, 64);
        if (lane >= d) h += v;
      }
      const int group_hits = __shfl(h, 63, 64);  // read by every lane, outside the branch below
      if (o < n_off) opre_s[(long long)mc * n_off + o] = cnt - group_hits + (h - my_hits);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (!FILL && lane == 0) count[i] = cnt;
}

// ---------------------------------------------------------------- scan
// Exclusive prefix sum of n int32 counts into out[0..n] (out[n] = total), three
// passes: per-block totals, one-block scan of the totals, per-block scan + offset.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int block_exclusive_scan(int v, int* sh, int& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    int x = (t >= o) ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  total = sh[kScanThreads - 1];
  int excl = sh[t] - v;
  __syncthreads();
  return excl;
}

__global__ void k_scan_partials(int n, const int* __restrict__ in, int* __restrict__ part) {
  __shared__ int sh[kScanThreads];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int s = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  int total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void k_scan_top(int nb, int* __restrict__ part) {
  __shared__ int sh[kScanThreads];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
    int idx = b0 + threadIdx.x;
    int v = idx < nb ? part[idx] : 0;
    int total;
    int ex = block_exclusive_scan(v, sh, total);
    if (idx < nb) part[idx] = carry + ex;
    carry += total;
  }
}

__global__ void k_scan_final(int n, const int* __restrict__ in, const int* __restrict__ part, int* __restrict__ out) {
  // scans n + 1 elements with a virtual zero at index n, so out[n] is the total
  __shared__ int sh[kScanThreads];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int total;
  int ex = block_exclusive_scan(s, sh, total) + part[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k <= n) out[base + k] = ex;
    ex += v[k];
  }
}

// one workgroup for n + 1 <= kScanSingle: out[0..n], out[n] = total
constexpr int kScanSingleThreads = 1024, kScanSingleItems = 16;
constexpr int kScanSingle = kScanSingleThreads * kScanSingleItems;

__global__ __launch_bounds__(kScanSingleThreads) void k_scan_single(int n, const int* __restrict__ in,
                                                                     int* __restrict__ out) {
  __shared__ int sh[kScanSingleThreads];
  const int t = threadIdx.x;
  const int per = (n + 1 + kScanSingleThreads - 1) / kScanSingleThreads;
  const int base = t * per;
  int v[kScanSingleItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanSingleItems; ++k) {
    v[k] = (k < per && base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  sh[t] = s;
  __syncthreads();
  for (int o = 1; o < kScanSingleThreads; o <<= 1) {
    const int x = (t >= o) ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int ex = sh[t] - s;
#pragma unroll
  for (int k = 0; k < kScanSingleItems; ++k) {
    if (k < per && base + k <= n) out[base + k] = ex;
    ex += v[k];
  }
}

// zero the bin counters, the bin cursors and the error word before a build
__global__ void k_init_build(int n_bins, int* __restrict__ bin_count, int* __restrict__ bin_cursor,
                             int* __restrict__ err) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_bins) {
    bin_count[t] = 0;
    bin_cursor[t] = 0;
  }
  if (t < 4) err[t] = 0;
}

// d_p = (r_j - r_i) + T cell for every listed pair from the current positions,
// with the expression and operation order of k_pairs, so unmoved atoms give the
// bits of a fresh build (a list reused under a Verlet skin)
__global__ __launch_bounds__(256) void k_pair_vectors(long long bound, const int* __restrict__ count,
                                                      const double* __restrict__ pos,
                                                      const StructMeta* __restrict__ meta,
                                                      const int* __restrict__ so, int n_struct,
                                                      const int* __restrict__ ncenter, const int* __restrict__ nj,
                                                      const int* __restrict__ nimg, double* __restrict__ ndx,
                                                      double* __restrict__ ndy, double* __restrict__ ndz) {
  const long long n_pairs = count ? min(bound, (long long)max(*count, 0)) : bound;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const int i = ncenter[p], j = nj[p];
  const StructMeta& M = meta[find_structure(so, n_struct, i)];
  int T[3];
  unpack_img(nimg[p], T);
  double tx, ty, tz;
  lattice_shift(T[0], T[1], T[2], M.cell, tx, ty, tz);
  ndx[p] = (pos[3 * j] - pos[3 * i]) + tx;
  ndy[p] = (pos[3 * j + 1] - pos[3 * i + 1]) + ty;
  ndz[p] = (pos[3 * j + 2] - pos[3 * i + 2]) + tz;
}

// out[0] = pair count, out[1] = error bits of the last build (out may be host-pinned memory)
__global__ void k_report(const int* __restrict__ total, const int* __restrict__ err, int* __restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = *total;
    out[1] = *err;
  }
}

}  // namespace

hipError_t launch_pair_vectors(long long bound, const int* count, const double* pos, const StructMeta* meta,
                               const int* so, int n_struct, const int* ncenter, const int* nj, const int* nimg,
                               double* ndx, double* ndy, double* ndz, hipStream_t st) {
  if (bound == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_vectors, dim3((unsigned)((bound + 255) / 256)), dim3(256), 0, st, bound, count, pos, meta,
                     so, n_struct, ncenter, nj, nimg, ndx, ndy, ndz);
  return hipGetLastError();
}

hipError_t launch_report(const int* total, const int* err, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, st, total, err, out);
  return hipGetLastError();
}

hipError_t launch_init_build(int n_bins, int* bin_count, int* bin_cursor, int* err, hipStream_t st) {
  const int n = n_bins > 4 ? n_bins : 4;
  hipLaunchKernelGGL(k_init_build, dim3((n + 255) / 256), dim3(256), 0, st, n_bins, bin_count, bin_cursor, err);
  return hipGetLastError();
}

hipError_t scan_exclusive(const int* in, int n, int* out, int* part, hipStream_t st) {
  if (n + 1 <= kScanSingle) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanSingleThreads), 0, st, n, in, out);
    return hipGetLastError();
  }
  const int nb = (n + kScanTile) / kScanTile;  // at least one block, covers index n
  hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kScanThreads), 0, st, n, in, part);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, nb, part);
  hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanThreads), 0, st, n, in, part, out);
  return hipGetLastError();
}

int scan_partials_needed(int n) { return (n + kScanTile) / kScanTile; }

size_t bin_small_lds_bytes(int n_atoms, int n_bins) { return sizeof(int) * ((size_t)n_atoms + 2 * (size_t)n_bins); }

bool bin_small_fits(int n_atoms, int n_bins) {
  return n_atoms > 0 && n_atoms <= kSmallAtoms && n_bins <= kSmallBins &&
         bin_small_lds_bytes(n_atoms, n_bins) <= kSmallBinLds;
}

hipError_t launch_bin_small(int n_atoms, const double* pos, const StructMeta* meta, const int* so, int n_struct,
                            int n_bins, int* atom_bin, int* atom_wrap, int* bin_start, Cand* cand, int* err,
                            hipStream_t st) {
  if (!bin_small_fits(n_atoms, n_bins)) return hipErrorInvalidValue;
  static bool attr = false;  // LDS beyond 64 KB needs the opt-in once per process
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_bin_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             kSmallBinLds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_bin_small, dim3(1), dim3(kSmallBinThreads), bin_small_lds_bytes(n_atoms, n_bins), st, n_atoms,
                     pos, meta, so, n_struct, n_bins, atom_bin, atom_wrap, bin_start, cand, err);
  return hipGetLastError();
}

hipError_t launch_bin_atoms(int n_atoms, const double* pos, const StructMeta* meta, const int* so, int n_struct,
                            int* atom_bin, int* atom_wrap, int* bin_count, int* err, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_atoms, dim3((n_atoms + 255) / 256), dim3(256), 0, st, n_atoms, pos, meta, so, n_struct,
                     atom_bin, atom_wrap, bin_count, err);
  return hipGetLastError();
}

hipError_t launch_fill_bins(int n_atoms, const double* pos, const int* atom_bin, const int* atom_wrap,
                            const int* bin_start, int* bin_cursor, int* unsorted, Cand* cand, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_bins, dim3((n_atoms + 255) / 256), dim3(256), 0, st, n_atoms, atom_bin, bin_start,
                     bin_cursor, unsorted);
  hipLaunchKernelGGL(k_rank_bins, dim3((n_atoms + 255) / 256), dim3(256), 0, st, n_atoms, pos, atom_bin, atom_wrap,
                     bin_start, unsorted, cand);
  return hipGetLastError();
}

hipError_t launch_pairs(bool fill, int n_atoms, const double* pos, const StructMeta* meta, const int* so,
                        int n_struct, double rc, const int* atom_bin, const int* atom_wrap, const int* bin_start,
                        const Cand* cand, int* count, int* opre, const int* offsets, long long capacity, int* nj,
                        int* nimg, int* ncenter, double* ndx, double* ndy, double* ndz, int* nrev, int* err,
                        hipStream_t st) {
  dim3 g((n_atoms + 3) / 4), b(256);
  if (fill)
    hipLaunchKernelGGL(k_pairs<true>, g, b, 0, st, n_atoms, pos, meta, so, n_struct, rc * rc, atom_bin, atom_wrap,
                       bin_start, cand, count, opre, offsets, capacity, nj, nimg, ncenter, ndx, ndy, ndz, nrev, err);
  else
    hipLaunchKernelGGL(k_pairs<false>, g, b, 0, st, n_atoms, pos, meta, so, n_struct, rc * rc, atom_bin, atom_wrap,
                       bin_start, cand, count, opre, offsets, capacity, nj, nimg, ncenter, ndx, ndy, ndz, nrev, err);
  return hipGetLastError();
}

}  // namespace soap
