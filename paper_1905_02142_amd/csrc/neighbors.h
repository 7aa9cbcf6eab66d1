// Host/device interface of the neighbour-list kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace soap {

// Geometry of one structure's cell list (host-built, device-read).
struct StructMeta {
  double cell[9];  // rows: lattice vectors a, b, c
  double inv[9];   // inverse of the cell matrix: fractional = position * inv
  int nbin[3];     // slabs per axis (1 on non-periodic axes)
  int R[3];        // slabs scanned either side (0 on non-periodic axes)
  int pbc[3];
  int bin0;        // first global bin of this structure
  int atom0, atom1;
  int n_off;       // slab offsets a centre scans: (2R0+1)(2R1+1)(2R2+1)
  int pad_;
  long long obase; // first entry of this structure's per-(centre, offset) hit prefixes
};

// One atom as a cell-list candidate, stored in bin order: its position (as
// given), index and the lattice wrap that brings it into the cell.
struct alignas(16) Cand {
  double x, y, z;
  int j, wrap;
};

// The lattice translation T cell (T integer, cell rows the lattice vectors),
// with explicit FMAs so that every kernel rounds it identically.
__device__ inline void lattice_shift(int t0, int t1, int t2, const double* cell, double& tx, double& ty,
                                     double& tz) {
  tx = __fma_rn((double)t2, cell[6], __fma_rn((double)t1, cell[3], (double)t0 * cell[0]));
  ty = __fma_rn((double)t2, cell[7], __fma_rn((double)t1, cell[4], (double)t0 * cell[1]));
  tz = __fma_rn((double)t2, cell[8], __fma_rn((double)t1, cell[5], (double)t0 * cell[2]));
}

// error bits raised by the kernels
constexpr int kErrNonFinite = 1;
constexpr int kErrCoincident = 2;
constexpr int kErrFarOutside = 8;

// lattice image (or cell wrap) packed in 30 bits, 10 bits per axis, |T| <= 511
constexpr int kWrapMax = 500;
__host__ __device__ inline int pack_img(int a, int b, int c) {
  return ((a + 512) << 20) | ((b + 512) << 10) | (c + 512);
}
__host__ __device__ inline void unpack_img(int v, int* t) {
  t[0] = ((v >> 20) & 1023) - 512;
  t[1] = ((v >> 10) & 1023) - 512;
  t[2] = (v & 1023) - 512;
}

// one-workgroup cell list for small systems (bin_small_fits)
constexpr int kSmallAtoms = 16384;
constexpr int kSmallBins = 16384;
constexpr int kSmallBinThreads = 1024;
constexpr int kSmallBinLds = 150 * 1024;  // dynamic LDS opt-in of one workgroup
bool bin_small_fits(int n_atoms, int n_bins);
// err[0..4) cleared; atom_bin, atom_wrap, bin_start (n_bins + 1) and cand
// (the atoms of each bin by ascending index) written
hipError_t launch_bin_small(int n_atoms, const double* pos, const StructMeta* meta, const int* so, int n_struct,
                            int n_bins, int* atom_bin, int* atom_wrap, int* bin_start, Cand* cand, int* err,
                            hipStream_t st);

// zero bin_count[0..n_bins), bin_cursor[0..n_bins) and err[0..4)
hipError_t launch_init_build(int n_bins, int* bin_count, int* bin_cursor, int* err, hipStream_t st);
hipError_t scan_exclusive(const int* in, int n, int* out, int* part, hipStream_t st);
int scan_partials_needed(int n);
hipError_t launch_bin_atoms(int n_atoms, const double* pos, const StructMeta* meta, const int* so, int n_struct,
                            int* atom_bin, int* atom_wrap, int* bin_count, int* err, hipStream_t st);
// cand: the atoms of each bin by ascending index (unsorted: n_atoms ints of scratch)
hipError_t launch_fill_bins(int n_atoms, const double* pos, const int* atom_bin, const int* atom_wrap,
                            const int* bin_start, int* bin_cursor, int* unsorted, Cand* cand, hipStream_t st);
// Count pass (fill false): count[i] = pairs of centre i, and opre (per
// structure from meta.obase, n_off entries per centre) = the hits of each centre
// before each slab offset.  Fill pass: the pairs of centre i from offsets[i],
// below capacity, with rev from offsets and opre.
hipError_t launch_pairs(bool fill, int n_atoms, const double* pos, const StructMeta* meta, const int* so,
                        int n_struct, double rc, const int* atom_bin, const int* atom_wrap, const int* bin_start,
                        const Cand* cand, int* count, int* opre, const int* offsets, long long capacity, int* nj,
                        int* nimg, int* ncenter, double* ndx, double* ndy, double* ndz, int* nrev, int* err,
                        hipStream_t st);
// pair vectors d_p = r_j + T cell - r_i of listed pairs 0..min(*count, bound) (count
// nullptr: 0..bound) from positions pos
hipError_t launch_pair_vectors(long long bound, const int* count, const double* pos, const StructMeta* meta,
                               const int* so, int n_struct, const int* ncenter, const int* nj, const int* nimg,
                               double* ndx, double* ndy, double* ndz, hipStream_t st);
// out[0] = *total, out[1] = *err, written by one kernel (out may be mapped host memory)
hipError_t launch_report(const int* total, const int* err, int* out, hipStream_t st);

}  // namespace soap
