// Host interface of the descriptor forward / adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "soap_device.h"

namespace soap {

size_t descriptor_lds_bytes(const DevParams& P);
size_t adjoint_lds_bytes(const DevParams& P);
// c and cbar workspace per atom: [species][lm < LL + 1][k < NMAX] doubles (NMAX =
// the compiled n_max bucket; the column lm = LL is a sink for unused records)
size_t c_doubles_per_atom(const DevParams& P);
// doubles per neighbour pair of the shared pair rows (radial values, ilexp, the
// direction u and their r-derivatives)
size_t pair_row_doubles(const DevParams& P);

// Every per-pair launch takes a pair bound: the exact pair count, or the list
// capacity when the count is still on the device.  Per-atom kernels cut each
// atom's range at the bound, so an overflowed list is read only where written.

// pair rows (pair_row_doubles fields each; blocks of 64 pairs stored
// field-major, pair_rows_bytes in all; FP64, or FP32 with rows_f32, which needs
// the FP64 radial stage) for n_pairs neighbours (or, with count
// non-null, for min(*count, n_pairs)), the derivative fields only if deriv, and
// the central-atom radial factors bc (n_max doubles); block: threads per block
// (64, 128 or 256); part 1: the radial fields and bc, part 2: the angular fields
// (two launches, both needed before the descriptor)
hipError_t launch_pair_prep(const DevParams& P, const DevTables* T, long long n_pairs, const int* count,
                            const double* dx, const double* dy, const double* dz, void* rows, bool rows_f32,
                            bool deriv, double* bc, int block, int part, hipStream_t st);
size_t pair_rows_bytes(const DevParams& P, long long n_pairs, bool f32 = false);

// c (n_atoms x c_doubles_per_atom), q (n_atoms rows of q_pitch >= K, zero beyond K) and |p|
// qc (nullable): a bf16 copy of q as well, row i at element i qc_pitch,
// (bf16)(float) q_ik and zero for the columns K..qc_pitch-1.  store_f32: the
// pair rows are read and c is written in FP32 (double otherwise); q stays FP64
hipError_t launch_descriptor(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, int bound,
                             const int* nj,
                             const int* species, const void* rows, bool store_f32, const double* bc, void* c,
                             double* q, int q_pitch, double* pnorm, void* qc, int qc_pitch, hipStream_t st);

// pair gradients g_p = dE/dd_p from qbar = dE/dq (n_atoms rows of
// qbar_pitch; with qbar2 non-null, qbar + qbar2, the two parts of a sliced GAP
// contraction), the forward c, q, |p| and the pair rows with derivatives; cbar
// is formed per atom inside the kernel.  gstride 1: three arrays gx, gy, gz;
// gstride 4: one record (x, y, z, 0) per pair at gx + 4 p (gy, gz unused).
// store_f32: the pair rows, c, qbar and qbar2 are FP32 (double otherwise)
hipError_t launch_pair_adjoint(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, int bound,
                               const int* nj, const int* species, const void* rows, bool store_f32, const void* c,
                               const double* q, int q_pitch, const double* pnorm, const void* qbar,
                               const void* qbar2, int qbar_pitch, double* gx, double* gy, double* gz,
                               int gstride, hipStream_t st);

// angular records (Qbar_lm polynomials) and ilexp series tables for these parameters
void build_angular_tables(const DevParams& P, DevTables& T);

// qbar (n_rows x K) = e_kset on every row; with kclear >= 0 only columns kset
// and kclear (the previous kset, set to zero) are written
hipError_t launch_unit_rows(int n_rows, int K, int kset, int kclear, double* qbar, hipStream_t st);

// out = F (overwrite) or pos_grad -= F (accumulate_grad), from the pair
// gradients as (x, y, z, 0) records (launch_pair_adjoint with gstride 4)
hipError_t launch_force_gather(int n_atoms, const int* offsets, int bound, const int* rev, const double* g,
                               double* out, bool accumulate_grad, hipStream_t st);

// p[0..n) = v, as a kernel (so that it may be captured in a graph)
hipError_t launch_fill(double* p, long long n, double v, hipStream_t st);

}  // namespace soap
