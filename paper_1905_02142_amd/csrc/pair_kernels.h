// Host interface of the descriptor forward / adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "soap_device.h"

namespace soap {

size_t descriptor_lds_bytes(const DevParams& P);
size_t adjoint_lds_bytes(const DevParams& P);

// c (n_atoms x nch x LL), q (n_atoms rows of q_pitch >= K, zero beyond K) and |p|
hipError_t launch_descriptor(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, const int* nj,
                             const double* dx, const double* dy, const double* dz, const int* species, double* c,
                             double* q, int q_pitch, double* pnorm, hipStream_t st);

// pair gradients g_p = dE/dd_p (SoA) from qbar = dE/dq and the forward c, q, |p|
hipError_t launch_pair_adjoint(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets,
                               const int* nj, const double* dx, const double* dy, const double* dz,
                               const int* species, const double* c, const double* q, int q_pitch,
                               const double* pnorm, const double* qbar, int qbar_pitch, double* gx, double* gy,
                               double* gz, hipStream_t st);

// angular slot order and ilexp series tables for these parameters
void build_angular_tables(const DevParams& P, DevTables& T);

// out = F (overwrite) or pos_grad -= F (accumulate_grad)
hipError_t launch_force_gather(int n_atoms, const int* offsets, const int* rev, const double* gx, const double* gy,
                               const double* gz, double* out, bool accumulate_grad, hipStream_t st);

}  // namespace soap
