// Host interface of the GAP kernel contractions.
#pragma once

#include <hip/hip_runtime.h>

namespace soap {

// FP64: e (N), Qbar (N x K, nullable), alpha_bar (M, nullable); work holds
// gap_fp64_workspace_doubles(N, M) doubles.
size_t gap_fp64_workspace_doubles(int N, int M);
hipError_t launch_gap_fp64(int N, int M, int K, const double* Q, const double* Qs, const double* alpha, int zeta,
                           double* e, double* Qbar, double* alpha_bar, double* work, hipStream_t st);

}  // namespace soap
