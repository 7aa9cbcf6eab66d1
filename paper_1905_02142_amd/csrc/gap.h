// Host interface of the GAP kernel contractions (MFMA).
#pragma once

#include <hip/hip_runtime.h>

namespace soap {

// prec: 0 FP64, 1 FP32, 2 BF16, 3 split BF16 (the soap_precision values).
// The workspace holds the converted, zero-padded operands, G and the per-tile
// partial sums.
size_t gap_workspace_bytes(int N, int M, int K, int prec);
// e (N) and alpha_bar (M, nullable); G stays in work for the qbar pass.  With
// sums false the per-tile partial sums are left in work for launch_gap_qbar to
// finish (e and alpha_bar are then written by that call)
// tile: the BF16 tile shapes (soap_tuning.gap_tile), 0 or 1; ignored in the other modes
hipError_t launch_gap_scores(int prec, int N, int M, int K, const double* Q, const double* Qs, const double* alpha,
                             int zeta, double* e, double* alpha_bar, bool sums, bool q_ready, void* work, int tile,
                             hipStream_t st);
// BF16 (prec 2) only: the N x gap_q_pitch(K) bf16 copy of Q inside work, for a
// producer of q that writes it itself (row i at element i Kp: (bf16)(float) q_ik,
// zero for the columns K..Kp-1), after which launch_gap_scores runs with q_ready
// and converts only the sparse set; nullptr for the other modes
void* gap_q_operand(int prec, int N, int M, int K, void* work);
int gap_q_pitch(int K);
// Qbar = G Q_s, from the operands the scores pass left in work, as `slices`
// parts (Qbar + s N K, s < slices, each N x K) that sum to it: part s contracts
// over the sparse points s Mp / slices .. (s + 1) Mp / slices - 1, which
// multiplies the workgroups of this long contraction.  With e non-null it also
// finishes e and alpha_bar (nullable) from the partial sums.  Qbar is FP32 with
// f32 (the modes that accumulate in FP32; not prec 0), FP64 otherwise
hipError_t launch_gap_qbar(int prec, int N, int M, int K, void* Qbar, bool f32, double* e, double* alpha_bar,
                           const void* work, int slices, int tile, hipStream_t st);
// the slice count launch_gap_qbar accepts and that pays off for an N x K output
// contracted over M sparse points: 1 or 2
int gap_qbar_slices(int N, int M, int K, int prec, int tile);

// Fused scores + Qbar (prec 1..3, padded K <= 352): e, alpha_bar (nullable) and
// Qbar in one pass with no N x M intermediate in HBM
bool gap_fused_supported(int K, int prec);
// target: number of workgroups the sparse-set slices should fill
size_t gap_fused_workspace_bytes(int N, int M, int K, int prec, int target);
// Qbar: FP32 with f32, FP64 otherwise
hipError_t launch_gap_fused(int prec, int N, int M, int K, const double* Q, const double* Qs, const double* alpha,
                            int zeta, double* e, double* alpha_bar, void* Qbar, bool f32, void* work, int target,
                            hipStream_t st);

}  // namespace soap
