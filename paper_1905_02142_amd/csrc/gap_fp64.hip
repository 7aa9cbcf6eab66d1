// GAP energy and its adjoint in FP64 (Sec. IV.A: e_i = sum_s alpha_s k(i, s),
// k = (q_i . q_s)^zeta, the dot-product SOAP kernel of Sec. I).
//
//   S = Q Q_s^T                      (N x M, contraction over the descriptor length K)
//   e_i = sum_s alpha_s S_is^zeta
//   G_is = zeta alpha_s S_is^(zeta-1)      -> Qbar = G Q_s = dE/dQ
//   alpha_bar_s = sum_i S_is^zeta           = dE/dalpha_s
//
// Two LDS-tiled VALU GEMMs with 64 x 64 output tiles and 4 x 4 register blocks;
// partial row / column sums of the epilogue are reduced in a fixed order, so the
// result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "gap.h"

namespace soap {

namespace {

constexpr int kT = 64;   // output tile
constexpr int kKT = 16;  // contraction tile

__device__ inline double ipow(double x, int e) {
  double r = 1.0;
  for (int t = 0; t < e; ++t) r *= x;
  return r;
}

// S tile, epilogue, G written; e_part[st][i], ab_part[it][s]
__global__ __launch_bounds__(256) void k_gap_scores(int N, int M, int K, const double* __restrict__ Q,
                                                    const double* __restrict__ Qs, const double* __restrict__ alpha,
                                                    int zeta, double* __restrict__ G, double* __restrict__ e_part,
                                                    double* __restrict__ ab_part) {
  __shared__ double As[kKT][kT + 1];
  __shared__ double Bs[kKT][kT + 1];
  __shared__ double colsum[4][kT];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int i0 = blockIdx.y * kT, s0 = blockIdx.x * kT;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += kKT) {
    for (int t = tid; t < kT * kKT; t += 256) {
      const int r = t / kKT, kk = t % kKT;
      const int gi = i0 + r, gs = s0 + r, gk = k0 + kk;
      As[kk][r] = (gi < N && gk < K) ? Q[(size_t)gi * K + gk] : 0.0;
      Bs[kk][r] = (gs < M && gk < K) ? Qs[(size_t)gs * K + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKT; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        a[x] = As[kk][ty + 16 * x];
        b[x] = Bs[kk][tx + 16 * x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
  double rows[4] = {0, 0, 0, 0}, cols[4] = {0, 0, 0, 0};
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int gi = i0 + ty + 16 * x;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int gs = s0 + tx + 16 * y;
      if (gi < N && gs < M) {
        const double s = acc[x][y];
        const double sz1 = ipow(s, zeta - 1);
        const double kv = sz1 * s;
        const double al = alpha[gs];
        G[(size_t)gi * M + gs] = (double)zeta * al * sz1;
        rows[x] = fma(al, kv, rows[x]);
        cols[y] += kv;
      }
    }
  }
  // row sums over the 16 threads sharing ty (consecutive lanes)
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    double v = rows[x];
    for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
    const int gi = i0 + ty + 16 * x;
    if (tx == 0 && gi < N) e_part[(size_t)blockIdx.x * N + gi] = v;
  }
  // column sums over ty: within the wave (4 ty values), then across the 4 waves
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    double v = cols[y];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if ((tid & 63) < 16) colsum[tid / 64][tx + 16 * y] = v;
  }
  __syncthreads();
  if (tid < kT) {
    const int gs = s0 + tid;
    if (gs < M) ab_part[(size_t)blockIdx.y * M + gs] = colsum[0][tid] + colsum[1][tid] + colsum[2][tid] + colsum[3][tid];
  }
}

// Qbar = G Q_s: tile over (atoms, descriptor index), contraction over sparse points
__global__ __launch_bounds__(256) void k_gap_qbar(int N, int M, int K, const double* __restrict__ G,
                                                  const double* __restrict__ Qs, double* __restrict__ Qbar) {
  __shared__ double As[kKT][kT + 1];
  __shared__ double Bs[kKT][kT + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int i0 = blockIdx.y * kT, k0 = blockIdx.x * kT;
  double acc[4][4] = {};
  for (int s0 = 0; s0 < M; s0 += kKT) {
    for (int t = tid; t < kT * kKT; t += 256) {
      const int r = t / kKT, ss = t % kKT;  // G[i0 + r][s0 + ss]
      const int gi = i0 + r, gs = s0 + ss;
      As[ss][r] = (gi < N && gs < M) ? G[(size_t)gi * M + gs] : 0.0;
      const int rr = t / kT, cc = t % kT;    // Qs[s0 + rr][k0 + cc]
      const int gs2 = s0 + rr, gk = k0 + cc;
      Bs[rr][cc] = (gs2 < M && gk < K) ? Qs[(size_t)gs2 * K + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ss = 0; ss < kKT; ++ss) {
      double a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        a[x] = As[ss][ty + 16 * x];
        b[x] = Bs[ss][tx + 16 * x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int gi = i0 + ty + 16 * x;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int gk = k0 + tx + 16 * y;
      if (gi < N && gk < K) Qbar[(size_t)gi * K + gk] = acc[x][y];
    }
  }
}

// out[j] = sum_t part[t * n + j], t = 0..nt-1 in order
__global__ void k_sum_parts(int n, int nt, const double* __restrict__ part, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int t = 0; t < nt; ++t) s += part[(size_t)t * n + j];
  out[j] = s;
}

}  // namespace

size_t gap_fp64_workspace_doubles(int N, int M) {
  const size_t nst = (M + kT - 1) / kT, nit = (N + kT - 1) / kT;
  return (size_t)N * M + nst * N + nit * M;
}

hipError_t launch_gap_fp64(int N, int M, int K, const double* Q, const double* Qs, const double* alpha, int zeta,
                           double* e, double* Qbar, double* alpha_bar, double* work, hipStream_t st) {
  if (N == 0) return hipSuccess;
  const int nst = (M + kT - 1) / kT, nit = (N + kT - 1) / kT;
  double* G = work;
  double* e_part = G + (size_t)N * M;
  double* ab_part = e_part + (size_t)nst * N;
  hipLaunchKernelGGL(k_gap_scores, dim3(nst, nit), dim3(256), 0, st, N, M, K, Q, Qs, alpha, zeta, G, e_part, ab_part);
  hipLaunchKernelGGL(k_sum_parts, dim3((N + 255) / 256), dim3(256), 0, st, N, nst, e_part, e);
  if (alpha_bar)
    hipLaunchKernelGGL(k_sum_parts, dim3((M + 255) / 256), dim3(256), 0, st, M, nit, ab_part, alpha_bar);
  if (Qbar) hipLaunchKernelGGL(k_gap_qbar, dim3((K + kT - 1) / kT, nit), dim3(256), 0, st, N, M, K, G, Qs, Qbar);
  return hipGetLastError();
}

}  // namespace soap
