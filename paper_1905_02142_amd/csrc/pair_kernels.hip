// Descriptor forward and adjoint kernels (FP64 VALU).
//
// Forward, one 64-lane wavefront per centre atom i (Sec. II, Eqs. (05), (08), (09)):
//   1. per-pair phase: lane t of a chunk of 16 neighbours computes
//        B_k = 4 pi A b_k              (radial recursion, orthonormal transform)
//        Ang_lm = w_l e_l Y_lm(u)      (ilexp and real spherical harmonics)
//      and stages them in LDS;
//   2. accumulation c[k][lm] += B_k Ang_lm: lane (pg, sl) owns the channels k of
//      the lm slice sl and the neighbours of pair group pg, so every LDS read of
//      a B row feeds LMS x n FMAs held in registers;
//   3. the PG partial sums are combined by DPP quad shuffles, the central atom is
//      added, c is stored (it is re-read by the adjoint), then p_{ab l} =
//      sum_m c[a][lm] c[b][lm] is formed from c in LDS and normalised in place.
// Channels of species s are accumulated together: neighbours are compacted per
// species with a wave ballot, so one register tile serves every species block.
//
// Adjoint, one wavefront per centre atom:
//   qbar -> vbar = (qbar - q (q.qbar)) / |p|  -> cbar = M c (M from vbar) in LDS,
//   then one lane per neighbour recomputes B, dB/dr, e_l, de_l/dz, Y_lm, grad Y_lm
//   and contracts them with cbar into the pair gradient g = dE/dd.
// Forces are gathered per atom through the reverse-pair index: no atomics, so
// FP64 results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "pair_kernels.h"
#include "soap_device.h"

namespace soap {

namespace {

template <int CTRL>
__device__ inline double dpp_move(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

// real spherical harmonics with the gradient of their polynomial extension:
// put(l, lm, Y, dY/dv_x, dY/dv_y, dY/dv_z)
template <int LM, typename F>
__device__ inline void real_ylm_grad(const DevTables* __restrict__ T, int lmax, double ux, double uy, double uz,
                                     F&& put) {
  double cr = 1.0, ci = 0.0;  // (u_x + i u_y)^m
  double pr = 0.0, pi = 0.0;  // (u_x + i u_y)^(m-1)
#pragma unroll
  for (int m = 0; m <= LM; ++m) {
    if (m <= lmax) {
      double q2 = 0.0, q1 = T->ymm[m];
      double d2 = 0.0, d1 = 0.0;  // d/dz of Qbar
#pragma unroll
      for (int l = m; l <= LM; ++l) {
        if (l <= lmax) {
          double q, d;
          if (l == m) {
            q = q1;
            d = d1;
          } else {
            const double a = T->ya[lm_tri(l, m)], b = T->yb[lm_tri(l, m)];
            q = a * uz * q1 - b * q2;
            d = a * (q1 + uz * d1) - b * d2;
            q2 = q1;
            q1 = q;
            d2 = d1;
            d1 = d;
          }
          if (m == 0) {
            put(l, l * l + l, q, 0.0, 0.0, d);
          } else {
            const double fm = (double)m;
            put(l, l * l + l + m, q * cr, q * fm * pr, -q * fm * pi, d * cr);
            put(l, l * l + l - m, q * ci, q * fm * pi, q * fm * pr, d * ci);
          }
        }
      }
    }
    pr = cr;
    pi = ci;
    const double nr = cr * ux - ci * uy;
    ci = cr * uy + ci * ux;
    cr = nr;
  }
}

template <int NMAX, int LMAX, int PG>
__global__ __launch_bounds__(64) void k_descriptor(DevParams P, const DevTables* __restrict__ T, int n_atoms,
                                                   const int* __restrict__ offsets, const int* __restrict__ nj,
                                                   const double* __restrict__ dx, const double* __restrict__ dy,
                                                   const double* __restrict__ dz, const int* __restrict__ species,
                                                   double* __restrict__ c_out, double* __restrict__ q_out,
                                                   double* __restrict__ pnorm_out) {
  constexpr int LLM = (LMAX + 1) * (LMAX + 1);
  constexpr int SL = 64 / PG;
  constexpr int LMS = (LLM + SL - 1) / SL;
  constexpr int CH = 16;
  constexpr int AST = LLM + 1;
  constexpr int BST = NMAX + 1;
  __shared__ double ang[CH * AST];
  __shared__ double bsh[CH * BST];
  __shared__ double bc[NMAX];
  __shared__ int idx[64];
  extern __shared__ double dyn[];

  const int i = blockIdx.x;
  if (i >= n_atoms) return;
  const int lane = threadIdx.x;
  const int pg = lane % PG, sl = lane / PG;
  const int n = P.n, LL = P.LL, nch = P.nch, LLP = LL + 1;
  double* csh = dyn;
  double* vsh = dyn + nch * LLP;
  const int p0 = offsets[i], p1 = offsets[i + 1];
  const int si = P.ns == 1 ? 0 : species[i];

  if (lane == 0) {
    double B[NMAX], dB[NMAX];
    radial<NMAX, false>(P, T, 0.0, B, dB);
    // r = 0: e_0 = 1, e_{l>0} = 0 and Y_00 = 1 / sqrt(4 pi)
#pragma unroll
    for (int k = 0; k < NMAX; ++k) bc[k] = P.cw * B[k] * T->lw[0] * 0.28209479177387814;
  }
  __syncthreads();

  for (int s = 0; s < P.ns; ++s) {
    double acc[LMS][NMAX];
#pragma unroll
    for (int kk = 0; kk < LMS; ++kk)
#pragma unroll
      for (int k = 0; k < NMAX; ++k) acc[kk][k] = 0.0;

    for (int w0 = p0; w0 < p1; w0 += 64) {
      const int p = w0 + lane;
      const bool take = p < p1 && (P.ns == 1 || species[nj[p]] == s);
      const unsigned long long mask = __ballot(take);
      if (take) idx[__popcll(mask & ((1ull << lane) - 1ull))] = p;
      const int cnt = __popcll(mask);
      __syncthreads();
      for (int c0 = 0; c0 < cnt; c0 += CH) {
        const int nc = min(CH, cnt - c0);
        if (lane < nc) {
          const int pp = idx[c0 + lane];
          const double x = dx[pp], y = dy[pp], z = dz[pp];
          const double r = sqrt(x * x + y * y + z * z), ir = 1.0 / r;
          double B[NMAX], dB[NMAX];
          radial<NMAX, false>(P, T, r, B, dB);
#pragma unroll
          for (int k = 0; k < NMAX; ++k) bsh[lane * BST + k] = B[k];
          const double sp = P.s0p + P.ap * r;
          double e[LMAX + 1];
          ilexp<LMAX>(r * r / (sp * sp), P.l, e);
          double we[LMAX + 1];
#pragma unroll
          for (int l = 0; l <= LMAX; ++l) we[l] = T->lw[l] * e[l];
          double* row = ang + lane * AST;
          real_ylm<LMAX>(T, P.l, x * ir, y * ir, z * ir, [&](int l, int lm, double v) { row[lm] = we[l] * v; });
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < CH / PG; ++t) {
          const int pi = pg + PG * t;
          if (pi < nc) {
            double b[NMAX];
#pragma unroll
            for (int k = 0; k < NMAX; ++k) b[k] = bsh[pi * BST + k];
#pragma unroll
            for (int kk = 0; kk < LMS; ++kk) {
              const int lm = sl + SL * kk;
              if (lm < LL) {
                const double a = ang[pi * AST + lm];
#pragma unroll
                for (int k = 0; k < NMAX; ++k) acc[kk][k] = fma(a, b[k], acc[kk][k]);
              }
            }
          }
        }
        __syncthreads();
      }
    }
    // combine the pair groups
#pragma unroll
    for (int kk = 0; kk < LMS; ++kk)
#pragma unroll
      for (int k = 0; k < NMAX; ++k) {
        double v = acc[kk][k];
        if (PG >= 2) v += dpp_move<kQuadXor1>(v);
        if (PG >= 4) v += dpp_move<kQuadXor2>(v);
        acc[kk][k] = v;
      }
    if (s == si && sl == 0) {
#pragma unroll
      for (int k = 0; k < NMAX; ++k) acc[0][k] += bc[k];
    }
#pragma unroll
    for (int kk = 0; kk < LMS; ++kk) {
      const int lm = sl + SL * kk;
      if (lm < LL) {
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
          if (k < n && (k % PG) == pg) {
            const int ch = s * n + k;
            c_out[((size_t)i * nch + ch) * LL + lm] = acc[kk][k];
            csh[ch * LLP + lm] = acc[kk][k];
          }
        }
      }
    }
  }
  __syncthreads();
  // power spectrum p_{ab l} (real form of Eq. (09)), packed a <= b then l,
  // off-diagonal scaled by sqrt(2); then q = p / |p|
  const int L1 = P.l + 1;
  double ss = 0.0;
  for (int k = lane; k < P.K; k += 64) {
    const int ab = k / L1, l = k - ab * L1;
    int a, b;
    ab_decode(ab, nch, a, b);
    const double* ca = csh + a * LLP + l * l;
    const double* cb = csh + b * LLP + l * l;
    double v = 0.0;
    for (int m = 0; m < 2 * l + 1; ++m) v = fma(ca[m], cb[m], v);
    if (a != b) v *= kSqrt2;
    vsh[k] = v;
    ss = fma(v, v, ss);
  }
  ss = wave_sum(ss);
  const double nrm = sqrt(ss);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int k = lane; k < P.K; k += 64) q_out[(size_t)i * P.K + k] = vsh[k] * inv;
  if (lane == 0 && pnorm_out) pnorm_out[i] = nrm;
}

template <int NMAX, int LMAX>
__global__ __launch_bounds__(64) void k_pair_adjoint(DevParams P, const DevTables* __restrict__ T, int n_atoms,
                                                     const int* __restrict__ offsets, const int* __restrict__ nj,
                                                     const double* __restrict__ dx, const double* __restrict__ dy,
                                                     const double* __restrict__ dz, const int* __restrict__ species,
                                                     const double* __restrict__ c, const double* __restrict__ q,
                                                     const double* __restrict__ pnorm,
                                                     const double* __restrict__ qbar, double* __restrict__ gx,
                                                     double* __restrict__ gy, double* __restrict__ gz) {
  extern __shared__ double dyn[];
  const int i = blockIdx.x;
  if (i >= n_atoms) return;
  const int lane = threadIdx.x;
  const int n = P.n, LL = P.LL, nch = P.nch, LLP = LL + 1, K = P.K, L1 = P.l + 1;
  double* csh = dyn;
  double* cbs = csh + nch * LLP;
  double* vb = cbs + nch * LLP;
  const int p0 = offsets[i], p1 = offsets[i + 1];

  for (int t = lane; t < nch * LL; t += 64) {
    const int ch = t / LL, lm = t - ch * LL;
    csh[ch * LLP + lm] = c[(size_t)i * nch * LL + t];
  }
  // vbar = (qbar - q (q . qbar)) / |p|
  const double nrm = pnorm[i];
  double dot = 0.0;
  for (int k = lane; k < K; k += 64) dot = fma(q[(size_t)i * K + k], qbar[(size_t)i * K + k], dot);
  dot = wave_sum(dot);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int k = lane; k < K; k += 64) vb[k] = (qbar[(size_t)i * K + k] - q[(size_t)i * K + k] * dot) * inv;
  __syncthreads();
  // cbar[a][lm] = sum_b M_ab(l) c[b][lm]; M_aa = 2 vbar_(aa,l), M_ab = sqrt(2) vbar_(ab,l)
  for (int t = lane; t < nch * LL; t += 64) {
    const int a = t / LL, lm = t - a * LL;
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    double s = 0.0;
    for (int b = 0; b < nch; ++b) {
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      const double w = (a == b) ? 2.0 : kSqrt2;
      s = fma(w * vb[ab_index(lo, hi, nch) * L1 + l], csh[b * LLP + lm], s);
    }
    cbs[a * LLP + lm] = s;
  }
  __syncthreads();
  for (int p = p0 + lane; p < p1; p += 64) {
    const double x = dx[p], y = dy[p], z = dz[p];
    const double r = sqrt(x * x + y * y + z * z), ir = 1.0 / r;
    const double ux = x * ir, uy = y * ir, uz = z * ir;
    double B[NMAX], dB[NMAX];
    radial<NMAX, true>(P, T, r, B, dB);
    const double sp = P.s0p + P.ap * r;
    const double zz = r * r / (sp * sp);
    const double dzdr = 2.0 * r / (sp * sp) - 2.0 * r * r * P.ap / (sp * sp * sp);
    double e[LMAX + 2];
    ilexp<LMAX + 1>(zz, P.l + 1, e);
    const int sj = P.ns == 1 ? 0 : species[nj[p]];
    if (sj < 0 || sj >= P.ns) {  // a label outside 0..n_species-1 contributes nothing
      gx[p] = gy[p] = gz[p] = 0.0;
      continue;
    }
    const double* base = cbs + sj * n * LLP;
    double gr = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
    real_ylm_grad<LMAX>(T, P.l, ux, uy, uz, [&](int l, int lm, double Y, double vx, double vy, double vz) {
      double U = 0.0, V = 0.0;
#pragma unroll
      for (int k = 0; k < NMAX; ++k) {
        if (k < n) {
          const double cb = base[k * LLP + lm];
          U = fma(cb, dB[k], U);
          V = fma(cb, B[k], V);
        }
      }
      const double wl = T->lw[l];
      const double de = e[l + 1] + ((double)l / zz - 1.0) * e[l];
      gr = fma(wl * (U * e[l] + V * de * dzdr), Y, gr);
      const double beta = wl * e[l] * V;
      tx = fma(beta, vx, tx);
      ty = fma(beta, vy, ty);
      tz = fma(beta, vz, tz);
    });
    // d u / d d = (I - u u^T) / r
    const double ut = ux * tx + uy * ty + uz * tz;
    gx[p] = gr * ux + (tx - ux * ut) * ir;
    gy[p] = gr * uy + (ty - uy * ut) * ir;
    gz[p] = gr * uz + (tz - uz * ut) * ir;
  }
}

// F_k = sum over k's pairs q of (g_q - g_rev(q)) (= -dE/dr_k); mode 1 adds -F_k into
// pos_grad.  16 lanes per atom stride over its pairs; the partial sums are
// combined by a fixed butterfly, so the result is the same on every run.
__global__ __launch_bounds__(256) void k_force_gather(int n_atoms, const int* __restrict__ offsets,
                                                      const int* __restrict__ rev, const double* __restrict__ gx,
                                                      const double* __restrict__ gy, const double* __restrict__ gz,
                                                      double* __restrict__ out, int accumulate_grad) {
  const int k = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int sub = threadIdx.x & 15;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (k < n_atoms) {
    for (int q = offsets[k] + sub; q < offsets[k + 1]; q += 16) {
      const int r = rev[q];
      fx += gx[q] - gx[r];
      fy += gy[q] - gy[r];
      fz += gz[q] - gz[r];
    }
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) {
    fx += __shfl_xor(fx, o, 16);
    fy += __shfl_xor(fy, o, 16);
    fz += __shfl_xor(fz, o, 16);
  }
  if (k < n_atoms && sub == 0) {
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

template <int NMAX, int LMAX>
hipError_t descriptor_impl(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, const int* nj,
                           const double* dx, const double* dy, const double* dz, const int* species, double* c,
                           double* q, double* pnorm, hipStream_t st) {
  const size_t dyn = sizeof(double) * ((size_t)P.nch * (P.LL + 1) + P.K);
  if (LMAX <= 8)
    hipLaunchKernelGGL((k_descriptor<NMAX, LMAX, 4>), dim3(n_atoms), dim3(64), dyn, st, P, T, n_atoms, offsets, nj,
                       dx, dy, dz, species, c, q, pnorm);
  else
    hipLaunchKernelGGL((k_descriptor<NMAX, LMAX, 2>), dim3(n_atoms), dim3(64), dyn, st, P, T, n_atoms, offsets, nj,
                       dx, dy, dz, species, c, q, pnorm);
  return hipGetLastError();
}

template <int NMAX, int LMAX>
hipError_t adjoint_impl(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, const int* nj,
                        const double* dx, const double* dy, const double* dz, const int* species, const double* c,
                        const double* q, const double* pnorm, const double* qbar, double* gx, double* gy, double* gz,
                        hipStream_t st) {
  const size_t dyn = sizeof(double) * (2 * (size_t)P.nch * (P.LL + 1) + P.K);
  hipLaunchKernelGGL((k_pair_adjoint<NMAX, LMAX>), dim3(n_atoms), dim3(64), dyn, st, P, T, n_atoms, offsets, nj, dx,
                     dy, dz, species, c, q, pnorm, qbar, gx, gy, gz);
  return hipGetLastError();
}

// compile-time (n_max, l_max) buckets: the kernel handles any n <= NMAX, l <= LMAX
template <typename F>
hipError_t dispatch(int n, int l, F&& f) {
  if (n <= 6 && l <= 6) return f.template operator()<6, 6>();
  if (n <= 8 && l <= 6) return f.template operator()<8, 6>();
  if (n <= 8 && l <= 8) return f.template operator()<8, 8>();
  if (n <= 10 && l <= 10) return f.template operator()<10, 10>();
  return f.template operator()<12, 12>();
}

}  // namespace

// static + dynamic LDS of one forward workgroup (static part of the (n, l) bucket used)
size_t descriptor_lds_bytes(const DevParams& P) {
  int NB = 12, LB = 12;
  if (P.n <= 6 && P.l <= 6) NB = 6, LB = 6;
  else if (P.n <= 8 && P.l <= 6) NB = 8, LB = 6;
  else if (P.n <= 8 && P.l <= 8) NB = 8, LB = 8;
  else if (P.n <= 10 && P.l <= 10) NB = 10, LB = 10;
  const size_t stat = sizeof(double) * (16 * ((LB + 1) * (LB + 1) + 1) + 16 * (NB + 1) + NB) + 64 * sizeof(int);
  return stat + sizeof(double) * ((size_t)P.nch * (P.LL + 1) + P.K);
}
size_t adjoint_lds_bytes(const DevParams& P) { return sizeof(double) * (2 * (size_t)P.nch * (P.LL + 1) + P.K); }

hipError_t launch_descriptor(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, const int* nj,
                             const double* dx, const double* dy, const double* dz, const int* species, double* c,
                             double* q, double* pnorm, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  auto f = [&]<int N, int LM>() {
    return descriptor_impl<N, LM>(P, T, n_atoms, offsets, nj, dx, dy, dz, species, c, q, pnorm, st);
  };
  return dispatch(P.n, P.l, f);
}

hipError_t launch_pair_adjoint(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets,
                               const int* nj, const double* dx, const double* dy, const double* dz,
                               const int* species, const double* c, const double* q, const double* pnorm,
                               const double* qbar, double* gx, double* gy, double* gz, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  auto f = [&]<int N, int LM>() {
    return adjoint_impl<N, LM>(P, T, n_atoms, offsets, nj, dx, dy, dz, species, c, q, pnorm, qbar, gx, gy, gz, st);
  };
  return dispatch(P.n, P.l, f);
}

hipError_t launch_force_gather(int n_atoms, const int* offsets, const int* rev, const double* gx, const double* gy,
                               const double* gz, double* out, bool accumulate_grad, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_force_gather, dim3((n_atoms + 15) / 16), dim3(256), 0, st, n_atoms, offsets, rev, gx, gy, gz,
                     out, accumulate_grad ? 1 : 0);
  return hipGetLastError();
}

}  // namespace soap
