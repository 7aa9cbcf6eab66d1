// Descriptor forward and adjoint kernels (FP64 VALU).
//
// Forward, one 64-lane wavefront per centre atom i (Sec. II, Eqs. (05), (08), (09)):
//   1. per-pair phase: each lane takes one neighbour of a 64-neighbour chunk and
//      computes B_k = 4 pi A b_k (radial recursion and orthonormal transform,
//      staged in LDS) and w_l e_l (ilexp, kept in registers);
//   2. the real spherical harmonics are produced in NP passes over fixed slices
//      of the angular slots (m-major order), so only one slice of the
//      64 x L^2 angular table sits in LDS at a time;
//   3. accumulation c[k][lm] += B_k Ang_lm: lane (pg, sl) owns the channels k of
//      the slots sl, sl + SL, .. of every pass and the neighbours of pair group
//      pg, so one LDS read of a B row feeds NMAX FMAs per owned slot;
//   4. the PG partial sums are combined by DPP quad shuffles, the central atom is
//      added, c is stored (the adjoint re-reads it), and p_{ab l} =
//      sum_m c[a][lm] c[b][lm] is formed from c in LDS and normalised.
// Neighbours of species s are compacted with a wave ballot and accumulated
// together, so one register tile serves every species block.
//
// Adjoint, one wavefront per centre atom:
//   qbar -> vbar = (qbar - q (q.qbar)) / |p| -> cbar = M c (M from vbar) in LDS,
//   then one lane per neighbour recomputes B, dB/dr, e_l, de_l/dz, Y_lm and
//   grad Y_lm and contracts them with cbar into the pair gradient g = dE/dd.
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

// Writes row[slot - s0] = we[l] Y(slot) for the angular slots s0 <= slot < s1.
// Slot order: m = 0 (l = 0..lmax), then for m = 1..lmax and l = m..lmax the
// pair (l, +m), (l, -m).  Y(l, +m) = Qbar_lm(u_z) Re (u_x + i u_y)^m,
// Y(l, -m) = Qbar_lm(u_z) Im (u_x + i u_y)^m, Y(l, 0) = Qbar_l0(u_z), with
// Qbar_lm = sqrt(2)^(m>0) N_lm d^m P_l/dz^m (pole-free; see the host tables).
// recursion factors staged in LDS once per workgroup (m-major, see ym_index)
struct YTab {
  double a[kMaxLM];
  double b[kMaxLM];
  double mm[kMaxL + 2];
};

__device__ inline void stage_ytab(const DevTables* __restrict__ T, YTab& y, int lane) {
  for (int t = lane; t < kMaxLM; t += 64) {
    y.a[t] = T->ym_a[t];
    y.b[t] = T->ym_b[t];
  }
  if (lane < kMaxL + 2) y.mm[lane] = T->ymm[lane];
}

template <int LMAX>
__device__ inline void angular_slots(const YTab& Y, int lmax, double ux, double uy, double uz,
                                     const double (&we)[LMAX + 1], int s0, int s1, double* __restrict__ row) {
  double cr = 1.0, ci = 0.0;
  int g = 0;
  for (int m = 0; m <= lmax && g < s1; ++m) {
    const int cnt = (m == 0) ? lmax + 1 : 2 * (lmax - m + 1);
    if (g + cnt > s0) {
      const double* ya = Y.a + ym_index(m, m) - m;  // ya[l] = factor of (l, m)
      const double* yb = Y.b + ym_index(m, m) - m;
      double q2 = 0.0, q1 = Y.mm[m];
      int slot = g;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        if (l >= m && l <= lmax) {
          double q = q1;
          if (l > m) {
            q = ya[l] * uz * q1 - yb[l] * q2;
            q2 = q1;
            q1 = q;
          }
          const double v = we[l] * q;
          if (m == 0) {
            if (slot >= s0 && slot < s1) row[slot - s0] = v;
            slot += 1;
          } else {
            if (slot >= s0 && slot < s1) row[slot - s0] = v * cr;
            if (slot + 1 >= s0 && slot + 1 < s1) row[slot + 1 - s0] = v * ci;
            slot += 2;
          }
        }
      }
    }
    g += cnt;
    const double nr = cr * ux - ci * uy;
    ci = cr * uy + ci * ux;
    cr = nr;
  }
}

template <int NMAX, int LMAX, int PG, int NP>
struct FwdShape {
  static constexpr int LLM = (LMAX + 1) * (LMAX + 1);
  static constexpr int S = (LLM + NP - 1) / NP;  // slots per pass
  static constexpr int SL = 64 / PG;
  static constexpr int LMSP = (S + SL - 1) / SL;
  static constexpr int AST = S + 1;
  static constexpr int BST = NMAX + 1;
};

template <int NMAX, int LMAX, int PG, int NP>
__global__ __launch_bounds__(64) void k_descriptor(DevParams P, const DevTables* __restrict__ T, int n_atoms,
                                                      const int* __restrict__ offsets, const int* __restrict__ nj,
                                                      const double* __restrict__ dx, const double* __restrict__ dy,
                                                      const double* __restrict__ dz, const int* __restrict__ species,
                                                      double* __restrict__ c_out, double* __restrict__ q_out,
                                                      int q_pitch, double* __restrict__ pnorm_out) {
  using Sh = FwdShape<NMAX, LMAX, PG, NP>;
  constexpr int S = Sh::S, SL = Sh::SL, LMSP = Sh::LMSP, AST = Sh::AST, BST = Sh::BST;
  __shared__ double ang[64 * AST];
  __shared__ double bsh[64 * BST];
  __shared__ double bc[NMAX];
  __shared__ int idx[64];
  __shared__ YTab ytab;
  extern __shared__ double dyn[];

  const int i = blockIdx.x;
  if (i >= n_atoms) return;
  const int lane = threadIdx.x;
  const int pg = lane % PG, sl = lane / PG;
  stage_ytab(T, ytab, lane);
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
    double acc[NP][LMSP][NMAX];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int kk = 0; kk < LMSP; ++kk)
#pragma unroll
        for (int k = 0; k < NMAX; ++k) acc[p][kk][k] = 0.0;

    for (int w0 = p0; w0 < p1; w0 += 64) {
      const int pp = w0 + lane;
      const bool take = pp < p1 && (P.ns == 1 || species[nj[pp]] == s);
      const unsigned long long mask = __ballot(take);
      if (take) idx[__popcll(mask & ((1ull << lane) - 1ull))] = pp;
      const int cnt = __popcll(mask);
      __syncthreads();
      if (cnt == 0) continue;
      // per-pair phase: radial factors to LDS, w_l e_l in registers
      double we[LMAX + 1];
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) we[l] = 0.0;
      double ux = 0.0, uy = 0.0, uz = 1.0;
      if (lane < cnt) {
        const int q = idx[lane];
        const double x = dx[q], y = dy[q], z = dz[q];
        const double r = sqrt(x * x + y * y + z * z), ir = 1.0 / r;
        ux = x * ir;
        uy = y * ir;
        uz = z * ir;
        double B[NMAX], dB[NMAX];
        radial<NMAX, false>(P, T, r, B, dB);
#pragma unroll
        for (int k = 0; k < NMAX; ++k) bsh[lane * BST + k] = B[k];
        __builtin_amdgcn_sched_barrier(0);  // keep the radial and ilexp temporaries apart
        const double sp = P.s0p + P.ap * r;
        double e[LMAX + 1];
        ilexp<LMAX>(r * r / (sp * sp), P.l, T->ilx_rec[1], T->ilx_rec[0], T->ilx_idf, e);
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) we[l] = T->lw[l] * e[l];
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int s0 = p * S, s1 = min(s0 + S, LL);
        if (s0 < LL) {
          if (lane < cnt) angular_slots<LMAX>(ytab, P.l, ux, uy, uz, we, s0, s1, ang + lane * AST);
          __syncthreads();
          for (int t = 0; t < 64 / PG; ++t) {
            const int pi = pg + PG * t;
            if (pi >= cnt) break;
            double b[NMAX];
#pragma unroll
            for (int k = 0; k < NMAX; ++k) b[k] = bsh[pi * BST + k];
#pragma unroll
            for (int kk = 0; kk < LMSP; ++kk) {
              const int sidx = sl + SL * kk;
              if (s0 + sidx < s1) {
                const double a = ang[pi * AST + sidx];
#pragma unroll
                for (int k = 0; k < NMAX; ++k) acc[p][kk][k] = fma(a, b[k], acc[p][kk][k]);
              }
            }
          }
          __syncthreads();
        }
      }
    }
    // combine the pair groups, add the central atom, scatter c into LDS
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int kk = 0; kk < LMSP; ++kk) {
        const int slot = p * S + sl + SL * kk;
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
          double v = acc[p][kk][k];
          if (PG >= 2) v += dpp_move<kQuadXor1>(v);
          if (PG >= 4) v += dpp_move<kQuadXor2>(v);
          if (slot == 0 && s == si) v += bc[k];
          if (sl + SL * kk < S && slot < LL && k < n && (k % PG) == pg) csh[(s * n + k) * LLP + T->slot_lm[slot]] = v;
        }
      }
  }
  __syncthreads();
  for (int t = lane; t < nch * LL; t += 64) {
    const int ch = t / LL, lm = t - ch * LL;
    c_out[(size_t)i * nch * LL + t] = csh[ch * LLP + lm];
  }
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
  for (int k = lane; k < q_pitch; k += 64) q_out[(size_t)i * q_pitch + k] = k < P.K ? vsh[k] * inv : 0.0;
  if (lane == 0 && pnorm_out) pnorm_out[i] = nrm;
}

template <int NMAX, int LMAX>
__global__ __launch_bounds__(64) void k_pair_adjoint(DevParams P, const DevTables* __restrict__ T, int n_atoms,
                                                        const int* __restrict__ offsets, const int* __restrict__ nj,
                                                        const double* __restrict__ dx, const double* __restrict__ dy,
                                                        const double* __restrict__ dz,
                                                        const int* __restrict__ species, const double* __restrict__ c,
                                                        const double* __restrict__ q, int q_pitch,
                                                        const double* __restrict__ pnorm,
                                                        const double* __restrict__ qbar, int qbar_pitch,
                                                        double* __restrict__ gx, double* __restrict__ gy,
                                                        double* __restrict__ gz) {
  extern __shared__ double dyn[];
  __shared__ YTab ytab;
  const int i = blockIdx.x;
  if (i >= n_atoms) return;
  const int lane = threadIdx.x;
  const int n = P.n, LL = P.LL, nch = P.nch, K = P.K, L1 = P.l + 1;
  stage_ytab(T, ytab, lane);
  const int CP = nch + (nch & 1);  // row pitch of the lm-major tables (16-byte rows)
  double* ct = dyn;                // c[lm][ch]
  double* cbt = ct + LL * CP;      // cbar[lm][ch]
  double* vb = cbt + LL * CP;      // vbar (K)
  const int p0 = offsets[i], p1 = offsets[i + 1];

  for (int t = lane; t < nch * LL; t += 64) {
    const int ch = t / LL, lm = t - ch * LL;
    ct[lm * CP + ch] = c[(size_t)i * nch * LL + t];
  }
  // vbar = (qbar - q (q . qbar)) / |p|
  const double nrm = pnorm[i];
  double dot = 0.0;
  for (int k = lane; k < K; k += 64) dot = fma(q[(size_t)i * q_pitch + k], qbar[(size_t)i * qbar_pitch + k], dot);
  dot = wave_sum(dot);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int k = lane; k < K; k += 64)
    vb[k] = (qbar[(size_t)i * qbar_pitch + k] - q[(size_t)i * q_pitch + k] * dot) * inv;
  __syncthreads();
  // cbar[a][lm] = sum_b M_ab(l) c[b][lm]; M_aa = 2 vbar_(aa,l), M_ab = sqrt(2) vbar_(ab,l)
  for (int t = lane; t < nch * LL; t += 64) {
    const int lm = t / nch, a = t - lm * nch;
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    double s = 0.0;
    for (int b = 0; b < nch; ++b) {
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      const double w = (a == b) ? 2.0 : kSqrt2;
      s = fma(w * vb[ab_index(lo, hi, nch) * L1 + l], ct[lm * CP + b], s);
    }
    cbt[lm * CP + a] = s;
  }
  __syncthreads();
  for (int p = p0 + lane; p < p1; p += 64) {
    const double x = dx[p], y = dy[p], z = dz[p];
    const int sj = P.ns == 1 ? 0 : species[nj[p]];
    if (sj < 0 || sj >= P.ns) {  // a label outside 0..n_species-1 contributes nothing
      gx[p] = gy[p] = gz[p] = 0.0;
      continue;
    }
    const double r = sqrt(x * x + y * y + z * z), ir = 1.0 / r;
    const double ux = x * ir, uy = y * ir, uz = z * ir;
    double B[NMAX], dB[NMAX];
    radial<NMAX, true>(P, T, r, B, dB);
    __builtin_amdgcn_sched_barrier(0);  // keep the radial and ilexp temporaries apart
    const double sp = P.s0p + P.ap * r;
    const double zz = r * r / (sp * sp), izz = 1.0 / zz;
    const double dzdr = 2.0 * r / (sp * sp) - 2.0 * r * r * P.ap / (sp * sp * sp);
    double e[LMAX + 2];
    ilexp<LMAX + 1>(zz, P.l + 1, T->ilx_rec[2], T->ilx_rec[1], T->ilx_idf, e);
    double we[LMAX + 1], wd[LMAX + 1];
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
      we[l] = T->lw[l] * e[l];
      // d e_l / dz = e_{l+1} + (l/z - 1) e_l
      wd[l] = T->lw[l] * (e[l + 1] + ((double)l * izz - 1.0) * e[l]) * dzdr;
    }
    const double* base = cbt + sj * n;
    double gr = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
    double cr = 1.0, ci = 0.0, pr = 0.0, pim = 0.0;  // (u_x + i u_y)^m and ^(m-1)
    for (int m = 0; m <= P.l; ++m) {
      const double* ya = ytab.a + ym_index(m, m) - m;
      const double* yb = ytab.b + ym_index(m, m) - m;
      double q2 = 0.0, q1 = ytab.mm[m], d2 = 0.0, d1 = 0.0;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        if (l >= m && l <= P.l) {
          double qv = q1, dv = d1;
          if (l > m) {
            const double a = ya[l], b = yb[l];
            qv = a * uz * q1 - b * q2;
            dv = a * (q1 + uz * d1) - b * d2;
            q2 = q1;
            q1 = qv;
            d2 = d1;
            d1 = dv;
          }
          // the two real harmonics of (l, m): cos part at l^2+l+m, sin part at l^2+l-m
#pragma unroll
          for (int part = 0; part < 2; ++part) {
            if (part == 1 && m == 0) break;
            const int lm = l * l + l + (part == 0 ? m : -m);
            const double* cbr = base + lm * CP;
            double U = 0.0, V = 0.0;
#pragma unroll
            for (int k = 0; k < NMAX; ++k) {
              if (k < n) {
                U = fma(cbr[k], dB[k], U);
                V = fma(cbr[k], B[k], V);
              }
            }
            const double fm = (double)m;
            double Y, vx, vy, vz;
            if (part == 0) {
              Y = qv * cr;
              vx = qv * fm * pr;
              vy = -qv * fm * pim;
              vz = dv * cr;
            } else {
              Y = qv * ci;
              vx = qv * fm * pim;
              vy = qv * fm * pr;
              vz = dv * ci;
            }
            gr = fma(U * we[l] + V * wd[l], Y, gr);
            const double beta = we[l] * V;
            tx = fma(beta, vx, tx);
            ty = fma(beta, vy, ty);
            tz = fma(beta, vz, tz);
          }
        }
      }
      pr = cr;
      pim = ci;
      const double nr = cr * ux - ci * uy;
      ci = cr * uy + ci * ux;
      cr = nr;
    }
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

// compile-time (n_max, l_max) buckets: the kernels handle any n <= NMAX, l <= LMAX
struct Bucket {
  int n, l, pg, np;
};
// pg: pair groups per wave; np: angular passes (chosen so that each lane owns
// one slot of every pass: ceil((l+1)^2 / np) <= 64 / pg)
Bucket bucket_of(int n, int l) {
  if (n <= 6 && l <= 6) return {6, 6, 2, 2};
  if (n <= 8 && l <= 6) return {8, 6, 2, 2};
  if (n <= 8 && l <= 8) return {8, 8, 2, 3};
  if (n <= 10 && l <= 10) return {10, 10, 2, 4};
  return {12, 12, 2, 6};
}

template <typename F>
hipError_t dispatch(int n, int l, F&& f) {
  const Bucket b = bucket_of(n, l);
  if (b.n == 6) return f.template operator()<6, 6, 2, 2>();
  if (b.n == 8 && b.l == 6) return f.template operator()<8, 6, 2, 2>();
  if (b.n == 8) return f.template operator()<8, 8, 2, 3>();
  if (b.n == 10) return f.template operator()<10, 10, 2, 4>();
  return f.template operator()<12, 12, 2, 6>();
}

size_t fwd_dyn_bytes(const DevParams& P) { return sizeof(double) * ((size_t)P.nch * (P.LL + 1) + P.K); }
size_t adj_dyn_bytes(const DevParams& P) {
  const size_t CP = P.nch + (P.nch & 1);
  return sizeof(double) * (2 * (size_t)P.LL * CP + P.K);
}

}  // namespace

size_t descriptor_lds_bytes(const DevParams& P) {
  const Bucket b = bucket_of(P.n, P.l);
  const int LLM = (b.l + 1) * (b.l + 1), S = (LLM + b.np - 1) / b.np;
  const size_t stat = sizeof(double) * (64 * (S + 1) + 64 * (b.n + 1) + b.n) + 64 * sizeof(int) + sizeof(YTab);
  return stat + fwd_dyn_bytes(P);
}
size_t adjoint_lds_bytes(const DevParams& P) { return adj_dyn_bytes(P) + sizeof(YTab); }

hipError_t launch_descriptor(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets, const int* nj,
                             const double* dx, const double* dy, const double* dz, const int* species, double* c,
                             double* q, int q_pitch, double* pnorm, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  const size_t dyn = fwd_dyn_bytes(P);
  auto f = [&]<int N, int LM, int PG, int NP>() {
    hipLaunchKernelGGL((k_descriptor<N, LM, PG, NP>), dim3(n_atoms), dim3(64), dyn, st, P, T, n_atoms, offsets, nj,
                       dx, dy, dz, species, c, q, q_pitch, pnorm);
    return hipGetLastError();
  };
  return dispatch(P.n, P.l, f);
}

hipError_t launch_pair_adjoint(const DevParams& P, const DevTables* T, int n_atoms, const int* offsets,
                               const int* nj, const double* dx, const double* dy, const double* dz,
                               const int* species, const double* c, const double* q, int q_pitch,
                               const double* pnorm, const double* qbar, int qbar_pitch, double* gx, double* gy,
                               double* gz, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  const size_t dyn = adj_dyn_bytes(P);
  auto f = [&]<int N, int LM, int PG, int NP>() {
    hipLaunchKernelGGL((k_pair_adjoint<N, LM>), dim3(n_atoms), dim3(64), dyn, st, P, T, n_atoms, offsets, nj, dx, dy,
                       dz, species, c, q, q_pitch, pnorm, qbar, qbar_pitch, gx, gy, gz);
    return hipGetLastError();
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

void build_angular_tables(const DevParams& P, DevTables& T) {
  int slot = 0;
  for (int m = 0; m <= P.l; ++m)
    for (int l = m; l <= P.l; ++l) {
      if (m == 0) T.slot_lm[slot++] = (short)(l * l + l);
      else {
        T.slot_lm[slot++] = (short)(l * l + l + m);
        T.slot_lm[slot++] = (short)(l * l + l - m);
      }
    }
  for (int o = 0; o < 3; ++o) {
    const int l = P.l - 1 + o;
    for (int k = 0; k < kIlexpTerms; ++k) T.ilx_rec[o][k] = 1.0 / ((double)(k + 1) * (double)(2 * l + 2 * k + 3));
  }
  double df = 1.0;  // (2l+1)!!
  for (int l = 0; l < kMaxL + 3; ++l) {
    if (l > 0) df *= (double)(2 * l + 1);
    T.ilx_idf[l] = 1.0 / df;
  }
}

}  // namespace soap
