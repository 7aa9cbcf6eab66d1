// Per-pair device arithmetic of the separable SOAP expansion (FP64).
//
// Caro 2019, arXiv:1905.02142:
//   radial overlaps        Eqs. (19), (02), (04) and the Gaussian-basis closed form (Sec. III.A)
//   buffer-zone smoothing  Sec. III.B (product of two Gaussians on [r_soft, r_hard])
//   amplitude and widths   Eq. (15)
//   ilexp                  Sec. III.C, evaluated in the numerically stable direction
//   spherical harmonics    Sec. III.C; real form, pole-free Cartesian recursion
#pragma once

#include <hip/hip_runtime.h>

namespace soap {

constexpr int kMaxN = 12;
constexpr int kMaxL = 12;
constexpr int kMaxLM = (kMaxL + 1) * (kMaxL + 2) / 2;
constexpr int kRecLanes = 16;               // lanes sharing one neighbour in the pair kernels
constexpr int kMaxRec = (kMaxLM + kRecLanes - 1) / kRecLanes;  // (l, m) records per lane
constexpr int kPolyTerms = kMaxL / 2 + 1;
// ilexp: below this z the upward l-recursion loses digits (about 1e-13 relative
// at z = 24, 6e-7 at z = 5.76); there the two highest orders come from the power
// series and the recursion runs downward, which is stable.
constexpr double kIlexpSeriesBelow = 25.0;
constexpr int kIlexpTerms = 40;  // series terms: relative tail < 1e-18 for z < 25, l <= 13

// Read-only tables built on the host at context creation.
struct DevTables {
  double W[kMaxN * kMaxN];  // W[n * kMaxN + alpha]; alpha = n_max - 1 is the Gaussian function
  double invN[kMaxN];       // 1 / N_alpha for alpha = 1..n_max-1, stored at alpha - 1
  double lw[kMaxL + 2];     // w_l: 2l+1 (Eq. (08) as printed) or 1
  // ilexp power series: ilx_rec[o][k] = 1 / ((k+1) (2l + 2k + 3)) for the order
  // l = l_max - 1 + o (o = 0, 1, 2), and ilx_idf[l] = 1 / (2l+1)!!
  double ilx_rec[3][kIlexpTerms];
  double ilx_idf[kMaxL + 3];
  // Angular records.  The real harmonics of one (l, m) are
  //   Y(l, +m) = Qbar_lm(u_z) Re (u_x + i u_y)^m,  Y(l, -m) = Qbar_lm(u_z) Im (u_x + i u_y)^m
  // with Qbar_lm = sqrt(2)^(m>0) N_lm d^m P_l/dz^m, a polynomial of degree l - m
  // and parity (l - m) mod 2: Qbar_lm(x) = x^par sum_i rec_coef[i] x^(2i).  No
  // 1/sin(theta) appears, so the poles need no special rule.  Record e of lane
  // j (16 lanes) is entry [j][e]; unused records have zero coefficients and
  // lm = -1.
  double rec_coef[kRecLanes][kMaxRec][kPolyTerms];
  int rec_lmp[kRecLanes][kMaxRec];     // l | m << 8 | par << 16
  short rec_lm[kRecLanes][kMaxRec][2];  // c index l^2+l+m (cos part) and l^2+l-m (sin part; -1 for m = 0)
};

// Scalars of the hyper-parameters, passed by value to every kernel.
struct DevParams {
  int n;        // n_max
  int l;        // l_max
  int ns;       // species
  int nch;      // ns * n
  int LL;       // (l+1)^2
  int K;        // descriptor length
  int buffer;   // r_soft < r_cut
  int l_weight;
  double rc, rs, nf;
  double inv_rc;
  double s0r, s0p, ar, ap, a;
  double cw;    // central-atom weight
};

// The per-pair tables of one (n_max, l_max) bucket, staged in LDS once per
// workgroup so that the radial transform and the ilexp series read them with
// broadcast LDS loads instead of holding them in scalar registers.
template <int NMAX, int LMAX>
struct PairTab {
  double W[NMAX][NMAX];
  double invN[NMAX];
  double lw[LMAX + 2];
  double rec[3][kIlexpTerms];
  double idf[LMAX + 3];
};

// every entry of the tables requested before any is stored, so a workgroup
// waits for memory once; the struct is read as one array of doubles
// (nthreads >= 64)
template <int NMAX, int LMAX>
__device__ inline void stage_pair_tables(const DevTables* __restrict__ T, PairTab<NMAX, LMAX>& t, int lane,
                                         int nthreads) {
  constexpr int nW = NMAX * NMAX, nI = NMAX, nL = LMAX + 2, nR = 3 * kIlexpTerms, nD = LMAX + 3;
  constexpr int total = nW + nI + nL + nR + nD;
  static_assert(sizeof(PairTab<NMAX, LMAX>) == total * sizeof(double), "PairTab is a plain array of doubles");
  constexpr int PER = (total + 63) / 64;
  double v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int y = lane + k * nthreads;
    const double* src = T->W;  // past the end: any valid address
    if (y < nW) src = T->W + (y / NMAX) * kMaxN + y % NMAX;
    else if ((y -= nW) < nI) src = T->invN + y;
    else if ((y -= nI) < nL) src = T->lw + y;
    else if ((y -= nL) < nR) src = &T->ilx_rec[0][0] + y;
    else if ((y -= nR) < nD) src = T->ilx_idf + y;
    v[k] = *src;
  }
  double* dst = reinterpret_cast<double*>(&t);
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (lane + k * nthreads < total) dst[lane + k * nthreads] = v[k];
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kSqrtPiOver2 = 1.25331413731550025121;

// erf(a) - erf(b) for a >= b without cancellation
__device__ inline double erf_diff(double a, double b) {
  if (b >= 0.0) return erfc(b) - erfc(a);
  if (a <= 0.0) return erfc(-a) - erfc(-b);
  return erf(a) - erf(b);
}

// Streams I_k = int_lo^hi (1 - t/rc)^k exp(-(t - mu)^2 / (2 s^2)) dt for
// k = 0..n+1 and adds, for the polynomial basis functions alpha = k - 2 >= 1,
//   ba[alpha - 1]  += scale I_k / N_alpha
//   dba[alpha - 1] += (dscale I_k + scale (dI_k/dmu dmu + dI_k/ds ds)) / N_alpha
// where dscale, dmu, ds are the r-derivatives of scale, mu and s.
// I_0 from erf, I_1 from the integration-by-parts identity with no k = -1 term,
// then I_{k+2} = (k+1) s^2/rc^2 I_k + (1 - mu/rc) I_{k+1} + (s^2/rc) [u^{k+1} G]_lo^hi
// (Eq. (04) multiplied through by N_alpha), u = 1 - t/rc.  The fixed-limit
// derivatives come from integrating dG/dmu = -dG/dt by parts:
//   dI_k/dmu = -[u^k G]_lo^hi - (k/rc) I_{k-1}
//   dI_k/ds  = (I_k - [u^k (t-mu) G]_lo^hi) / s - (k s/rc) dI_{k-1}/dmu
// which avoid the cancellation of ((rc-mu) I_k - rc I_{k+1}) / s^2 (about two
// digits for narrow Gaussians, before W amplifies the error).  Only the last
// two terms are kept, so the stream needs a handful of registers.
template <int NMAX, bool DERIV, typename Tab>
__device__ inline void overlap_stream(const Tab& T, int n, double lo, double hi, double mu,
                                      double s, double rc, double scale, double dscale, double dmu_dr, double ds_dr,
                                      double (&ba)[NMAX], double (&dba)[NMAX]) {
  const double s2 = s * s;
  const double is = 1.0 / (kSqrt2 * s);
  const double ah = (hi - mu) * is, al = (lo - mu) * is;
  const double gh = exp(-ah * ah), gl = exp(-al * al);
  const double uh = 1.0 - hi / rc, ul = 1.0 - lo / rc;
  const double c1 = s2 / (rc * rc), c2 = 1.0 - mu / rc, c3 = s2 / rc;
  const double th = (hi - mu) * gh, tl = (lo - mu) * gl;
  const double krc = 1.0 / rc, is_ = 1.0 / s;
  double Im2 = 0.0, Im1 = 0.0;   // I_{k-2}, I_{k-1}
  double Dm1 = 0.0;              // dI_{k-1}/dmu
  double qh = 1.0, ql = 1.0;     // u^k at the limits
  double qh1 = 1.0, ql1 = 1.0;   // u^(k-1) at the limits (k >= 1)
#pragma unroll
  for (int k = 0; k <= NMAX + 1; ++k) {
    double I;
    if (k == 0) I = s * kSqrtPiOver2 * erf_diff(ah, al);
    else I = (double)(k - 1) * c1 * Im2 + c2 * Im1 + c3 * (qh1 * gh - ql1 * gl);
    double Dmu = 0.0, Ds = 0.0;
    if (DERIV) {
      Dmu = -(qh * gh - ql * gl) - (double)k * krc * Im1;
      Ds = (I - (qh * th - ql * tl)) * is_ - (double)k * s * krc * Dm1;
    }
    if (k >= 3 && k - 2 < n) {
      const double iN = T.invN[k - 3];
      ba[k - 3] += scale * I * iN;
      if (DERIV) dba[k - 3] += (dscale * I + scale * (Dmu * dmu_dr + Ds * ds_dr)) * iN;
    }
    Im2 = Im1;
    Im1 = I;
    Dm1 = Dmu;
    qh1 = qh;
    ql1 = ql;
    qh *= uh;
    ql *= ul;
  }
}

// Overlap of exp(-(t-mu)^2/(2 s^2)) with the Gaussian basis function of Eq. (06)
// over [0, inf) in closed form, and its mu and s derivatives.
__device__ inline void gauss_basis(double mu, double s, double s0, double& B, double& dBmu, double& dBs) {
  const double ss2 = s0 * s0 + s * s, ss = sqrt(ss2);
  const double c0 = 1.3313353638003897 / sqrt(s0);  // pi^(1/4) / sqrt(sigma0)
  const double E = exp(-mu * mu / (2.0 * ss2));
  const double w = s0 * mu / (kSqrt2 * s * ss);
  const double F = 1.0 + erf(w);
  const double H = s0 * s / ss;
  B = c0 * E * H * F;
  const double dF = 1.1283791670955126 * exp(-w * w);  // 2/sqrt(pi) e^{-w^2}
  dBmu = c0 * H * (-mu / ss2 * E * F + E * dF * (s0 / (kSqrt2 * s * ss)));
  const double dss = s / ss;
  const double dE = E * (mu * mu / (ss2 * ss)) * dss;
  const double dH = s0 / ss - s0 * s / ss2 * dss;
  const double dw = -w / s - w / ss * dss;
  dBs = c0 * (dE * H * F + E * dH * F + E * H * dF * dw);
}

// Radial factor of one neighbour at distance r:
//   Bk[k] = 4 pi A(r) b_k(r), k < n_max, b = W b_alpha   (Eqs. (01), (08), (15))
// and, with DERIV, dBk[k] = d Bk[k] / dr (through mu = r, sigma_r(r) and A(r)).
template <int NMAX, bool DERIV, typename Tab>
__device__ inline void radial(const DevParams& P, const Tab& T, double r, double (&Bk)[NMAX], double (&dBk)[NMAX]) {
  const int n = P.n;
  const double s = P.s0r + P.ar * r;
  double ba[NMAX], dba[NMAX];
#pragma unroll
  for (int a = 0; a < NMAX; ++a) {
    ba[a] = 0.0;
    dba[a] = 0.0;
  }
  // [0, r_soft]: the neighbour's Gaussian itself (mu = r, width sigma_r(r))
  overlap_stream<NMAX, DERIV>(T, n, 0.0, P.rs, r, s, P.rc, 1.0, 0.0, 1.0, P.ar, ba, dba);
  if (P.buffer) {
    // f(t) G(t) on [r_soft, r_hard] = C exp(-(t - mu')^2 / (2 s'^2))
    const double D = P.rc - P.rs, d2 = D * D / (P.nf * P.nf);
    const double s2 = s * s, sp2 = 1.0 / (1.0 / s2 + 1.0 / d2), sp = sqrt(sp2);
    const double mup = sp2 * (r / s2 + P.rs / d2);
    const double C = exp(-(r - P.rs) * (r - P.rs) / (2.0 * (s2 + d2)));
    double dC = 0.0, dmup = 0.0, dsp = 0.0;
    if (DERIV) {
      const double dC_mu = -C * (r - P.rs) / (s2 + d2);
      const double dC_s = C * (r - P.rs) * (r - P.rs) * s / ((s2 + d2) * (s2 + d2));
      const double dsp_s = sp2 * sp / (s2 * s);
      const double dmup_mu = sp2 / s2;
      const double dmup_s = 2.0 * sp * dsp_s * (r / s2 + P.rs / d2) - 2.0 * sp2 * r / (s2 * s);
      dC = dC_mu + dC_s * P.ar;
      dmup = dmup_mu + dmup_s * P.ar;
      dsp = dsp_s * P.ar;
    }
    overlap_stream<NMAX, DERIV>(T, n, P.rs, P.rc, mup, sp, P.rc, C, dC, dmup, dsp, ba, dba);
  }
  {
    double B, dBmu, dBs;
    gauss_basis(r, s, P.s0r, B, dBmu, dBs);
#pragma unroll
    for (int al = 0; al < NMAX; ++al)
      if (al == n - 1) {
        ba[al] = B;
        if (DERIV) dba[al] = dBmu + dBs * P.ar;
      }
  }
  // amplitude (Eq. (15)); a = 0 means no (1+2x^3-3x^2)^a factor
  const double sr = s, sp = P.s0p + P.ap * r;
  double A = 1.0 / (sr * sp * sp), dlogA = 0.0;
  if (P.a != 0.0) {
    const double x = r / P.rc, h = 1.0 + 2.0 * x * x * x - 3.0 * x * x;
    A *= pow(h, P.a);
    dlogA = P.a * (6.0 * x * x - 6.0 * x) / (h * P.rc);
  }
  dlogA += -P.ar / sr - 2.0 * P.ap / sp;
  const double fA = 4.0 * kPi * A;
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k < n) {
      double acc = 0.0, dacc = 0.0;
#pragma unroll
      for (int al = 0; al < NMAX; ++al) {
        if (al < n) {
          const double w = T.W[k][al];
          acc = fma(w, ba[al], acc);
          if (DERIV) dacc = fma(w, dba[al], dacc);
        }
      }
      Bk[k] = fA * acc;
      if (DERIV) dBk[k] = fA * (dacc + dlogA * acc);
    }
  }
}

// e_l(z) = exp(-z) i_l(z) for l = 0..lmax (lmax <= LM), z > 0.
// Large z: the recursion e_l = e_{l-2} - (2l-1)/z e_{l-1} upward from the
// closed forms of e_0 and e_1 (Sec. III.C).  Small z, where that direction
// loses digits: the power series of the two highest orders, with tabulated
// reciprocals rec_top (order lmax) and rec_sub (order lmax - 1), then the same
// recursion downward, which is stable.
template <int LM>
__device__ inline void ilexp(double z, int lmax, const double* __restrict__ rec_top,
                             const double* __restrict__ rec_sub, const double* __restrict__ idf,
                             double (&e)[LM + 1]) {
  const double iz = 1.0 / z;
  if (lmax == 0 || z >= kIlexpSeriesBelow) {
    const double em = expm1(-2.0 * z);
    e[0] = -em * 0.5 * iz;
    if (lmax >= 1) e[1] = (z - 1.0 + (em + 1.0) * (z + 1.0)) * 0.5 * iz * iz;
#pragma unroll
    for (int l = 2; l <= LM; ++l)
      if (l <= lmax) e[l] = e[l - 2] - (double)(2 * l - 1) * iz * e[l - 1];
    return;
  }
  // i_l(z) = z^l / (2l+1)!! sum_k (z^2/2)^k / (k! (2l+3)(2l+5)..(2l+2k+1))
  const int L = lmax;
  double zl = 1.0;
  for (int j = 1; j < L; ++j) zl *= z;
  double t1 = zl * idf[L - 1];  // z^(L-1) / (2L-1)!!
  double t0 = zl * z * idf[L];  // z^L / (2L+1)!!
  const double h = 0.5 * z * z;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int k = 0; k < kIlexpTerms; ++k) {
    s0 += t0;
    s1 += t1;
    t0 *= h * rec_top[k];
    t1 *= h * rec_sub[k];
  }
  const double ez = exp(-z);
  double up = ez * s0, cur = ez * s1;  // e_L, e_{L-1}
#pragma unroll
  for (int l = LM; l >= 0; --l) {
    if (l == L) e[l] = up;
    if (l == L - 1) e[l] = cur;
  }
#pragma unroll
  for (int l = LM - 1; l >= 1; --l) {
    if (l <= L - 1) {
      const double nxt = up + (double)(2 * l + 1) * iz * cur;  // e_{l-1}
      e[l - 1] = nxt;
      up = cur;
      cur = nxt;
    }
  }
}

}  // namespace soap
