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

#include <type_traits>

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
  // double-double parts for the radial stage in extended precision: W = W + Wl and
  // 1 / N_alpha = invN + invNl to about 106 bits; rcinv = (1/rc, its remainder,
  // 1/rc^2, its remainder)
  double Wl[kMaxN * kMaxN];
  double invNl[kMaxN];
  double rcinv[4];
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
  int radial_dd;  // radial recursion and W b in double-double arithmetic
  int ps_mfma;    // power spectrum and its adjoint on the matrix cores (BF16 operands, FP32 accumulation)
  double rc, rs, nf;
  double inv_rc;
  double s0r, s0p, ar, ap, a;
  double cw;    // central-atom weight
  // the adjoint's partial rounds give each pair R = 2, 4, 8 lanes; lane sub takes
  // the degrees l set in tail_deg[log2 R - 1][sub], the records of 0..l_max dealt
  // out longest first to the least loaded lane
  unsigned short tail_deg[3][8];
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
  double Wl[NMAX][NMAX];
  double invNl[NMAX];
  double rcinv[4];
};

// every entry of the tables requested before any is stored, so a workgroup
// waits for memory once; the struct is read as one array of doubles
// (nthreads >= 64)
template <int NMAX, int LMAX>
__device__ inline void stage_pair_tables(const DevTables* __restrict__ T, PairTab<NMAX, LMAX>& t, int lane,
                                         int nthreads) {
  constexpr int nW = NMAX * NMAX, nI = NMAX, nL = LMAX + 2, nR = 3 * kIlexpTerms, nD = LMAX + 3;
  constexpr int total = 2 * nW + 2 * nI + nL + nR + nD + 4;
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
    else if ((y -= nD) < nW) src = T->Wl + (y / NMAX) * kMaxN + y % NMAX;
    else if ((y -= nW) < nI) src = T->invNl + y;
    else if ((y -= nI) < 4) src = T->rcinv + y;
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
__host__ __device__ inline double erf_diff(double a, double b) {
  if (b >= 0.0) return erfc(b) - erfc(a);
  if (a <= 0.0) return erfc(-a) - erfc(-b);
  return erf(a) - erf(b);
}

// ------------------------------------------------------------ double-double
// A value hi + lo with |lo| <= ulp(hi) / 2, about 106 significant bits, built
// from the error-free transformations of FP64 sums (Knuth's TwoSum) and
// products (the FMA leaves the product's rounding error exactly).  These rely on
// every sum and product being rounded exactly as written, so floating-point
// contraction is off inside them: fusing the product a*b of TwoProd into the
// sum of a following FastTwoSum (which the AMDGPU backend does once they are
// inlined) counts the product's rounding error twice and leaves a result no
// better than plain FP64.
struct dd {
  double hi, lo;
};

// a + b exactly
__host__ __device__ inline dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
// a + b exactly, for |a| >= |b| (or a = 0)
__host__ __device__ inline dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return {s, b - (s - a)};
}
// a b exactly
__host__ __device__ inline dd two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
// a + b with an error below 2^-104 (|a| + |b|)
__host__ __device__ inline dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return fast_two_sum(s.hi, s.lo);
}
__host__ __device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__host__ __device__ inline dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b.hi);
  p.lo = fma(a.hi, b.lo, fma(a.lo, b.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}
__host__ __device__ inline dd dd_mul_d(dd a, double b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b);
  p.lo = fma(a.lo, b, p.lo);
  return fast_two_sum(p.hi, p.lo);
}
// 1 / a: the residual 1 - q a of the rounded quotient q is exact
__host__ __device__ inline dd dd_recip(double a) {
#pragma clang fp contract(off)
  const double q = 1.0 / a;
  const double r = fma(-q, a, 1.0);
  return fast_two_sum(q, r * q);
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
__host__ __device__ inline void overlap_stream(const Tab& T, int n, double lo, double hi, double mu,
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

// overlap_stream with the recursion, its derivatives and the sums into b_alpha
// carried in double-double arithmetic.  The seeds (erf and the Gaussians at the
// limits) stay FP64: their rounding moves b_n = W b_alpha by about an FP64 ulp,
// whereas every rounding inside the recursion is multiplied by the entries of
// W (up to ~5e6 at n_max = 10, ~2e8 at 12; the overlap matrix of the basis is
// nearly singular, Sec. III.A).  The limit factors u = 1 - t/rc and the
// coefficients s^2/rc^2, 1 - mu/rc, s^2/rc are formed from 1/rc in
// double-double, so the recursion is that of one consistent (mu, s, rc).
template <int NMAX, bool DERIV, typename Tab>
__host__ __device__ inline void overlap_stream_dd(const Tab& T, int n, double lo, double hi, double mu, double s,
                                         double scale, double dscale, double dmu_dr, double ds_dr,
                                         dd (&ba)[NMAX], dd (&dba)[NMAX]) {
#pragma clang fp contract(off)
  const dd irc{T.rcinv[0], T.rcinv[1]}, irc2{T.rcinv[2], T.rcinv[3]};
  const dd one{1.0, 0.0};
  const double is = 1.0 / (kSqrt2 * s);
  const double ah = (hi - mu) * is, al = (lo - mu) * is;
  const double gh = exp(-ah * ah), gl = exp(-al * al);
  const dd I0{s * kSqrtPiOver2 * erf_diff(ah, al), 0.0};
  const dd uh = dd_sub(one, dd_mul_d(irc, hi)), ul = dd_sub(one, dd_mul_d(irc, lo));
  const dd s2 = two_prod(s, s);
  const dd c1 = dd_mul(s2, irc2), c2 = dd_sub(one, dd_mul_d(irc, mu)), c3 = dd_mul(s2, irc);
  // the s-derivative is needed only when the width depends on r
  const bool wide = DERIV && ds_dr != 0.0;
  dd th{0.0, 0.0}, tl{0.0, 0.0}, is_{0.0, 0.0};
  if (wide) {
    th = dd_mul_d(two_sum(hi, -mu), gh);
    tl = dd_mul_d(two_sum(lo, -mu), gl);
    is_ = dd_recip(s);
  }
  dd Im2{0.0, 0.0}, Im1{0.0, 0.0}, Dm1{0.0, 0.0};
  dd qh = one, ql = one, qh1 = one, ql1 = one;
#pragma unroll
  for (int k = 0; k <= NMAX + 1; ++k) {
    dd I = I0;
    if (k > 0) {
      const dd bnd = dd_sub(dd_mul_d(qh1, gh), dd_mul_d(ql1, gl));
      I = dd_add(dd_add(dd_mul(dd_mul_d(c1, (double)(k - 1)), Im2), dd_mul(c2, Im1)), dd_mul(c3, bnd));
    }
    dd Dmu{0.0, 0.0}, Ds{0.0, 0.0};
    if (DERIV) {
      const dd kr = dd_mul_d(irc, (double)k);
      Dmu = dd_neg(dd_add(dd_sub(dd_mul_d(qh, gh), dd_mul_d(ql, gl)), dd_mul(kr, Im1)));
      if (wide)
        Ds = dd_sub(dd_mul(dd_sub(I, dd_sub(dd_mul(qh, th), dd_mul(ql, tl))), is_), dd_mul(dd_mul_d(kr, s), Dm1));
    }
    if (k >= 3 && k - 2 < n) {
      const dd iN{T.invN[k - 3], T.invNl[k - 3]};
      ba[k - 3] = dd_add(ba[k - 3], dd_mul(dd_mul_d(I, scale), iN));
      if (DERIV) {
        dd t = dd_mul_d(Dmu, dmu_dr);
        if (wide) t = dd_add(t, dd_mul_d(Ds, ds_dr));
        t = dd_add(dd_mul_d(I, dscale), dd_mul_d(t, scale));
        dba[k - 3] = dd_add(dba[k - 3], dd_mul(t, iN));
      }
    }
    Im2 = Im1;
    Im1 = I;
    Dm1 = Dmu;
    qh1 = qh;
    ql1 = ql;
    qh = dd_mul(qh, uh);
    ql = dd_mul(ql, ul);
  }
}

// Overlap of exp(-(t-mu)^2/(2 s^2)) with the Gaussian basis function of Eq. (06)
// over [0, inf) in closed form, and its mu and s derivatives.
__host__ __device__ inline void gauss_basis(double mu, double s, double s0, double& B, double& dBmu, double& dBs) {
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
// DD: b_alpha and W b_alpha in double-double (overlap_stream_dd), W b_alpha as a
// compensated dot product with W = W + Wl, rounded once to FP64.
template <int NMAX, bool DERIV, bool DD, typename Tab>
__host__ __device__ inline void radial(const DevParams& P, const Tab& T, double r, double (&Bk)[NMAX], double (&dBk)[NMAX]) {
  using A_t = typename std::conditional<DD, dd, double>::type;
  const int n = P.n;
  const double s = P.s0r + P.ar * r;
  A_t ba[NMAX], dba[NMAX];
#pragma unroll
  for (int a = 0; a < NMAX; ++a) {
    ba[a] = A_t{};
    dba[a] = A_t{};
  }
  // [0, r_soft]: the neighbour's Gaussian itself (mu = r, width sigma_r(r))
  if constexpr (DD) overlap_stream_dd<NMAX, DERIV>(T, n, 0.0, P.rs, r, s, 1.0, 0.0, 1.0, P.ar, ba, dba);
  else overlap_stream<NMAX, DERIV>(T, n, 0.0, P.rs, r, s, P.rc, 1.0, 0.0, 1.0, P.ar, ba, dba);
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
    if constexpr (DD) overlap_stream_dd<NMAX, DERIV>(T, n, P.rs, P.rc, mup, sp, C, dC, dmup, dsp, ba, dba);
    else overlap_stream<NMAX, DERIV>(T, n, P.rs, P.rc, mup, sp, P.rc, C, dC, dmup, dsp, ba, dba);
  }
  {
    // the Gaussian function's column of W is small (below ~1e3), so its FP64
    // closed form suffices in both arithmetics
    double B, dBmu, dBs;
    gauss_basis(r, s, P.s0r, B, dBmu, dBs);
#pragma unroll
    for (int al = 0; al < NMAX; ++al)
      if (al == n - 1) {
        ba[al] = A_t{B};
        if (DERIV) dba[al] = A_t{dBmu + dBs * P.ar};
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
      if constexpr (DD) {
        // compensated dot products (the sum of the exact products kept as an
        // unevaluated hi + lo, in the manner of Ogita, Rump and Oishi's Dot2)
#pragma clang fp contract(off)
        double c = 0.0, dc = 0.0;
#pragma unroll
        for (int al = 0; al < NMAX; ++al) {
          if (al < n) {
            const double wh = T.W[k][al], wl = T.Wl[k][al];
            const dd p = two_prod(wh, ba[al].hi), t = two_sum(acc, p.hi);
            acc = t.hi;
            c = fma(wh, ba[al].lo, fma(wl, ba[al].hi, c + (t.lo + p.lo)));
            if (DERIV) {
              const dd dp = two_prod(wh, dba[al].hi), dt = two_sum(dacc, dp.hi);
              dacc = dt.hi;
              dc = fma(wh, dba[al].lo, fma(wl, dba[al].hi, dc + (dt.lo + dp.lo)));
            }
          }
        }
        acc += c;
        dacc += dc;
      } else {
#pragma unroll
        for (int al = 0; al < NMAX; ++al) {
          if (al < n) {
            const double w = T.W[k][al];
            acc = fma(w, ba[al], acc);
            if (DERIV) dacc = fma(w, dba[al], dacc);
          }
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
