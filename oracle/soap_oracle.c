/*
 * Oracle for the separable SOAP descriptor and its GAP energy / forces.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library.  The product path never calls
 * it, and it shares no code, header or table with the HIP library.
 *
 * Plain, slow, obviously correct.  Every per-pair and per-atom quantity is
 * computed in x87 extended precision (long double, 64-bit mantissa): the
 * polynomial radial basis is so badly conditioned (Sec. "Radial expansion
 * coefficients": S is nearly singular as n_max grows) that double precision
 * b_n would carry relative errors of 1e-11 (n_max = 8) to 1e-9 (n_max = 10),
 * too close to the 1e-10 bar the GPU path is checked against.  Building with
 * -DORACLE_REAL=double gives the double-precision variant for error studies.
 *
 * Structure of a call (Caro 2019, arXiv 1905.02142):
 *   per pair i -> j (vector d = r_j + T - r_i, r = |d|):
 *     widths / amplitude                     Eq. (15)
 *     I_k = int_lo^hi (1 - t/r_c)^k G(t) dt  integration-by-parts recursion, Eqs. (02), (04),
 *                                            erf seed for k = 0
 *     b_alpha = I_{alpha+2} / N_alpha        Eq. (19), polynomial basis phi_alpha
 *     b_{n_max}: Gaussian basis overlap      closed form below Eq. (04), auxiliary Eq. (06)
 *     b_n = sum_alpha W_{n alpha} b_alpha    orthonormalisation W = S^{-1/2}
 *     e_l(z) = exp(-z) i_l(z), z = r^2/sigma_perp^2   ("ilexp"), from the power series of i_l
 *     Y*_lm(r_hat) for m >= 0                definition with the associated Legendre functions
 *     c^j_{nlm} = 4 pi A w_l b_n e_l Y*_lm   Eq. (08); w_l = 2l+1 as printed, or 1
 *   per atom:
 *     c_nlm = sum_j c^j_nlm (+ central atom) density sum, Sec. I
 *     p_{n n' l} = sum_m c_nlm c*_{n'lm}     Eq. (09): m = 0 term + 2 Re of m > 0 terms
 *     q = p / |p|
 *   GAP: e_i = sum_s alpha_s (q_i . q_s)^zeta  (Sec. "Cohesive energy model")
 *   forces: the exact derivative of the above, by the chain rule, per pair.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_REAL
#define ORACLE_REAL long double
#endif
typedef ORACLE_REAL R;

#define PI_R 3.141592653589793238462643383279502884L
#define MAXN 16
#define MAXL 16
#define MAXK (MAXN + 8)

/* hyper-parameters; field names follow the paper's symbols */
typedef struct {
  int n_max, l_max, n_species;
  double r_cut;          /* r_hard */
  double r_soft;         /* == r_cut: no buffer zone */
  double n_f;            /* buffer filter parameter */
  double sigma0_r, sigma0_perp, alpha_r, alpha_perp, a;
  double central_weight; /* weight of the central-atom Gaussian, 0 drops it */
  int l_weight;          /* 0: w_l = 2l+1 (Eq. 08 as printed); 1: w_l = 1 */
} or_params;

static R r_exp(R x) { return (R)expl((long double)x); }
static R r_erf(R x) { return (R)erfl((long double)x); }
static R r_sqrt(R x) { return (R)sqrtl((long double)x); }
static R r_pow(R x, R y) { return (R)powl((long double)x, (long double)y); }

/* ------------------------------------------------------------------ radial */

/* Gaussian G(t) = exp(-(t - mu)^2 / (2 s^2)) */
static R gauss(R t, R mu, R s) { return r_exp(-(t - mu) * (t - mu) / (2 * s * s)); }

/*
 * I_k = int_lo^hi (1 - t/rc)^k exp(-(t-mu)^2/(2 s^2)) dt for k = 0..kmax.
 * Seed: I_0 from erf; I_1 from the same integration by parts with the k = -1
 * term absent.  Then, for k >= 0,
 *   I_{k+2} = (k+1) s^2/rc^2 I_k + (1 - mu/rc) I_{k+1} + (s^2/rc) [u^{k+1} G]_lo^hi,
 * u = 1 - t/rc, which is Eq. (04) multiplied through by N_alpha.
 */
static void overlap_integrals(R lo, R hi, R mu, R s, R rc, int kmax, R* I) {
  R s2 = s * s;
  R ulo = 1 - lo / rc, uhi = 1 - hi / rc;
  R glo = gauss(lo, mu, s), ghi = gauss(hi, mu, s);
  I[0] = s * r_sqrt(PI_R / 2) * (r_erf((hi - mu) / (r_sqrt(2) * s)) - r_erf((lo - mu) / (r_sqrt(2) * s)));
  if (kmax >= 1) I[1] = (s2 / rc) * (ghi - glo) + (1 - mu / rc) * I[0];
  R pl = ulo, ph = uhi; /* u^{k+1} at the limits, k = 0 */
  for (int k = 0; k + 2 <= kmax; ++k) {
    I[k + 2] = (R)(k + 1) * s2 / (rc * rc) * I[k] + (1 - mu / rc) * I[k + 1] + (s2 / rc) * (ph * ghi - pl * glo);
    pl *= ulo;
    ph *= uhi;
  }
}

/* d I_k / d mu and d I_k / d s with fixed limits (derivative under the integral):
 *   dI_k/dmu = ((rc - mu)/s^2) I_k - (rc/s^2) I_{k+1}
 *   dI_k/ds  = s^-3 [ (rc-mu)^2 I_k - 2 rc (rc-mu) I_{k+1} + rc^2 I_{k+2} ]
 * because (t - mu) = (rc - mu) - rc u.  Needs I up to k+2. */
static void overlap_derivs(R mu, R s, R rc, int kmax, const R* I, R* dmu, R* ds) {
  R s2 = s * s, w = rc - mu;
  for (int k = 0; k <= kmax; ++k) {
    dmu[k] = (w / s2) * I[k] - (rc / s2) * I[k + 1];
    ds[k] = (w * w * I[k] - 2 * rc * w * I[k + 1] + rc * rc * I[k + 2]) / (s2 * s);
  }
}

/*
 * Overlap of exp(-(t-mu)^2/(2 s^2)) with the auxiliary Gaussian basis function
 * phi_G(t) = sqrt(2)/(sqrt(sigma0) pi^(1/4)) exp(-t^2/(2 sigma0^2)) over [0, inf),
 * the closed form printed below Eq. (04), with its mu and s derivatives.
 */
static void gauss_basis_overlap(R mu, R s, R s0, R* B, R* dB_dmu, R* dB_ds) {
  R ss2 = s0 * s0 + s * s, ss = r_sqrt(ss2);
  R c0 = r_pow(PI_R, 0.25L) / r_sqrt(s0);
  R E = r_exp(-mu * mu / (2 * ss2));
  R w = s0 * mu / (r_sqrt(2) * s * ss);
  R F = 1 + r_erf(w);
  R H = s0 * s / ss;
  *B = c0 * E * H * F;
  /* derivatives */
  R dE_dmu = -mu / ss2 * E;
  R dw_dmu = s0 / (r_sqrt(2) * s * ss);
  R dF_dw = 2 / r_sqrt(PI_R) * r_exp(-w * w);
  *dB_dmu = c0 * H * (dE_dmu * F + E * dF_dw * dw_dmu);
  R dss_ds = s / ss;
  R dE_ds = E * (mu * mu / (ss2 * ss)) * dss_ds;
  R dH_ds = s0 / ss - s0 * s / ss2 * dss_ds;
  R dw_ds = -w / s - w / ss * dss_ds;
  *dB_ds = c0 * (dE_ds * H * F + E * dH_ds * F + E * H * dF_dw * dw_ds);
}

/*
 * b_n(r) for n = 1..n_max (returned 0-based) and d b_n / d r.
 * Both b_alpha and W b_alpha are formed in R precision; W is given as a
 * double-double (hi + lo) so that it carries more than 53 bits.
 */
static void radial(const or_params* P, const double* Whi, const double* Wlo, R r, R* bn, R* dbn) {
  int n = P->n_max;
  R rc = P->r_cut, rs = P->r_soft;
  R s = P->sigma0_r + P->alpha_r * r;
  R ds_dr = P->alpha_r;
  int kmax = n + 1;      /* b_alpha needs I_3 .. I_{n+1} */
  int kder = kmax + 2;   /* the s-derivative of I_k needs I_{k+2} */
  R I[MAXK], dImu[MAXK], dIs[MAXK];
  R J[MAXK], dJmu[MAXK], dJs[MAXK];
  overlap_integrals(0, rs, r, s, rc, kder, I);
  overlap_derivs(r, s, rc, kmax, I, dImu, dIs);
  if (rs < rc) {
    /* buffer zone [r_soft, r_hard]: f(t) G(t) is a Gaussian of mean mu', width s'
     * times the constant C (Sec. "Density smoothing at the cutoff"). */
    R D = rc - rs, d2 = D * D / ((R)P->n_f * (R)P->n_f);
    R sp2 = 1 / (1 / (s * s) + 1 / d2), sp = r_sqrt(sp2);
    R mup = sp2 * (r / (s * s) + rs / d2);
    R C = r_exp(-(r - rs) * (r - rs) / (2 * (s * s + d2)));
    overlap_integrals(rs, rc, mup, sp, rc, kder, J);
    overlap_derivs(mup, sp, rc, kmax, J, dJmu, dJs);
    /* chain rule through mu' (mu, s), s' (s) and C (mu, s) */
    R dC_dmu = -C * (r - rs) / (s * s + d2);
    R dC_ds = C * (r - rs) * (r - rs) * s / ((s * s + d2) * (s * s + d2));
    R dsp_ds = sp2 * sp / (s * s * s);
    R dmup_dmu = sp2 / (s * s);
    R dmup_ds = 2 * sp * dsp_ds * (r / (s * s) + rs / d2) - 2 * sp2 * r / (s * s * s);
    for (int k = 0; k <= kmax; ++k) {
      R v = C * J[k];
      R vmu = dC_dmu * J[k] + C * dJmu[k] * dmup_dmu;
      R vs = dC_ds * J[k] + C * (dJmu[k] * dmup_ds + dJs[k] * dsp_ds);
      I[k] += v;
      dImu[k] += vmu;
      dIs[k] += vs;
    }
  }
  R ba[MAXN], dba[MAXN];
  for (int al = 1; al <= n - 1; ++al) {
    R Na = r_sqrt(rc / (R)(2 * al + 5));
    ba[al - 1] = I[al + 2] / Na;
    dba[al - 1] = (dImu[al + 2] + dIs[al + 2] * ds_dr) / Na;
  }
  R B, dBmu, dBs;
  gauss_basis_overlap(r, s, P->sigma0_r, &B, &dBmu, &dBs);
  ba[n - 1] = B;
  dba[n - 1] = dBmu + dBs * ds_dr;
  for (int i = 0; i < n; ++i) {
    R acc = 0, dacc = 0;
    for (int al = 0; al < n; ++al) {
      R w = (R)Whi[i * n + al] + (R)Wlo[i * n + al];
      acc += w * ba[al];
      dacc += w * dba[al];
    }
    bn[i] = acc;
    if (dbn) dbn[i] = dacc;
  }
}

/* ----------------------------------------------------------------- angular */

/* e_l(z) = exp(-z) i_l(z), l = 0..lmax+1, and de_l/dz for l = 0..lmax, from the
 * power series i_l(z) = sum_k z^(l+2k) / (2^k k! (2l+2k+1)!!) and its
 * term-by-term derivative. */
static void ilexp(R z, int lmax, R* e, R* de) {
  R ez = r_exp(-z);
  for (int l = 0; l <= lmax + 1; ++l) {
    if (z == 0) {
      e[l] = (l == 0) ? 1 : 0;
      if (l <= lmax) de[l] = (l == 0) ? -1 : (l == 1 ? (R)1 / 3 : 0);
      continue;
    }
    R t = 1; /* z^l / (2l+1)!! */
    for (int j = 1; j <= l; ++j) t *= z / (R)(2 * j + 1);
    R sum = 0, dsum = 0;
    for (int k = 0; k < 100000; ++k) {
      sum += t;
      dsum += t * (R)(l + 2 * k) / z;
      R nt = t * (z * z / 2) / ((R)(k + 1) * (R)(2 * l + 2 * k + 3));
      if (k > 2 && nt < sum * 1e-24L && nt < t) break;
      t = nt;
    }
    e[l] = ez * sum;
    if (l <= lmax) de[l] = ez * (dsum - sum);
  }
}

/* m-th derivative of the Legendre polynomial P_l at x:
 *   P_l(x) = 2^-l sum_k (-1)^k (2l-2k)! / (k! (l-k)! (l-2k)!) x^(l-2k)  */
static R fact(int n) {
  /* n! for 0 <= n <= 40, tabulated on first use */
  static R table[41];
  static int ready = 0;
  if (!ready) {
#pragma omp critical(oracle_fact)
    if (!ready) {
      table[0] = 1;
      for (int i = 1; i <= 40; ++i) table[i] = table[i - 1] * i;
      __atomic_store_n(&ready, 1, __ATOMIC_RELEASE);
    }
  }
  return table[n];
}
static R legendre_deriv(int l, int m, R x) {
  if (m > l) return 0;
  R s = 0;
  for (int k = 0; 2 * k <= l - m; ++k) {
    R coef = fact(2 * l - 2 * k) / (fact(k) * fact(l - k) * fact(l - 2 * k - m));
    R term = coef;
    for (int i = 0; i < l - 2 * k - m; ++i) term *= x;
    s += (k % 2) ? -term : term;
  }
  for (int i = 0; i < l; ++i) s /= 2;
  return s;
}

/* Y*_lm(u) for a unit vector u and 0 <= m <= l, with its gradient on the sphere.
 * With P_lm(cos th) = (-1)^m sin^m th P_l^(m)(cos th) (Condon-Shortley phase, the
 * paper's P_11 = -sqrt(1 - x^2)) and sin th e^{-i phi} = u_x - i u_y:
 *   Y*_lm = N_lm (-1)^m P_l^(m)(u_z) (u_x - i u_y)^m,
 *   N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
 * grad[c] = d Y*_lm / d v_c of the same polynomial in v = (v_x, v_y, v_z). */
static void ylm_conj(int l, int m, const R* u, R* re, R* im, R* gre, R* gim) {
  R N = r_sqrt((R)(2 * l + 1) / (4 * PI_R) * fact(l - m) / fact(l + m));
  if (m % 2) N = -N;
  R pm = legendre_deriv(l, m, u[2]);
  R pm1 = legendre_deriv(l, m + 1, u[2]);
  /* (u_x - i u_y)^k for k = m and m - 1 */
  R wr = 1, wi = 0, vr = 1, vi = 0;
  for (int k = 0; k < m; ++k) {
    vr = wr; vi = wi;
    R nr = wr * u[0] + wi * u[1];
    R ni = wi * u[0] - wr * u[1];
    wr = nr; wi = ni;
  }
  *re = N * pm * wr;
  *im = N * pm * wi;
  if (gre) {
    /* d/dv_x (v_x - i v_y)^m = m (.)^(m-1); d/dv_y = -i m (.)^(m-1) */
    gre[0] = N * pm * m * vr;
    gim[0] = N * pm * m * vi;
    gre[1] = N * pm * m * vi;   /* -i (vr + i vi) = vi - i vr */
    gim[1] = -N * pm * m * vr;
    gre[2] = N * pm1 * wr;
    gim[2] = N * pm1 * wi;
  }
}

/* ---------------------------------------------------------- per-pair terms */

static R amplitude(const or_params* P, R r, R* dA) {
  R sr = P->sigma0_r + P->alpha_r * r, sp = P->sigma0_perp + P->alpha_perp * r;
  R x = r / P->r_cut;
  R h = 1 + 2 * x * x * x - 3 * x * x;
  R ha = (P->a == 0) ? 1 : r_pow(h, P->a);
  R A = ha / (sr * sp * sp);
  if (dA) {
    R dlog = -P->alpha_r / sr - 2 * P->alpha_perp / sp;
    if (P->a != 0) dlog += P->a * (6 * x * x - 6 * x) / (h * P->r_cut);
    *dA = A * dlog;
  }
  return A;
}

static R lweight(const or_params* P, int l) { return P->l_weight ? 1 : (R)(2 * l + 1); }

/* index of (l, m), 0 <= m <= l */
static int lm_index(int l, int m) { return l * (l + 1) / 2 + m; }

/* ------------------------------------------------------------ descriptor */

typedef struct {
  R* cre; /* n_ch x LM */
  R* cim;
} cbuf;

/* c_nlm of one centre atom (complex, m >= 0), including the central atom. */
static void centre_coefficients(const or_params* P, const double* Whi, const double* Wlo, int spec_i,
                                long p0, long p1, const int* pair_spec, const double* d, R* cre, R* cim) {
  int n = P->n_max, L = P->l_max;
  int LM = (L + 1) * (L + 2) / 2;
  int nch = n * P->n_species;
  memset(cre, 0, sizeof(R) * nch * LM);
  memset(cim, 0, sizeof(R) * nch * LM);
  R bn[MAXN], e[MAXL + 2], de[MAXL + 2];
  for (long p = p0; p < p1; ++p) {
    R v[3] = {d[3 * p], d[3 * p + 1], d[3 * p + 2]};
    R r = r_sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    R u[3] = {v[0] / r, v[1] / r, v[2] / r};
    R A = amplitude(P, r, NULL);
    radial(P, Whi, Wlo, r, bn, NULL);
    R sp = P->sigma0_perp + P->alpha_perp * r;
    ilexp(r * r / (sp * sp), L, e, de);
    int ch0 = pair_spec[p] * n;
    for (int l = 0; l <= L; ++l)
      for (int m = 0; m <= l; ++m) {
        R yr, yi;
        ylm_conj(l, m, u, &yr, &yi, NULL, NULL);
        R ang = 4 * PI_R * A * lweight(P, l) * e[l];
        for (int k = 0; k < n; ++k) {
          cre[(ch0 + k) * LM + lm_index(l, m)] += ang * bn[k] * yr;
          cim[(ch0 + k) * LM + lm_index(l, m)] += ang * bn[k] * yi;
        }
      }
  }
  if (P->central_weight != 0) {
    /* r_j = 0: mu = 0, sigma_r = sigma0_r, e_0 = 1, e_{l>0} = 0, Y*_00 = 1/sqrt(4 pi) */
    R A0 = amplitude(P, 0, NULL);
    radial(P, Whi, Wlo, 0, bn, NULL);
    for (int k = 0; k < n; ++k)
      cre[(spec_i * n + k) * LM] += (R)P->central_weight * 4 * PI_R * A0 * lweight(P, 0) * bn[k] / r_sqrt(4 * PI_R);
  }
}

/* p_{a b l} = c_{al0} c_{bl0} + 2 sum_{m>=1} Re(c_{alm} c*_{blm}), packed a <= b,
 * then l; off-diagonal entries scaled by sqrt(2) so that the packed dot
 * product equals the full (a, b) sum. */
static void power_spectrum(const or_params* P, const R* cre, const R* cim, R* v) {
  int n = P->n_max, L = P->l_max, nch = n * P->n_species;
  int LM = (L + 1) * (L + 2) / 2;
  int k = 0;
  for (int a = 0; a < nch; ++a)
    for (int b = a; b < nch; ++b)
      for (int l = 0; l <= L; ++l) {
        R s = cre[a * LM + lm_index(l, 0)] * cre[b * LM + lm_index(l, 0)];
        for (int m = 1; m <= l; ++m)
          s += 2 * (cre[a * LM + lm_index(l, m)] * cre[b * LM + lm_index(l, m)] +
                    cim[a * LM + lm_index(l, m)] * cim[b * LM + lm_index(l, m)]);
        v[k++] = (a == b) ? s : r_sqrt(2) * s;
      }
}

int or_descriptor_dim(const or_params* P) {
  int nch = P->n_max * P->n_species;
  return nch * (nch + 1) / 2 * (P->l_max + 1);
}

static int check_params(const or_params* P) {
  if (P->n_max < 2 || P->n_max > 12 || P->l_max < 0 || P->l_max > 12 || P->n_species < 1) return -1;
  if (!(P->r_cut > 0) || !(P->sigma0_r > 0) || !(P->sigma0_perp > 0)) return -1;
  if (P->r_soft > P->r_cut || !(P->r_soft > 0)) return -1;
  return 0;
}

/*
 * Descriptor of n_centres atoms.  Pairs of centre c are offsets[c]..offsets[c+1]-1
 * with neighbour species pair_spec[p] and vector d[3p..3p+2] = r_j + T - r_i.
 * Outputs q (n_centres x K), |p| (n_centres), and optionally c (complex, m >= 0).
 */
int or_descriptor(const or_params* P, const double* Whi, const double* Wlo, int n_centres,
                  const int* centre_spec, const long* offsets, const int* pair_spec, const double* d,
                  double* q, double* pnorm, double* c_re, double* c_im) {
  if (check_params(P)) return -1;
  int K = or_descriptor_dim(P);
  int nch = P->n_max * P->n_species;
  int LM = (P->l_max + 1) * (P->l_max + 2) / 2;
#pragma omp parallel
  {
    R* cre = malloc(sizeof(R) * nch * LM);
    R* cim = malloc(sizeof(R) * nch * LM);
    R* v = malloc(sizeof(R) * K);
#pragma omp for schedule(dynamic, 4)
    for (int c = 0; c < n_centres; ++c) {
      centre_coefficients(P, Whi, Wlo, centre_spec[c], offsets[c], offsets[c + 1], pair_spec, d, cre, cim);
      power_spectrum(P, cre, cim, v);
      R nrm = 0;
      for (int k = 0; k < K; ++k) nrm += v[k] * v[k];
      nrm = r_sqrt(nrm);
      for (int k = 0; k < K; ++k) q[(long)c * K + k] = (nrm > 0) ? (double)(v[k] / nrm) : 0.0;
      if (pnorm) pnorm[c] = (double)nrm;
      if (c_re)
        for (int i = 0; i < nch * LM; ++i) {
          c_re[(long)c * nch * LM + i] = (double)cre[i];
          c_im[(long)c * nch * LM + i] = (double)cim[i];
        }
    }
    free(cre);
    free(cim);
    free(v);
  }
  return 0;
}

/*
 * Vector-Jacobian product of the descriptor: given qbar = dE/dq (n_centres x K),
 * returns g[3p..3p+2] = dE/dd_p for every pair p, by the chain rule
 *   qbar -> vbar = (qbar - q (q . qbar)) / |v| -> pbar -> cbar -> g.
 */
int or_descriptor_vjp(const or_params* P, const double* Whi, const double* Wlo, int n_centres,
                      const int* centre_spec, const long* offsets, const int* pair_spec, const double* d,
                      const double* qbar, double* g) {
  if (check_params(P)) return -1;
  int K = or_descriptor_dim(P);
  int n = P->n_max, L = P->l_max, nch = n * P->n_species;
  int LM = (L + 1) * (L + 2) / 2;
#pragma omp parallel
  {
    R* cre = malloc(sizeof(R) * nch * LM);
    R* cim = malloc(sizeof(R) * nch * LM);
    R* gre = malloc(sizeof(R) * nch * LM); /* dE / d Re c */
    R* gim = malloc(sizeof(R) * nch * LM); /* dE / d Im c */
    R* v = malloc(sizeof(R) * K);
    R* vb = malloc(sizeof(R) * K);
#pragma omp for schedule(dynamic, 4)
    for (int c = 0; c < n_centres; ++c) {
      long p0 = offsets[c], p1 = offsets[c + 1];
      for (long p = p0; p < p1; ++p) g[3 * p] = g[3 * p + 1] = g[3 * p + 2] = 0;
      centre_coefficients(P, Whi, Wlo, centre_spec[c], p0, p1, pair_spec, d, cre, cim);
      power_spectrum(P, cre, cim, v);
      R nrm = 0;
      for (int k = 0; k < K; ++k) nrm += v[k] * v[k];
      nrm = r_sqrt(nrm);
      if (!(nrm > 0)) continue;
      /* q = v / |v| -> vbar = (qbar - q (q . qbar)) / |v| */
      R qq = 0;
      for (int k = 0; k < K; ++k) qq += (v[k] / nrm) * (R)qbar[(long)c * K + k];
      for (int k = 0; k < K; ++k) vb[k] = ((R)qbar[(long)c * K + k] - (v[k] / nrm) * qq) / nrm;
      /* packed v -> dE/dc through p_{abl} */
      memset(gre, 0, sizeof(R) * nch * LM);
      memset(gim, 0, sizeof(R) * nch * LM);
      int k = 0;
      for (int a = 0; a < nch; ++a)
        for (int b = a; b < nch; ++b)
          for (int l = 0; l <= L; ++l) {
            R pb = (a == b) ? vb[k] : r_sqrt(2) * vb[k]; /* dE/dp_{abl} */
            ++k;
            for (int m = 0; m <= l; ++m) {
              R kap = (m == 0) ? 1 : 2;
              int ia = a * LM + lm_index(l, m), ib = b * LM + lm_index(l, m);
              /* p_{abl} contains kap (Re_a Re_b + Im_a Im_b); a == b counts the square */
              gre[ia] += pb * kap * cre[ib];
              gre[ib] += pb * kap * cre[ia];
              if (m > 0) {
                gim[ia] += pb * kap * cim[ib];
                gim[ib] += pb * kap * cim[ia];
              }
            }
          }
      /* per pair: c^p = 4 pi w_l A(r) b_n(r) e_l(z(r)) Y*_lm(u), u = d / r */
      R bn[MAXN], dbn[MAXN], e[MAXL + 2], de[MAXL + 2];
      for (long p = p0; p < p1; ++p) {
        R vv[3] = {d[3 * p], d[3 * p + 1], d[3 * p + 2]};
        R r = r_sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
        R u[3] = {vv[0] / r, vv[1] / r, vv[2] / r};
        R dA;
        R A = amplitude(P, r, &dA);
        radial(P, Whi, Wlo, r, bn, dbn);
        R sp = P->sigma0_perp + P->alpha_perp * r;
        R z = r * r / (sp * sp);
        R dz = 2 * r / (sp * sp) - 2 * r * r * P->alpha_perp / (sp * sp * sp);
        ilexp(z, L, e, de);
        int ch0 = pair_spec[p] * n;
        R gr = 0;           /* coefficient of u in g (radial derivative part) */
        R gt[3] = {0, 0, 0}; /* sum of cbar R_nl grad Y (then projected) */
        for (int l = 0; l <= L; ++l)
          for (int m = 0; m <= l; ++m) {
            R yr, yi, gyr[3], gyi[3];
            ylm_conj(l, m, u, &yr, &yi, gyr, gyi);
            R w = 4 * PI_R * lweight(P, l);
            for (int kk = 0; kk < n; ++kk) {
              int idx = (ch0 + kk) * LM + lm_index(l, m);
              R Rnl = w * A * bn[kk] * e[l];
              R dRnl = w * (dA * bn[kk] * e[l] + A * dbn[kk] * e[l] + A * bn[kk] * de[l] * dz);
              gr += dRnl * (gre[idx] * yr + gim[idx] * yi);
              for (int x = 0; x < 3; ++x) gt[x] += Rnl * (gre[idx] * gyr[x] + gim[idx] * gyi[x]);
            }
          }
        /* d u / d d = (I - u u^T) / r */
        R ug = u[0] * gt[0] + u[1] * gt[1] + u[2] * gt[2];
        for (int x = 0; x < 3; ++x) g[3 * p + x] = (double)(gr * u[x] + (gt[x] - u[x] * ug) / r);
      }
    }
    free(cre);
    free(cim);
    free(gre);
    free(gim);
    free(v);
    free(vb);
  }
  return 0;
}

/*
 * GAP local energies e_i = sum_s alpha_s (q_i . q_s)^zeta and, optionally,
 * qbar_i = dE/dq_i = sum_s alpha_s zeta (q_i . q_s)^(zeta-1) q_s and
 * alpha_bar_s = dE/dalpha_s = sum_i (q_i . q_s)^zeta.
 */
void or_gap(int N, int K, const double* q, int M, const double* qs, const double* alpha, int zeta,
            double* e, double* qbar, double* alpha_bar) {
  if (alpha_bar)
    for (int s = 0; s < M; ++s) alpha_bar[s] = 0;
#pragma omp parallel
  {
    R* ab = calloc((size_t)M, sizeof(R));
    R* qb = malloc(sizeof(R) * K);
#pragma omp for schedule(static)
    for (int i = 0; i < N; ++i) {
      R ei = 0;
      for (int k = 0; k < K; ++k) qb[k] = 0;
      for (int s = 0; s < M; ++s) {
        R x = 0;
        for (int k = 0; k < K; ++k) x += (R)q[(long)i * K + k] * (R)qs[(long)s * K + k];
        R xz1 = 1;
        for (int t = 0; t < zeta - 1; ++t) xz1 *= x;
        ei += alpha[s] * xz1 * x;
        ab[s] += xz1 * x;
        if (qbar) {
          R gcoef = alpha[s] * zeta * xz1;
          for (int k = 0; k < K; ++k) qb[k] += gcoef * (R)qs[(long)s * K + k];
        }
      }
      e[i] = (double)ei;
      if (qbar)
        for (int k = 0; k < K; ++k) qbar[(long)i * K + k] = (double)qb[k];
    }
#pragma omp critical
    if (alpha_bar)
      for (int s = 0; s < M; ++s) alpha_bar[s] += (double)ab[s];
    free(ab);
    free(qb);
  }
}

/* ------------------------------------------------------------- neighbours */

/*
 * Brute-force neighbour list: for each centre i (in the given order), every
 * atom j and every lattice translation T = n_a a + n_b b + n_c c with
 * |n_x| <= ceil(r_cut / w_x) on periodic axes (w_x = cell width perpendicular
 * to the other two lattice vectors), keep 0 < |r_j + T - r_i| < r_cut.
 * Returns the number of pairs; writes at most cap of them.
 */
long or_neighbors(int n_atoms, const double* pos, const double* cell, const int* pbc, double rc,
                  int n_centres, const int* centres, long cap, long* offsets, int* pj, int* shift,
                  double* d) {
  int R_[3];
  double vol = cell[0] * (cell[4] * cell[8] - cell[5] * cell[7]) - cell[1] * (cell[3] * cell[8] - cell[5] * cell[6]) +
               cell[2] * (cell[3] * cell[7] - cell[4] * cell[6]);
  vol = fabs(vol);
  for (int a = 0; a < 3; ++a) {
    const double* u = cell + 3 * ((a + 1) % 3);
    const double* v = cell + 3 * ((a + 2) % 3);
    double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
    double w = vol / sqrt(cx * cx + cy * cy + cz * cz);
    R_[a] = pbc[a] ? (int)ceil(rc / w) : 0;
  }
  long np = 0;
  for (int c = 0; c < n_centres; ++c) {
    int i = centres[c];
    offsets[c] = np;
    for (int j = 0; j < n_atoms; ++j)
      for (int na = -R_[0]; na <= R_[0]; ++na)
        for (int nb = -R_[1]; nb <= R_[1]; ++nb)
          for (int nc = -R_[2]; nc <= R_[2]; ++nc) {
            double dv[3];
            for (int x = 0; x < 3; ++x)
              dv[x] = pos[3 * j + x] + na * cell[x] + nb * cell[3 + x] + nc * cell[6 + x] - pos[3 * i + x];
            double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
            if (r2 > 0 && r2 < rc * rc) {
              if (np < cap) {
                pj[np] = j;
                shift[3 * np] = na;
                shift[3 * np + 1] = nb;
                shift[3 * np + 2] = nc;
                d[3 * np] = dv[0];
                d[3 * np + 1] = dv[1];
                d[3 * np + 2] = dv[2];
              }
              ++np;
            }
          }
  }
  offsets[n_centres] = np;
  return np;
}

/* ---------------------------------------------- pieces exposed for pinning */

void or_overlap_integrals(double lo, double hi, double mu, double s, double rc, int kmax, double* out) {
  R I[64];
  overlap_integrals(lo, hi, mu, s, rc, kmax, I);
  for (int k = 0; k <= kmax; ++k) out[k] = (double)I[k];
}

void or_radial(const or_params* P, const double* Whi, const double* Wlo, double r, double* bn, double* dbn) {
  R b[MAXN], db[MAXN];
  radial(P, Whi, Wlo, r, b, db);
  for (int i = 0; i < P->n_max; ++i) {
    bn[i] = (double)b[i];
    if (dbn) dbn[i] = (double)db[i];
  }
}

void or_ilexp(double z, int lmax, double* e, double* de) {
  R ee[MAXL + 2], dd[MAXL + 2];
  ilexp(z, lmax, ee, dd);
  for (int l = 0; l <= lmax; ++l) {
    e[l] = (double)ee[l];
    if (de) de[l] = (double)dd[l];
  }
}

void or_ylm_conj(int l, int m, const double* u, double* re, double* im, double* gre, double* gim) {
  R uu[3] = {u[0], u[1], u[2]}, a, b, ga[3], gb[3];
  ylm_conj(l, m, uu, &a, &b, ga, gb);
  *re = (double)a;
  *im = (double)b;
  if (gre)
    for (int x = 0; x < 3; ++x) {
      gre[x] = (double)ga[x];
      gim[x] = (double)gb[x];
    }
}

void or_gauss_basis_overlap(double mu, double s, double s0, double* out3) {
  R B, a, b;
  gauss_basis_overlap(mu, s, s0, &B, &a, &b);
  out3[0] = (double)B;
  out3[1] = (double)a;
  out3[2] = (double)b;
}

double or_amplitude(const or_params* P, double r, double* dA) {
  R d;
  R A = amplitude(P, r, &d);
  if (dA) *dA = (double)d;
  return (double)A;
}

int or_real_bits(void) { return (int)(sizeof(R) == sizeof(double) ? 53 : 64); }

/* threads for the following parallel regions of this library (n >= 1) */
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* threads an OpenMP parallel region of this library uses */
int or_num_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}
