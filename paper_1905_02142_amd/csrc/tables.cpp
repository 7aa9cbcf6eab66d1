// Host tables of the radial basis (Sec. III.A "Radial expansion coefficients").
//
// The basis is phi_alpha(r) = (1 - r/r_c)^(alpha+2) / N_alpha, alpha = 1..n_max-1,
// N_alpha = sqrt(r_c / (2 alpha + 5)), plus the Gaussian phi_{n_max} of Eq. (06).
// g_n = sum_alpha W_{n alpha} phi_alpha with W = S^{-1/2} (symmetric, Loewdin) and
// S_{ab} = int_0^{r_c} phi_a phi_b dr.
//
// S becomes nearly singular as n_max grows (smallest eigenvalue ~1e-11 at
// n_max = 8, ~1e-15 at 10, ~1e-17 at 12), so W carries huge entries of
// alternating sign.  Forming S and its eigendecomposition in double precision
// would leave W wrong in the 6th digit at n_max = 8.  Here everything is done in
// IEEE binary128 (__float128, 113-bit mantissa) and only the final W is rounded.
//
// Compiled by the host compiler only (no device code).

#include <quadmath.h>

#include <cmath>
#include <cstring>

namespace {

typedef __float128 Q;

// I_k = int_0^{r_c} (1 - t/r_c)^k exp(-t^2 / (2 s^2)) dt for k = 0..kmax, by the
// integration-by-parts recursion of Eq. (04) with the neighbour at the origin:
//   I_{k+2} = (k+1) s^2/r_c^2 I_k + I_{k+1} - s^2/r_c,
// seeded by I_0 (erf) and I_1 (the same identity with the k = -1 term absent).
void origin_overlaps(Q rc, Q s, int kmax, Q* I) {
  Q s2 = s * s;
  I[0] = s * sqrtq(M_PIq / 2) * erfq(rc / (sqrtq((Q)2) * s));
  Q grc = expq(-rc * rc / (2 * s2));
  if (kmax >= 1) I[1] = (s2 / rc) * (grc - 1) + I[0];
  for (int k = 0; k + 2 <= kmax; ++k) I[k + 2] = (Q)(k + 1) * s2 / (rc * rc) * I[k] + I[k + 1] - s2 / rc;
}

// Cyclic Jacobi eigendecomposition of a symmetric n x n matrix A (destroyed):
// on return A's diagonal holds the eigenvalues and V the eigenvectors (columns).
void jacobi(int n, Q* A, Q* V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1 : 0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    Q off = 0, diag = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (i != j) off += A[i * n + j] * A[i * n + j];
        else diag += A[i * n + j] * A[i * n + j];
      }
    if (off <= diag * (Q)1e-70) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        Q apq = A[p * n + q];
        if (apq == 0) continue;
        Q theta = (A[q * n + q] - A[p * n + p]) / (2 * apq);
        Q t = (theta >= 0 ? 1 : -1) / (fabsq(theta) + sqrtq(theta * theta + 1));
        Q c = 1 / sqrtq(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          Q akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          Q apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          Q vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

}  // namespace

// Builds W (n x n, row-major, rounded to double) and, optionally, W's rounding
// remainder Wlo (W ~ W + Wlo) and the eigenvalues of S (ascending).
// Returns 0, or -1 if S is not positive definite in binary128.
extern "C" int soap_host_basis_table(int n_max, double r_cut, double sigma0_r, double* W, double* Wlo,
                                     double* eig) {
  const int n = n_max;
  if (n < 2 || n > 16) return -1;
  Q rc = r_cut, s0 = sigma0_r;
  Q S[16 * 16], V[16 * 16], I[24];
  // polynomial block in closed form: sqrt((2a+5)(2b+5)) / (a+b+5)
  for (int a = 1; a < n; ++a)
    for (int b = 1; b < n; ++b) S[(a - 1) * n + (b - 1)] = sqrtq((Q)((2 * a + 5) * (2 * b + 5))) / (Q)(a + b + 5);
  // polynomial x Gaussian: (c_g / N_a) I_{a+2}(origin, sigma0_r), c_g = sqrt(2)/(sqrt(s0) pi^(1/4))
  origin_overlaps(rc, s0, n + 1, I);
  Q cg = sqrtq((Q)2) / (sqrtq(s0) * powq(M_PIq, (Q)0.25));
  for (int a = 1; a < n; ++a) {
    Q Na = sqrtq(rc / (Q)(2 * a + 5));
    S[(a - 1) * n + (n - 1)] = S[(n - 1) * n + (a - 1)] = cg * I[a + 2] / Na;
  }
  // Gaussian x Gaussian over [0, r_c]: erf(r_c / sigma0)
  S[(n - 1) * n + (n - 1)] = erfq(rc / s0);
  Q A[16 * 16];
  std::memcpy(A, S, sizeof(Q) * n * n);
  jacobi(n, A, V);
  Q lam[16];
  for (int i = 0; i < n; ++i) {
    lam[i] = A[i * n + i];
    if (!(lam[i] > 0)) return -1;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      Q w = 0;
      for (int k = 0; k < n; ++k) w += V[i * n + k] * V[j * n + k] / sqrtq(lam[k]);
      double hi = (double)w;
      W[i * n + j] = hi;
      if (Wlo) Wlo[i * n + j] = (double)(w - (Q)hi);
    }
  if (eig) {
    double e[16];
    for (int i = 0; i < n; ++i) e[i] = (double)lam[i];
    // ascending order (insertion sort of at most 16 values)
    for (int i = 1; i < n; ++i)
      for (int k = i; k > 0 && e[k] < e[k - 1]; --k) {
        double t = e[k];
        e[k] = e[k - 1];
        e[k - 1] = t;
      }
    for (int i = 0; i < n; ++i) eig[i] = e[i];
  }
  return 0;
}

// Constants of the radial stage in double-double form (value = hi + lo to about
// 106 bits, from binary128): 1 / N_alpha = sqrt((2 alpha + 5) / r_c) for
// alpha = 1..n_max-1 (stored at alpha - 1), and rc4 = (1/r_c, remainder,
// 1/r_c^2, remainder).  Returns 0, or -1 for invalid sizes.
extern "C" int soap_host_radial_consts(int n_max, double r_cut, double* invN_hi, double* invN_lo, double* rc4) {
  if (n_max < 2 || n_max > 16 || !(r_cut > 0)) return -1;
  Q rc = r_cut;
  auto split = [](Q x, double* hi, double* lo) {
    *hi = (double)x;
    *lo = (double)(x - (Q)*hi);
  };
  for (int a = 1; a < n_max; ++a) split(sqrtq((Q)(2 * a + 5) / rc), invN_hi + a - 1, invN_lo + a - 1);
  split(1 / rc, rc4, rc4 + 1);
  split(1 / (rc * rc), rc4 + 2, rc4 + 3);
  return 0;
}
