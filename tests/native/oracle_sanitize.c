/* Memory and undefined-behaviour check of the oracle's C on the host (built with
 * AddressSanitizer and UBSan by tests/test_sanitize.py; CPU only).  Runs the
 * neighbour search, descriptor, its vector-Jacobian product, the GAP sums and the
 * pinned pieces on a small random periodic box and on a buffer-zone parameter
 * set; the orthonormalisation table is the identity, which exercises the same
 * memory accesses as any other table.  Exit status 0 when every call returns. */
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int n_max, l_max, n_species;
  double r_cut, r_soft, n_f, sigma0_r, sigma0_perp, alpha_r, alpha_perp, a, central_weight;
  int l_weight;
} or_params;

int or_descriptor_dim(const or_params* P);
int or_descriptor(const or_params* P, const double* Whi, const double* Wlo, int n_centres, const int* centre_spec,
                  const long* offsets, const int* pair_spec, const double* d, double* q, double* pnorm,
                  double* c_re, double* c_im);
int or_descriptor_vjp(const or_params* P, const double* Whi, const double* Wlo, int n_centres,
                      const int* centre_spec, const long* offsets, const int* pair_spec, const double* d,
                      const double* qbar, double* g);
void or_gap(int N, int K, const double* q, int M, const double* qs, const double* alpha, int zeta, double* e,
            double* qbar, double* alpha_bar);
long or_neighbors(int n_atoms, const double* pos, const double* cell, const int* pbc, double rc, int n_centres,
                  const int* centres, long cap, long* offsets, int* pj, int* shift, double* d);
void or_radial(const or_params* P, const double* Whi, const double* Wlo, double r, double* bn, double* dbn);
void or_ilexp(double z, int lmax, double* e, double* de);
void or_ylm_conj(int l, int m, const double* u, double* re, double* im, double* gre, double* gim);

static unsigned long long rng = 88172645463325252ULL;
static double uniform(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int run(const or_params* P, int n_atoms, double box) {
  const int n = P->n_max;
  double* W = calloc((size_t)n * n, sizeof(double));
  double* Wlo = calloc((size_t)n * n, sizeof(double));
  for (int i = 0; i < n; ++i) W[i * n + i] = 1.0;
  double* pos = malloc(sizeof(double) * 3 * n_atoms);
  int* spec = malloc(sizeof(int) * n_atoms);
  int* cen = malloc(sizeof(int) * n_atoms);
  for (int i = 0; i < n_atoms; ++i) {
    for (int x = 0; x < 3; ++x) pos[3 * i + x] = box * uniform();
    spec[i] = (int)(uniform() * P->n_species);
    cen[i] = i;
  }
  double cell[9] = {box, 0, 0, 0.3, box, 0, -0.2, 0.1, box};
  int pbc[3] = {1, 1, 1};
  long* off = malloc(sizeof(long) * (n_atoms + 1));
  const long np = or_neighbors(n_atoms, pos, cell, pbc, P->r_cut, n_atoms, cen, 0, off, NULL, NULL, NULL);
  int* pj = malloc(sizeof(int) * (np + 1));
  int* sh = malloc(sizeof(int) * 3 * (np + 1));
  double* d = malloc(sizeof(double) * 3 * (np + 1));
  or_neighbors(n_atoms, pos, cell, pbc, P->r_cut, n_atoms, cen, np, off, pj, sh, d);
  int* pspec = malloc(sizeof(int) * (np + 1));
  for (long p = 0; p < np; ++p) pspec[p] = spec[pj[p]];
  const int K = or_descriptor_dim(P);
  const int LM = (P->l_max + 1) * (P->l_max + 2) / 2, nch = P->n_max * P->n_species;
  double* q = calloc((size_t)n_atoms * K, sizeof(double));
  double* pn = calloc(n_atoms, sizeof(double));
  double* cre = calloc((size_t)n_atoms * nch * LM, sizeof(double));
  double* cim = calloc((size_t)n_atoms * nch * LM, sizeof(double));
  if (or_descriptor(P, W, Wlo, n_atoms, spec, off, pspec, d, q, pn, cre, cim)) return 1;
  const int M = 7;
  double* qs = malloc(sizeof(double) * M * K);
  double* al = malloc(sizeof(double) * M);
  for (int i = 0; i < M * K; ++i) qs[i] = uniform() - 0.5;
  for (int i = 0; i < M; ++i) al[i] = uniform();
  double* e = calloc(n_atoms, sizeof(double));
  double* qbar = calloc((size_t)n_atoms * K, sizeof(double));
  double* ab = calloc(M, sizeof(double));
  or_gap(n_atoms, K, q, M, qs, al, 3, e, qbar, ab);
  double* g = calloc((size_t)3 * (np + 1), sizeof(double));
  if (or_descriptor_vjp(P, W, Wlo, n_atoms, spec, off, pspec, d, qbar, g)) return 2;
  double bn[16], dbn[16], el[32], de[32], u[3] = {0.48, -0.6, 0.64}, re, im, gre[3], gim[3];
  or_radial(P, W, Wlo, 0.5 * P->r_cut, bn, dbn);
  or_ilexp(3.0, P->l_max, el, de);
  for (int l = 0; l <= P->l_max; ++l)
    for (int m = 0; m <= l; ++m) or_ylm_conj(l, m, u, &re, &im, gre, gim);
  printf("n_max %d l_max %d species %d: %ld pairs, K %d\n", P->n_max, P->l_max, P->n_species, np, K);
  free(W); free(Wlo); free(pos); free(spec); free(cen); free(off); free(pj); free(sh); free(d); free(pspec);
  free(q); free(pn); free(cre); free(cim); free(qs); free(al); free(e); free(qbar); free(ab); free(g);
  return 0;
}

int main(void) {
  or_params a = {6, 6, 2, 3.7, 3.7, 4.0, 0.5, 0.5, 0.0, 0.0, 0.0, 1.0, 0};
  or_params b = {12, 12, 1, 4.3, 3.8, 4.0, 0.12, 0.55, 0.14, 0.06, 1.6, 0.0, 1};
  if (run(&a, 24, 7.0)) return 1;
  if (run(&b, 10, 6.0)) return 1;
  return 0;
}
