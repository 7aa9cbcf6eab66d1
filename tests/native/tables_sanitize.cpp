// Memory and undefined-behaviour check of the library's host table builder
// (paper_1905_02142_amd/csrc/tables.cpp: the radial basis table in binary128 and
// the double-double constants), built with AddressSanitizer and UBSan by
// tests/test_sanitize.py; CPU only.  Every n_max the library accepts, two
// cutoffs and widths.  Exit status 0 when every table is built.
#include <cmath>
#include <cstdio>
#include <initializer_list>

extern "C" int soap_host_basis_table(int n_max, double r_cut, double sigma0_r, double* W, double* Wlo, double* eig);
extern "C" int soap_host_radial_consts(int n_max, double r_cut, double* invN_hi, double* invN_lo, double* rc4);

int main() {
  for (int n = 2; n <= 12; ++n)
    for (double rc : {3.7, 5.5})
      for (double s0 : {0.12, 0.5}) {
        double W[16 * 16], Wl[16 * 16], eig[16], iN[16], iNl[16], rc4[4];
        if (soap_host_basis_table(n, rc, s0, W, Wl, eig) != 0) return 1;
        if (soap_host_radial_consts(n, rc, iN, iNl, rc4) != 0) return 2;
        for (int i = 0; i < n * n; ++i)
          if (!std::isfinite(W[i]) || !std::isfinite(Wl[i])) return 3;
      }
  // sizes the builders refuse
  double W[16 * 16], iN[16], iNl[16], rc4[4];
  if (soap_host_basis_table(1, 5.0, 0.5, W, nullptr, nullptr) == 0) return 4;
  if (soap_host_radial_consts(17, 5.0, iN, iNl, rc4) == 0) return 5;
  std::printf("tables: n_max 2..12 built\n");
  return 0;
}
