// Test-only C shim over the host linear algebra of the library.
#include <complex>
#include <vector>

#include "hostla.h"

extern "C" int shim_eig(int m, const double *A, double *lre, double *lim, double *zre, double *zim, int *isreal) {
  std::vector<std::complex<double>> lam, Z;
  std::vector<int> r;
  const int rc = hla::eig_real(m, A, m, lam, Z, r);
  if (rc) return rc;
  for (int i = 0; i < m; ++i) {
    lre[i] = lam[i].real();
    lim[i] = lam[i].imag();
    isreal[i] = r[i];
  }
  for (size_t i = 0; i < Z.size(); ++i) {
    zre[i] = Z[i].real();
    zim[i] = Z[i].imag();
  }
  return 0;
}

extern "C" int shim_svd(int m, const double *A, double *U, double *S) {
  std::vector<double> u, s;
  const int rc = hla::svd_left(m, A, m, u, s);
  if (rc) return rc;
  for (size_t i = 0; i < u.size(); ++i) U[i] = u[i];
  for (int i = 0; i < m; ++i) S[i] = s[i];
  return 0;
}

extern "C" int shim_solve(int m, const double *Mre, const double *Mim, double *bre, double *bim) {
  std::vector<std::complex<double>> M((size_t)m * m), b(m);
  for (size_t i = 0; i < M.size(); ++i) M[i] = {Mre[i], Mim[i]};
  for (int i = 0; i < m; ++i) b[i] = {bre[i], bim[i]};
  const int rc = hla::solve_complex(m, M, b);
  for (int i = 0; i < m; ++i) {
    bre[i] = b[i].real();
    bim[i] = b[i].imag();
  }
  return rc;
}
