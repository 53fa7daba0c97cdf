// Host FP64 dense linear algebra for the small k x k problems of FOA-based
// DMD (k <= 512): SVD of beta for rank truncation, eigenpairs of the
// projected matrix, and the small complex solve for the mode coefficients.
// Written from textbook methods (one-sided Jacobi SVD; Householder
// Hessenberg reduction + Francis double-shift QR + quasi-triangular back
// substitution); no external LAPACK.  All matrices are column-major.
#pragma once

#include <complex>
#include <vector>

namespace hla {

using cd = std::complex<double>;

// Singular values (descending) and left singular vectors of the m x m matrix A.
// U: m x m (column j belongs to S[j]).  Returns 0 on success, -1 if the
// sweeps did not converge.
int svd_left(int m, const double *A, int lda, std::vector<double> &U, std::vector<double> &S);

// Eigenvalues and right eigenvectors of the real m x m matrix A.
// lam[i] and column i of Z (m x m complex, unit 2-norm) form a pair;
// is_real[i] is 1 for eigenvalues of 1x1 blocks of the real Schur form (their
// imaginary part is exactly 0), 0 for members of a complex-conjugate pair.
// Returns 0 on success, -1 if the QR iteration did not converge.
int eig_real(int m, const double *A, int lda, std::vector<cd> &lam, std::vector<cd> &Z,
             std::vector<int> &is_real);

// Solve the complex m x m system M x = b in place (b <- x) by LU with partial
// pivoting.  Returns 0, or -1 for an exactly singular pivot.
int solve_complex(int m, std::vector<cd> M, std::vector<cd> &b);

}  // namespace hla
