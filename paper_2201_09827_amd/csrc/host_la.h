// Small dense linear algebra on the host (float64), for the per-cycle
// problems of GMRES / GCRO-DR: Givens least squares, thin QR, Cholesky,
// and the harmonic Ritz eigenproblem.  All matrices are column-major.
#pragma once

#include <complex>
#include <vector>

namespace gir {
namespace la {

// y minimising ||beta e1 - Hbar y||_2 for the (j+1) x j upper Hessenberg Hbar
// (leading dimension ldh), by Givens rotations; returns the residual norm.
double givens_lsq(const double* H, int ldh, int j, double beta, double* y);

// Householder thin QR of the m x k matrix A (m >= k): Q (m x k), R (k x k,
// upper) with a non-negative diagonal.  Returns false if A is rank deficient
// (a zero diagonal entry of R).
bool qr_thin(const double* A, int lda, int m, int k, double* Q, double* R);

// upper Cholesky factor R of the symmetric positive definite k x k G
// (G = R^T R); false if a pivot is not positive.
bool cholesky_upper(const double* G, int k, double* R);

// inverse of the k x k upper triangular R (in place allowed)
void inv_upper(const double* R, int k, double* Rinv);

// eigenvalues and (unit) eigenvectors of a real N x N matrix: complex Schur
// form by Hessenberg reduction and shifted QR, then back substitution.
bool eig_real(const double* A, int N, std::vector<std::complex<double>>& w,
              std::vector<std::complex<double>>& V);

// Harmonic Ritz vectors of GCRO-DR: the eigenvectors of
// G^T G z = theta G^T M z (G, M rows x cols) for the k values of smallest
// |theta|.  Solved as the standard problem R^-T (G^T M) R^-1 w = (1/theta) w
// with G = Q R.  Infinite theta come last; a complex pair contributes
// (Re z, Im z) or is dropped whole when it does not fit.  P (cols x kout,
// column-major) receives the real basis; returns kout (0 on failure).
int harmonic_ritz(const double* G, const double* M, int rows, int cols, int k, double* P);

}  // namespace la
}  // namespace gir
