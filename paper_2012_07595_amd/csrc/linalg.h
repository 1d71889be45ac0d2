// Small dense FP64 linear algebra on the host for the projected problem
// (Algorithm 5 step (i)) and the small factors of the block
// orthogonalisation.  Matrices are row-major unless stated.
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace bks {
namespace la {

using Mat = std::vector<double>;

// Symmetric eigendecomposition A = V diag(w) V^T (A n x n row-major, only
// read).  Eigenvalues in descending order; V(:, i) is column i of the
// row-major V.  Householder tridiagonalisation + implicit QL.
void sym_eig(int n, const double *A, double *w, double *V);
// The same by cyclic Jacobi rotations: slower, unconditionally convergent;
// sym_eig falls back to it if the QL iteration stalls.
void sym_eig_jacobi(int n, const double *A, double *w, double *V);

// Leading r eigenvectors (descending eigenvalues) as an n x r row-major
// matrix.  From order 24, with r <= n / 2: Householder reduction, the
// eigenvalues alone by the QL iteration, the r vectors by inverse iteration
// on the tridiagonal and back through the reflectors, accepted when the
// residuals and orthonormality are within 64 n eps (else sym_eig).
void top_eigvecs(int n, const double *A, int r, double *Vr, double *wr = nullptr);

// Cholesky A = U^T U in place (row-major: U in the upper triangle, the
// strict lower triangle set to zero; U^T = L of A = L L^T).  false if A is
// not numerically positive definite (then *fail_pivot, if given, is the
// offending Schur-complement diagonal).
bool cholesky(int n, double *A, double *fail_pivot = nullptr);
// Solve U^T U x = b in place (U from cholesky).
void chol_solve(int n, const double *U, double *b);

// Householder QR of an m x n (m >= n) row-major matrix: returns the full
// m x m orthogonal Q (row-major) whose first n columns span the columns.
void qr_full(int m, int n, const double *A, double *Q);
// Thin orthonormalisation (first n columns of qr_full).
void orthonormalize(int m, int n, double *A);

// Host threads for the parallel loops and products below, per calling
// thread (0: the default, BKS_HOST_THREADS or the hardware concurrency, at
// most 8; 1: no threads).  Results never depend on it: every output element
// is computed by one thread, in a fixed order.
void set_threads(int n);
int threads();
// fn(i) for every i in [0, n), split over threads() threads.
void parallel_for(int n, const std::function<void(int)> &fn);

// C (m x n, ldc) = alpha op(A) op(B) + beta C (beta = 0: C is not read).
// op(A) is m x k: A row-major with leading dimension lda, or A^T if ta;
// op(B) k x n likewise.  Register-blocked (4 x 8, AVX2 FMA); `parallel`
// spreads the output panels over threads().
void dgemm(bool ta, bool tb, int m, int n, int k, double alpha, const double *A, int lda,
           const double *B, int ldb, double beta, double *C, int ldc, bool parallel = false);

// C (m x n) = A (m x k) * B (k x n), all row-major.
void gemm(int m, int n, int k, const double *A, const double *B, double *C);
// C (m x n) = A^T (A: k x m) * B (k x n)
void gemm_tn(int m, int n, int k, const double *A, const double *B, double *C);

}  // namespace la
}  // namespace bks
