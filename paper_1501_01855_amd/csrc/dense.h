// Small dense complex linear algebra on the host (n up to a few hundred):
// the Rayleigh-Ritz problems of the eigensolvers and of eigSUMR.
// Matrices are row-major std::complex<double>, A[i*n + j].
#pragma once
#include <complex>
#include <vector>

namespace ovl {
namespace dense {

using zc = std::complex<double>;

// Hermitian eigenproblem by cyclic complex Jacobi rotations.  On return
// evals ascend and column k of V (V[i*n + k]) is the k-th eigenvector.
void eigh(int n, const std::vector<zc> &A, std::vector<double> &evals, std::vector<zc> &V);

// Cholesky factor of a Hermitian positive-definite matrix: A = R^H R, R upper
// triangular.  Returns false if A is not numerically positive definite.
bool cholesky_upper(int n, const std::vector<zc> &A, std::vector<zc> &R);

// Inverse of an upper-triangular matrix.
std::vector<zc> inv_upper(int n, const std::vector<zc> &R);

// C = A B (m x k times k x n).
std::vector<zc> matmul(int m, int k, int n, const std::vector<zc> &A, const std::vector<zc> &B);

// C = A^H B (A: k x m, B: k x n) -> m x n.
std::vector<zc> matmul_ah(int k, int m, int n, const std::vector<zc> &A, const std::vector<zc> &B);

}  // namespace dense
}  // namespace ovl
