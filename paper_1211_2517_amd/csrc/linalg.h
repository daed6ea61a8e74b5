// Dense FP64 linear algebra for the plan-time operator precompute (host only).
#pragma once
#include <cstdint>
#include <vector>

namespace kifmm {

// One-sided (Hestenes) Jacobi SVD of a square or tall matrix A (m x n, m >= n,
// row-major). On return s holds the n singular values in descending order,
// U (m x n, row-major) the left and V (n x n, row-major) the right singular
// vectors, A = U diag(s) V^T. Columns of U for zero singular values are zero.
void svd_jacobi(int m, int n, const double* A, std::vector<double>& s, std::vector<double>& U,
                std::vector<double>& V);

// Singular values (descending) and left singular vectors (rows x rows,
// row-major, column i = vector i) of a wide matrix W (rows x cols, cols >= rows,
// row-major): Householder QR of W^T = Q R, then Jacobi SVD of R^T, whose left
// singular vectors are those of W.
void svd_wide_left(int rows, int64_t cols, const double* W, std::vector<double>& s,
                   std::vector<double>& U);

// Truncated-SVD pseudo-inverse of a square n x n matrix (row-major): singular
// values below rcond * s_max are dropped.
std::vector<double> pinv(int n, const double* A, double rcond);

// C = A B with A (m x k) and B (k x n), all row-major.
std::vector<double> matmul(int m, int k, int n, const double* A, const double* B);
// C = A^T B with A (k x m) and B (k x n), all row-major.
std::vector<double> matmul_tn(int m, int k, int n, const double* A, const double* B);

}  // namespace kifmm
