// Dense FP64 linear algebra for the plan-time operator precompute (host only).
#include "linalg.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace kifmm {

namespace {

// One-sided Jacobi on the columns of a column-major m x n matrix `a`,
// accumulating the rotations in the column-major n x n matrix `v`.
void jacobi_columns(int m, int n, std::vector<double>& a, std::vector<double>& v) {
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    const double tol = 1e-15;
    for (int sweep = 0; sweep < 80; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n - 1; ++p) {
            double* ap = &a[(size_t)p * m];
            for (int q = p + 1; q < n; ++q) {
                double* aq = &a[(size_t)q * m];
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int i = 0; i < m; ++i) {
                    alpha += ap[i] * ap[i];
                    beta += aq[i] * aq[i];
                    gamma += ap[i] * aq[i];
                }
                if (alpha == 0.0 || beta == 0.0) continue;
                double c = std::fabs(gamma) / std::sqrt(alpha * beta);
                if (!(c > tol)) continue;
                off = std::max(off, c);
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / std::sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int i = 0; i < m; ++i) {
                    double x = ap[i], y = aq[i];
                    ap[i] = cs * x - sn * y;
                    aq[i] = sn * x + cs * y;
                }
                double* vp = &v[(size_t)p * n];
                double* vq = &v[(size_t)q * n];
                for (int i = 0; i < n; ++i) {
                    double x = vp[i], y = vq[i];
                    vp[i] = cs * x - sn * y;
                    vq[i] = sn * x + cs * y;
                }
            }
        }
        if (off <= tol) break;
    }
}

}  // namespace

void svd_jacobi(int m, int n, const double* A, std::vector<double>& s, std::vector<double>& U,
                std::vector<double>& V) {
    std::vector<double> a((size_t)m * n);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) a[(size_t)j * m + i] = A[(size_t)i * n + j];
    std::vector<double> v;
    jacobi_columns(m, n, a, v);
    std::vector<double> norms(n);
    for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += a[(size_t)j * m + i] * a[(size_t)j * m + i];
        norms[j] = std::sqrt(acc);
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return norms[x] > norms[y]; });
    s.assign(n, 0.0);
    U.assign((size_t)m * n, 0.0);
    V.assign((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        int j = order[c];
        s[c] = norms[j];
        for (int i = 0; i < m; ++i) U[(size_t)i * n + c] = norms[j] > 0 ? a[(size_t)j * m + i] / norms[j] : 0.0;
        for (int i = 0; i < n; ++i) V[(size_t)i * n + c] = v[(size_t)j * n + i];
    }
}

void svd_wide_left(int rows, int64_t cols, const double* W, std::vector<double>& s,
                   std::vector<double>& U) {
    const int n = rows;
    const int64_t m = cols;
    // B = W^T stored column-major: column c of B is row c of W (contiguous).
    std::vector<double> B(W, W + (size_t)m * n);
    std::vector<double> R((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double* bj = &B[(size_t)j * m];
        double norm2 = 0.0;
        for (int64_t i = j; i < m; ++i) norm2 += bj[i] * bj[i];
        double norm = std::sqrt(norm2);
        double alpha = bj[j] >= 0 ? -norm : norm;
        if (norm == 0.0) {
            R[(size_t)j * n + j] = 0.0;
            continue;
        }
        // v = x - alpha e1 stored in place of column j (rows j..m-1);
        // v^T v = 2 |x| (|x| + |x0|) since alpha = -sign(x0) |x|.
        const double x0 = bj[j];
        bj[j] -= alpha;
        const double vtv = 2.0 * norm * (norm + std::fabs(x0));
        const double beta = vtv > 0 ? 2.0 / vtv : 0.0;
#pragma omp parallel for schedule(dynamic, 4)
        for (int c = j + 1; c < n; ++c) {
            double* bc = &B[(size_t)c * m];
            double w = 0.0;
            for (int64_t i = j; i < m; ++i) w += bj[i] * bc[i];
            w *= beta;
            for (int64_t i = j; i < m; ++i) bc[i] -= w * bj[i];
        }
        R[(size_t)j * n + j] = alpha;
        for (int c = j + 1; c < n; ++c) R[(size_t)j * n + c] = B[(size_t)c * m + j];
    }
    // W = R^T Q^T: left singular vectors of W are those of R^T (n x n).
    std::vector<double> Rt((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Rt[(size_t)i * n + j] = R[(size_t)j * n + i];
    std::vector<double> V;
    svd_jacobi(n, n, Rt.data(), s, U, V);
}

std::vector<double> pinv(int n, const double* A, double rcond) {
    std::vector<double> s, U, V;
    svd_jacobi(n, n, A, s, U, V);
    const double cut = rcond * (s.empty() ? 0.0 : s[0]);
    std::vector<double> P((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        if (!(s[c] > cut) || s[c] == 0.0) continue;
        const double inv = 1.0 / s[c];
        for (int i = 0; i < n; ++i) {
            const double vi = V[(size_t)i * n + c] * inv;
            double* Pi = &P[(size_t)i * n];
            for (int j = 0; j < n; ++j) Pi[j] += vi * U[(size_t)j * n + c];
        }
    }
    return P;
}

std::vector<double> matmul(int m, int k, int n, const double* A, const double* B) {
    std::vector<double> C((size_t)m * n, 0.0);
    for (int i = 0; i < m; ++i) {
        double* Ci = &C[(size_t)i * n];
        for (int l = 0; l < k; ++l) {
            const double a = A[(size_t)i * k + l];
            const double* Bl = &B[(size_t)l * n];
            for (int j = 0; j < n; ++j) Ci[j] += a * Bl[j];
        }
    }
    return C;
}

std::vector<double> matmul_tn(int m, int k, int n, const double* A, const double* B) {
    std::vector<double> C((size_t)m * n, 0.0);
    for (int l = 0; l < k; ++l) {
        const double* Al = &A[(size_t)l * m];
        const double* Bl = &B[(size_t)l * n];
        for (int i = 0; i < m; ++i) {
            const double a = Al[i];
            double* Ci = &C[(size_t)i * n];
            for (int j = 0; j < n; ++j) Ci[j] += a * Bl[j];
        }
    }
    return C;
}

}  // namespace kifmm
