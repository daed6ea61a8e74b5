// GMRES(m) on a plan's operator (the BEM systems of Sec. 4 are solved by
// GMRES, Sec. 5): restarted GMRES with classical Gram-Schmidt applied twice
// (one pass of products against every basis vector, one update), Givens
// rotations of the small Hessenberg matrix on the host in FP64, and the
// basis in device memory in the plan's precision. The products and updates
// are the kernels below; the matvec is kifmm_apply.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/kifmm.h"

namespace kifmm {
int solve_fail(int code, const std::string& msg);
int plan_precision_bytes(kifmm_plan_t plan, int64_t* n);
}  // namespace kifmm

namespace {

constexpr int kDotBlocks = 240;

// partial[j * gridDim.x + bx] = sum over this block's share of k of V[j][k] w[k]
template <typename T>
__global__ void __launch_bounds__(256) dots_kernel(const T* __restrict__ V, int64_t n, const T* __restrict__ w,
                                                   double* __restrict__ partial) {
    __shared__ double red[256];
    const int j = blockIdx.y;
    const T* v = V + (int64_t)j * n;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        acc += (double)v[k] * (double)w[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

// h[j] = sum of the partial sums of row j (one block per j, fixed order)
__global__ void __launch_bounds__(256) sum_rows_kernel(const double* __restrict__ partial, int nb,
                                                       double* __restrict__ h) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) acc += partial[(int64_t)blockIdx.x * nb + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[blockIdx.x] = red[0];
}

// w[k] += sign * sum_j c[j] V[j][k]
template <typename T>
__global__ void __launch_bounds__(256) combine_kernel(T* __restrict__ w, const T* __restrict__ V, int nv, int64_t n,
                                                      const double* __restrict__ c, double sign) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    double acc = 0.0;
    for (int j = 0; j < nv; ++j) acc += c[j] * (double)V[(int64_t)j * n + k];
    w[k] = (T)((double)w[k] + sign * acc);
}

// dst[k] = s * (a[k] - (b ? b[k] : 0))
template <typename T>
__global__ void __launch_bounds__(256) scaled_diff_kernel(T* __restrict__ dst, const T* __restrict__ a,
                                                          const T* __restrict__ b, double s, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const double v = (double)a[k] - (b ? (double)b[k] : 0.0);
    dst[k] = (T)(s * v);
}

struct Bufs {
    void* V = nullptr;
    void* w = nullptr;
    void* r = nullptr;
    double* partial = nullptr;
    double* h = nullptr;
    ~Bufs() {
        (void)hipFree(V);
        (void)hipFree(w);
        (void)hipFree(r);
        (void)hipFree(partial);
        (void)hipFree(h);
    }
};

#define KIFMM_SOLVE_HIP(call)                                                                        \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return kifmm::solve_fail(KIFMM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int gmres_t(kifmm_plan_t plan, int64_t n, const T* b, T* x, double tol, int m, int max_iter, hipStream_t st,
            int* iters_out, double* resid_out) {
    Bufs B;
    KIFMM_SOLVE_HIP(hipMalloc(&B.V, (size_t)(m + 1) * n * sizeof(T)));
    KIFMM_SOLVE_HIP(hipMalloc(&B.w, (size_t)n * sizeof(T)));
    KIFMM_SOLVE_HIP(hipMalloc(&B.r, (size_t)n * sizeof(T)));
    KIFMM_SOLVE_HIP(hipMalloc((void**)&B.partial, (size_t)(m + 1) * kDotBlocks * sizeof(double)));
    KIFMM_SOLVE_HIP(hipMalloc((void**)&B.h, (size_t)(m + 1) * sizeof(double)));
    T* V = static_cast<T*>(B.V);
    T* w = static_cast<T*>(B.w);
    T* r = static_cast<T*>(B.r);
    const dim3 g1((unsigned)((n + 255) / 256));
    std::vector<double> hh(m + 1);
    // <V[0..nv), v> into hh (host)
    auto dots = [&](const T* Vs, int nv, const T* v) -> int {
        hipLaunchKernelGGL((dots_kernel<T>), dim3(kDotBlocks, nv), dim3(256), 0, st, Vs, n, v, B.partial);
        KIFMM_SOLVE_HIP(hipGetLastError());
        hipLaunchKernelGGL(sum_rows_kernel, dim3(nv), dim3(256), 0, st, B.partial, kDotBlocks, B.h);
        KIFMM_SOLVE_HIP(hipGetLastError());
        KIFMM_SOLVE_HIP(hipMemcpyAsync(hh.data(), B.h, nv * sizeof(double), hipMemcpyDeviceToHost, st));
        KIFMM_SOLVE_HIP(hipStreamSynchronize(st));
        return KIFMM_OK;
    };
    auto apply = [&](const T* in, T* out) -> int { return kifmm_apply(plan, in, out, st); };
    int rc = dots(b, 1, b);
    if (rc) return rc;
    const double bnorm = std::sqrt(hh[0]);
    if (bnorm == 0.0) {
        hipLaunchKernelGGL((scaled_diff_kernel<T>), g1, dim3(256), 0, st, x, x, x, 0.0, n);
        KIFMM_SOLVE_HIP(hipStreamSynchronize(st));
        if (iters_out) *iters_out = 0;
        if (resid_out) *resid_out = 0.0;
        return KIFMM_OK;
    }
    int used = 0;
    double rel = 1.0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    for (;;) {
        // r = b - A x, v0 = r / |r|
        if ((rc = apply(x, w))) return rc;
        ++used;
        hipLaunchKernelGGL((scaled_diff_kernel<T>), g1, dim3(256), 0, st, r, b, w, 1.0, n);
        KIFMM_SOLVE_HIP(hipGetLastError());
        if ((rc = dots(r, 1, r))) return rc;
        const double beta = std::sqrt(hh[0]);
        rel = beta / bnorm;
        if (rel <= tol || used >= max_iter) break;
        hipLaunchKernelGGL((scaled_diff_kernel<T>), g1, dim3(256), 0, st, V, r, (const T*)nullptr, 1.0 / beta, n);
        KIFMM_SOLVE_HIP(hipGetLastError());
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (; k < m && used < max_iter; ++k) {
            if ((rc = apply(V + (int64_t)k * n, w))) return rc;
            ++used;
            // classical Gram-Schmidt, twice
            for (int pass = 0; pass < 2; ++pass) {
                if ((rc = dots(V, k + 1, w))) return rc;
                for (int j = 0; j <= k; ++j) H[(size_t)j * m + k] = (pass ? H[(size_t)j * m + k] : 0.0) + hh[j];
                KIFMM_SOLVE_HIP(hipMemcpyAsync(B.h, hh.data(), (k + 1) * sizeof(double), hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL((combine_kernel<T>), g1, dim3(256), 0, st, w, V, k + 1, n, B.h, -1.0);
                KIFMM_SOLVE_HIP(hipGetLastError());
            }
            if ((rc = dots(w, 1, w))) return rc;
            const double hn = std::sqrt(hh[0]);
            H[(size_t)(k + 1) * m + k] = hn;
            if (hn > 0.0) {
                hipLaunchKernelGGL((scaled_diff_kernel<T>), g1, dim3(256), 0, st, V + (int64_t)(k + 1) * n, w,
                                   (const T*)nullptr, 1.0 / hn, n);
                KIFMM_SOLVE_HIP(hipGetLastError());
            }
            // Givens rotations
            for (int j = 0; j < k; ++j) {
                const double a = H[(size_t)j * m + k], c = H[(size_t)(j + 1) * m + k];
                H[(size_t)j * m + k] = cs[j] * a + sn[j] * c;
                H[(size_t)(j + 1) * m + k] = -sn[j] * a + cs[j] * c;
            }
            const double a = H[(size_t)k * m + k], c = H[(size_t)(k + 1) * m + k];
            const double d = std::hypot(a, c);
            cs[k] = d > 0 ? a / d : 1.0;
            sn[k] = d > 0 ? c / d : 0.0;
            H[(size_t)k * m + k] = d;
            H[(size_t)(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (std::fabs(g[k + 1]) / bnorm <= tol || hn == 0.0) {
                ++k;
                break;
            }
        }
        // x += V y, H(0:k, 0:k) y = g(0:k)
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * m + j] * y[j];
            y[i] = s / H[(size_t)i * m + i];
        }
        KIFMM_SOLVE_HIP(hipMemcpyAsync(B.h, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL((combine_kernel<T>), g1, dim3(256), 0, st, x, V, k, n, B.h, 1.0);
        KIFMM_SOLVE_HIP(hipGetLastError());
        KIFMM_SOLVE_HIP(hipStreamSynchronize(st));
    }
    if (iters_out) *iters_out = used;
    if (resid_out) *resid_out = rel;
    return KIFMM_OK;
}

}  // namespace

extern "C" int kifmm_solve_gmres(kifmm_plan_t plan, const void* b, void* x, double tol, int restart, int max_iter,
                                 void* stream, int* iterations, double* residual) {
    int64_t n = 0;
    const int eb = kifmm::plan_precision_bytes(plan, &n);
    if (eb < 0) return eb;
    if (!b || !x || b == x) return kifmm::solve_fail(KIFMM_EINVAL, "b and x must be non-NULL and distinct");
    if (!(tol > 0.0) || restart < 1 || restart > 200 || max_iter < 1)
        return kifmm::solve_fail(KIFMM_EINVAL, "need tol > 0, 1 <= restart <= 200 and max_iter >= 1");
    hipStream_t st = (hipStream_t)stream;
    if (eb == 8)
        return gmres_t<double>(plan, n, (const double*)b, (double*)x, tol, restart, max_iter, st, iterations, residual);
    return gmres_t<float>(plan, n, (const float*)b, (float*)x, tol, restart, max_iter, st, iterations, residual);
}
