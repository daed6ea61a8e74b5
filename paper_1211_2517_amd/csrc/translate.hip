// M2M as one product per parent (Sec. 2.2 in the reduced form of Sec. 3.3):
// q~_P = sum over the octants o of M~^o q~_{child o}, for FP32 plans with one
// right-hand side. The grouped GEMM of gemm.hip walks a parent's eight octant
// classes as eight chunks of its pipeline, which costs about as much per
// launch on the coarse levels (a few to a few hundred parents) as on the
// finest. Here a workgroup of 4 waves takes 16 parents and one row block of
// 16 output rows; wave w multiplies octants 2w and 2w+1, with the children's
// rows loaded straight into the B operand, and the four partial tiles are
// summed through LDS. Every workgroup reads its row block of all eight octant
// matrices, so the form pays where launch latency dominates: the coarse
// levels. The FP32 16x16x4 MFMA: lane (j, g) supplies
// A[j][4g+e] and B[4g+e][j] of a K-step of 16 and holds rows 4g+q of
// column j of the result.
#include "kernels.h"

namespace kifmm {

namespace {

typedef float tv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ tv4 tr_mfma(float a, float b, tv4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int KP16>
__global__ void __launch_bounds__(256) m2m_direct_kernel(int n_par, const int32_t* __restrict__ par_row,
                                                         const int32_t* __restrict__ child,
                                                         const float* __restrict__ A, const float* __restrict__ X,
                                                         float* __restrict__ Y) {
    constexpr int KDIM = KP16 * 16;
    __shared__ __align__(16) tv4 part[3 * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    const int p = blockIdx.x * 16 + j;
    const int blk = blockIdx.y;
    tv4 acc0 = tv4{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int o = 2 * wave + h;
        const int ch = p < n_par ? child[8 * (int64_t)p + o] : -1;
        const float* xr = X + (int64_t)(ch < 0 ? 0 : ch) * KDIM + 4 * g;
        const float* ar = A + ((int64_t)o * KDIM + blk * 16 + j) * KDIM + 4 * g;
        tv4 a[KP16], b[KP16];
#pragma unroll
        for (int t = 0; t < KP16; ++t) {
            a[t] = *reinterpret_cast<const tv4*>(ar + 16 * t);
            b[t] = ch < 0 ? tv4{0.f, 0.f, 0.f, 0.f} : *reinterpret_cast<const tv4*>(xr + 16 * t);
        }
#pragma unroll
        for (int t = 0; t < KP16; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (t & 1)
                    acc1 = tr_mfma(a[t][e], b[t][e], acc1);
                else
                    acc0 = tr_mfma(a[t][e], b[t][e], acc0);
            }
    }
    if (wave > 0) part[(wave - 1) * 64 + lane] = acc0 + acc1;
    __syncthreads();
    if (wave > 0 || p >= n_par) return;
    const tv4 s = acc0 + acc1 + part[lane] + part[64 + lane] + part[128 + lane];
    *reinterpret_cast<tv4*>(Y + (int64_t)par_row[p] * KDIM + blk * 16 + 4 * g) = s;
}

template <int KP16>
hipError_t m2m_direct_t(int n_par, const int32_t* par_row, const int32_t* child, const void* A, const void* X,
                        void* Y, hipStream_t st) {
    const dim3 grid((unsigned)((n_par + 15) / 16), (unsigned)KP16);
    hipLaunchKernelGGL((m2m_direct_kernel<KP16>), grid, dim3(256), 0, st, n_par, par_row, child, (const float*)A,
                       (const float*)X, (float*)Y);
    return hipGetLastError();
}

}  // namespace

bool m2m_direct_supported(int kp) { return kp % 16 == 0 && kp >= 16 && kp <= 160; }

hipError_t launch_m2m_direct(int n_par, const int32_t* par_row, const int32_t* child, const void* A, int kp,
                             const void* X, void* Y, hipStream_t st) {
    if (n_par == 0) return hipSuccess;
    switch (kp / 16) {
        case 1: return m2m_direct_t<1>(n_par, par_row, child, A, X, Y, st);
        case 2: return m2m_direct_t<2>(n_par, par_row, child, A, X, Y, st);
        case 3: return m2m_direct_t<3>(n_par, par_row, child, A, X, Y, st);
        case 4: return m2m_direct_t<4>(n_par, par_row, child, A, X, Y, st);
        case 5: return m2m_direct_t<5>(n_par, par_row, child, A, X, Y, st);
        case 6: return m2m_direct_t<6>(n_par, par_row, child, A, X, Y, st);
        case 7: return m2m_direct_t<7>(n_par, par_row, child, A, X, Y, st);
        case 8: return m2m_direct_t<8>(n_par, par_row, child, A, X, Y, st);
        case 9: return m2m_direct_t<9>(n_par, par_row, child, A, X, Y, st);
        case 10: return m2m_direct_t<10>(n_par, par_row, child, A, X, Y, st);
        default: return hipErrorNotSupported;
    }
}

}  // namespace kifmm
