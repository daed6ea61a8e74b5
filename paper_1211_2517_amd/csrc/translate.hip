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
//
// L2L (and the adjoint's M2M^T) in the direct form: every child takes one
// product, p~_child += L~^o p~_parent with o its octant. The children of a
// level are sorted by octant and cut into segments of up to 16*kDownMaxBlocks
// of one
// octant; a workgroup of 4 waves takes a segment, each wave two (more for
// k_pad > 128) 16-row blocks of L~^o in registers, loaded once, and walks the
// segment's 16-column blocks: the rows of a block two blocks ahead, the
// parents' rows (straight into the B operand) and the children's old rows
// one block ahead of the MFMAs. No LDS and no barrier: the waves of a
// workgroup never wait for each other.
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

template <int KP16>
__global__ void __launch_bounds__(256) down_direct_kernel(const int32_t* __restrict__ seg,
                                                          const int32_t* __restrict__ tgt,
                                                          const int32_t* __restrict__ src,
                                                          const float* __restrict__ A, const float* __restrict__ X,
                                                          float* __restrict__ Y) {
    constexpr int KDIM = KP16 * 16;
    constexpr int RBW = (KP16 + 3) / 4;   // row blocks per wave
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    const int cls = seg[3 * blockIdx.x], i0 = seg[3 * blockIdx.x + 1], n = seg[3 * blockIdx.x + 2];
    const int ncb = (n + 15) >> 4;
    // Every load is issued unconditionally and in the same order for every
    // block (indices clamped into the segment, row blocks past k_pad clamped
    // to the last one): loads under a branch would make the compiler drain
    // all loads in flight where the branches join, the prefetched ones too.
    // An empty slot computes on the segment's last item and is not stored;
    // MFMA columns are independent, so nothing else sees it.
    auto load_idx = [&](int c, int& sr, int& row) {
        const int i = min(16 * c + j, n - 1);
        sr = src[i0 + i];
        row = tgt[i0 + i];
    };
    auto load_ops = [&](int sr, int row, tv4 (&b)[KP16], tv4 (&y)[RBW]) {
        const float* xr = X + (int64_t)sr * KDIM + 4 * g;
#pragma unroll
        for (int t = 0; t < KP16; ++t) b[t] = *reinterpret_cast<const tv4*>(xr + 16 * t);
        const float* yr = Y + (int64_t)row * KDIM + 4 * g;
#pragma unroll
        for (int r = 0; r < RBW; ++r) y[r] = *reinterpret_cast<const tv4*>(yr + min(wave + 4 * r, KP16 - 1) * 16);
    };
    // register sets by block parity: the rows (source, target) of blocks c
    // and c+1, the operands of blocks c and c+1
    int sr0, row0, sr1, row1;
    tv4 b0[KP16], b1[KP16], y0[RBW], y1[RBW];
    load_idx(0, sr0, row0);
    load_idx(min(1, ncb - 1), sr1, row1);
    tv4 a[RBW][KP16];
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
        const int blk = min(wave + 4 * r, KP16 - 1);
        const float* ar = A + ((int64_t)cls * KDIM + blk * 16 + j) * KDIM + 4 * g;
#pragma unroll
        for (int t = 0; t < KP16; ++t) a[r][t] = *reinterpret_cast<const tv4*>(ar + 16 * t);
    }
    load_ops(sr0, row0, b0, y0);
    // block c: the rows of block c+2 are loaded first (into block c's set,
    // after its target row is taken), then the operands of block c+1 (whose
    // rows arrived one block earlier), then block c is multiplied; its
    // operands were loaded one block earlier. Blocks past the segment run
    // the same loads and skip the MFMAs and the store.
    auto step = [&](int c, int& src_c, int& row_c, const int& src_n, const int& row_n, const tv4 (&bc)[KP16],
                    const tv4 (&yc)[RBW], tv4 (&bn)[KP16], tv4 (&yn)[RBW]) {
        const int rc = row_c;
        load_idx(min(c + 2, ncb - 1), src_c, row_c);
        load_ops(src_n, row_n, bn, yn);
        if (c >= ncb) return;
        const bool live = 16 * c + j < n;
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
            const int blk = wave + 4 * r;
            if (blk >= KP16) break;
            tv4 d0 = tv4{0.f, 0.f, 0.f, 0.f}, d1 = d0;
#pragma unroll
            for (int t = 0; t < KP16; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (t & 1)
                        d1 = tr_mfma(a[r][t][e], bc[t][e], d1);
                    else
                        d0 = tr_mfma(a[r][t][e], bc[t][e], d0);
                }
            if (live) *reinterpret_cast<tv4*>(Y + (int64_t)rc * KDIM + blk * 16 + 4 * g) = yc[r] + (d0 + d1);
        }
    };
    for (int c = 0; c < ncb; c += 2) {
        step(c, sr0, row0, sr1, row1, b0, y0, b1, y1);
        step(c + 1, sr1, row1, sr0, row0, b1, y1, b0, y0);
    }
}

template <int KP16>
hipError_t down_direct_t(int n_seg, const int32_t* seg, const int32_t* tgt, const int32_t* src, const void* A,
                         const void* X, void* Y, hipStream_t st) {
    hipLaunchKernelGGL((down_direct_kernel<KP16>), dim3((unsigned)n_seg), dim3(256), 0, st, seg, tgt, src,
                       (const float*)A, (const float*)X, (float*)Y);
    return hipGetLastError();
}

}  // namespace

bool m2m_direct_supported(int kp) { return kp % 16 == 0 && kp >= 16 && kp <= 160; }

hipError_t launch_down_direct(int n_seg, const int32_t* seg, const int32_t* tgt, const int32_t* src, const void* A,
                              int kp, const void* X, void* Y, hipStream_t st) {
    if (n_seg == 0) return hipSuccess;
    switch (kp / 16) {
        case 1: return down_direct_t<1>(n_seg, seg, tgt, src, A, X, Y, st);
        case 2: return down_direct_t<2>(n_seg, seg, tgt, src, A, X, Y, st);
        case 3: return down_direct_t<3>(n_seg, seg, tgt, src, A, X, Y, st);
        case 4: return down_direct_t<4>(n_seg, seg, tgt, src, A, X, Y, st);
        case 5: return down_direct_t<5>(n_seg, seg, tgt, src, A, X, Y, st);
        case 6: return down_direct_t<6>(n_seg, seg, tgt, src, A, X, Y, st);
        case 7: return down_direct_t<7>(n_seg, seg, tgt, src, A, X, Y, st);
        case 8: return down_direct_t<8>(n_seg, seg, tgt, src, A, X, Y, st);
        case 9: return down_direct_t<9>(n_seg, seg, tgt, src, A, X, Y, st);
        case 10: return down_direct_t<10>(n_seg, seg, tgt, src, A, X, Y, st);
        default: return hipErrorNotSupported;
    }
}

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
