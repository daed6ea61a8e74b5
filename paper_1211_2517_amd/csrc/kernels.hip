// Device kernels of the KIFMM evaluation for gfx950 (CDNA4, wave64).
//
// gg_kernel      grouped gather GEMM on MFMA: the S2M/L2T reduced-operator
//                products (Sec. 3.3), M2M and L2L (eqs. (4), (6)) and the
//                compressed M2L (eq. (13) with the level scaling of Sec. 3.1).
// eval_surface   potential of the points of a leaf on the (3-2d) cube surface:
//                the check potential of S2M (eq. (3)) and, in the adjoint,
//                the transpose of the L2T evaluation.
// eval_targets   near-field direct sum of eq. (1) over the near field (S2T)
//                plus the potential of the downward equivalent densities on
//                the leaf's points (L2T, eq. (7)), scattered to caller order.
#include "kernels.h"

namespace kifmm {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

// Output row of accumulator element q held by lane group g (column = lane % 16):
// the FP32 form stores 4 consecutive rows per lane group, the FP64 form
// interleaves the lane groups row by row.
template <>
struct Mfma<float> {
    using V4 = f32x4;
    static __device__ __forceinline__ V4 step(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int g) { return 4 * g + q; }
};

template <>
struct Mfma<double> {
    using V4 = f64x4;
    static __device__ __forceinline__ V4 step(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int g) { return 4 * q + g; }
};

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

template <typename T>
struct alignas(4 * sizeof(T)) P4 {
    T x, y, z, w;
};

struct GGParams {
    const void* A;
    int64_t a_stride;
    int lda;
    const void* X;
    int ldx;
    void* Y;
    int ldy;
    int MB;
    int R;
    int cp;
    int accumulate;
    const int32_t* tile_tgt0;
    const int32_t* tile_ntgt;
    const int32_t* tile_chunk0;
    const void* tile_scale;
    const int32_t* chunk_cls;
    const int32_t* chunk_src;
    const int32_t* chunk_col;
};

constexpr int kMBW = 2;  // 16-row output blocks owned by one wave

// One workgroup owns one tile of target rows; its (MB*16) x (ntgt*R)
// accumulator lives in LDS. Wave w owns output row blocks [2w, 2w+2) and walks
// every chunk of the tile: per class it keeps its rows of A in registers, per
// chunk it gathers up to 16 columns of X, runs the 16x16x4 MFMA chain over the
// K dimension and adds the result into its own LDS rows (no two lanes or
// waves touch the same LDS word in one step, so no atomics are needed).
//
// MFMA operand layout (v_mfma_*_16x16x4): lane l supplies A[l%16][kk] and
// B[kk][l%16] of one K-step and holds D[Mfma<T>::row(q, l/16)][l%16]. The K
// order is permuted so that both operands are read as 4-wide vectors: in
// K-chunk t, lane group g = l/16 supplies indices 16t + 4g + e for the 4
// consecutive MFMA steps e = 0..3.
template <typename T, int KP16>
__global__ void __launch_bounds__(1024) gg_kernel(GGParams p) {
    using M = Mfma<T>;
    using V4 = typename M::V4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* acc = reinterpret_cast<T*>(smem_raw);
    const int tile = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rows = p.MB * 16;
    const int ldl = rows + 4;
    const int R = p.R;
    const int t0 = p.tile_tgt0[tile];
    const int ncol = p.tile_ntgt[tile] * R;
    const T* __restrict__ X = static_cast<const T*>(p.X);
    const T* __restrict__ A = static_cast<const T*>(p.A);
    T* __restrict__ Y = static_cast<T*>(p.Y);

    const int64_t ybase = (int64_t)t0 * R;
    for (int idx = threadIdx.x; idx < ncol * rows; idx += blockDim.x) {
        const int col = idx / rows;
        const int row = idx - col * rows;
        acc[col * ldl + row] = p.accumulate ? Y[(ybase + col) * p.ldy + row] : T(0);
    }
    __syncthreads();

    const int j = lane & 15;
    const int grp = lane >> 4;
    const int mb0 = wave * kMBW;
    const T scale = static_cast<const T*>(p.tile_scale)[tile];
    const int cb = p.tile_chunk0[tile];
    const int ce = p.tile_chunk0[tile + 1];
    const int pj = j / R;
    const int rj = j - pj * R;

    V4 a[kMBW][KP16];
    int cur = -1;
    for (int ch = cb; ch < ce; ++ch) {
        const int cls = p.chunk_cls[ch];
        if (cls != cur) {
            cur = cls;
            const T* Ac = A + (int64_t)cls * p.a_stride;
#pragma unroll
            for (int m = 0; m < kMBW; ++m) {
                const int mb = mb0 + m;
                const T* ar = Ac + (int64_t)(mb * 16 + j) * p.lda + 4 * grp;
#pragma unroll
                for (int t = 0; t < KP16; ++t) {
                    if (mb < p.MB)
                        a[m][t] = *reinterpret_cast<const V4*>(ar + 16 * t);
                    else
                        a[m][t] = V4{0, 0, 0, 0};
                }
            }
        }
        const int src = p.chunk_src[ch * p.cp + pj];
        const int col = p.chunk_col[ch * p.cp + pj];
        V4 b[KP16];
        if (src >= 0) {
            const T* xs = X + ((int64_t)src * R + rj) * p.ldx + 4 * grp;
#pragma unroll
            for (int t = 0; t < KP16; ++t) b[t] = *reinterpret_cast<const V4*>(xs + 16 * t);
        } else {
#pragma unroll
            for (int t = 0; t < KP16; ++t) b[t] = V4{0, 0, 0, 0};
        }
        V4 d[kMBW];
#pragma unroll
        for (int m = 0; m < kMBW; ++m) d[m] = V4{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < KP16; ++t) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
#pragma unroll
                for (int m = 0; m < kMBW; ++m) d[m] = M::step(a[m][t][e], b[t][e], d[m]);
            }
        }
        if (col >= 0) {
#pragma unroll
            for (int m = 0; m < kMBW; ++m) {
                if (mb0 + m < p.MB) {
                    T* dst = acc + (col * R + rj) * ldl + (mb0 + m) * 16;
#pragma unroll
                    for (int q = 0; q < 4; ++q) dst[M::row(q, grp)] += scale * d[m][q];
                }
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < ncol * rows; idx += blockDim.x) {
        const int col = idx / rows;
        const int row = idx - col * rows;
        Y[(ybase + col) * p.ldy + row] = acc[col * ldl + row];
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) permute_in_kernel(int64_t n, const int32_t* __restrict__ perm,
                                                         const T* __restrict__ sigma, int64_t ld,
                                                         int nrhs, T* __restrict__ sig_s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t src = perm[i];
#pragma unroll
    for (int r = 0; r < R; ++r) sig_s[i * R + r] = r < nrhs ? sigma[src + r * ld] : T(0);
}

// one wave per leaf; lanes run over the surface points
template <typename T, int R>
__global__ void __launch_bounds__(256) eval_surface_kernel(int64_t n_leaf, const P4<T>* __restrict__ pts,
                                                           const T* __restrict__ sig,
                                                           const int32_t* __restrict__ leaf_ptr,
                                                           const T* __restrict__ surf, int n_eq,
                                                           int nep, T* __restrict__ C) {
    const int64_t leaf = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (leaf >= n_leaf) return;
    const int lane = threadIdx.x & 63;
    const int p0 = leaf_ptr[leaf];
    const int p1 = leaf_ptr[leaf + 1];
    for (int a0 = 0; a0 < nep; a0 += 64) {
        const int a = a0 + lane;
        const bool valid = a < n_eq;
        T sx = 0, sy = 0, sz = 0;
        if (valid) {
            sx = surf[3 * a];
            sy = surf[3 * a + 1];
            sz = surf[3 * a + 2];
        }
        T acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0;
        for (int jj = p0; jj < p1; ++jj) {
            const P4<T> q = pts[jj];
            const T dx = sx - q.x, dy = sy - q.y, dz = sz - q.z;
            const T rinv = rsq(dx * dx + dy * dy + dz * dz);
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += sig[(int64_t)jj * R + r] * rinv;
        }
        if (a < nep) {
#pragma unroll
            for (int r = 0; r < R; ++r) C[(leaf * R + r) * nep + a] = valid ? acc[r] : T(0);
        }
    }
}

// one wave per target leaf; `lpt` lanes per target split the sources
template <typename T, int R>
__global__ void __launch_bounds__(256) eval_targets_kernel(
    int64_t n_leaf, const P4<T>* __restrict__ pts, const T* __restrict__ sig,
    const int32_t* __restrict__ leaf_ptr, const int32_t* __restrict__ near_ptr,
    const int32_t* __restrict__ near_leaf, const int32_t* __restrict__ near_code,
    const T* __restrict__ E, const T* __restrict__ surf, int n_eq, int nep, T near_scale,
    T far_scale, const int32_t* __restrict__ perm, T* __restrict__ out, int64_t ld, int nrhs) {
    const int64_t leaf = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (leaf >= n_leaf) return;
    const int lane = threadIdx.x & 63;
    const int p0 = leaf_ptr[leaf];
    const int ne = leaf_ptr[leaf + 1] - p0;
    int lpt = 64;
    while (lpt > 1 && (64 / lpt) < ne) lpt >>= 1;
    const int tpr = 64 / lpt;
    const int sub = lane & (lpt - 1);
    const int q0 = near_ptr[leaf];
    const int q1 = near_ptr[leaf + 1];
    for (int tb = 0; tb < ne; tb += tpr) {
        const int tl = tb + lane / lpt;
        const bool valid = tl < ne;
        const int i = p0 + (valid ? tl : 0);
        const P4<T> ui = pts[i];
        T acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0;
        for (int q = q0; q < q1; ++q) {
            const int nb = near_leaf[q];
            const int code = near_code[q];
            const T wx = ui.x + T(2 * (code / 9 - 1));
            const T wy = ui.y + T(2 * ((code / 3) % 3 - 1));
            const T wz = ui.z + T(2 * (code % 3 - 1));
            const int b1 = leaf_ptr[nb + 1];
            for (int jj = leaf_ptr[nb] + sub; jj < b1; jj += lpt) {
                const P4<T> s = pts[jj];
                const T dx = wx - s.x, dy = wy - s.y, dz = wz - s.z;
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T rinv = r2 > T(0) ? rsq(r2) : T(0);
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += sig[(int64_t)jj * R + r] * rinv;
            }
        }
        T far[R];
#pragma unroll
        for (int r = 0; r < R; ++r) far[r] = 0;
        if (E != nullptr) {
            for (int a = sub; a < n_eq; a += lpt) {
                const T dx = ui.x - surf[3 * a], dy = ui.y - surf[3 * a + 1], dz = ui.z - surf[3 * a + 2];
                const T rinv = rsq(dx * dx + dy * dy + dz * dz);
#pragma unroll
                for (int r = 0; r < R; ++r) far[r] += E[(leaf * R + r) * nep + a] * rinv;
            }
        }
        for (int off = lpt >> 1; off > 0; off >>= 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc[r] += __shfl_xor(acc[r], off);
                far[r] += __shfl_xor(far[r], off);
            }
        }
        if (valid && sub == 0) {
            const int64_t dst = perm[i];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nrhs) out[dst + r * ld] = near_scale * acc[r] + far_scale * far[r];
        }
    }
}

template <typename T, int KP16>
hipError_t gg_launch_t(const GGParams& p, int n_tiles, int waves, size_t lds, hipStream_t st) {
    static size_t attr_set = 0;
    if (lds > 65536 && lds > attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gg_kernel<T, KP16>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = lds;
    }
    hipLaunchKernelGGL((gg_kernel<T, KP16>), dim3(n_tiles), dim3(64 * waves), lds, st, p);
    return hipGetLastError();
}

template <typename T>
hipError_t gg_dispatch(int KP16, const GGParams& p, int n_tiles, int waves, size_t lds, hipStream_t st) {
    switch (KP16) {
#define KIFMM_GG_CASE(K) \
    case K:              \
        return gg_launch_t<T, K>(p, n_tiles, waves, lds, st);
        KIFMM_GG_CASE(1) KIFMM_GG_CASE(2) KIFMM_GG_CASE(3) KIFMM_GG_CASE(4) KIFMM_GG_CASE(5)
        KIFMM_GG_CASE(6) KIFMM_GG_CASE(7) KIFMM_GG_CASE(8) KIFMM_GG_CASE(9) KIFMM_GG_CASE(10)
        KIFMM_GG_CASE(11) KIFMM_GG_CASE(12) KIFMM_GG_CASE(13) KIFMM_GG_CASE(14) KIFMM_GG_CASE(15)
        KIFMM_GG_CASE(16) KIFMM_GG_CASE(17) KIFMM_GG_CASE(18) KIFMM_GG_CASE(19)
#undef KIFMM_GG_CASE
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace

size_t gg_lds_limit() { return 160 * 1024; }

size_t gg_lds_bytes(int elt, int MB, int cols) { return (size_t)cols * (MB * 16 + 4) * elt; }

hipError_t launch_gg(const DevSched& s, int elt, const void* A, int MB, int KP16, const void* X,
                     int ldx, void* Y, int ldy, int R, int accumulate, hipStream_t st) {
    if (s.n_tiles == 0) return hipSuccess;
    GGParams p;
    p.A = A;
    p.a_stride = (int64_t)MB * 16 * KP16 * 16;
    p.lda = KP16 * 16;
    p.X = X;
    p.ldx = ldx;
    p.Y = Y;
    p.ldy = ldy;
    p.MB = MB;
    p.R = R;
    p.cp = s.cp;
    p.accumulate = accumulate;
    p.tile_tgt0 = s.tile_tgt0;
    p.tile_ntgt = s.tile_ntgt;
    p.tile_chunk0 = s.tile_chunk0;
    p.tile_scale = s.tile_scale;
    p.chunk_cls = s.chunk_cls;
    p.chunk_src = s.chunk_src;
    p.chunk_col = s.chunk_col;
    const int waves = (MB + kMBW - 1) / kMBW;
    const size_t lds = gg_lds_bytes(elt, MB, s.max_tile * R);
    if (lds > gg_lds_limit() || waves > 16) return hipErrorInvalidValue;
    if (elt == 4) return gg_dispatch<float>(KP16, p, s.n_tiles, waves, lds, st);
    return gg_dispatch<double>(KP16, p, s.n_tiles, waves, lds, st);
}

#define KIFMM_R_SWITCH(R, BODY)                      \
    switch (R) {                                     \
        case 1: { constexpr int RR = 1; BODY; break; }  \
        case 2: { constexpr int RR = 2; BODY; break; }  \
        case 4: { constexpr int RR = 4; BODY; break; }  \
        case 8: { constexpr int RR = 8; BODY; break; }  \
        case 16: { constexpr int RR = 16; BODY; break; } \
        default: return hipErrorInvalidValue;        \
    }

hipError_t launch_permute_in(int elt, int R, int64_t n, const int32_t* perm, const void* sigma,
                             int64_t ld, int nrhs, void* sig_s, hipStream_t st) {
    const dim3 grid((unsigned)((n + 255) / 256));
    if (elt == 4) {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((permute_in_kernel<float, RR>), grid, dim3(256), 0, st, n, perm,
                                             (const float*)sigma, ld, nrhs, (float*)sig_s))
    } else {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((permute_in_kernel<double, RR>), grid, dim3(256), 0, st, n, perm,
                                             (const double*)sigma, ld, nrhs, (double*)sig_s))
    }
    return hipGetLastError();
}

hipError_t launch_eval_surface(int elt, int R, int64_t n_leaf, const void* pts, const void* sig_s,
                               const int32_t* leaf_ptr, const void* surf, int n_eq, int nep, void* C,
                               hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_leaf + 3) / 4));
    if (elt == 4) {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_surface_kernel<float, RR>), grid, dim3(256), 0, st, n_leaf,
                                             (const P4<float>*)pts, (const float*)sig_s, leaf_ptr,
                                             (const float*)surf, n_eq, nep, (float*)C))
    } else {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_surface_kernel<double, RR>), grid, dim3(256), 0, st, n_leaf,
                                             (const P4<double>*)pts, (const double*)sig_s, leaf_ptr,
                                             (const double*)surf, n_eq, nep, (double*)C))
    }
    return hipGetLastError();
}

hipError_t launch_eval_targets(int elt, int R, int64_t n_leaf, const void* pts, const void* sig_s,
                               const int32_t* leaf_ptr, const int32_t* near_ptr, const int32_t* near_leaf,
                               const int32_t* near_code, const void* E, const void* surf, int n_eq, int nep,
                               double near_scale, double far_scale, const int32_t* perm, void* out,
                               int64_t ld, int nrhs, hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_leaf + 3) / 4));
    if (elt == 4) {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_targets_kernel<float, RR>), grid, dim3(256), 0, st, n_leaf,
                                             (const P4<float>*)pts, (const float*)sig_s, leaf_ptr, near_ptr,
                                             near_leaf, near_code, (const float*)E, (const float*)surf, n_eq,
                                             nep, (float)near_scale, (float)far_scale, perm, (float*)out, ld,
                                             nrhs))
    } else {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_targets_kernel<double, RR>), grid, dim3(256), 0, st, n_leaf,
                                             (const P4<double>*)pts, (const double*)sig_s, leaf_ptr, near_ptr,
                                             near_leaf, near_code, (const double*)E, (const double*)surf, n_eq,
                                             nep, near_scale, far_scale, perm, (double*)out, ld, nrhs))
    }
    return hipGetLastError();
}

}  // namespace kifmm
