// Device kernels of the KIFMM evaluation for gfx950 (CDNA4, wave64).
//
// gg_kernel      grouped gather GEMM on MFMA: the S2M/L2T reduced-operator
//                products (Sec. 3.3), M2M and L2L (Sec. 2.2 and their reduced forms) and the
//                compressed M2L (Sec. 3.1, K~ applied with the homogeneous level scaling).
// eval_surface   potential of the points of a leaf on the (3-2d) cube surface:
//                the check potential of S2M (Sec. 2.2) and, in the adjoint,
//                the transpose of the L2T evaluation.
// eval_targets   near-field direct sum of eq. (1) over the near field (S2T)
//                plus the potential of the downward equivalent densities on
//                the leaf's points (L2T, Sec. 2.2), scattered to caller order.
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
    int n_tiles;
    int n_rg;
    const int32_t* tile_tgt0;
    const int32_t* tile_ntgt;
    const int32_t* tile_chunk0;
    const int32_t* chunk_cls;
    const int32_t* chunk_next;
    const int32_t* chunk_nblk;
    const void* chunk_scale;
    const int32_t* chunk_src;
    const int32_t* chunk_col;
};

// Loads through the constant address space: with a wave-uniform index the
// compiler emits scalar loads, which are counted apart from the vector loads
// (lgkmcnt, not vmcnt) and so never force the vector-load queue to drain.
template <typename T>
__device__ __forceinline__ T uload(const void* base, int idx) {
    typedef const T __attribute__((address_space(4))) CT;
    return reinterpret_cast<CT*>(reinterpret_cast<uintptr_t>(base))[idx];
}

// Grouped gather GEMM: Y[t] (+)= scale * sum_chunks A[cls] X[src].
//
// A workgroup owns one (tile, row group): the targets of the tile and WAVES
// 16-row blocks of the output, one per wave. Its accumulator (rows x ntgt*R
// columns) lives in LDS. The chunks of a tile are sorted by class; a chunk
// holds up to 32 columns (two 16-column MFMA blocks, the second one only when
// used) of one class. Per chunk the workgroup
//   - stages the gathered source columns of X in an LDS buffer, loaded by all
//     threads one chunk ahead (double buffer, one barrier per chunk);
//   - each wave multiplies its 16 rows of A[cls], held in registers for the
//     whole run of chunks of one class (the next class's rows are prefetched
//     one chunk ahead of a class change), by the staged columns on 16x16x4
//     MFMA and adds the result into its own LDS rows.
// Chunk metadata that is uniform across a wave (class, next class, block
// count, scale and the source index of each staged column) is read with
// scalar loads; only the gathered data and the per-lane target column are
// vector loads, issued so that every wait retires only what it needs.
// Within a chunk the target columns are distinct and each wave owns its
// rows, so no two lanes or waves update the same LDS word at the same time
// and the summation order is fixed (results are bitwise reproducible).
//
// MFMA operand layout (v_mfma_*_16x16x4): lane l supplies A[l%16][kk] and
// B[kk][l%16] of one K-step and holds D[Mfma<T>::row(q, l/16)][l%16]. The K
// order is permuted so that both operands are read as 4-wide vectors: in
// K-chunk t, lane group g = l/16 supplies indices 16t + 4g + e for the 4
// consecutive MFMA steps e = 0..3.
//
// Block b maps to tile (b / (8*n_rg))*8 + b%8 and row group (b/8) % n_rg, so
// the row groups of a tile run on the same XCD (blocks are dealt to the 8 XCDs
// round-robin) and share its L2 for the gathered columns.
template <typename T, int KP16, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) gg_kernel(GGParams p) {
    using M = Mfma<T>;
    using V4 = typename M::V4;
    constexpr int NT = 64 * WAVES;
    constexpr int KDIM = KP16 * 16;
    constexpr int LDB = KDIM + 4;          // LDS stride of one staged column
    constexpr int V4C = KDIM / 4;          // 4-vectors per column
    constexpr int CPL = V4C >= 64 ? 1 : 64 / V4C;   // columns covered by one wave-wide load
    constexpr int LPC = (V4C + 63) / 64;             // wave-wide loads per column (wide K)
    constexpr int GRP = CPL * WAVES;                 // columns covered per load round by the workgroup
    constexpr int NLD = ((32 + GRP - 1) / GRP) * LPC;   // loads per lane per chunk
    const int b = blockIdx.x;
    const int rg = (b >> 3) % p.n_rg;
    const int tile = (b / (8 * p.n_rg)) * 8 + (b & 7);
    if (tile >= p.n_tiles) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* bbuf = reinterpret_cast<T*>(smem_raw);   // [2][32][LDB]
    T* acc = bbuf + 2 * 32 * LDB;               // [ncol][ldl]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int mb_lo = rg * WAVES;
    const int nmb = min(WAVES, p.MB - mb_lo);
    const int rows = nmb * 16;
    const int ldl = WAVES * 16 + 4;
    const int R = p.R;
    const int cp = p.cp;
    const int t0 = uload<int32_t>(p.tile_tgt0, tile);
    const int ncol = uload<int32_t>(p.tile_ntgt, tile) * R;
    const T* __restrict__ X = static_cast<const T*>(p.X);
    const T* __restrict__ A = static_cast<const T*>(p.A);
    T* __restrict__ Y = static_cast<T*>(p.Y);

    const int64_t ybase = (int64_t)t0 * R;
    const int row0 = mb_lo * 16;
    for (int idx = threadIdx.x; idx < ncol * rows; idx += NT) {
        const int col = idx / rows;
        const int row = idx - col * rows;
        acc[col * ldl + row] = p.accumulate ? Y[(ybase + col) * p.ldy + row0 + row] : T(0);
    }

    const int cb = uload<int32_t>(p.tile_chunk0, tile);
    const int ce = uload<int32_t>(p.tile_chunk0, tile + 1);
    const int j = lane & 15;
    const int grp = lane >> 4;
    const bool wact = wave < nmb;
    const T* arow = A + (int64_t)(row0 + (wact ? wave : 0) * 16 + j) * p.lda + 4 * grp;

    // staging map: load i of this lane covers staged column sc[i] (0..31),
    // 4-vector part sp[i] of it. In load i the wave covers the CPL columns
    // scb[i] .. scb[i]+CPL-1 (lane / V4C picks one). Lanes beyond them repeat
    // a valid (column, part), so every lane issues the same loads and stores
    // (duplicates write identical values); no load is predicated.
    int sc[NLD], sp[NLD], scb[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int unit = i / LPC;                       // which column round
        const int sub = i - unit * LPC;                 // which 64-wide slice of a long column
        scb[i] = (unit * WAVES + wave) * CPL;
        const int q = CPL > 1 ? min(lane / V4C, CPL - 1) : 0;
        sc[i] = min(scb[i] + q, 31);
        sp[i] = min((CPL > 1 ? lane - q * V4C : lane) + sub * 64, V4C - 1);
    }
    V4 stg[NLD];
    // Empty pair slots hold source -1 and load row 0 (a valid row): their
    // products land only in output columns that are never stored. All source
    // indices are fetched first (scalar loads), then all gathers are issued.
    auto stage_load = [&](int ch) {
        int src[NLD];
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            int s = 0;
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int c = min(scb[i] + q, 31);
                const int sq = uload<int32_t>(p.chunk_src, ch * cp + c / R);
                if (sc[i] == c) s = sq;
            }
            src[i] = max(s, 0);
        }
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int c = sc[i];
            const int pj = c / R;
            stg[i] = *reinterpret_cast<const V4*>(X + ((int64_t)src[i] * R + (c - pj * R)) * p.ldx + 4 * sp[i]);
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) *reinterpret_cast<V4*>(bbuf + (buf * 32 + sc[i]) * LDB + 4 * sp[i]) = stg[i];
    };
    // A rows of the current class run and of the next one; the two register
    // sets swap roles from run to run (the run loop below is unrolled by two),
    // so a prefetch lands directly in the registers that will use it.
    V4 a0[KP16];
    V4 a1[KP16];
    auto load_a = [&](V4 (&dst)[KP16], int cls) {
        const T* ar = arow + (int64_t)cls * p.a_stride;
#pragma unroll
        for (int t = 0; t < KP16; ++t) dst[t] = *reinterpret_cast<const V4*>(ar + 16 * t);
    };

    const int pj16 = j / R;
    const int rj = j - pj16 * R;
    int col0 = -1, col1 = -1;   // target columns of the current chunk (both blocks)
    if (cb < ce) {
        load_a(a0, uload<int32_t>(p.chunk_cls, cb));
        stage_load(cb);
        stage_store(0);
        col0 = p.chunk_col[cb * cp + pj16];
        col1 = p.chunk_col[cb * cp + (16 / R) + pj16];
    }
    __syncthreads();

    // one chunk: stage chunk ch+1 (and its target columns) while the MFMAs of chunk ch run
    auto step = [&](int ch, const V4 (&a)[KP16]) {
        const int buf = (ch - cb) & 1;
        // scalar metadata first: scalar and LDS loads share one counter, and
        // scalar ones return out of order, so none may be pending at the MFMAs
        const int nb = uload<int32_t>(p.chunk_nblk, ch);
        const T scale = uload<T>(p.chunk_scale, ch);
        const int chn = min(ch + 1, ce - 1);
        const int ncol0 = p.chunk_col[chn * cp + pj16];
        const int ncol1 = p.chunk_col[chn * cp + (16 / R) + pj16];
        stage_load(chn);
        if (wact) {
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                if (blk < nb) {
                    const T* bcol = bbuf + (buf * 32 + blk * 16 + j) * LDB + 4 * grp;
                    V4 bv[KP16];
#pragma unroll
                    for (int t = 0; t < KP16; ++t) bv[t] = *reinterpret_cast<const V4*>(bcol + 16 * t);
                    // issue every LDS read of the block before the first MFMA
                    __builtin_amdgcn_sched_barrier(0);
                    V4 d0 = V4{0, 0, 0, 0};
                    V4 d1 = V4{0, 0, 0, 0};
#pragma unroll
                    for (int t = 0; t < KP16; ++t) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            if (t & 1)
                                d1 = M::step(a[t][e], bv[t][e], d1);
                            else
                                d0 = M::step(a[t][e], bv[t][e], d0);
                        }
                    }
                    const int col = blk ? col1 : col0;
                    if (col >= 0) {
                        T* dst = acc + (col * R + rj) * ldl + wave * 16;
#pragma unroll
                        for (int q = 0; q < 4; ++q) dst[M::row(q, grp)] += scale * (d0[q] + d1[q]);
                    }
                }
            }
        }
        stage_store(buf ^ 1);
        col0 = ncol0;
        col1 = ncol1;
        __syncthreads();
    };
    // one class run: prefetch the next run's A rows, then its chunks
    auto run = [&](int ch, const V4 (&a)[KP16], V4 (&nxt)[KP16]) {
        const int cls = uload<int32_t>(p.chunk_cls, ch);
        const int nx = uload<int32_t>(p.chunk_next, ch);
        load_a(nxt, nx >= 0 ? nx : cls);   // unconditional, so every path issues the same loads
        do {
            step(ch, a);
            ++ch;
        } while (ch < ce && uload<int32_t>(p.chunk_cls, ch) == cls);
        return ch;
    };
    for (int ch = cb; ch < ce;) {
        ch = run(ch, a0, a1);
        if (ch < ce) ch = run(ch, a1, a0);
    }
    for (int idx = threadIdx.x; idx < ncol * rows; idx += NT) {
        const int col = idx / rows;
        const int row = idx - col * rows;
        Y[(ybase + col) * p.ldy + row0 + row] = acc[col * ldl + row];
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

template <typename T, int KP16, int WAVES>
hipError_t gg_launch_t(const GGParams& p, int blocks, size_t lds, hipStream_t st) {
    static size_t attr_set = 0;
    if (lds > 65536 && lds > attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gg_kernel<T, KP16, WAVES>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = lds;
    }
    hipLaunchKernelGGL((gg_kernel<T, KP16, WAVES>), dim3(blocks), dim3(64 * WAVES), lds, st, p);
    return hipGetLastError();
}

template <typename T, int WAVES>
hipError_t gg_dispatch(int KP16, const GGParams& p, int blocks, size_t lds, hipStream_t st) {
    switch (KP16) {
#define KIFMM_GG_CASE(K) \
    case K:              \
        return gg_launch_t<T, K, WAVES>(p, blocks, lds, st);
        KIFMM_GG_CASE(1) KIFMM_GG_CASE(2) KIFMM_GG_CASE(3) KIFMM_GG_CASE(4) KIFMM_GG_CASE(5)
        KIFMM_GG_CASE(6) KIFMM_GG_CASE(7) KIFMM_GG_CASE(8) KIFMM_GG_CASE(9) KIFMM_GG_CASE(10)
        KIFMM_GG_CASE(11) KIFMM_GG_CASE(12) KIFMM_GG_CASE(13) KIFMM_GG_CASE(14) KIFMM_GG_CASE(15)
        KIFMM_GG_CASE(16) KIFMM_GG_CASE(17) KIFMM_GG_CASE(18) KIFMM_GG_CASE(19)
#undef KIFMM_GG_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t gg_variant(int variant, int KP16, const GGParams& p, int blocks, size_t lds, hipStream_t st) {
    switch (variant) {
        case 0: return gg_dispatch<T, 8>(KP16, p, blocks, lds, st);
        case 1: return gg_dispatch<T, 4>(KP16, p, blocks, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int gg_variant_rows(int variant) {
    switch (variant) {
        case 0: return 8 * 16;
        case 1: return 4 * 16;
        default: return 0;
    }
}

size_t gg_lds_limit() { return 160 * 1024; }

size_t gg_lds_bytes(int elt, int variant, int KP16, int cols) {
    return ((size_t)2 * 32 * (KP16 * 16 + 4) + (size_t)cols * (gg_variant_rows(variant) + 4)) * elt;
}

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
    p.n_tiles = s.n_tiles;
    const int mbg = gg_variant_rows(s.variant) / 16;
    if (mbg == 0 || s.cp * R != 32) return hipErrorInvalidValue;
    p.n_rg = (MB + mbg - 1) / mbg;
    p.tile_tgt0 = s.tile_tgt0;
    p.tile_ntgt = s.tile_ntgt;
    p.tile_chunk0 = s.tile_chunk0;
    p.chunk_cls = s.chunk_cls;
    p.chunk_next = s.chunk_next;
    p.chunk_nblk = s.chunk_nblk;
    p.chunk_scale = s.chunk_scale;
    p.chunk_src = s.chunk_src;
    p.chunk_col = s.chunk_col;
    const size_t lds = gg_lds_bytes(elt, s.variant, KP16, s.max_tile * R);
    if (lds > gg_lds_limit() || KP16 < 1 || KP16 > 19) return hipErrorInvalidValue;
    const int blocks = (s.n_tiles + 7) / 8 * 8 * p.n_rg;
    if (elt == 4) return gg_variant<float>(s.variant, KP16, p, blocks, lds, st);
    return gg_variant<double>(s.variant, KP16, p, blocks, lds, st);
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
