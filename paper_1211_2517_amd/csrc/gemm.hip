// Grouped gather GEMM kernels of the KIFMM evaluation for gfx950 (CDNA4, wave64).
//
// gg_kernel      grouped gather GEMM on MFMA: the S2M/L2T reduced-operator
//                products (Sec. 3.3), M2M and L2L (Sec. 2.2 and their reduced forms) and the
//                compressed M2L (Sec. 3.1, K~ applied with the homogeneous level scaling).
// rs_kernel      row-slab form of the same product (FP32 data): every wave
//                loads its own operands and owns its rows of the accumulator.
// gd_kernel      the same product when every target has one pair (direct form).
// The point evaluations (surface potentials, near and far fields, M2T, S2L)
// are in eval.hip.
#include "kernels.h"

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#ifndef GG_XCD_RUN
#define GG_XCD_RUN 1
#endif
#ifndef GG_GD
#define GG_GD 3
#endif
#ifndef GG_LA
#define GG_LA 2
#endif
#ifndef GG_TSMALL
#define GG_TSMALL (KP16 > 1 ? 1 : 0)
#endif
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


struct GGParams {
    const void* A;
    int64_t a_stride;
    int lda;
    int a_rows, a_cols;   // rows and columns of A that hold data (the rest is zero)
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
    int xcd_run;     // consecutive tiles given to one XCD
    int nbuf;        // LDS staging buffers (2: double buffer; 1: wide K in FP64)
    int trash_col;   // first of R accumulator columns that take the products of empty slots
    // extents (bytes) of the buffer resources: loads past them return zero
    uint32_t x_bytes, a_bytes, meta_bytes, list_bytes;
    const int32_t* tile_tgt0;
    const int32_t* tile_ntgt;
    const int32_t* tile_chunk0;
    const int32_t* chunk_meta;   // per chunk: class, 16-column blocks, scale (bits, 1 or 2 words)
    const int32_t* chunk_src;
    const int32_t* chunk_col;
};

// Loads through the constant address space: with a wave-uniform index the
// compiler emits scalar loads. Used only outside the chunk loop.
template <typename T>
__device__ __forceinline__ T uload(const void* base, int idx) {
    typedef const T __attribute__((address_space(4))) CT;
    return reinterpret_cast<CT*>(reinterpret_cast<uintptr_t>(base))[idx];
}

// A lane offset at or past every buffer extent: the load returns zero and
// makes no memory request (used for zero padding and empty slots).
constexpr uint32_t kOffNone = 0x80000000u;

// Word 3 of a raw buffer resource (32-bit data format; offsets are checked
// against the record count, out-of-range loads return zero).
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}

// 4-vector load through a buffer resource at byte offset voff + soff.
template <typename T>
__device__ __forceinline__ typename Mfma<T>::V4 bload4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ f32x4 bload4<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ f64x4 bload4<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    typedef int i32x8 __attribute__((ext_vector_type(8)));
    const i32x4 lo = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    const i32x4 hi = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0));
    const i32x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(f64x4, v);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));

// 2-wide load through a buffer resource (the last K-chunk of the trimmed form).
__device__ __forceinline__ float2 bload2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// A 2-vector as the first two elements of a 4-vector (the other two undefined).
__device__ __forceinline__ f32x4 widen2(f32x2 v) { return __builtin_shufflevector(v, v, 0, 1, -1, -1); }

__device__ __forceinline__ int bload1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}

// Split-BF16 product of one 32-wide K-chunk on v_mfma_f32_16x16x32_bf16:
// d += ah*bh + ah*bl + al*bh, where (ah, al) and (bh, bl) are the high and low
// BF16 parts of A and B (x = hi + lo + O(2^-16 |x|)); the dropped al*bl term
// is of the same order. Lane l supplies A[l%16][8*(l/16) + j] and
// B[8*(l/16) + j][l%16], j = 0..7, and holds D[4*(l/16) + q][l%16] as in the
// FP32 form.
__device__ __forceinline__ f32x4 mfma_b3(f32x4 ah, f32x4 al, f32x4 bh, f32x4 bl, f32x4 d) {
    typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
    const bf8 AH = __builtin_bit_cast(bf8, ah), AL = __builtin_bit_cast(bf8, al);
    const bf8 BH = __builtin_bit_cast(bf8, bh), BL = __builtin_bit_cast(bf8, bl);
    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, BH, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BL, d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BH, d, 0, 0, 0);
    return d;
}

// The same three products into two accumulators (da += al*bh + ah*bh,
// db += ah*bl), so that consecutive MFMAs of one block do not all wait for
// each other's results.
__device__ __forceinline__ void mfma_b3x(f32x4 ah, f32x4 al, f32x4 bh, f32x4 bl, f32x4& da, f32x4& db) {
    typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
    const bf8 AH = __builtin_bit_cast(bf8, ah), AL = __builtin_bit_cast(bf8, al);
    const bf8 BH = __builtin_bit_cast(bf8, bh), BL = __builtin_bit_cast(bf8, bl);
    da = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, BH, da, 0, 0, 0);
    db = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BL, db, 0, 0, 0);
    da = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, BH, da, 0, 0, 0);
}

// High and low BF16 parts (round to nearest even) of 4 floats, packed two per word.
__device__ __forceinline__ void split_bf16(const f32x4& v, uint2& hi, uint2& lo) {
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    const bf2 h01 = __builtin_convertvector(f2{v[0], v[1]}, bf2);
    const bf2 h23 = __builtin_convertvector(f2{v[2], v[3]}, bf2);
    const f2 r01 = f2{v[0], v[1]} - __builtin_convertvector(h01, f2);
    const f2 r23 = f2{v[2], v[3]} - __builtin_convertvector(h23, f2);
    hi = uint2{__builtin_bit_cast(uint32_t, h01), __builtin_bit_cast(uint32_t, h23)};
    lo = uint2{__builtin_bit_cast(uint32_t, __builtin_convertvector(r01, bf2)),
               __builtin_bit_cast(uint32_t, __builtin_convertvector(r23, bf2))};
}

// Scheduling pattern for an MFMA sequence of N K-chunks: DS0 LDS reads first,
// then per K-chunk MF MFMAs, DS LDS reads (operands of a later K-chunk; none
// in the last LA chunks) and LD vector-memory reads, so that loads issued
// inside the sequence stay spread over it instead of leaving in one burst.
template <int N, int LA, int MF, int DS, int LD>
__device__ __forceinline__ void sched_chain() {
    if constexpr (N > 0) {
        __builtin_amdgcn_sched_group_barrier(0x008, MF, 0);
        if constexpr (N > LA) __builtin_amdgcn_sched_group_barrier(0x100, DS, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, LD, 0);
        sched_chain<N - 1, LA, MF, DS, LD>();
    }
}
template <int N, int LA, int MF, int DS, int LD>
__device__ __forceinline__ void sched_interleave() {
    __builtin_amdgcn_sched_group_barrier(0x100, DS * LA, 0);
    sched_chain<N, LA, MF, DS, LD>();
}

template <typename T>
__device__ __forceinline__ T meta_scale(int lo, int hi);
template <>
__device__ __forceinline__ float meta_scale<float>(int lo, int) { return __int_as_float(lo); }
template <>
__device__ __forceinline__ double meta_scale<double>(int lo, int hi) {
    return __hiloint2double(hi, lo);
}

// Grouped gather GEMM: Y[t] (+)= scale * sum_chunks A[cls] X[src].
//
// A workgroup owns one (tile, row group): the targets of the tile and
// WAVES*MBW 16-row blocks of the output, MBW per wave. Its accumulator (rows x
// ntgt*R columns) lives in LDS. The chunks of a tile are sorted by class; a chunk
// holds up to 32 columns (two 16-column MFMA blocks, the second one only when
// used) of one class. The chunk loop is a software pipeline; while the MFMAs of
// chunk c run, the workgroup has in flight
//   - the gathered source columns of chunks c+1 .. c+GD (all threads, into
//     register sets; chunk c+1's are stored to the other LDS staging buffer
//     after the MFMAs),
//   - the A rows of chunk c+1 for each wave (second register set),
//   - the target columns of chunk c+1, the metadata of chunk c+3 and the
//     source rows of chunk c+GD+2.
// A value is first needed one iteration after the one that loads it (A rows,
// target columns, source rows) or two (gathers, metadata).
// Every load of the loop is a buffer load with a lane offset fixed for the
// kernel and a scalar offset per chunk (little address arithmetic), issued
// in the same order each iteration, so the waits retire exactly the loads
// that are needed next; the loop has no scalar loads, whose out-of-order
// returns would share the LDS counter and stall the MFMAs' operand reads.
// One barrier per chunk.
// Empty slots of a chunk gather row 0 (a valid row) and add their products
// into R spare accumulator columns that are never stored. Within a chunk the
// real target columns are distinct and each wave owns its rows, so no two
// lanes or waves update the same live LDS word at the same time and the
// summation order is fixed (results are bitwise reproducible).
//
// MFMA operand layout (v_mfma_*_16x16x4): lane l supplies A[l%16][kk] and
// B[kk][l%16] of one K-step and holds D[Mfma<T>::row(q, l/16)][l%16]. The K
// order is permuted so that both operands are read as 4-wide vectors: in
// K-chunk t, lane group g = l/16 supplies indices 16t + 4g + e for the 4
// consecutive MFMA steps e = 0..3.
//
// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Runs of xcd_run consecutive tiles go to one XCD, with the row groups of a
// tile next to each other: for k = b/8 and q = k/n_rg, block b is row group
// k % n_rg of tile ((q / xcd_run)*8 + b%8)*xcd_run + q % xcd_run. Tiles are
// Morton-ordered ranges of targets, so the row groups of a tile, and
// neighbouring tiles of a run, share their source columns in one L2.
//
// B3 (split BF16, FP32 data): A holds per row and 32-wide K-chunk c the 32
// high BF16 parts then the 32 low parts (the 128 bytes of two FP32 16-wide
// K-chunks); the staging converts the gathered FP32 columns into the same
// layout in LDS. Register sets and LDS addresses are those of the FP32 form;
// K-chunk pair (2c, 2c+1) of the FP32 form is (hi, lo) of 32-wide chunk c.
template <typename T, int KP16, int WAVES, int MBW, bool B3 = false, bool TAIL8 = false>
__global__ void __launch_bounds__(64 * WAVES, MBW == 1 ? 2 : 1) gg_kernel(GGParams p) {
    static_assert(!B3 || (sizeof(T) == 4 && KP16 % 2 == 0), "split BF16 needs FP32 data and 32-wide K-chunks");
    static_assert(!TAIL8 || (!B3 && sizeof(T) == 4 && KP16 >= 2 && KP16 * 4 <= 32),
                  "the trimmed last K-chunk exists in the FP32 pipelined form only");
    using M = Mfma<T>;
    using V4 = typename M::V4;
    constexpr int NT = 64 * WAVES;
    constexpr int KDIM = KP16 * 16;
    constexpr int LDB = KDIM + 4;          // LDS stride of one staged column
    constexpr int V4C = KDIM / 4;          // 4-vectors per staged column
    constexpr int NSV = 32 * V4C;          // 4-vectors staged per chunk
    constexpr int NLD = (NSV + NT - 1) / NT;
    // second A register set and both blocks' B operands read ahead, where the
    // registers allow it (256 per lane at two waves per SIMD, MBW = 1; 512 at
    // one wave per SIMD, MBW = 2)
    constexpr bool ADBL = KP16 * sizeof(T) <= 64;
    constexpr bool PRE2 = KP16 * sizeof(T) <= 32;
    const int b = blockIdx.x;
    const int kx = b >> 3;
    const int rg = kx % p.n_rg;
    const int q = kx / p.n_rg;
    const int tile = ((q / p.xcd_run) * 8 + (b & 7)) * p.xcd_run + q % p.xcd_run;
    if (tile >= p.n_tiles) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* bbuf = reinterpret_cast<T*>(smem_raw);   // [nbuf][32][LDB]
    T* acc = bbuf + p.nbuf * 32 * LDB;          // [ncol + R][ldl]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int mb_lo = rg * WAVES * MBW;
    const int nmb = min(WAVES * MBW, p.MB - mb_lo);
    const int rows = nmb * 16;
    const int ldl = WAVES * MBW * 16 + 4;
    const int R = p.R;
    const int cp = p.cp;
    const int t0 = uload<int32_t>(p.tile_tgt0, tile);
    const int ncol = uload<int32_t>(p.tile_ntgt, tile) * R;
    const int cb = uload<int32_t>(p.tile_chunk0, tile);
    const int ce = uload<int32_t>(p.tile_chunk0, tile + 1);
    T* __restrict__ Y = static_cast<T*>(p.Y);

    const int64_t ybase = (int64_t)t0 * R;
    const int row0 = mb_lo * 16;
    for (int idx = tid; idx < ncol * rows; idx += NT) {
        const int col = idx / rows;
        const int row = idx - col * rows;
        acc[col * ldl + row] = p.accumulate ? Y[(ybase + col) * p.ldy + row0 + row] : T(0);
    }
    if (cb >= ce) {
        __syncthreads();
        for (int idx = tid; idx < ncol * rows; idx += NT) {
            const int col = idx / rows;
            Y[(ybase + col) * p.ldy + row0 + idx - col * rows] = acc[col * ldl + idx - col * rows];
        }
        return;
    }

    const int j = lane & 15;
    const int grp = lane >> 4;
    // a wave works when its first row block holds output rows; a second row
    // block past the last one reads a valid row of A and accumulates into LDS
    // rows that are never stored
    const bool wact = wave * MBW < nmb;
    // buffer resources: every load of the chunk loop takes a 32-bit lane
    // offset that is fixed for the kernel plus a scalar offset per chunk
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(p.X, p.x_bytes);
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(p.A, p.a_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(p.chunk_meta, p.meta_bytes);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(p.chunk_src, p.list_bytes);
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(p.chunk_col, p.list_bytes);
    // A loads skip the zero padding: rows past a_rows, and the 4-wide K pieces
    // past a_cols (only the last K-chunk can hold those)
    uint32_t aoff[MBW], aofl[MBW];
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
        const int blk = min(wave * MBW + m, nmb - 1);
        const int row = row0 + blk * 16 + j;
        aoff[m] = row < p.a_rows ? (uint32_t)((row * p.lda + 4 * grp) * (int)sizeof(T)) : kOffNone;
        if constexpr (TAIL8)
            aofl[m] = (row < p.a_rows && 16 * (KP16 - 1) + 2 * grp < p.a_cols)
                          ? (uint32_t)((row * p.lda + 16 * (KP16 - 1) + 2 * grp) * (int)sizeof(T)) : kOffNone;
        else
            aofl[m] = (row < p.a_rows && (B3 || 16 * (KP16 - 1) + 4 * grp < p.a_cols))
                          ? aoff[m] + 16 * (KP16 - 1) * (int)sizeof(T) : kOffNone;
    }
    // TAIL8: the data end within 8 of the last K-chunk's start, so that
    // K-chunk is read as 2-vectors (k = 16 (KP16-1) + 2 g + e, e = 0, 1, in
    // the first two elements; the other two are never read) and takes two
    // MFMA steps instead of four: lane group g supplies the same k for A and B.
    auto a_last = [&](uint32_t off, uint32_t so) -> V4 {
        if constexpr (TAIL8) {
            return widen2(__builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(ra, off, so, 0)));
        } else {
            return bload4<T>(ra, off, so);
        }
    };
    const uint32_t a_cls_bytes = (uint32_t)(p.a_stride * (int64_t)sizeof(T));
    const uint32_t xrow_bytes = (uint32_t)(R * p.ldx * (int)sizeof(T));

    // staging map: 4-vector f = i*NT + tid of the chunk is part f % V4C of
    // staged column f / V4C (pair f / V4C / R, right-hand side f / V4C % R).
    // Threads past the end repeat the last 4-vector (identical stores).
    int spair[NLD], soff[NLD];   // soff: FP32 offset, or (B3) offset of the high parts
    uint32_t xoff[NLD];
    bool xpad[NLD];     // 4-vector entirely in the zero padding past a_cols
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int f = min(i * NT + tid, NSV - 1);
        const int c = f / V4C;
        spair[i] = c / R;
        const int rhs = c - spair[i] * R;
        const int part = 4 * (f - c * V4C);
        soff[i] = B3 ? c * LDB + (part / 32) * 32 + (part % 32) / 2 : c * LDB + part;
        xoff[i] = (uint32_t)((rhs * p.ldx + part) * (int)sizeof(T));
        xpad[i] = part >= p.a_cols;
    }
    const int pj16 = j / R;
    const int rj = j - pj16 * R;
    const int colb1 = 16 / R;   // pair index of the first column of block 1

    // pipeline state entering the iteration of chunk c: the class, block count
    // and scale of chunks c and c+1 (scalars), the gathered columns of chunks
    // c+1 .. c+GD-1 (in flight), and in two sets of registers by chunk parity
    // (set (x - cb) & 1 for chunk x) the metadata words of chunks c+2 and c+3,
    // the target columns of chunks c and c+1 and the source rows of chunks
    // c+GD and c+GD+1. A loaded value stays in the register its load wrote
    // until it is used: a register copy of a value still in flight would make
    // the copy wait for it, and with it for every load issued before it.
    struct Ring {
        int src[NLD];   // source rows of a chunk
        int meta;       // metadata word of a chunk (lanes 0..3)
        int col0, col1; // target columns of this lane in a chunk (blocks 0 and 1)
    };
    Ring ring[2];
    int cls_c, nb_c, cls_n, nb_n;
    T sc_c, sc_n;
    // gathered columns: GD = 3 or 4 chunks ahead in four register sets (chunk
    // index mod 4) in the FP32 8-wave shape up to K = 224 (measured: 8% faster
    // than GD = 2 there, slower in the 4-wave shapes, whose waves issue twice
    // the gathers), else GD = 2 in two sets (chunk parity)
    constexpr bool SETS4_FIT = sizeof(T) == 4 && WAVES == 8 && KP16 <= 14;
    constexpr int GD = SETS4_FIT ? GG_GD : 2;
    static_assert(GD >= 2 && GD <= 4, "gather distance");
    constexpr int FILL = GD == 2 ? 2 : 4;   // pipeline-fill iterations before chunk cb
    V4 g0[NLD], g1[NLD], g2[GD > 2 ? NLD : 1], g3[GD > 2 ? NLD : 1];
    V4 a0[MBW][KP16];
    V4 a1[ADBL ? MBW : 1][KP16];

    // metadata of a chunk: lanes 0..3 load its four words (a vector load), then
    // they are broadcast to scalars once the loads have drained
    auto load_meta = [&](int ch) { return bload1(rm, 4 * (lane & 3), 16 * ch); };
    auto unpack_meta = [&](int v, int& cls, int& nb, T& sc) {
        cls = __builtin_amdgcn_readlane(v, 0);
        nb = __builtin_amdgcn_readlane(v, 1);
        sc = meta_scale<T>(__builtin_amdgcn_readlane(v, 2), __builtin_amdgcn_readlane(v, 3));
    };
    auto load_src = [&](int ch, int (&dst)[NLD]) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) dst[i] = bload1(rs, 4 * spair[i], 4 * ch * cp);
    };
    auto gather = [&](V4 (&dst)[NLD], const int (&src)[NLD]) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const uint32_t off = (src[i] < 0 || xpad[i]) ? kOffNone
                                                         : (uint32_t)__umul24((uint32_t)src[i], xrow_bytes) + xoff[i];
            dst[i] = bload4<T>(rx, off, 0);
        }
    };
    auto stage_store = [&](int buf, const V4 (&v)[NLD]) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            if constexpr (B3) {
                uint2 hi, lo;
                split_bf16(v[i], hi, lo);
                *reinterpret_cast<uint2*>(bbuf + buf * 32 * LDB + soff[i]) = hi;
                *reinterpret_cast<uint2*>(bbuf + buf * 32 * LDB + soff[i] + 16) = lo;
            } else {
                *reinterpret_cast<V4*>(bbuf + buf * 32 * LDB + soff[i]) = v[i];
            }
        }
    };
    auto load_a = [&](V4 (&dst)[MBW][KP16], int cls) {
        const uint32_t so = (uint32_t)cls * a_cls_bytes;
#pragma unroll
        for (int m = 0; m < MBW; ++m) {
#pragma unroll
            for (int t = 0; t < KP16 - 1; ++t) dst[m][t] = bload4<T>(ra, aoff[m] + 16 * t * (int)sizeof(T), so);
            dst[m][KP16 - 1] = a_last(aofl[m], so);
        }
    };
    auto tcol = [&](int ch, int& c0, int& c1) {
        c0 = bload1(rc, 4 * pj16, 4 * ch * cp);
        c1 = bload1(rc, 4 * (colb1 + pj16), 4 * ch * cp);
    };
    // accumulator column `col` at this wave's rows; empty slots go to the spare columns
    auto acc_ptr = [&](int col) {
        return acc + ((col >= 0 ? col : p.trash_col) * R + rj) * ldl + wave * MBW * 16;
    };

    // acc[col][rows of this wave] += scale * (u + v), read-modify-write of one
    // lane's 4 accumulator elements
    auto acc_add = [&](T* ptr, const V4& u, const V4& v, T scale) {
        if constexpr (sizeof(T) == 4) {
            V4* q4 = reinterpret_cast<V4*>(ptr + 4 * grp);   // rows 4*grp .. 4*grp+3
            const V4 o = *q4;
            V4 r;
#pragma unroll
            for (int q = 0; q < 4; ++q) r[q] = __builtin_fmaf(scale, u[q] + v[q], o[q]);
            *q4 = r;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) ptr[M::row(q, grp)] = __builtin_fma(scale, u[q] + v[q], ptr[M::row(q, grp)]);
        }
    };

    // MFMAs of one chunk whose B operands sit in LDS buffer `buf`: for each of
    // the wave's MBW row blocks and each 16-column block, two accumulation
    // chains over K (even and odd K-chunks). `on` (uniform) says whether the
    // chunk is computed; hook(t) runs in every case, in one code path, so that
    // the loads it issues write their registers directly (a load issued on
    // two branches would need a register copy at the join, and the copy a
    // wait for the load).
    //
    // PRE2 shapes issue their memory traffic inside the MFMA sequence, in
    // program order between fences (sched_barrier), so that the loads of all
    // waves reach the memory pipelines spread over the MFMAs instead of in one
    // burst after the barrier: the LDS operands LA K-chunks ahead of their use,
    // and after K-chunk t the call hook(t) (the A rows of the next chunk and
    // this iteration's other loads). Other shapes call hook(t) for every t
    // before the MFMAs.
    constexpr int LA = GG_LA;
    auto mfma_chunk = [&](int buf, const V4 (&a)[MBW][KP16], const Ring& cur, bool on, auto&& hook) {
        const T* bcol = bbuf + (buf * 32 + j) * LDB + 4 * grp;
        const T scale = sc_c;
        // metadata word 1: 16-column blocks holding data, and (bits 8..) the
        // K-chunks holding data when fewer than KP16 (stage-2 factors of rank
        // below the padded rank); the other K-chunks multiply zeros only
        // (read only for K up to 96, the padded stage-2 ranks; wider kernels
        // always run every K-chunk, which multiplies zeros there)
        const bool two = on && (nb_c & 0xff) > 1;
        const int kc = (KP16 <= 6 && (nb_c >> 8)) ? (nb_c >> 8) : KP16;
        if constexpr (PRE2) {
            V4 b0[KP16], b1[KP16];
            // B operand of K-chunk t for column block cb (the trimmed last
            // K-chunk: 2-vectors at k = 16 (KP16-1) + 2 g, as for A)
            auto ldsb = [&](int cbk, int t) -> V4 {
                if constexpr (TAIL8) {
                    if (t == KP16 - 1)
                        return widen2(*reinterpret_cast<const f32x2*>(bcol + cbk * 16 * LDB + 16 * t - 2 * grp));
                }
                return *reinterpret_cast<const V4*>(bcol + cbk * 16 * LDB + 16 * t);
            };
#pragma unroll
            for (int t = 0; t < LA && t < KP16; ++t) {
                b0[t] = ldsb(0, t);
                b1[t] = ldsb(1, t);
            }
            V4 d[MBW][4];
#pragma unroll
            for (int m = 0; m < MBW; ++m)
#pragma unroll
                for (int q = 0; q < 4; ++q) d[m][q] = V4{0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < KP16; ++t) {
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (B3) {
                    if (t & 1) {
                        if (two) {
#pragma unroll
                            for (int m = 0; m < MBW; ++m) {
                                mfma_b3x(a[m][t - 1], a[m][t], b0[t - 1], b0[t], d[m][0], d[m][1]);
                                mfma_b3x(a[m][t - 1], a[m][t], b1[t - 1], b1[t], d[m][2], d[m][3]);
                            }
                        } else if (on) {
#pragma unroll
                            for (int m = 0; m < MBW; ++m) mfma_b3x(a[m][t - 1], a[m][t], b0[t - 1], b0[t], d[m][0], d[m][1]);
                        }
                    }
                } else {
                    // two accumulation chains per block (step parity), so that
                    // consecutive MFMAs of a block are independent
                    constexpr int NE = TAIL8 ? 2 : 4;   // MFMA steps of the last K-chunk
                    if (two && t < kc) {
#pragma unroll
                        for (int e = 0; e < (t == KP16 - 1 ? NE : 4); ++e) {
#pragma unroll
                            for (int m = 0; m < MBW; ++m) {
                                d[m][e & 1] = M::step(a[m][t][e], b0[t][e], d[m][e & 1]);
                                d[m][2 + (e & 1)] = M::step(a[m][t][e], b1[t][e], d[m][2 + (e & 1)]);
                            }
                        }
                    } else if (on && t < kc) {
#pragma unroll
                        for (int e = 0; e < (t == KP16 - 1 ? NE : 4); ++e) {
#pragma unroll
                            for (int m = 0; m < MBW; ++m) d[m][e & 1] = M::step(a[m][t][e], b0[t][e], d[m][e & 1]);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                if (t + LA < KP16) {
                    b0[t + LA] = ldsb(0, t + LA);
                    b1[t + LA] = ldsb(1, t + LA);
                }
                hook(t);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (on) {
                T* p0 = acc_ptr(cur.col0);
#pragma unroll
                for (int m = 0; m < MBW; ++m) acc_add(p0 + 16 * m, d[m][0], d[m][1], scale);
            }
            if (two) {
                T* p1 = acc_ptr(cur.col1);
#pragma unroll
                for (int m = 0; m < MBW; ++m) acc_add(p1 + 16 * m, d[m][2], d[m][3], scale);
            }
        } else {
#pragma unroll
            for (int t = 0; t < KP16; ++t) hook(t);
            if (on) {
                for (int blk = 0; blk < (nb_c & 0xff); ++blk) {
                    V4 d[MBW][2];
#pragma unroll
                    for (int m = 0; m < MBW; ++m) d[m][0] = d[m][1] = V4{0, 0, 0, 0};
                    if constexpr (B3) {
#pragma unroll
                        for (int t = 0; t < KP16; t += 2) {
                            const V4 bh = *reinterpret_cast<const V4*>(bcol + blk * 16 * LDB + 16 * t);
                            const V4 bl = *reinterpret_cast<const V4*>(bcol + blk * 16 * LDB + 16 * (t + 1));
#pragma unroll
                            for (int m = 0; m < MBW; ++m)
                                d[m][(t >> 1) & 1] = mfma_b3(a[m][t], a[m][t + 1], bh, bl, d[m][(t >> 1) & 1]);
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < KP16; ++t) {
                            if (t < kc) {
                                const V4 bv = *reinterpret_cast<const V4*>(bcol + blk * 16 * LDB + 16 * t);
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
#pragma unroll
                                    for (int m = 0; m < MBW; ++m) d[m][t & 1] = M::step(a[m][t][e], bv[e], d[m][t & 1]);
                                }
                            }
                        }
                    }
                    T* pp = acc_ptr(blk ? cur.col1 : cur.col0);
#pragma unroll
                    for (int m = 0; m < MBW; ++m) acc_add(pp + 16 * m, d[m][0], d[m][1], scale);
                }
            }
        }
    };

    // The loop starts FILL chunks early, at c = cb-FILL: those iterations
    // only fill the pipeline (chunk indices are clamped into the tile, their
    // MFMAs are skipped), so every load of the loop is issued by the same code
    // in the same order, and the wait counts are the same on every iteration.
    // A clamped chunk index past the last chunk only repeats valid loads.
    auto clampc = [&](int ch) { return min(max(ch, cb), ce - 1); };
    static_assert(FILL % 2 == 0, "the first iteration has parity 0");
    unpack_meta(load_meta(cb), cls_n, nb_n, sc_n);
    ring[0].meta = load_meta(cb);
    ring[1].meta = 0;
    cls_c = -1;
    nb_c = 0;
    sc_c = T(0);
    ring[0].col0 = ring[0].col1 = ring[1].col0 = ring[1].col1 = -1;
    load_src(clampc(cb - FILL + GD), ring[GD & 1].src);
    load_src(clampc(cb - FILL + GD + 1), ring[(GD + 1) & 1].src);
    // drain the prologue's loads (s_waitcnt vmcnt(0)), so that the wait
    // counts computed for the loop follow its steady state only
    __builtin_amdgcn_s_waitcnt(0x0F70);

    // one iteration: chunk ch with its A rows in `a`; `an` receives chunk
    // ch+1's rows, `gi` holds chunk ch+1's gathered columns (in flight) and
    // `go` receives chunk ch+GD's. `cur` is the ring set of chunk ch's parity.
    auto step = [&](int ch, int buf, V4 (&a)[MBW][KP16], V4 (&an)[MBW][KP16], V4 (&gi)[NLD], V4 (&go)[NLD],
                    Ring& cur, Ring& oth) {
        // Every iteration issues the same loads in the same order (the A rows
        // of the next chunk are loaded even when its class is unchanged; they
        // then come from L2): vmcnt retires loads in issue order, so with a
        // fixed sequence each wait covers exactly the loads it needs, while a
        // data-dependent load count would make the compiler's waits drain
        // loads issued in the same iteration. The order is: the A rows of chunk
        // c+1, K-chunk by K-chunk (hook(t), spread over the MFMAs; needed by
        // the next iteration's MFMAs), with the gathers of chunk c+GD (stored
        // at the end of iteration c+GD-1) and the indices consumed one or two
        // iterations later issued after K-chunk GG_TSMALL. So no wait ever
        // retires a load of its own iteration that it does not need.
        // source rows of chunk ch+GD (used here), reloaded with those of
        // chunk ch+GD+2 (same parity)
        int (&sq)[NLD] = (GD % 2 == 0) ? cur.src : oth.src;
        auto hook = [&](int t) {
            if (ADBL) {
                const uint32_t so = (uint32_t)cls_n * a_cls_bytes;
#pragma unroll
                for (int m = 0; m < MBW; ++m)
                    an[m][t] = t == KP16 - 1 ? a_last(aofl[m], so) : bload4<T>(ra, aoff[m] + 16 * t * (int)sizeof(T), so);
            }
            // the gathers and the small loads (source rows, metadata, target
            // columns) go out right after the first K-chunks' MFMAs, so they
            // have most of an extra iteration to return (issued after the last
            // K-chunk they left the next iteration waiting on memory latency)
            if (t == GG_TSMALL) {
                gather(go, sq);
                load_src(clampc(ch + GD + 2), sq);
                oth.meta = load_meta(clampc(ch + 3));
                tcol(clampc(ch + 1), oth.col0, oth.col1);
            }
        };
        // with one staging buffer every chunk uses buffer 0, and the store of
        // the next chunk waits until all waves have read the current one
        const bool one = p.nbuf == 1;
        mfma_chunk(one ? 0 : buf, a, cur, wact && ch >= cb && ch < ce, hook);
        if (one) __syncthreads();
        stage_store(one ? 0 : buf ^ 1, gi);
        if (!ADBL && cls_n != cls_c) load_a(a, cls_n);
        cls_c = cls_n;
        nb_c = nb_n;
        sc_c = sc_n;
        unpack_meta(cur.meta, cls_n, nb_n, sc_n);   // chunk ch+2
        __syncthreads();
    };
    // all iterations of the unrolled group always run (up to three past the
    // last chunk; their MFMAs are skipped), so the loop has a single back edge
    // and the wait counts stay exact. Iteration ch stores the gathers of chunk
    // ch+1 (set (ch+1-cb) mod 4) and issues those of chunk ch+GD.
    if constexpr (GD == 2) {
        if constexpr (ADBL) {
            for (int ch = cb - FILL; ch < ce; ch += 2) {
                step(ch, 0, a0, a1, g1, g0, ring[0], ring[1]);
                step(ch + 1, 1, a1, a0, g0, g1, ring[1], ring[0]);
            }
        } else {
            for (int ch = cb - FILL; ch < ce; ch += 2) {
                step(ch, 0, a0, a0, g1, g0, ring[0], ring[1]);
                step(ch + 1, 1, a0, a0, g0, g1, ring[1], ring[0]);
            }
        }
    } else {
        // four sets: chunk ch0 + i (ch0 the first chunk of an unrolled group)
        // has its gathers in set i mod 4
        auto gs = [&](auto idx) -> V4 (&)[NLD] {
            constexpr int i = decltype(idx)::value % 4;
            if constexpr (i == 0)
                return g0;
            else if constexpr (i == 1)
                return g1;
            else if constexpr (i == 2)
                return g2;
            else
                return g3;
        };
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        using G0 = std::integral_constant<int, GD>;
        using G1 = std::integral_constant<int, GD + 1>;
        using G2 = std::integral_constant<int, GD + 2>;
        using G3 = std::integral_constant<int, GD + 3>;
        if constexpr (ADBL) {
            for (int ch = cb - FILL; ch < ce; ch += 4) {
                step(ch, 0, a0, a1, gs(I1{}), gs(G0{}), ring[0], ring[1]);
                step(ch + 1, 1, a1, a0, gs(I2{}), gs(G1{}), ring[1], ring[0]);
                step(ch + 2, 0, a0, a1, gs(I3{}), gs(G2{}), ring[0], ring[1]);
                step(ch + 3, 1, a1, a0, gs(I4{}), gs(G3{}), ring[1], ring[0]);
            }
        } else {
            for (int ch = cb - FILL; ch < ce; ch += 4) {
                step(ch, 0, a0, a0, gs(I1{}), gs(G0{}), ring[0], ring[1]);
                step(ch + 1, 1, a0, a0, gs(I2{}), gs(G1{}), ring[1], ring[0]);
                step(ch + 2, 0, a0, a0, gs(I3{}), gs(G2{}), ring[0], ring[1]);
                step(ch + 3, 1, a0, a0, gs(I4{}), gs(G3{}), ring[1], ring[0]);
            }
        }
    }
    for (int idx = tid; idx < ncol * rows; idx += NT) {
        const int col = idx / rows;
        const int row = idx - col * rows;
        Y[(ybase + col) * p.ldy + row0 + row] = acc[col * ldl + row];
    }
}

// Row-slab grouped gather GEMM (FP32 data; FP32 MFMA, or split BF16 with B3):
// the product of gg_kernel, Y[t] (+)= scale * sum_chunks A[cls] X[src], on the
// same tiles, chunks and workgroup-to-XCD mapping, organised so that the waves
// of a workgroup never wait for each other.
//
// Wave w owns MBW 16-row blocks of the row group and, in the LDS accumulator,
// those rows of every target column of the tile; it walks the tile's chunks
// on its own. For each chunk it takes its rows of A[cls] and the chunk's
// gathered source columns straight from memory into MFMA operand registers
// (no staging in LDS), and adds its 16*MBW x 32 product into its own rows of
// the accumulator. Waves share no LDS words, so the kernel has no barrier; the
// four waves' gathers of a chunk meet in the CU's vector L1.
//
// Pipeline: the operands of chunk c+1 are loaded while the MFMAs of chunk c
// run, K-chunk by K-chunk into the registers that K-chunk t of chunk c has just
// finished with (one register set). Chunk metadata, source rows and target
// columns are vector loads issued one to three chunks ahead, in two register
// sets by chunk parity, so every value stays in the register its load wrote
// and every iteration issues the same loads in the same order (the waits then
// retire exactly the loads that are needed).
//
// Operand layout (v_mfma_f32_16x16x4f32): lane l = 16 g + j supplies A[j][kk]
// and B[kk][j]; in K-chunk t the lane's 4-vector holds k = 16 t + 4 g + e for
// the MFMA steps e = 0..3. TAIL8: the data end within 8 of the last K-chunk's
// start, so that K-chunk is read as 2-vectors (k = 16 t + 2 g + e, e = 0, 1)
// and takes two MFMA steps instead of four.
// B3: A holds per row and 32-wide K-chunk c the 32 high BF16 parts, then the
// 32 low parts; register K-chunks (2c, 2c+1) are (hi, lo) of A's chunk c, and
// the lane's 8 gathered FP32 values k = 32 c + 8 g + i (i = 0..7, two
// 4-vectors) are split into BF16 high and low parts in registers; each 32-wide
// chunk is three v_mfma_f32_16x16x32_bf16 (hi*hi + hi*lo + lo*hi).
template <int KP16, int WAVES, int MBW, bool B3, bool TAIL8>
__global__ void __launch_bounds__(64 * WAVES, 1) rs_kernel(GGParams p) {
    static_assert(!B3 || (KP16 % 2 == 0 && !TAIL8), "split BF16 needs 32-wide K-chunks");
    using V4 = f32x4;
    constexpr int ROWS = WAVES * MBW * 16;
    constexpr int LDL = ROWS + 4;                // LDS stride of one accumulator column
    constexpr int KF = TAIL8 ? KP16 - 1 : KP16;  // K-chunks read as 4-vectors
    const int bid = blockIdx.x;
    const int kx = bid >> 3;
    const int rg = kx % p.n_rg;
    const int qq = kx / p.n_rg;
    const int tile = ((qq / p.xcd_run) * 8 + (bid & 7)) * p.xcd_run + qq % p.xcd_run;
    if (tile >= p.n_tiles) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* acc = reinterpret_cast<float*>(smem_raw);   // [ncol][LDL]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int mb_lo = rg * WAVES * MBW;
    const int nmb = min(WAVES * MBW, p.MB - mb_lo);
    // waves without output rows have nothing to do (there is no barrier)
    if (wave * MBW >= nmb) return;
    const int wr0 = wave * MBW * 16;                   // first row of this wave in the group
    const int wrows = min(MBW * 16, nmb * 16 - wr0);   // its rows that hold output
    const int R = p.R;
    const int cp = p.cp;
    const int t0 = uload<int32_t>(p.tile_tgt0, tile);
    const int ncol = uload<int32_t>(p.tile_ntgt, tile) * R;
    const int cb = uload<int32_t>(p.tile_chunk0, tile);
    const int ce = uload<int32_t>(p.tile_chunk0, tile + 1);
    float* __restrict__ Y = static_cast<float*>(p.Y);
    const int64_t ybase = (int64_t)t0 * R;
    const int row0 = mb_lo * 16;
    const int pieces = wrows / 4;
    for (int idx = lane; idx < ncol * pieces; idx += 64) {
        const int col = idx / pieces;
        const int r = wr0 + 4 * (idx - col * pieces);
        V4 v = V4{0, 0, 0, 0};
        if (p.accumulate) v = *reinterpret_cast<const V4*>(Y + (ybase + col) * p.ldy + row0 + r);
        *reinterpret_cast<V4*>(acc + col * LDL + r) = v;
    }

    if (cb < ce) {
        const int j = lane & 15;
        const int g = lane >> 4;
        const __amdgpu_buffer_rsrc_t rx = make_rsrc(p.X, p.x_bytes);
        const __amdgpu_buffer_rsrc_t ra = make_rsrc(p.A, p.a_bytes);
        const __amdgpu_buffer_rsrc_t rm = make_rsrc(p.chunk_meta, p.meta_bytes);
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(p.chunk_src, p.list_bytes);
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(p.chunk_col, p.list_bytes);
        // lane byte offsets of K-chunk t: A (both forms) and B (gathered columns)
        auto koff_a = [&](int t) -> uint32_t { return (uint32_t)(64 * t + 16 * g); };
        auto koff_b = [&](int t) -> uint32_t {
            return B3 ? (uint32_t)(128 * (t >> 1) + 32 * g + 16 * (t & 1)) : (uint32_t)(64 * t + 16 * g);
        };
        // K pieces wholly past a_cols hold zeros in A and X: not read
        auto kvalid = [&](int t) { return B3 ? true : (16 * t + 4 * g < p.a_cols); };
        const uint32_t ktail = (uint32_t)(64 * (KP16 - 1) + 8 * g);
        const bool tvalid = 16 * (KP16 - 1) + 2 * g < p.a_cols;
        uint32_t arow[MBW];
#pragma unroll
        for (int m = 0; m < MBW; ++m) {
            const int row = row0 + wr0 + 16 * m + j;
            arow[m] = row < p.a_rows ? (uint32_t)(row * p.lda * 4) : kOffNone;
        }
        const uint32_t a_cls_bytes = (uint32_t)(p.a_stride * 4);
        const uint32_t xrow_bytes = (uint32_t)(R * p.ldx * 4);
        // column 16 bb + j of a chunk: pair pj[bb] of the chunk, right-hand side rh[bb]
        int pj[2], rh[2];
        uint32_t xcol[2];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            pj[bb] = (16 * bb + j) / R;
            rh[bb] = 16 * bb + j - pj[bb] * R;
            xcol[bb] = (uint32_t)(rh[bb] * p.ldx * 4);
        }
        struct Ring {
            int src[2];   // source rows of a chunk (columns 16 bb + j)
            int col[2];   // target columns of a chunk
            int meta;     // metadata word (lane & 3) of a chunk
        };
        Ring ring[2];
        auto clampc = [&](int ch) { return min(max(ch, cb), ce - 1); };
        auto load_src = [&](int ch, int (&dst)[2]) {
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) dst[bb] = bload1(rs, 4 * pj[bb], 4 * ch * cp);
        };
        auto load_col = [&](int ch, int (&dst)[2]) {
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) dst[bb] = bload1(rc, 4 * pj[bb], 4 * ch * cp);
        };
        auto load_meta = [&](int ch) { return bload1(rm, 4 * (lane & 3), 16 * ch); };
        int cls_n, nb_c, nb_n;
        float sc_c, sc_n;
        auto unpack = [&](int v, int& cls, int& nb, float& sc) {
            cls = __builtin_amdgcn_readlane(v, 0);
            nb = __builtin_amdgcn_readlane(v, 1);
            sc = __int_as_float(__builtin_amdgcn_readlane(v, 2));
        };
        // operand registers of the chunk whose MFMAs run next
        V4 a[MBW][KF];
        V4 bq[2][KF];
        float2 at[TAIL8 ? MBW : 1], bt[TAIL8 ? 2 : 1];
        // pipeline fill: the loop starts two chunks early (those iterations
        // load and compute nothing new; chunk indices are clamped into the tile)
        {
            int v0 = load_meta(cb);
            ring[0].meta = v0;
            ring[1].meta = 0;
            load_src(cb, ring[1].src);
            ring[0].src[0] = ring[0].src[1] = -1;
            ring[0].col[0] = ring[0].col[1] = ring[1].col[0] = ring[1].col[1] = -1;
            __builtin_amdgcn_s_waitcnt(0x0F70);
            unpack(v0, cls_n, nb_n, sc_n);
            nb_c = 0;
            sc_c = 0.f;
        }
        // one iteration: the MFMAs of chunk ch (operands in a/bq), the loads of
        // chunk ch+1's operands, then the accumulation of chunk ch.
        auto step = [&](int ch, Ring& cur, Ring& oth) {
            const bool on = ch >= cb && ch < ce;
            const bool two = on && (nb_c & 0xff) > 1;
            const float scale = sc_c;
            V4 d[MBW][2][2];
#pragma unroll
            for (int m = 0; m < MBW; ++m)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb) d[m][bb][0] = d[m][bb][1] = V4{0, 0, 0, 0};
            const uint32_t aso = (uint32_t)cls_n * a_cls_bytes;   // class of chunk ch+1
            uint32_t bro[2];
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
                bro[bb] = oth.src[bb] < 0 ? kOffNone : (uint32_t)__umul24((uint32_t)oth.src[bb], xrow_bytes) + xcol[bb];
            auto small_loads = [&]() {
                load_src(clampc(ch + 2), cur.src);
                load_col(clampc(ch + 1), oth.col);
                oth.meta = load_meta(clampc(ch + 3));
            };
            if constexpr (B3) {
#pragma unroll
                for (int c2 = 0; c2 < KP16 / 2; ++c2) {
                    const int t = 2 * c2;
                    __builtin_amdgcn_sched_barrier(0);
                    if (on) {
                        f32x4 bh[2], bl[2];
#pragma unroll
                        for (int bb = 0; bb < 2; ++bb) {
                            uint2 h0, l0, h1, l1;
                            split_bf16(bq[bb][t], h0, l0);
                            split_bf16(bq[bb][t + 1], h1, l1);
                            bh[bb] = __builtin_bit_cast(f32x4, uint4{h0.x, h0.y, h1.x, h1.y});
                            bl[bb] = __builtin_bit_cast(f32x4, uint4{l0.x, l0.y, l1.x, l1.y});
                        }
                        if (two) {
#pragma unroll
                            for (int m = 0; m < MBW; ++m) {
                                mfma_b3x(a[m][t], a[m][t + 1], bh[0], bl[0], d[m][0][0], d[m][0][1]);
                                mfma_b3x(a[m][t], a[m][t + 1], bh[1], bl[1], d[m][1][0], d[m][1][1]);
                            }
                        } else {
#pragma unroll
                            for (int m = 0; m < MBW; ++m)
                                mfma_b3x(a[m][t], a[m][t + 1], bh[0], bl[0], d[m][0][0], d[m][0][1]);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = t; u < t + 2; ++u) {
#pragma unroll
                        for (int m = 0; m < MBW; ++m) a[m][u] = bload4<float>(ra, arow[m] + koff_a(u), aso);
#pragma unroll
                        for (int bb = 0; bb < 2; ++bb) bq[bb][u] = bload4<float>(rx, bro[bb] + koff_b(u), 0);
                    }
                    if (c2 == 0) small_loads();
                }
            } else {
#pragma unroll
                for (int t = 0; t < KF; ++t) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (two) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
#pragma unroll
                            for (int m = 0; m < MBW; ++m) {
                                d[m][0][e & 1] = Mfma<float>::step(a[m][t][e], bq[0][t][e], d[m][0][e & 1]);
                                d[m][1][e & 1] = Mfma<float>::step(a[m][t][e], bq[1][t][e], d[m][1][e & 1]);
                            }
                    } else if (on) {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
#pragma unroll
                            for (int m = 0; m < MBW; ++m)
                                d[m][0][e & 1] = Mfma<float>::step(a[m][t][e], bq[0][t][e], d[m][0][e & 1]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    const bool kv = kvalid(t);
#pragma unroll
                    for (int m = 0; m < MBW; ++m)
                        a[m][t] = bload4<float>(ra, kv ? arow[m] + koff_a(t) : kOffNone, aso);
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb) bq[bb][t] = bload4<float>(rx, kv ? bro[bb] + koff_b(t) : kOffNone, 0);
                    if (t == 0) small_loads();
                }
                if constexpr (TAIL8) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (two) {
#pragma unroll
                        for (int e = 0; e < 2; ++e)
#pragma unroll
                            for (int m = 0; m < MBW; ++m) {
                                d[m][0][e] = Mfma<float>::step(at[m][e], bt[0][e], d[m][0][e]);
                                d[m][1][e] = Mfma<float>::step(at[m][e], bt[1][e], d[m][1][e]);
                            }
                    } else if (on) {
#pragma unroll
                        for (int e = 0; e < 2; ++e)
#pragma unroll
                            for (int m = 0; m < MBW; ++m) d[m][0][e] = Mfma<float>::step(at[m][e], bt[0][e], d[m][0][e]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int m = 0; m < MBW; ++m) at[m] = bload2(ra, tvalid ? arow[m] + ktail : kOffNone, aso);
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb) bt[bb] = bload2(rx, tvalid ? bro[bb] + ktail : kOffNone, 0);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            // chunk ch into this wave's rows of the accumulator; empty slots
            // (column -1) are skipped
            if (on) {
#pragma unroll
                for (int bb = 0; bb < 2; ++bb) {
                    if (bb == 1 && !two) break;
                    const int col = cur.col[bb];
                    if (col >= 0) {
                        float* pc = acc + (col * R + rh[bb]) * LDL + wr0 + 4 * g;
#pragma unroll
                        for (int m = 0; m < MBW; ++m) {
                            V4* q4 = reinterpret_cast<V4*>(pc + 16 * m);
                            const V4 o = *q4;
                            V4 r;
#pragma unroll
                            for (int e = 0; e < 4; ++e) r[e] = __builtin_fmaf(scale, d[m][bb][0][e] + d[m][bb][1][e], o[e]);
                            *q4 = r;
                        }
                    }
                }
            }
            nb_c = nb_n;
            sc_c = sc_n;
            unpack(cur.meta, cls_n, nb_n, sc_n);   // chunk ch+2
        };
        for (int ch = cb - 2; ch < ce; ch += 2) {
            step(ch, ring[0], ring[1]);
            step(ch + 1, ring[1], ring[0]);
        }
    }
    for (int idx = lane; idx < ncol * pieces; idx += 64) {
        const int col = idx / pieces;
        const int r = wr0 + 4 * (idx - col * pieces);
        *reinterpret_cast<V4*>(Y + (ybase + col) * p.ldy + row0 + r) = *reinterpret_cast<const V4*>(acc + col * LDL + r);
    }
}

// Grouped GEMM of a schedule in which every target has exactly one pair (the
// leaf S~ and T~ products, L2L and, in the adjoint, the transposed M2M):
// nothing is summed across chunks, so a workgroup computes one chunk for all
// output rows and writes (or adds into) Y directly, without an accumulator in
// LDS. The workgroups are small and run no pipeline; the loads of one are
// hidden behind the MFMAs of the others on its CU.
//
// The workgroup stages the chunk's 32 source columns in LDS; wave w computes
// the 16-row blocks w, w+4, ... of the output for the 16-column blocks that
// hold data, with the A rows of a block in registers and the same K-permuted
// operand layout as gg_kernel. Empty slots have no target and are not
// written. Targets are distinct within and across chunks, so every output
// element is written once by one lane.
struct GDParams {
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
    int unit_scale;             // 1: ignore the chunk scale (products written unscaled)
    const int32_t* chunk_meta;
    const int32_t* chunk_src;
    const int32_t* chunk_tgt;   // per chunk slot: target row (box), -1 for an empty slot
};

template <typename T, int KP16>
__global__ void __launch_bounds__(256) gd_kernel(GDParams p) {
    using M = Mfma<T>;
    using V4 = typename M::V4;
    constexpr int KDIM = KP16 * 16;
    constexpr int LDB = KDIM + 4;
    constexpr int V4C = KDIM / 4;
    constexpr int NSV = 32 * V4C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* bb = reinterpret_cast<T*>(smem_raw);   // [32][LDB]
    const int ch = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int j = lane & 15;
    const int grp = lane >> 4;
    const int R = p.R;
    const int cp = p.cp;
    const int cls = uload<int32_t>(p.chunk_meta, 4 * ch);
    // word 1: 16-column blocks holding data and (bits 8..) the 16-row blocks
    // of A holding data when fewer than MB (stage-2 factors)
    const int w1 = uload<int32_t>(p.chunk_meta, 4 * ch + 1);
    const int nblk = w1 & 0xff;
    const int nrb = (w1 >> 8) ? min(w1 >> 8, p.MB) : p.MB;
    const T scale = p.unit_scale ? T(1)
                                 : meta_scale<T>(uload<int32_t>(p.chunk_meta, 4 * ch + 2),
                                                 uload<int32_t>(p.chunk_meta, 4 * ch + 3));
    const T* __restrict__ X = static_cast<const T*>(p.X);
    for (int f = tid; f < NSV; f += 256) {
        const int c = f / V4C;
        const int part = 4 * (f - c * V4C);
        const int pr = c / R;
        const int src = p.chunk_src[ch * cp + pr];
        V4 v = V4{0, 0, 0, 0};
        if (src >= 0) v = *reinterpret_cast<const V4*>(X + ((int64_t)src * R + (c - pr * R)) * p.ldx + part);
        *reinterpret_cast<V4*>(bb + c * LDB + part) = v;
    }
    // output row (target row * R + right-hand side) of this lane's column in
    // each 16-column block, -1 for an empty slot
    int64_t orow[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int c = b * 16 + j;
        const int pr = c / R;
        const int tgt = p.chunk_tgt[ch * cp + pr];
        orow[b] = tgt >= 0 ? (int64_t)tgt * R + (c - pr * R) : -1;
    }
    __syncthreads();
    const T* __restrict__ A = static_cast<const T*>(p.A) + (int64_t)cls * p.a_stride;
    T* __restrict__ Y = static_cast<T*>(p.Y);
    for (int blk = wave; blk < nrb; blk += 4) {
        V4 a[KP16];
        const T* ar = A + (int64_t)(blk * 16 + j) * p.lda + 4 * grp;
#pragma unroll
        for (int t = 0; t < KP16; ++t) a[t] = *reinterpret_cast<const V4*>(ar + 16 * t);
        for (int cb = 0; cb < nblk; ++cb) {
            V4 d0 = V4{0, 0, 0, 0}, d1 = V4{0, 0, 0, 0};
            const T* bc = bb + (cb * 16 + j) * LDB + 4 * grp;
#pragma unroll
            for (int t = 0; t < KP16; ++t) {
                const V4 bv = *reinterpret_cast<const V4*>(bc + 16 * t);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (t & 1)
                        d1 = M::step(a[t][e], bv[e], d1);
                    else
                        d0 = M::step(a[t][e], bv[e], d0);
                }
            }
            const int64_t o = cb ? orow[1] : orow[0];
            if (o >= 0) {
                T* yp = Y + o * p.ldy + blk * 16;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = M::row(q, grp);
                    const T v = scale * (d0[q] + d1[q]);
                    yp[r] = p.accumulate ? yp[r] + v : v;
                }
            }
        }
    }
}

// Raise the dynamic-LDS limit of kernel `fn` on the current device to at
// least `lds` bytes (no call below 64 KiB). Safe to call from several
// threads: the limits already set are kept per (kernel, device) under a lock.
hipError_t ensure_lds(const void* fn, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    size_t& cur = done[{fn, dev}];
    if (lds <= cur) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) cur = lds;
    return e;
}

template <typename T, int KP16>
hipError_t gd_launch_t(const GDParams& p, int blocks, size_t lds, hipStream_t st) {
    hipError_t e = ensure_lds(reinterpret_cast<const void*>(&gd_kernel<T, KP16>), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gd_kernel<T, KP16>), dim3(blocks), dim3(256), lds, st, p);
    return hipGetLastError();
}

template <typename T>
hipError_t gd_dispatch(int KP16, const GDParams& p, int blocks, size_t lds, hipStream_t st) {
    switch (KP16) {
#define KIFMM_GD_CASE(K) \
    case K:              \
        return gd_launch_t<T, K>(p, blocks, lds, st);
        KIFMM_GD_CASE(1) KIFMM_GD_CASE(2) KIFMM_GD_CASE(3) KIFMM_GD_CASE(4) KIFMM_GD_CASE(5)
        KIFMM_GD_CASE(6) KIFMM_GD_CASE(7) KIFMM_GD_CASE(8) KIFMM_GD_CASE(9) KIFMM_GD_CASE(10)
        KIFMM_GD_CASE(11) KIFMM_GD_CASE(12) KIFMM_GD_CASE(13) KIFMM_GD_CASE(14) KIFMM_GD_CASE(15)
        KIFMM_GD_CASE(16) KIFMM_GD_CASE(17) KIFMM_GD_CASE(18) KIFMM_GD_CASE(19)
#undef KIFMM_GD_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T, int KP16, int WAVES, int MBW, bool B3>
hipError_t gg_launch_t(const GGParams& p, int blocks, size_t lds, hipStream_t st) {
    if constexpr (B3 && (KP16 % 2 != 0 || sizeof(T) != 4)) {
        return hipErrorInvalidValue;
    } else {
        // FP32 pipelined form with the data ending within 8 of the last
        // K-chunk's start: the trimmed last K-chunk
        constexpr bool can_trim = !B3 && sizeof(T) == 4 && KP16 >= 2 && KP16 * 4 <= 32;
        if constexpr (can_trim) {
            if (p.a_cols <= 16 * (KP16 - 1) + 8) {
                hipError_t e = ensure_lds(reinterpret_cast<const void*>(&gg_kernel<T, KP16, WAVES, MBW, false, true>), lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL((gg_kernel<T, KP16, WAVES, MBW, false, true>), dim3(blocks), dim3(64 * WAVES), lds, st, p);
                return hipGetLastError();
            }
        }
        hipError_t e = ensure_lds(reinterpret_cast<const void*>(&gg_kernel<T, KP16, WAVES, MBW, B3>), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((gg_kernel<T, KP16, WAVES, MBW, B3>), dim3(blocks), dim3(64 * WAVES), lds, st, p);
        return hipGetLastError();
    }
}

template <typename T, int WAVES, int MBW, bool B3 = false>
hipError_t gg_dispatch(int KP16, const GGParams& p, int blocks, size_t lds, hipStream_t st) {
    switch (KP16) {
#define KIFMM_GG_CASE(K) \
    case K:              \
        return gg_launch_t<T, K, WAVES, MBW, B3>(p, blocks, lds, st);
        KIFMM_GG_CASE(1) KIFMM_GG_CASE(2) KIFMM_GG_CASE(3) KIFMM_GG_CASE(4) KIFMM_GG_CASE(5)
        KIFMM_GG_CASE(6) KIFMM_GG_CASE(7) KIFMM_GG_CASE(8) KIFMM_GG_CASE(9) KIFMM_GG_CASE(10)
        KIFMM_GG_CASE(11) KIFMM_GG_CASE(12) KIFMM_GG_CASE(13) KIFMM_GG_CASE(14) KIFMM_GG_CASE(15)
        KIFMM_GG_CASE(16) KIFMM_GG_CASE(17) KIFMM_GG_CASE(18) KIFMM_GG_CASE(19)
#undef KIFMM_GG_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <int KP16, int WAVES, int MBW, bool B3, bool TAIL8>
hipError_t rs_launch_t(const GGParams& p, int blocks, size_t lds, hipStream_t st) {
    if constexpr ((B3 && (KP16 % 2 != 0 || TAIL8)) || (TAIL8 && KP16 < 2)) {
        return hipErrorInvalidValue;
    } else {
        hipError_t e = ensure_lds(reinterpret_cast<const void*>(&rs_kernel<KP16, WAVES, MBW, B3, TAIL8>), lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((rs_kernel<KP16, WAVES, MBW, B3, TAIL8>), dim3(blocks), dim3(64 * WAVES), lds, st, p);
        return hipGetLastError();
    }
}

template <int WAVES, int MBW>
hipError_t rs_dispatch(int KP16, bool b3, bool tail8, const GGParams& p, int blocks, size_t lds, hipStream_t st) {
    switch (KP16) {
#define KIFMM_RS_CASE(K)                                                                  \
    case K:                                                                               \
        if (b3) return rs_launch_t<K, WAVES, MBW, true, false>(p, blocks, lds, st);       \
        if (tail8) return rs_launch_t<K, WAVES, MBW, false, true>(p, blocks, lds, st);    \
        return rs_launch_t<K, WAVES, MBW, false, false>(p, blocks, lds, st);
        KIFMM_RS_CASE(1) KIFMM_RS_CASE(2) KIFMM_RS_CASE(3) KIFMM_RS_CASE(4) KIFMM_RS_CASE(5)
        KIFMM_RS_CASE(6) KIFMM_RS_CASE(7) KIFMM_RS_CASE(8) KIFMM_RS_CASE(9) KIFMM_RS_CASE(10)
#undef KIFMM_RS_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t gg_variant(int variant, int KP16, const GGParams& p, int blocks, size_t lds, hipStream_t st,
                      bool b3) {
    if (variant == 4 || variant == 5) {
        // row-slab form: FP32 data only, K up to 160
        if constexpr (sizeof(T) == 4) {
            const bool tail8 = !b3 && KP16 >= 2 && p.a_cols <= 16 * (KP16 - 1) + 8;
            if (variant == 4) return rs_dispatch<4, 2>(KP16, b3, tail8, p, blocks, lds, st);
            return rs_dispatch<8, 1>(KP16, b3, tail8, p, blocks, lds, st);
        }
        return hipErrorInvalidValue;
    }
    if (b3) {
        if constexpr (sizeof(T) == 4) {
            switch (variant) {
                case 0: return gg_dispatch<T, 8, 1, true>(KP16, p, blocks, lds, st);
                case 1:
                case 2: return gg_dispatch<T, 4, 1, true>(KP16, p, blocks, lds, st);
                case 3: return gg_dispatch<T, 4, 2, true>(KP16, p, blocks, lds, st);
                default: return hipErrorInvalidValue;
            }
        }
        return hipErrorInvalidValue;
    }
    switch (variant) {
        case 0: return gg_dispatch<T, 8, 1>(KP16, p, blocks, lds, st);
        case 1:
        case 2: return gg_dispatch<T, 4, 1>(KP16, p, blocks, lds, st);
        case 3:
            // two row blocks per wave: FP32 only (the FP64 registers would spill)
            if constexpr (sizeof(T) == 4) return gg_dispatch<T, 4, 2>(KP16, p, blocks, lds, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int gg_variant_rows(int variant) {
    switch (variant) {
        case 0: return 8 * 16;
        case 1:
        case 2: return 4 * 16;
        case 3: return 4 * 2 * 16;
        case 4: return 4 * 2 * 16;
        case 5: return 8 * 16;
        default: return 0;
    }
}

bool gg_variant_supported(int variant, int elt, int kp16) {
    if (variant < 0 || variant >= kGGVariants) return false;
    if (variant == 3) return elt == 4;
    if (variant == 4 || variant == 5) return elt == 4 && kp16 <= 10;
    return true;
}

bool gg_variant_staged(int variant) { return variant < 4; }

int gg_variant_wgs_per_cu(int variant) { return variant == 2 ? 2 : 1; }

size_t gg_lds_limit(int variant) { return (160 * 1024) / gg_variant_wgs_per_cu(variant); }

int gg_nbuf(int elt, int variant, int KP16) {
    if (!gg_variant_staged(variant)) return 0;
    const size_t stage = (size_t)32 * (KP16 * 16 + 4) * elt;
    return 2 * stage <= gg_lds_limit(variant) / 2 ? 2 : 1;
}

size_t gg_lds_bytes(int elt, int variant, int KP16, int cols) {
    return ((size_t)gg_nbuf(elt, variant, KP16) * 32 * (KP16 * 16 + 4) +
            (size_t)cols * (gg_variant_rows(variant) + 4)) * elt;
}

hipError_t launch_gg(const DevSched& s, int elt, const void* A, int MB, int KP16, int a_rows, int a_cols,
                     const void* X, int ldx, void* Y, int ldy, int R, int accumulate, hipStream_t st,
                     bool b3) {
    if (s.n_tiles == 0) return hipSuccess;
    if (b3 && (elt != 4 || KP16 % 2 != 0)) return hipErrorInvalidValue;
    if (a_rows < 1 || a_rows > MB * 16 || a_cols < 1 || a_cols > KP16 * 16) return hipErrorInvalidValue;
    if (s.direct && !b3) {
        // one pair per target: one workgroup per chunk, results written directly
        if (KP16 < 1 || KP16 > 19 || s.cp * R != 32 || s.chunk_tgt == nullptr) return hipErrorInvalidValue;
        GDParams g;
        g.A = A;
        g.a_stride = (int64_t)MB * 16 * KP16 * 16;
        g.lda = KP16 * 16;
        g.X = X;
        g.ldx = ldx;
        g.Y = Y;
        g.ldy = ldy;
        g.MB = MB;
        g.R = R;
        g.cp = s.cp;
        g.accumulate = accumulate;
        g.unit_scale = s.unit_scale ? 1 : 0;
        g.chunk_meta = s.chunk_meta;
        g.chunk_src = s.chunk_src;
        g.chunk_tgt = s.chunk_tgt;
        const size_t lds = (size_t)32 * (KP16 * 16 + 4) * elt;
        if (elt == 4) return gd_dispatch<float>(KP16, g, s.n_chunks, lds, st);
        return gd_dispatch<double>(KP16, g, s.n_chunks, lds, st);
    }
    GGParams p;
    p.A = A;
    p.a_stride = (int64_t)MB * 16 * KP16 * 16;
    p.lda = KP16 * 16;
    p.a_rows = a_rows;
    p.a_cols = a_cols;
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
    if (!gg_variant_supported(s.variant, elt, KP16) || s.cp * R != 32 || s.max_tile < 1) return hipErrorInvalidValue;
    p.n_rg = (MB + mbg - 1) / mbg;
    p.nbuf = gg_nbuf(elt, s.variant, KP16);
    p.trash_col = s.max_tile;
    p.tile_tgt0 = s.tile_tgt0;
    p.tile_ntgt = s.tile_ntgt;
    p.tile_chunk0 = s.tile_chunk0;
    p.chunk_meta = s.chunk_meta;
    p.chunk_src = s.chunk_src;
    p.chunk_col = s.chunk_col;
    // buffer extents: rows of X up to the largest source row of the schedule,
    // classes of A up to the largest class; each must fit 32-bit offsets
    const int64_t xb = (int64_t)(s.max_src + 1) * R * ldx * elt;
    const int64_t ab = (int64_t)(s.max_cls + 1) * p.a_stride * elt;
    const int64_t lb = (int64_t)s.n_chunks * s.cp * 4;
    const int64_t lim = (int64_t)1 << 31;
    if (xb >= lim || ab >= lim || lb >= lim || (int64_t)R * ldx * elt >= (1 << 24) || s.max_src >= (1 << 24))
        return hipErrorInvalidValue;
    p.x_bytes = (uint32_t)xb;
    p.a_bytes = (uint32_t)ab;
    p.meta_bytes = (uint32_t)((int64_t)s.n_chunks * 16);
    p.list_bytes = (uint32_t)lb;
    // accumulator columns: the largest tile plus the spare columns of empty slots
    const size_t lds = gg_lds_bytes(elt, s.variant, KP16, (s.max_tile + 1) * R);
    if (lds > gg_lds_limit(s.variant) || KP16 < 1 || KP16 > 19) return hipErrorInvalidValue;
    p.xcd_run = GG_XCD_RUN;
    const int blocks = (s.n_tiles + 8 * p.xcd_run - 1) / (8 * p.xcd_run) * 8 * p.xcd_run * p.n_rg;
    if (elt == 4) return gg_variant<float>(s.variant, KP16, p, blocks, lds, st, b3);
    return gg_variant<double>(s.variant, KP16, p, blocks, lds, st, false);
}

}  // namespace kifmm
