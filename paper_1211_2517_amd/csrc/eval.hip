// Point-evaluation kernels of the KIFMM for gfx950 (CDNA4, wave64).
//
// permute_in     densities into the sorted point order.
// eval_surface   potential of the points of a leaf on the (3-2d) cube surface:
//                the check potential of S2M (Sec. 2.2) and, in the adjoint,
//                the transpose of the L2T evaluation.
// eval_targets   near-field direct sum of eq. (1) over the near field (S2T)
//                plus the potential of the downward equivalent densities on
//                the leaf's points (L2T, Sec. 2.2), scattered to caller order.
// eval_m2t       adaptive trees: equivalent densities of W-list cubes at a
//                leaf's points (M2T).
// eval_s2l       adaptive trees: check potentials of a cube from the points of
//                its X-list leaves (S2L).
#include "kernels.h"

#include <type_traits>

namespace kifmm {

namespace {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

template <typename T>
struct alignas(4 * sizeof(T)) P4 {
    T x, y, z, w;
};

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

// Check potential of a leaf's points on its (3-2d) surface: one wave per
// leaf, lanes over the surface points. The wave stages the leaf's points as
// (x, y, z, sigma) 4-vectors in LDS (sigmas of further right-hand sides in a
// second array), in batches of at most CAP points, so each interaction reads
// one broadcast LDS vector.
template <typename T, int R>
__global__ void __launch_bounds__(256) eval_surface_kernel(int64_t n_leaf, const P4<T>* __restrict__ pts,
                                                           const T* __restrict__ sig,
                                                           const int32_t* __restrict__ leaf_ptr,
                                                           const T* __restrict__ surf, int n_eq,
                                                           int nep, T* __restrict__ C) {
    constexpr int WPB = 4;
    constexpr int CAP = 64;
    __shared__ P4<T> sp[WPB][CAP];
    __shared__ T ss[WPB][R > 1 ? CAP * R : 1];
    const int wave = threadIdx.x >> 6;
    const int64_t leaf = (int64_t)blockIdx.x * WPB + wave;
    if (leaf >= n_leaf) return;
    const int lane = threadIdx.x & 63;
    P4<T>* st = sp[wave];
    T* sst = ss[wave];
    const int p0 = leaf_ptr[leaf];
    const int p1 = leaf_ptr[leaf + 1];
    constexpr int NA = (19 * 16 + 63) / 64;   // surface points per lane, at most
    T sx[NA], sy[NA], sz[NA];
    T acc[NA][R];
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int a = k * 64 + lane;
        const bool valid = a < n_eq;
        sx[k] = valid ? surf[3 * a] : T(0);
        sy[k] = valid ? surf[3 * a + 1] : T(0);
        sz[k] = valid ? surf[3 * a + 2] : T(0);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[k][r] = 0;
    }
    const int na = (nep + 63) / 64;
    for (int base = p0; base < p1; base += CAP) {
        const int cnt = min(CAP, p1 - base);
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const P4<T> v = pts[base + lane];
            T w0 = T(0);
            if constexpr (R == 1) {
                w0 = sig[base + lane];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) sst[lane * R + r] = sig[(int64_t)(base + lane) * R + r];
            }
            st[lane] = P4<T>{v.x, v.y, v.z, w0};
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll 2
        for (int jj = 0; jj < cnt; ++jj) {
            const P4<T> f = st[jj];
#pragma unroll
            for (int k = 0; k < NA; ++k) {
                if (k < na) {
                    const T dx = sx[k] - f.x, dy = sy[k] - f.y, dz = sz[k] - f.z;
                    const T rinv = rsq(dx * dx + dy * dy + dz * dz);
                    if constexpr (R == 1) {
                        acc[k][0] += f.w * rinv;
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[k][r] += sst[jj * R + r] * rinv;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int a = k * 64 + lane;
        if (k < na && a < nep) {
#pragma unroll
            for (int r = 0; r < R; ++r) C[(leaf * R + r) * nep + a] = a < n_eq ? acc[k][r] : T(0);
        }
    }
}

// Near field (S2T, MODE bit 1) and far field (L2T, MODE bit 2) at the points
// of a target leaf: one wave per target leaf, `lpt` lanes per target splitting
// the sources. MODE 1 writes the near field, MODE 2 adds the far field to
// what is there, MODE 3 writes both.
// The wave stages the points of its near-field leaves in its own LDS slots
// as 4-vectors (x, y, z in target-leaf units, sigma for one right-hand side;
// the sigmas of several right-hand sides sit in a second array), so each
// interaction reads one broadcast LDS vector; batches of at most CAP points
// are staged and consumed in turn. The near-field entries (at most 27 in a
// uniform tree, at most 64 here) are resolved in parallel, one per lane, and
// a prefix sum of their point counts numbers the staged points, so every
// staged point is one independent load: a batch costs one memory latency. For the far field the wave stages the
// leaf's downward equivalent surface as (x, y, z, E) vectors the same way
// (one right-hand side), or reads E from global memory (several).
// FP32 near field: the points are also given in fixed point, q = round(u 2^28)
// (int32; |u| <= 1 in leaf units), and the staged sources carry q - 2^29 d, so
// every coordinate difference of a near pair is an exact integer that is
// converted to FP32 once: the distance of a nearly coincident pair keeps full
// FP32 relative accuracy (with FP32 leaf-unit coordinates it would lose the
// digits the two coordinates share). The 2^28 scale is taken out in the
// near-field factor.
template <typename T, int R, int MODE, bool AD = false>
__global__ void __launch_bounds__(256) eval_targets_kernel(
    int64_t n_leaf, const P4<T>* __restrict__ pts, const P4<int32_t>* __restrict__ qpts, const T* __restrict__ sig,
    const int32_t* __restrict__ leaf_ptr, const int32_t* __restrict__ near_ptr,
    const int32_t* __restrict__ near_leaf, const int32_t* __restrict__ near_code,
    const int32_t* __restrict__ leaf_level, const T* __restrict__ leaf_scale, const T* __restrict__ E,
    const T* __restrict__ surf, int n_eq, int nep, T near_scale, T far_scale, const int32_t* __restrict__ perm,
    T* __restrict__ out, int64_t ld, int nrhs) {
    constexpr int WPB = 4;
    constexpr int CAP = (R >= 8 ? 64 : R >= 2 ? 128 : 256) / (int)(sizeof(T) / 4);
    constexpr int MAXEQ = 19 * 16;
    constexpr bool FIX = sizeof(T) == 4;   // fixed-point near-field differences
    using SP = typename std::conditional<FIX, P4<int32_t>, P4<T>>::type;
    __shared__ SP sp[(MODE & 1) ? WPB : 1][(MODE & 1) ? CAP : 1];
    __shared__ T ss[(MODE & 1) ? WPB : 1][(MODE & 1) && R > 1 ? CAP * R : 1];
    __shared__ P4<T> fs[(MODE & 2) && R == 1 ? WPB : 1][(MODE & 2) && R == 1 ? MAXEQ : 1];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t leaf = (int64_t)blockIdx.x * WPB + wave;
    if (leaf >= n_leaf) return;
    SP* st = sp[(MODE & 1) ? wave : 0];
    // adaptive form: every leaf has its own near-field scale (its unit), and
    // leaves above level 2 have no local expansion
    int lev = 0;
    T nsc = near_scale;
    if constexpr (AD) {
        lev = leaf_level[leaf];
        nsc = leaf_scale[leaf];
    }
    // fixed-point differences are in units of 2^-28 leaf half-widths
    const T nscale = (FIX && (MODE & 1)) ? nsc * T(268435456.0f) : nsc;
    T* sst = ss[(MODE & 1) ? wave : 0];
    const int p0 = leaf_ptr[leaf];
    const int ne = leaf_ptr[leaf + 1] - p0;
    int lpt = 64;
    while (lpt > 1 && (64 / lpt) < ne) lpt >>= 1;
    const int tpr = 64 / lpt;
    const int sub = lane & (lpt - 1);
    const int q0 = near_ptr[leaf];
    const int q1 = near_ptr[leaf + 1];
    const bool far_on = (MODE & 2) && E != nullptr && (!AD || lev >= 2);
    // near-field entries, one per lane: first point, point count, offset code,
    // and the inclusive prefix sum of the counts (the entries' staged ranges).
    // Adaptive trees take the entries in two passes: sources at the target's
    // level or coarser (differences in target-leaf units), then sources one
    // level finer (differences in their units, so the target coordinates are
    // doubled and the source weights too: exact in both arithmetics).
    int e_b0 = 0, e_code = 0, e_cnt[2] = {0, 0}, e_incl[2] = {0, 0}, n_near[2] = {0, 0};
    if constexpr ((MODE & 1) != 0) {
        const int nq = min(q1 - q0, 64);
        int cnt = 0, pass = 0;
        if (lane < nq) {
            const int nb = near_leaf[q0 + lane];
            e_code = near_code[q0 + lane];
            e_b0 = leaf_ptr[nb];
            cnt = leaf_ptr[nb + 1] - e_b0;
            if constexpr (AD) pass = (e_code / 729 == 1) ? 1 : 0;
        }
        e_cnt[0] = pass == 0 ? cnt : 0;
        e_cnt[1] = pass == 1 ? cnt : 0;
#pragma unroll
        for (int ps = 0; ps < (AD ? 2 : 1); ++ps) {
            int v0 = e_cnt[ps];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(v0, off);
                if (lane >= off) v0 += v;
            }
            e_incl[ps] = v0;
            n_near[ps] = __shfl(v0, 63);
        }
    }
    if constexpr ((MODE & 2) && R == 1) {
        if (far_on) {
            for (int a = lane; a < n_eq; a += 64)
                fs[wave][a] = P4<T>{surf[3 * a], surf[3 * a + 1], surf[3 * a + 2], E[leaf * nep + a]};
        }
    }
    for (int tb = 0; tb < ne; tb += tpr) {
        const int tl = tb + lane / lpt;
        const bool valid = tl < ne;
        const int i = p0 + (valid ? tl : 0);
        const P4<T> ui = pts[i];
        P4<int32_t> qi{0, 0, 0, 0};
        if constexpr (FIX && (MODE & 1)) qi = qpts[i];
        P4<T> ut = ui;          // target coordinates of the current pass
        P4<int32_t> qt = qi;
        T acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0;
        // consume the staged batch of n points
        auto consume = [&](int n) {
            __builtin_amdgcn_wave_barrier();
#pragma unroll 4
            for (int jj = sub; jj < n; jj += lpt) {
                const SP f = st[jj];
                T dx, dy, dz, fw;
                if constexpr (FIX) {
                    dx = (T)(qt.x - f.x);
                    dy = (T)(qt.y - f.y);
                    dz = (T)(qt.z - f.z);
                    fw = __int_as_float(f.w);
                } else {
                    dx = ut.x - f.x;
                    dy = ut.y - f.y;
                    dz = ut.z - f.z;
                    fw = f.w;
                }
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T rinv = r2 > T(0) ? rsq(r2) : T(0);
                if constexpr (R == 1) {
                    acc[0] += fw * rinv;
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] += sst[jj * R + r] * rinv;
                }
            }
            __builtin_amdgcn_wave_barrier();
        };
#pragma unroll 1
        for (int ps = 0; ps < (AD ? 2 : 1); ++ps) {
            const int incl = e_incl[ps], ecnt = e_cnt[ps], nn = n_near[ps];
            if (ps == 1) {
                qt = P4<int32_t>{2 * qi.x, 2 * qi.y, 2 * qi.z, 0};
                ut = P4<T>{T(2) * ui.x, T(2) * ui.y, T(2) * ui.z, T(0)};
            }
            // stage and consume the near-field points in batches of CAP
            for (int base = 0; base < nn; base += CAP) {
                const int cnt = min(CAP, nn - base);
#pragma unroll
                for (int k = 0; k < CAP / 64; ++k) {
                    const int slot = k * 64 + lane;
                    const int sidx = base + slot;
                    // entry of staged point sidx: the number of entries whose
                    // range ends at or before it (binary search over the lanes)
                    int e = 0;
#pragma unroll
                    for (int stp = 32; stp > 0; stp >>= 1) {
                        const int v = __shfl(incl, e + stp - 1);
                        if (v <= sidx) e += stp;
                    }
                    e = min(e, 63);
                    const int b0 = __shfl(e_b0, e);
                    const int ex = __shfl(incl, e) - __shfl(ecnt, e);
                    const int code = __shfl(e_code, e);
                    if (slot < cnt) {
                        const int jj = b0 + (sidx - ex);
                        // the source in the units of the pass: a s + o, where a = 2
                        // for a coarser source (adaptive), and o = (source centre -
                        // target centre) in those units (uniform: o = -2 d, d =
                        // target - source cube)
                        int ox, oy, oz, as = 1;
                        T wm = T(1);
                        if constexpr (AD) {
                            const int m = code / 729, rem = code - 729 * m;
                            ox = rem / 81 - 4;
                            oy = (rem / 9) % 9 - 4;
                            oz = rem % 9 - 4;
                            as = m == 2 ? 2 : 1;
                            wm = m == 1 ? T(2) : T(1);
                        } else {
                            ox = -2 * (code / 9 - 1);
                            oy = -2 * ((code / 3) % 3 - 1);
                            oz = -2 * (code % 3 - 1);
                        }
                        T w0 = T(0);
                        if constexpr (R == 1) {
                            w0 = wm * sig[jj];
                        } else {
#pragma unroll
                            for (int r = 0; r < R; ++r) sst[slot * R + r] = wm * sig[(int64_t)jj * R + r];
                        }
                        if constexpr (FIX) {
                            const P4<int32_t> sq = qpts[jj];
                            st[slot] = SP{as * sq.x + ox * (1 << 28), as * sq.y + oy * (1 << 28),
                                          as * sq.z + oz * (1 << 28), __float_as_int(w0)};
                        } else {
                            const P4<T> sv = pts[jj];
                            st[slot] = SP{T(as) * sv.x + T(ox), T(as) * sv.y + T(oy), T(as) * sv.z + T(oz), w0};
                        }
                    }
                }
                consume(cnt);
            }
        }
        T far[R];
#pragma unroll
        for (int r = 0; r < R; ++r) far[r] = 0;
        if (far_on) {
            if constexpr ((MODE & 2) && R == 1) {
                __builtin_amdgcn_wave_barrier();
#pragma unroll 4
                for (int a = sub; a < n_eq; a += lpt) {
                    const P4<T> f = fs[wave][a];
                    const T dx = ui.x - f.x, dy = ui.y - f.y, dz = ui.z - f.z;
                    far[0] += f.w * rsq(dx * dx + dy * dy + dz * dz);
                }
            } else {
                for (int a = sub; a < n_eq; a += lpt) {
                    const T dx = ui.x - surf[3 * a], dy = ui.y - surf[3 * a + 1], dz = ui.z - surf[3 * a + 2];
                    const T rinv = rsq(dx * dx + dy * dy + dz * dz);
#pragma unroll
                    for (int r = 0; r < R; ++r) far[r] += E[(leaf * R + r) * nep + a] * rinv;
                }
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
            for (int r = 0; r < R; ++r) {
                if (r < nrhs) {
                    if constexpr (MODE == 1)
                        out[dst + r * ld] = nscale * acc[r];
                    else if constexpr (MODE == 2)
                        out[dst + r * ld] += far_scale * far[r];
                    else
                        out[dst + r * ld] = nscale * acc[r] + far_scale * far[r];
                }
            }
        }
    }
}

// Near field (S2T) of FP32 uniform plans with one right-hand side, the form
// of eval_targets_kernel's near mode (fixed-point differences, entries one
// per lane, prefix sum, binary search) with its batches of 64 staged sources
// held in registers, one per lane, and read across lanes (ds_bpermute)
// instead of from LDS. It allocates no LDS, so its workgroups can share a CU
// with a launch that holds the CU's LDS (the M2L launch) and use the vector
// ALU that launch leaves idle. Every lane runs the same number of steps per
// batch (sources past the batch are masked), so the cross-lane reads never
// execute under divergence; the per-lane sums are those of
// eval_targets_kernel in the same order (bitwise the same result).
__global__ void __launch_bounds__(256) near_reg_kernel(int64_t n_leaf, const P4<int32_t>* __restrict__ qpts,
                                                       const float* __restrict__ sig,
                                                       const int32_t* __restrict__ leaf_ptr,
                                                       const int32_t* __restrict__ near_ptr,
                                                       const int32_t* __restrict__ near_leaf,
                                                       const int32_t* __restrict__ near_code, float near_scale,
                                                       const int32_t* __restrict__ perm, float* __restrict__ out) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t leaf = (int64_t)blockIdx.x * 4 + wave;
    if (leaf >= n_leaf) return;
    const float nscale = near_scale * 268435456.0f;
    const int p0 = leaf_ptr[leaf];
    const int ne = leaf_ptr[leaf + 1] - p0;
    int lpt = 64;
    while (lpt > 1 && (64 / lpt) < ne) lpt >>= 1;
    const int tpr = 64 / lpt;
    const int sub = lane & (lpt - 1);
    const int q0 = near_ptr[leaf], q1 = near_ptr[leaf + 1];
    const int nq = min(q1 - q0, 64);
    int e_b0 = 0, e_code = 0, e_cnt = 0;
    if (lane < nq) {
        const int nb = near_leaf[q0 + lane];
        e_code = near_code[q0 + lane];
        e_b0 = leaf_ptr[nb];
        e_cnt = leaf_ptr[nb + 1] - e_b0;
    }
    int incl = e_cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    const int n_near = __shfl(incl, 63);
    for (int tb = 0; tb < ne; tb += tpr) {
        const int tl = tb + lane / lpt;
        const bool valid = tl < ne;
        const int i = p0 + (valid ? tl : 0);
        const P4<int32_t> qi = qpts[i];
        float acc = 0.0f;
        for (int base = 0; base < n_near; base += 64) {
            const int cnt = min(64, n_near - base);
            // this lane's staged source: slot = lane of the batch
            const int sidx = base + lane;
            int e = 0;
#pragma unroll
            for (int stp = 32; stp > 0; stp >>= 1) {
                const int v = __shfl(incl, e + stp - 1);
                if (v <= sidx) e += stp;
            }
            e = min(e, 63);
            const int b0 = __shfl(e_b0, e);
            const int ex = __shfl(incl, e) - __shfl(e_cnt, e);
            const int code = __shfl(e_code, e);
            int sx = 0, sy = 0, sz = 0;
            float sw = 0.0f;
            if (lane < cnt) {
                const int jj = b0 + (sidx - ex);
                // the source in target-leaf units: s - 2 d (d = target - source cube)
                const int ox = -2 * (code / 9 - 1), oy = -2 * ((code / 3) % 3 - 1), oz = -2 * (code % 3 - 1);
                const P4<int32_t> sq = qpts[jj];
                sx = sq.x + ox * (1 << 28);
                sy = sq.y + oy * (1 << 28);
                sz = sq.z + oz * (1 << 28);
                sw = sig[jj];
            }
            const int steps = (cnt + lpt - 1) / lpt;
#pragma unroll 4
            for (int k = 0; k < steps; ++k) {
                const int jj = sub + k * lpt;
                const int src = jj < cnt ? jj : 0;
                const int fx = __shfl(sx, src), fy = __shfl(sy, src), fz = __shfl(sz, src);
                const float fw = __shfl(sw, src);
                const float dx = (float)(qi.x - fx), dy = (float)(qi.y - fy), dz = (float)(qi.z - fz);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = r2 > 0.0f ? rsq(r2) : 0.0f;
                if (jj < cnt) acc += fw * rinv;
            }
        }
        for (int off = lpt >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (valid && sub == 0) out[perm[i]] = nscale * acc;
    }
}

// M2T at the points of the leaves in `lf_list` (one wave per leaf, `lpt`
// lanes per target point splitting the surface points): for every W entry of
// the leaf, the U~ q~ values Psi of its cube, placed on the cube's (1+d)
// surface mapped into the leaf's units (rho s + o), are evaluated at the
// leaf's points; the sum times leaf_scale[leaf] (1/(4 pi r_leaf)) is added
// to out. One right-hand side stages (x, y, z, Psi) in LDS; several
// read Psi from global memory.
template <typename T, int R>
__global__ void __launch_bounds__(256) eval_m2t_kernel(
    int64_t n_lf, const int32_t* __restrict__ lf_list, const P4<T>* __restrict__ pts,
    const int32_t* __restrict__ leaf_ptr, const T* __restrict__ leaf_scale,
    const int32_t* __restrict__ ent_ptr, const int32_t* __restrict__ ent_cube, const T* __restrict__ ent_geo,
    const T* __restrict__ Psi, const T* __restrict__ surf_in, int n_eq, int nep,
    const int32_t* __restrict__ perm, T* __restrict__ out, int64_t ld, int nrhs) {
    constexpr int WPB = 4;
    constexpr int MAXEQ = 19 * 16;
    __shared__ P4<T> fs[WPB][MAXEQ];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t wi = (int64_t)blockIdx.x * WPB + wave;
    if (wi >= n_lf) return;
    const int leaf = lf_list[wi];
    const T scale = leaf_scale[leaf];
    const int p0 = leaf_ptr[leaf];
    const int ne = leaf_ptr[leaf + 1] - p0;
    int lpt = 64;
    while (lpt > 1 && (64 / lpt) < ne) lpt >>= 1;
    const int tpr = 64 / lpt;
    const int sub = lane & (lpt - 1);
    const int k0 = ent_ptr[wi], k1 = ent_ptr[wi + 1];
    P4<T>* st = fs[wave];
    if constexpr (R == 1) {
        // one right-hand side: the surface in registers (lane a, a + 64, ...),
        // the entries' cubes and geometry one per lane (batches of 64), and
        // the Psi values of the next entry loaded while the current one is
        // evaluated (unconditional loads, the entry index clamped)
        constexpr int NS = MAXEQ / 64 + 1;
        T sx[NS], sy[NS], sz[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int a = min(q * 64 + lane, n_eq - 1);
            sx[q] = surf_in[3 * a];
            sy[q] = surf_in[3 * a + 1];
            sz[q] = surf_in[3 * a + 2];
        }
        const int nsq = (n_eq + 63) / 64;
        for (int tb = 0; tb < ne; tb += tpr) {
            const int tl = tb + lane / lpt;
            const bool valid = tl < ne;
            const int i = p0 + (valid ? tl : 0);
            const P4<T> ui = pts[i];
            T acc = 0;
            for (int kb = k0; kb < k1; kb += 64) {
                const int nk = min(64, k1 - kb);
                const int kl = kb + min(lane, nk - 1);
                const int e_cube = ent_cube[kl];
                const T g_rho = ent_geo[4 * kl], g_ox = ent_geo[4 * kl + 1], g_oy = ent_geo[4 * kl + 2],
                        g_oz = ent_geo[4 * kl + 3];
                auto load_psi = [&](int e, T (&v)[NS]) {
                    const T* ps = Psi + (int64_t)__builtin_amdgcn_readlane(e_cube, min(e, nk - 1)) * nep;
#pragma unroll
                    for (int q = 0; q < NS; ++q) v[q] = ps[min(q * 64 + lane, n_eq - 1)];
                };
                T pn[NS];
                load_psi(0, pn);
                for (int e = 0; e < nk; ++e) {
                    T pc[NS];
#pragma unroll
                    for (int q = 0; q < NS; ++q) pc[q] = pn[q];
                    load_psi(e + 1, pn);
                    const T rho = __shfl(g_rho, e), ox = __shfl(g_ox, e), oy = __shfl(g_oy, e), oz = __shfl(g_oz, e);
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        const int a = q * 64 + lane;
                        if (q < nsq && a < n_eq) st[a] = P4<T>{rho * sx[q] + ox, rho * sy[q] + oy, rho * sz[q] + oz, pc[q]};
                    }
                    __builtin_amdgcn_wave_barrier();
#pragma unroll 4
                    for (int a = sub; a < n_eq; a += lpt) {
                        const P4<T> f = st[a];
                        const T dx = ui.x - f.x, dy = ui.y - f.y, dz = ui.z - f.z;
                        acc += f.w * rsq(dx * dx + dy * dy + dz * dz);
                    }
                }
            }
            for (int off = lpt >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if (valid && sub == 0 && nrhs > 0) out[perm[i]] += scale * acc;
        }
        return;
    }
    for (int tb = 0; tb < ne; tb += tpr) {
        const int tl = tb + lane / lpt;
        const bool valid = tl < ne;
        const int i = p0 + (valid ? tl : 0);
        const P4<T> ui = pts[i];
        T acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0;
        for (int k = k0; k < k1; ++k) {
            const int cube = ent_cube[k];
            const T rho = ent_geo[4 * k], ox = ent_geo[4 * k + 1], oy = ent_geo[4 * k + 2], oz = ent_geo[4 * k + 3];
            const T* ps = Psi + (int64_t)cube * R * nep;
            __builtin_amdgcn_wave_barrier();
            for (int a = lane; a < n_eq; a += 64)
                st[a] = P4<T>{rho * surf_in[3 * a] + ox, rho * surf_in[3 * a + 1] + oy, rho * surf_in[3 * a + 2] + oz,
                              R == 1 ? ps[a] : T(0)};
            __builtin_amdgcn_wave_barrier();
#pragma unroll 4
            for (int a = sub; a < n_eq; a += lpt) {
                const P4<T> f = st[a];
                const T dx = ui.x - f.x, dy = ui.y - f.y, dz = ui.z - f.z;
                const T rinv = rsq(dx * dx + dy * dy + dz * dz);
                if constexpr (R == 1) {
                    acc[0] += f.w * rinv;
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] += ps[(int64_t)r * nep + a] * rinv;
                }
            }
        }
        for (int off = lpt >> 1; off > 0; off >>= 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += __shfl_xor(acc[r], off);
        }
        if (valid && sub == 0) {
            const int64_t dst = perm[i];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nrhs) out[dst + r * ld] += scale * acc[r];
        }
    }
}

// S2L check potentials of the W cubes (one wave per cube, lanes over the
// (1+d) surface points): CX[(w*R + r)*nep + a] = sum over the cube's X
// entries of sum_j sig_s[j*R + r] / |s_a - (rho u_j + o)| for a < n_eq, 0 up
// to nep; the points of each X leaf are mapped into the cube's units and
// staged in LDS in batches of at most CAP.
template <typename T, int R>
__global__ void __launch_bounds__(256) eval_s2l_kernel(
    int64_t n_cube, const P4<T>* __restrict__ pts, const T* __restrict__ sig, const int32_t* __restrict__ leaf_ptr,
    const int32_t* __restrict__ ent_ptr, const int32_t* __restrict__ ent_leaf, const T* __restrict__ ent_geo,
    const T* __restrict__ surf_in, int n_eq, int nep, T* __restrict__ CX) {
    constexpr int WPB = 4;
    constexpr int CAP = 64;
    __shared__ P4<T> sp[WPB][CAP];
    __shared__ T ss[WPB][R > 1 ? CAP * R : 1];
    const int wave = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * WPB + wave;
    if (w >= n_cube) return;
    const int lane = threadIdx.x & 63;
    P4<T>* st = sp[wave];
    T* sst = ss[wave];
    constexpr int NA = (19 * 16 + 63) / 64;
    T sx[NA], sy[NA], sz[NA];
    T acc[NA][R];
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int a = k * 64 + lane;
        const bool ok = a < n_eq;
        sx[k] = ok ? surf_in[3 * a] : T(0);
        sy[k] = ok ? surf_in[3 * a + 1] : T(0);
        sz[k] = ok ? surf_in[3 * a + 2] : T(0);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[k][r] = 0;
    }
    const int na = (nep + 63) / 64;
    const int k0 = ent_ptr[w], k1 = ent_ptr[w + 1];
    for (int ke = k0; ke < k1; ++ke) {
        const int leaf = ent_leaf[ke];
        const T rho = ent_geo[4 * ke], ox = ent_geo[4 * ke + 1], oy = ent_geo[4 * ke + 2], oz = ent_geo[4 * ke + 3];
        const int p0 = leaf_ptr[leaf], p1 = leaf_ptr[leaf + 1];
        for (int base = p0; base < p1; base += CAP) {
            const int cnt = min(CAP, p1 - base);
            __builtin_amdgcn_wave_barrier();
            if (lane < cnt) {
                const P4<T> v = pts[base + lane];
                T w0 = T(0);
                if constexpr (R == 1) {
                    w0 = sig[base + lane];
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) sst[lane * R + r] = sig[(int64_t)(base + lane) * R + r];
                }
                st[lane] = P4<T>{rho * v.x + ox, rho * v.y + oy, rho * v.z + oz, w0};
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll 2
            for (int jj = 0; jj < cnt; ++jj) {
                const P4<T> f = st[jj];
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    if (k < na) {
                        const T dx = sx[k] - f.x, dy = sy[k] - f.y, dz = sz[k] - f.z;
                        const T rinv = rsq(dx * dx + dy * dy + dz * dz);
                        if constexpr (R == 1) {
                            acc[k][0] += f.w * rinv;
                        } else {
#pragma unroll
                            for (int r = 0; r < R; ++r) acc[k][r] += sst[jj * R + r] * rinv;
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int a = k * 64 + lane;
        if (k < na && a < nep) {
#pragma unroll
            for (int r = 0; r < R; ++r) CX[(w * R + r) * nep + a] = a < n_eq ? acc[k][r] : T(0);
        }
    }
}

// BEM S2M check potentials (Sec. 4.2): one wave per leaf, lanes over the
// (3-2d) surface; the sources are the 7 quadrature points of every triangle of
// the leaf, staged as (x, y, z, W q) in leaf units (W = rule weight x area,
// divided by r_L for the double layer), with the triangle's unit normal for
// the double layer, whose kernel n.(s - y) / |s - y|^3 replaces 1/|s - y|.
template <typename T, bool DL>
__global__ void __launch_bounds__(256) eval_surface_bem_kernel(
    int64_t n_leaf, const P4<T>* __restrict__ qp, const P4<T>* __restrict__ tn, const T* __restrict__ sig,
    const int32_t* __restrict__ leaf_ptr, const T* __restrict__ surf, int n_eq, int nep, T* __restrict__ C) {
    constexpr int WPB = 4;
    constexpr int CAP = 64;
    __shared__ P4<T> sp[WPB][CAP];
    __shared__ P4<T> sn[WPB][DL ? CAP : 1];
    const int wave = threadIdx.x >> 6;
    const int64_t leaf = (int64_t)blockIdx.x * WPB + wave;
    if (leaf >= n_leaf) return;
    const int lane = threadIdx.x & 63;
    P4<T>* st = sp[wave];
    P4<T>* stn = sn[DL ? wave : 0];
    constexpr int NA = (19 * 16 + 63) / 64;
    T sx[NA], sy[NA], sz[NA], acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int a = k * 64 + lane;
        const bool ok = a < n_eq;
        sx[k] = ok ? surf[3 * a] : T(0);
        sy[k] = ok ? surf[3 * a + 1] : T(0);
        sz[k] = ok ? surf[3 * a + 2] : T(0);
        acc[k] = 0;
    }
    const int na = (nep + 63) / 64;
    const int q0 = 7 * leaf_ptr[leaf], q1 = 7 * leaf_ptr[leaf + 1];
    for (int base = q0; base < q1; base += CAP) {
        const int cnt = min(CAP, q1 - base);
        __builtin_amdgcn_wave_barrier();
        if (lane < cnt) {
            const int qi = base + lane;
            const P4<T> v = qp[qi];
            st[lane] = P4<T>{v.x, v.y, v.z, v.w * sig[qi / 7]};
            if constexpr (DL) stn[lane] = tn[qi / 7];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll 2
        for (int jj = 0; jj < cnt; ++jj) {
            const P4<T> f = st[jj];
            P4<T> nv{0, 0, 0, 0};
            if constexpr (DL) nv = stn[jj];
#pragma unroll
            for (int k = 0; k < NA; ++k) {
                if (k < na) {
                    const T dx = sx[k] - f.x, dy = sy[k] - f.y, dz = sz[k] - f.z;
                    const T rinv = rsq(dx * dx + dy * dy + dz * dz);
                    if constexpr (DL)
                        acc[k] += f.w * (nv.x * dx + nv.y * dy + nv.z * dz) * rinv * rinv * rinv;
                    else
                        acc[k] += f.w * rinv;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int a = k * 64 + lane;
        if (k < na && a < nep) C[leaf * nep + a] = a < n_eq ? acc[k] : T(0);
    }
}

// Elementary functions of the BEM element integrals. FP32: the hardware
// square root, reciprocal and log2 (about 1 ulp each), and an arctangent
// from a degree-8 polynomial in t^2 (atan(t) ~ t P(t^2) on [0, 1], fitted by
// fit_atan.py; largest error 9e-8) with the octant reduction of atan2; the
// integrals are sums of many such terms checked against the FP64 oracle at
// 1e-5. FP64: the library functions.
__device__ __forceinline__ float bem_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double bem_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float bem_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double bem_div(double a, double b) { return a / b; }
__device__ __forceinline__ float bem_log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ double bem_log(double x) { return log(x); }
__device__ __forceinline__ float bem_atan2(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float s = t * t;
    float p = 0.0024567225482314825f;
    p = __builtin_fmaf(p, s, -0.01440135296434164f);
    p = __builtin_fmaf(p, s, 0.039781223982572556f);
    p = __builtin_fmaf(p, s, -0.07234857976436615f);
    p = __builtin_fmaf(p, s, 0.10498946905136108f);
    p = __builtin_fmaf(p, s, -0.14161229133605957f);
    p = __builtin_fmaf(p, s, 0.19985906779766083f);
    p = __builtin_fmaf(p, s, -0.33332598209381104f);
    p = __builtin_fmaf(p, s, 0.9999998807907104f);
    float r = t * p;
    if (ay > ax) r = 1.5707963267948966f - r;
    if (x < 0.0f) r = 3.1415926535897932f - r;
    return copysignf(r, y);
}
__device__ __forceinline__ double bem_atan2(double y, double x) { return atan2(y, x); }

// int_T 1/|x - y| dS_y over a flat triangle (vertices a, b, c, unit normal n)
// in closed form: for the projection x0 of x on the plane and its height h,
// every edge with in-plane outward normal m and unit tangent t adds
// p ln((R+ + s+)/(R- + s-)) - |h| (atan(p s+ / (R0^2 + |h| R+)) - atan(p s- /
// (R0^2 + |h| R-))), p = (start - x0).m, s = (end points - x0).t, R0^2 = p^2 +
// h^2, R = sqrt(s^2 + R0^2) (Wilton et al. 1984); R + s is formed as R0^2 /
// (R - s) for s < 0, which has no cancellation. Evaluated with fewer
// transcendentals: R- and R+ are the distances from x to the edge's end
// points (three square roots per triangle, not two per edge), and the
// difference of the two arctangents is one atan2: with D = R0^2 + |h| R > 0,
// atan(p s+ / D+) - atan(p s- / D-) = atan2(p (s+ D- - s- D+), D+ D- + p^2 s+ s-)
// (both angles lie in (-pi/2, pi/2), so the difference is the angle of the
// point (cos, sin) ~ (D+ D- + p^2 s+ s-, p (s+ D- - s- D+)), scaled by D+ D-).
template <typename T>
__device__ __forceinline__ T tri_inv_r(T x, T y, T z, const P4<T>& a, const P4<T>& b, const P4<T>& c,
                                       const P4<T>& n, const P4<T> (&te)[3], const P4<T> (&me)[3]) {
    // te[e]: unit tangent of edge e (vertex e to e+1) and its length in w;
    // me[e]: the in-plane outward normal t x n
    const T h = (x - a.x) * n.x + (y - a.y) * n.y + (z - a.z) * n.z;
    const T x0 = x - h * n.x, y0 = y - h * n.y, z0 = z - h * n.z;
    const T ah = fabs(h);
    const P4<T>* vs[3] = {&a, &b, &c};
    T dist[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const T dx = vs[e]->x - x, dy = vs[e]->y - y, dz = vs[e]->z - z;
        dist[e] = bem_sqrt(dx * dx + dy * dy + dz * dz);
    }
    T total = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const P4<T>& u = *vs[e];
        const T dx = u.x - x0, dy = u.y - y0, dz = u.z - z0;
        const T p = dx * me[e].x + dy * me[e].y + dz * me[e].z;
        const T sm = dx * te[e].x + dy * te[e].y + dz * te[e].z;
        const T sp = sm + te[e].w;
        const T r0 = p * p + h * h;
        const T rm = dist[e], rp = dist[(e + 1) % 3];
        if (p != T(0)) {
            const T num = sp >= T(0) ? rp + sp : bem_div(r0, rp - sp);
            const T den = sm >= T(0) ? rm + sm : bem_div(r0, rm - sm);
            total += p * bem_log(bem_div(num, den));
            if (ah > T(0)) {
                const T dp = r0 + ah * rp, dm = r0 + ah * rm;
                total -= ah * bem_atan2(p * (sp * dm - sm * dp), dp * dm + p * p * sp * sm);
            }
        }
    }
    return total;
}

// Edge data of a triangle for tri_inv_r: unit tangents with lengths, and
// in-plane outward normals.
template <typename T>
__device__ __forceinline__ void tri_edges(const P4<T>& a, const P4<T>& b, const P4<T>& c, const P4<T>& n,
                                          P4<T> (&te)[3], P4<T> (&me)[3]) {
    const P4<T>* vs[3] = {&a, &b, &c};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const P4<T>& u = *vs[e];
        const P4<T>& w = *vs[(e + 1) % 3];
        const T ex = w.x - u.x, ey = w.y - u.y, ez = w.z - u.z;
        const T len = bem_sqrt(ex * ex + ey * ey + ez * ez);
        const T il = bem_div(T(1), len);
        const T tx = ex * il, ty = ey * il, tz = ez * il;
        te[e] = P4<T>{tx, ty, tz, len};
        me[e] = P4<T>{ty * n.z - tz * n.y, tz * n.x - tx * n.z, tx * n.y - ty * n.x, T(0)};
    }
}

// signed solid angle of the triangle (a, b, c) seen from x (Van Oosterom and
// Strackee 1983): positive when x is on the side the normal points away from
template <typename T>
__device__ __forceinline__ T tri_solid_angle(T x, T y, T z, const P4<T>& a, const P4<T>& b, const P4<T>& c) {
    const T r1x = a.x - x, r1y = a.y - y, r1z = a.z - z;
    const T r2x = b.x - x, r2y = b.y - y, r2z = b.z - z;
    const T r3x = c.x - x, r3y = c.y - y, r3z = c.z - z;
    const T l1 = bem_sqrt(r1x * r1x + r1y * r1y + r1z * r1z);
    const T l2 = bem_sqrt(r2x * r2x + r2y * r2y + r2z * r2z);
    const T l3 = bem_sqrt(r3x * r3x + r3y * r3y + r3z * r3z);
    const T num = r1x * (r2y * r3z - r2z * r3y) + r1y * (r2z * r3x - r2x * r3z) + r1z * (r2x * r3y - r2y * r3x);
    const T den = l1 * l2 * l3 + (r1x * r2x + r1y * r2y + r1z * r2z) * l3 + (r1x * r3x + r1y * r3y + r1z * r3z) * l2 +
                  (r2x * r3x + r2y * r3y + r2z * r3z) * l1;
    return T(2) * bem_atan2(num, den);
}

// BEM near field (S2T, Sec. 4.2): one wave per target leaf, `lpt` lanes per
// collocation point splitting the near-field triangles. The triangles of all
// near-field leaves are staged in batches of CAP, one per lane, as the near
// field of points is (entries resolved one per lane, a prefix sum of their
// triangle counts, each staged triangle's entry found by a binary search over
// the lanes): one memory latency per batch. A staged triangle is its vertices
// shifted into the target leaf's units by the cube offset, its unit normal
// (q in the first vertex's w, the triangle's index in the second's) and, for
// the single layer, its edge tangents, lengths and in-plane normals, formed
// once per staged triangle instead of once per pair. Single layer: out =
// scale * sum_j q_j int_T 1/|x - y| (scale = r_L / (4 pi)); double layer:
// scale * sum_j q_j Omega_j (scale = -1/(4 pi)), the self triangle
// contributing 0 (principal value). Writes out.
template <typename T, bool DL>
__global__ void __launch_bounds__(256) eval_near_bem_kernel(
    int64_t n_leaf, const P4<T>* __restrict__ pts, const P4<T>* __restrict__ tri, const T* __restrict__ sig,
    const int32_t* __restrict__ leaf_ptr, const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_leaf,
    const int32_t* __restrict__ near_code, T scale, const int32_t* __restrict__ perm, T* __restrict__ out) {
    constexpr int WPB = 4;
    constexpr int CAP = sizeof(T) == 4 ? 64 : 32;
    constexpr int NP = DL ? 4 : 10;   // 4-vectors per staged triangle
    __shared__ P4<T> sp[WPB][NP * CAP];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t leaf = (int64_t)blockIdx.x * WPB + wave;
    if (leaf >= n_leaf) return;
    P4<T>* st = sp[wave];
    const int p0 = leaf_ptr[leaf];
    const int ne = leaf_ptr[leaf + 1] - p0;
    int lpt = 64;
    while (lpt > 1 && (64 / lpt) < ne) lpt >>= 1;
    const int tpr = 64 / lpt;
    const int sub = lane & (lpt - 1);
    const int q0 = near_ptr[leaf], q1 = near_ptr[leaf + 1];
    // near-field entries, one per lane: first triangle, count, offset code,
    // and the inclusive prefix sum of the counts
    const int nq = min(q1 - q0, 64);
    int e_b0 = 0, e_code = 0, e_cnt = 0;
    if (lane < nq) {
        const int nb = near_leaf[q0 + lane];
        e_code = near_code[q0 + lane];
        e_b0 = leaf_ptr[nb];
        e_cnt = leaf_ptr[nb + 1] - e_b0;
    }
    int incl = e_cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    const int n_near = __shfl(incl, 63);
    for (int tb = 0; tb < ne; tb += tpr) {
        const int tl = tb + lane / lpt;
        const bool valid = tl < ne;
        const int i = p0 + (valid ? tl : 0);
        const P4<T> ui = pts[i];
        T acc = 0;
        for (int base = 0; base < n_near; base += CAP) {
            const int cnt = min(CAP, n_near - base);
            __builtin_amdgcn_wave_barrier();
            for (int slot = lane; slot < CAP; slot += 64) {
                const int sidx = base + slot;
                int e = 0;
#pragma unroll
                for (int stp = 32; stp > 0; stp >>= 1) {
                    const int v = __shfl(incl, e + stp - 1);
                    if (v <= sidx) e += stp;
                }
                e = min(e, 63);
                const int b0 = __shfl(e_b0, e);
                const int ex = __shfl(incl, e) - __shfl(e_cnt, e);
                const int code = __shfl(e_code, e);
                if (slot < cnt) {
                    const int j = b0 + (sidx - ex);
                    // source shifted into target-leaf units: s - 2 d, d = target - source cube
                    const T ox = T(-2 * (code / 9 - 1)), oy = T(-2 * ((code / 3) % 3 - 1)), oz = T(-2 * (code % 3 - 1));
                    P4<T> v[4];
#pragma unroll
                    for (int part = 0; part < 4; ++part) v[part] = tri[4 * (int64_t)j + part];
#pragma unroll
                    for (int part = 0; part < 3; ++part) {
                        v[part].x += ox;
                        v[part].y += oy;
                        v[part].z += oz;
                    }
                    v[0].w = sig[j];
                    v[1].w = T(j);
#pragma unroll
                    for (int part = 0; part < 4; ++part) st[NP * slot + part] = v[part];
                    if constexpr (!DL) {
                        P4<T> te[3], me[3];
                        tri_edges(v[0], v[1], v[2], v[3], te, me);
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            st[NP * slot + 4 + k] = te[k];
                            st[NP * slot + 7 + k] = me[k];
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            for (int t = sub; t < cnt; t += lpt) {
                const P4<T> a = st[NP * t], b = st[NP * t + 1], c = st[NP * t + 2];
                if constexpr (DL) {
                    if ((int)b.w != i) acc += a.w * tri_solid_angle(ui.x, ui.y, ui.z, a, b, c);
                } else {
                    const P4<T> n = st[NP * t + 3];
                    P4<T> te[3], me[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        te[k] = st[NP * t + 4 + k];
                        me[k] = st[NP * t + 7 + k];
                    }
                    acc += a.w * tri_inv_r(ui.x, ui.y, ui.z, a, b, c, n, te, me);
                }
            }
        }
        for (int off = lpt >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (valid && sub == 0) out[perm[i]] = scale * acc;
    }
}

// ------------------------------------------------------------------------
// Leaf stages fused with their reduced-operator products (FP32 plans, one
// right-hand side). The products use the FP32 16x16x4 MFMA: lane (j, g)
// supplies A[j][4 g + e] and B[4 g + e][j] of each K-step and holds the
// output rows 4 g + q of column j.
typedef float fv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ fv4 leaf_mfma(float a, float b, fv4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// S2M: the check potentials of LB leaves on the (3-2d) surface (one wave per
// leaf in turn, as eval_surface_kernel) are kept in LDS as the columns of
// C (KDIM x LB), then Y[leaf_row[leaf]] = scale * A C[leaf] for the k_pad rows
// of A (the reduced S~, or T~^T in the adjoint; row-major, lda = KDIM).
// Leaves with leaf_row < 0 are computed and not stored.
template <int KP16>
__global__ void __launch_bounds__(256) s2m_fused_kernel(int64_t n_leaf, const P4<float>* __restrict__ pts,
                                                        const float* __restrict__ sig,
                                                        const int32_t* __restrict__ leaf_ptr,
                                                        const float* __restrict__ surf, int n_eq,
                                                        const float* __restrict__ A, int MB,
                                                        const int32_t* __restrict__ leaf_row, float scale,
                                                        float* __restrict__ Y, int ldy) {
    constexpr int LB = 32, WPB = 4, CAP = 64;
    constexpr int KDIM = KP16 * 16, LDB = KDIM + 4;
    constexpr int NA = (KDIM + 63) / 64;
    __shared__ P4<float> sp[WPB][CAP];
    __shared__ __align__(16) float cs[LB * LDB];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t l0 = (int64_t)blockIdx.x * LB;
    const int nl = (int)min((int64_t)LB, n_leaf - l0);
    float sx[NA], sy[NA], sz[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int a = k * 64 + lane;
        const bool ok = a < n_eq;
        sx[k] = ok ? surf[3 * a] : 0.0f;
        sy[k] = ok ? surf[3 * a + 1] : 0.0f;
        sz[k] = ok ? surf[3 * a + 2] : 0.0f;
    }
    P4<float>* st = sp[wave];
    // point ranges of the workgroup's leaves: lane l holds leaf_ptr[l0 + l]
    // (l <= nl), read back with readlane
    const int lp = leaf_ptr[l0 + min(lane, nl)];
    // the first batch of a leaf's points is loaded one leaf ahead (the next
    // leaf of this wave while the current one is computed); the loads are
    // unconditional (index clamped into the leaf, or into the last leaf past
    // the workgroup's end) so that the compiler's wait for them is exact
    auto load_first = [&](int ll, P4<float>& v, float& w) {
        const int l = min(ll, nl - 1);
        const int p0 = __builtin_amdgcn_readlane(lp, l), p1 = __builtin_amdgcn_readlane(lp, l + 1);
        const int i = p1 > p0 ? min(p0 + lane, p1 - 1) : 0;
        v = pts[i];
        w = sig[i];
    };
    P4<float> vn;
    float wn;
    load_first(wave, vn, wn);
    for (int ll = wave; ll < LB; ll += WPB) {
        float acc[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k] = 0.0f;
        const P4<float> v0 = vn;
        const float w0 = wn;
        load_first(ll + WPB, vn, wn);
        auto batch = [&](int cnt) {
#pragma unroll 2
            for (int jj = 0; jj < cnt; ++jj) {
                const P4<float> f = st[jj];
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    const float dx = sx[k] - f.x, dy = sy[k] - f.y, dz = sz[k] - f.z;
                    acc[k] += f.w * rsq(dx * dx + dy * dy + dz * dz);
                }
            }
        };
        if (ll < nl) {
            const int p0 = __builtin_amdgcn_readlane(lp, ll), p1 = __builtin_amdgcn_readlane(lp, ll + 1);
            // first batch from the prefetched registers, further ones (leaves of
            // more than CAP points) loaded in place
            const int cnt0 = min(CAP, p1 - p0);
            __builtin_amdgcn_wave_barrier();
            if (lane < cnt0) st[lane] = P4<float>{v0.x, v0.y, v0.z, w0};
            __builtin_amdgcn_wave_barrier();
            batch(cnt0);
            for (int base = p0 + CAP; base < p1; base += CAP) {
                const int cnt = min(CAP, p1 - base);
                __builtin_amdgcn_wave_barrier();
                if (lane < cnt) {
                    const P4<float> v = pts[base + lane];
                    st[lane] = P4<float>{v.x, v.y, v.z, sig[base + lane]};
                }
                __builtin_amdgcn_wave_barrier();
                batch(cnt);
            }
        }
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int a = k * 64 + lane;
            if (a < KDIM) cs[ll * LDB + a] = (a < n_eq && ll < nl) ? acc[k] : 0.0f;
        }
    }
    // rows of A for this wave's first 16-row block, issued before the barrier
    // so that they arrive while the other waves finish their leaves (a fence
    // keeps the compiler from spreading the loads over the MFMAs, which would
    // wait for each in turn); further blocks load theirs in place
    const int j = lane & 15, grp = lane >> 4;
    fv4 a0[KP16];
    {
        const float* ar = A + (int64_t)(min(wave, MB - 1) * 16 + j) * KDIM + 4 * grp;
#pragma unroll
        for (int t = 0; t < KP16; ++t) a0[t] = *reinterpret_cast<const fv4*>(ar + 16 * t);
    }
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    int orow[LB / 16];
#pragma unroll
    for (int b = 0; b < LB / 16; ++b) {
        const int c = b * 16 + j;
        orow[b] = c < nl ? leaf_row[l0 + c] : -1;
    }
    auto rows = [&](int blk, const fv4 (&a)[KP16]) {
#pragma unroll
        for (int cb = 0; cb < LB / 16; ++cb) {
            if (cb * 16 >= nl) break;
            fv4 d0 = fv4{0, 0, 0, 0}, d1 = fv4{0, 0, 0, 0};
            const float* bc = cs + (cb * 16 + j) * LDB + 4 * grp;
#pragma unroll
            for (int t = 0; t < KP16; ++t) {
                const fv4 bv = *reinterpret_cast<const fv4*>(bc + 16 * t);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (t & 1)
                        d1 = leaf_mfma(a[t][e], bv[e], d1);
                    else
                        d0 = leaf_mfma(a[t][e], bv[e], d0);
                }
            }
            const int o = orow[cb];
            if (o >= 0) {
                float* yp = Y + (int64_t)o * ldy + blk * 16;
#pragma unroll
                for (int q = 0; q < 4; ++q) yp[4 * grp + q] = scale * (d0[q] + d1[q]);
            }
        }
    };
    if (wave < MB) rows(wave, a0);
    for (int blk = wave + WPB; blk < MB; blk += WPB) {
        fv4 a[KP16];
        const float* ar = A + (int64_t)(blk * 16 + j) * KDIM + 4 * grp;
#pragma unroll
        for (int t = 0; t < KP16; ++t) a[t] = *reinterpret_cast<const fv4*>(ar + 16 * t);
        __builtin_amdgcn_sched_barrier(0);
        rows(blk, a);
    }
}

// L2P: E (the leaves' downward equivalent densities) of LB leaves on MFMA,
// E[leaf] = A X[leaf_row[leaf]] (A = T~, or S~^T in the adjoint: NR16 * 16
// rows of K = KP16 * 16; X rows of ldx), kept in LDS, then the far field at
// each leaf's points (one wave per leaf in turn, the surface and E staged as
// 4-vectors) added to out: out[perm[i]] += far_scale * sum_a E_a / |u_i - s_a|.
// Leaves with leaf_row < 0 get no far field.
template <int KP16, int NR16, int LB>
__global__ void __launch_bounds__(256) l2p_fused_kernel(int64_t n_leaf, const P4<float>* __restrict__ pts,
                                                        const int32_t* __restrict__ leaf_ptr,
                                                        const int32_t* __restrict__ leaf_row,
                                                        const float* __restrict__ A,
                                                        const float* __restrict__ X, int ldx,
                                                        const float* __restrict__ surf, int n_eq, float far_scale,
                                                        const int32_t* __restrict__ perm, float* __restrict__ out) {
    constexpr int WPB = 4;
    constexpr int KDIM = KP16 * 16, LDB = KDIM + 4;
    constexpr int NROW = NR16 * 16, LDE = NROW + 4;
    constexpr int BB = LB * LDB, FS = WPB * NROW * 4;
    __shared__ __align__(16) float xs[BB > FS ? BB : FS];   // gathered X columns, then the staged surfaces
    __shared__ __align__(16) float es[LB * LDE];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t l0 = (int64_t)blockIdx.x * LB;
    const int nl = (int)min((int64_t)LB, n_leaf - l0);
    const int j = lane & 15, grp = lane >> 4;
    // the loads of this phase before its first wait: the rows of A of this
    // wave's first 16-row block, then the gathered X columns (unconditional:
    // a leaf without a row, or past the end, reads row 0 and stages zeros);
    // further blocks load their rows of A in place
    constexpr int NG = (LB * (KDIM / 4) + 255) / 256;
    auto load_a = [&](int blk, fv4 (&a)[KP16]) {
        const float* ar = A + (int64_t)(blk * 16 + j) * KDIM + 4 * grp;
#pragma unroll
        for (int t = 0; t < KP16; ++t) a[t] = *reinterpret_cast<const fv4*>(ar + 16 * t);
    };
    fv4 a0[KP16];
    load_a(min(wave, NR16 - 1), a0);
    fv4 gv[NG];
    bool gz[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) {
        const int f = min(tid + 256 * i, LB * (KDIM / 4) - 1);
        const int c = f / (KDIM / 4), part = 4 * (f - c * (KDIM / 4));
        const int r = c < nl ? leaf_row[l0 + c] : -1;
        gz[i] = r < 0;
        gv[i] = *reinterpret_cast<const fv4*>(X + (int64_t)(r < 0 ? 0 : r) * ldx + part);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
        const int f = tid + 256 * i;
        if (f < LB * (KDIM / 4)) {
            const int c = f / (KDIM / 4), part = 4 * (f - c * (KDIM / 4));
            *reinterpret_cast<fv4*>(xs + c * LDB + part) = gz[i] ? fv4{0, 0, 0, 0} : gv[i];
        }
    }
    __syncthreads();
    for (int blk = wave; blk < NR16; blk += WPB) {
        fv4 a[KP16];
        if (blk == wave) {
#pragma unroll
            for (int t = 0; t < KP16; ++t) a[t] = a0[t];
        } else {
            load_a(blk, a);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int cb = 0; cb < LB / 16; ++cb) {
            fv4 d0 = fv4{0, 0, 0, 0}, d1 = fv4{0, 0, 0, 0};
            const float* bc = xs + (cb * 16 + j) * LDB + 4 * grp;
#pragma unroll
            for (int t = 0; t < KP16; ++t) {
                const fv4 bv = *reinterpret_cast<const fv4*>(bc + 16 * t);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (t & 1)
                        d1 = leaf_mfma(a[t][e], bv[e], d1);
                    else
                        d0 = leaf_mfma(a[t][e], bv[e], d0);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) es[(cb * 16 + j) * LDE + blk * 16 + 4 * grp + q] = d0[q] + d1[q];
        }
    }
    __syncthreads();
    P4<float>* fs = reinterpret_cast<P4<float>*>(xs) + wave * NROW;
    // point ranges and Q/P rows of the workgroup's leaves: lane l holds those
    // of leaf l, read back with readlane
    const int lp = leaf_ptr[l0 + min(lane, nl)];
    const int lr = leaf_row[l0 + min(lane, nl - 1)];
    // the surface in registers (lane a, a + 64, ...), staged with each leaf's E
    constexpr int NS = (NROW + 63) / 64;
    float fx[NS], fy[NS], fz[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int a = min(k * 64 + lane, n_eq - 1);
        fx[k] = surf[3 * a];
        fy[k] = surf[3 * a + 1];
        fz[k] = surf[3 * a + 2];
    }
    // lanes per target (a power of two) so that one pass covers the leaf's
    // points where it can. The first pass's target point and output index
    // are loaded one leaf ahead, unconditionally (the index clamped into the
    // leaf, or into the last leaf past the workgroup's end), and the old
    // output value before the next leaf's loads, so that each wait covers
    // exactly the loads it needs; further passes (leaves of more than 64
    // points) load in place.
    auto lanes_per_target = [](int ne) {
        int lpt = 64;
        while (lpt > 1 && (64 / lpt) < ne) lpt >>= 1;
        return lpt;
    };
    auto load_first = [&](int ll, P4<float>& u, int& pi) {
        const int l = min(ll, nl - 1);
        const int p0 = __builtin_amdgcn_readlane(lp, l), ne = __builtin_amdgcn_readlane(lp, l + 1) - p0;
        const int i = ne > 0 ? p0 + min(lane / lanes_per_target(ne), ne - 1) : 0;
        u = pts[i];
        pi = perm[i];
    };
    auto far_at = [&](const P4<float>& ui, int lpt, int sub) {
        float far = 0.0f;
#pragma unroll 4
        for (int a = sub; a < n_eq; a += lpt) {
            const P4<float> f = fs[a];
            const float dx = ui.x - f.x, dy = ui.y - f.y, dz = ui.z - f.z;
            far += f.w * rsq(dx * dx + dy * dy + dz * dz);
        }
        for (int off = lpt >> 1; off > 0; off >>= 1) far += __shfl_xor(far, off);
        return far;
    };
    P4<float> un;
    int pn;
    load_first(wave, un, pn);
    for (int ll = wave; ll < nl; ll += WPB) {
        const P4<float> u0 = un;
        const int pi0 = pn;
        const float old0 = out[pi0];
        load_first(ll + WPB, un, pn);
        if (__builtin_amdgcn_readlane(lr, ll) < 0) continue;
        const int p0 = __builtin_amdgcn_readlane(lp, ll);
        const int ne = __builtin_amdgcn_readlane(lp, ll + 1) - p0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int a = k * 64 + lane;
            if (a < n_eq) fs[a] = P4<float>{fx[k], fy[k], fz[k], es[ll * LDE + a]};
        }
        __builtin_amdgcn_wave_barrier();
        const int lpt = lanes_per_target(ne);
        const int tpr = 64 / lpt;
        const int sub = lane & (lpt - 1);
        {
            const float far = far_at(u0, lpt, sub);
            if (lane / lpt < ne && sub == 0) out[pi0] = old0 + far_scale * far;
        }
        for (int tb = tpr; tb < ne; tb += tpr) {
            const int tl = tb + lane / lpt;
            const bool valid = tl < ne;
            const int i = p0 + (valid ? tl : 0);
            const float far = far_at(pts[i], lpt, sub);
            if (valid && sub == 0) out[perm[i]] += far_scale * far;
        }
    }
}

// Vectors of several plans joined into one (gather) and split back
// (scatter): element i of the joined vector belongs to segment s with
// off[s] <= i < off[s+1], at index i - off[s] of that segment's pointer.
template <typename T>
__global__ void __launch_bounds__(256) gather_segments_kernel(int64_t n, SegTable seg, T* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s = 0;
    for (int stp = kMaxSegments / 2; stp > 0; stp >>= 1)
        if (s + stp < seg.count && seg.off[s + stp] <= i) s += stp;
    dst[i] = static_cast<const T*>(seg.ptr[s])[i - seg.off[s]];
}

template <typename T>
__global__ void __launch_bounds__(256) scatter_segments_kernel(int64_t n, SegTable seg, const T* __restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s = 0;
    for (int stp = kMaxSegments / 2; stp > 0; stp >>= 1)
        if (s + stp < seg.count && seg.off[s + stp] <= i) s += stp;
    static_cast<T*>(const_cast<void*>(seg.ptr[s]))[i - seg.off[s]] = src[i];
}

}  // namespace

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

hipError_t launch_eval_targets(int mode, int elt, int R, int64_t n_leaf, const void* pts, const void* qpts,
                               const void* sig_s,
                               const int32_t* leaf_ptr, const int32_t* near_ptr, const int32_t* near_leaf,
                               const int32_t* near_code, const int32_t* leaf_level, const void* leaf_scale,
                               const void* E, const void* surf, int n_eq, int nep, double near_scale,
                               double far_scale, const int32_t* perm, void* out, int64_t ld, int nrhs,
                               hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    if (mode < 1 || mode > 3 || (mode == 2 && E == nullptr)) return hipErrorInvalidValue;
    if (elt == 4 && (mode & 1) && qpts == nullptr) return hipErrorInvalidValue;
    if ((leaf_level == nullptr) != (leaf_scale == nullptr)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_leaf + 3) / 4));
#define KIFMM_EVT(TT, M, AD)                                                                                  \
    KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_targets_kernel<TT, RR, M, AD>), grid, dim3(256), 0, st, n_leaf, \
                                         (const P4<TT>*)pts, (const P4<int32_t>*)qpts, (const TT*)sig_s, leaf_ptr, near_ptr, near_leaf, \
                                         near_code, leaf_level, (const TT*)leaf_scale, (const TT*)E, (const TT*)surf, n_eq, nep, (TT)near_scale, \
                                         (TT)far_scale, perm, (TT*)out, ld, nrhs))
#define KIFMM_EVT_AD(TT, M) \
    if (leaf_level) { KIFMM_EVT(TT, M, true) } else { KIFMM_EVT(TT, M, false) }
    if (elt == 4) {
        if (mode == 1) { KIFMM_EVT_AD(float, 1) } else if (mode == 2) { KIFMM_EVT_AD(float, 2) } else { KIFMM_EVT_AD(float, 3) }
    } else {
        if (mode == 1) { KIFMM_EVT_AD(double, 1) } else if (mode == 2) { KIFMM_EVT_AD(double, 2) } else { KIFMM_EVT_AD(double, 3) }
    }
#undef KIFMM_EVT_AD
#undef KIFMM_EVT
    return hipGetLastError();
}

hipError_t launch_near_reg(int64_t n_leaf, const void* qpts, const void* sig_s, const int32_t* leaf_ptr,
                           const int32_t* near_ptr, const int32_t* near_leaf, const int32_t* near_code,
                           double near_scale, const int32_t* perm, void* out, hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_leaf + 3) / 4));
    hipLaunchKernelGGL(near_reg_kernel, grid, dim3(256), 0, st, n_leaf, (const P4<int32_t>*)qpts,
                       (const float*)sig_s, leaf_ptr, near_ptr, near_leaf, near_code, (float)near_scale, perm,
                       (float*)out);
    return hipGetLastError();
}

hipError_t launch_eval_m2t(int elt, int R, int64_t n_lf, const int32_t* lf_list, const void* pts,
                           const int32_t* leaf_ptr, const void* leaf_scale, const int32_t* ent_ptr,
                           const int32_t* ent_cube, const void* ent_geo, const void* Psi, const void* surf_in,
                           int n_eq, int nep, const int32_t* perm, void* out, int64_t ld, int nrhs,
                           hipStream_t st) {
    if (n_lf == 0) return hipSuccess;
    if (n_eq > 19 * 16) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_lf + 3) / 4));
    if (elt == 4) {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_m2t_kernel<float, RR>), grid, dim3(256), 0, st, n_lf, lf_list,
                                             (const P4<float>*)pts, leaf_ptr, (const float*)leaf_scale, ent_ptr,
                                             ent_cube, (const float*)ent_geo, (const float*)Psi,
                                             (const float*)surf_in, n_eq, nep, perm, (float*)out, ld, nrhs))
    } else {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_m2t_kernel<double, RR>), grid, dim3(256), 0, st, n_lf, lf_list,
                                             (const P4<double>*)pts, leaf_ptr, (const double*)leaf_scale, ent_ptr,
                                             ent_cube, (const double*)ent_geo, (const double*)Psi,
                                             (const double*)surf_in, n_eq, nep, perm, (double*)out, ld, nrhs))
    }
    return hipGetLastError();
}

hipError_t launch_eval_s2l(int elt, int R, int64_t n_cube, const void* pts, const void* sig_s,
                           const int32_t* leaf_ptr, const int32_t* ent_ptr, const int32_t* ent_leaf,
                           const void* ent_geo, const void* surf_in, int n_eq, int nep, void* CX, hipStream_t st) {
    if (n_cube == 0) return hipSuccess;
    if (n_eq > 19 * 16 || nep > 19 * 16) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_cube + 3) / 4));
    if (elt == 4) {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_s2l_kernel<float, RR>), grid, dim3(256), 0, st, n_cube,
                                             (const P4<float>*)pts, (const float*)sig_s, leaf_ptr, ent_ptr, ent_leaf,
                                             (const float*)ent_geo, (const float*)surf_in, n_eq, nep, (float*)CX))
    } else {
        KIFMM_R_SWITCH(R, hipLaunchKernelGGL((eval_s2l_kernel<double, RR>), grid, dim3(256), 0, st, n_cube,
                                             (const P4<double>*)pts, (const double*)sig_s, leaf_ptr, ent_ptr, ent_leaf,
                                             (const double*)ent_geo, (const double*)surf_in, n_eq, nep, (double*)CX))
    }
    return hipGetLastError();
}

hipError_t launch_gather_segments(int elt, int64_t n, const SegTable& seg, void* dst, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (seg.count < 1 || seg.count > kMaxSegments) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (elt == 4)
        hipLaunchKernelGGL((gather_segments_kernel<float>), grid, dim3(256), 0, st, n, seg, (float*)dst);
    else
        hipLaunchKernelGGL((gather_segments_kernel<double>), grid, dim3(256), 0, st, n, seg, (double*)dst);
    return hipGetLastError();
}

hipError_t launch_scatter_segments(int elt, int64_t n, const SegTable& seg, const void* src, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (seg.count < 1 || seg.count > kMaxSegments) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (elt == 4)
        hipLaunchKernelGGL((scatter_segments_kernel<float>), grid, dim3(256), 0, st, n, seg, (const float*)src);
    else
        hipLaunchKernelGGL((scatter_segments_kernel<double>), grid, dim3(256), 0, st, n, seg, (const double*)src);
    return hipGetLastError();
}

hipError_t launch_eval_surface_bem(int elt, int layer, int64_t n_leaf, const void* qp, const void* tn,
                                   const void* sig_s, const int32_t* leaf_ptr, const void* surf, int n_eq, int nep,
                                   void* C, hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    if (n_eq > 19 * 16 || nep > 19 * 16 || (layer == 1 && tn == nullptr)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_leaf + 3) / 4));
#define KIFMM_SB(TT, DLV)                                                                              \
    hipLaunchKernelGGL((eval_surface_bem_kernel<TT, DLV>), grid, dim3(256), 0, st, n_leaf, (const P4<TT>*)qp, \
                       (const P4<TT>*)tn, (const TT*)sig_s, leaf_ptr, (const TT*)surf, n_eq, nep, (TT*)C)
    if (elt == 4) {
        if (layer == 1) KIFMM_SB(float, true); else KIFMM_SB(float, false);
    } else {
        if (layer == 1) KIFMM_SB(double, true); else KIFMM_SB(double, false);
    }
#undef KIFMM_SB
    return hipGetLastError();
}

hipError_t launch_eval_near_bem(int elt, int layer, int64_t n_leaf, const void* pts, const void* tri,
                                const void* sig_s, const int32_t* leaf_ptr, const int32_t* near_ptr,
                                const int32_t* near_leaf, const int32_t* near_code, double scale,
                                const int32_t* perm, void* out, hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_leaf + 3) / 4));
#define KIFMM_NB(TT, DLV)                                                                                   \
    hipLaunchKernelGGL((eval_near_bem_kernel<TT, DLV>), grid, dim3(256), 0, st, n_leaf, (const P4<TT>*)pts,  \
                       (const P4<TT>*)tri, (const TT*)sig_s, leaf_ptr, near_ptr, near_leaf, near_code, (TT)scale, \
                       perm, (TT*)out)
    if (elt == 4) {
        if (layer == 1) KIFMM_NB(float, true); else KIFMM_NB(float, false);
    } else {
        if (layer == 1) KIFMM_NB(double, true); else KIFMM_NB(double, false);
    }
#undef KIFMM_NB
    return hipGetLastError();
}

namespace {

template <int KP16>
hipError_t s2m_fused_t(int64_t n_leaf, const void* pts, const void* sig_s, const int32_t* leaf_ptr, const void* surf,
                       int n_eq, const void* A, int kp, const int32_t* leaf_row, double scale, void* Y, int ldy,
                       hipStream_t st) {
    const dim3 grid((unsigned)((n_leaf + 31) / 32));
    hipLaunchKernelGGL((s2m_fused_kernel<KP16>), grid, dim3(256), 0, st, n_leaf, (const P4<float>*)pts,
                       (const float*)sig_s, leaf_ptr, (const float*)surf, n_eq, (const float*)A, kp / 16, leaf_row,
                       (float)scale, (float*)Y, ldy);
    return hipGetLastError();
}

template <int KP16, int NR16>
hipError_t l2p_fused_t(int64_t n_leaf, const void* pts, const int32_t* leaf_ptr, const int32_t* leaf_row,
                       const void* A, const void* X, int kp, const void* surf, int n_eq, double far_scale,
                       const int32_t* perm, void* out, hipStream_t st) {
    constexpr int LB = 16;   // leaves per workgroup: 16 keeps 8 workgroups (32 waves) on a CU
    const dim3 grid((unsigned)((n_leaf + LB - 1) / LB));
    hipLaunchKernelGGL((l2p_fused_kernel<KP16, NR16, LB>), grid, dim3(256), 0, st, n_leaf, (const P4<float>*)pts,
                       leaf_ptr, leaf_row, (const float*)A, (const float*)X, kp, (const float*)surf, n_eq,
                       (float)far_scale, perm, (float*)out);
    return hipGetLastError();
}

template <int NR16>
hipError_t l2p_fused_nr(int kp16, int64_t n_leaf, const void* pts, const int32_t* leaf_ptr, const int32_t* leaf_row,
                        const void* A, const void* X, int kp, const void* surf, int n_eq, double far_scale,
                        const int32_t* perm, void* out, hipStream_t st) {
#define KIFMM_L2PF(K) \
    case K: return l2p_fused_t<K, NR16>(n_leaf, pts, leaf_ptr, leaf_row, A, X, kp, surf, n_eq, far_scale, perm, out, st);
    switch (kp16) {
        KIFMM_L2PF(1) KIFMM_L2PF(2) KIFMM_L2PF(3) KIFMM_L2PF(4) KIFMM_L2PF(5)
        KIFMM_L2PF(6) KIFMM_L2PF(7) KIFMM_L2PF(8) KIFMM_L2PF(9) KIFMM_L2PF(10)
        default: return hipErrorNotSupported;
    }
#undef KIFMM_L2PF
}

}  // namespace

bool s2m_fused_supported(int nep, int kp) {
    const int r = nep / 16;
    return nep % 16 == 0 && kp % 16 == 0 && kp <= 19 * 16 &&
           (r == 1 || r == 2 || r == 4 || r == 7 || r == 10 || r == 14 || r == 19);
}

bool l2p_fused_supported(int nep, int kp) {
    const int r = nep / 16;
    return nep % 16 == 0 && kp % 16 == 0 && kp <= nep && kp / 16 <= 10 && (r == 4 || r == 7 || r == 10);
}

hipError_t launch_s2m_fused(int64_t n_leaf, const void* pts, const void* sig_s, const int32_t* leaf_ptr,
                            const void* surf, int n_eq, int nep, const void* A, int kp, const int32_t* leaf_row,
                            double scale, void* Y, int ldy, hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    if (nep % 16 || kp % 16 || n_eq > nep || kp > 19 * 16) return hipErrorInvalidValue;
#define KIFMM_S2MF(K) \
    case K: return s2m_fused_t<K>(n_leaf, pts, sig_s, leaf_ptr, surf, n_eq, A, kp, leaf_row, scale, Y, ldy, st);
    switch (nep / 16) {
        KIFMM_S2MF(1) KIFMM_S2MF(2) KIFMM_S2MF(4) KIFMM_S2MF(7) KIFMM_S2MF(10)
        KIFMM_S2MF(14) KIFMM_S2MF(19)
        default: return hipErrorNotSupported;
    }
#undef KIFMM_S2MF
}

hipError_t launch_l2p_fused(int64_t n_leaf, const void* pts, const int32_t* leaf_ptr, const int32_t* leaf_row,
                            const void* A, int kp, int nep, const void* X, const void* surf, int n_eq,
                            double far_scale, const int32_t* perm, void* out, hipStream_t st) {
    if (n_leaf == 0) return hipSuccess;
    if (nep % 16 || kp % 16 || n_eq > nep || kp > nep) return hipErrorInvalidValue;
    switch (nep / 16) {
        case 4: return l2p_fused_nr<4>(kp / 16, n_leaf, pts, leaf_ptr, leaf_row, A, X, kp, surf, n_eq, far_scale, perm, out, st);
        case 7: return l2p_fused_nr<7>(kp / 16, n_leaf, pts, leaf_ptr, leaf_row, A, X, kp, surf, n_eq, far_scale, perm, out, st);
        case 10: return l2p_fused_nr<10>(kp / 16, n_leaf, pts, leaf_ptr, leaf_row, A, X, kp, surf, n_eq, far_scale, perm, out, st);
        default: return hipErrorNotSupported;
    }
}

}  // namespace kifmm
