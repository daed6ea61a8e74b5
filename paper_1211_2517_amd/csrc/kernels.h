// Device kernels of the KIFMM evaluation (gfx950) and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kifmm {

// Device view of a grouped gather GEMM schedule (see GGSched in plan.h).
struct DevSched {
    int n_tiles = 0;
    int n_chunks = 0;
    int cp = 16;
    int max_tile = 0;
    int variant = 0;                    // kernel shape, see gg_variant_rows
    int max_src = 0;                    // largest source row index in the chunks
    int max_cls = 0;                    // largest class in the chunks
    const int32_t* tile_tgt0 = nullptr;
    const int32_t* tile_ntgt = nullptr;
    const int32_t* tile_chunk0 = nullptr;
    // per chunk 4 words: class; 16-column blocks holding data (bits 0..7) and,
    // when nonzero, the 16-wide K-chunks (gg form) or 16-row blocks of A
    // (direct form) holding data (bits 8..); scale (float bits in word 2, or
    // the low and high words of a double in words 2 and 3)
    const int32_t* chunk_meta = nullptr;
    const int32_t* chunk_src = nullptr;
    const int32_t* chunk_col = nullptr;
    // every target of the schedule has exactly one pair: launch_gg runs one
    // workgroup per chunk and writes the results directly (no LDS
    // accumulator); chunk_tgt holds the target row of each chunk slot (-1 empty)
    bool direct = false;
    const int32_t* chunk_tgt = nullptr;
    // direct form only: write the products unscaled (the chunk scale is ignored)
    bool unit_scale = false;
};

// Y[tgt] (+)= scale * sum_chunks A[cls] X[src] for every tile of `s`.
//  A: per-class (MB*16) x (KP16*16) row-major blocks, of which the leading
//  a_rows x a_cols hold data and the rest is zero (the padding is not read);
//  X rows of length ldx (>= KP16*16, zero past a_cols), Y rows of length
//  ldy (>= MB*16); row of (box b, right-hand side r) is b*R + r.
// elt = 4 (FP32 MFMA) or 8 (FP64 MFMA). With b3 (elt 4, KP16 even) A is in
// the split-BF16 layout (per row and 32-wide K-chunk: 32 high BF16 parts, then
// 32 low parts) and the products run on BF16 MFMA with FP32 accumulation.
// Returns a hipError_t.
hipError_t launch_gg(const DevSched& s, int elt, const void* A, int MB, int KP16, int a_rows, int a_cols,
                     const void* X, int ldx, void* Y, int ldy, int R, int accumulate, hipStream_t st,
                     bool b3 = false);

// Kernel shapes (chunks hold 32 / R pairs). Staged forms (gg_kernel: the
// gathered columns are staged in LDS and shared by the waves, one barrier per
// chunk), one 16-row block per wave unless stated:
//   0 = 8 waves (128 output rows per workgroup), all of a CU's LDS;
//   1 = 4 waves (64 rows), all of a CU's LDS;
//   2 = 4 waves (64 rows), half of a CU's LDS, so two workgroups share a CU;
//   3 = 4 waves with two 16-row blocks each (128 rows), all of a CU's LDS,
//       one wave per SIMD (FP32 only).
// Row-slab forms (rs_kernel: every wave loads its operands itself and owns
// its rows of the accumulator, no barrier; FP32 data, K up to 160):
//   4 = 4 waves with two 16-row blocks each (128 rows), one wave per SIMD;
//   5 = 8 waves (128 rows), two waves per SIMD.
constexpr int kGGVariants = 6;
// Whether shape `variant` exists for element size `elt` (4 or 8 bytes) and
// K dimension kp16 * 16.
bool gg_variant_supported(int variant, int elt, int kp16);
// Whether the shape stages the gathered columns in LDS.
bool gg_variant_staged(int variant);
// Output rows per workgroup of a shape (0 for an unknown shape).
int gg_variant_rows(int variant);
// Workgroups of a shape that run on one CU at a time.
int gg_variant_wgs_per_cu(int variant);
// Largest dynamic LDS a workgroup of the shape may use (bytes).
size_t gg_lds_limit(int variant);
// LDS staging buffers (2, or 1 when two would take over half the budget).
int gg_nbuf(int elt, int variant, int KP16);
// Per-workgroup LDS bytes with `cols` accumulator columns (spare columns
// included) and K dimension KP16*16.
size_t gg_lds_bytes(int elt, int variant, int KP16, int cols);

// BEM plans (Sec. 4). Check potentials of the leaves' triangles on the
// (3-2d) surface from their 7-point rules: qp holds 7 (x, y, z, W) per
// triangle in leaf units (sorted order), tn the unit normal per triangle
// (double layer, layer = 1: kernel n.(s - y)/|s - y|^3); C as eval_surface.
hipError_t launch_eval_surface_bem(int elt, int layer, int64_t n_leaf, const void* qp, const void* tn,
                                   const void* sig_s, const int32_t* leaf_ptr, const void* surf, int n_eq, int nep,
                                   void* C, hipStream_t st);
// Near field of BEM plans: out[perm[i]] = scale * sum over the triangles j of
// the near field of q_j int_{T_j} 1/|x_i - y| (layer 0) or q_j Omega_ij (layer
// 1, signed solid angle, self term 0), in leaf units. tri holds 4 (x, y, z, -)
// per triangle: the vertices in its own leaf's units and the unit normal.
hipError_t launch_eval_near_bem(int elt, int layer, int64_t n_leaf, const void* pts, const void* tri,
                                const void* sig_s, const int32_t* leaf_ptr, const int32_t* near_ptr,
                                const int32_t* near_leaf, const int32_t* near_code, double scale,
                                const int32_t* perm, void* out, hipStream_t st);

// FP32 plans with one right-hand side: S2M in one launch. The check
// potentials of the leaves (as launch_eval_surface) stay in LDS and
// Y[leaf_row[e] * ldy + i] = scale * sum_a A[i][a] C_e[a] for i < kp (A: kp x nep
// row-major, zero past n_eq and k); leaves with leaf_row < 0 are not stored.
// Whether the fused leaf kernels exist for n_eq padded to nep and k to kp.
bool s2m_fused_supported(int nep, int kp);
bool l2p_fused_supported(int nep, int kp);
hipError_t launch_s2m_fused(int64_t n_leaf, const void* pts, const void* sig_s, const int32_t* leaf_ptr,
                            const void* surf, int n_eq, int nep, const void* A, int kp, const int32_t* leaf_row,
                            double scale, void* Y, int ldy, hipStream_t st);
// FP32 plans with one right-hand side: L2P in one launch. E_e = A X[leaf_row[e]]
// (A: nep x kp row-major; X rows of kp) stays in LDS and the far field of
// launch_eval_targets mode 2 is added to out (leaves with leaf_row < 0: none).
// hipErrorNotSupported for a (kp, nep) pair that has no instance.
hipError_t launch_l2p_fused(int64_t n_leaf, const void* pts, const int32_t* leaf_ptr, const int32_t* leaf_row,
                            const void* A, int kp, int nep, const void* X, const void* surf, int n_eq,
                            double far_scale, const int32_t* perm, void* out, hipStream_t st);

// FP32 M2M with one right-hand side as one product per parent:
// Y[par_row[i]] = sum_o A_o X[child[8 i + o]] (child -1: absent), A_o the kp x kp
// blocks of octant o (row-major, consecutive), X and Y rows of kp. For
// 16 <= kp <= 160 (m2m_direct_supported).
bool m2m_direct_supported(int kp);
hipError_t launch_m2m_direct(int n_par, const int32_t* par_row, const int32_t* child, const void* A, int kp,
                             const void* X, void* Y, hipStream_t st);

// FP32 direct-form product with one right-hand side, one class per segment:
// for segment s = (cls, i0, n) of seg (3 words each, n <= 16 kDownMaxBlocks)
// and i0 <= i < i0 + n (n >= 1), Y[tgt[i]] += A_cls X[src[i]], A_cls the
// kp x kp block of class cls (row-major, consecutive), X and Y rows of kp,
// the tgt rows distinct and none of them a src row. 16 <= kp <= 160,
// kp % 16 == 0.
constexpr int kDownMaxBlocks = 16;
hipError_t launch_down_direct(int n_seg, const int32_t* seg, const int32_t* tgt, const int32_t* src, const void* A,
                              int kp, const void* X, void* Y, hipStream_t st);

// A joined vector of up to kMaxSegments plans' vectors (passed by value to
// the kernels): segment s holds elements [off[s], off[s+1]) at ptr[s].
constexpr int kMaxSegments = 64;
struct SegTable {
    const void* ptr[kMaxSegments];
    int64_t off[kMaxSegments + 1];
    int count;
};
// dst[i] = ptr[s][i - off[s]] for i < n = off[count] (the joined vector)
hipError_t launch_gather_segments(int elt, int64_t n, const SegTable& seg, void* dst, hipStream_t st);
// ptr[s][i - off[s]] = src[i]
hipError_t launch_scatter_segments(int elt, int64_t n, const SegTable& seg, const void* src, hipStream_t st);

// sig_s[i*R + r] = r < nrhs ? sigma[perm[i] + r*ld] : 0
hipError_t launch_permute_in(int elt, int R, int64_t n, const int32_t* perm, const void* sigma,
                             int64_t ld, int nrhs, void* sig_s, hipStream_t st);

// C[(leaf*R + r)*nep + a] = sum_{j in leaf} sig_s[j*R+r] / |surf_a - u_j|   (a < n_eq; 0 for a < nep)
hipError_t launch_eval_surface(int elt, int R, int64_t n_leaf, const void* pts, const void* sig_s,
                               const int32_t* leaf_ptr, const void* surf, int n_eq, int nep,
                               void* C, hipStream_t st);

// Evaluation at the points of every leaf (i in the leaf, caller index perm[i]):
//   near(i) = near_scale * sum_{near j != i} sig_s[j] / |u_i - u_j + 2 d|
//   far(i)  = far_scale  * sum_a E[(leaf*R+r)*nep + a] / |u_i - surf_a|
// mode 1: out[perm[i] + r*ld] = near(i); mode 2: out[...] += far(i) (E must
// not be null); mode 3: out[...] = near(i) + far(i) (far omitted if E is null).
// pts: leaf-unit coordinates (4 values per point, the last unused); qpts (FP32
// only, modes 1 and 3): the same coordinates in fixed point, 4 int32 per point,
// round(u * 2^28), for exact near-field differences.
// leaf_level and leaf_scale (adaptive form, else both null): the level of
// every leaf and its near-field scale 1/(4 pi r_leaf), which replaces
// near_scale; near codes are those of HostTree's adaptive form (sources one
// level finer or coarser), and leaves above level 2 get no far(i).
hipError_t launch_eval_targets(int mode, int elt, int R, int64_t n_leaf, const void* pts, const void* qpts,
                               const void* sig_s,
                               const int32_t* leaf_ptr, const int32_t* near_ptr,
                               const int32_t* near_leaf, const int32_t* near_code, const int32_t* leaf_level,
                               const void* leaf_scale, const void* E, const void* surf, int n_eq, int nep,
                               double near_scale, double far_scale, const int32_t* perm, void* out, int64_t ld,
                               int nrhs, hipStream_t st);

// Near field of an FP32 uniform plan with one right-hand side (launch_eval_targets
// mode 1 with R = 1 and no adaptive form), its staged sources in registers:
// no LDS. Writes out; the same result bit for bit.
hipError_t launch_near_reg(int64_t n_leaf, const void* qpts, const void* sig_s, const int32_t* leaf_ptr,
                           const int32_t* near_ptr, const int32_t* near_leaf, const int32_t* near_code,
                           double near_scale, const int32_t* perm, void* out, hipStream_t st);

// M2T (adaptive trees): for every leaf lf_list[w] and each of its entries k in
// [ent_ptr[w], ent_ptr[w+1]), the values Psi[(ent_cube[k]*R + r)*nep + a] on the
// surface points rho * surf_in[a] + o (ent_geo[4k..4k+3] = rho, o; leaf units)
// are evaluated at the leaf's points: out[perm[i] + r*ld] += leaf_scale[leaf] *
// sum_k sum_a Psi / |u_i - (rho s_a + o)|.
hipError_t launch_eval_m2t(int elt, int R, int64_t n_lf, const int32_t* lf_list, const void* pts,
                           const int32_t* leaf_ptr, const void* leaf_scale, const int32_t* ent_ptr,
                           const int32_t* ent_cube, const void* ent_geo, const void* Psi, const void* surf_in,
                           int n_eq, int nep, const int32_t* perm, void* out, int64_t ld, int nrhs,
                           hipStream_t st);

// S2L (adaptive trees): CX[(w*R + r)*nep + a] = sum over entries k in
// [ent_ptr[w], ent_ptr[w+1]) and points j of leaf ent_leaf[k] of
// sig_s[j*R + r] / |surf_in[a] - (rho u_j + o)| for a < n_eq, 0 for a < nep.
hipError_t launch_eval_s2l(int elt, int R, int64_t n_cube, const void* pts, const void* sig_s,
                           const int32_t* leaf_ptr, const int32_t* ent_ptr, const int32_t* ent_leaf,
                           const void* ent_geo, const void* surf_in, int n_eq, int nep, void* CX, hipStream_t st);

}  // namespace kifmm
