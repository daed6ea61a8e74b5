/*
 * kifmm.h - C ABI of the MI355X (gfx950) SVD-accelerated kernel-independent FMM.
 *
 * The library evaluates the single-layer Laplace potential of N point sources
 * at the same N points (eq. (1) of Cao, Wen, Rong, "A SVD accelerated
 * kernel-independent fast multipole method and its application to BEM",
 * with G(x,y) = 1/(4 pi |x-y|) of Sec. 4 and the self pair contributing 0):
 *
 *     phi_i = sum_{j != i} sigma_j / (4 pi |x_i - x_j|)
 *
 * by the KIFMM of Sec. 2 whose M2L translations are compressed by the
 * stage-1 SVD of Sec. 3.1 and whose upward and downward passes use the
 * reduced operators of Sec. 3.3 (or, with opts.dense_m2l, the uncompressed
 * operators). The evaluation order is the complete algorithm of Sec. 4.3.
 *
 * Conventions shared by every entry point:
 *  - Every call returns an int status (KIFMM_OK = 0 or a negative code); no
 *    C++ exception crosses the ABI. kifmm_last_error() gives a thread-local
 *    message for the last failing call on the calling thread.
 *  - Host pointers are read during the call only and may be freed after it.
 *  - Device pointers (sigma, phi, g, out) point to memory of the plan's device;
 *    they hold float for KIFMM_FP32 and KIFMM_BF16X3 plans and double for
 *    KIFMM_FP64 plans, in the caller's point order. The caller keeps them alive
 *    until the stream has finished the work.
 *  - The apply calls are asynchronous on `stream` (a hipStream_t, 0 for the
 *    null stream), allocate nothing, copy nothing between host and device and
 *    may be captured in a HIP graph. Applies of one plan must not overlap in
 *    time (they share the plan's workspace): issue them on one stream or
 *    order them with events.
 *  - Threads: plans may be built, applied and destroyed from several host
 *    threads at once (process-wide state - the autotuner's cache and the
 *    kernels' LDS limits - is guarded by locks), but the calls on one plan or
 *    one group must not run concurrently with each other.
 */
#ifndef KIFMM_H
#define KIFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kifmm_plan_s* kifmm_plan_t;   /* opaque; owns its device memory */
typedef struct kifmm_group_s* kifmm_group_t; /* opaque; several plans in one HIP graph */

enum {
    KIFMM_OK = 0,
    KIFMM_EINVAL = -1,     /* invalid argument (sizes, null pointers, ranges) */
    KIFMM_ENOMEM = -2,     /* host or device allocation failed, or opts.mem_limit exceeded */
    KIFMM_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
    KIFMM_ENONFINITE = -4, /* a point coordinate is NaN or infinite */
    KIFMM_ESTATE = -5      /* call not valid for this plan (e.g. apply on a host-only plan) */
};

enum {
    KIFMM_FP64 = 0,  /* every device stage in double */
    KIFMM_FP32 = 1,  /* every device stage in float; M2L/translation GEMMs on FP32 MFMA */
    KIFMM_BF16X3 = 2 /* as FP32, but the M2L GEMM as three BF16 MFMA products (hi*hi + hi*lo +
                        lo*hi) with FP32 accumulation: K~ is split into BF16 high and low parts at
                        plan time, the gathered q~ columns when they are staged; each product then
                        carries a relative error of order 2^-16 (the compressed space is padded to
                        a multiple of 32) */
};

enum {
    KIFMM_SINGLE_LAYER = 0, /* BEM plans: G(x, y) = 1 / (4 pi |x - y|) */
    KIFMM_DOUBLE_LAYER = 1  /* BEM plans: dG(x, y)/dn(y) */
};

typedef struct {
    int precision;      /* KIFMM_FP64 / KIFMM_FP32 / KIFMM_BF16X3; default KIFMM_FP32 */
    double cd;          /* surface constant C_d of d = C_d / sqrt(leaf_size) (Sec. 4.1); default 0.5 */
    double pinv_rcond;  /* relative cutoff of the truncated-SVD pseudo-inverses of the
                           check-to-equivalent matrices; default 1e-10 */
    int depth;          /* 0 = automatic (smallest level whose cubes all hold <= leaf_size
                           points); > 0 forces the leaf level */
    int max_depth;      /* cap of the automatic depth; default 16, at most 20 */
    int dense_m2l;      /* 1 = uncompressed operators (n_eq-dimensional, the baseline); default 0 */
    int max_nrhs;       /* largest nrhs accepted by kifmm_apply_batched; default 1, at most 16 */
    int device;         /* HIP device ordinal; default 0; -1 builds a host-only plan (tree,
                           lists and operators, no device memory: info/export calls only) */
    size_t mem_limit;   /* fail with KIFMM_ENOMEM if the plan's device memory would exceed
                           this many bytes; 0 = no limit */
    int tile_targets;   /* target boxes per M2L work tile; 0 = autotune on the device */
    int m2l_shape;      /* M2L kernel shape (see kifmm_info_t.m2l_variant); -1 = autotuned
                           (default), 0..5 forces one shape (the tile count is still tuned
                           unless tile_targets > 0); KIFMM_EINVAL if the shape does not
                           exist in the requested precision or for the compressed dimension */
    double c2;          /* stage-2 low rank of the compressed M2L matrices (Sec. 3.2): each
                           K~^(t) is replaced by U^ V^ from its SVD, keeping the singular
                           values >= eps2 * Sigma_00 with eps2 = c2 * eps / k (the paper's
                           eps2 = C2 eps1 / k); M2L then runs as two thin products per pair
                           (w = V^ q into a per-pair buffer, then p += U^ w). 0 = off
                           (default). KIFMM_EINVAL with dense_m2l or KIFMM_BF16X3 */
    int adaptive;       /* 1 = adaptive octree (Sec. 2.1 read cube by cube): a cube holding more
                           than leaf_size points is split into its nonempty children, down to
                           max_depth, and the tree is 2:1 balanced (in rounds, every leaf sharing a
                           vertex with a leaf two or more levels finer is split) so that leaves sit
                           at several levels. Near fields then join leaves of neighbouring levels,
                           and the far field between leaves of different levels runs through the
                           W and X lists of the kernel-independent FMM: the upward equivalent
                           densities U~ q~ of a cube evaluated at a coarser leaf's points (M2T),
                           and a coarser leaf's points giving a cube's downward check potential,
                           projected by U~^T (S2L). 0 = uniform depth (default). KIFMM_EINVAL with
                           depth > 0 */
    int fused_leaf;     /* FP32 plans with max_nrhs 1: bit 0 runs S2M (check potentials and S~) as
                           one launch, bit 1 L2P (T~ and the far field) as one launch, where the
                           kernels exist (p <= 6 for L2P); other plans ignore it. Default 3
                           (both); 0 = separate launches (for checks and profiling). The fused
                           and separate forms compute the same sums in the same order */
    int direct_passes;  /* FP32 plans with max_nrhs 1: 1 (default) runs M2M (the adjoint: L2L^T) on
                           the levels of at most 3072 parents as one product per parent over its
                           eight children, and L2L (the adjoint: M2M^T) by segments of one octant
                           with the operator rows held in registers; 0 = the grouped GEMM for both,
                           as in other plans. The forms sum in different orders (results agree to
                           FP32 rounding) */
    int near_overlap;   /* FP32 uniform point plans with max_nrhs 1 and c2 = 0: 1 (default) runs the near field
                           with its staged sources in registers (no LDS) and forks it just before
                           M2L, so it shares the CUs of the M2L launch (which holds their LDS and
                           leaves the vector ALU idle); 0 forks it after the permute, alongside S2M
                           and M2M. The same result bit for bit */
} kifmm_opts_t;

/* Per-stage counters; index with the KIFMM_STAGE_* values. */
enum {
    KIFMM_STAGE_P2M = 0, KIFMM_STAGE_M2M = 1, KIFMM_STAGE_M2L = 2, KIFMM_STAGE_L2L = 3,
    KIFMM_STAGE_L2P = 4, KIFMM_STAGE_P2P = 5, KIFMM_STAGE_PERM = 6, KIFMM_STAGE_COUNT = 7
};

typedef struct {
    int depth;              /* leaf level L */
    int k;                  /* reduced dimension (n_eq when dense_m2l) */
    int n_eq;               /* surface points per cube, p^3 - (p-2)^3 */
    int k_pad;              /* k rounded up to a multiple of 16 (device row stride) */
    int precision;
    int dense_m2l;
    int64_t n;              /* points */
    int64_t n_leaf;         /* nonempty leaves */
    int64_t n_box;          /* nonempty cubes at levels 0..L */
    int64_t near_pairs;     /* (target leaf, source leaf) near-field pairs */
    int64_t p2p_interactions; /* point-point interactions of the near field (self included) */
    int64_t v_pairs;        /* M2L (target, source) pairs over levels 2..L */
    int64_t v_pairs_level[21];
    int64_t boxes_level[21];
    double r0;              /* root half-width */
    double flops[KIFMM_STAGE_COUNT];  /* algorithmic flops per apply (unpadded) */
    double bytes[KIFMM_STAGE_COUNT];  /* algorithmic HBM bytes per apply */
    size_t device_bytes;    /* device memory owned by the plan */
    int m2l_tile_targets;   /* tile size in use */
    double sigma0;          /* largest singular value of K_fat (svd mode), else 0 */
    double plan_seconds;    /* wall time of the plan call */
    int m2l_variant;        /* M2L kernel shape in use. Gathered columns staged in LDS and shared
                               by the waves: 0 = 8 waves x 16 rows per workgroup, 1 = 4 waves x 16
                               rows, 2 = 4 waves x 16 rows at two workgroups per CU, 3 = 4 waves x
                               32 rows (FP32 only). Row slabs, every wave loading its own operands
                               (FP32 and BF16X3, k_pad <= 160): 4 = 4 waves x 32 rows, 5 = 8 waves
                               x 16 rows */
    int m2l_tiles;          /* M2L target tiles (workgroups = tiles x row groups) */
    int m2l_rank_max;       /* stage 2: largest rank of the factored M2L matrices, else 0 */
    double m2l_rank_mean;   /* stage 2: mean rank over the 316 classes, else 0 */
    int adaptive;           /* opts.adaptive of the plan */
    int leaf_level_min;     /* coarsest leaf level (depth for uniform plans) */
    int64_t w_pairs;        /* adaptive: (leaf, cube) W-list pairs = X-list pairs */
    int64_t w_cubes;        /* adaptive: cubes in some W list (their U~ q~ is formed once) */
    double m2t_flops;       /* adaptive: M2T (U~ products and point evaluations) per apply */
    double s2l_flops;       /* adaptive: S2L (point evaluations and U~^T products) per apply */
    int layer;              /* -1 point sources; BEM plans: KIFMM_SINGLE_LAYER / KIFMM_DOUBLE_LAYER */
    int64_t m2l_chunks;     /* M2L chunks (runs of at most 32 pairs of one class in a tile) */
    int64_t m2l_blocks;     /* their 16-column MFMA blocks */
} kifmm_info_t;

/* Fill `o` with the defaults listed above. Returns KIFMM_EINVAL if o is NULL. */
int kifmm_opts_default(kifmm_opts_t* o);

/* Build a plan (Alg. Step 1, Sec. 4.3): octree over the points (Sec. 2.1), near
 * and interaction fields, surfaces (Sec. 2.1 with d of Sec. 4.1), operators in
 * FP64 (S, M, K, L, T of Sec. 2.2; stage-1 SVD of Sec. 3.1 keeping singular
 * values >= eps * Sigma_00; reduced operators of Sec. 3.3), the M2L work
 * schedule, and the upload of all of it to the device.
 *   points:    host, n x 3 row-major doubles (x0,y0,z0,x1,...); copied.
 *   n >= 1; 2 <= p <= 16 (points per cube side; n_eq = p^3 - (p-2)^3);
 *   0 <= eps < 1 (eps = 0 keeps every singular vector); leaf_size >= 1.
 *   out:       receives the plan; set to NULL on failure.
 * Errors: KIFMM_EINVAL, KIFMM_ENONFINITE, KIFMM_ENOMEM, KIFMM_EHIP. */
int kifmm_plan(const double* points, int64_t n, int p, double eps, int leaf_size,
               kifmm_plan_t* out);
/* As kifmm_plan with options (NULL = defaults). */
int kifmm_plan_ex(const double* points, int64_t n, int p, double eps, int leaf_size,
                  const kifmm_opts_t* opts, kifmm_plan_t* out);

/* BEM plan (Sec. 4): the collocation operator of piecewise-constant densities
 * on a mesh of flat triangles, evaluated at the triangles' centroids,
 *     phi_i = sum_j q_j int_{T_j} K(x_i, y) dS_y,
 * K = G (KIFMM_SINGLE_LAYER, eq. of Sec. 4) or dG/dn(y) (KIFMM_DOUBLE_LAYER,
 * n the unit normal given by the vertex order of T_j; the self term is its
 * principal value, 0 on a flat triangle; the free term of a boundary integral
 * equation is the caller's). The octree is built over the centroids (Sec. 4.1,
 * with d = C_d / sqrt(leaf_size)); S2M evaluates the check potentials of the
 * leaf's triangles by a 7-point degree-5 rule on each triangle (with the
 * double-layer kernel for KIFMM_DOUBLE_LAYER, the first step of S2M in
 * Sec. 4.2), S2T the near-field integrals in closed form (single layer: the
 * edge formula of the integral of 1/|x - y| over a flat triangle; double
 * layer: the signed solid angle); the other steps are those of kifmm_plan.
 *   vertices:  host, n_vertices x 3 doubles; triangles: host, n_triangles x 3
 *              vertex indices (0-based); both copied. Point i of the plan (the
 *              order of sigma and phi in kifmm_apply) is triangle i.
 *   opts:      as kifmm_plan_ex; adaptive must be 0 and max_nrhs 1.
 * kifmm_apply, kifmm_apply_noalloc, kifmm_apply_batched (nrhs = 1) and groups
 * (not merged) work on BEM plans; kifmm_apply_adjoint returns KIFMM_ESTATE.
 * Errors: KIFMM_EINVAL (unknown layer, index out of range, zero-area
 * triangle, adaptive or max_nrhs > 1), KIFMM_ENONFINITE, KIFMM_ENOMEM,
 * KIFMM_EHIP. */
int kifmm_plan_bem(const double* vertices, int64_t n_vertices, const int32_t* triangles, int64_t n_triangles,
                   int layer, int p, double eps, int leaf_size, const kifmm_opts_t* opts, kifmm_plan_t* out);

/* phi = F sigma, the FMM approximation of eq. (1) (Alg. Steps 2-4, Sec. 4.3).
 *   sigma, phi: device, n elements each, caller order; must not alias. */
int kifmm_apply(kifmm_plan_t plan, const void* sigma, void* phi, void* stream);

/* As kifmm_apply, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the apply's
 * workspace - permuted densities, surface values, upward and downward
 * coefficients, the device memory kifmm_apply takes from the plan - comes
 * from a static device array of the library (64 MiB, one copy per GPU, held
 * until the process ends), and the call allocates nothing.
 *   sigma, phi: device, n elements each, caller order; must not alias.
 * Every call on one GPU shares that GPU's array, so calls that overlap in time
 * on one GPU (any plans, any streams) race: serialise them. The array keeps
 * the last call's contents; nothing in it needs to start at zero.
 * Errors: KIFMM_EINVAL if the plan's workspace exceeds 64 MiB (see
 * kifmm_plan_info's n, n_leaf, n_box: about 190 bytes per point at p = 6 and
 * max_nrhs = 1) or the plan uses stage 2 (c2 > 0); KIFMM_ESTATE if profiling
 * is on; as kifmm_apply otherwise. */
int kifmm_apply_noalloc(kifmm_plan_t plan, const void* sigma, void* phi, void* stream);

/* out = F^T g by the transposed passes (L2T^T, L2L^T up the tree, M2L with
 * the transposed class matrices, M2M^T down the tree, S2M^T, S2T^T).
 *   g, out: device, n elements each, caller order; must not alias. */
int kifmm_apply_adjoint(kifmm_plan_t plan, const void* g, void* out, void* stream);

/* nrhs right-hand sides at once (1 <= nrhs <= opts.max_nrhs of the plan).
 *   sigma, phi: device, column-major n x nrhs with leading dimension ld >= n. */
int kifmm_apply_batched(kifmm_plan_t plan, const void* sigma, void* phi, int nrhs, int64_t ld,
                        void* stream);

/* Group several plans (for instance independent point sets) so that one call
 * runs all their applies from one captured HIP graph. The plans must outlive
 * the group and must use one device and one precision.
 * When 2 to 64 plans also share the operators (p, eps, leaf_size, opts.cd,
 * opts.pinv_rcond, opts.dense_m2l), the right-hand-side width (max_nrhs
 * rounded up to a power of two) and none uses stage 2 (opts.c2 = 0), the
 * group is merged: one synthetic plan holds the cubes, leaves and points of
 * all of them one after the other (device copies of their lists and
 * schedules, a workspace of the summed size), and every stage of an apply is
 * one launch over all the plans (M2M and L2L one per level); the inputs are
 * joined and the outputs split back by two small kernels. The results equal
 * the plans' own applies up to the summation order of the M2L products (its
 * work tiles differ). Otherwise each plan's apply is captured on a stream of
 * its own. */
int kifmm_group_create(const kifmm_plan_t* plans, int nplans, kifmm_group_t* out);
/* sigma[i], phi[i]: device vectors of plan i (as in kifmm_apply). The first call
 * with a given set of pointers captures the graph; later calls with the same
 * pointers replay it, other pointers re-capture it. */
int kifmm_group_apply(kifmm_group_t group, const void* const* sigma, void* const* phi,
                      void* stream);
void kifmm_group_destroy(kifmm_group_t group); /* NULL-safe */

/* Solve A x = b for the plan's operator A (the BEM systems of Sec. 4 are
 * solved by GMRES, Sec. 5) with restarted GMRES(restart): classical
 * Gram-Schmidt applied twice, the Krylov basis in device memory in the plan's
 * precision (restart + 1 vectors of n elements, allocated by this call and
 * freed before it returns), the small Hessenberg problem on the host in FP64.
 *   b:  device, n elements, caller order (not modified).
 *   x:  device, n elements: the initial guess on entry, the solution on return.
 *   Stops when the relative residual |b - A x| / |b| (recomputed explicitly at
 *   every restart and at the end) is <= tol, or after max_iter applies.
 *   iterations (may be NULL): applies used; residual (may be NULL): the final
 *   relative residual. The call synchronizes `stream` (it reads the inner
 *   products on the host every iteration) and cannot be captured in a graph.
 * Errors: KIFMM_EINVAL (tol <= 0, restart outside [1, 200], max_iter < 1,
 * NULL or equal pointers), KIFMM_ESTATE (host-only plan), KIFMM_EHIP. Not
 * reaching tol is not an error: check *residual. */
int kifmm_solve_gmres(kifmm_plan_t plan, const void* b, void* x, double tol, int restart, int max_iter,
                      void* stream, int* iterations, double* residual);

/* Sizes, counts and per-stage algorithmic flops/bytes of a plan. */
int kifmm_plan_info(kifmm_plan_t plan, kifmm_info_t* info);

/* Leaf cube of every point (caller order) as integer coordinates at level
 * info.depth: leaf_coords is a host array of n x 3 int32. (In an adaptive
 * plan: the level-depth cube holding the point, not its leaf.) */
int kifmm_plan_export_tree(kifmm_plan_t plan, int32_t* leaf_coords);

/* Leaf of every point (caller order) as (level, i, j, k), the cube's integer
 * coordinates at its own level: out is a host array of n x 4 int32. */
int kifmm_plan_export_point_leaves(kifmm_plan_t plan, int32_t* out);

/* The cubes of the tree (Sec. 2.1) in the plan's global order, 5 int32 per
 * cube: level, i, j, k (integer coordinates at that level) and the leaf index
 * (-1 for a split cube). With out == NULL only *count (cubes) is set; else
 * out must hold 5 * count values. count must not be NULL. */
int kifmm_plan_export_boxes(kifmm_plan_t plan, int32_t* out, int64_t* count);

/* The interaction lists as (target, source) pairs of global cube indices (the
 * order of kifmm_plan_export_boxes), 2 int32 per pair. which:
 *   0 U: near field (Sec. 2.1), target leaf and source leaf
 *   1 V: interaction field (Sec. 2.1), target and source cube, levels >= 2
 *   2 W (adaptive plans; empty otherwise): target leaf, source cube
 *   3 X (adaptive plans; empty otherwise): target cube, source leaf
 * With out == NULL only *count (pairs) is set; else out must hold 2 * count
 * values. KIFMM_EINVAL for another `which` or count == NULL. */
int kifmm_plan_export_list(kifmm_plan_t plan, int which, int32_t* out, int64_t* count);

/* Host FP64 copies of the plan's operators (for checks). `which`:
 *   0 singular values of K_fat (n_eq values; dense plans: zeros)
 *   1 U~ (n_eq x k, row-major; dense: identity)
 *   2 S~  (k x n_eq)      3 T~ (n_eq x k)
 *   4 M~^o (8 x k x k; o = 4*ox + 2*oy + oz, child position bits)
 *   5 L~^o (8 x k x k)    6 K~^(t) (316 x k x k; t in lexicographic order over
 *                            [-3,3]^3 with max|t_a| >= 2)
 *   stage-2 plans only (opts.c2 > 0; KIFMM_EINVAL otherwise), r = info.m2l_rank_max:
 *   7 ranks of the 316 classes (as doubles)
 *   8 U^ (316 x k x r, zero past each class's rank)
 *   9 V^ = S^ Q^^T (316 x r x k, zero past each class's rank)
 * `out` must hold the number of doubles stated; `count` (may be NULL) receives it. */
int kifmm_plan_export_operator(kifmm_plan_t plan, int which, double* out, int64_t* count);

/* Stage timing with HIP events (the tracing facility). While enabled, every
 * apply of the plan records an event before and after each stage
 * (KIFMM_STAGE_* order: P2M = surface evaluation + S~ GEMM, M2M, M2L, L2L,
 * L2P = T~ GEMM + far-field evaluation at the points, P2P = near field,
 * PERM = permute-in). The near field runs on a stream of the plan, forked from
 * the caller's stream after the permute and joined back before the far-field
 * evaluation, so its time overlaps the other stages'.
 * Enabled applies cannot be captured in a HIP graph: an apply of such a plan
 * on a capturing stream, and kifmm_group_apply on a group holding one, return
 * KIFMM_ESTATE without recording anything. kifmm_profile(plan, 0/1) switches
 * it and clears the totals. */
int kifmm_profile(kifmm_plan_t plan, int enable);
/* Waits for the recorded events and returns the summed milliseconds per stage
 * since profiling was enabled (ms[KIFMM_STAGE_COUNT]) and the number of
 * profiled applies (*calls, may be NULL). */
int kifmm_profile_read(kifmm_plan_t plan, double* ms, int64_t* calls);

/* Release a plan and its device memory. NULL-safe; the plan must not be in use. */
void kifmm_destroy(kifmm_plan_t plan);

/* Message of the last failing call on this thread ("" if none). */
const char* kifmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KIFMM_H */
