// Host-side plan: octree, near/interaction fields, FP64 operators and the
// work schedules of the grouped GEMM kernel. Nothing here touches the GPU.
#pragma once
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

namespace kifmm {

constexpr int QBITS = 21;     // integer coordinate bits per axis
constexpr int NCLASS = 316;   // M2L offset classes (Sec. 3.1)
constexpr int MAX_LEVEL = 20;

struct PlanError {
    int code;
    std::string msg;
};

// Class id of an M2L offset t in [-3,3]^3 with max|t_a| >= 2 (lexicographic), else -1.
int class_of_offset(int tx, int ty, int tz);
// Inverse of class_of_offset.
void offset_of_class(int c, int* t);

struct HostTree {
    int depth = 0;
    int64_t n = 0;
    double centre[3] = {0, 0, 0};
    double r0 = 1.0;
    std::vector<int32_t> perm;          // sorted position -> caller index
    std::vector<int64_t> level_begin;   // depth+2 entries: global box index range of each level
    std::vector<uint64_t> box_key;      // Morton key of each box at its own level
    std::vector<int32_t> box_parent;    // global index of the parent, -1 for the root
    std::vector<int32_t> box_child;     // 8 per box (octant 4*ox+2*oy+oz), -1 if empty
    std::vector<int32_t> leaf_ptr;      // n_leaf+1 offsets into the sorted points
    std::vector<double> u;              // sorted points in leaf units: (x - c_leaf)/r_L, 3 per point
    std::vector<int32_t> near_ptr;      // CSR over leaves
    std::vector<int32_t> near_leaf;     // source leaf (leaf index)
    std::vector<int32_t> near_code;     // (dx+1)*9+(dy+1)*3+(dz+1), d = target - source cube
    std::vector<int32_t> v_ptr;         // CSR over global boxes (levels 2..depth)
    std::vector<int32_t> v_src;         // source box (global index)
    std::vector<int32_t> v_cls;         // offset class of (target - source)
    std::vector<int32_t> leaf_coords;   // per caller point: level-depth cube (3 ints)
    // Adaptive trees (build_adaptive_host_tree): leaves at several levels. The
    // boxes of a level are its leaves, then its split cubes, each in Morton
    // order; leaf indices follow the sorted points. Points are in the units of
    // their own leaf. Near-field codes there are m * 729 + (ox+4) * 81 +
    // (oy+4) * 9 + (oz+4): m = 0 source at the target's level, 1 one level
    // finer, 2 one level coarser; o = (source centre - target centre) in
    // half-widths of the finer of the two leaves.
    bool adaptive = false;
    std::vector<int64_t> level_leaves;  // leaves of each level
    std::vector<int32_t> box_leaf;      // leaf index of a box, -1 for a split cube
    std::vector<int32_t> leaf_box;      // global box index of a leaf
    std::vector<int32_t> leaf_level;    // level of a leaf
    std::vector<int32_t> w_ptr, w_src;  // W lists: CSR over leaves, source cube (global index)
    std::vector<int32_t> x_ptr, x_src;  // X lists: CSR over boxes, source leaf (leaf index)

    int64_t n_box() const { return level_begin.back(); }
    int64_t n_leaf() const { return (int64_t)leaf_ptr.size() - 1; }
    int64_t level_count(int l) const { return level_begin[l + 1] - level_begin[l]; }
    double half_width(int l) const { return r0 / double(int64_t(1) << l); }
};

// Level of global box g and its integer coordinates at that level.
int box_cube(const HostTree& t, int64_t g, int64_t c[3]);
// Leaf index of global box g (-1 for a split cube) and global box of leaf e,
// for both kinds of tree.
int64_t leaf_of_box(const HostTree& t, int64_t g);
int64_t box_of_leaf(const HostTree& t, int64_t e);

// Builds the tree; throws PlanError on invalid input.
HostTree build_host_tree(const double* pts, int64_t n, int leaf_size, int depth_override,
                         int max_depth);

// Adaptive octree (Sec. 2.1 read cube by cube): a cube holding more than
// leaf_size points is split into its nonempty children, down to max_depth;
// then 2:1 balance in rounds, every leaf sharing a vertex with a leaf two or
// more levels finer being split, all at once, until none is left. Lists of
// the kernel-independent FMM between leaves of different levels: U (near
// field: leaves of any level sharing a vertex), V (as the uniform tree, at
// every level >= 2), W (cubes below a same-level neighbour of a leaf whose
// parent shares a vertex with the leaf but which do not) and X (the dual of
// W). Throws PlanError on invalid input.
HostTree build_adaptive_host_tree(const double* pts, int64_t n, int leaf_size, int max_depth);

struct HostOps {
    int p = 0, n_eq = 0, k = 0;
    bool dense = false;
    double d = 0, rcond = 0, eps = 0, sigma0 = 0;
    std::vector<double> E;      // unit surface template (n_eq x 3)
    std::vector<double> outer;  // (3-2d) E: upward check = downward equivalent surface
    std::vector<double> sing;   // singular values of K_fat (n_eq; zeros in dense mode)
    std::vector<double> U;      // n_eq x k
    std::vector<double> S;      // k x n_eq
    std::vector<double> T;      // n_eq x k
    std::vector<double> M, L;   // 8 x k x k (octant 4*ox+2*oy+oz)
    std::vector<double> K;      // 316 x k x k
    // stage-2 factors (Sec. 3.2), empty unless build_stage2 ran
    double c2 = 0, eps2 = 0;    // constant C2 and the absolute cutoff C2 eps / k * sigma0
    int r2max = 0;              // largest rank
    std::vector<int32_t> rank2; // 316 ranks
    std::vector<double> U2;     // 316 x k x r2max: U^ (zero past the rank)
    std::vector<double> V2;     // 316 x r2max x k: V^ = S^ Q^^T (zero past the rank)
};

HostOps build_host_ops(int p, double eps, int leaf_size, double cd, double rcond, bool dense);

// The operators of (p, eps, leaf_size, cd, rcond, dense, c2) from a
// process-wide cache: they are fixed by the equivalent and check surfaces
// alone, not by the points or the boundary (the remark on the translating
// matrices in Sec. 5.1), so plans with equal parameters
// share one FP64 copy instead of repeating the SVD of K_fat. The most recently
// used parameter sets stay cached; c2 > 0 adds the stage-2 factors. Safe to
// call from several threads. Throws PlanError as build_host_ops.
std::shared_ptr<const HostOps> host_ops_shared(int p, double eps, int leaf_size, double cd, double rcond,
                                               bool dense, double c2);

// Stage-2 low rank of the compressed M2L matrices (Sec. 3.2): per class the SVD
// K~ = U S Q^T, keeping the singular values not below C2 eps / k * sigma0.
// Requires compressed operators (not dense); c2 > 0.
void build_stage2(HostOps& o, double c2);

// Work schedule of the grouped gather GEMM Y[t] (+)= scale * sum A[cls] X[src].
// `cp` pairs of one class form a chunk; `rhs` right-hand-side columns per pair.
// Targets are split into tiles of consecutive rows; inside a tile the
// (target, source, class) pairs are sorted by (scale group, class) and cut
// into chunks of at most `cp` pairs that share one class and one scale.
struct GGSched {
    int cp = 32;
    int rhs = 1;
    int max_tile = 0;
    int variant = 0;                   // grouped-GEMM kernel shape
    std::vector<int32_t> tile_tgt0;    // first target row of the tile
    std::vector<int32_t> tile_ntgt;    // targets in the tile
    std::vector<int32_t> tile_chunk0;  // n_tiles + 1
    std::vector<int32_t> chunk_cls;
    std::vector<int32_t> chunk_next;   // class of the next chunk of the tile whose class differs, -1 if none
    std::vector<int32_t> chunk_nblk;   // 16-column blocks holding data (ceil(pairs * R / 16))
    std::vector<double> chunk_scale;
    std::vector<int32_t> chunk_src;    // n_chunks * cp (-1 = empty slot)
    std::vector<int32_t> chunk_col;    // n_chunks * cp (target column in the tile, -1 = empty)
    int64_t pairs = 0;
    int n_tiles() const { return (int)tile_tgt0.size(); }
    int n_chunks() const { return (int)chunk_cls.size(); }
};

// Append the targets [0, n_tgt) (rows tgt_row0 + i of Y), whose pairs are
// given in CSR form (ptr over targets, absolute indices into src/cls), cut
// into tiles at `cuts` (strictly increasing, 0 ... n_tgt). Target i uses the
// scale group_scale[group ? group[i] : 0].
void gg_build(GGSched& s, int64_t tgt_row0, int64_t n_tgt, const int32_t* ptr, const int32_t* src,
              const int32_t* cls, const int32_t* group, const std::vector<double>& group_scale,
              const std::vector<int64_t>& cuts);

// Tiles of `tile` consecutive targets.
std::vector<int64_t> uniform_cuts(int64_t n_tgt, int tile);
// About `n_tiles` tiles of equal cost (pairs + `per_target` per target), none
// larger than `max_tile` targets.
std::vector<int64_t> balanced_cuts(int64_t n_tgt, const int32_t* ptr, int n_tiles, int max_tile,
                                   double per_target);

// Estimated kernel cost of a tile: per chunk, per 16-column block and per
// target (accumulator set-up and store).
struct TileCost {
    double per_chunk = 1.0;
    double per_block = 0.0;
    double per_target = 0.0;
};
// About `n_tiles` tiles of equal estimated cost, none larger than `max_tile`
// targets; chunks and blocks are counted as gg_build forms them (`cp` pairs
// per chunk, `rhs` columns per pair; classes are read as in gg_build).
std::vector<int64_t> chunk_cuts(int64_t n_tgt, const int32_t* ptr, const int32_t* cls, const int32_t* group,
                                int cp, int rhs, int n_tiles, int max_tile, const TileCost& w);

// Consecutive tile ranges of a schedule whose chunk slots (cp per chunk,
// slot_bytes each) span less than max_bytes and fewer than max_slots per
// range: the first tile of every range, then the tile count. Each range is
// the longest that fits, in order. Empty if one tile alone does not fit.
std::vector<int> split_tile_ranges(const std::vector<int32_t>& tile_chunk0, int cp, int64_t slot_bytes,
                                   int64_t max_bytes, int64_t max_slots);

}  // namespace kifmm
