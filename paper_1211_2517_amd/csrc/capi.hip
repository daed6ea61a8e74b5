// C ABI of the MI355X KIFMM library: plan construction, device upload and the
// evaluation passes (complete algorithm of Sec. 4.3) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/kifmm.h"
#include "kernels.h"
#include "plan.h"

using namespace kifmm;

namespace {

thread_local std::string g_last_error;

// Workspace of kifmm_apply_noalloc: a device array of the library, one copy on
// every GPU the library runs on, held until the process ends. In host code
// `scratch` names a host-side stand-in, never the device memory: its device
// address is looked up once per device (scratch_address) and only that
// address is used.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex& scratch_mutex() {
    static std::mutex m;
    return m;
}
std::map<int, void*>& scratch_ptrs() {
    static std::map<int, void*> m;   // device ordinal -> device address of `scratch`
    return m;
}

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

constexpr double kFourPi = 12.566370614359172953850573533118;

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace

// Device copies of a plan's operator tables. Plans whose operators, element
// type, split-BF16 choice and device agree share one copy (see
// shared_tables); the memory is freed with the last plan that uses it.
struct DevTables {
    int device = 0;
    size_t bytes = 0;
    std::shared_ptr<const HostOps> ops;   // keeps the cache key's operators alive
    std::vector<void*> allocs;
    void *Kt = nullptr, *KtT = nullptr, *Mt = nullptr, *MtT = nullptr, *Lt = nullptr, *LtT = nullptr;
    void *Sop = nullptr, *SopT = nullptr, *Top = nullptr, *TopT = nullptr;
    void *V2t = nullptr, *U2t = nullptr, *U2tT = nullptr, *V2tT = nullptr, *surf = nullptr;
    void *Ut = nullptr, *UtT = nullptr, *surf_in = nullptr;   // U~, U~^T and the (1+d) surface (M2T, S2L)
    ~DevTables() {
        if (allocs.empty()) return;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        for (void* p : allocs) (void)hipFree(p);
        (void)hipSetDevice(cur);
    }
};

struct kifmm_plan_s {
    kifmm_opts_t opts{};
    int p = 0;
    double eps = 0;
    int leaf_size = 0;
    HostTree tree;
    std::shared_ptr<const HostOps> ops_sp;   // cached FP64 operators (shared by plans with equal parameters)
    const HostOps& ops() const { return *ops_sp; }
    int k = 0, kp = 0, nep = 0, R = 1, elt = 4;
    bool b3 = false;    // M2L in split BF16 (KIFMM_BF16X3); all other stages FP32
    bool st2 = false;   // stage-2 low-rank M2L (opts.c2 > 0)
    int rp = 0;         // stage-2 rank padded to 16
    bool on_device = false;
    int device = 0;
    int num_cu = 256;   // compute units of the device (MI355X: 256)
    float tuned_ms = 0;  // M2L launch time of the autotuned shape (0 = not tuned)
    // host schedules
    GGSched h_leafup, h_leafdown, h_m2l;
    std::vector<GGSched> h_up, h_down;   // indexed by target level
    // device schedules
    DevSched d_leafup, d_leafdown, d_m2l;
    // stage-2 M2L: w = V^ q per chunk slot (d_s2a), then p += scale U^ w, as
    // launches over tile ranges (d_s2b), each reading the W rows of its own
    // slots from byte offset s2b_xoff[r] of W
    DevSched d_s2a;
    std::vector<DevSched> d_s2b;
    std::vector<size_t> s2b_xoff;
    std::vector<DevSched> d_up, d_down;
    // device data
    void* pts = nullptr;
    void* qpts = nullptr;   // FP32 plans: fixed-point leaf-unit coordinates (near field)
    void* surf = nullptr;
    int32_t* perm = nullptr;
    int32_t* leaf_ptr = nullptr;
    int32_t* near_ptr = nullptr;
    int32_t* near_leaf = nullptr;
    int32_t* near_code = nullptr;
    void *Kt = nullptr, *KtT = nullptr, *Mt = nullptr, *MtT = nullptr, *Lt = nullptr, *LtT = nullptr;
    void *Sop = nullptr, *SopT = nullptr, *Top = nullptr, *TopT = nullptr;
    void *V2t = nullptr, *U2t = nullptr, *U2tT = nullptr, *V2tT = nullptr;   // stage-2 factors
    void* W = nullptr;   // stage-2 per-slot products w = V^ q (n_chunks x 32 rows of rp)
    // Adaptive trees. The cubes that appear in some W list are exactly those
    // with a nonempty X list; they are numbered as "W cubes" in box order.
    // M2T: Psi[w] = U~ q~ of W cube w (h_m2t), evaluated at the points of the
    // leaves that list it (m2t_*); S2L: CX[w] = check potential of W cube w
    // from the points of its X leaves (s2l_*), then P += U~^T CX / (4 pi r)
    // (h_s2l). The adjoint runs the same steps with the roles of Q and P swapped.
    std::vector<int32_t> w_cube_box;     // W cube -> global box
    GGSched h_m2t, h_s2l;
    DevSched d_m2t, d_s2l;
    int64_t n_m2t_leaf = 0;              // leaves with a nonempty W list
    int32_t* leaf_level = nullptr;
    void* leaf_scale = nullptr;          // per leaf 1/(4 pi r_leaf), element type
    int32_t *m2t_leaf = nullptr, *m2t_ptr = nullptr, *m2t_cube = nullptr;
    int32_t *s2l_ptr = nullptr, *s2l_leaf = nullptr;
    void *m2t_geo = nullptr, *s2l_geo = nullptr;   // per entry (rho, ox, oy, oz) in the element type
    void *Ut = nullptr, *UtT = nullptr, *surf_in = nullptr;
    // BEM plans (Sec. 4): the points are the triangles' centroids; per
    // triangle (sorted order, leaf units) its 7-point rule (x, y, z, W), its
    // unit normal, and its vertices and normal for the near-field integrals
    int layer = -1;                      // -1 point sources, 0 single layer, 1 double layer
    // leaf stages fused with their products (FP32, one right-hand side): the
    // check potentials with S~ (S2M), T~ with the far field (L2P); leaf_row is
    // the Q/P row of every leaf (-1: no local expansion)
    bool fuse_s2m = false, fuse_l2p = false;
    int32_t* leaf_row = nullptr;
    // M2M by one product per parent (FP32, one right-hand side) on the levels
    // of at most kM2MDirectMax parents: per level, m2m_n parents (0: the
    // grouped GEMM of d_up), and at d_m2m their Q rows followed by 8 child
    // rows each
    bool m2m_direct = false;
    std::vector<int32_t> m2m_n;
    std::vector<int32_t*> d_m2m;
    // L2L in the direct form (FP32, one right-hand side): per level, dd_nseg
    // segments of one octant of up to 16 * dd_ncb children; d_dd holds the
    // segments (class, first item, items), the items' child rows, then their
    // parent rows (dd_nitem items)
    bool down_direct = false;
    std::vector<int32_t> dd_nseg, dd_ncb, dd_nitem;
    std::vector<int32_t*> d_dd;
    // near field with register-staged sources, forked just before M2L so that
    // it runs on the CUs the M2L launch holds (opts.near_overlap)
    bool near_late = false;
    void *bem_qp = nullptr, *bem_tn = nullptr, *bem_tri = nullptr;
    void *sig_s = nullptr, *C = nullptr, *Q = nullptr, *P = nullptr, *E = nullptr;
    void *CX = nullptr, *Psi = nullptr;   // adaptive: per W cube, S2L check potentials and U~ q~
    std::vector<void*> allocs;
    std::shared_ptr<DevTables> tables;   // operator tables (possibly shared with other plans)
    size_t device_bytes = 0;
    // the near field runs on a stream of its own, forked from and joined back
    // into the caller's stream, so that it overlaps the far-field passes
    hipStream_t near_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    kifmm_info_t info{};
    // stage profiling
    bool profiling = false;
    std::vector<std::array<hipEvent_t, 2 * KIFMM_STAGE_COUNT>> prof_events;  // per pending apply
    std::vector<std::array<hipEvent_t, 2 * KIFMM_STAGE_COUNT>> prof_free;
    double prof_ms[KIFMM_STAGE_COUNT] = {0};
    int64_t prof_calls = 0;
};

struct kifmm_group_s {
    std::vector<kifmm_plan_t> plans;
    // merged form (see build_fused): one synthetic plan over the cubes,
    // leaves and points of all the plans, with joined input and output vectors
    kifmm_plan_s* fused = nullptr;
    void *sig_u = nullptr, *out_u = nullptr;
    std::vector<int64_t> pt_off;
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<const void*> key_sigma;
    std::vector<void*> key_phi;
    hipStream_t key_stream = nullptr;
};

namespace {

void release_streams(kifmm_plan_s* pl) {
    if (pl->near_stream) (void)hipStreamDestroy(pl->near_stream);
    if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
    if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
    pl->near_stream = nullptr;
    pl->ev_fork = pl->ev_join = nullptr;
}

void release_device(kifmm_plan_s* pl) {
    if (!pl->allocs.empty()) {
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(pl->device);
        for (void* p : pl->allocs) hipFree(p);
        hipSetDevice(cur);
    }
    pl->allocs.clear();
}

struct Uploader {
    kifmm_plan_s* pl;
    size_t limit;
    int err = KIFMM_OK;
    std::string msg;
    std::vector<void*>* scratch = nullptr;   // when set, allocations go here instead of the plan
    size_t scratch_bytes = 0;                // bytes allocated into `scratch`
    void* alloc(size_t bytes) {
        if (err != KIFMM_OK) return nullptr;
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~size_t(255);
        if (limit && pl->device_bytes + bytes > limit) {
            err = KIFMM_ENOMEM;
            msg = "opts.mem_limit exceeded (" + std::to_string(pl->device_bytes + bytes) + " bytes needed)";
            return nullptr;
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            err = KIFMM_ENOMEM;
            msg = std::string("hipMalloc failed: ") + hipGetErrorString(e);
            return nullptr;
        }
        if (scratch) {
            scratch->push_back(p);
            scratch_bytes += bytes;
        } else {
            pl->allocs.push_back(p);
            pl->device_bytes += bytes;
        }
        return p;
    }
    template <class V>
    void* put(const V& v) {
        size_t bytes = v.size() * sizeof(typename V::value_type);
        void* p = alloc(bytes);
        if (p && bytes) {
            hipError_t e = hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                err = KIFMM_EHIP;
                msg = std::string("hipMemcpy failed: ") + hipGetErrorString(e);
            }
        }
        return p;
    }
    void* zeros(size_t bytes) {
        void* p = alloc(bytes);
        if (p) {
            hipError_t e = hipMemset(p, 0, (bytes + 255) & ~size_t(255));
            if (e != hipSuccess) {
                err = KIFMM_EHIP;
                msg = std::string("hipMemset failed: ") + hipGetErrorString(e);
            }
        }
        return p;
    }
};

// padded table of `nblk` blocks rows x cols (row-major) from FP64 values
template <typename T>
std::vector<T> pad_blocks(int nblk, int rows, int cols, int rows_pad, int cols_pad,
                          const std::function<double(int, int, int)>& f) {
    std::vector<T> out((size_t)nblk * rows_pad * cols_pad, T(0));
    for (int b = 0; b < nblk; ++b)
        for (int i = 0; i < rows; ++i)
            for (int j = 0; j < cols; ++j) out[((size_t)b * rows_pad + i) * cols_pad + j] = (T)f(b, i, j);
    return out;
}

// With row_map, the schedule's target rows are indices into row_map, which
// gives the rows the kernel writes; the schedule must then have one pair per
// target (the direct form), or the upload fails.
DevSched upload_sched(Uploader& up, const GGSched& s, int elt, const std::vector<int32_t>* row_map = nullptr) {
    DevSched d;
    d.n_tiles = s.n_tiles();
    d.n_chunks = s.n_chunks();
    d.cp = s.cp;
    d.max_tile = s.max_tile;
    d.variant = s.variant;
    if (d.n_tiles == 0) return d;
    d.tile_tgt0 = (const int32_t*)up.put(s.tile_tgt0);
    d.tile_ntgt = (const int32_t*)up.put(s.tile_ntgt);
    d.tile_chunk0 = (const int32_t*)up.put(s.tile_chunk0);
    for (int32_t v : s.chunk_src) d.max_src = std::max(d.max_src, v);
    for (int32_t v : s.chunk_cls) d.max_cls = std::max(d.max_cls, v);
    std::vector<int32_t> meta((size_t)4 * d.n_chunks, 0);
    for (int c = 0; c < d.n_chunks; ++c) {
        meta[4 * c] = s.chunk_cls[c];
        meta[4 * c + 1] = s.chunk_nblk[c];
        if (elt == 4) {
            const float f = (float)s.chunk_scale[c];
            std::memcpy(&meta[4 * c + 2], &f, sizeof f);
        } else {
            std::memcpy(&meta[4 * c + 2], &s.chunk_scale[c], sizeof(double));
        }
    }
    d.chunk_meta = (const int32_t*)up.put(meta);
    d.chunk_src = (const int32_t*)up.put(s.chunk_src);
    d.chunk_col = (const int32_t*)up.put(s.chunk_col);
    // one pair for every target of every tile: the direct form of the kernel
    int64_t lo = INT64_MAX, hi = 0;
    for (int t = 0; t < d.n_tiles; ++t) {
        lo = std::min<int64_t>(lo, s.tile_tgt0[t]);
        hi = std::max<int64_t>(hi, (int64_t)s.tile_tgt0[t] + s.tile_ntgt[t]);
    }
    std::vector<int32_t> seen((size_t)(hi - lo), 0), tgt(s.chunk_col.size(), -1);
    int64_t need = 0;
    for (int t = 0; t < d.n_tiles; ++t) need += s.tile_ntgt[t];
    int64_t got = 0;
    bool direct = true;
    for (int t = 0; t < d.n_tiles && direct; ++t) {
        for (int c = s.tile_chunk0[t]; c < s.tile_chunk0[t + 1] && direct; ++c) {
            for (int i = 0; i < s.cp; ++i) {
                const int32_t col = s.chunk_col[(size_t)c * s.cp + i];
                if (col < 0) continue;
                const int64_t g = (int64_t)s.tile_tgt0[t] + col;
                if (++seen[(size_t)(g - lo)] > 1) {
                    direct = false;
                    break;
                }
                tgt[(size_t)c * s.cp + i] = row_map ? (*row_map)[(size_t)g] : (int32_t)g;
                ++got;
            }
        }
    }
    if (direct && got == need) {
        d.direct = true;
        d.chunk_tgt = (const int32_t*)up.put(tgt);
    } else if (row_map && up.err == KIFMM_OK) {
        up.err = KIFMM_EINVAL;
        up.msg = "internal: a row-mapped schedule must have one pair per target";
    }
    return d;
}

int neg_class(int c) {
    int t[3];
    offset_of_class(c, t);
    return class_of_offset(-t[0], -t[1], -t[2]);
}

// BF16 bits of a float, rounded to nearest even (finite inputs).
uint16_t bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Split-BF16 table of `nblk` zero-padded rows_pad x cols_pad blocks (cols_pad a
// multiple of 32): per row and 32-wide column chunk, the 32 high parts
// hi = bf16(x), then the 32 low parts lo = bf16(x - hi), so a row takes the
// bytes of cols_pad floats.
std::vector<uint16_t> split_blocks(int nblk, int rows, int cols, int rows_pad, int cols_pad,
                                   const std::function<double(int, int, int)>& f) {
    std::vector<uint16_t> out((size_t)nblk * rows_pad * cols_pad * 2, 0);
    for (int b = 0; b < nblk; ++b)
        for (int i = 0; i < rows; ++i)
            for (int j = 0; j < cols; ++j) {
                const double x = f(b, i, j);
                const uint16_t hi = bf16_bits((float)x);
                const uint16_t lo = bf16_bits((float)(x - bf16_value(hi)));
                const size_t row = ((size_t)b * rows_pad + i) * cols_pad * 2;
                const size_t at = row + (size_t)(j / 32) * 64 + (j % 32);
                out[at] = hi;
                out[at + 32] = lo;
            }
    return out;
}

template <typename T>
void upload_op_tables(const kifmm_plan_s* pl, Uploader& up, DevTables& d) {
    const HostOps& o = pl->ops();
    const int k = o.k, ne = o.n_eq, kp = pl->kp, nep = pl->nep;
    auto K = [&](int c, int i, int j) { return o.K[((size_t)c * k + i) * k + j]; };
    if (pl->b3) {
        d.Kt = up.put(split_blocks(NCLASS, k, k, kp, kp, [&](int c, int i, int j) { return K(c, i, j); }));
        d.KtT = up.put(split_blocks(NCLASS, k, k, kp, kp, [&](int c, int i, int j) { return K(neg_class(c), j, i); }));
    } else {
        d.Kt = up.put(pad_blocks<T>(NCLASS, k, k, kp, kp, [&](int c, int i, int j) { return K(c, i, j); }));
        d.KtT = up.put(pad_blocks<T>(NCLASS, k, k, kp, kp, [&](int c, int i, int j) { return K(neg_class(c), j, i); }));
    }
    auto Mf = [&](int b, int i, int j) { return o.M[((size_t)b * k + i) * k + j]; };
    auto Lf = [&](int b, int i, int j) { return o.L[((size_t)b * k + i) * k + j]; };
    d.Mt = up.put(pad_blocks<T>(8, k, k, kp, kp, Mf));
    d.MtT = up.put(pad_blocks<T>(8, k, k, kp, kp, [&](int b, int i, int j) { return Mf(b, j, i); }));
    d.Lt = up.put(pad_blocks<T>(8, k, k, kp, kp, Lf));
    d.LtT = up.put(pad_blocks<T>(8, k, k, kp, kp, [&](int b, int i, int j) { return Lf(b, j, i); }));
    d.Sop = up.put(pad_blocks<T>(1, k, ne, kp, nep, [&](int, int i, int a) { return o.S[(size_t)i * ne + a]; }));
    d.SopT = up.put(pad_blocks<T>(1, ne, k, nep, kp, [&](int, int a, int i) { return o.S[(size_t)i * ne + a]; }));
    d.Top = up.put(pad_blocks<T>(1, ne, k, nep, kp, [&](int, int a, int i) { return o.T[(size_t)a * k + i]; }));
    d.TopT = up.put(pad_blocks<T>(1, k, ne, kp, nep, [&](int, int i, int a) { return o.T[(size_t)a * k + i]; }));
    if (pl->st2) {
        // stage-2 factors (Sec. 3.2), zero-padded to rp: phase A multiplies by V^
        // (rp x kp per class), phase B by U^ (kp x rp); the adjoint applies the
        // class -t transposed: U^(-t)^T in phase A and V^(-t)^T in phase B
        const int rm = o.r2max, rp = pl->rp;
        auto U2 = [&](int c, int i, int j) { return j < rm ? o.U2[((size_t)c * k + i) * rm + j] : 0.0; };
        auto V2 = [&](int c, int j, int i) { return j < rm ? o.V2[((size_t)c * rm + j) * k + i] : 0.0; };
        d.V2t = up.put(pad_blocks<T>(NCLASS, rm, k, rp, kp, V2));
        d.U2t = up.put(pad_blocks<T>(NCLASS, k, rm, kp, rp, U2));
        d.U2tT = up.put(pad_blocks<T>(NCLASS, rm, k, rp, kp, [&](int c, int j, int i) { return U2(neg_class(c), i, j); }));
        d.V2tT = up.put(pad_blocks<T>(NCLASS, k, rm, kp, rp, [&](int c, int i, int j) { return V2(neg_class(c), j, i); }));
    }
    std::vector<T> surf(3 * ne);
    for (int i = 0; i < 3 * ne; ++i) surf[i] = (T)o.outer[i];
    d.surf = up.put(surf);
    // M2T and S2L (adaptive trees): U~, U~^T and the upward-equivalent /
    // downward-check surface (1 + d) E
    auto Uf = [&](int, int a, int i) { return o.U[(size_t)a * k + i]; };
    d.Ut = up.put(pad_blocks<T>(1, ne, k, nep, kp, Uf));
    d.UtT = up.put(pad_blocks<T>(1, k, ne, kp, nep, [&](int, int i, int a) { return o.U[(size_t)a * k + i]; }));
    std::vector<T> sin(3 * ne);
    for (int i = 0; i < 3 * ne; ++i) sin[i] = (T)((1.0 + o.d) * o.E[i]);
    d.surf_in = up.put(sin);
}

// The operator tables of the plan from the process-wide cache of device
// tables, uploading them when no live plan on this device has them.
template <typename T>
std::shared_ptr<DevTables> shared_tables(const kifmm_plan_s* pl, Uploader& up) {
    using Key = std::tuple<const HostOps*, int, bool, int, int, int, int>;
    static std::mutex mu;
    static std::map<Key, std::weak_ptr<DevTables>> cache;
    const Key key{pl->ops_sp.get(), pl->elt, pl->b3, pl->device, pl->kp, pl->nep, pl->rp};
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            if (auto d = it->second.lock()) return d;
            cache.erase(it);
        }
    }
    auto d = std::make_shared<DevTables>();
    d->device = pl->device;
    d->ops = pl->ops_sp;
    std::vector<void*>* saved = up.scratch;
    const size_t saved_bytes = up.scratch_bytes;
    up.scratch = &d->allocs;
    up.scratch_bytes = 0;
    upload_op_tables<T>(pl, up, *d);
    d->bytes = up.scratch_bytes;
    up.scratch = saved;
    up.scratch_bytes = saved_bytes;
    if (up.err != KIFMM_OK) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end())
        if (auto other = it->second.lock()) return other;   // another thread uploaded them meanwhile
    cache[key] = d;
    return d;
}

template <typename T>
int upload_tables(kifmm_plan_s* pl, Uploader& up) {
    pl->tables = shared_tables<T>(pl, up);
    if (!pl->tables) return up.err;
    const DevTables& d = *pl->tables;
    pl->device_bytes += d.bytes;
    if (up.limit && pl->device_bytes > up.limit) {
        up.err = KIFMM_ENOMEM;
        up.msg = "opts.mem_limit exceeded by the operator tables (" + std::to_string(pl->device_bytes) + " bytes)";
        return up.err;
    }
    pl->Kt = d.Kt;
    pl->KtT = d.KtT;
    pl->Mt = d.Mt;
    pl->MtT = d.MtT;
    pl->Lt = d.Lt;
    pl->LtT = d.LtT;
    pl->Sop = d.Sop;
    pl->SopT = d.SopT;
    pl->Top = d.Top;
    pl->TopT = d.TopT;
    pl->V2t = d.V2t;
    pl->U2t = d.U2t;
    pl->U2tT = d.U2tT;
    pl->V2tT = d.V2tT;
    pl->surf = d.surf;
    pl->Ut = d.Ut;
    pl->UtT = d.UtT;
    pl->surf_in = d.surf_in;
    std::vector<T> pts(4 * (size_t)pl->tree.n, T(0));
    for (int64_t i = 0; i < pl->tree.n; ++i)
        for (int a = 0; a < 3; ++a) pts[4 * i + a] = (T)pl->tree.u[3 * i + a];
    pl->pts = up.put(pts);
    if (sizeof(T) == 4) {
        // fixed point for the near field: q = round(u 2^28), |u| <= 1
        std::vector<int32_t> q(4 * (size_t)pl->tree.n, 0);
        for (int64_t i = 0; i < pl->tree.n; ++i)
            for (int a = 0; a < 3; ++a) {
                const double v = std::nearbyint(pl->tree.u[3 * i + a] * 268435456.0);
                q[4 * i + a] = (int32_t)std::min(268435456.0, std::max(-268435456.0, v));
            }
        pl->qpts = up.put(q);
    }
    return up.err;
}

// Host form of the per-leaf data of the adaptive evaluation kernels (level and
// near-field scale 1/(4 pi r_leaf)) and of the M2T and S2L entries; for a
// uniform tree every leaf is at the leaf level and there are no entries.
template <typename T>
struct AdaptiveLists {
    std::vector<int32_t> level;
    std::vector<T> scale;
    std::vector<int32_t> mleaf, mptr{0}, mcube, sptr{0}, sleaf;
    std::vector<T> mgeo, sgeo;
};

template <typename T>
AdaptiveLists<T> adaptive_lists(const kifmm_plan_s* pl) {
    const HostTree& t = pl->tree;
    AdaptiveLists<T> a;
    const int64_t nl = t.n_leaf();
    a.level.resize(nl);
    a.scale.resize(nl);
    for (int64_t e = 0; e < nl; ++e) {
        a.level[e] = t.adaptive ? t.leaf_level[e] : t.depth;
        a.scale[e] = (T)(1.0 / (kFourPi * t.half_width(a.level[e])));
    }
    const int64_t nw = (int64_t)pl->w_cube_box.size();
    if (!t.adaptive || nw == 0) return a;
    std::vector<int32_t> cube_of_box(t.n_box(), -1);
    for (int64_t w = 0; w < nw; ++w) cube_of_box[pl->w_cube_box[w]] = (int32_t)w;
    for (int64_t e = 0; e < nl; ++e) {
        if (t.w_ptr[e + 1] == t.w_ptr[e]) continue;
        int64_t c[3], ec[3];
        const int l = box_cube(t, t.leaf_box[e], c);
        a.mleaf.push_back((int32_t)e);
        for (int32_t k = t.w_ptr[e]; k < t.w_ptr[e + 1]; ++k) {
            const int m = box_cube(t, t.w_src[k], ec);
            const double rho = std::ldexp(1.0, l - m);
            a.mcube.push_back(cube_of_box[t.w_src[k]]);
            a.mgeo.push_back((T)rho);
            for (int d = 0; d < 3; ++d) a.mgeo.push_back((T)((2.0 * ec[d] + 1.0) * rho - (2.0 * c[d] + 1.0)));
        }
        a.mptr.push_back((int32_t)a.mcube.size());
    }
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t g = pl->w_cube_box[w];
        int64_t c[3], ec[3];
        const int m = box_cube(t, g, ec);
        for (int32_t k = t.x_ptr[g]; k < t.x_ptr[g + 1]; ++k) {
            const int32_t e = t.x_src[k];
            const int l = box_cube(t, t.leaf_box[e], c);
            const double rho = std::ldexp(1.0, m - l);
            a.sleaf.push_back(e);
            a.sgeo.push_back((T)rho);
            for (int d = 0; d < 3; ++d) a.sgeo.push_back((T)((2.0 * c[d] + 1.0) * rho - (2.0 * ec[d] + 1.0)));
        }
        a.sptr.push_back((int32_t)a.sleaf.size());
    }
    return a;
}

// Device lists of an adaptive plan: leaf levels and scales, the M2T entries
// of every leaf with a W list and the S2L entries of every W cube, each with
// the geometry (rho, o) that maps the source into the target's units: for M2T
// the W cube's surface point s becomes rho s + o in the units of the target
// leaf (rho = r_cube / r_leaf), for S2L a point u of the source leaf becomes
// rho u + o in the units of the W cube (rho = r_leaf / r_cube); rho is a power
// of two and o a multiple of rho or an integer, so both are exact.
template <typename T>
void upload_adaptive(kifmm_plan_s* pl, Uploader& up) {
    const AdaptiveLists<T> a = adaptive_lists<T>(pl);
    pl->leaf_level = (int32_t*)up.put(a.level);
    pl->leaf_scale = up.put(a.scale);
    const int64_t nw = (int64_t)pl->w_cube_box.size();
    if (nw == 0) return;
    pl->n_m2t_leaf = (int64_t)a.mleaf.size();
    pl->m2t_leaf = (int32_t*)up.put(a.mleaf);
    pl->m2t_ptr = (int32_t*)up.put(a.mptr);
    pl->m2t_cube = (int32_t*)up.put(a.mcube);
    pl->m2t_geo = up.put(a.mgeo);
    pl->s2l_ptr = (int32_t*)up.put(a.sptr);
    pl->s2l_leaf = (int32_t*)up.put(a.sleaf);
    pl->s2l_geo = up.put(a.sgeo);
    pl->d_m2t = upload_sched(up, pl->h_m2t, pl->elt);
    pl->d_s2l = upload_sched(up, pl->h_s2l, pl->elt, &pl->w_cube_box);
    const size_t bytes = (size_t)nw * pl->R * pl->nep * pl->elt;
    pl->CX = up.zeros(bytes);
    pl->Psi = up.zeros(bytes);
}

// Triangles of a BEM plan in the plan's point order, in the units of each
// triangle's leaf (the leaf of its centroid): the 7-point rule of Radon
// (degree 5; weights x area, divided by r_L for the double layer, whose S2M
// kernel carries one more inverse length), the unit normal, and the vertices.
struct BemMesh {
    std::vector<double> verts;   // 3 per vertex
    std::vector<int32_t> tris;   // 3 per triangle (caller order)
};

template <typename T>
void upload_bem(kifmm_plan_s* pl, Uploader& up, const BemMesh& m) {
    const HostTree& t = pl->tree;
    const int64_t n = t.n;
    const double r = t.half_width(t.depth);
    const double s15 = std::sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, b1 = (9.0 + 2.0 * s15) / 21.0;
    const double a2 = (6.0 + s15) / 21.0, b2 = (9.0 - 2.0 * s15) / 21.0;
    const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
    const double bary[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, a1, b1}, {a1, b1, a1}, {b1, a1, a1},
                               {a2, a2, b2}, {a2, b2, a2}, {b2, a2, a2}};
    const double wq[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
    std::vector<T> qp(28 * (size_t)n), tn(4 * (size_t)n, T(0)), tri(16 * (size_t)n, T(0));
    for (int64_t e = 0; e < t.n_leaf(); ++e) {
        int64_t c[3];
        box_cube(t, t.level_begin[t.depth] + e, c);
        double cen[3];
        for (int a = 0; a < 3; ++a) cen[a] = (t.centre[a] - t.r0) + (2.0 * double(c[a]) + 1.0) * r;
        for (int32_t i = t.leaf_ptr[e]; i < t.leaf_ptr[e + 1]; ++i) {
            const int32_t* f = &m.tris[3 * (size_t)t.perm[i]];
            double v[3][3];
            for (int k = 0; k < 3; ++k)
                for (int a = 0; a < 3; ++a) v[k][a] = (m.verts[3 * (size_t)f[k] + a] - cen[a]) / r;
            const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
            const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
            const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                  e1[0] * e2[1] - e1[1] * e2[0]};
            const double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            const double area = 0.5 * len * r * r;   // physical area
            const double wscale = pl->layer == 1 ? area / r : area;
            for (int k = 0; k < 7; ++k) {
                for (int a = 0; a < 3; ++a)
                    qp[28 * (size_t)i + 4 * k + a] =
                        (T)(bary[k][0] * v[0][a] + bary[k][1] * v[1][a] + bary[k][2] * v[2][a]);
                qp[28 * (size_t)i + 4 * k + 3] = (T)(wq[k] * wscale);
            }
            for (int a = 0; a < 3; ++a) {
                tn[4 * (size_t)i + a] = (T)(cr[a] / len);
                for (int k = 0; k < 3; ++k) tri[16 * (size_t)i + 4 * k + a] = (T)v[k][a];
                tri[16 * (size_t)i + 12 + a] = (T)(cr[a] / len);
            }
        }
    }
    pl->bem_qp = up.put(qp);
    pl->bem_tn = up.put(tn);
    pl->bem_tri = up.put(tri);
}

// Device schedules and buffer of the stage-2 M2L (Sec. 3.2), from the M2L
// schedule (same tiles and chunks): phase A writes w = V^ q of every pair into
// its own chunk slot (direct form: one output row per slot), phase B adds
// scale * U^ w into the targets. Phase B reads W through 32-bit buffer
// offsets, so it runs as launches over consecutive tile ranges whose W rows
// each span less than 2 GiB, with slot numbers relative to the range. Word 1
// of the chunk metadata carries, above the block count, the 16-blocks of the
// class's rank (phase A: rows of V^; phase B: K-chunks of U^); the rank of a
// class and of its negation are equal up to rounding at the cutoff, and the
// larger one is used for both.
void upload_stage2(kifmm_plan_s* pl, Uploader& up) {
    const GGSched& s = pl->h_m2l;
    const int nch = s.n_chunks();
    if (nch == 0) return;
    const HostOps& o = pl->ops();
    const int64_t row_bytes = (int64_t)pl->rp * pl->elt;          // one W row (slot x rhs)
    const int64_t slot_bytes = (int64_t)pl->R * row_bytes;
    const int64_t wbytes = (int64_t)nch * s.cp * slot_bytes;
    DevSched a = upload_sched(up, s, pl->elt);
    if (up.err != KIFMM_OK) return;
    std::vector<int32_t> meta((size_t)4 * nch, 0), slot(s.chunk_src.size(), -1);
    for (int c = 0; c < nch; ++c) {
        const int cls = s.chunk_cls[c];
        const int rb = (std::max(o.rank2[cls], o.rank2[neg_class(cls)]) + 15) / 16;
        meta[4 * c] = cls;
        meta[4 * c + 1] = s.chunk_nblk[c] | (rb << 8);
        if (pl->elt == 4) {
            const float f = (float)s.chunk_scale[c];
            std::memcpy(&meta[4 * c + 2], &f, sizeof f);
        } else {
            std::memcpy(&meta[4 * c + 2], &s.chunk_scale[c], sizeof(double));
        }
    }
    for (size_t i = 0; i < slot.size(); ++i)
        if (s.chunk_src[i] >= 0) slot[i] = (int32_t)i;
    // tile ranges of phase B: the W rows of a range's slots stay below 2 GiB,
    // and its slot numbers below 2^24 (the kernel's 24-bit row multiply)
    const std::vector<int> rbeg = split_tile_ranges(s.tile_chunk0, s.cp, slot_bytes,
                                                    ((int64_t)1 << 31) - ((int64_t)1 << 20), ((int64_t)1 << 24) - 1);
    if (rbeg.empty()) {
        up.err = KIFMM_EINVAL;
        up.msg = "stage-2: the products of one M2L tile exceed the 32-bit offsets of the kernel";
        return;
    }
    std::vector<int32_t> rel(slot.size(), -1);
    std::vector<int32_t> rel_max(rbeg.size() - 1, 0);
    for (size_t r = 0; r + 1 < rbeg.size(); ++r) {
        const int64_t c0 = s.tile_chunk0[rbeg[r]], c1 = s.tile_chunk0[rbeg[r + 1]];
        for (int64_t i = c0 * s.cp; i < c1 * s.cp; ++i)
            if (slot[i] >= 0) {
                rel[i] = (int32_t)(slot[i] - c0 * s.cp);
                rel_max[r] = std::max(rel_max[r], rel[i]);
            }
    }
    a.chunk_meta = (const int32_t*)up.put(meta);
    const int32_t* dslot = (const int32_t*)up.put(slot);
    const int32_t* drel = (const int32_t*)up.put(rel);
    DevSched b = a;
    a.direct = true;          // target of a slot = the slot's row of w
    a.unit_scale = true;      // the level scale is applied in phase B
    a.chunk_tgt = dslot;
    b.direct = false;
    b.chunk_tgt = nullptr;
    b.chunk_src = drel;       // source of a slot = its row of w, from the range's first slot
    pl->d_s2a = a;
    pl->d_s2b.clear();
    pl->s2b_xoff.clear();
    for (size_t r = 0; r + 1 < rbeg.size(); ++r) {
        DevSched br = b;
        br.n_tiles = rbeg[r + 1] - rbeg[r];
        br.tile_tgt0 = b.tile_tgt0 + rbeg[r];
        br.tile_ntgt = b.tile_ntgt + rbeg[r];
        br.tile_chunk0 = b.tile_chunk0 + rbeg[r];
        br.max_src = rel_max[r];
        pl->d_s2b.push_back(br);
        pl->s2b_xoff.push_back((size_t)((int64_t)s.tile_chunk0[rbeg[r]] * s.cp * slot_bytes));
    }
    pl->W = up.zeros((size_t)wbytes);
}

void fill_info(kifmm_plan_s* pl, double seconds) {
    kifmm_info_t& in = pl->info;
    const HostTree& t = pl->tree;
    std::memset(&in, 0, sizeof(in));
    in.depth = t.depth;
    in.k = pl->ops().k;
    in.n_eq = pl->ops().n_eq;
    in.k_pad = pl->kp;
    in.precision = pl->opts.precision;
    in.dense_m2l = pl->opts.dense_m2l;
    in.n = t.n;
    in.n_leaf = t.n_leaf();
    in.n_box = t.n_box();
    in.near_pairs = (int64_t)t.near_leaf.size();
    int64_t inter = 0;
    for (int64_t e = 0; e < t.n_leaf(); ++e) {
        int64_t ne = t.leaf_ptr[e + 1] - t.leaf_ptr[e];
        for (int32_t q = t.near_ptr[e]; q < t.near_ptr[e + 1]; ++q)
            inter += ne * (int64_t)(t.leaf_ptr[t.near_leaf[q] + 1] - t.leaf_ptr[t.near_leaf[q]]);
    }
    in.p2p_interactions = inter;
    for (int l = 0; l <= t.depth; ++l) {
        in.boxes_level[l] = t.level_count(l);
        in.v_pairs_level[l] = t.v_ptr[t.level_begin[l + 1]] - t.v_ptr[t.level_begin[l]];
        in.v_pairs += in.v_pairs_level[l];
    }
    in.r0 = t.r0;
    const double k = pl->ops().k, ne = pl->ops().n_eq, nl = (double)t.n_leaf(), N = (double)t.n;
    const double elt = pl->elt;
    int64_t nbox_up = 0;
    for (int l = 2; l < t.depth; ++l) nbox_up += t.level_count(l + 1);
    const bool far = t.depth >= 2;
    // 11 flops per point-surface or point-point kernel evaluation (3 sub, 3 mul,
    // 2 add, rsqrt, multiply-add)
    in.flops[KIFMM_STAGE_P2M] = far ? 11.0 * N * ne + 2.0 * k * ne * nl : 0;
    in.flops[KIFMM_STAGE_M2M] = far ? 2.0 * k * k * (double)nbox_up : 0;
    in.flops[KIFMM_STAGE_M2L] = 2.0 * k * k * (double)in.v_pairs;
    if (pl->st2) {
        // two thin products per pair: 2 k r (w = V^ q) + 2 k r (U^ w), r the class rank
        double f = 0.0, rs = 0.0;
        for (int32_t c : t.v_cls) f += 4.0 * k * pl->ops().rank2[c];
        for (int32_t r : pl->ops().rank2) rs += r;
        in.flops[KIFMM_STAGE_M2L] = f;
        in.m2l_rank_max = pl->ops().r2max;
        in.m2l_rank_mean = rs / NCLASS;
    }
    in.flops[KIFMM_STAGE_L2L] = far ? 2.0 * k * k * (double)nbox_up : 0;
    in.flops[KIFMM_STAGE_L2P] = far ? 11.0 * N * ne + 2.0 * k * ne * nl : 0;
    in.flops[KIFMM_STAGE_P2P] = 11.0 * (double)inter;
    int64_t nbox_m2l = 0;
    for (int l = 2; l <= t.depth; ++l) nbox_m2l += t.level_count(l);
    in.bytes[KIFMM_STAGE_P2M] = far ? N * (16 + elt) + nl * k * elt : 0;
    in.bytes[KIFMM_STAGE_M2M] = far ? 2.0 * nbox_up * k * elt : 0;
    in.bytes[KIFMM_STAGE_M2L] = 2.0 * nbox_m2l * k * elt + (double)NCLASS * k * k * elt;
    in.bytes[KIFMM_STAGE_L2L] = far ? 3.0 * nbox_up * k * elt : 0;
    in.bytes[KIFMM_STAGE_L2P] = far ? nl * k * elt + N * (16 + elt) : 0;
    in.bytes[KIFMM_STAGE_P2P] = N * (16 + 2 * elt + 4);
    in.bytes[KIFMM_STAGE_PERM] = N * (2 * elt + 4);
    in.device_bytes = pl->device_bytes;
    in.m2l_tile_targets = pl->h_m2l.max_tile;
    in.sigma0 = pl->ops().sigma0;
    in.plan_seconds = seconds;
    in.m2l_variant = pl->h_m2l.variant;
    in.m2l_tiles = pl->h_m2l.n_tiles();
    in.m2l_chunks = pl->h_m2l.n_chunks();
    for (int32_t b : pl->h_m2l.chunk_nblk) in.m2l_blocks += b & 0xff;
    in.adaptive = t.adaptive ? 1 : 0;
    in.layer = pl->layer;
    in.leaf_level_min = t.depth;
    if (t.adaptive) {
        for (int32_t l : t.leaf_level) in.leaf_level_min = std::min(in.leaf_level_min, (int)l);
        in.w_pairs = (int64_t)t.w_src.size();
        in.w_cubes = (int64_t)pl->w_cube_box.size();
        // M2T: U~ q~ per W cube, then every (point, surface point) of the W
        // entries of its leaf; S2L: every (source point, surface point) of the
        // X entries, then U~^T per W cube
        double pts_w = 0.0, pts_x = 0.0;
        for (int64_t e = 0; e < t.n_leaf(); ++e)
            pts_w += (double)(t.leaf_ptr[e + 1] - t.leaf_ptr[e]) * (t.w_ptr[e + 1] - t.w_ptr[e]);
        for (int32_t e : t.x_src) pts_x += (double)(t.leaf_ptr[e + 1] - t.leaf_ptr[e]);
        in.m2t_flops = 2.0 * k * ne * (double)in.w_cubes + 11.0 * ne * pts_w;
        in.s2l_flops = 11.0 * ne * pts_x + 2.0 * k * ne * (double)in.w_cubes;
    }
}

// Largest tile (targets) whose LDS accumulator (plus the R spare columns of
// empty slots) fits one workgroup of the shape.
int max_tile_for(const kifmm_plan_s* pl, int variant, int kdim) {
    const size_t fixed = gg_lds_bytes(pl->elt, variant, kdim / 16, pl->R);
    const size_t per_col = (gg_lds_bytes(pl->elt, variant, kdim / 16, 1) - gg_lds_bytes(pl->elt, variant, kdim / 16, 0)) * pl->R;
    if (gg_lds_limit(variant) <= fixed + per_col) return 1;
    return std::max(1, (int)((gg_lds_limit(variant) - fixed) / per_col));
}

int row_groups(int rows_pad, int variant) {
    const int mbg = gg_variant_rows(variant) / 16;
    return (rows_pad / 16 + mbg - 1) / mbg;
}

// M2L schedule over every box of levels 2..L (one contiguous target range);
// tiles are cut at equal estimated kernel cost (chunks, blocks, targets) into
// at most `n_tiles` tiles, or uniformly into `tile` targets when tile > 0.
GGSched build_m2l_sched(const kifmm_plan_s* pl, int variant, int n_tiles, int tile) {
    const HostTree& t = pl->tree;
    GGSched s;
    s.cp = 32 / pl->R;
    s.rhs = pl->R;
    s.variant = variant;
    const int L = t.depth;
    if (L < 2) return s;
    const int64_t b0 = t.level_begin[2], nb = t.n_box() - b0;
    std::vector<int32_t> group(nb);
    std::vector<double> scale(L - 1);
    for (int l = 2; l <= L; ++l) {
        scale[l - 2] = 1.0 / t.half_width(l);
        for (int64_t b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b) group[b - b0] = l - 2;
    }
    const int cap = max_tile_for(pl, variant, pl->kp);
    // The loop of the kernel costs about the same per chunk whatever its fill,
    // plus a share per 16-column block of MFMA work and a little per target
    // (accumulator set-up and store); tiles of equal pair counts would differ
    // by up to 2.3x in chunks (coarse levels have short class runs).
    TileCost w;
    w.per_chunk = 1.0;
    w.per_block = 0.5;
    w.per_target = 0.05;
    std::vector<int64_t> cuts = tile > 0 ? uniform_cuts(nb, std::min(tile, cap))
                                         : chunk_cuts(nb, &t.v_ptr[b0], t.v_cls.data(), group.data(), s.cp,
                                                      pl->R, n_tiles, cap, w);
    gg_build(s, b0, nb, &t.v_ptr[b0], t.v_src.data(), t.v_cls.data(), group.data(), scale, cuts);
    return s;
}

// Tiles for `variant` so that the launch fills the CUs in whole rounds.
int m2l_tiles_for(const kifmm_plan_s* pl, int variant, int extra_rounds) {
    const HostTree& t = pl->tree;
    const int64_t nb = t.n_box() - t.level_begin[2];
    const int n_rg = row_groups(pl->kp, variant);
    const int slots = std::max(1, pl->num_cu * gg_variant_wgs_per_cu(variant) / n_rg);
    const int cap = max_tile_for(pl, variant, pl->kp);
    int rounds = 1;
    while ((int64_t)rounds * slots * cap < nb * 11 / 10) ++rounds;
    return (rounds + extra_rounds) * slots;
}

void build_uniform_passes(kifmm_plan_s* pl, const std::function<int(int64_t)>& level_tile);

// The parents of level l (cubes with at least one child) and their eight
// child rows (-1: no child), every row offset by off, appended to par / ch.
void m2m_lists(const HostTree& t, int l, int32_t off, std::vector<int32_t>& par, std::vector<int32_t>& ch) {
    for (int64_t b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b) {
        bool any = false;
        for (int o = 0; o < 8; ++o) any = any || t.box_child[8 * b + o] >= 0;
        if (!any) continue;
        par.push_back((int32_t)b + off);
        for (int o = 0; o < 8; ++o) {
            const int32_t c = t.box_child[8 * b + o];
            ch.push_back(c < 0 ? -1 : c + off);
        }
    }
}

// Above this many parents a level's M2M runs as the grouped GEMM, which reads
// each octant matrix once per tile of up to a few hundred parents; the direct
// kernel reads it once per 16 parents and only wins where launch latency
// dominates (measured at p = 6: 6-12 us against 26 us per launch up to about
// 1200 parents, 32 against 27 us at 4700).
constexpr int64_t kM2MDirectMax = 3072;

void upload_m2m(kifmm_plan_s* pl, Uploader& up, const std::vector<std::vector<int32_t>>& par,
                const std::vector<std::vector<int32_t>>& ch) {
    pl->m2m_n.assign(par.size(), 0);
    pl->d_m2m.assign(par.size(), nullptr);
    for (size_t l = 0; l < par.size(); ++l) {
        if (par[l].empty() || (int64_t)par[l].size() > kM2MDirectMax) continue;
        std::vector<int32_t> v(par[l]);
        v.insert(v.end(), ch[l].begin(), ch[l].end());
        pl->m2m_n[l] = (int32_t)par[l].size();
        pl->d_m2m[l] = (int32_t*)up.put(v);
    }
    pl->m2m_direct = up.err == KIFMM_OK;
}

// One L2L product of the direct form: child row tgt from parent row src with
// the octant class cls.
struct DownItem {
    int32_t cls, tgt, src;
};

// The L2L items of level l (every cube of the level from its parent), rows
// offset by off, appended to v.
void down_items(const HostTree& t, int l, int32_t off, std::vector<DownItem>& v) {
    for (int64_t b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b)
        v.push_back({(int32_t)(t.box_key[b] & 7), (int32_t)b + off, t.box_parent[b] + off});
}

// Segments of the direct L2L kernel per level: the items sorted by class
// (stable: Morton order within a class), cut into runs of one class of up to
// 16 * nb items, nb (at most kDownMaxBlocks) the fewest 16-column blocks per
// segment that let every segment of the level be resident at once (two
// workgroups per CU up to k_pad = 144, one above, by the kernel's register
// count): a second, partial round of workgroups would double the launch, and
// longer segments amortise the operator rows a workgroup loads.
void upload_down(kifmm_plan_s* pl, Uploader& up, std::vector<std::vector<DownItem>>& items) {
    const size_t nl = items.size();
    pl->dd_nseg.assign(nl, 0);
    pl->dd_ncb.assign(nl, 1);
    pl->dd_nitem.assign(nl, 0);
    pl->d_dd.assign(nl, nullptr);
    for (size_t l = 0; l < nl; ++l) {
        std::vector<DownItem>& v = items[l];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [](const DownItem& a, const DownItem& b) { return a.cls < b.cls; });
        int64_t nblk = 0;
        for (size_t i = 0; i < v.size();) {
            size_t e = i;
            while (e < v.size() && v[e].cls == v[i].cls) ++e;
            nblk += (int64_t)(e - i + 15) / 16;
            i = e;
        }
        const int64_t slots = (int64_t)pl->num_cu * (pl->kp <= 144 ? 2 : 1);
        // the class runs add up to 8 partial segments
        const int ncb = (int)std::min<int64_t>(kDownMaxBlocks, std::max<int64_t>(1, (nblk + slots - 9) / (slots - 8)));
        std::vector<int32_t> segs;
        for (size_t i = 0; i < v.size();) {
            size_t e = i;
            while (e < v.size() && v[e].cls == v[i].cls && e - i < (size_t)16 * ncb) ++e;
            segs.insert(segs.end(), {v[i].cls, (int32_t)i, (int32_t)(e - i)});
            i = e;
        }
        std::vector<int32_t> buf(segs);
        for (const DownItem& d : v) buf.push_back(d.tgt);
        for (const DownItem& d : v) buf.push_back(d.src);
        pl->dd_nseg[l] = (int32_t)(segs.size() / 3);
        pl->dd_ncb[l] = ncb;
        pl->dd_nitem[l] = (int32_t)v.size();
        pl->d_dd[l] = (int32_t*)up.put(buf);
    }
    pl->down_direct = up.err == KIFMM_OK;
}

// Schedules of the upward and downward passes of an adaptive tree (the M2L
// schedule is the uniform tree's: every cube of levels >= 2). S2M at the
// leaves of levels >= 2 (a level's leaves come first among its cubes), M2M
// into its split cubes, L2L into every cube of levels >= 3, L2T at the leaves
// of levels >= 2 (coarser leaves take their far field from W alone), and the
// M2T / S2L products of the W cubes.
void build_adaptive_passes(kifmm_plan_s* pl, const std::function<int(int64_t)>& level_tile) {
    const HostTree& t = pl->tree;
    const int L = t.depth;
    const int64_t nleaf = t.n_leaf();
    const std::vector<double> one{1.0}, inv4pi{1.0 / kFourPi};
    int64_t n_up = 0;
    for (int l = 2; l <= L; ++l) n_up += t.level_leaves[l];
    const int per_cu = (int)std::max<int64_t>(1, (n_up + pl->num_cu - 1) / pl->num_cu);
    const int tile_up = std::min(std::max(16 / pl->R + 1, per_cu), max_tile_for(pl, 0, pl->nep));
    const int tile_dn = std::min(std::max(16 / pl->R + 1, per_cu), max_tile_for(pl, 0, pl->kp));
    for (int l = 2; l <= L; ++l) {
        const int64_t b0 = t.level_begin[l], nl = t.level_leaves[l];
        if (nl == 0) continue;
        std::vector<int32_t> ptr(nl + 1), src(nl), cls(nl, 0);
        for (int64_t e = 0; e <= nl; ++e) ptr[e] = (int32_t)e;
        for (int64_t e = 0; e < nl; ++e) src[e] = t.box_leaf[b0 + e];
        gg_build(pl->h_leafup, b0, nl, ptr.data(), src.data(), cls.data(), nullptr, inv4pi, uniform_cuts(nl, tile_up));
    }
    for (int64_t e0 = 0; e0 < nleaf;) {
        if (t.leaf_level[e0] < 2) {
            ++e0;
            continue;
        }
        int64_t e1 = e0;
        while (e1 < nleaf && t.leaf_level[e1] >= 2) ++e1;
        const int64_t nr = e1 - e0;
        std::vector<int32_t> ptr(nr + 1), src(nr), cls(nr, 0);
        for (int64_t e = 0; e <= nr; ++e) ptr[e] = (int32_t)e;
        for (int64_t e = 0; e < nr; ++e) src[e] = t.leaf_box[e0 + e];
        gg_build(pl->h_leafdown, e0, nr, ptr.data(), src.data(), cls.data(), nullptr, one, uniform_cuts(nr, tile_dn));
        e0 = e1;
    }
    for (int l = 2; l < L; ++l) {
        const int64_t b0 = t.level_begin[l] + t.level_leaves[l], nb = t.level_begin[l + 1] - b0;
        if (nb == 0) continue;
        std::vector<int32_t> ptr(1, 0), src, cls;
        for (int64_t b = 0; b < nb; ++b) {
            for (int o = 0; o < 8; ++o) {
                const int32_t ch = t.box_child[8 * (b0 + b) + o];
                if (ch >= 0) {
                    src.push_back(ch);
                    cls.push_back(o);
                }
            }
            ptr.push_back((int32_t)src.size());
        }
        gg_build(pl->h_up[l], b0, nb, ptr.data(), src.data(), cls.data(), nullptr, one,
                 uniform_cuts(nb, level_tile(nb)));
    }
    for (int l = 3; l <= L; ++l) {
        const int64_t b0 = t.level_begin[l], nb = t.level_count(l);
        std::vector<int32_t> ptr(nb + 1), src(nb), cls(nb);
        for (int64_t b = 0; b < nb; ++b) {
            ptr[b] = (int32_t)b;
            src[b] = t.box_parent[b0 + b];
            cls[b] = (int32_t)(t.box_key[b0 + b] & 7);
        }
        ptr[nb] = (int32_t)nb;
        // one tile: the direct form runs a workgroup per chunk, so the chunks
        // of a level are best full (32 children of one octant each)
        gg_build(pl->h_down[l], b0, nb, ptr.data(), src.data(), cls.data(), nullptr, one, uniform_cuts(nb, nb));
    }
    // W cubes: Psi = U~ q~ (one product each) and P += U~^T CX / (4 pi r_l)
    pl->w_cube_box.clear();
    for (int64_t g = 0; g < t.n_box(); ++g)
        if (t.x_ptr[g + 1] > t.x_ptr[g]) pl->w_cube_box.push_back((int32_t)g);
    const int64_t nw = (int64_t)pl->w_cube_box.size();
    pl->h_m2t = GGSched();
    pl->h_s2l = GGSched();
    for (GGSched* s : {&pl->h_m2t, &pl->h_s2l}) {
        s->cp = 32 / pl->R;
        s->rhs = pl->R;
    }
    if (nw > 0) {
        std::vector<int32_t> ptr(nw + 1), src(nw), cls(nw, 0), grp(nw);
        for (int64_t w = 0; w <= nw; ++w) ptr[w] = (int32_t)w;
        std::vector<double> scale(L + 1);
        for (int l = 0; l <= L; ++l) scale[l] = 1.0 / (kFourPi * t.half_width(l));
        for (int64_t w = 0; w < nw; ++w) {
            const int64_t g = pl->w_cube_box[w];
            src[w] = (int32_t)g;
            int l = 0;
            while (t.level_begin[l + 1] <= g) ++l;
            grp[w] = l;
        }
        gg_build(pl->h_m2t, 0, nw, ptr.data(), src.data(), cls.data(), nullptr, one, uniform_cuts(nw, 64));
        for (int64_t w = 0; w < nw; ++w) src[w] = (int32_t)w;
        gg_build(pl->h_s2l, 0, nw, ptr.data(), src.data(), cls.data(), grp.data(), scale, uniform_cuts(nw, 64));
    }
}

int build_schedules(kifmm_plan_s* pl, int m2l_tile, int m2l_shape) {
    const HostTree& t = pl->tree;
    const int L = t.depth;
    pl->h_leafup = GGSched();
    pl->h_leafdown = GGSched();
    pl->h_m2l = GGSched();
    pl->h_up.assign(L + 1, GGSched());
    pl->h_down.assign(L + 1, GGSched());
    const int cp = 32 / pl->R;
    for (GGSched* s : {&pl->h_leafup, &pl->h_leafdown, &pl->h_m2l}) {
        s->cp = cp;
        s->rhs = pl->R;
    }
    for (auto& s : pl->h_up) {
        s.cp = cp;
        s.rhs = pl->R;
    }
    for (auto& s : pl->h_down) {
        s.cp = cp;
        s.rhs = pl->R;
    }
    if (L < 2) return KIFMM_OK;
    // tiles of a per-level launch: about one workgroup per CU for the large
    // levels (a workgroup's fixed costs - pipeline fill, accumulator load and
    // store - then amortise over many chunks), small ones for small levels so
    // that they still spread over the chip
    auto level_tile = [&](int64_t nb) {
        const int64_t per_cu = (nb + pl->num_cu - 1) / pl->num_cu;
        const int64_t tl = std::max<int64_t>(16 / pl->R + 1, per_cu);
        return (int)std::min<int64_t>(tl, max_tile_for(pl, 0, pl->kp));
    };
    if (t.adaptive) {
        build_adaptive_passes(pl, level_tile);
    } else {
        build_uniform_passes(pl, level_tile);
    }
    // M2L: default shape (the device autotuner may replace it)
    if (m2l_tile > 0)
        pl->h_m2l = build_m2l_sched(pl, m2l_shape, 0, m2l_tile);
    else
        pl->h_m2l = build_m2l_sched(pl, m2l_shape, m2l_tiles_for(pl, m2l_shape, 0), 0);
    return KIFMM_OK;
}

// Schedules of the upward and downward passes of a uniform tree.
void build_uniform_passes(kifmm_plan_s* pl, const std::function<int(int64_t)>& level_tile) {
    const HostTree& t = pl->tree;
    const int L = t.depth;
    const int64_t nleaf = t.n_leaf();
    const int64_t lb = t.level_begin[L];
    const std::vector<double> one{1.0}, inv4pi{1.0 / kFourPi};
    {
        std::vector<int32_t> ptr(nleaf + 1), src(nleaf), cls(nleaf, 0);
        for (int64_t e = 0; e <= nleaf; ++e) ptr[e] = (int32_t)e;
        for (int64_t e = 0; e < nleaf; ++e) src[e] = (int32_t)e;
        const int per_cu = (int)((nleaf + pl->num_cu - 1) / pl->num_cu);
        const int tile_up = std::min(std::max(16 / pl->R + 1, per_cu), max_tile_for(pl, 0, pl->nep));
        gg_build(pl->h_leafup, lb, nleaf, ptr.data(), src.data(), cls.data(), nullptr, inv4pi,
                 uniform_cuts(nleaf, tile_up));
        for (int64_t e = 0; e < nleaf; ++e) src[e] = (int32_t)(lb + e);
        const int tile_dn = std::min(std::max(16 / pl->R + 1, per_cu), max_tile_for(pl, 0, pl->kp));
        gg_build(pl->h_leafdown, 0, nleaf, ptr.data(), src.data(), cls.data(), nullptr, one,
                 uniform_cuts(nleaf, tile_dn));
    }
    for (int l = 2; l < L; ++l) {
        // targets at level l, sources their children at level l+1 (class = octant)
        const int64_t b0 = t.level_begin[l], nb = t.level_count(l);
        std::vector<int32_t> ptr(1, 0), src, cls;
        for (int64_t b = 0; b < nb; ++b) {
            for (int o = 0; o < 8; ++o) {
                int32_t ch = t.box_child[8 * (b0 + b) + o];
                if (ch >= 0) {
                    src.push_back(ch);
                    cls.push_back(o);
                }
            }
            ptr.push_back((int32_t)src.size());
        }
        gg_build(pl->h_up[l], b0, nb, ptr.data(), src.data(), cls.data(), nullptr, one,
                 uniform_cuts(nb, level_tile(nb)));
    }
    for (int l = 3; l <= L; ++l) {
        // targets at level l, source their parent at level l-1 (class = own octant)
        const int64_t b0 = t.level_begin[l], nb = t.level_count(l);
        std::vector<int32_t> ptr(nb + 1), src(nb), cls(nb);
        for (int64_t b = 0; b < nb; ++b) {
            ptr[b] = (int32_t)b;
            src[b] = t.box_parent[b0 + b];
            cls[b] = (int32_t)(t.box_key[b0 + b] & 7);
        }
        ptr[nb] = (int32_t)nb;
        // one pair per target (the direct form: one workgroup per chunk), so
        // one tile per level, whose chunks are full: 32 children of one octant
        gg_build(pl->h_down[l], b0, nb, ptr.data(), src.data(), cls.data(), nullptr, one, uniform_cuts(nb, nb));
    }
}

// M2L tile-shape autotuner: time the M2L launch for a few (row blocks per
// workgroup, workgroup rounds) shapes on the device and keep the fastest.
// Results are cached per (problem size, k, precision, nrhs width, CU count)
// for the life of the process.
struct TuneKey {
    int64_t n, n_box, v_pairs;
    int kp, elt, R, num_cu, shape;
    bool operator<(const TuneKey& o) const {
        return std::tie(n, n_box, v_pairs, kp, elt, R, num_cu, shape) <
               std::tie(o.n, o.n_box, o.v_pairs, o.kp, o.elt, o.R, o.num_cu, o.shape);
    }
};
// The cache is shared by every plan of the process; plans may be built from
// several threads, so every access holds tune_mutex().
std::map<TuneKey, std::pair<int, int>>& tune_cache() {
    static std::map<TuneKey, std::pair<int, int>> c;
    return c;
}
std::mutex& tune_mutex() {
    static std::mutex m;
    return m;
}

void autotune_m2l(kifmm_plan_s* pl, Uploader& up) {
    const HostTree& t = pl->tree;
    const int shape = pl->opts.m2l_shape;
    const TuneKey key{t.n, t.n_box(), (int64_t)t.v_src.size(), pl->kp, pl->elt, pl->R, pl->num_cu, shape};
    std::vector<std::pair<int, int>> cands;   // (kernel shape, extra rounds)
    bool cached = false;
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            cands.push_back(it->second);
            cached = true;
        }
    }
    if (!cached) {
        for (int v = 0; v < kGGVariants; ++v)
            if ((shape < 0 || v == shape) && gg_variant_supported(v, pl->elt, pl->kp / 16))
                for (int r = 0; r < 3; ++r) cands.push_back({v, r});
    }
    if (cands.size() == 1) {
        pl->h_m2l = build_m2l_sched(pl, cands[0].first, m2l_tiles_for(pl, cands[0].first, cands[0].second), 0);
        pl->d_m2l = upload_sched(up, pl->h_m2l, pl->elt);
        return;
    }
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best_ms = 1e30f;
    std::pair<int, int> best = {0, 0};
    GGSched best_sched;
    const int kp16 = pl->kp / 16;
    for (auto c : cands) {
        GGSched hs = build_m2l_sched(pl, c.first, m2l_tiles_for(pl, c.first, c.second), 0);
        std::vector<void*> scratch;
        Uploader tmp{pl, 0};
        tmp.scratch = &scratch;
        DevSched ds = upload_sched(tmp, hs, pl->elt);
        float ms = 1e30f;
        if (tmp.err == KIFMM_OK) {
            bool ok = launch_gg(ds, pl->elt, pl->Kt, kp16, kp16, pl->k, pl->k, pl->Q, pl->kp, pl->P, pl->kp, pl->R, 0, st, pl->b3) == hipSuccess;
            for (int rep = 0; ok && rep < 3; ++rep) {
                ok = hipEventRecord(e0, st) == hipSuccess &&
                     launch_gg(ds, pl->elt, pl->Kt, kp16, kp16, pl->k, pl->k, pl->Q, pl->kp, pl->P, pl->kp, pl->R, 0, st, pl->b3) == hipSuccess &&
                     hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
                float one = 0.f;
                if (ok && hipEventElapsedTime(&one, e0, e1) == hipSuccess) ms = std::min(ms, one);
            }
        }
        (void)hipStreamSynchronize(st);
        for (void* q : scratch) (void)hipFree(q);
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
            best_sched = std::move(hs);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (best_ms < 1e29f) {
        {
            std::lock_guard<std::mutex> lock(tune_mutex());
            tune_cache()[key] = best;
        }
        pl->h_m2l = std::move(best_sched);
        pl->tuned_ms = best_ms;
    }
    pl->d_m2l = upload_sched(up, pl->h_m2l, pl->elt);
}

// Device workspace of one apply: the permuted densities, the check and
// equivalent surface values of the leaves, the upward (Q~) and downward (P~)
// coefficients of every box and, in stage-2 plans, the per-pair products.
// Every element an apply reads is written earlier in the same apply, except
// the rows of W past a class's rank, which must hold zeros.
struct Work {
    void *sig_s = nullptr, *C = nullptr, *E = nullptr, *Q = nullptr, *P = nullptr, *W = nullptr;
    void *CX = nullptr, *Psi = nullptr;
};

Work plan_work(const kifmm_plan_s* pl) {
    Work w;
    w.sig_s = pl->sig_s;
    w.C = pl->C;
    w.E = pl->E;
    w.Q = pl->Q;
    w.P = pl->P;
    w.W = pl->W;
    w.CX = pl->CX;
    w.Psi = pl->Psi;
    return w;
}

// Device address of `scratch` on device `dev`, which must be the current
// device; looked up with hipGetSymbolAddress on the first call per device.
int scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lock(scratch_mutex());
    auto it = scratch_ptrs().find(dev);
    if (it != scratch_ptrs().end()) {
        *out = it->second;
        return KIFMM_OK;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return fail(KIFMM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    scratch_ptrs()[dev] = ptr;
    *out = ptr;
    return KIFMM_OK;
}

// Workspace of a plan carved out of `base` (256-byte aligned pieces); returns
// the bytes it needs. With base == nullptr only the size is computed.
size_t carve_work(const kifmm_plan_s* pl, char* base, Work* w) {
    const HostTree& t = pl->tree;
    const size_t elt = pl->elt, R = pl->R;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return p;
    };
    Work v;
    v.sig_s = take((size_t)t.n * R * elt);
    if (t.depth >= 2) {
        v.C = take((size_t)t.n_leaf() * R * pl->nep * elt);
        v.E = take((size_t)t.n_leaf() * R * pl->nep * elt);
        v.Q = take((size_t)t.n_box() * R * pl->kp * elt);
        v.P = take((size_t)t.n_box() * R * pl->kp * elt);
        if (!pl->w_cube_box.empty()) {
            v.CX = take(pl->w_cube_box.size() * R * pl->nep * elt);
            v.Psi = take(pl->w_cube_box.size() * R * pl->nep * elt);
        }
    }
    if (w) *w = v;
    return off;
}

int check_plan_for_apply(kifmm_plan_t plan) {
    if (!plan) return fail(KIFMM_EINVAL, "plan is NULL");
    if (!plan->on_device) return fail(KIFMM_ESTATE, "plan was built host-only (opts.device = -1)");
    return KIFMM_OK;
}

#define KIFMM_HIP(call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return fail(KIFMM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int run_passes(kifmm_plan_s* pl, const Work& w, const void* in, void* out, int nrhs, int64_t ld, bool adjoint,
               hipStream_t st) {
    const HostTree& t = pl->tree;
    const int L = t.depth;
    const int elt = pl->elt, R = pl->R, kp = pl->kp, nep = pl->nep;
    const int MBk = kp / 16, KPk = kp / 16, MBe = nep / 16, KPe = nep / 16;
    const int64_t nleaf = t.n_leaf();
    // Profiled applies record timing events that are read back later; an
    // event recorded inside a stream capture must not be used outside it, so
    // a profiled plan refuses to be captured.
    hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
    KIFMM_HIP(hipStreamIsCapturing(st, &cap_status));
    if (pl->profiling && cap_status != hipStreamCaptureStatusNone)
        return fail(KIFMM_ESTATE, "a plan with profiling on cannot be applied inside a stream capture");
    if (adjoint && pl->layer >= 0)
        return fail(KIFMM_ESTATE, "BEM plans have no adjoint apply (the collocation operator is not symmetric)");
    int cur = 0;
    KIFMM_HIP(hipGetDevice(&cur));
    if (cur != pl->device) KIFMM_HIP(hipSetDevice(pl->device));
    std::array<hipEvent_t, 2 * KIFMM_STAGE_COUNT>* ev = nullptr;
    if (pl->profiling) {
        if (pl->prof_free.empty()) {
            std::array<hipEvent_t, 2 * KIFMM_STAGE_COUNT> a{};
            for (auto& e : a) KIFMM_HIP(hipEventCreate(&e));
            pl->prof_free.push_back(a);
        }
        pl->prof_events.push_back(pl->prof_free.back());
        pl->prof_free.pop_back();
        ev = &pl->prof_events.back();
    }
    auto mark = [&](int stage, int end) -> hipError_t {
        return ev ? hipEventRecord((*ev)[2 * stage + end], st) : hipSuccess;
    };
    // Stages without work still record both events so that every pair is valid.
    KIFMM_HIP(mark(KIFMM_STAGE_PERM, 0));
    KIFMM_HIP(launch_permute_in(elt, R, t.n, pl->perm, in, ld, nrhs, w.sig_s, st));
    KIFMM_HIP(mark(KIFMM_STAGE_PERM, 1));
    const bool far = L >= 2;
    const double rL = t.half_width(L);
    // adaptive form: per-leaf levels and scales, and the W/X steps
    const bool ad = t.adaptive;
    const int64_t nw = (int64_t)pl->w_cube_box.size();
    const double near_scale = 1.0 / (kFourPi * rL);   // uniform form (the adaptive form has per-leaf scales)
    const int32_t* lev = ad ? pl->leaf_level : nullptr;
    const void* lsc = ad ? pl->leaf_scale : nullptr;
    const int n_eq = pl->ops().n_eq;
    // BEM plans (Sec. 4): triangles as sources; near-field scale of the
    // closed-form integrals in leaf units
    const bool bem = pl->layer >= 0;
    const double bem_scale = pl->layer == 1 ? -1.0 / kFourPi : rL / kFourPi;
    // M2T at the points (after the far field, adding to it)
    auto m2t_eval = [&]() -> hipError_t {
        if (!far || !ad || pl->n_m2t_leaf == 0) return hipSuccess;
        return launch_eval_m2t(elt, R, pl->n_m2t_leaf, pl->m2t_leaf, pl->pts, pl->leaf_ptr, pl->leaf_scale,
                               pl->m2t_ptr, pl->m2t_cube, pl->m2t_geo, w.Psi, pl->surf_in, n_eq, nep, pl->perm, out,
                               ld, nrhs, st);
    };
    // The near field (S2T) runs on the plan's own stream, concurrent with the
    // far-field passes, and the far-field evaluation waits for it. Under
    // stream capture everything stays on the capturing stream instead (near
    // and far fields in one kernel at the end): the fork and join events are
    // also recorded by eager applies, and an event recorded during a capture
    // must not be reused outside it.
    const bool fork = far && cap_status == hipStreamCaptureStatusNone;
    // the near field on the plan's own stream: forked after the permute, or
    // (near_late) just before M2L with the register-staged kernel; its launch
    // is then submitted after the M2L launch's (the fork event recorded before
    // it), so the M2L workgroups are dispatched first (measured 0.6% faster)
    const bool late = fork && pl->near_late && !adjoint;
    auto launch_near = [&]() -> int {
        hipStream_t ns = pl->near_stream;
        if (!late) KIFMM_HIP(hipEventRecord(pl->ev_fork, st));
        KIFMM_HIP(hipStreamWaitEvent(ns, pl->ev_fork, 0));
        if (ev) KIFMM_HIP(hipEventRecord((*ev)[2 * KIFMM_STAGE_P2P], ns));
        if (bem)
            KIFMM_HIP(launch_eval_near_bem(elt, pl->layer, nleaf, pl->pts, pl->bem_tri, w.sig_s, pl->leaf_ptr,
                                           pl->near_ptr, pl->near_leaf, pl->near_code, bem_scale, pl->perm, out, ns));
        else if (late)
            KIFMM_HIP(launch_near_reg(nleaf, pl->qpts, w.sig_s, pl->leaf_ptr, pl->near_ptr, pl->near_leaf,
                                      pl->near_code, near_scale, pl->perm, out, ns));
        else
            KIFMM_HIP(launch_eval_targets(1, elt, R, nleaf, pl->pts, pl->qpts, w.sig_s, pl->leaf_ptr, pl->near_ptr,
                                          pl->near_leaf, pl->near_code, lev, lsc, nullptr, pl->surf, n_eq, nep,
                                          near_scale, 1.0 / kFourPi, pl->perm, out, ld, nrhs, ns));
        if (ev) KIFMM_HIP(hipEventRecord((*ev)[2 * KIFMM_STAGE_P2P + 1], ns));
        KIFMM_HIP(hipEventRecord(pl->ev_join, ns));
        return KIFMM_OK;
    };
    if (fork && !late) {
        const int rc = launch_near();
        if (rc != KIFMM_OK) return rc;
    }
    KIFMM_HIP(mark(KIFMM_STAGE_P2M, 0));
    if (far) {
        // upward (forward) / L2T^T (adjoint): surface evaluation and the leaf
        // GEMM, in one launch when the fused kernel exists for this plan
        if (!bem && pl->fuse_s2m) {
            KIFMM_HIP(launch_s2m_fused(nleaf, pl->pts, w.sig_s, pl->leaf_ptr, pl->surf, n_eq, nep,
                                       adjoint ? pl->TopT : pl->Sop, kp, pl->leaf_row, 1.0 / kFourPi,
                                       adjoint ? w.P : w.Q, kp, st));
        } else {
            if (bem)
                KIFMM_HIP(launch_eval_surface_bem(elt, pl->layer, nleaf, pl->bem_qp, pl->bem_tn, w.sig_s,
                                                  pl->leaf_ptr, pl->surf, n_eq, nep, w.C, st));
            else
                KIFMM_HIP(launch_eval_surface(elt, R, nleaf, pl->pts, w.sig_s, pl->leaf_ptr, pl->surf, n_eq, nep,
                                              w.C, st));
            KIFMM_HIP(launch_gg(pl->d_leafup, elt, adjoint ? pl->TopT : pl->Sop, MBk, KPe, pl->k, n_eq, w.C, nep,
                                adjoint ? w.P : w.Q, kp, R, 0, st));
        }
    }
    KIFMM_HIP(mark(KIFMM_STAGE_P2M, 1));
    KIFMM_HIP(mark(KIFMM_STAGE_M2M, 0));
    if (far) {
        // M2M (forward) / L2L^T (adjoint): parents at l from children at l+1,
        // by one product per parent on the levels that have the direct lists
        const void* A = adjoint ? pl->LtT : pl->Mt;
        void* X = adjoint ? w.P : w.Q;
        for (int l = L - 1; l >= 2; --l) {
            const int32_t n = pl->m2m_direct && l < (int)pl->m2m_n.size() ? pl->m2m_n[l] : 0;
            if (n > 0)
                KIFMM_HIP(launch_m2m_direct(n, pl->d_m2m[l], pl->d_m2m[l] + n, A, kp, X, X, st));
            else
                KIFMM_HIP(launch_gg(pl->d_up[l], elt, A, MBk, KPk, pl->k, pl->k, X, kp, X, kp, R, 0, st));
        }
    }
    KIFMM_HIP(mark(KIFMM_STAGE_M2M, 1));
    if (late) KIFMM_HIP(hipEventRecord(pl->ev_fork, st));
    KIFMM_HIP(mark(KIFMM_STAGE_M2L, 0));
    if (far && ad && nw > 0) {
        // M2T: U~ q~ of every W cube (the adjoint: of the upward pass of its transpose, in P)
        KIFMM_HIP(launch_gg(pl->d_m2t, elt, pl->Ut, MBe, KPk, n_eq, pl->k, adjoint ? w.P : w.Q, kp, w.Psi, nep, R,
                            0, st));
    }
    if (far && pl->st2) {
        // stage 2 (Sec. 3.2): w = V^ q per pair, then p += r_l^-1 U^ w
        const int MBr = pl->rp / 16;
        KIFMM_HIP(launch_gg(pl->d_s2a, elt, adjoint ? pl->U2tT : pl->V2t, MBr, KPk, pl->rp, pl->k,
                            adjoint ? w.P : w.Q, kp, w.W, pl->rp, R, 0, st));
        for (size_t r = 0; r < pl->d_s2b.size(); ++r)
            KIFMM_HIP(launch_gg(pl->d_s2b[r], elt, adjoint ? pl->V2tT : pl->U2t, MBk, MBr, pl->k, pl->rp,
                                static_cast<const char*>(w.W) + pl->s2b_xoff[r], pl->rp,
                                adjoint ? w.Q : w.P, kp, R, 0, st));
    } else if (far) {
        if (!adjoint)
            KIFMM_HIP(launch_gg(pl->d_m2l, elt, pl->Kt, MBk, KPk, pl->k, pl->k, w.Q, kp, w.P, kp, R, 0, st, pl->b3));
        else
            KIFMM_HIP(launch_gg(pl->d_m2l, elt, pl->KtT, MBk, KPk, pl->k, pl->k, w.P, kp, w.Q, kp, R, 0, st, pl->b3));
    }
    if (far && ad && nw > 0) {
        // S2L: check potentials of the W cubes from the points of their X
        // leaves, projected by U~^T and added to the M2L result (the adjoint:
        // the transpose of M2T, into Q)
        KIFMM_HIP(launch_eval_s2l(elt, R, nw, pl->pts, w.sig_s, pl->leaf_ptr, pl->s2l_ptr, pl->s2l_leaf, pl->s2l_geo,
                                  pl->surf_in, n_eq, nep, w.CX, st));
        KIFMM_HIP(launch_gg(pl->d_s2l, elt, pl->UtT, MBk, KPe, pl->k, n_eq, w.CX, nep, adjoint ? w.Q : w.P, kp, R,
                            1, st));
    }
    KIFMM_HIP(mark(KIFMM_STAGE_M2L, 1));
    if (late) {
        const int rc = launch_near();
        if (rc != KIFMM_OK) return rc;
    }
    KIFMM_HIP(mark(KIFMM_STAGE_L2L, 0));
    if (far) {
        // L2L (forward) / M2M^T (adjoint): children at l from parents at l-1,
        // one product each, added
        const void* A = adjoint ? pl->MtT : pl->Lt;
        void* X = adjoint ? w.Q : w.P;
        for (int l = 3; l <= L; ++l) {
            const int32_t ns = pl->down_direct && l < (int)pl->dd_nseg.size() ? pl->dd_nseg[l] : 0;
            if (ns > 0) {
                const int32_t* d = pl->d_dd[l];
                KIFMM_HIP(launch_down_direct(ns, d, d + 3 * ns, d + 3 * ns + pl->dd_nitem[l], A, kp, X, X, st));
            } else {
                KIFMM_HIP(launch_gg(pl->d_down[l], elt, A, MBk, KPk, pl->k, pl->k, X, kp, X, kp, R, 1, st));
            }
        }
    }
    KIFMM_HIP(mark(KIFMM_STAGE_L2L, 1));
    KIFMM_HIP(mark(KIFMM_STAGE_L2P, 0));
    // L2P: the T~ product and the far field at the points in one launch when
    // the fused kernel exists for this plan (else the product into E, then the
    // far-field evaluation)
    const bool fl2p = far && pl->fuse_l2p;
    auto l2p = [&]() -> hipError_t {
        if (fl2p)
            return launch_l2p_fused(nleaf, pl->pts, pl->leaf_ptr, pl->leaf_row, adjoint ? pl->SopT : pl->Top, kp, nep,
                                    adjoint ? w.Q : w.P, pl->surf, n_eq, 1.0 / kFourPi, pl->perm, out, st);
        return launch_eval_targets(2, elt, R, nleaf, pl->pts, pl->qpts, w.sig_s, pl->leaf_ptr, pl->near_ptr,
                                   pl->near_leaf, pl->near_code, lev, lsc, w.E, pl->surf, n_eq, nep, near_scale,
                                   1.0 / kFourPi, pl->perm, out, ld, nrhs, st);
    };
    if (far) {
        if (!fl2p) {
            if (!adjoint)
                KIFMM_HIP(launch_gg(pl->d_leafdown, elt, pl->Top, MBe, KPk, n_eq, pl->k, w.P, kp, w.E, nep, R, 0, st));
            else
                KIFMM_HIP(launch_gg(pl->d_leafdown, elt, pl->SopT, MBe, KPk, n_eq, pl->k, w.Q, kp, w.E, nep, R, 0, st));
        }
        if (fork) {
            // far field at the points (L2T), added to the near field
            KIFMM_HIP(hipStreamWaitEvent(st, pl->ev_join, 0));
            KIFMM_HIP(l2p());
            KIFMM_HIP(m2t_eval());
        }
    }
    KIFMM_HIP(mark(KIFMM_STAGE_L2P, 1));
    if (!fork) {
        KIFMM_HIP(mark(KIFMM_STAGE_P2P, 0));
        if (bem) {
            // BEM: the near-field integrals, then the far field added
            KIFMM_HIP(launch_eval_near_bem(elt, pl->layer, nleaf, pl->pts, pl->bem_tri, w.sig_s, pl->leaf_ptr,
                                           pl->near_ptr, pl->near_leaf, pl->near_code, bem_scale, pl->perm, out, st));
            if (far) KIFMM_HIP(l2p());
        } else if (fl2p) {
            // the near field, then the fused L2P added
            KIFMM_HIP(launch_eval_targets(1, elt, R, nleaf, pl->pts, pl->qpts, w.sig_s, pl->leaf_ptr, pl->near_ptr,
                                          pl->near_leaf, pl->near_code, lev, lsc, nullptr, pl->surf, n_eq, nep,
                                          near_scale, 1.0 / kFourPi, pl->perm, out, ld, nrhs, st));
            KIFMM_HIP(l2p());
        } else {
            // near field and (when there is one) far field in one kernel
            KIFMM_HIP(launch_eval_targets(3, elt, R, nleaf, pl->pts, pl->qpts, w.sig_s, pl->leaf_ptr, pl->near_ptr,
                                          pl->near_leaf, pl->near_code, lev, lsc, far ? w.E : nullptr, pl->surf,
                                          n_eq, nep, near_scale, 1.0 / kFourPi, pl->perm, out, ld, nrhs, st));
        }
        KIFMM_HIP(m2t_eval());
        KIFMM_HIP(mark(KIFMM_STAGE_P2P, 1));
    }
    if (cur != pl->device) KIFMM_HIP(hipSetDevice(cur));
    return KIFMM_OK;
}

// ------------------------------------------------------------ merged groups
// Plans of a group that share device, precision, operators (p, eps, leaf
// size, C_d, pseudo-inverse cutoff, dense), right-hand-side width and have no
// stage 2 run as one merged plan: the cubes, leaves and points of all of them
// numbered one after the other, every stage one launch over all of them (M2M
// and L2L one per level). The per-plan scales travel with the work: the M2L
// chunks carry their own r_l^-1, the leaves their near-field scale (the
// adaptive form of the evaluation kernels, which the merged plan always uses).
bool fusable(const std::vector<kifmm_plan_t>& ps) {
    if (ps.size() < 2 || ps.size() > (size_t)kMaxSegments) return false;
    const kifmm_plan_s* a = ps[0];
    for (const kifmm_plan_s* b : ps) {
        if (b->device != a->device || b->opts.precision != a->opts.precision || b->R != a->R || b->st2 ||
            b->p != a->p || b->eps != a->eps || b->leaf_size != a->leaf_size || b->opts.cd != a->opts.cd ||
            b->opts.pinv_rcond != a->opts.pinv_rcond || b->opts.dense_m2l != a->opts.dense_m2l ||
            b->kp != a->kp || b->nep != a->nep || b->profiling || b->layer >= 0)
            return false;
    }
    return true;
}

// Appends src's tiles and chunks to dst, target rows shifted by tgt_off and
// source rows by src_off.
void append_sched(GGSched& dst, const GGSched& src, int64_t tgt_off, int64_t src_off) {
    if (src.n_tiles() == 0) return;
    if (dst.tile_chunk0.empty()) dst.tile_chunk0.push_back(0);
    const int32_t base = (int32_t)dst.chunk_cls.size();
    for (int t = 0; t < src.n_tiles(); ++t) {
        dst.tile_tgt0.push_back((int32_t)(src.tile_tgt0[t] + tgt_off));
        dst.tile_ntgt.push_back(src.tile_ntgt[t]);
        dst.tile_chunk0.push_back(base + src.tile_chunk0[t + 1]);
    }
    dst.chunk_cls.insert(dst.chunk_cls.end(), src.chunk_cls.begin(), src.chunk_cls.end());
    dst.chunk_next.insert(dst.chunk_next.end(), src.chunk_next.begin(), src.chunk_next.end());
    dst.chunk_nblk.insert(dst.chunk_nblk.end(), src.chunk_nblk.begin(), src.chunk_nblk.end());
    dst.chunk_scale.insert(dst.chunk_scale.end(), src.chunk_scale.begin(), src.chunk_scale.end());
    dst.chunk_col.insert(dst.chunk_col.end(), src.chunk_col.begin(), src.chunk_col.end());
    for (int32_t v : src.chunk_src) dst.chunk_src.push_back(v < 0 ? v : (int32_t)(v + src_off));
    dst.max_tile = std::max(dst.max_tile, src.max_tile);
    dst.pairs += src.pairs;
    dst.variant = src.variant;
}

void destroy_fused(kifmm_group_s* g) {
    if (!g->fused) return;
    release_streams(g->fused);
    release_device(g->fused);
    delete g->fused;
    g->fused = nullptr;
}

template <typename T>
int build_fused_t(kifmm_group_s* g) {
    const std::vector<kifmm_plan_t>& ps = g->plans;
    const kifmm_plan_s* p0 = ps[0];
    const int np = (int)ps.size();
    kifmm_plan_s* fp = new (std::nothrow) kifmm_plan_s();
    if (!fp) return fail(KIFMM_ENOMEM, "host allocation failed");
    g->fused = fp;
    fp->opts = p0->opts;
    fp->p = p0->p;
    fp->eps = p0->eps;
    fp->leaf_size = p0->leaf_size;
    fp->ops_sp = p0->ops_sp;
    fp->k = p0->k;
    fp->kp = p0->kp;
    fp->nep = p0->nep;
    fp->R = p0->R;
    fp->elt = p0->elt;
    fp->b3 = p0->b3;
    fp->device = p0->device;
    fp->num_cu = p0->num_cu;
    fp->tables = p0->tables;
    fp->Kt = p0->Kt; fp->KtT = p0->KtT; fp->Mt = p0->Mt; fp->MtT = p0->MtT; fp->Lt = p0->Lt; fp->LtT = p0->LtT;
    fp->Sop = p0->Sop; fp->SopT = p0->SopT; fp->Top = p0->Top; fp->TopT = p0->TopT;
    fp->surf = p0->surf; fp->Ut = p0->Ut; fp->UtT = p0->UtT; fp->surf_in = p0->surf_in;
    // offsets of every plan's points, leaves, cubes, W cubes and near entries
    std::vector<int64_t> pt(np + 1, 0), lf(np + 1, 0), bx(np + 1, 0), wc(np + 1, 0), ne(np + 1, 0);
    int D = 0;
    for (int i = 0; i < np; ++i) {
        const HostTree& t = ps[i]->tree;
        pt[i + 1] = pt[i] + t.n;
        lf[i + 1] = lf[i] + t.n_leaf();
        bx[i + 1] = bx[i] + t.n_box();
        wc[i + 1] = wc[i] + (int64_t)ps[i]->w_cube_box.size();
        ne[i + 1] = ne[i] + (int64_t)t.near_leaf.size();
        D = std::max(D, t.depth);
    }
    if (pt[np] > INT32_MAX / 2 || bx[np] > INT32_MAX / 2 || ne[np] > INT32_MAX / 2)
        return fail(KIFMM_EINVAL, "the plans of the group are too large to merge");
    g->pt_off = pt;
    HostTree& U = fp->tree;
    U.adaptive = true;
    U.depth = D;
    U.n = pt[np];
    U.r0 = 1.0;
    U.level_begin.assign(D + 2, 0);
    U.level_begin[D + 1] = bx[np];
    U.leaf_ptr.assign(1, 0);
    for (int i = 0; i < np; ++i) {
        const HostTree& t = ps[i]->tree;
        for (int64_t e = 1; e <= t.n_leaf(); ++e) U.leaf_ptr.push_back((int32_t)(t.leaf_ptr[e] + pt[i]));
    }
    // schedules
    const int cp = 32 / fp->R;
    for (GGSched* s : {&fp->h_leafup, &fp->h_leafdown, &fp->h_m2l, &fp->h_m2t, &fp->h_s2l}) {
        *s = GGSched();
        s->cp = cp;
        s->rhs = fp->R;
    }
    fp->h_up.assign(D + 1, GGSched());
    fp->h_down.assign(D + 1, GGSched());
    for (auto* v : {&fp->h_up, &fp->h_down})
        for (auto& s : *v) {
            s.cp = cp;
            s.rhs = fp->R;
        }
    const int variant = p0->h_m2l.variant;
    int64_t nb2 = 0;
    for (int i = 0; i < np; ++i) {
        const HostTree& t = ps[i]->tree;
        if (t.depth >= 2) nb2 += t.n_box() - t.level_begin[2];
    }
    const int n_rg = row_groups(fp->kp, variant);
    const int slots = std::max(1, fp->num_cu * gg_variant_wgs_per_cu(variant) / n_rg);
    const int cap = max_tile_for(p0, variant, fp->kp);
    int rounds = 1;
    while ((int64_t)rounds * slots * cap < nb2 * 11 / 10) ++rounds;
    const int64_t tiles = (int64_t)rounds * slots;
    for (int i = 0; i < np; ++i) {
        const kifmm_plan_s* m = ps[i];
        const HostTree& t = m->tree;
        if (t.depth < 2) continue;
        append_sched(fp->h_leafup, m->h_leafup, bx[i], lf[i]);
        append_sched(fp->h_leafdown, m->h_leafdown, lf[i], bx[i]);
        for (int l = 0; l <= t.depth; ++l) {
            append_sched(fp->h_up[l], m->h_up[l], bx[i], bx[i]);
            append_sched(fp->h_down[l], m->h_down[l], bx[i], bx[i]);
        }
        const int64_t nbi = t.n_box() - t.level_begin[2];
        const int ti = (int)std::max<int64_t>(1, (tiles * nbi + nb2 / 2) / std::max<int64_t>(1, nb2));
        append_sched(fp->h_m2l, build_m2l_sched(m, variant, ti, 0), bx[i], bx[i]);
        append_sched(fp->h_m2t, m->h_m2t, wc[i], bx[i]);
        append_sched(fp->h_s2l, m->h_s2l, wc[i], wc[i]);
        for (int32_t b : m->w_cube_box) fp->w_cube_box.push_back((int32_t)(b + bx[i]));
    }
    // host lists
    std::vector<int32_t> perm, near_ptr(1, 0), near_leaf, near_code, level, mleaf, mptr(1, 0), mcube, sptr(1, 0), sleaf;
    std::vector<T> scale, mgeo, sgeo;
    for (int i = 0; i < np; ++i) {
        const kifmm_plan_s* m = ps[i];
        const HostTree& t = m->tree;
        for (int32_t v : t.perm) perm.push_back((int32_t)(v + pt[i]));
        for (int64_t e = 1; e <= t.n_leaf(); ++e) near_ptr.push_back((int32_t)(t.near_ptr[e] + ne[i]));
        for (int32_t v : t.near_leaf) near_leaf.push_back((int32_t)(v + lf[i]));
        for (int32_t c : t.near_code) {
            if (t.adaptive) {
                near_code.push_back(c);
            } else {
                // uniform code of d = target - source cube; adaptive form o = -2 d
                const int dx = c / 9 - 1, dy = (c / 3) % 3 - 1, dz = c % 3 - 1;
                near_code.push_back((4 - 2 * dx) * 81 + (4 - 2 * dy) * 9 + (4 - 2 * dz));
            }
        }
        const AdaptiveLists<T> a = adaptive_lists<T>(m);
        level.insert(level.end(), a.level.begin(), a.level.end());
        scale.insert(scale.end(), a.scale.begin(), a.scale.end());
        const int32_t m0 = (int32_t)mcube.size(), s0 = (int32_t)sleaf.size();
        for (int32_t v : a.mleaf) mleaf.push_back((int32_t)(v + lf[i]));
        for (size_t k = 1; k < a.mptr.size(); ++k) mptr.push_back(a.mptr[k] + m0);
        for (int32_t v : a.mcube) mcube.push_back((int32_t)(v + wc[i]));
        mgeo.insert(mgeo.end(), a.mgeo.begin(), a.mgeo.end());
        if (t.adaptive && !m->w_cube_box.empty())
            for (size_t k = 1; k < a.sptr.size(); ++k) sptr.push_back(a.sptr[k] + s0);
        for (int32_t v : a.sleaf) sleaf.push_back((int32_t)(v + lf[i]));
        sgeo.insert(sgeo.end(), a.sgeo.begin(), a.sgeo.end());
    }
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(fp->device);
    Uploader up{fp, 0};
    fp->perm = (int32_t*)up.put(perm);
    fp->leaf_ptr = (int32_t*)up.put(U.leaf_ptr);
    fp->near_ptr = (int32_t*)up.put(near_ptr);
    fp->near_leaf = (int32_t*)up.put(near_leaf);
    fp->near_code = (int32_t*)up.put(near_code);
    fp->leaf_level = (int32_t*)up.put(level);
    fp->leaf_scale = up.put(scale);
    fp->pts = up.alloc((size_t)pt[np] * 4 * sizeof(T));
    if (fp->elt == 4) fp->qpts = up.alloc((size_t)pt[np] * 4 * sizeof(int32_t));
    for (int i = 0; i < np && up.err == KIFMM_OK; ++i) {
        const size_t n = (size_t)ps[i]->tree.n;
        hipError_t e = hipMemcpy(static_cast<char*>(fp->pts) + (size_t)pt[i] * 4 * sizeof(T), ps[i]->pts,
                                 n * 4 * sizeof(T), hipMemcpyDeviceToDevice);
        if (e == hipSuccess && fp->qpts)
            e = hipMemcpy(static_cast<char*>(fp->qpts) + (size_t)pt[i] * 4 * sizeof(int32_t), ps[i]->qpts,
                          n * 4 * sizeof(int32_t), hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {
            up.err = KIFMM_EHIP;
            up.msg = std::string("hipMemcpy (merging the group's points): ") + hipGetErrorString(e);
        }
    }
    const size_t elt = fp->elt, R = fp->R;
    fp->sig_s = up.zeros((size_t)pt[np] * R * elt);
    if (D >= 2) {
        fp->C = up.zeros((size_t)lf[np] * R * fp->nep * elt);
        fp->E = up.zeros((size_t)lf[np] * R * fp->nep * elt);
        fp->Q = up.zeros((size_t)bx[np] * R * fp->kp * elt);
        fp->P = up.zeros((size_t)bx[np] * R * fp->kp * elt);
    }
    fp->d_leafup = upload_sched(up, fp->h_leafup, fp->elt);
    fp->d_leafdown = upload_sched(up, fp->h_leafdown, fp->elt);
    fp->d_m2l = upload_sched(up, fp->h_m2l, fp->elt);
    fp->d_up.resize(D + 1);
    fp->d_down.resize(D + 1);
    for (int l = 0; l <= D; ++l) {
        fp->d_up[l] = upload_sched(up, fp->h_up[l], fp->elt);
        fp->d_down[l] = upload_sched(up, fp->h_down[l], fp->elt);
    }
    if (!fp->w_cube_box.empty()) {
        fp->n_m2t_leaf = (int64_t)mleaf.size();
        fp->m2t_leaf = (int32_t*)up.put(mleaf);
        fp->m2t_ptr = (int32_t*)up.put(mptr);
        fp->m2t_cube = (int32_t*)up.put(mcube);
        fp->m2t_geo = up.put(mgeo);
        fp->s2l_ptr = (int32_t*)up.put(sptr);
        fp->s2l_leaf = (int32_t*)up.put(sleaf);
        fp->s2l_geo = up.put(sgeo);
        fp->d_m2t = upload_sched(up, fp->h_m2t, fp->elt);
        fp->d_s2l = upload_sched(up, fp->h_s2l, fp->elt, &fp->w_cube_box);
        fp->CX = up.zeros(fp->w_cube_box.size() * R * fp->nep * elt);
        fp->Psi = up.zeros(fp->w_cube_box.size() * R * fp->nep * elt);
    }
    if (D >= 2) {
        std::vector<int32_t> rows;
        for (int i = 0; i < np; ++i) {
            const HostTree& t = ps[i]->tree;
            for (int64_t e = 0; e < t.n_leaf(); ++e) {
                int64_t r = -1;
                if (t.depth >= 2) r = t.adaptive ? (t.leaf_level[e] >= 2 ? t.leaf_box[e] : -1) : t.level_begin[t.depth] + e;
                rows.push_back(r < 0 ? -1 : (int32_t)(r + bx[i]));
            }
        }
        fp->leaf_row = (int32_t*)up.put(rows);
        const bool ok = fp->elt == 4 && fp->R == 1 && p0->opts.fused_leaf;
        fp->fuse_s2m = ok && (p0->opts.fused_leaf & 1) && s2m_fused_supported(fp->nep, fp->kp);
        fp->fuse_l2p = ok && (p0->opts.fused_leaf & 2) && l2p_fused_supported(fp->nep, fp->kp);
    }
    if (D >= 3 && fp->elt == 4 && fp->R == 1 && p0->opts.direct_passes && m2m_direct_supported(fp->kp)) {
        std::vector<std::vector<int32_t>> par(D), ch(D);
        for (int i = 0; i < np; ++i)
            for (int l = 2; l < std::min(D, ps[i]->tree.depth); ++l)
                m2m_lists(ps[i]->tree, l, (int32_t)bx[i], par[l], ch[l]);
        upload_m2m(fp, up, par, ch);
        std::vector<std::vector<DownItem>> dn(D + 1);
        for (int i = 0; i < np; ++i)
            for (int l = 3; l <= ps[i]->tree.depth; ++l) down_items(ps[i]->tree, l, (int32_t)bx[i], dn[l]);
        upload_down(fp, up, dn);
    }
    g->sig_u = up.zeros((size_t)pt[np] * elt);
    g->out_u = up.zeros((size_t)pt[np] * elt);
    if (up.err == KIFMM_OK &&
        (hipStreamCreateWithFlags(&fp->near_stream, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&fp->ev_fork, hipEventDisableTiming) != hipSuccess ||
         hipEventCreateWithFlags(&fp->ev_join, hipEventDisableTiming) != hipSuccess)) {
        up.err = KIFMM_EHIP;
        up.msg = "creating the merged plan's stream or events failed";
    }
    hipDeviceSynchronize();
    hipSetDevice(cur);
    if (up.err != KIFMM_OK) return fail(up.err, up.msg);
    fp->on_device = true;
    return KIFMM_OK;
}

int collect_profile(kifmm_plan_s* pl) {
    for (auto& a : pl->prof_events) {
        for (int s = 0; s < KIFMM_STAGE_COUNT; ++s) {
            float ms = 0.f;
            KIFMM_HIP(hipEventSynchronize(a[2 * s + 1]));
            KIFMM_HIP(hipEventElapsedTime(&ms, a[2 * s], a[2 * s + 1]));
            pl->prof_ms[s] += ms;
        }
        pl->prof_calls++;
        pl->prof_free.push_back(a);
    }
    pl->prof_events.clear();
    return KIFMM_OK;
}

void destroy_profile_events(kifmm_plan_s* pl) {
    for (auto& a : pl->prof_events)
        for (auto e : a) (void)hipEventDestroy(e);
    for (auto& a : pl->prof_free)
        for (auto e : a) (void)hipEventDestroy(e);
    pl->prof_events.clear();
    pl->prof_free.clear();
}

}  // namespace

extern "C" {

}  // extern "C"

namespace kifmm {
int solve_fail(int code, const std::string& msg) { return fail(code, msg); }
// element bytes of a plan that can be applied (and its point count), or an error code
int plan_precision_bytes(kifmm_plan_t plan, int64_t* n) {
    const int rc = check_plan_for_apply(plan);
    if (rc) return rc;
    *n = plan->tree.n;
    return plan->elt;
}
}  // namespace kifmm

extern "C" {

int kifmm_opts_default(kifmm_opts_t* o) {
    if (!o) return fail(KIFMM_EINVAL, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->precision = KIFMM_FP32;
    o->cd = 0.5;
    o->pinv_rcond = 1e-10;
    o->depth = 0;
    o->max_depth = 16;
    o->dense_m2l = 0;
    o->max_nrhs = 1;
    o->device = 0;
    o->mem_limit = 0;
    o->tile_targets = 0;
    o->m2l_shape = -1;
    o->fused_leaf = 3;
    o->direct_passes = 1;
    o->near_overlap = 1;
    return KIFMM_OK;
}

int kifmm_plan(const double* points, int64_t n, int p, double eps, int leaf_size, kifmm_plan_t* out) {
    return kifmm_plan_ex(points, n, p, eps, leaf_size, nullptr, out);
}

static int plan_build(const double* points, int64_t n, int p, double eps, int leaf_size, const kifmm_opts_t* opts,
                      const BemMesh* bem, int layer, kifmm_plan_t* out) {
    g_last_error.clear();
    if (!out) return fail(KIFMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!points) return fail(KIFMM_EINVAL, "points is NULL");
    kifmm_opts_t o;
    kifmm_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision != KIFMM_FP64 && o.precision != KIFMM_FP32 && o.precision != KIFMM_BF16X3)
        return fail(KIFMM_EINVAL, "unknown precision");
    if (o.max_nrhs < 1 || o.max_nrhs > 16) return fail(KIFMM_EINVAL, "max_nrhs must be in [1, 16]");
    if (o.tile_targets < 0 || o.tile_targets > 4096) return fail(KIFMM_EINVAL, "tile_targets must be in [0, 4096]");
    if (o.device < -1) return fail(KIFMM_EINVAL, "device must be >= -1");
    if (o.m2l_shape < -1 || o.m2l_shape >= kGGVariants)
        return fail(KIFMM_EINVAL, "m2l_shape must be -1 or in [0, " + std::to_string(kGGVariants - 1) + "]");
    if (o.m2l_shape >= 0 && !gg_variant_supported(o.m2l_shape, o.precision == KIFMM_FP64 ? 8 : 4, 1))
        return fail(KIFMM_EINVAL, "m2l_shape " + std::to_string(o.m2l_shape) + " is not available in this precision");
    if (!(o.c2 >= 0.0) || !std::isfinite(o.c2)) return fail(KIFMM_EINVAL, "c2 must be finite and >= 0");
    if (o.c2 > 0.0 && (o.dense_m2l || o.precision == KIFMM_BF16X3))
        return fail(KIFMM_EINVAL, "c2 > 0 (stage-2 low rank) needs compressed operators in FP32 or FP64");
    if (o.adaptive != 0 && o.adaptive != 1) return fail(KIFMM_EINVAL, "adaptive must be 0 or 1");
    if (o.fused_leaf < 0 || o.fused_leaf > 3) return fail(KIFMM_EINVAL, "fused_leaf must be in [0, 3]");
    if (o.direct_passes != 0 && o.direct_passes != 1) return fail(KIFMM_EINVAL, "direct_passes must be 0 or 1");
    if (o.near_overlap != 0 && o.near_overlap != 1) return fail(KIFMM_EINVAL, "near_overlap must be 0 or 1");
    if (o.adaptive && o.depth > 0) return fail(KIFMM_EINVAL, "adaptive trees take no forced depth (opts.depth)");
    if (bem && (o.adaptive || o.max_nrhs != 1))
        return fail(KIFMM_EINVAL, "BEM plans take uniform trees and one right-hand side (adaptive = 0, max_nrhs = 1)");
    const auto t0 = std::chrono::steady_clock::now();
    kifmm_plan_s* pl = new (std::nothrow) kifmm_plan_s();
    if (!pl) return fail(KIFMM_ENOMEM, "host allocation failed");
    pl->opts = o;
    pl->p = p;
    pl->eps = eps;
    pl->leaf_size = leaf_size;
    pl->elt = o.precision == KIFMM_FP64 ? 8 : 4;
    pl->b3 = o.precision == KIFMM_BF16X3;
    pl->layer = bem ? layer : -1;
    pl->R = 1;
    while (pl->R < o.max_nrhs) pl->R <<= 1;
    try {
        if (p < 2 || p > 16) throw PlanError{KIFMM_EINVAL, "p must be in [2, 16]"};
        if (!(eps >= 0.0 && eps < 1.0)) throw PlanError{KIFMM_EINVAL, "eps must be in [0, 1)"};
        pl->tree = o.adaptive ? build_adaptive_host_tree(points, n, leaf_size, o.max_depth)
                              : build_host_tree(points, n, leaf_size, o.depth, o.max_depth);
        pl->ops_sp = host_ops_shared(p, eps, leaf_size, o.cd, o.pinv_rcond, o.dense_m2l != 0, o.c2);
    } catch (const PlanError& e) {
        delete pl;
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        delete pl;
        return fail(KIFMM_ENOMEM, "host allocation failed");
    }
    {
        // the near-field kernel takes at most 64 entries per leaf (27 in a
        // uniform tree, 57 in a 2:1-balanced one)
        const HostTree& t = pl->tree;
        for (int64_t e = 0; e < t.n_leaf(); ++e)
            if (t.near_ptr[e + 1] - t.near_ptr[e] > 64) {
                delete pl;
                return fail(KIFMM_EINVAL, "internal: a leaf has more than 64 near-field leaves");
            }
    }
    pl->k = pl->ops().k;
    pl->st2 = o.c2 > 0.0;
    pl->rp = pl->st2 ? (pl->ops().r2max + 15) / 16 * 16 : 0;
    // split-BF16 M2L works on 32-wide K-chunks
    pl->kp = pl->b3 ? (pl->k + 31) / 32 * 32 : (pl->k + 15) / 16 * 16;
    pl->nep = (pl->ops().n_eq + 15) / 16 * 16;
    if (pl->kp > 19 * 16 || pl->nep > 19 * 16) {
        delete pl;
        return fail(KIFMM_EINVAL, "n_eq too large for the device kernels (p <= 8 supported)");
    }
    if (o.m2l_shape >= 0 && !gg_variant_supported(o.m2l_shape, pl->elt, pl->kp / 16)) {
        delete pl;
        return fail(KIFMM_EINVAL, "m2l_shape " + std::to_string(o.m2l_shape) +
                                      " does not support the compressed dimension " + std::to_string(pl->kp));
    }
    if (o.device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || o.device >= ndev) {
            delete pl;
            return fail(KIFMM_EHIP, "HIP device " + std::to_string(o.device) + " not available");
        }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, o.device) == hipSuccess && ncu > 0)
            pl->num_cu = ncu;
    }
    build_schedules(pl, o.tile_targets, std::max(o.m2l_shape, 0));
    if (o.device >= 0) {
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(o.device);
        pl->device = o.device;
        Uploader up{pl, o.mem_limit};
        const HostTree& t = pl->tree;
        pl->perm = (int32_t*)up.put(t.perm);
        pl->leaf_ptr = (int32_t*)up.put(t.leaf_ptr);
        pl->near_ptr = (int32_t*)up.put(t.near_ptr);
        pl->near_leaf = (int32_t*)up.put(t.near_leaf);
        pl->near_code = (int32_t*)up.put(t.near_code);
        if (pl->elt == 4)
            upload_tables<float>(pl, up);
        else
            upload_tables<double>(pl, up);
        const size_t elt = pl->elt, R = pl->R;
        pl->sig_s = up.zeros((size_t)t.n * R * elt);
        if (t.depth >= 2) {
            pl->C = up.zeros((size_t)t.n_leaf() * R * pl->nep * elt);
            pl->E = up.zeros((size_t)t.n_leaf() * R * pl->nep * elt);
            pl->Q = up.zeros((size_t)t.n_box() * R * pl->kp * elt);
            pl->P = up.zeros((size_t)t.n_box() * R * pl->kp * elt);
        }
        pl->d_leafup = upload_sched(up, pl->h_leafup, pl->elt);
        pl->d_leafdown = upload_sched(up, pl->h_leafdown, pl->elt);
        const bool tune = o.tile_targets == 0 && t.depth >= 2;
        if (!tune) pl->d_m2l = upload_sched(up, pl->h_m2l, pl->elt);
        pl->d_up.resize(pl->h_up.size());
        pl->d_down.resize(pl->h_down.size());
        for (size_t l = 0; l < pl->h_up.size(); ++l) pl->d_up[l] = upload_sched(up, pl->h_up[l], pl->elt);
        for (size_t l = 0; l < pl->h_down.size(); ++l) pl->d_down[l] = upload_sched(up, pl->h_down[l], pl->elt);
        if (up.err == KIFMM_OK && tune) autotune_m2l(pl, up);
        if (up.err == KIFMM_OK && pl->st2 && t.depth >= 2) upload_stage2(pl, up);
        if (up.err == KIFMM_OK && t.adaptive) {
            if (pl->elt == 4)
                upload_adaptive<float>(pl, up);
            else
                upload_adaptive<double>(pl, up);
        }
        if (up.err == KIFMM_OK && bem) {
            if (pl->elt == 4)
                upload_bem<float>(pl, up, *bem);
            else
                upload_bem<double>(pl, up, *bem);
        }
        if (up.err == KIFMM_OK && t.depth >= 2) {
            // the Q/P row of every leaf for the fused leaf kernels
            std::vector<int32_t> rows(t.n_leaf());
            for (int64_t e = 0; e < t.n_leaf(); ++e)
                rows[e] = t.adaptive ? (t.leaf_level[e] >= 2 ? t.leaf_box[e] : -1)
                                     : (int32_t)(t.level_begin[t.depth] + e);
            pl->leaf_row = (int32_t*)up.put(rows);
            const bool ok = pl->elt == 4 && pl->R == 1 && o.fused_leaf;
            pl->fuse_s2m = ok && (o.fused_leaf & 1) && !bem && s2m_fused_supported(pl->nep, pl->kp);
            pl->fuse_l2p = ok && (o.fused_leaf & 2) && l2p_fused_supported(pl->nep, pl->kp);
            // not for stage-2 plans: beside their two M2L phases the near field
            // costs more than it hides (measured 2.14 -> 2.21 ms at C2 = 10)
            pl->near_late = o.near_overlap && pl->elt == 4 && pl->R == 1 && !bem && !t.adaptive && !pl->st2;
        }
        if (up.err == KIFMM_OK && t.depth >= 3 && pl->elt == 4 && pl->R == 1 && o.direct_passes &&
            m2m_direct_supported(pl->kp)) {
            std::vector<std::vector<int32_t>> par(t.depth), ch(t.depth);
            for (int l = 2; l < t.depth; ++l) m2m_lists(t, l, 0, par[l], ch[l]);
            upload_m2m(pl, up, par, ch);
            std::vector<std::vector<DownItem>> dn(t.depth + 1);
            for (int l = 3; l <= t.depth; ++l) down_items(t, l, 0, dn[l]);
            upload_down(pl, up, dn);
        }
        if (up.err == KIFMM_OK &&
            (hipStreamCreateWithFlags(&pl->near_stream, hipStreamNonBlocking) != hipSuccess ||
             hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming) != hipSuccess)) {
            up.err = KIFMM_EHIP;
            up.msg = "creating the near-field stream or its events failed";
        }
        hipDeviceSynchronize();
        hipSetDevice(cur);
        if (up.err != KIFMM_OK) {
            int code = up.err;
            std::string msg = up.msg;
            release_streams(pl);
            release_device(pl);
            delete pl;
            return fail(code, msg);
        }
        pl->on_device = true;
        // the static workspace of kifmm_apply_noalloc on this device
        int cur2 = 0;
        hipGetDevice(&cur2);
        hipSetDevice(o.device);
        void* sp = nullptr;
        const int src = scratch_address(o.device, &sp);
        hipSetDevice(cur2);
        if (src != KIFMM_OK) {
            const std::string msg = g_last_error;
            kifmm_destroy(pl);
            return fail(src, msg);
        }
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(pl, secs);
    *out = pl;
    return KIFMM_OK;
}

int kifmm_plan_ex(const double* points, int64_t n, int p, double eps, int leaf_size, const kifmm_opts_t* opts,
                  kifmm_plan_t* out) {
    return plan_build(points, n, p, eps, leaf_size, opts, nullptr, -1, out);
}

int kifmm_plan_bem(const double* vertices, int64_t n_vertices, const int32_t* triangles, int64_t n_triangles,
                   int layer, int p, double eps, int leaf_size, const kifmm_opts_t* opts, kifmm_plan_t* out) {
    g_last_error.clear();
    if (!out) return fail(KIFMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!vertices || !triangles) return fail(KIFMM_EINVAL, "vertices and triangles must be non-NULL");
    if (layer != KIFMM_SINGLE_LAYER && layer != KIFMM_DOUBLE_LAYER) return fail(KIFMM_EINVAL, "unknown layer");
    if (n_vertices < 3 || n_triangles < 1 || n_triangles > (int64_t)INT32_MAX / 2)
        return fail(KIFMM_EINVAL, "need at least 3 vertices and 1 triangle");
    BemMesh m;
    try {
        m.verts.assign(vertices, vertices + 3 * n_vertices);
        m.tris.assign(triangles, triangles + 3 * n_triangles);
    } catch (const std::bad_alloc&) {
        return fail(KIFMM_ENOMEM, "host allocation failed");
    }
    for (double v : m.verts)
        if (!std::isfinite(v)) return fail(KIFMM_ENONFINITE, "non-finite vertex coordinate");
    std::vector<double> cen(3 * (size_t)n_triangles);
    for (int64_t j = 0; j < n_triangles; ++j) {
        const int32_t* f = &m.tris[3 * (size_t)j];
        for (int k = 0; k < 3; ++k)
            if (f[k] < 0 || f[k] >= n_vertices)
                return fail(KIFMM_EINVAL, "triangle " + std::to_string(j) + " has a vertex index out of range");
        double e1[3], e2[3];
        for (int a = 0; a < 3; ++a) {
            const double v0 = m.verts[3 * (size_t)f[0] + a];
            e1[a] = m.verts[3 * (size_t)f[1] + a] - v0;
            e2[a] = m.verts[3 * (size_t)f[2] + a] - v0;
            cen[3 * (size_t)j + a] = (v0 + m.verts[3 * (size_t)f[1] + a] + m.verts[3 * (size_t)f[2] + a]) / 3.0;
        }
        const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                     cz = e1[0] * e2[1] - e1[1] * e2[0];
        if (!(cx * cx + cy * cy + cz * cz > 0.0))
            return fail(KIFMM_EINVAL, "triangle " + std::to_string(j) + " has zero area");
    }
    return plan_build(cen.data(), n_triangles, p, eps, leaf_size, opts, &m, layer, out);
}

int kifmm_apply(kifmm_plan_t plan, const void* sigma, void* phi, void* stream) {
    int rc = check_plan_for_apply(plan);
    if (rc) return rc;
    if (!sigma || !phi) return fail(KIFMM_EINVAL, "sigma and phi must be non-NULL");
    if (sigma == phi) return fail(KIFMM_EINVAL, "sigma and phi must not alias");
    return run_passes(plan, plan_work(plan), sigma, phi, 1, plan->tree.n, false, (hipStream_t)stream);
}

int kifmm_apply_noalloc(kifmm_plan_t plan, const void* sigma, void* phi, void* stream) {
    int rc = check_plan_for_apply(plan);
    if (rc) return rc;
    if (!sigma || !phi) return fail(KIFMM_EINVAL, "sigma and phi must be non-NULL");
    if (sigma == phi) return fail(KIFMM_EINVAL, "sigma and phi must not alias");
    if (plan->st2)
        return fail(KIFMM_EINVAL, "stage-2 plans (c2 > 0) keep per-pair products that must start at zero: use kifmm_apply");
    if (plan->profiling) return fail(KIFMM_ESTATE, "profiled applies create timing events: use kifmm_apply");
    const size_t need = carve_work(plan, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(KIFMM_EINVAL, "the plan's workspace (" + std::to_string(need) + " bytes) exceeds the " +
                                      std::to_string(kScratchBytes) + "-byte static workspace of kifmm_apply_noalloc");
    int cur = 0;
    KIFMM_HIP(hipGetDevice(&cur));
    if (cur != plan->device) KIFMM_HIP(hipSetDevice(plan->device));
    void* base = nullptr;
    rc = scratch_address(plan->device, &base);
    if (cur != plan->device) KIFMM_HIP(hipSetDevice(cur));
    if (rc) return rc;
    Work w;
    carve_work(plan, static_cast<char*>(base), &w);
    return run_passes(plan, w, sigma, phi, 1, plan->tree.n, false, (hipStream_t)stream);
}

int kifmm_apply_adjoint(kifmm_plan_t plan, const void* g, void* out, void* stream) {
    int rc = check_plan_for_apply(plan);
    if (rc) return rc;
    if (!g || !out) return fail(KIFMM_EINVAL, "g and out must be non-NULL");
    if (g == out) return fail(KIFMM_EINVAL, "g and out must not alias");
    return run_passes(plan, plan_work(plan), g, out, 1, plan->tree.n, true, (hipStream_t)stream);
}

int kifmm_apply_batched(kifmm_plan_t plan, const void* sigma, void* phi, int nrhs, int64_t ld, void* stream) {
    int rc = check_plan_for_apply(plan);
    if (rc) return rc;
    if (!sigma || !phi) return fail(KIFMM_EINVAL, "sigma and phi must be non-NULL");
    if (sigma == phi) return fail(KIFMM_EINVAL, "sigma and phi must not alias");
    if (nrhs < 1 || nrhs > plan->opts.max_nrhs)
        return fail(KIFMM_EINVAL, "nrhs must be in [1, opts.max_nrhs] (" + std::to_string(plan->opts.max_nrhs) + ")");
    if (ld < plan->tree.n) return fail(KIFMM_EINVAL, "ld must be >= n");
    return run_passes(plan, plan_work(plan), sigma, phi, nrhs, ld, false, (hipStream_t)stream);
}

int kifmm_plan_info(kifmm_plan_t plan, kifmm_info_t* info) {
    if (!plan || !info) return fail(KIFMM_EINVAL, "plan and info must be non-NULL");
    *info = plan->info;
    return KIFMM_OK;
}

int kifmm_plan_export_tree(kifmm_plan_t plan, int32_t* leaf_coords) {
    if (!plan || !leaf_coords) return fail(KIFMM_EINVAL, "plan and leaf_coords must be non-NULL");
    std::memcpy(leaf_coords, plan->tree.leaf_coords.data(), sizeof(int32_t) * 3 * plan->tree.n);
    return KIFMM_OK;
}

int kifmm_plan_export_point_leaves(kifmm_plan_t plan, int32_t* out) {
    if (!plan || !out) return fail(KIFMM_EINVAL, "plan and out must be non-NULL");
    const HostTree& t = plan->tree;
    for (int64_t e = 0; e < t.n_leaf(); ++e) {
        int64_t c[3];
        const int l = box_cube(t, box_of_leaf(t, e), c);
        for (int32_t i = t.leaf_ptr[e]; i < t.leaf_ptr[e + 1]; ++i) {
            int32_t* o = out + 4 * (int64_t)t.perm[i];
            o[0] = l;
            o[1] = (int32_t)c[0];
            o[2] = (int32_t)c[1];
            o[3] = (int32_t)c[2];
        }
    }
    return KIFMM_OK;
}

int kifmm_plan_export_boxes(kifmm_plan_t plan, int32_t* out, int64_t* count) {
    if (!plan || !count) return fail(KIFMM_EINVAL, "plan and count must be non-NULL");
    const HostTree& t = plan->tree;
    *count = t.n_box();
    if (!out) return KIFMM_OK;
    for (int64_t g = 0; g < t.n_box(); ++g) {
        int64_t c[3];
        int32_t* o = out + 5 * g;
        o[0] = box_cube(t, g, c);
        o[1] = (int32_t)c[0];
        o[2] = (int32_t)c[1];
        o[3] = (int32_t)c[2];
        o[4] = (int32_t)leaf_of_box(t, g);
    }
    return KIFMM_OK;
}

int kifmm_plan_export_list(kifmm_plan_t plan, int which, int32_t* out, int64_t* count) {
    if (!plan || !count) return fail(KIFMM_EINVAL, "plan and count must be non-NULL");
    if (which < 0 || which > 3) return fail(KIFMM_EINVAL, "which must be in [0, 3]");
    const HostTree& t = plan->tree;
    // CSR over targets: U and W over leaves, V and X over boxes
    const std::vector<int32_t>* ptr = nullptr;
    const std::vector<int32_t>* src = nullptr;
    bool tgt_leaf = false, src_leaf = false;
    if (which == 0) { ptr = &t.near_ptr; src = &t.near_leaf; tgt_leaf = src_leaf = true; }
    if (which == 1) { ptr = &t.v_ptr; src = &t.v_src; }
    if (which == 2) { ptr = &t.w_ptr; src = &t.w_src; tgt_leaf = true; }
    if (which == 3) { ptr = &t.x_ptr; src = &t.x_src; src_leaf = true; }
    *count = (int64_t)src->size();
    if (!out || src->empty()) return KIFMM_OK;
    int64_t q = 0;
    for (size_t i = 0; i + 1 < ptr->size(); ++i)
        for (int32_t k = (*ptr)[i]; k < (*ptr)[i + 1]; ++k, ++q) {
            out[2 * q] = (int32_t)(tgt_leaf ? box_of_leaf(t, (int64_t)i) : (int64_t)i);
            out[2 * q + 1] = (int32_t)(src_leaf ? box_of_leaf(t, (*src)[k]) : (*src)[k]);
        }
    return KIFMM_OK;
}

int kifmm_plan_export_operator(kifmm_plan_t plan, int which, double* out, int64_t* count) {
    if (!plan) return fail(KIFMM_EINVAL, "plan is NULL");
    const HostOps& o = plan->ops();
    const std::vector<double>* v = nullptr;
    switch (which) {
        case 0: v = &o.sing; break;
        case 1: v = &o.U; break;
        case 2: v = &o.S; break;
        case 3: v = &o.T; break;
        case 4: v = &o.M; break;
        case 5: v = &o.L; break;
        case 6: v = &o.K; break;
        case 8: v = &o.U2; break;
        case 9: v = &o.V2; break;
        case 7: {
            if (o.rank2.empty()) return fail(KIFMM_EINVAL, "operator 7 exists only in stage-2 plans (c2 > 0)");
            if (count) *count = (int64_t)o.rank2.size();
            if (out)
                for (size_t i = 0; i < o.rank2.size(); ++i) out[i] = o.rank2[i];
            return KIFMM_OK;
        }
        default: return fail(KIFMM_EINVAL, "unknown operator id");
    }
    if ((which == 8 || which == 9) && v->empty())
        return fail(KIFMM_EINVAL, "operators 8 and 9 exist only in stage-2 plans (c2 > 0)");
    if (count) *count = (int64_t)v->size();
    if (out) std::memcpy(out, v->data(), sizeof(double) * v->size());
    return KIFMM_OK;
}

int kifmm_profile(kifmm_plan_t plan, int enable) {
    int rc = check_plan_for_apply(plan);
    if (rc) return rc;
    if (!plan->prof_events.empty()) {
        rc = collect_profile(plan);
        if (rc) return rc;
    }
    plan->profiling = enable != 0;
    std::fill(plan->prof_ms, plan->prof_ms + KIFMM_STAGE_COUNT, 0.0);
    plan->prof_calls = 0;
    return KIFMM_OK;
}

int kifmm_profile_read(kifmm_plan_t plan, double* ms, int64_t* calls) {
    int rc = check_plan_for_apply(plan);
    if (rc) return rc;
    if (!ms) return fail(KIFMM_EINVAL, "ms is NULL");
    rc = collect_profile(plan);
    if (rc) return rc;
    std::copy(plan->prof_ms, plan->prof_ms + KIFMM_STAGE_COUNT, ms);
    if (calls) *calls = plan->prof_calls;
    return KIFMM_OK;
}

void kifmm_destroy(kifmm_plan_t plan) {
    if (!plan) return;
    if (plan->on_device) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(plan->device);
        destroy_profile_events(plan);
        release_streams(plan);
        (void)hipSetDevice(cur);
    }
    release_device(plan);
    delete plan;
}

const char* kifmm_last_error(void) { return g_last_error.c_str(); }

int kifmm_group_create(const kifmm_plan_t* plans, int nplans, kifmm_group_t* out) {
    if (!out) return fail(KIFMM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans || nplans < 1) return fail(KIFMM_EINVAL, "need at least one plan");
    for (int i = 0; i < nplans; ++i) {
        int rc = check_plan_for_apply(plans[i]);
        if (rc) return rc;
        if (plans[i]->device != plans[0]->device || plans[i]->opts.precision != plans[0]->opts.precision)
            return fail(KIFMM_EINVAL, "plans of a group must share device and precision");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(KIFMM_EINVAL, "a plan appears twice in the group");
    }
    kifmm_group_s* g = new (std::nothrow) kifmm_group_s();
    if (!g) return fail(KIFMM_ENOMEM, "host allocation failed");
    g->plans.assign(plans, plans + nplans);
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(plans[0]->device);
    bool ok = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess;
    g->side.resize(nplans, nullptr);
    g->join.resize(nplans, nullptr);
    for (int i = 0; ok && i < nplans; ++i) {
        ok = hipStreamCreateWithFlags(&g->side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&g->join[i], hipEventDisableTiming) == hipSuccess;
    }
    hipSetDevice(cur);
    if (!ok) {
        kifmm_group_destroy(g);
        return fail(KIFMM_EHIP, "stream/event creation failed");
    }
    if (fusable(g->plans)) {
        const int rc = g->plans[0]->elt == 4 ? build_fused_t<float>(g) : build_fused_t<double>(g);
        if (rc != KIFMM_OK) {
            const std::string msg = g_last_error;
            kifmm_group_destroy(g);
            return fail(rc, msg);
        }
    }
    *out = g;
    return KIFMM_OK;
}

int kifmm_group_apply(kifmm_group_t g, const void* const* sigma, void* const* phi, void* stream) {
    if (!g || !sigma || !phi) return fail(KIFMM_EINVAL, "group, sigma and phi must be non-NULL");
    const int np = (int)g->plans.size();
    for (int i = 0; i < np; ++i)
        if (!sigma[i] || !phi[i] || sigma[i] == phi[i]) return fail(KIFMM_EINVAL, "bad sigma/phi pointer");
    for (int i = 0; i < np; ++i)
        if (g->plans[i]->profiling)
            return fail(KIFMM_ESTATE, "plan " + std::to_string(i) +
                                          " of the group has profiling on; profiled applies cannot be captured");
    hipStream_t st = (hipStream_t)stream;
    bool same = g->exec != nullptr && g->key_stream == st;
    for (int i = 0; same && i < np; ++i) same = g->key_sigma[i] == sigma[i] && g->key_phi[i] == phi[i];
    int cur = 0;
    KIFMM_HIP(hipGetDevice(&cur));
    KIFMM_HIP(hipSetDevice(g->plans[0]->device));
    if (!same) {
        if (g->exec) hipGraphExecDestroy(g->exec);
        if (g->graph) hipGraphDestroy(g->graph);
        g->exec = nullptr;
        g->graph = nullptr;
        hipStream_t cap = st;
        hipStream_t own = nullptr;
        if (cap == nullptr) {   // the null stream cannot be captured: capture on a private stream
            KIFMM_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
            cap = own;
        }
        KIFMM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        int rc = KIFMM_OK;
        if (g->fused) {
            // the joined input, the merged plan's passes, the joined output split back
            SegTable in{}, outs{};
            in.count = outs.count = np;
            for (int i = 0; i <= np; ++i) in.off[i] = outs.off[i] = g->pt_off[i];
            for (int i = 0; i < np; ++i) {
                in.ptr[i] = sigma[i];
                outs.ptr[i] = phi[i];
            }
            const int64_t n = g->pt_off[np];
            hipError_t e = launch_gather_segments(g->fused->elt, n, in, g->sig_u, cap);
            if (e != hipSuccess) rc = fail(KIFMM_EHIP, std::string("gather launch: ") + hipGetErrorString(e));
            if (rc == KIFMM_OK) rc = run_passes(g->fused, plan_work(g->fused), g->sig_u, g->out_u, 1, n, false, cap);
            if (rc == KIFMM_OK) {
                e = launch_scatter_segments(g->fused->elt, n, outs, g->out_u, cap);
                if (e != hipSuccess) rc = fail(KIFMM_EHIP, std::string("scatter launch: ") + hipGetErrorString(e));
            }
        } else {
            hipEventRecord(g->fork, cap);
            for (int i = 0; i < np && rc == KIFMM_OK; ++i) {
                hipStreamWaitEvent(g->side[i], g->fork, 0);
                rc = run_passes(g->plans[i], plan_work(g->plans[i]), sigma[i], phi[i], 1, g->plans[i]->tree.n, false,
                                g->side[i]);
                hipEventRecord(g->join[i], g->side[i]);
                hipStreamWaitEvent(cap, g->join[i], 0);
            }
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(cap, &graph);
        if (rc != KIFMM_OK || e != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            if (own) hipStreamDestroy(own);
            hipSetDevice(cur);
            return rc != KIFMM_OK ? rc : fail(KIFMM_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
        }
        if (own) hipStreamDestroy(own);
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(graph);
            hipSetDevice(cur);
            return fail(KIFMM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        g->graph = graph;
        g->key_sigma.assign(sigma, sigma + np);
        g->key_phi.assign(phi, phi + np);
        g->key_stream = st;
    }
    KIFMM_HIP(hipGraphLaunch(g->exec, st));
    KIFMM_HIP(hipSetDevice(cur));
    return KIFMM_OK;
}

void kifmm_group_destroy(kifmm_group_t g) {
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    destroy_fused(g);
    for (auto s : g->side)
        if (s) hipStreamDestroy(s);
    for (auto e : g->join)
        if (e) hipEventDestroy(e);
    if (g->fork) hipEventDestroy(g->fork);
    delete g;
}

}  // extern "C"
