// Host-side plan construction: octree and lists (Sec. 2.1), FP64 operators
// (Sec. 2.2, 3.1, 3.3, 4.1) and grouped-GEMM work schedules.
#include "plan.h"

#include <list>
#include <mutex>
#include <tuple>
#include <unordered_map>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "linalg.h"

namespace kifmm {

namespace {

constexpr double kFourPi = 12.566370614359172953850573533118;

template <class F>
void parallel_for(int64_t n, F&& f) {
    unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 2 || hw == 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    int nt = (int)std::min<int64_t>(hw, n);
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int64_t i = t; i < n; i += nt) f(i);
        });
    for (auto& x : th) x.join();
}

inline uint64_t spread3(uint64_t v) {
    // spread the low 21 bits of v so that bit b lands on bit 3b
    v &= 0x1fffff;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

inline uint64_t compact3(uint64_t v) {
    v &= 0x1249249249249249ULL;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
    v = (v ^ (v >> 32)) & 0x1fffff;
    return v;
}

inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) {
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

inline void unmorton(uint64_t key, int64_t* c) {
    c[0] = (int64_t)compact3(key >> 2);
    c[1] = (int64_t)compact3(key >> 1);
    c[2] = (int64_t)compact3(key);
}

// index of `key` in the sorted range [b, e) of `keys`, or -1
inline int64_t find_key(const std::vector<uint64_t>& keys, int64_t b, int64_t e, uint64_t key) {
    auto it = std::lower_bound(keys.begin() + b, keys.begin() + e, key);
    if (it != keys.begin() + e && *it == key) return it - keys.begin();
    return -1;
}

inline double kernel(const double* x, const double* y) {
    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    double r = std::sqrt(dx * dx + dy * dy + dz * dz);
    return r > 0 ? 1.0 / (kFourPi * r) : 0.0;
}

// G(X, Y) for point lists X (m x 3) and Y (n x 3), row-major m x n
std::vector<double> kernel_matrix(int m, const double* X, int n, const double* Y) {
    std::vector<double> G((size_t)m * n);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) G[(size_t)i * n + j] = kernel(X + 3 * i, Y + 3 * j);
    return G;
}

std::vector<double> transpose(int m, int n, const double* A) {
    std::vector<double> B((size_t)m * n);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) B[(size_t)j * m + i] = A[(size_t)i * n + j];
    return B;
}

}  // namespace

int class_of_offset(int tx, int ty, int tz) {
    if (std::max(std::abs(tx), std::max(std::abs(ty), std::abs(tz))) < 2) return -1;
    if (std::abs(tx) > 3 || std::abs(ty) > 3 || std::abs(tz) > 3) return -1;
    int id = 0;
    for (int a = -3; a <= 3; ++a)
        for (int b = -3; b <= 3; ++b)
            for (int c = -3; c <= 3; ++c) {
                if (std::max(std::abs(a), std::max(std::abs(b), std::abs(c))) < 2) continue;
                if (a == tx && b == ty && c == tz) return id;
                ++id;
            }
    return -1;
}

void offset_of_class(int cls, int* t) {
    int id = 0;
    for (int a = -3; a <= 3; ++a)
        for (int b = -3; b <= 3; ++b)
            for (int c = -3; c <= 3; ++c) {
                if (std::max(std::abs(a), std::max(std::abs(b), std::abs(c))) < 2) continue;
                if (id == cls) {
                    t[0] = a; t[1] = b; t[2] = c;
                    return;
                }
                ++id;
            }
    t[0] = t[1] = t[2] = 0;
}

int box_cube(const HostTree& t, int64_t g, int64_t c[3]) {
    int l = 0;
    while (t.level_begin[l + 1] <= g) ++l;
    unmorton(t.box_key[g], c);
    return l;
}

int64_t leaf_of_box(const HostTree& t, int64_t g) {
    if (t.adaptive) return t.box_leaf[g];
    return g >= t.level_begin[t.depth] ? g - t.level_begin[t.depth] : -1;
}

int64_t box_of_leaf(const HostTree& t, int64_t e) {
    return t.adaptive ? t.leaf_box[e] : t.level_begin[t.depth] + e;
}

namespace {

// Checks of the arguments shared by both tree builders.
void check_tree_args(int64_t n, int leaf_size, int max_depth) {
    if (n < 1) throw PlanError{-1, "n must be >= 1"};
    if (leaf_size < 1) throw PlanError{-1, "leaf_size must be >= 1"};
    if (max_depth < 0 || max_depth > MAX_LEVEL) throw PlanError{-1, "max_depth must be in [0, 20]"};
    if (n > (int64_t)INT32_MAX / 2) throw PlanError{-1, "n too large"};
}

// Root cube, integer coordinates (caller order, 3 per point, into q) and the
// Morton order of the points: fills t.n, t.centre, t.r0 and t.perm and
// returns the sorted Morton keys.
std::vector<uint64_t> sort_points(const double* pts, int64_t n, HostTree& t, std::vector<int64_t>& q) {
    t.n = n;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = pts[3 * i + a];
            if (!std::isfinite(v)) throw PlanError{-4, "non-finite point coordinate at index " + std::to_string(i)};
            lo[a] = std::min(lo[a], v);
            hi[a] = std::max(hi[a], v);
        }
    double ext = 0;
    for (int a = 0; a < 3; ++a) {
        t.centre[a] = (lo[a] + hi[a]) / 2.0;
        ext = std::max(ext, hi[a] - lo[a]);
    }
    t.r0 = ext > 0 ? ext / 2.0 * (1.0 + std::ldexp(1.0, -20)) : 1.0;
    const double qmax = double((1 << QBITS) - 1);
    std::vector<uint64_t> key(n);
    q.resize(3 * n);
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            double base = t.centre[a] - t.r0;
            double v = std::floor((pts[3 * i + a] - base) / (2.0 * t.r0) * double(1 << QBITS));
            v = std::min(std::max(v, 0.0), qmax);
            q[3 * i + a] = (int64_t)v;
        }
        key[i] = morton(q[3 * i], q[3 * i + 1], q[3 * i + 2]);
    }
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    std::vector<uint64_t> skey(n);
    for (int64_t i = 0; i < n; ++i) skey[i] = key[order[i]];
    t.perm = std::move(order);
    return skey;
}

}  // namespace

HostTree build_host_tree(const double* pts, int64_t n, int leaf_size, int depth_override,
                         int max_depth) {
    check_tree_args(n, leaf_size, max_depth);
    if (depth_override < 0 || depth_override > MAX_LEVEL) throw PlanError{-1, "depth must be in [0, 20]"};
    HostTree t;
    std::vector<int64_t> q;
    const std::vector<uint64_t> skey = sort_points(pts, n, t, q);
    const std::vector<int32_t>& order = t.perm;

    int L = depth_override;
    if (L == 0 && depth_override == 0) {
        L = max_depth;
        for (int l = 0; l <= max_depth; ++l) {
            int shift = 3 * (QBITS - l);
            int64_t run = 1, worst = 1;
            for (int64_t i = 1; i < n; ++i) {
                if ((skey[i] >> shift) == (skey[i - 1] >> shift)) {
                    ++run;
                } else {
                    run = 1;
                }
                worst = std::max(worst, run);
            }
            if (worst <= leaf_size) {
                L = l;
                break;
            }
        }
    }
    t.depth = L;

    // per-level unique keys, leaves first
    std::vector<std::vector<uint64_t>> lk(L + 1);
    const int lshift = 3 * (QBITS - L);
    t.leaf_ptr.clear();
    for (int64_t i = 0; i < n; ++i) {
        uint64_t k = skey[i] >> lshift;
        if (lk[L].empty() || lk[L].back() != k) {
            lk[L].push_back(k);
            t.leaf_ptr.push_back((int32_t)i);
        }
    }
    t.leaf_ptr.push_back((int32_t)n);
    for (int l = L - 1; l >= 0; --l) {
        for (uint64_t k : lk[l + 1]) {
            uint64_t pk = k >> 3;
            if (lk[l].empty() || lk[l].back() != pk) lk[l].push_back(pk);
        }
    }
    t.level_begin.assign(L + 2, 0);
    for (int l = 0; l <= L; ++l) t.level_begin[l + 1] = t.level_begin[l] + (int64_t)lk[l].size();
    const int64_t nb = t.level_begin[L + 1];
    t.box_key.resize(nb);
    for (int l = 0; l <= L; ++l)
        std::copy(lk[l].begin(), lk[l].end(), t.box_key.begin() + t.level_begin[l]);
    t.box_parent.assign(nb, -1);
    t.box_child.assign(8 * nb, -1);
    for (int l = 1; l <= L; ++l) {
        for (int64_t b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b) {
            int64_t p = find_key(t.box_key, t.level_begin[l - 1], t.level_begin[l], t.box_key[b] >> 3);
            t.box_parent[b] = (int32_t)p;
            t.box_child[8 * p + (t.box_key[b] & 7)] = (int32_t)b;
        }
    }

    // leaf-unit coordinates of the sorted points
    const double rL = t.half_width(L);
    t.u.resize(3 * n);
    const int64_t nleaf = t.n_leaf();
    for (int64_t e = 0; e < nleaf; ++e) {
        int64_t c[3];
        unmorton(t.box_key[t.level_begin[L] + e], c);
        for (int32_t i = t.leaf_ptr[e]; i < t.leaf_ptr[e + 1]; ++i) {
            for (int a = 0; a < 3; ++a) {
                double centre = (t.centre[a] - t.r0) + (2.0 * double(c[a]) + 1.0) * rL;
                t.u[3 * (int64_t)i + a] = (pts[3 * (int64_t)order[i] + a] - centre) / rL;
            }
        }
    }
    t.leaf_coords.resize(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) t.leaf_coords[3 * i + a] = (int32_t)(q[3 * i + a] >> (QBITS - L));

    // near fields of the leaves
    const int64_t side = int64_t(1) << L;
    t.near_ptr.assign(nleaf + 1, 0);
    {
        std::vector<std::vector<int32_t>> nl(nleaf), nc(nleaf);
        parallel_for(nleaf, [&](int64_t e) {
            int64_t c[3];
            unmorton(t.box_key[t.level_begin[L] + e], c);
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int64_t b[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                        if (b[0] < 0 || b[1] < 0 || b[2] < 0 || b[0] >= side || b[1] >= side || b[2] >= side) continue;
                        int64_t j = find_key(t.box_key, t.level_begin[L], t.level_begin[L + 1],
                                             morton(b[0], b[1], b[2]));
                        if (j < 0) continue;
                        nl[e].push_back((int32_t)(j - t.level_begin[L]));
                        // code of (target - source) = -d
                        nc[e].push_back((1 - dx) * 9 + (1 - dy) * 3 + (1 - dz));
                    }
        });
        for (int64_t e = 0; e < nleaf; ++e) t.near_ptr[e + 1] = t.near_ptr[e] + (int32_t)nl[e].size();
        t.near_leaf.reserve(t.near_ptr[nleaf]);
        t.near_code.reserve(t.near_ptr[nleaf]);
        for (int64_t e = 0; e < nleaf; ++e) {
            t.near_leaf.insert(t.near_leaf.end(), nl[e].begin(), nl[e].end());
            t.near_code.insert(t.near_code.end(), nc[e].begin(), nc[e].end());
        }
    }

    // interaction fields of every box at levels 2..L: children of the parent's
    // near field that are not adjacent to the box
    t.v_ptr.assign(nb + 1, 0);
    {
        std::vector<std::vector<int32_t>> vs(nb), vc(nb);
        for (int l = 2; l <= L; ++l) {
            const int64_t pside = int64_t(1) << (l - 1);
            const int64_t b0 = t.level_begin[l], b1 = t.level_begin[l + 1];
            parallel_for(b1 - b0, [&](int64_t off) {
                const int64_t b = b0 + off;
                int64_t c[3];
                unmorton(t.box_key[b], c);
                int64_t pc[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
                for (int dx = -1; dx <= 1; ++dx)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dz = -1; dz <= 1; ++dz) {
                            int64_t pn[3] = {pc[0] + dx, pc[1] + dy, pc[2] + dz};
                            if (pn[0] < 0 || pn[1] < 0 || pn[2] < 0 || pn[0] >= pside || pn[1] >= pside || pn[2] >= pside) continue;
                            int64_t p = find_key(t.box_key, t.level_begin[l - 1], t.level_begin[l],
                                                 morton(pn[0], pn[1], pn[2]));
                            if (p < 0) continue;
                            for (int o = 0; o < 8; ++o) {
                                int32_t ch = t.box_child[8 * p + o];
                                if (ch < 0) continue;
                                int64_t cc[3] = {2 * pn[0] + ((o >> 2) & 1), 2 * pn[1] + ((o >> 1) & 1), 2 * pn[2] + (o & 1)};
                                int tx = (int)(c[0] - cc[0]), ty = (int)(c[1] - cc[1]), tz = (int)(c[2] - cc[2]);
                                if (std::max(std::abs(tx), std::max(std::abs(ty), std::abs(tz))) < 2) continue;
                                vs[b].push_back(ch);
                                vc[b].push_back(class_of_offset(tx, ty, tz));
                            }
                        }
            });
        }
        for (int64_t b = 0; b < nb; ++b) t.v_ptr[b + 1] = t.v_ptr[b] + (int32_t)vs[b].size();
        t.v_src.reserve(t.v_ptr[nb]);
        t.v_cls.reserve(t.v_ptr[nb]);
        for (int64_t b = 0; b < nb; ++b) {
            t.v_src.insert(t.v_src.end(), vs[b].begin(), vs[b].end());
            t.v_cls.insert(t.v_cls.end(), vc[b].begin(), vc[b].end());
        }
    }
    return t;
}

namespace {

// Whether the closed cubes (la, ca) and (lb, cb), la <= lb, share a point.
inline bool cubes_touch(int la, const int64_t* ca, int lb, const int64_t* cb) {
    const int s = lb - la;
    for (int a = 0; a < 3; ++a) {
        const int64_t lo = ca[a] << s, hi = (ca[a] + 1) << s;
        if (cb[a] > hi || cb[a] + 1 < lo) return false;
    }
    return true;
}

struct ANode {
    uint64_t key;    // Morton key at the node's level
    int32_t b, e;    // range of sorted points
    bool leaf;
};

}  // namespace

HostTree build_adaptive_host_tree(const double* pts, int64_t n, int leaf_size, int max_depth) {
    check_tree_args(n, leaf_size, max_depth);
    HostTree t;
    t.adaptive = true;
    std::vector<int64_t> q;
    const std::vector<uint64_t> skey = sort_points(pts, n, t, q);
    std::vector<std::vector<ANode>> lv(max_depth + 1);
    std::vector<std::unordered_map<uint64_t, int32_t>> at(max_depth + 1);
    auto add = [&](int l, uint64_t key, int32_t b, int32_t e) {
        at[l][key] = (int32_t)lv[l].size();
        lv[l].push_back(ANode{key, b, e, true});
    };
    // the nonempty children of node idx at level l (a contiguous run of the
    // sorted points each), all new leaves
    auto split = [&](int l, int32_t idx) {
        lv[l][idx].leaf = false;
        const int32_t b = lv[l][idx].b, e = lv[l][idx].e;
        const int shift = 3 * (QBITS - l - 1);
        int32_t i = b;
        while (i < e) {
            const uint64_t ck = skey[i] >> shift;
            int32_t j = i + 1;
            while (j < e && (skey[j] >> shift) == ck) ++j;
            add(l + 1, ck, i, j);
            i = j;
        }
    };
    add(0, 0, 0, (int32_t)n);
    {
        std::vector<std::pair<int, int32_t>> work{{0, 0}};
        while (!work.empty()) {
            const auto [l, idx] = work.back();
            work.pop_back();
            if (lv[l][idx].e - lv[l][idx].b > leaf_size && l < max_depth) {
                const size_t first = lv[l + 1].size();
                split(l, idx);
                for (size_t c = first; c < lv[l + 1].size(); ++c) work.push_back({l + 1, (int32_t)c});
            }
        }
    }
    // 2:1 balance in rounds. A leaf A touching a leaf F two or more levels
    // finer contains a same-level neighbour cube of F; it is the deepest
    // existing cube holding that neighbour cube, so F's 26 neighbours find it.
    for (;;) {
        std::vector<std::pair<int, int32_t>> marks;
        for (int l = 2; l <= max_depth; ++l) {
            const int64_t side = int64_t(1) << l;
            for (const ANode& f : lv[l]) {
                if (!f.leaf) continue;
                int64_t c[3];
                unmorton(f.key, c);
                for (int d = 0; d < 27; ++d) {
                    if (d == 13) continue;
                    const int64_t nb[3] = {c[0] + d / 9 - 1, c[1] + (d / 3) % 3 - 1, c[2] + d % 3 - 1};
                    if (nb[0] < 0 || nb[1] < 0 || nb[2] < 0 || nb[0] >= side || nb[1] >= side || nb[2] >= side) continue;
                    const uint64_t nk = morton(nb[0], nb[1], nb[2]);
                    for (int m = l; m >= 0; --m) {
                        auto it = at[m].find(nk >> (3 * (l - m)));
                        if (it == at[m].end()) continue;
                        if (m <= l - 2 && lv[m][it->second].leaf) marks.push_back({m, it->second});
                        break;
                    }
                }
            }
        }
        if (marks.empty()) break;
        std::sort(marks.begin(), marks.end());
        marks.erase(std::unique(marks.begin(), marks.end()), marks.end());
        for (const auto& [m, idx] : marks) split(m, idx);
    }
    int D = 0;
    for (int l = 0; l <= max_depth; ++l)
        if (!lv[l].empty()) D = l;
    t.depth = D;
    // global numbering: per level the leaves, then the split cubes, each in Morton order
    std::vector<std::vector<int32_t>> gid(D + 1);
    t.level_begin.assign(D + 2, 0);
    t.level_leaves.assign(D + 1, 0);
    std::vector<std::pair<int, int32_t>> node_of;   // global box -> (level, node)
    for (int l = 0; l <= D; ++l) {
        std::vector<int32_t> idx(lv[l].size());
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
            if (lv[l][a].leaf != lv[l][b].leaf) return lv[l][a].leaf;
            return lv[l][a].key < lv[l][b].key;
        });
        gid[l].assign(lv[l].size(), -1);
        for (int32_t i : idx) {
            gid[l][i] = (int32_t)node_of.size();
            node_of.push_back({l, i});
            if (lv[l][i].leaf) ++t.level_leaves[l];
        }
        t.level_begin[l + 1] = (int64_t)node_of.size();
    }
    const int64_t nb = t.n_box();
    t.box_key.resize(nb);
    t.box_parent.assign(nb, -1);
    t.box_child.assign(8 * nb, -1);
    t.box_leaf.assign(nb, -1);
    for (int64_t g = 0; g < nb; ++g) {
        const auto [l, i] = node_of[g];
        t.box_key[g] = lv[l][i].key;
        if (l > 0) {
            const int32_t p = gid[l - 1][at[l - 1].at(lv[l][i].key >> 3)];
            t.box_parent[g] = p;
            t.box_child[8 * (int64_t)p + (lv[l][i].key & 7)] = (int32_t)g;
        }
    }
    // leaves in the order of their points
    std::vector<int32_t> leaves;
    for (int64_t g = 0; g < nb; ++g)
        if (lv[node_of[g].first][node_of[g].second].leaf) leaves.push_back((int32_t)g);
    auto first_point = [&](int32_t g) { return lv[node_of[g].first][node_of[g].second].b; };
    std::sort(leaves.begin(), leaves.end(), [&](int32_t a, int32_t b) { return first_point(a) < first_point(b); });
    const int64_t nleaf = (int64_t)leaves.size();
    t.leaf_ptr.resize(nleaf + 1);
    t.leaf_box = leaves;
    t.leaf_level.resize(nleaf);
    for (int64_t e = 0; e < nleaf; ++e) {
        const auto [l, i] = node_of[leaves[e]];
        t.leaf_ptr[e] = lv[l][i].b;
        t.leaf_level[e] = l;
        t.box_leaf[leaves[e]] = (int32_t)e;
        if (e > 0 && lv[node_of[leaves[e - 1]].first][node_of[leaves[e - 1]].second].e != lv[l][i].b)
            throw PlanError{-1, "internal: leaves do not partition the points"};
    }
    t.leaf_ptr[nleaf] = (int32_t)n;
    // coordinates in the units of each point's own leaf
    t.u.resize(3 * n);
    for (int64_t e = 0; e < nleaf; ++e) {
        const int l = t.leaf_level[e];
        const double r = t.half_width(l);
        int64_t c[3];
        unmorton(t.box_key[t.leaf_box[e]], c);
        for (int32_t i = t.leaf_ptr[e]; i < t.leaf_ptr[e + 1]; ++i)
            for (int a = 0; a < 3; ++a) {
                const double centre = (t.centre[a] - t.r0) + (2.0 * double(c[a]) + 1.0) * r;
                t.u[3 * (int64_t)i + a] = (pts[3 * (int64_t)t.perm[i] + a] - centre) / r;
            }
    }
    t.leaf_coords.resize(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) t.leaf_coords[3 * i + a] = (int32_t)(q[3 * i + a] >> (QBITS - D));
    auto find = [&](int l, uint64_t key) -> int32_t {
        if (l < 0 || l > D) return -1;
        auto it = at[l].find(key);
        return it == at[l].end() ? -1 : gid[l][it->second];
    };
    auto level_of = [&](int64_t g) {
        int l = 0;
        while (t.level_begin[l + 1] <= g) ++l;
        return l;
    };
    // U (near field with codes) and W lists of every leaf
    t.near_ptr.assign(nleaf + 1, 0);
    t.w_ptr.assign(nleaf + 1, 0);
    {
        std::vector<std::vector<int32_t>> nl(nleaf), nc(nleaf), wl(nleaf);
        std::vector<std::string> errs(nleaf);
        parallel_for(nleaf, [&](int64_t e) {
            const int l = t.leaf_level[e];
            const int64_t side = int64_t(1) << l;
            int64_t c[3];
            unmorton(t.box_key[t.leaf_box[e]], c);
            auto add_near = [&](int32_t g, int ls) {
                const int32_t s = t.box_leaf[g];
                for (int32_t v : nl[e])
                    if (v == s) return;
                int64_t sc[3];
                unmorton(t.box_key[g], sc);
                int m = 0, off[3];
                for (int a = 0; a < 3; ++a) {
                    if (ls == l) {
                        off[a] = (int)(2 * (sc[a] - c[a]));
                    } else if (ls == l + 1) {
                        m = 1;
                        off[a] = (int)((2 * sc[a] + 1) - (4 * c[a] + 2));
                    } else if (ls == l - 1) {
                        m = 2;
                        off[a] = (int)((4 * sc[a] + 2) - (2 * c[a] + 1));
                    } else {
                        errs[e] = "internal: near-field leaves more than one level apart";
                        return;
                    }
                    if (off[a] < -4 || off[a] > 4) {
                        errs[e] = "internal: near-field offset out of range";
                        return;
                    }
                }
                nl[e].push_back(s);
                nc[e].push_back(m * 729 + (off[0] + 4) * 81 + (off[1] + 4) * 9 + (off[2] + 4));
            };
            std::vector<std::pair<int32_t, int>> stack;
            for (int d = 0; d < 27; ++d) {
                const int64_t pc[3] = {c[0] + d / 9 - 1, c[1] + (d / 3) % 3 - 1, c[2] + d % 3 - 1};
                if (pc[0] < 0 || pc[1] < 0 || pc[2] < 0 || pc[0] >= side || pc[1] >= side || pc[2] >= side) continue;
                const uint64_t pk = morton(pc[0], pc[1], pc[2]);
                const int32_t g = find(l, pk);
                if (g >= 0) {
                    // a same-level neighbour (or the leaf itself): its touching leaves
                    // are near, its first descendants that do not touch are W
                    stack.assign(1, {g, l});
                    while (!stack.empty()) {
                        const auto [h, lh] = stack.back();
                        stack.pop_back();
                        if (t.box_leaf[h] >= 0) {
                            add_near(h, lh);
                            continue;
                        }
                        for (int o = 0; o < 8; ++o) {
                            const int32_t ch = t.box_child[8 * (int64_t)h + o];
                            if (ch < 0) continue;
                            int64_t cc[3];
                            unmorton(t.box_key[ch], cc);
                            if (cubes_touch(l, c, lh + 1, cc))
                                stack.push_back({ch, lh + 1});
                            else
                                wl[e].push_back(ch);
                        }
                    }
                } else {
                    // the coarser leaf holding the neighbour cube, if any
                    for (int m = l - 1; m >= 0; --m) {
                        const int32_t h = find(m, pk >> (3 * (l - m)));
                        if (h < 0) continue;
                        if (t.box_leaf[h] >= 0) add_near(h, m);
                        break;
                    }
                }
            }
        });
        for (int64_t e = 0; e < nleaf; ++e)
            if (!errs[e].empty()) throw PlanError{-1, errs[e]};
        for (int64_t e = 0; e < nleaf; ++e) {
            t.near_ptr[e + 1] = t.near_ptr[e] + (int32_t)nl[e].size();
            t.w_ptr[e + 1] = t.w_ptr[e] + (int32_t)wl[e].size();
        }
        for (int64_t e = 0; e < nleaf; ++e) {
            t.near_leaf.insert(t.near_leaf.end(), nl[e].begin(), nl[e].end());
            t.near_code.insert(t.near_code.end(), nc[e].begin(), nc[e].end());
            std::sort(wl[e].begin(), wl[e].end());
            t.w_src.insert(t.w_src.end(), wl[e].begin(), wl[e].end());
        }
    }
    // X lists: the dual of W
    {
        std::vector<int32_t> cnt(nb + 1, 0);
        for (int32_t g : t.w_src) ++cnt[g + 1];
        t.x_ptr.assign(nb + 1, 0);
        for (int64_t g = 0; g < nb; ++g) t.x_ptr[g + 1] = t.x_ptr[g] + cnt[g + 1];
        t.x_src.assign(t.w_src.size(), -1);
        std::vector<int32_t> fill(t.x_ptr.begin(), t.x_ptr.end() - 1);
        for (int64_t e = 0; e < nleaf; ++e)
            for (int32_t k = t.w_ptr[e]; k < t.w_ptr[e + 1]; ++k) t.x_src[fill[t.w_src[k]]++] = (int32_t)e;
    }
    // V lists of every box at levels 2..D: children of the parent's
    // same-level neighbours that do not share a vertex with the box
    t.v_ptr.assign(nb + 1, 0);
    {
        std::vector<std::vector<int32_t>> vs(nb), vc(nb);
        const int64_t b2 = D >= 2 ? t.level_begin[2] : nb;
        parallel_for(nb - b2, [&](int64_t off) {
            const int64_t b = b2 + off;
            const int l = level_of(b);
            const int64_t pside = int64_t(1) << (l - 1);
            int64_t c[3];
            unmorton(t.box_key[b], c);
            const int64_t pc[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
            for (int d = 0; d < 27; ++d) {
                const int64_t pn[3] = {pc[0] + d / 9 - 1, pc[1] + (d / 3) % 3 - 1, pc[2] + d % 3 - 1};
                if (pn[0] < 0 || pn[1] < 0 || pn[2] < 0 || pn[0] >= pside || pn[1] >= pside || pn[2] >= pside) continue;
                const int32_t p = find(l - 1, morton(pn[0], pn[1], pn[2]));
                if (p < 0) continue;
                for (int o = 0; o < 8; ++o) {
                    const int32_t ch = t.box_child[8 * (int64_t)p + o];
                    if (ch < 0) continue;
                    const int64_t cc[3] = {2 * pn[0] + ((o >> 2) & 1), 2 * pn[1] + ((o >> 1) & 1), 2 * pn[2] + (o & 1)};
                    const int tx = (int)(c[0] - cc[0]), ty = (int)(c[1] - cc[1]), tz = (int)(c[2] - cc[2]);
                    if (std::max(std::abs(tx), std::max(std::abs(ty), std::abs(tz))) < 2) continue;
                    vs[b].push_back(ch);
                    vc[b].push_back(class_of_offset(tx, ty, tz));
                }
            }
        });
        for (int64_t b = 0; b < nb; ++b) t.v_ptr[b + 1] = t.v_ptr[b] + (int32_t)vs[b].size();
        for (int64_t b = 0; b < nb; ++b) {
            t.v_src.insert(t.v_src.end(), vs[b].begin(), vs[b].end());
            t.v_cls.insert(t.v_cls.end(), vc[b].begin(), vc[b].end());
        }
    }
    return t;
}

HostOps build_host_ops(int p, double eps, int leaf_size, double cd, double rcond, bool dense) {
    if (p < 2 || p > 16) throw PlanError{-1, "p must be in [2, 16]"};
    if (!(eps >= 0.0 && eps < 1.0)) throw PlanError{-1, "eps must be in [0, 1)"};
    if (!(cd >= 0.0) || !(rcond >= 0.0)) throw PlanError{-1, "cd and pinv_rcond must be >= 0"};
    HostOps o;
    o.p = p;
    o.dense = dense;
    o.eps = eps;
    o.rcond = rcond;
    o.d = cd / std::sqrt(double(leaf_size));
    if (!(o.d <= 2.0 / 3.0)) throw PlanError{-1, "surface offset d = cd/sqrt(leaf_size) must be <= 2/3"};
    // boundary nodes of the p^3 grid on [-1,1]^3, lexicographic
    std::vector<double> g(p);
    for (int i = 0; i < p; ++i) g[i] = -1.0 + 2.0 * double(i) / double(p - 1);
    g[p - 1] = 1.0;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int k = 0; k < p; ++k)
                if (std::min(i, std::min(j, k)) == 0 || std::max(i, std::max(j, k)) == p - 1) {
                    o.E.push_back(g[i]);
                    o.E.push_back(g[j]);
                    o.E.push_back(g[k]);
                }
    const int ne = (int)o.E.size() / 3;
    o.n_eq = ne;
    std::vector<double> inner(3 * ne), outer(3 * ne);
    for (int i = 0; i < 3 * ne; ++i) {
        inner[i] = (1.0 + o.d) * o.E[i];
        outer[i] = (3.0 - 2.0 * o.d) * o.E[i];
    }
    o.outer = outer;
    // S2M / L2T check-to-equivalent pseudo-inverses (unit cube)
    std::vector<double> Gup = kernel_matrix(ne, outer.data(), ne, inner.data());  // G(UC, UE)
    std::vector<double> Gdn = kernel_matrix(ne, inner.data(), ne, outer.data());  // G(DC, DE)
    std::vector<double> Pup = pinv(ne, Gup.data(), rcond);
    std::vector<double> Pdn = pinv(ne, Gdn.data(), rcond);
    // M2M and L2L for the 8 child octants (parent units)
    std::vector<double> M8((size_t)8 * ne * ne), L8((size_t)8 * ne * ne);
    parallel_for(8, [&](int64_t oc) {
        double s[3] = {((oc >> 2) & 1) ? 1.0 : -1.0, ((oc >> 1) & 1) ? 1.0 : -1.0, (oc & 1) ? 1.0 : -1.0};
        std::vector<double> child(3 * ne);
        for (int i = 0; i < ne; ++i)
            for (int a = 0; a < 3; ++a) child[3 * i + a] = 0.5 * (s[a] + inner[3 * i + a]);
        std::vector<double> Gm = kernel_matrix(ne, outer.data(), ne, child.data());   // G(UC, child UE)
        std::vector<double> Mo = matmul(ne, ne, ne, Pup.data(), Gm.data());
        std::vector<double> Gl = kernel_matrix(ne, child.data(), ne, outer.data());   // G(child DC, DE)
        std::vector<double> Lo = matmul(ne, ne, ne, Gl.data(), Pdn.data());
        std::copy(Mo.begin(), Mo.end(), M8.begin() + oc * ne * ne);
        std::copy(Lo.begin(), Lo.end(), L8.begin() + oc * ne * ne);
    });
    // M2L matrices K^(t) = G(DC + 2t, UE)
    std::vector<double> K((size_t)NCLASS * ne * ne);
    parallel_for(NCLASS, [&](int64_t c) {
        int t[3];
        offset_of_class((int)c, t);
        std::vector<double> tgt(3 * ne);
        for (int i = 0; i < ne; ++i)
            for (int a = 0; a < 3; ++a) tgt[3 * i + a] = inner[3 * i + a] + 2.0 * t[a];
        std::vector<double> Kc = kernel_matrix(ne, tgt.data(), ne, inner.data());
        std::copy(Kc.begin(), Kc.end(), K.begin() + c * ne * ne);
    });
    o.sing.assign(ne, 0.0);
    if (dense) {
        o.k = ne;
        o.U.assign((size_t)ne * ne, 0.0);
        for (int i = 0; i < ne; ++i) o.U[(size_t)i * ne + i] = 1.0;
        o.S = Pup;
        o.T = Pdn;
        o.M = std::move(M8);
        o.L = std::move(L8);
        o.K = std::move(K);
        return o;
    }
    // stage-1 compression: U from the SVD of K_fat = [K^(1) ... K^(316)]
    std::vector<double> Kfat((size_t)ne * NCLASS * ne);
    for (int c = 0; c < NCLASS; ++c)
        for (int i = 0; i < ne; ++i)
            std::memcpy(&Kfat[(size_t)i * NCLASS * ne + (size_t)c * ne], &K[(size_t)c * ne * ne + (size_t)i * ne],
                        sizeof(double) * ne);
    std::vector<double> s, Ufull;
    svd_wide_left(ne, (int64_t)NCLASS * ne, Kfat.data(), s, Ufull);
    Kfat.clear();
    Kfat.shrink_to_fit();
    o.sing = s;
    o.sigma0 = s[0];
    int k = 0;
    for (int i = 0; i < ne; ++i)
        if (s[i] >= eps * s[0]) ++k;
    if (k < 1) k = 1;
    o.k = k;
    o.U.resize((size_t)ne * k);
    for (int i = 0; i < ne; ++i)
        for (int j = 0; j < k; ++j) o.U[(size_t)i * k + j] = Ufull[(size_t)i * ne + j];
    const double* U = o.U.data();
    o.S = matmul_tn(k, ne, ne, U, Pup.data());         // U~^T P_up
    o.T = matmul(ne, ne, k, Pdn.data(), U);            // P_dn U~
    o.M.resize((size_t)8 * k * k);
    o.L.resize((size_t)8 * k * k);
    parallel_for(8, [&](int64_t oc) {
        std::vector<double> MU = matmul(ne, ne, k, &M8[oc * ne * ne], U);
        std::vector<double> Mr = matmul_tn(k, ne, k, U, MU.data());
        std::vector<double> LU = matmul(ne, ne, k, &L8[oc * ne * ne], U);
        std::vector<double> Lr = matmul_tn(k, ne, k, U, LU.data());
        std::copy(Mr.begin(), Mr.end(), o.M.begin() + oc * k * k);
        std::copy(Lr.begin(), Lr.end(), o.L.begin() + oc * k * k);
    });
    o.K.resize((size_t)NCLASS * k * k);
    parallel_for(NCLASS, [&](int64_t c) {
        std::vector<double> KU = matmul(ne, ne, k, &K[(size_t)c * ne * ne], U);
        std::vector<double> Kr = matmul_tn(k, ne, k, U, KU.data());
        std::copy(Kr.begin(), Kr.end(), o.K.begin() + c * k * k);
    });
    return o;
}

std::shared_ptr<const HostOps> host_ops_shared(int p, double eps, int leaf_size, double cd, double rcond,
                                               bool dense, double c2) {
    using Key = std::tuple<int, double, int, double, double, bool, double>;
    static std::mutex mu;
    static std::list<std::pair<Key, std::shared_ptr<const HostOps>>> lru;   // most recent first
    constexpr size_t kKeep = 4;
    const Key key{p, eps, leaf_size, cd, rcond, dense, c2};
    {
        std::lock_guard<std::mutex> lock(mu);
        for (auto it = lru.begin(); it != lru.end(); ++it)
            if (it->first == key) {
                lru.splice(lru.begin(), lru, it);
                return lru.front().second;
            }
    }
    // built outside the lock (seconds); two threads asking for one new key
    // both build it and the first to finish is cached
    auto ops = std::make_shared<HostOps>(build_host_ops(p, eps, leaf_size, cd, rcond, dense));
    if (c2 > 0.0) build_stage2(*ops, c2);
    std::lock_guard<std::mutex> lock(mu);
    for (auto it = lru.begin(); it != lru.end(); ++it)
        if (it->first == key) return it->second;
    lru.emplace_front(key, ops);
    if (lru.size() > kKeep) lru.pop_back();
    return ops;
}

void build_stage2(HostOps& o, double c2) {
    if (o.dense) throw PlanError{-1, "stage-2 low rank needs the compressed operators (dense_m2l = 0)"};
    if (!(c2 > 0.0) || !std::isfinite(c2)) throw PlanError{-1, "c2 must be finite and > 0"};
    const int k = o.k;
    o.c2 = c2;
    o.eps2 = c2 * o.eps / double(k) * o.sigma0;
    std::vector<std::vector<double>> Us(NCLASS), Vs(NCLASS), ss(NCLASS);
    o.rank2.assign(NCLASS, 0);
    parallel_for(NCLASS, [&](int64_t c) {
        svd_jacobi(k, k, &o.K[(size_t)c * k * k], ss[c], Us[c], Vs[c]);
        int r = 0;
        for (int i = 0; i < k; ++i)
            if (ss[c][i] >= o.eps2) ++r;
        o.rank2[c] = std::max(r, 1);
    });
    o.r2max = *std::max_element(o.rank2.begin(), o.rank2.end());
    const int rm = o.r2max;
    o.U2.assign((size_t)NCLASS * k * rm, 0.0);
    o.V2.assign((size_t)NCLASS * rm * k, 0.0);
    for (int c = 0; c < NCLASS; ++c) {
        const int r = o.rank2[c];
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < r; ++j) o.U2[((size_t)c * k + i) * rm + j] = Us[c][(size_t)i * k + j];
        // V^ = S^ Q^^T: row j is s_j times column j of the right singular vectors
        for (int j = 0; j < r; ++j)
            for (int i = 0; i < k; ++i) o.V2[((size_t)c * rm + j) * k + i] = ss[c][j] * Vs[c][(size_t)i * k + j];
    }
}

std::vector<int> split_tile_ranges(const std::vector<int32_t>& tile_chunk0, int cp, int64_t slot_bytes,
                                   int64_t max_bytes, int64_t max_slots) {
    const int n_tiles = tile_chunk0.empty() ? 0 : (int)tile_chunk0.size() - 1;
    auto fits = [&](int t0, int t1) {
        const int64_t slots = (int64_t)(tile_chunk0[t1] - tile_chunk0[t0]) * cp;
        return slots * slot_bytes < max_bytes && slots < max_slots;
    };
    std::vector<int> starts{0};
    for (int t = 0; t < n_tiles; ++t) {
        if (!fits(t, t + 1)) return {};
        if (!fits(starts.back(), t + 1)) starts.push_back(t);
    }
    starts.push_back(n_tiles);
    return starts;
}

std::vector<int64_t> uniform_cuts(int64_t n_tgt, int tile) {
    std::vector<int64_t> cuts;
    for (int64_t t = 0; t < n_tgt; t += tile) cuts.push_back(t);
    cuts.push_back(n_tgt);
    return cuts;
}

std::vector<int64_t> balanced_cuts(int64_t n_tgt, const int32_t* ptr, int n_tiles, int max_tile,
                                   double per_target) {
    std::vector<int64_t> cuts{0};
    if (n_tgt == 0) return cuts;
    const double total = double(ptr[n_tgt] - ptr[0]) + per_target * double(n_tgt);
    const double quota = total / std::max(1, n_tiles);
    double acc = 0.0;
    int64_t start = 0;
    for (int64_t t = 0; t < n_tgt; ++t) {
        acc += double(ptr[t + 1] - ptr[t]) + per_target;
        const bool full = (t + 1 - start) >= max_tile;
        if (t + 1 < n_tgt && (full || acc >= quota * double(cuts.size()))) {
            cuts.push_back(t + 1);
            start = t + 1;
        }
    }
    cuts.push_back(n_tgt);
    return cuts;
}

std::vector<int64_t> chunk_cuts(int64_t n_tgt, const int32_t* ptr, const int32_t* cls, const int32_t* group,
                                int cp, int rhs, int n_tiles, int max_tile, const TileCost& w) {
    std::vector<int64_t> cuts{0};
    if (n_tgt == 0) return cuts;
    int n_groups = 1;
    if (group)
        for (int64_t t = 0; t < n_tgt; ++t) n_groups = std::max(n_groups, group[t] + 1);
    const int cpb = std::max(1, 16 / std::max(1, rhs));   // pairs per 16-column block (rhs <= 16)
    std::vector<int32_t> cnt((size_t)n_groups * NCLASS * 8, 0);
    std::vector<int32_t> touched;
    // cost of adding target t to the current tile (counts not yet updated)
    auto delta = [&](int64_t t) {
        double d = w.per_target;
        const int64_t g = group ? group[t] : 0;
        for (int32_t q = ptr[t]; q < ptr[t + 1]; ++q) {
            const int32_t n = cnt[(size_t)(g * NCLASS * 8 + cls[q])];
            if (n % cp == 0) d += w.per_chunk;
            if (n % cpb == 0) d += w.per_block;
        }
        return d;
    };
    auto add = [&](int64_t t) {
        const int64_t g = group ? group[t] : 0;
        for (int32_t q = ptr[t]; q < ptr[t + 1]; ++q) {
            int32_t& n = cnt[(size_t)(g * NCLASS * 8 + cls[q])];
            if (n == 0) touched.push_back((int32_t)(g * NCLASS * 8 + cls[q]));
            ++n;
        }
    };
    auto reset = [&]() {
        for (int32_t k : touched) cnt[(size_t)k] = 0;
        touched.clear();
    };
    // greedy cut at cost threshold T: a tile closes before the target that
    // would take it over T or past max_tile targets
    auto greedy = [&](double T, std::vector<int64_t>* out) {
        int64_t tiles = 1, start = 0;
        double cost = 0.0;
        reset();
        for (int64_t t = 0; t < n_tgt; ++t) {
            double d = delta(t);
            if (t > start && (cost + d > T || t - start >= max_tile)) {
                if (out) out->push_back(t);
                ++tiles;
                start = t;
                cost = 0.0;
                reset();
                d = delta(t);
            }
            add(t);
            cost += d;
        }
        reset();
        return tiles;
    };
    // smallest threshold giving at most n_tiles tiles (bisection)
    double hi = 0.0;
    {
        reset();
        for (int64_t t = 0; t < n_tgt; ++t) {
            hi += delta(t);
            add(t);
        }
        reset();
    }
    double lo = 0.0;
    for (int it = 0; it < 40 && hi - lo > 1e-3 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (greedy(mid, nullptr) <= std::max(1, n_tiles))
            hi = mid;
        else
            lo = mid;
    }
    greedy(hi, &cuts);
    cuts.push_back(n_tgt);
    return cuts;
}

void gg_build(GGSched& s, int64_t tgt_row0, int64_t n_tgt, const int32_t* ptr, const int32_t* src,
              const int32_t* cls, const int32_t* group, const std::vector<double>& group_scale,
              const std::vector<int64_t>& cuts) {
    if (s.tile_chunk0.empty()) s.tile_chunk0.push_back(0);
    struct Item {
        int64_t key;
        int32_t q;
        int32_t col;
    };
    std::vector<Item> items;
    for (size_t c = 0; c + 1 < cuts.size(); ++c) {
        const int64_t t0 = cuts[c], t1 = cuts[c + 1];
        if (t1 <= t0) continue;
        s.tile_tgt0.push_back((int32_t)(tgt_row0 + t0));
        s.tile_ntgt.push_back((int32_t)(t1 - t0));
        s.max_tile = std::max<int>(s.max_tile, (int)(t1 - t0));
        items.clear();
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t g = group ? group[t] : 0;
            for (int32_t q = ptr[t]; q < ptr[t + 1]; ++q)
                items.push_back({g * NCLASS * 8 + cls[q], q, (int32_t)(t - t0)});
        }
        std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.key < b.key; });
        const size_t first_chunk = s.chunk_cls.size();
        size_t i = 0;
        std::vector<int32_t> slot(s.cp);
        while (i < items.size()) {
            const int64_t key = items[i].key;
            const int64_t g = key / (NCLASS * 8);
            s.chunk_cls.push_back(cls[items[i].q]);
            s.chunk_scale.push_back(group_scale[g]);
            size_t e = i;
            while (e < items.size() && e - i < (size_t)s.cp && items[e].key == key) ++e;
            const int used = (int)(e - i);
            // Slot order inside the chunk: the kernels add the products of the
            // slots of a 16-column block into their target columns of an LDS
            // accumulator whose column stride is 1 modulo 16 banks' groups of
            // four words, so a block whose columns are distinct modulo 16 (best:
            // column = slot mod 16) is free of bank conflicts. Every column has
            // one slot per chunk, so the order changes no sum.
            std::fill(slot.begin(), slot.end(), -1);
            const int nslot = s.rhs == 1 ? (used > 16 ? 32 : 16) : s.cp;
            if (s.rhs == 1 && s.cp == 32) {
                std::vector<size_t> rest;
                for (size_t k = i; k < e; ++k) {
                    const int r = items[k].col & 15;
                    if (slot[r] < 0)
                        slot[r] = (int32_t)k;
                    else if (nslot == 32 && slot[16 + r] < 0)
                        slot[16 + r] = (int32_t)k;
                    else
                        rest.push_back(k);
                }
                size_t f = 0;
                for (int j = 0; j < nslot && f < rest.size(); ++j)
                    if (slot[j] < 0) slot[j] = (int32_t)rest[f++];
            } else {
                for (int j = 0; j < used; ++j) slot[j] = (int32_t)(i + j);
            }
            for (int j = 0; j < s.cp; ++j) {
                if (slot[j] >= 0) {
                    s.chunk_src.push_back(src[items[slot[j]].q]);
                    s.chunk_col.push_back(items[slot[j]].col);
                } else {
                    s.chunk_src.push_back(-1);
                    s.chunk_col.push_back(-1);
                }
            }
            s.chunk_nblk.push_back(s.rhs == 1 && s.cp == 32 ? nslot / 16 : (used * s.rhs + 15) / 16);
            i = e;
        }
        // class of the next chunk with a different class, within this tile
        const size_t last = s.chunk_cls.size();
        s.chunk_next.resize(last, -1);
        int next = -1;
        for (size_t ch = last; ch-- > first_chunk;) {
            s.chunk_next[ch] = next;
            if (ch > first_chunk && s.chunk_cls[ch - 1] != s.chunk_cls[ch]) next = s.chunk_cls[ch];
        }
        s.pairs += (int64_t)items.size();
        s.tile_chunk0.push_back((int32_t)s.chunk_cls.size());
    }
}

}  // namespace kifmm
