// Host plan construction (octree, lists, FP64 operators, stage-2 factors and
// the M2L work schedule) on seeded point sets, with checks of its structural
// invariants. Built with the address and undefined-behaviour sanitizers and
// run by tests/test_host_sanitized.py; any out-of-bounds access, leak or
// undefined operation in plan.cpp or linalg.cpp fails the run.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_1211_2517_amd/csrc/plan.h"

using namespace kifmm;

static int fails = 0;
#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            std::printf("check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                              \
        }                                                         \
    } while (0)

static void run(const std::vector<double>& pts, int leaf, const char* name) {
    const int64_t n = (int64_t)pts.size() / 3;
    HostTree t = build_host_tree(pts.data(), n, leaf, 0, 16);
    CHECK(t.n == n && (int64_t)t.perm.size() == n);
    CHECK(t.leaf_ptr.front() == 0 && t.leaf_ptr.back() == n);
    std::vector<int> seen(n, 0);
    for (int32_t p : t.perm) {
        CHECK(p >= 0 && p < n);
        if (p >= 0 && p < n) ++seen[p];
    }
    for (int v : seen) CHECK(v == 1);
    for (double u : t.u) CHECK(std::fabs(u) <= 1.0);
    // every near entry names a leaf; every interaction entry a box of the same level
    for (int32_t s : t.near_leaf) CHECK(s >= 0 && s < t.n_leaf());
    for (int l = 2; l <= t.depth; ++l)
        for (int64_t b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b)
            for (int32_t q = t.v_ptr[b]; q < t.v_ptr[b + 1]; ++q) {
                const int32_t s = t.v_src[q];
                CHECK(s >= t.level_begin[l] && s < t.level_begin[l + 1]);
                CHECK(t.v_cls[q] >= 0 && t.v_cls[q] < NCLASS);
            }
    // M2L schedule over levels 2..L: every pair lands in exactly one chunk slot
    if (t.depth >= 2) {
        const int64_t b0 = t.level_begin[2], nb = t.n_box() - b0;
        std::vector<int32_t> group(nb);
        std::vector<double> scale(t.depth - 1);
        for (int l = 2; l <= t.depth; ++l) {
            scale[l - 2] = 1.0 / t.half_width(l);
            for (int64_t b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b) group[b - b0] = l - 2;
        }
        TileCost w;
        w.per_block = 0.5;
        w.per_target = 0.05;
        GGSched s;
        s.cp = 32;
        const std::vector<int64_t> cuts = chunk_cuts(nb, &t.v_ptr[b0], t.v_cls.data(), group.data(), 32, 1, 64, 300, w);
        gg_build(s, b0, nb, &t.v_ptr[b0], t.v_src.data(), t.v_cls.data(), group.data(), scale, cuts);
        int64_t slots = 0;
        for (int32_t v : s.chunk_src) slots += v >= 0;
        CHECK(slots == (int64_t)t.v_src.size());
        CHECK(s.max_tile <= 300);
    }
    HostOps o = build_host_ops(4, 1e-6, leaf, 0.5, 1e-10, false);
    CHECK(o.n_eq == 56 && o.k > 0 && o.k <= 56);
    build_stage2(o, 10.0);
    CHECK(o.r2max >= 1 && o.r2max <= o.k);
    HostOps d = build_host_ops(4, 1e-6, leaf, 0.5, 1e-10, true);
    CHECK(d.k == 56);
    std::printf("%s: n=%lld depth=%d leaves=%lld boxes=%lld pairs=%zu k=%d r2max=%d\n", name, (long long)n, t.depth,
                (long long)t.n_leaf(), (long long)t.n_box(), t.v_src.size(), o.k, o.r2max);
}

// Adaptive tree: structure and list invariants (leaves partition the points,
// points within their leaf, near sources within one level, W/X duality).
static void run_adaptive(const std::vector<double>& pts, int leaf, const char* name) {
    const int64_t n = (int64_t)pts.size() / 3;
    HostTree t = build_adaptive_host_tree(pts.data(), n, leaf, 16);
    CHECK(t.adaptive && t.n == n && t.leaf_ptr.front() == 0 && t.leaf_ptr.back() == n);
    const int64_t nl = t.n_leaf();
    CHECK((int64_t)t.leaf_box.size() == nl && (int64_t)t.leaf_level.size() == nl);
    for (int64_t e = 0; e < nl; ++e) {
        CHECK(t.leaf_ptr[e] < t.leaf_ptr[e + 1]);
        CHECK(t.box_leaf[t.leaf_box[e]] == e);
        CHECK(t.leaf_ptr[e + 1] - t.leaf_ptr[e] <= leaf || t.leaf_level[e] == 16);
        CHECK(t.near_ptr[e + 1] - t.near_ptr[e] <= 64);
        for (int32_t q = t.near_ptr[e]; q < t.near_ptr[e + 1]; ++q) {
            const int32_t s = t.near_leaf[q];
            CHECK(s >= 0 && s < nl);
            if (s >= 0 && s < nl) CHECK(std::abs(t.leaf_level[s] - t.leaf_level[e]) <= 1);
            CHECK(t.near_code[q] >= 0 && t.near_code[q] < 3 * 729);
        }
    }
    for (double u : t.u) CHECK(std::fabs(u) <= 1.0);
    int64_t wx = 0;
    for (int32_t g : t.w_src) CHECK(g >= 0 && g < t.n_box());
    for (int64_t g = 0; g < t.n_box(); ++g)
        for (int32_t k = t.x_ptr[g]; k < t.x_ptr[g + 1]; ++k, ++wx) {
            const int32_t e = t.x_src[k];
            CHECK(e >= 0 && e < nl);
            bool found = false;
            for (int32_t q = t.w_ptr[e]; q < t.w_ptr[e + 1]; ++q) found |= t.w_src[q] == g;
            CHECK(found);
        }
    CHECK(wx == (int64_t)t.w_src.size());
    std::printf("%s (adaptive): n=%lld depth=%d leaves=%lld boxes=%lld v=%zu w=%zu\n", name, (long long)n, t.depth,
                (long long)nl, (long long)t.n_box(), t.v_src.size(), t.w_src.size());
}

int main() {
    std::mt19937_64 rng(1211);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    std::vector<double> cube, sphere;
    for (int i = 0; i < 3000; ++i)
        for (int a = 0; a < 3; ++a) cube.push_back(u(rng));
    for (int i = 0; i < 3000; ++i) {
        double x = u(rng), y = u(rng), z = u(rng);
        const double r = std::sqrt(x * x + y * y + z * z) + 1e-12;
        sphere.push_back(x / r);
        sphere.push_back(y / r);
        sphere.push_back(z / r);
    }
    // duplicates and a tight cluster
    for (int i = 0; i < 30; ++i)
        for (int a = 0; a < 3; ++a) sphere.push_back(sphere[a]);
    run(cube, 32, "cube");
    run(sphere, 16, "sphere+duplicates");
    // a tight cluster in a sparse background: leaves over many levels
    std::vector<double> clus(cube.begin(), cube.begin() + 3 * 500);
    std::normal_distribution<double> g(0.0, 0.01);
    for (int i = 0; i < 2000; ++i)
        for (int a = 0; a < 3; ++a) clus.push_back(0.5 + g(rng));
    run_adaptive(clus, 16, "cluster");
    run_adaptive(sphere, 16, "sphere+duplicates");
    try {
        std::vector<double> bad{0.0, 0.0, NAN};
        build_host_tree(bad.data(), 1, 8, 0, 16);
        CHECK(false);
    } catch (const PlanError&) {
    }
    std::printf("%s\n", fails ? "FAILED" : "OK");
    return fails ? 1 : 0;
}
