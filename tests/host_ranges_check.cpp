// Host check of kifmm::split_tile_ranges, the tile ranges over which the
// second stage-2 phase is launched so that each launch's products stay within
// 32-bit buffer offsets. Built and run by tests/test_host_ranges.py.
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_1211_2517_amd/csrc/plan.h"

using kifmm::split_tile_ranges;

int main() {
    std::mt19937 rng(7);
    int bad = 0;
    for (int trial = 0; trial < 2000; ++trial) {
        const int nt = 1 + (int)(rng() % 60);
        std::vector<int32_t> c0{0};
        for (int t = 0; t < nt; ++t) c0.push_back(c0.back() + (int)(rng() % 50));   // empty tiles allowed
        const int cp = 1 + (int)(rng() % 32);
        const int64_t sb = 1 + (int64_t)(rng() % 100);
        const int64_t max_bytes = 1 + (int64_t)(rng() % 200000), max_slots = 1 + (int64_t)(rng() % 3000);
        const std::vector<int> r = split_tile_ranges(c0, cp, sb, max_bytes, max_slots);
        auto fits = [&](int a, int b) {
            const int64_t s = (int64_t)(c0[b] - c0[a]) * cp;
            return s * sb < max_bytes && s < max_slots;
        };
        bool each = true;
        for (int t = 0; t < nt; ++t) each = each && fits(t, t + 1);
        if (!each) {
            bad += !r.empty();   // a tile that does not fit alone: refused
            continue;
        }
        if (r.size() < 2 || r.front() != 0 || r.back() != nt) {
            ++bad;
            continue;
        }
        for (size_t i = 0; i + 1 < r.size(); ++i) {
            bad += r[i + 1] <= r[i];                               // in order, nonempty
            bad += !fits(r[i], r[i + 1]);                          // each range fits
            bad += i + 2 < r.size() && fits(r[i], r[i + 1] + 1);   // and is the longest that fits
        }
    }
    // the 2^20-point sphere at p = 8: 512 tiles of 358 chunks of 32 slots,
    // FP32 rows of 96 values: 2.25 GB, two ranges below 2 GiB
    std::vector<int32_t> c0{0};
    for (int t = 0; t < 512; ++t) c0.push_back(c0.back() + 358);
    const std::vector<int> r = split_tile_ranges(c0, 32, 96 * 4, (int64_t(1) << 31) - (int64_t(1) << 20),
                                                 (int64_t(1) << 24) - 1);
    bad += r.size() != 3;
    std::printf("mismatches: %d; sphere p=8 ranges: %zu\n", bad, r.size() - 1);
    return bad != 0;
}
