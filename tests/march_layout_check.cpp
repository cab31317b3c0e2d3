// Host check of the row-marching task layout (march_layout.h): for many grid shapes, depths, lane
// widths, device sizes and segment minimums, every band's segments tile its rows exactly once, the
// stored columns of the bands cover every column, bands that start or end at the grid's sides load
// inside it, the middle segments of a zoned layout stay r * levels rows from the grid's top and
// bottom, and the task count fits 32 bits.  Prints one line and exits 0 on success.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../paper_2605_07954_amd/csrc/march_layout.h"

using st::march::BandCols;
using st::march::TaskMap;
using st::march::TaskRows;

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64() {  // splitmix64
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static int64_t pick(int64_t lo, int64_t hi) { return lo + int64_t(next_u64() % uint64_t(hi - lo + 1)); }

static int fail(const char* what, int64_t rows, int64_t cols, int V, int r, int levels, int64_t waves, int64_t seg_min,
                int zs) {
    std::printf("FAIL %s: rows %lld cols %lld V %d r %d levels %d waves %lld seg_min %lld zero_sides %d\n", what,
                (long long)rows, (long long)cols, V, r, levels, (long long)waves, (long long)seg_min, zs);
    return 1;
}

int main() {
    const int64_t row_set[] = {1, 2, 3, 5, 7, 8, 9, 13, 40, 97, 129, 300, 512, 1000, 2050, 8192, 16384};
    const int64_t waves_set[] = {256, 2048, 3072, 4096, 5120, 8192};
    long configs = 0, tasks_total = 0;
    for (int it = 0; it < 6000; ++it) {
        const int V = it % 3 == 0 ? 1 : it % 3 == 1 ? 4 : 8;
        const int r = int(pick(1, 4));
        const int levels = int(pick(1, 8));
        const int H = st::march::halo_lanes(r, levels, V);
        if (64 - 2 * H < 2) continue;
        const bool box = next_u64() & 1;
        const int taps = box ? (2 * r + 1) * (2 * r + 1) : 4 * r + 1;
        const int64_t rows = next_u64() % 3 ? row_set[next_u64() % 17] : pick(1, 20000);
        int64_t cols = next_u64() % 2 ? pick(1, 6000) : pick(1, 40) * 64 * V + pick(0, 64 * V);
        if (V > 1) cols = std::max<int64_t>(V, cols / V * V);  // whole lanes, as the vector kernels need
        const int64_t waves = waves_set[next_u64() % 6];
        const int64_t seg_min_set[] = {0, 0, 3, 7, 40, rows, 3 * rows};
        const int64_t seg_min = seg_min_set[next_u64() % 7];
        const bool zs = cols >= 2 * 64 * V && (next_u64() & 1);
        TaskMap m{};
        if (!st::march::plan_march_tasks(m, rows, cols, V, r, levels, taps, waves, seg_min, zs))
            return fail("no layout", rows, cols, V, r, levels, waves, seg_min, zs);
        if (m.tasks <= 0 || m.tasks >= (int64_t(1) << 31)) return fail("task count", rows, cols, V, r, levels, waves, seg_min, zs);
        std::vector<std::vector<std::pair<int64_t, int64_t>>> seg(size_t(m.bands));
        const int64_t reach = int64_t(r) * levels;
        for (int64_t t = 0; t < m.tasks; ++t) {
            const TaskRows tr = st::march::task_rows(m, t);
            if (tr.band < 0 || tr.band >= m.bands || tr.y0 < 0 || tr.y0 >= tr.y1 || tr.y1 > rows)
                return fail("task rows", rows, cols, V, r, levels, waves, seg_min, zs);
            seg[size_t(tr.band)].push_back({tr.y0, tr.y1});
            // a zoned layout's middle segments (seg rows, not at the grid's ends) take no edge checks
            if (m.ends_first && t >= m.tasks_outer && tr.y1 - tr.y0 == m.seg && m.seg != m.seg_short &&
                (tr.y0 < reach || tr.y1 > rows - reach) && rows > 2 * reach + m.seg)
                return fail("middle segment in an edge zone", rows, cols, V, r, levels, waves, seg_min, zs);
        }
        for (auto& s : seg) {
            std::sort(s.begin(), s.end());
            int64_t pos = 0;
            for (auto& q : s) {
                if (q.first != pos) return fail("rows not tiled", rows, cols, V, r, levels, waves, seg_min, zs);
                pos = q.second;
            }
            if (pos != rows) return fail("rows not covered", rows, cols, V, r, levels, waves, seg_min, zs);
        }
        // columns: the union of the bands' stored lanes covers [0, cols)
        std::vector<int64_t> lo_hi;
        std::vector<std::pair<int64_t, int64_t>> spans;
        for (int b = 0; b < m.bands; ++b) {
            const BandCols c = st::march::band_cols(m, b, V, H);
            const int lo = c.lo < 0 ? H : c.lo, hi = c.hi < 0 ? 64 - H : c.hi;
            if (m.zero_sides && (c.x0 < 0 || c.x0 + 64 * V > cols))
                return fail("zero-side band loads outside the grid", rows, cols, V, r, levels, waves, seg_min, zs);
            spans.push_back({std::max<int64_t>(0, c.x0 + int64_t(V) * lo), std::min<int64_t>(cols, c.x0 + int64_t(V) * hi)});
        }
        std::sort(spans.begin(), spans.end());
        int64_t covered = 0;
        for (auto& q : spans) {
            if (q.first > covered) return fail("columns not covered", rows, cols, V, r, levels, waves, seg_min, zs);
            covered = std::max(covered, q.second);
        }
        if (covered < cols) return fail("last columns not covered", rows, cols, V, r, levels, waves, seg_min, zs);
        ++configs;
        tasks_total += m.tasks;
    }
    std::printf("ok: %ld layouts, %ld tasks\n", configs, tasks_total);
    return 0;
}
