// Task layout of the row-marching pass: how its (band, segment) tasks cover a grid.  Shared by the
// host, which sizes a pass, and the kernel, which maps its task index to rows and columns; the host
// side also compiles without a device (a CPU test checks that every layout covers its grid).
//
// A band is 64 lanes of V columns; the r * levels columns next to its loaded edge are exact only at
// the lower levels, so a band stores lanes [H, 64 - H) (H = halo_lanes), except that with a constant
// halo of +0 the lane shifts bring 0 into lanes 0 and 63, which is the halo's value at every level:
// then the first band starts at column 0 and stores its first H lanes too, and the last band ends at
// the last column and stores its last H ("zero sides": a grid needs up to two bands fewer and its
// side bands take no column checks).
//
// Tasks that take the edge checks (the two outer bands unless the sides are zero, and the segments
// within r * levels rows of the grid's top or bottom) spend about 1.5 more instructions per cell and
// level than the footprint's taps (measured: star r = 2 edge tasks run 17 % longer than inner ones
// of the same length).  A pass lasts as long as its slowest wavefront, so those tasks get segments
// of seg_short rows, with kappa (seg_short + lag) = seg + lag, kappa = 1 + 1.5 / taps and lag =
// 2r(levels - 1) the rows a task recomputes (in whole loop groups of 2r + 1 rows).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace st {
namespace march {

__host__ __device__ constexpr int halo_lanes(int R, int TB, int V) { return (R * TB + V - 1) / V; }

// Tasks: first the outer bands' (band 0 and bands - 1 alternating, segments of seg_short rows),
// then the inner bands' (task t: band band0 + t % inner, row of tasks q = t / inner).  An inner band
// runs n_top segments of seg_short rows from its top, then n_mid of seg rows, then n_bot of
// seg_short rows (the last one cut at the grid's end); with ends_first the rows of tasks q take the
// top segments, then the bottom ones, then the middle ones, else they go in order.  The short
// segments cover the rows that take the edge checks, and they come first: the oldest wavefronts on
// a SIMD are issued first.  (The uniform layout: no outer tasks, every band inner from band0 = 0,
// n_top = 0, segments of seg rows in order and the rest.)
struct TaskMap {
    int64_t rows, cols;
    int64_t tasks;
    int64_t tasks_outer;  // outer * ceil(rows / seg_short)
    int64_t seg;          // rows of an inner band's middle segments
    int64_t seg_short;    // rows of the segments at the grid's top and bottom and of the outer bands
    int n_top, n_mid, n_bot;
    int bands;
    int inner;       // inner bands
    int band0;       // the first inner band (1, or 0 when every band is inner)
    int outer;       // outer bands: 0, 1 or 2
    int ends_first;  // inner bands run their top and bottom segments first
    int zero_sides;  // see the top of this file
};

struct TaskRows {
    int64_t band, y0, y1;
};

// Band and output rows [y0, y1) of task `task` (< m.tasks).  Task indices fit 32 bits (checked on
// the host): one 32-bit division, on the path to the task's first load.
__host__ __device__ inline TaskRows task_rows(const TaskMap& m, int64_t task) {
    TaskRows r;
    if (task < m.tasks_outer) {
        const bool two = m.outer == 2;
        r.band = two && (task & 1) ? m.bands - 1 : 0;
        r.y0 = (two ? task >> 1 : task) * m.seg_short;
        r.y1 = r.y0 + m.seg_short < m.rows ? r.y0 + m.seg_short : m.rows;
        return r;
    }
    const uint32_t t = uint32_t(task - m.tasks_outer), q = t / uint32_t(m.inner);
    r.band = m.band0 + int64_t(t - q * uint32_t(m.inner));
    const uint32_t nt = uint32_t(m.n_top), nm = uint32_t(m.n_mid), nb = uint32_t(m.n_bot);
    // k: the segment's place from the top
    const uint32_t k = !m.ends_first || q < nt ? q : q < nt + nb ? q + nm : q - nb;
    int64_t len;
    if (k < nt) {
        r.y0 = int64_t(k) * m.seg_short;
        len = m.seg_short;
    } else if (k < nt + nm) {
        r.y0 = int64_t(nt) * m.seg_short + int64_t(k - nt) * m.seg;
        len = m.seg;
    } else {
        r.y0 = int64_t(nt) * m.seg_short + int64_t(nm) * m.seg + int64_t(k - nt - nm) * m.seg_short;
        len = m.seg_short;
    }
    r.y1 = r.y0 + len < m.rows ? r.y0 + len : m.rows;
    return r;
}

struct BandCols {
    int64_t x0;  // first loaded column (negative: the band starts in the halo)
    int lo, hi;  // stored lanes [lo, hi); -1: the default [H, 64 - H)
};

// Columns of band `band` with V columns per lane and H halo lanes.  With zero sides the bands
// between the first and the last follow the first at V (64 - 2H) columns each, the last of them
// moved left where it would pass the last band's end (the overlap stores the same values).
__host__ __device__ inline BandCols band_cols(const TaskMap& m, int64_t band, int V, int H) {
    const int64_t outw = int64_t(V) * (64 - 2 * H);
    BandCols c{band * outw - int64_t(V) * H, -1, -1};
    if (m.zero_sides) {
        const int64_t last = m.cols - 64 * int64_t(V);
        if (band == 0) {
            c.x0 = 0;
            c.lo = 0;
        } else if (band == m.bands - 1) {
            c.x0 = last;
            c.hi = 64;
        } else {
            c.x0 = (band - 1) * outw + int64_t(V) * (64 - 2 * H);
            if (c.x0 > last) c.x0 = last;
        }
    }
    return c;
}

// ---- host side: choosing a layout

// Every band split into segments of seg rows, in order, bands minor.  Returns false when a band
// would need 2^31 segments or more.
inline bool uniform_map(TaskMap& m, int64_t seg) {
    if (m.rows / seg + 1 >= (int64_t(1) << 31)) return false;
    m.seg = m.seg_short = seg;
    m.n_top = 0;
    m.n_mid = int(m.rows / seg);
    m.n_bot = m.rows % seg ? 1 : 0;
    m.inner = m.bands;
    m.band0 = 0;
    m.outer = 0;
    m.ends_first = 0;
    m.tasks_outer = 0;
    m.tasks = int64_t(m.bands) * (m.n_mid + m.n_bot);
    return true;
}

// Short segments (seg - cut rows) for the outer bands (`outer_edges`) and over the `reach` rows at
// an inner band's top and bottom; the middle segments, of seg rows, then take no edge checks.
// Returns false when a band would need 2^31 segments or more.
inline bool zoned_map(TaskMap& m, int64_t seg, int64_t cut, int64_t reach, bool outer_edges) {
    const int64_t rows = m.rows, ss = std::max<int64_t>(seg - cut, 1);
    m.seg = seg;
    m.seg_short = ss;
    m.inner = !outer_edges ? m.bands : m.bands >= 3 ? m.bands - 2 : 0;
    m.band0 = outer_edges ? 1 : 0;
    m.outer = !outer_edges ? 0 : m.bands >= 2 ? 2 : 1;
    m.ends_first = 1;
    int64_t nt = std::max<int64_t>(1, (reach + ss - 1) / ss), nm = 0, nb = 0;
    if (nt * ss >= rows) {  // short segments only
        nt = (rows + ss - 1) / ss;
    } else {
        // middle segments end at least `reach` rows above the grid's end; the rest (at least `reach`
        // rows, or all that is left) is cut into short ones
        const int64_t top = nt * ss;
        nm = std::max<int64_t>(0, (rows - top - reach) / seg);
        nb = (rows - top - nm * seg + ss - 1) / ss;
    }
    if (nt + nm + nb >= (int64_t(1) << 31)) return false;
    m.n_top = int(nt);
    m.n_mid = int(nm);
    m.n_bot = int(nb);
    m.tasks_outer = m.outer ? m.outer * ((rows + ss - 1) / ss) : 0;
    m.tasks = m.tasks_outer + int64_t(m.inner) * (nt + nm + nb);
    return true;
}

// The layout of one pass: `waves` wavefronts the device holds at once, `seg_min` the plan's least
// segment, `zero_sides` as above (the caller decides it: a constant halo of +0 and whole-lane
// accesses, cols >= 2 * 64 V), `taps` the footprint's taps.  Returns false when the pass would need
// 2^31 tasks or more.
inline bool plan_march_tasks(TaskMap& m, int64_t rows, int64_t cols, int V, int r, int levels, int taps,
                             int64_t waves, int64_t seg_min, bool zero_sides) {
    constexpr double edge_cost = 1.5;  // extra instructions per cell and level of an edge task
    const int H = halo_lanes(r, levels, V);
    const int64_t outw = int64_t(V) * (64 - 2 * H);
    m.rows = rows;
    m.cols = cols;
    m.zero_sides = zero_sides;
    int64_t bands = (cols + outw - 1) / outw;
    if (zero_sides) {
        const int64_t sides = 2 * int64_t(V) * (64 - H);
        bands = 2 + (cols > sides ? (cols - sides + outw - 1) / outw : 0);
    }
    if (bands >= (int64_t(1) << 31)) return false;
    m.bands = int(bands);
    const int64_t per_band = std::max<int64_t>(1, waves / bands);  // segments per band
    const int64_t natural = (rows + per_band - 1) / per_band;
    // a segment recomputes r (levels - 1) rows of the lower levels at either end: on small grids
    // longer segments (fewer tasks than wavefronts) cost less than the recomputation they avoid
    int64_t seg = std::max<int64_t>(natural, std::min<int64_t>(seg_min, rows));
    // A task's row loop runs whole groups of 2r + 1 iterations (seg + lag of them, rounded up), so
    // the segment is rounded up to fill its last group: every task runs the same iterations as
    // before and there are fewer tasks (rounding down measured slower even on small grids, where
    // the extra tasks cost more than the shorter ones save).
    const int64_t ring = 2 * r + 1, lag = 2 * int64_t(r) * (levels - 1), reach = int64_t(r) * levels;
    const int64_t part = (seg + lag) % ring;
    if (part && seg < rows) seg += ring - part;
    const double kappa = 1.0 + edge_cost / taps;
    int64_t groups = std::llround(double(seg + lag) * (1.0 - 1.0 / kappa) / double(ring));
    // Segments raised by the plan's minimum (small grids, fewer tasks than wavefronts: the tuner has
    // weighed segment length against task count) keep the uniform layout, unless the sides are zero
    // (then only the few segments at the grid's top and bottom get shorter).  The shorter segments
    // add tasks: give up groups of the cut until they fit the wavefronts the device holds at once,
    // else keep the uniform layout.
    if (seg_min > natural && !zero_sides) groups = 0;
    if (!uniform_map(m, seg)) return false;
    const int64_t uniform_tasks = m.tasks;
    for (; groups > 0; --groups) {
        if (groups * ring >= seg) continue;
        TaskMap c = m;
        if (zoned_map(c, seg, groups * ring, reach, !zero_sides) && c.tasks <= std::max(waves, uniform_tasks)) {
            m = c;
            break;
        }
    }
    return m.tasks < (int64_t(1) << 31);
}

}  // namespace march
}  // namespace st
