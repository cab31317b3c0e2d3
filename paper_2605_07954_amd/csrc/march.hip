// Row-marching Jacobi pass (paper Sec. II-C update with the fixed halo of Sec. IV-A; per cell the
// FP32 order of Sec. IV-E: the centre product, then one FMA per footprint tap in row-major order, the
// same order as the tiled kernels, so results agree bit for bit).  Fields may be stored as FP32,
// BF16 or FP16; arithmetic is FP32 and every level is rounded to the storage type.
//
// One wavefront owns a band of columns, V per lane (V = 8 or 4 with one or two 16-byte loads, or one
// 8-byte load, per lane and row; for any other width or alignment V = 4 with one element access
// per column; or V = 1, many short tasks for small grids), and walks down a segment of rows.  Each
// input row is read from HBM once per band; the r columns a lane needs on either side
// come from neighbouring lanes through DPP wave shifts (the value at column c < 0 is the previous
// lane's value at column c + V, so the side columns are produced nearest first, one shift each),
// and the pass uses neither LDS nor barriers.  The rows a lane needs sit in a register ring whose
// slots become fixed registers because the row loop is unrolled over the ring length.  With several
// levels per pass further rings hold the intermediate levels.  Level l is exact on columns at
// least r*l away from the band's loaded edge, so a band writes V (64 - 2 H) columns with
// H = ceil(r tb / V) halo lanes per side.
//
// Segments are sized on the host so that the number of (band, segment) tasks is close to the number
// of wavefronts the device holds at once: every wavefront runs one task of about equal duration (the
// tasks that take the grid's edge checks get proportionally shorter segments, see march_layout).  A
// plan may ask for longer segments (stencil_set_march_segment), which the autotuner does for small
// grids.

#include <algorithm>
#include <cmath>

#include "march_kern.h"

namespace st {

using march_k::MarchArgs;
using march_k::MarchFn;
using march_k::MWAVES;

namespace {

MarchFn march_lookup(int storage, int mode, int shape, int r, int levels, bool xbc) {
    const bool box = shape == SHAPE_BOX;
    if (xbc) {
        if (storage == ST_F32) return box ? march_lookup_xbc_f32_box(mode, r, levels) : march_lookup_xbc_f32_star(mode, r, levels);
        if (storage == ST_BF16)
            return box ? march_lookup_xbc_bf16_box(mode, r, levels) : march_lookup_xbc_bf16_star(mode, r, levels);
        if (storage == ST_F16) return box ? march_lookup_xbc_f16_box(mode, r, levels) : march_lookup_xbc_f16_star(mode, r, levels);
        return nullptr;
    }
    if (storage == ST_F32) return box ? march_lookup_f32_box(mode, r, levels) : march_lookup_f32_star(mode, r, levels);
    if (storage == ST_BF16) return box ? march_lookup_bf16_box(mode, r, levels) : march_lookup_bf16_star(mode, r, levels);
    if (storage == ST_F16) return box ? march_lookup_f16_box(mode, r, levels) : march_lookup_f16_star(mode, r, levels);
    return nullptr;
}

// How a pass's tasks cover the grid (see MarchArgs).
struct MarchLayout {
    int64_t seg, seg_short, tasks_outer, tasks;
    int64_t n_top, n_mid, n_bot;
    int inner, band0, outer, ends_first;
};

// Every band split into segments of seg rows, in order, bands minor.
MarchLayout uniform_layout(int64_t rows, int bands, int64_t seg) {
    MarchLayout L;
    L.seg = L.seg_short = seg;
    L.n_top = 0;
    L.n_mid = rows / seg;
    L.n_bot = rows % seg ? 1 : 0;
    L.inner = bands;
    L.band0 = 0;
    L.outer = 0;
    L.ends_first = 0;
    L.tasks_outer = 0;
    L.tasks = int64_t(bands) * (L.n_mid + L.n_bot);
    return L;
}

// Tasks that take the edge checks (the two outer bands, and the segments of an inner band that lie
// within `reach` = r * levels rows of the grid's top or bottom) spend about 1.5 more instructions
// per cell and level than the footprint's taps (measured: star r = 2 edge tasks run 17 % longer
// than inner ones of the same length).  A launch lasts as long as its slowest wavefront, so those
// tasks get segments of seg_short = seg - cut rows: the outer bands' segments, and the segments
// that cover an inner band's top and bottom `reach` rows; the middle segments, of seg rows, then
// take no edge checks.  `outer_edges`: the first and last bands take the column checks (else every
// band is inner).
MarchLayout march_layout(int64_t rows, int bands, int64_t seg, int64_t cut, int64_t reach, bool outer_edges) {
    MarchLayout L;
    L.seg = seg;
    const int64_t ss = L.seg_short = std::max<int64_t>(seg - cut, 1);
    L.inner = !outer_edges ? bands : bands >= 3 ? bands - 2 : 0;
    L.band0 = outer_edges ? 1 : 0;
    L.outer = !outer_edges ? 0 : bands >= 2 ? 2 : 1;
    L.ends_first = 1;
    L.n_top = std::max<int64_t>(1, (reach + ss - 1) / ss);
    if (L.n_top * ss >= rows) {  // short segments only
        L.n_top = (rows + ss - 1) / ss;
        L.n_mid = L.n_bot = 0;
    } else {
        // middle segments end at least `reach` rows above the grid's end; the rest (at least
        // `reach` rows, or all that is left) is cut into short ones
        const int64_t top = L.n_top * ss;
        L.n_mid = std::max<int64_t>(0, (rows - top - reach) / seg);
        L.n_bot = (rows - top - L.n_mid * seg + ss - 1) / ss;
    }
    L.tasks_outer = L.outer ? L.outer * ((rows + ss - 1) / ss) : 0;
    L.tasks = L.tasks_outer + int64_t(L.inner) * (L.n_top + L.n_mid + L.n_bot);
    return L;
}

}  // namespace

int march_max_tb(int shape, int radius, int vmax) {
    if (vmax == 8) {  // never deeper than the four-column kernels it falls back to
        if (shape == SHAPE_STAR) return radius == 1 ? 8 : radius == 2 ? 4 : radius == 3 ? 3 : 2;
        return radius == 1 ? 3 : radius == 2 ? 2 : radius == 3 ? 2 : 1;
    }
    if (shape == SHAPE_STAR) return radius == 1 ? 8 : radius == 2 ? 6 : radius == 3 ? 4 : 3;
    return radius == 1 ? 6 : radius == 2 ? 3 : 2;
}

bool march_usable(const st_plan* p) { return p->kind == KIND_CONST && p->radius <= 4; }

int launch_march(const st_plan* p, const void* src, void* dst, int levels, int vmax, hipStream_t s) {
    // V columns per lane with one vector access per lane and row when every row starts on a
    // 16-byte boundary (cols % V == 0 and aligned buffers; four 16-bit cells are 8 bytes, which the
    // same condition covers); else four columns per lane with element accesses (mode 0); vmax 1:
    // one column per lane, any width and alignment
    // (periodic and framed grids have no eight-column kernels: they take four columns per lane)
    const bool xbc = p->bc != ST_BC_CONST;
    if (xbc && vmax == 8) vmax = 4;
    const bool aligned = (reinterpret_cast<uintptr_t>(src) % 16) == 0 && (reinterpret_cast<uintptr_t>(dst) % 16) == 0;
    const int mode = vmax == 1 ? 1 : aligned && vmax == 8 && p->cols % 8 == 0 ? 8 : aligned && p->cols % 4 == 0 ? 4 : 0;
    const int V = mode == 8 ? 8 : mode == 1 ? 1 : 4;
    MarchFn fn = march_lookup(p->storage, mode, p->shape, p->radius, levels, xbc);
    if (!fn) return fail(ST_EUNSUPPORTED, "no row-marching kernel for this shape/radius/depth");
    MarchArgs a;
    a.src = src;
    a.dst = dst;
    a.rows = p->rows;
    a.cols = p->cols;
    a.b = p->bq;
    a.bc = p->bc;
    a.frame = p->frame;
    a.stop = p->stop;
    std::memcpy(a.w, p->w, sizeof(a.w));
    const int64_t H = march::halo_lanes(p->radius, levels, V), outw = V * (64 - 2 * H);
    a.bands = int((p->cols + outw - 1) / outw);
    // A constant halo of +0 with whole-lane accesses (vector, or one column per lane): the first
    // band starts at column 0 and the last ends at the last column, storing the lanes a halo would
    // otherwise take (see MarchArgs), so a grid needs up to two bands fewer and its side bands take
    // no column checks.
    const float zero = 0.0f;
    a.zero_sides = !xbc && mode != 0 && std::memcmp(&p->bq, &zero, sizeof(float)) == 0 && p->cols >= 2 * 64 * V;
    if (a.zero_sides) {
        const int64_t sides = 2 * V * (64 - H);
        a.bands = int(2 + (p->cols > sides ? (p->cols - sides + outw - 1) / outw : 0));
    }
    int blocks = 0;
    if (int rc = resident_blocks(reinterpret_cast<const void*>(fn), 0, &blocks)) return rc;
    const int64_t waves = int64_t(blocks) * MWAVES;
    const int64_t per_band = std::max<int64_t>(1, waves / a.bands);  // segments per band
    const int64_t natural = (p->rows + per_band - 1) / per_band;
    // a segment recomputes r (levels - 1) rows of the lower levels at either end: on small grids
    // longer segments (fewer tasks than wavefronts) cost less than the recomputation they avoid
    int64_t seg = std::max<int64_t>(natural, std::min<int64_t>(p->seg_min, p->rows));
    // A task's row loop runs whole groups of 2r + 1 iterations (seg + 2r(levels - 1) of them, rounded
    // up), so the segment is rounded up to fill its last group: every task runs the same iterations
    // as before and there are fewer tasks (rounding down measured slower even on small grids, where
    // the extra tasks cost more than the shorter ones save).
    const int64_t ring = 2 * p->radius + 1, part = (seg + 2 * p->radius * (levels - 1)) % ring;
    if (part && seg < p->rows) seg += ring - part;
    const int taps = p->shape == SHAPE_STAR ? 4 * p->radius + 1 : (2 * p->radius + 1) * (2 * p->radius + 1);

    const int64_t lag = 2 * p->radius * (levels - 1), reach = int64_t(p->radius) * levels;
    // an edge task of seg_short rows runs as long as an inner one of seg rows:
    // kappa (seg_short + lag) = seg + lag, kappa = 1 + 1.5 / taps (in whole loop groups)
    const double kappa = 1.0 + 1.5 / taps;
    int64_t groups = std::llround(double(seg + lag) * (1.0 - 1.0 / kappa) / double(ring));
    // Segments raised by the plan's minimum (small grids, fewer tasks than wavefronts: the tuner
    // has weighed segment length against task count) keep the uniform layout, unless the side
    // bands take no column checks (then only the few segments at the grid's top and bottom get
    // shorter).  The shorter segments add tasks: give up groups of the cut until they fit the
    // wavefronts the device holds at once, else keep the uniform layout.
    if (p->seg_min > natural && !a.zero_sides) groups = 0;
    MarchLayout L = uniform_layout(p->rows, a.bands, seg);
    for (; groups > 0; --groups) {
        if (groups * ring >= seg) continue;
        const MarchLayout C = march_layout(p->rows, a.bands, seg, groups * ring, reach, !a.zero_sides);
        if (C.tasks <= std::max(waves, L.tasks)) {
            L = C;
            break;
        }
    }
    if (L.n_top + L.n_mid + L.n_bot >= (int64_t(1) << 31) / std::max(1, L.inner))
        return fail(ST_EUNSUPPORTED, "too many marching tasks for one pass");
    a.seg = L.seg;
    a.seg_short = L.seg_short;
    a.n_top = int(L.n_top);
    a.n_mid = int(L.n_mid);
    a.n_bot = int(L.n_bot);
    a.inner = L.inner;
    a.outer = L.outer;
    a.tasks_outer = L.tasks_outer;
    a.band0 = L.band0;
    a.ends_first = L.ends_first;
    a.tasks = L.tasks;
    if (a.tasks >= (int64_t(1) << 31)) return fail(ST_EUNSUPPORTED, "too many marching tasks for one pass");
    const int64_t grid = (a.tasks + MWAVES - 1) / MWAVES;
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(grid)), dim3(64 * MWAVES), 0, s, a);
    ST_LAUNCH_CHECK("sweep_march");
    return ST_OK;
}

}  // namespace st
