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
// H = ceil(r tb / V) halo lanes per side (with a halo of +0 the bands at the grid's sides write
// theirs too, see march_layout.h).  A wavefront lowers its priority as its task progresses, so the
// tasks sharing a SIMD finish together (march_body.h).
//
// Segments are sized on the host so that the number of (band, segment) tasks is close to the number
// of wavefronts the device holds at once: every wavefront runs one task of about equal duration (the
// tasks that take the grid's edge checks get proportionally shorter segments, see march_layout.h).  A
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

MarchFn march_lookup(int storage, int mode, int shape, int r, int levels, bool xbc, bool periodic) {
    const bool box = shape == SHAPE_BOX;
    if (xbc) {
        if (storage == ST_F32)
            return box ? march_lookup_xbc_f32_box(mode, r, levels, periodic) : march_lookup_xbc_f32_star(mode, r, levels, periodic);
        if (storage == ST_BF16)
            return box ? march_lookup_xbc_bf16_box(mode, r, levels, periodic) : march_lookup_xbc_bf16_star(mode, r, levels, periodic);
        if (storage == ST_F16)
            return box ? march_lookup_xbc_f16_box(mode, r, levels, periodic) : march_lookup_xbc_f16_star(mode, r, levels, periodic);
        return nullptr;
    }
    if (storage == ST_F32) return box ? march_lookup_f32_box(mode, r, levels) : march_lookup_f32_star(mode, r, levels);
    if (storage == ST_BF16) return box ? march_lookup_bf16_box(mode, r, levels) : march_lookup_bf16_star(mode, r, levels);
    if (storage == ST_F16) return box ? march_lookup_f16_box(mode, r, levels) : march_lookup_f16_star(mode, r, levels);
    return nullptr;
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
    MarchFn fn = march_lookup(p->storage, mode, p->shape, p->radius, levels, xbc, p->bc == ST_BC_PERIODIC);
    if (!fn) return fail(ST_EUNSUPPORTED, "no row-marching kernel for this shape/radius/depth");
    MarchArgs a;
    a.src = src;
    a.dst = dst;
    a.b = p->bq;
    a.bc = p->bc;
    a.frame = p->frame;
    a.stop = p->stop;
    std::memcpy(a.w, p->w, sizeof(a.w));
    // A constant halo of +0 with whole-lane accesses (vector, or one column per lane): the first
    // band starts at column 0 and the last ends at the last column (march_layout.h).
    const float zero = 0.0f;
    const bool zero_sides =
        !xbc && mode != 0 && std::memcmp(&p->bq, &zero, sizeof(float)) == 0 && p->cols >= 2 * 64 * V;
    int blocks = 0;
    if (int rc = resident_blocks(reinterpret_cast<const void*>(fn), 0, &blocks)) return rc;
    const int taps = p->shape == SHAPE_STAR ? 4 * p->radius + 1 : (2 * p->radius + 1) * (2 * p->radius + 1);
    if (!march::plan_march_tasks(a.map, p->rows, p->cols, V, p->radius, levels, taps, int64_t(blocks) * MWAVES,
                                 p->seg_min, zero_sides))
        return fail(ST_EUNSUPPORTED, "too many marching tasks for one pass");
    const int64_t grid = (a.map.tasks + MWAVES - 1) / MWAVES;
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(grid)), dim3(64 * MWAVES), 0, s, a);
    ST_LAUNCH_CHECK("sweep_march");
    return ST_OK;
}

}  // namespace st
