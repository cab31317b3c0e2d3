// Row-marching Jacobi pass (paper Sec. II-C update with the fixed halo of Sec. IV-A; per cell the
// FP32 order of Sec. IV-E: the centre product, then one FMA per footprint tap in row-major order, the
// same order as the tiled kernels, so results agree bit for bit).  Fields may be stored as FP32,
// BF16 or FP16; arithmetic is FP32 and every level is rounded to the storage type.
//
// One wavefront owns a band of columns, V per lane (V = 4 with one 16-byte or 8-byte load per lane
// and row; V = 1 with one element per lane, for any width and alignment), and walks down a segment
// of rows.  Each input row is read from HBM once per band; the r columns a lane needs on either side
// come from neighbouring lanes through DPP wave shifts (the value at column c < 0 is the previous
// lane's value at column c + V, so the side columns are produced nearest first, one shift each),
// and the pass uses neither LDS nor barriers.  The rows a lane needs sit in a register ring whose
// slots become fixed registers because the row loop is unrolled over the ring length.  With several
// levels per pass further rings hold the intermediate levels.  Level l is exact on columns at
// least r*l away from the band's loaded edge, so a band writes V (64 - 2 H) columns with
// H = ceil(r tb / V) halo lanes per side.
//
// Segments are sized on the host so that the number of (band, segment) tasks is close to the number
// of wavefronts the device holds at once: every wavefront runs one task of equal length.

#include <algorithm>

#include "march_body.h"

namespace st {
namespace {

using namespace march;

constexpr int MWAVES = 4;  // wavefronts per workgroup, each with its own task

struct MarchArgs {
    const void* src;
    void* dst;
    int64_t rows, cols;
    int64_t tasks;  // bands * segments
    int64_t seg;    // output rows per task
    int bands;
    float b;
    float w[MAXK];
};

// Input rows a wavefront keeps in flight: one ring length (2r+1 rows, loaded that many iterations
// before use) wherever the registers allow; box r >= 3 with several levels needs them for its
// rings, and its long per-row arithmetic hides a one-row lead.
constexpr int fifo_rows(int R, int SHAPE, int TB) {
    return SHAPE == SHAPE_STAR || R <= 2 || TB == 1 ? 2 * R + 1 : 0;
}

template <int S, int R, int V, int SHAPE, int TB>
__device__ __forceinline__ void sweep_march_body(const MarchArgs& a) {
    const int lane = int(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t task = int64_t(blockIdx.x) * MWAVES + wave;
    if (task >= a.tasks) return;
    constexpr int H = halo_lanes(R, TB, V);
    constexpr int OUTW = V * (64 - 2 * H);
    const int64_t band = task % a.bands;
    const int64_t y0 = (task / a.bands) * a.seg;
    const int64_t y1 = y0 + a.seg < a.rows ? y0 + a.seg : a.rows;
    const int64_t X0 = band * OUTW - V * H;
    const MarchView v{a.src, a.dst, a.rows, a.cols, a.b};
    march_task<S, R, V, SHAPE, TB, fifo_rows(R, SHAPE, TB)>(v, a.w, lane, y0, y1, X0);
}

template <int S, int R, int V, int SHAPE, int TB>
__global__ __launch_bounds__(64 * MWAVES) void sweep_march(MarchArgs a) {
    sweep_march_body<S, R, V, SHAPE, TB>(a);
}

// r = 3 with two levels and four columns per lane needs about 174 registers, just over the 168
// that let three wavefronts share a SIMD; held to 168, the compiler keeps six values in scratch (one
// access per 192 FMAs), and the third wavefront hides more load latency than that costs (measured
// +2 % on box49).
template <int S, int R, int V, int SHAPE, int TB>
__global__ __launch_bounds__(64 * MWAVES) __attribute__((amdgpu_waves_per_eu(3))) void sweep_march_w3(MarchArgs a) {
    sweep_march_body<S, R, V, SHAPE, TB>(a);
}

using MarchFn = void (*)(MarchArgs);

template <int S, int R, int V, int SH, int TB>
MarchFn march_kernel() {
    if constexpr (V == 4 && R == 3 && TB == 2) return sweep_march_w3<S, R, V, SH, TB>;
    else return sweep_march<S, R, V, SH, TB>;
}

// Depths per shape and radius: the rings of TB levels must fit the register file next to each
// other (a star ring row holds V values, a box ring row V + 2r).
template <int S, int V, int SH>
MarchFn march_fn(int r, int levels) {
#define ST_MARCH(R, TB) \
    if (r == R && levels == TB) return march_kernel<S, R, V, SH, TB>();
    if constexpr (SH == SHAPE_STAR) {
        ST_MARCH(1, 1) ST_MARCH(1, 2) ST_MARCH(1, 3) ST_MARCH(1, 4) ST_MARCH(1, 5) ST_MARCH(1, 6) ST_MARCH(1, 7) ST_MARCH(1, 8)
        ST_MARCH(2, 1) ST_MARCH(2, 2) ST_MARCH(2, 3) ST_MARCH(2, 4) ST_MARCH(2, 5) ST_MARCH(2, 6)
        ST_MARCH(3, 1) ST_MARCH(3, 2) ST_MARCH(3, 3) ST_MARCH(3, 4)
        ST_MARCH(4, 1) ST_MARCH(4, 2) ST_MARCH(4, 3)
    } else {
        ST_MARCH(1, 1) ST_MARCH(1, 2) ST_MARCH(1, 3) ST_MARCH(1, 4)
        ST_MARCH(2, 1) ST_MARCH(2, 2) ST_MARCH(2, 3)
        ST_MARCH(3, 1) ST_MARCH(3, 2)
        ST_MARCH(4, 1) ST_MARCH(4, 2)
    }
#undef ST_MARCH
    return nullptr;
}

template <int S, int V>
MarchFn march_lookup_s(int shape, int r, int levels) {
    return shape == SHAPE_BOX ? march_fn<S, V, SHAPE_BOX>(r, levels) : march_fn<S, V, SHAPE_STAR>(r, levels);
}

MarchFn march_lookup(int storage, int V, int shape, int r, int levels) {
    if (V == 4) {
        if (storage == ST_F32) return march_lookup_s<ST_F32, 4>(shape, r, levels);
        if (storage == ST_BF16) return march_lookup_s<ST_BF16, 4>(shape, r, levels);
        if (storage == ST_F16) return march_lookup_s<ST_F16, 4>(shape, r, levels);
    } else {
        if (storage == ST_F32) return march_lookup_s<ST_F32, 1>(shape, r, levels);
        if (storage == ST_BF16) return march_lookup_s<ST_BF16, 1>(shape, r, levels);
        if (storage == ST_F16) return march_lookup_s<ST_F16, 1>(shape, r, levels);
    }
    return nullptr;
}

}  // namespace

int march_max_tb(int shape, int radius) {
    if (shape == SHAPE_STAR) return radius == 1 ? 8 : radius == 2 ? 6 : radius == 3 ? 4 : 3;
    return radius == 1 ? 4 : radius == 2 ? 3 : 2;
}

bool march_usable(const st_plan* p) { return p->kind == KIND_CONST && p->radius <= 4; }

int launch_march(const st_plan* p, const void* src, void* dst, int levels, hipStream_t s) {
    // four columns per lane when every row starts on a 16-byte boundary (cols % 4 == 0 and aligned
    // buffers; a 16-bit row of four cells is 8 bytes, which the same condition covers); else one
    const bool wide = p->cols % 4 == 0 && (reinterpret_cast<uintptr_t>(src) % 16) == 0 &&
                      (reinterpret_cast<uintptr_t>(dst) % 16) == 0;
    const int V = wide ? 4 : 1;
    MarchFn fn = march_lookup(p->storage, V, p->shape, p->radius, levels);
    if (!fn) return fail(ST_EUNSUPPORTED, "no row-marching kernel for this shape/radius/depth");
    MarchArgs a;
    a.src = src;
    a.dst = dst;
    a.rows = p->rows;
    a.cols = p->cols;
    a.b = p->bq;
    std::memcpy(a.w, p->w, sizeof(a.w));
    const int64_t outw = V * (64 - 2 * halo_lanes(p->radius, levels, V));
    a.bands = int((p->cols + outw - 1) / outw);
    int blocks = 0;
    if (int rc = resident_blocks(reinterpret_cast<const void*>(fn), 0, &blocks)) return rc;
    const int64_t waves = int64_t(blocks) * MWAVES;
    const int64_t per_band = std::max<int64_t>(1, waves / a.bands);  // segments per band
    a.seg = (p->rows + per_band - 1) / per_band;
    const int64_t segs = (p->rows + a.seg - 1) / a.seg;
    a.tasks = segs * a.bands;
    const int64_t grid = (a.tasks + MWAVES - 1) / MWAVES;
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(grid)), dim3(64 * MWAVES), 0, s, a);
    ST_LAUNCH_CHECK("sweep_march");
    return ST_OK;
}

}  // namespace st
