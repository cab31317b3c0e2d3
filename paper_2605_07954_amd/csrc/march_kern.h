// Row-marching kernels and their instantiation tables; included by one translation unit per
// storage type and shape (march_f32_star.hip, march_f32_box.hip, ...), which instantiate those
// kernels, and by march.hip for the launch arguments.  The design is described in march.hip.
#pragma once

#include "march_body.h"

namespace st {
namespace march_k {

using namespace march;

constexpr int MWAVES = 4;  // wavefronts per workgroup, each with its own task

struct MarchArgs {
    const void* src;
    void* dst;
    TaskMap map;        // how the pass's tasks cover the grid (march_layout.h)
    float b;
    int bc;             // boundary rule (march::BC_*)
    const int* stop;    // nullable: when it holds a nonzero value the pass does nothing
    const void* frame;  // BC_FRAME: the caller's halo frame
    float w[MAXK];
};

// Input rows a wavefront keeps in flight: one ring length (2r+1 rows, loaded that many iterations
// before use) wherever the registers allow; box r >= 3 with several levels needs them for its
// rings, and its long per-row arithmetic hides a one-row lead.
constexpr int fifo_rows(int R, int SHAPE, int TB) {
    return SHAPE == SHAPE_STAR || R <= 2 || TB == 1 ? 2 * R + 1 : 0;
}

template <int S, int R, int V, int SHAPE, int TB, bool VEC, int XBC>
__device__ __forceinline__ void sweep_march_body(const MarchArgs& a) {
    const int lane = int(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t task = int64_t(blockIdx.x) * MWAVES + wave;
    if (task >= a.map.tasks) return;
    if (a.stop && __hip_atomic_load(a.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    constexpr int H = halo_lanes(R, TB, V);
    const TaskRows tr = task_rows(a.map, task);
    const BandCols bc = band_cols(a.map, tr.band, V, H);
    const MarchView v{a.src, a.dst, a.map.rows, a.map.cols, a.b, a.bc, a.frame};
    march_task<S, R, V, SHAPE, TB, fifo_rows(R, SHAPE, TB), VEC, XBC>(v, a.w, lane, tr.y0, tr.y1, bc.x0, bc.lo, bc.hi);
}

template <int S, int R, int V, int SHAPE, int TB, bool VEC, int XBC>
__global__ __launch_bounds__(64 * MWAVES) void sweep_march(MarchArgs a) {
    sweep_march_body<S, R, V, SHAPE, TB, VEC, XBC>(a);
}

// r = 3 with two levels and four columns per lane needs about 174 registers, just over the 168
// that let three wavefronts share a SIMD; held to 168, the compiler keeps six values in scratch (one
// access per 192 FMAs), and the third wavefront hides more load latency than that costs (measured
// +2 % on box49).
template <int S, int R, int V, int SHAPE, int TB, bool VEC, int XBC>
__global__ __launch_bounds__(64 * MWAVES) __attribute__((amdgpu_waves_per_eu(3))) void sweep_march_w3(MarchArgs a) {
    sweep_march_body<S, R, V, SHAPE, TB, VEC, XBC>(a);
}

using MarchFn = void (*)(MarchArgs);

template <int S, int R, int V, int SH, int TB, bool VEC = true, int XBC = XBC_CONST>
MarchFn march_kernel() {
    if constexpr (V == 4 && R == 3 && TB == 2 && VEC) return sweep_march_w3<S, R, V, SH, TB, VEC, XBC>;
    else return sweep_march<S, R, V, SH, TB, VEC, XBC>;
}

// Depths per shape and radius: the rings of TB levels must fit the register file next to each
// other (a star ring row holds V values, a box ring row V + 2r).
template <int S, int V, int SH, bool VEC, int XBC = XBC_CONST>
MarchFn march_fn(int r, int levels) {
#define ST_MARCH(R, TB) \
    if (r == R && levels == TB) return march_kernel<S, R, V, SH, TB, VEC, XBC>();
    if constexpr (SH == SHAPE_STAR) {
        ST_MARCH(1, 1) ST_MARCH(1, 2) ST_MARCH(1, 3) ST_MARCH(1, 4) ST_MARCH(1, 5) ST_MARCH(1, 6) ST_MARCH(1, 7) ST_MARCH(1, 8)
        ST_MARCH(2, 1) ST_MARCH(2, 2) ST_MARCH(2, 3) ST_MARCH(2, 4) ST_MARCH(2, 5) ST_MARCH(2, 6)
        ST_MARCH(3, 1) ST_MARCH(3, 2) ST_MARCH(3, 3) ST_MARCH(3, 4)
        ST_MARCH(4, 1) ST_MARCH(4, 2) ST_MARCH(4, 3)
    } else {
        ST_MARCH(1, 1) ST_MARCH(1, 2) ST_MARCH(1, 3) ST_MARCH(1, 4) ST_MARCH(1, 5) ST_MARCH(1, 6)
        ST_MARCH(2, 1) ST_MARCH(2, 2) ST_MARCH(2, 3)
        ST_MARCH(3, 1) ST_MARCH(3, 2)
        ST_MARCH(4, 1) ST_MARCH(4, 2)
    }
#undef ST_MARCH
    return nullptr;
}

// Eight columns per lane: twice the arithmetic per lane shift, load and halo lane, and twice the
// ring registers, so the depths are lower.
template <int S, int SH>
MarchFn march8_fn(int r, int levels) {
#define ST_MARCH8(R, TB) \
    if (r == R && levels == TB) return march_kernel<S, R, 8, SH, TB>();
    if constexpr (SH == SHAPE_STAR) {
        ST_MARCH8(1, 1) ST_MARCH8(1, 2) ST_MARCH8(1, 3) ST_MARCH8(1, 4) ST_MARCH8(1, 5) ST_MARCH8(1, 6)
        ST_MARCH8(1, 7) ST_MARCH8(1, 8)
        ST_MARCH8(2, 1) ST_MARCH8(2, 2) ST_MARCH8(2, 3) ST_MARCH8(2, 4)
        ST_MARCH8(3, 1) ST_MARCH8(3, 2) ST_MARCH8(3, 3)
        ST_MARCH8(4, 1) ST_MARCH8(4, 2)
    } else {
        ST_MARCH8(1, 1) ST_MARCH8(1, 2) ST_MARCH8(1, 3)
        ST_MARCH8(2, 1) ST_MARCH8(2, 2)
        ST_MARCH8(3, 1) ST_MARCH8(3, 2)
        ST_MARCH8(4, 1)
    }
#undef ST_MARCH8
    return nullptr;
}

// The kernel of storage type S and shape SH for `mode` (8 or 4: that many columns per lane with
// vector accesses; 0: four columns per lane with element accesses; 1: one column per lane), radius
// and depth (nullptr if none).
template <int S, int SH>
MarchFn march_lookup_shape(int mode, int r, int levels) {
    if (mode == 8) return march8_fn<S, SH>(r, levels);
    if (mode == 4) return march_fn<S, 4, SH, true>(r, levels);
    if (mode == 1) return march_fn<S, 1, SH, true>(r, levels);
    return march_fn<S, 4, SH, false>(r, levels);
}

// The same kernels built with the periodic or the framed boundary rule in their edge tasks (four
// columns per lane with vector or element accesses, or one; no eight-column form).
template <int S, int SH, int XBC>
MarchFn march_lookup_shape_rule(int mode, int r, int levels) {
    if (mode == 4) return march_fn<S, 4, SH, true, XBC>(r, levels);
    if (mode == 1) return march_fn<S, 1, SH, true, XBC>(r, levels);
    if (mode == 0) return march_fn<S, 4, SH, false, XBC>(r, levels);
    return nullptr;
}
template <int S, int SH>
MarchFn march_lookup_shape_xbc(int mode, int r, int levels, bool periodic) {
    return periodic ? march_lookup_shape_rule<S, SH, XBC_PERIODIC>(mode, r, levels)
                    : march_lookup_shape_rule<S, SH, XBC_FRAME>(mode, r, levels);
}

}  // namespace march_k

// Lookups per storage type and shape, one per translation unit.
march_k::MarchFn march_lookup_f32_star(int mode, int r, int levels);
march_k::MarchFn march_lookup_f32_box(int mode, int r, int levels);
march_k::MarchFn march_lookup_bf16_star(int mode, int r, int levels);
march_k::MarchFn march_lookup_bf16_box(int mode, int r, int levels);
march_k::MarchFn march_lookup_f16_star(int mode, int r, int levels);
march_k::MarchFn march_lookup_f16_box(int mode, int r, int levels);
march_k::MarchFn march_lookup_xbc_f32_star(int mode, int r, int levels, bool periodic);
march_k::MarchFn march_lookup_xbc_f32_box(int mode, int r, int levels, bool periodic);
march_k::MarchFn march_lookup_xbc_bf16_star(int mode, int r, int levels, bool periodic);
march_k::MarchFn march_lookup_xbc_bf16_box(int mode, int r, int levels, bool periodic);
march_k::MarchFn march_lookup_xbc_f16_star(int mode, int r, int levels, bool periodic);
march_k::MarchFn march_lookup_xbc_f16_box(int mode, int r, int levels, bool periodic);

}  // namespace st
