// Device body of the row-marching Jacobi pass (paper Sec. II-C update with the fixed halo of
// Sec. IV-A; per cell the FP32 order of Sec. IV-E), shared by the single-grid kernel and the batched
// multi-grid kernel.  See march.hip for the design; this file holds the per-wavefront task:
// march_one (one level) and march_levels (TB >= 2 levels) walk one band of columns over a
// segment of rows.
#pragma once

#include "internal.h"
#include "storage.h"

namespace st {
namespace march {

// What a task needs of its grid.
struct MarchView {
    const void* src;
    void* dst;
    int64_t rows, cols;
    float b;  // halo value, already rounded to the storage type
};

__host__ __device__ constexpr int halo_lanes(int R, int TB, int V) { return (R * TB + V - 1) / V; }

// DPP wave shifts over the whole wavefront: lane l receives lane l-1 (resp. l+1); lane 0 (resp. 63)
// receives 0, which only feeds outputs that are never stored.
__device__ __forceinline__ float from_prev_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

// One ring row as seen by a lane: v[R + c] is the row's value at column c of the lane's V, for
// c in [-R, V + R).
template <int R, int V>
struct Row {
    float v[V + 2 * R];
};

template <int R, int V>
__device__ __forceinline__ void fill_sides(Row<R, V>& x) {
#pragma unroll
    for (int c = -1; c >= -R; --c) x.v[R + c] = from_prev_lane(x.v[R + c + V]);
#pragma unroll
    for (int c = V; c < V + R; ++c) x.v[R + c] = from_next_lane(x.v[R + c - V]);
}

__device__ __forceinline__ bool tap_on(int shape, int dy, int dx) { return shape == SHAPE_BOX || dy == 0 || dx == 0; }

template <int V>
struct Cells {
    float c[V];
};

// The V outputs of a lane for one row; `ring[(base + R + dy) % N]` holds input row dy.
template <int R, int V, int SHAPE, int N>
__device__ __forceinline__ Cells<V> apply(const Row<R, V>* ring, int base, const float* w) {
    constexpr int K = 2 * R + 1;
    Cells<V> o;
    const Row<R, V>& mid = ring[(base + R) % N];
#pragma unroll
    for (int c = 0; c < V; ++c) o.c[c] = w[R * K + R] * mid.v[R + c];
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
        const Row<R, V>& x = ring[(base + R + dy) % N];
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            if ((dy == 0 && dx == 0) || !tap_on(SHAPE, dy, dx)) continue;
            const float wt = w[(dy + R) * K + dx + R];
#pragma unroll
            for (int c = 0; c < V; ++c) o.c[c] = __builtin_fmaf(wt, x.v[R + c + dx], o.c[c]);
        }
    }
    return o;
}

// V consecutive cells of the storage type from element offset `off`, widened to FP32 (exact).
template <int S, int V>
__device__ __forceinline__ Cells<V> load_cells(const void* src, int64_t off) {
    Cells<V> q;
    if constexpr (V == 1) {
        q.c[0] = Fmt<S>::ld(static_cast<const typename Fmt<S>::T*>(src)[off]);
    } else if constexpr (S == ST_F32) {
        const float4 f = *reinterpret_cast<const float4*>(static_cast<const float*>(src) + off);
        q.c[0] = f.x; q.c[1] = f.y; q.c[2] = f.z; q.c[3] = f.w;
    } else {
        const uint2 h = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(src) + off);
        q.c[0] = Fmt<S>::ld(uint16_t(h.x & 0xffffu));
        q.c[1] = Fmt<S>::ld(uint16_t(h.x >> 16));
        q.c[2] = Fmt<S>::ld(uint16_t(h.y & 0xffffu));
        q.c[3] = Fmt<S>::ld(uint16_t(h.y >> 16));
    }
    return q;
}

template <int S, int V>
__device__ __forceinline__ void store_cells(void* dst, int64_t off, const Cells<V>& q) {
    using T = typename Fmt<S>::T;
    if constexpr (V == 1) {
        static_cast<T*>(dst)[off] = Fmt<S>::st(q.c[0]);
    } else {
        store4<S>(static_cast<T*>(dst) + off, q.c);
    }
}

template <int R, int V>
__device__ __forceinline__ void set_own(Row<R, V>& x, const Cells<V>& q) {
#pragma unroll
    for (int c = 0; c < V; ++c) x.v[R + c] = q.c[c];
}

// Loads one input row into `x` (own columns).  EDGE tasks may touch rows or columns outside the
// grid: those cells hold b.  Interior tasks only clamp the row of a prefetch past the grid's end.
template <int S, int R, int V, bool EDGE>
__device__ __forceinline__ void load_row(Row<R, V>& x, const void* src, int64_t gy, int64_t rows, int64_t cols,
                                         int64_t gx, bool col_in, float b) {
    Cells<V> q;
    if (EDGE) {
        if (gy >= 0 && gy < rows && col_in) {
            q = load_cells<S, V>(src, gy * cols + gx);
        } else {
#pragma unroll
            for (int c = 0; c < V; ++c) q.c[c] = b;
        }
    } else {
        const int64_t g = gy < rows ? gy : rows - 1;
        q = load_cells<S, V>(src, g * cols + gx);
    }
    set_own<R, V>(x, q);
}

// One level: output rows [y0, y1) of the band whose first loaded column is X0.
template <int S, int R, int V, int SHAPE, bool EDGE>
__device__ __forceinline__ void march_one(const MarchView& a, const float* w, int lane, int64_t y0, int64_t y1,
                                          int64_t X0) {
    constexpr int N = 2 * R + 2;  // window of 2R+1 rows plus one row in flight
    constexpr int H = halo_lanes(R, 1, V);
    const int64_t rows = a.rows, cols = a.cols;
    const int64_t gx = X0 + V * lane;
    const bool col_in = gx >= 0 && gx + V <= cols;  // V = 4 only with cols % 4 == 0: all or none
    const bool writer = lane >= H && lane < 64 - H && (!EDGE || col_in);
    const float b = a.b;
    Row<R, V> ring[N];
    const int64_t j0 = y0 - R;  // input row held by slot 0 at the start; row j lives in slot (j - j0) % N
#pragma unroll
    for (int t = 0; t < N; ++t) load_row<S, R, V, EDGE>(ring[t], a.src, j0 + t, rows, cols, gx, col_in, b);
#pragma unroll
    for (int t = 0; t < 2 * R; ++t) fill_sides<R, V>(ring[t]);
    for (int64_t k0 = y0; k0 < y1; k0 += N) {
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const int64_t k = k0 + u;
            if (k >= y1) break;
            fill_sides<R, V>(ring[(u + 2 * R) % N]);  // row k+R enters the window
            const Cells<V> o = apply<R, V, SHAPE, N>(ring, u, w);
            if (writer) store_cells<S, V>(a.dst, k * cols + gx, o);
            load_row<S, R, V, EDGE>(ring[u], a.src, k - R + N, rows, cols, gx, col_in, b);  // row k-R is done
        }
    }
}

// TB >= 2 levels.  Level l (0 = input, TB = output) keeps its own ring of N = 2R+1 rows.  Iteration i
// computes level-1 row m1 = y0 - R(TB-1) + i from the input rows m1-R .. m1+R, then, once enough rows
// of the level below exist, level-l row m1 - (l-1)R for l = 2 .. TB.  Within level l the row of
// iteration i sits in slot (i + l - 1) % N (because -2R = 1 mod N), so every slot index is a
// compile-time constant of the loop unrolled N times.
template <int S, int R, int V, int SHAPE, int TB, bool EDGE>
__device__ __forceinline__ void march_levels(const MarchView& a, const float* w, int lane, int64_t y0, int64_t y1,
                                             int64_t X0) {
    constexpr int N = 2 * R + 1;
    constexpr int H = halo_lanes(R, TB, V);
    const int64_t rows = a.rows, cols = a.cols;
    const int64_t gx = X0 + V * lane;
    const bool col_in = gx >= 0 && gx + V <= cols;
    const bool writer = lane >= H && lane < 64 - H && (!EDGE || col_in);
    const float b = a.b;
    Row<R, V> lv[TB][N];  // lv[0]: input rows; lv[l]: level l < TB (the output level is stored directly)
    const int64_t j0 = y0 - R * TB;  // input row in slot 0 at the start
#pragma unroll
    for (int t = 0; t < N; ++t) load_row<S, R, V, EDGE>(lv[0][t], a.src, j0 + t, rows, cols, gx, col_in, b);
#pragma unroll
    for (int t = 0; t < 2 * R; ++t) fill_sides<R, V>(lv[0][t]);
    const int64_t iters = (y1 - y0) + 2 * R * (TB - 1);
    for (int64_t i0 = 0; i0 < iters; i0 += N) {
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const int64_t i = i0 + u;
            if (i >= iters) break;
            fill_sides<R, V>(lv[0][(u + 2 * R) % N]);  // input row m1 + R enters the window
#pragma unroll
            for (int l = 1; l <= TB; ++l) {
                if (i < 2 * R * (l - 1)) break;  // level l - 1 does not have 2R+1 rows yet
                const int64_t m = y0 - R * (TB - 1) + i - int64_t(l - 1) * R;  // row of level l
                Cells<V> q = apply<R, V, SHAPE, N>(lv[l - 1], u + l - 1, w);
                if (l == TB) {
                    if (writer) store_cells<S, V>(a.dst, m * cols + gx, q);
                } else {
                    Row<R, V>& x = lv[l][(u + l - 1) % N];
                    // every level is rounded to the storage type; cells outside the grid keep b
                    const bool inside = !EDGE || (m >= 0 && m < rows && col_in);
#pragma unroll
                    for (int c = 0; c < V; ++c) q.c[c] = inside ? Fmt<S>::rnd(q.c[c]) : b;
                    set_own<R, V>(x, q);
                    fill_sides<R, V>(x);
                }
                if (l == 1)  // input row m1 - R is no longer needed: fetch the row N further down
                    load_row<S, R, V, EDGE>(lv[0][u], a.src, j0 + i + N, rows, cols, gx, col_in, b);
            }
        }
    }
}

// Weights of a task: scalar registers (a VOP2 FMA reads one scalar operand) unless the footprint
// is large and each weight feeds a single FMA per row (V = 1): then they would spill out of the
// scalar file and cost a lane read per use, so they are copied into vector registers once.
template <int R, int V, int SHAPE>
__device__ __forceinline__ void load_weights(const float* w, float* wv) {
    constexpr int K = 2 * R + 1;
#pragma unroll
    for (int q = 0; q < K * K; ++q) {
        if constexpr (V == 1 && SHAPE == SHAPE_BOX && R >= 3) {
            const float sw = w[q];
            asm volatile("v_mov_b32 %0, %1" : "=v"(wv[q]) : "s"(sw));
        } else {
            wv[q] = w[q];
        }
    }
}

// One task: output rows [y0, y1) of the band whose first loaded column is X0, TB levels.
template <int S, int R, int V, int SHAPE, int TB>
__device__ __forceinline__ void march_task(const MarchView& a, const float* w, int lane, int64_t y0, int64_t y1,
                                           int64_t X0) {
    const bool edge = y0 - R * TB < 0 || y1 + R * TB > a.rows || X0 < 0 || X0 + 64 * V > a.cols;
    float wv[(2 * R + 1) * (2 * R + 1)];
    load_weights<R, V, SHAPE>(w, wv);
    if constexpr (TB == 1) {
        if (edge) march_one<S, R, V, SHAPE, true>(a, wv, lane, y0, y1, X0);
        else march_one<S, R, V, SHAPE, false>(a, wv, lane, y0, y1, X0);
    } else {
        if (edge) march_levels<S, R, V, SHAPE, TB, true>(a, wv, lane, y0, y1, X0);
        else march_levels<S, R, V, SHAPE, TB, false>(a, wv, lane, y0, y1, X0);
    }
}

}  // namespace march
}  // namespace st
