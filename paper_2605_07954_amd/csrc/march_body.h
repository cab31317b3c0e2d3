// Device body of the row-marching Jacobi pass (paper Sec. II-C update with the fixed halo of
// Sec. IV-A; per cell the FP32 order of Sec. IV-E), shared by the single-grid kernel and the batched
// multi-grid kernel.  See march.hip for the design; this file holds the per-wavefront task:
// march_levels walks one band of columns over a segment of rows, TB levels per pass.
#pragma once

#include <type_traits>

#include "internal.h"
#include "march_layout.h"
#include "star_centre.h"
#include "storage.h"

namespace st {
namespace march {

// Boundary rules for the cells outside the grid.
enum { BC_CONST = ST_BC_CONST, BC_PERIODIC = ST_BC_PERIODIC, BC_FRAME = ST_BC_FRAME };

// What a task needs of its grid.
struct MarchView {
    const void* src;
    void* dst;
    int64_t rows, cols;
    float b;            // halo value (BC_CONST), already rounded to the storage type
    int bc;             // BC_CONST, BC_PERIODIC or BC_FRAME
    const void* frame;  // BC_FRAME: the caller's halo frame, storage type (see frame_value)
};

// i reduced into [0, n) (a grid smaller than the halo may wrap more than once).
__device__ __forceinline__ int64_t wrap_index(int64_t i, int64_t n) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

// The fixed value of the out-of-grid cell (gy, gx) from the caller's frame of depth R: top strip
// R x (cols + 2R), bottom strip R x (cols + 2R), left strip rows x R, right strip rows x R, each
// row-major, one after another.  Cells farther out feed only cells outside the grid, which take
// their frame value again at every level, so they read 0.
template <int S>
__device__ __forceinline__ float frame_value(const MarchView& a, int R, int64_t gy, int64_t gx) {
    const int64_t rows = a.rows, cols = a.cols;
    if (gy < -R || gy >= rows + R || gx < -R || gx >= cols + R) return 0.0f;
    const int64_t wf = cols + 2 * R;
    int64_t k;
    if (gy < 0) k = (gy + R) * wf + (gx + R);
    else if (gy >= rows) k = int64_t(R) * wf + (gy - rows) * wf + (gx + R);
    else if (gx < 0) k = 2 * int64_t(R) * wf + gy * R + (gx + R);
    else k = 2 * int64_t(R) * wf + rows * R + gy * R + (gx - cols);
    return Fmt<S>::ld(static_cast<const typename Fmt<S>::T*>(a.frame)[k]);
}

// Value that an out-of-grid cell holds at every level: b, or its frame value.  (Periodic grids
// have none: their outside cells are loaded from, and computed like, the cells they wrap to.)
// XBC: the boundary rule the kernel is built for (XBC_CONST: the constant halo b; XBC_PERIODIC;
// XBC_FRAME), so that each kernel carries the edge code of one rule only (the others' would cost it
// registers: built for both, the periodic edge loop ran ten times the instructions of the inner one).
constexpr int XBC_CONST = 0, XBC_PERIODIC = 1, XBC_FRAME = 2;
template <int S, int XBC>
__device__ __forceinline__ float outside_value(const MarchView& a, int R, int64_t gy, int64_t gx) {
    if constexpr (XBC == XBC_FRAME) return frame_value<S>(a, R, gy, gx);
    return a.b;
}
template <int XBC>
__device__ __forceinline__ constexpr bool periodic(const MarchView&) {
    return XBC == XBC_PERIODIC;
}


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

// What one load of V cells returns, still in the storage type: a prefetched row is widened to FP32
// only when it enters the window, so the load need not complete before that.
template <int S, int V>
struct RawSel {
    using type = typename Fmt<S>::T;
};
template <>
struct RawSel<ST_F32, 4> {
    using type = float4;
};
template <>
struct RawSel<ST_BF16, 4> {
    using type = uint2;
};
template <>
struct RawSel<ST_F16, 4> {
    using type = uint2;
};
struct F32x8 {
    float4 a, b;
};
template <>
struct RawSel<ST_F32, 8> {
    using type = F32x8;
};
template <>
struct RawSel<ST_BF16, 8> {
    using type = uint4;
};
template <>
struct RawSel<ST_F16, 8> {
    using type = uint4;
};
template <int S, int V>
using Raw = typename RawSel<S, V>::type;

// A lane's V cells loaded one element at a time (any width and alignment).
template <int S, int V>
struct Elems {
    typename Fmt<S>::T v[V];
};
// VEC: one vector access per lane and row (cols % V == 0, 16-byte aligned rows); otherwise V
// element accesses.  V = 1 is the same either way.
template <int S, int V, bool VEC>
struct RawTSel {
    using type = Elems<S, V>;
};
template <int S, int V>
struct RawTSel<S, V, true> {
    using type = Raw<S, V>;
};
template <int S>
struct RawTSel<S, 1, false> {
    using type = Raw<S, 1>;
};
template <int S, int V, bool VEC>
using RawT = typename RawTSel<S, V, VEC>::type;

// Which of a lane's V columns lie inside the grid.  With vector accesses (and V = 1) all or none,
// since cols % V == 0; with element accesses each column on its own.
template <int V>
struct ColMask {
    bool ok[V];
    bool any;
};

template <int V, bool VEC>
__device__ __forceinline__ ColMask<V> col_mask(int64_t gx, int64_t cols) {
    ColMask<V> m;
    const bool all = gx >= 0 && gx + V <= cols;
#pragma unroll
    for (int c = 0; c < V; ++c) m.ok[c] = (VEC || V == 1) ? all : (gx + c >= 0 && gx + c < cols);
    m.any = (VEC || V == 1) ? all : (gx + V > 0 && gx < cols);
    return m;
}

// The fields live in global memory, and every access goes through a global-qualified pointer: the
// compiler then emits global loads and stores even where it cannot trace a pointer to a kernel
// argument (the batched kernels read theirs from a descriptor table).  Flat accesses would also count
// against the LDS counter, so every wait for an LDS read would wait for the loads in flight too.
template <typename T>
using Glob = __attribute__((address_space(1))) T;
template <int B>
struct Bits;  // a native type of B bytes
template <>
struct Bits<2> {
    using type = unsigned short;
};
template <>
struct Bits<4> {
    using type = unsigned;
};
template <>
struct Bits<8> {
    using type = unsigned __attribute__((ext_vector_type(2)));
};
template <>
struct Bits<16> {
    using type = unsigned __attribute__((ext_vector_type(4)));
};
template <typename X>
__device__ __forceinline__ X gload(const void* p) {
    if constexpr (sizeof(X) == 32) {  // two 16-byte halves
        using H = typename Bits<16>::type;
        struct Two {
            H a, b;
        } t;
        t.a = ((const Glob<H>*)p)[0];
        t.b = ((const Glob<H>*)p)[1];
        return __builtin_bit_cast(X, t);
    } else {
        using B = typename Bits<sizeof(X)>::type;
        return __builtin_bit_cast(X, *(const Glob<B>*)p);
    }
}
template <typename X>
__device__ __forceinline__ void gstore(void* p, const X& x) {
    using B = typename Bits<sizeof(X)>::type;
    *(Glob<B>*)p = __builtin_bit_cast(B, x);
}

template <int S, int V>
__device__ __forceinline__ Raw<S, V> load_raw(const void* src, int64_t off) {
    return gload<Raw<S, V>>(static_cast<const typename Fmt<S>::T*>(src) + off);
}

// Interior tasks address a lane's cells as a wavefront-uniform pointer (row start plus the band's
// first column, scalar registers) plus the lane's byte offset V * lane * sizeof(T) < 2 KiB, which the
// global loads and stores take as their 32-bit vector offset: no per-lane 64-bit address arithmetic.
template <int S, int V>
__device__ __forceinline__ uint32_t lane_bytes() {
    return uint32_t(V * int(threadIdx.x & 63) * int(sizeof(typename Fmt<S>::T)));
}
template <int S, int V>
__device__ __forceinline__ Raw<S, V> load_lane(const void* src, int64_t first, uint32_t loff) {
    const char* p = reinterpret_cast<const char*>(static_cast<const typename Fmt<S>::T*>(src) + first);
    return gload<Raw<S, V>>(p + loff);
}

// The rows a task loads: its input rows y0 - R TB .. y1 - 1 + R TB, cut to the grid.  Fetches past
// them (the FIFO's lead beyond the last row needed and the last group's extra iterations) re-read
// the nearest needed row, which the cache holds, rather than rows of the neighbouring segment.
struct RowSpan {
    int64_t lo, hi;
};
// Input rows [o0, o1) that a neighbouring wavefront of the workgroup staged in LDS (one 16-byte raw
// lane vector per lane and row, row-major): fetched from there instead of HBM.  lds == nullptr: none.
struct SharedRows {
    const float4* lds;
    int64_t o0, o1;
};

// d < 0 from the high word of d: a scalar compare where a 64-bit one would take a vector compare
__device__ __forceinline__ bool negative(int64_t d) { return int32_t(uint32_t(uint64_t(d) >> 32)) < 0; }
// An interior task's rows only run past its span on the side it marches towards.
template <bool UP>
__device__ __forceinline__ int64_t clamp_interior(int64_t gy, const RowSpan& sp) {
    return UP ? (negative(gy - sp.lo) ? sp.lo : gy) : (negative(sp.hi - gy) ? sp.hi : gy);
}
__device__ __forceinline__ int64_t clamp_span(int64_t gy, const RowSpan& sp) {
    return gy < sp.lo ? sp.lo : gy > sp.hi ? sp.hi : gy;
}

// Exact widening to FP32.
template <int S, int V>
__device__ __forceinline__ Cells<V> widen(Raw<S, V> r) {
    Cells<V> q;
    if constexpr (V == 1) {
        q.c[0] = Fmt<S>::ld(r);
    } else if constexpr (S == ST_F32 && V == 8) {
        q.c[0] = r.a.x; q.c[1] = r.a.y; q.c[2] = r.a.z; q.c[3] = r.a.w;
        q.c[4] = r.b.x; q.c[5] = r.b.y; q.c[6] = r.b.z; q.c[7] = r.b.w;
    } else if constexpr (S == ST_F32) {
        q.c[0] = r.x; q.c[1] = r.y; q.c[2] = r.z; q.c[3] = r.w;
    } else if constexpr (V == 8) {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            q.c[2 * k] = Fmt<S>::ld(uint16_t(w[k] & 0xffffu));
            q.c[2 * k + 1] = Fmt<S>::ld(uint16_t(w[k] >> 16));
        }
    } else {
        q.c[0] = Fmt<S>::ld(uint16_t(r.x & 0xffffu));
        q.c[1] = Fmt<S>::ld(uint16_t(r.x >> 16));
        q.c[2] = Fmt<S>::ld(uint16_t(r.y & 0xffffu));
        q.c[3] = Fmt<S>::ld(uint16_t(r.y >> 16));
    }
    return q;
}

template <int S, int V>
__device__ __forceinline__ Cells<V> widen(const Elems<S, V>& r) {
    Cells<V> q;
#pragma unroll
    for (int c = 0; c < V; ++c) q.c[c] = Fmt<S>::ld(r.v[c]);
    return q;
}

template <int S, int V>
__device__ __forceinline__ void store_cells(void* dst, int64_t off, const Cells<V>& q) {
    using T = typename Fmt<S>::T;
    if constexpr (V == 1) {
        gstore(static_cast<T*>(dst) + off, Fmt<S>::st(q.c[0]));
    } else if constexpr (S != ST_F32) {  // four (eight) 16-bit cells: one 8-byte (16-byte) store
        uint32_t w[V / 2];
#pragma unroll
        for (int k = 0; k < V / 2; ++k) w[k] = Fmt<S>::st2(q.c[2 * k], q.c[2 * k + 1]);
        gstore(static_cast<T*>(dst) + off, w);
    } else {
#pragma unroll
        for (int k = 0; k < V; k += 4) {
            const float v4[4] = {q.c[k], q.c[k + 1], q.c[k + 2], q.c[k + 3]};
            gstore(static_cast<T*>(dst) + off + k, v4);
        }
    }
}

// A register copy that the compiler cannot fold away.  An FP32 row moves from its FIFO slot into the
// ring unchanged; folded, the two slots become one register set live for D + 2R + 1 iterations,
// longer than the unrolled loop, and the copies that restore the allocation at the loop's back edge
// then wait for every load in flight.  Copied, each set lives for at most U iterations.
template <int V>
__device__ __forceinline__ void pin_copy(Cells<V>& q) {
#pragma unroll
    for (int c = 0; c < V; ++c) asm volatile("v_mov_b32 %0, %1" : "=v"(q.c[c]) : "v"(q.c[c]));
}

// A level's V cells rounded to the storage type (16-bit types two at a time).
template <int S, int V>
__device__ __forceinline__ void round_cells(Cells<V>& q) {
    if constexpr (S != ST_F32 && V % 2 == 0) {
#pragma unroll
        for (int c = 0; c < V; c += 2) Fmt<S>::rnd2(q.c[c], q.c[c + 1]);
    } else {
#pragma unroll
        for (int c = 0; c < V; ++c) q.c[c] = Fmt<S>::rnd(q.c[c]);
    }
}

template <int R, int V>
__device__ __forceinline__ void set_own(Row<R, V>& x, const Cells<V>& q) {
#pragma unroll
    for (int c = 0; c < V; ++c) x.v[R + c] = q.c[c];
}

// Input row gy as raw storage values, for the FIFO: the row is clamped into the task's row span
// (which EDGE tasks cut to the grid; the cells a clamped row stands for are replaced by their
// outside value when it is used, see `cells_of`, or never feed a stored output), and EDGE tasks
// clamp columns into the grid too, or wrap row and columns on a periodic grid.  A lane's vector
// never straddles the grid's side (cols % V == 0, and so is its first column), so it wraps whole.
template <int S, int V, bool VEC, bool EDGE, int XBC, bool UP = false>
__device__ __forceinline__ RawT<S, V, VEC> fetch_raw(const MarchView& a, int64_t gy, int64_t gx, const ColMask<V>& m,
                                                     int64_t X0, const RowSpan& sp) {
    const int64_t rows = a.rows, cols = a.cols;
    const bool wrap = EDGE && periodic<XBC>(a);
    int64_t g;
    if (wrap) g = wrap_index(gy, rows);
    else if (EDGE) g = clamp_span(gy, sp);
    else g = clamp_interior<UP>(gy, sp);
    if constexpr (!EDGE && (VEC || V == 1)) {
        return load_lane<S, V>(a.src, g * cols + X0, lane_bytes<S, V>());
    } else if constexpr (VEC || V == 1) {
        const int64_t x = wrap ? wrap_index(gx, cols) : (EDGE && !m.ok[0] ? 0 : gx);
        return load_raw<S, V>(a.src, g * cols + x);
    } else {
        RawT<S, V, VEC> r;
        const typename Fmt<S>::T* row = static_cast<const typename Fmt<S>::T*>(a.src) + g * cols;
#pragma unroll
        for (int c = 0; c < V; ++c)
            r.v[c] = gload<typename Fmt<S>::T>(row + (wrap ? wrap_index(gx + c, cols) : (EDGE && !m.ok[c] ? 0 : gx + c)));
        return r;
    }
}

template <int S, int R, int V, bool EDGE, int XBC, typename RawRow>
__device__ __forceinline__ Cells<V> cells_of(const MarchView& a, const RawRow& r, int64_t gy, int64_t gx,
                                             const ColMask<V>& m) {
    Cells<V> q = widen<S, V>(r);
    if (EDGE && !periodic<XBC>(a)) {
        const bool row_ok = gy >= 0 && gy < a.rows;
#pragma unroll
        for (int c = 0; c < V; ++c) q.c[c] = row_ok && m.ok[c] ? q.c[c] : outside_value<S, XBC>(a, R, gy, gx + c);
    }
    return q;
}

// Input row gy loaded and widened at once (the ring rows and the one-row lead).  With vector
// accesses EDGE tasks skip the load for cells outside the grid, which take their outside value (a
// periodic grid loads the cells they wrap to); with element accesses they load clamped (or wrapped)
// addresses and substitute.  Rows are clamped into the task's row span as in `fetch_raw`.
template <int S, int R, int V, bool VEC, bool EDGE, int XBC, bool UP = false>
__device__ __forceinline__ Cells<V> load_now(const MarchView& a, int64_t gy, int64_t gx, const ColMask<V>& m,
                                             int64_t X0, const RowSpan& sp) {
    const int64_t rows = a.rows, cols = a.cols;
    if constexpr (VEC || V == 1) {
        Cells<V> q;
        if (EDGE) {
            if (periodic<XBC>(a)) {
                q = widen<S, V>(load_raw<S, V>(a.src, wrap_index(gy, rows) * cols + wrap_index(gx, cols)));
            } else if (gy >= 0 && gy < rows && m.ok[0]) {
                q = widen<S, V>(load_raw<S, V>(a.src, clamp_span(gy, sp) * cols + gx));
            } else {
#pragma unroll
                for (int c = 0; c < V; ++c) q.c[c] = outside_value<S, XBC>(a, R, gy, gx + c);
            }
        } else {
            q = widen<S, V>(load_lane<S, V>(a.src, clamp_interior<UP>(gy, sp) * cols + X0, lane_bytes<S, V>()));
        }
        return q;
    } else {
        return cells_of<S, R, V, EDGE, XBC>(a, fetch_raw<S, V, VEC, EDGE, XBC, UP>(a, gy, gx, m, X0, sp), gy, gx, m);
    }
}

// A lane's V outputs of one row: one vector store, or one element store per column inside the grid.
template <int S, int V, bool VEC, bool EDGE>
__device__ __forceinline__ void store_row(void* dst, int64_t row_off, int64_t gx, const Cells<V>& q,
                                          const ColMask<V>& m, int64_t X0) {
    if constexpr (!EDGE && (VEC || V == 1)) {
        char* p = reinterpret_cast<char*>(static_cast<typename Fmt<S>::T*>(dst) + row_off + X0);
        store_cells<S, V>(p + lane_bytes<S, V>(), 0, q);
    } else if constexpr (VEC || V == 1) {
        store_cells<S, V>(dst, row_off + gx, q);
    } else {
        typename Fmt<S>::T* row = static_cast<typename Fmt<S>::T*>(dst) + row_off;
#pragma unroll
        for (int c = 0; c < V; ++c)
            if (!EDGE || m.ok[c]) gstore(row + gx + c, Fmt<S>::st(q.c[c]));
    }
}

// The V outputs of a lane for one row; `ring[(base + R + dy) % N]` holds input row dy.  A box
// footprint reads the side columns of every row, which each ring row therefore carries from the
// moment it enters; a star footprint reads them on the centre row only, so ring rows hold their own
// columns and the centre row's sides are produced here, once per row and level as well.
template <int R, int V, int SHAPE, int N, bool UP = false>
__device__ __forceinline__ Cells<V> apply(const Row<R, V>* ring, int base, const float* w) {
    constexpr int K = 2 * R + 1;
    constexpr int DS = UP ? -1 : 1;  // marching upwards the ring holds the rows in the other order
    if constexpr (SHAPE == SHAPE_STAR && V >= 4) {
        // the centre row's side taps take the neighbouring lanes' columns as DPP-shifted FMA operands
        // (star_centre.h), which saves the 2R lane moves per row and level; same order of operations
        const Row<R, V>& mid = ring[(base + R) % N];
        Cells<V> o;
#pragma unroll
        for (int c = 0; c < V; ++c) o.c[c] = w[R * K + R] * mid.v[R + c];
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
            if (dy == 0) {
                float x[V], ws[2 * R];
#pragma unroll
                for (int c = 0; c < V; ++c) x[c] = mid.v[R + c];
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    ws[t] = w[R * K + t];              // dx = t - R
                    ws[R + t] = w[R * K + R + 1 + t];  // dx = t + 1
                }
                StarCentre<R, V>::apply(o.c, x, ws);
                continue;
            }
            const Row<R, V>& x = ring[(base + R + DS * dy) % N];
            const float wt = w[(dy + R) * K + R];
#pragma unroll
            for (int c = 0; c < V; ++c) o.c[c] = __builtin_fmaf(wt, x.v[R + c], o.c[c]);
        }
        return o;
    }
    Row<R, V> mid = ring[(base + R) % N];
    if constexpr (SHAPE == SHAPE_STAR) fill_sides<R, V>(mid);
    Cells<V> o;
#pragma unroll
    for (int c = 0; c < V; ++c) o.c[c] = w[R * K + R] * mid.v[R + c];
#pragma unroll
    for (int dy = -R; dy <= R; ++dy) {
        const Row<R, V>& x = dy == 0 ? mid : ring[(base + R + DS * dy) % N];
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

// TB levels over output rows [y0, y1) of the band whose first loaded column is X0.  Level l (0 =
// input, TB = output) keeps its own ring of N = 2R+1 rows.  Iteration i computes level-1 row
// m1 = y0 - R(TB-1) + i from the input rows m1-R .. m1+R, then, once enough rows of the level below
// exist, level-l row m1 - (l-1)R for l = 2 .. TB.  Within level l the row of iteration i sits in slot
// (i + l - 1) % N (because -2R = 1 mod N), so with the loop unrolled a multiple of N times every
// slot index is a compile-time constant.
//
// Input rows are loaded D iterations before they enter the window, into a FIFO of D raw rows (D a
// multiple of N; the loop is unrolled D times).  With D = 0 a row is loaded into the ring slot that
// level 1 has just released, one iteration ahead.
//
// UP marches the segment from its last row to its first: the same steps with the row order
// reversed (iteration i computes level-1 row y1 - 1 + R(TB-1) - i, and so on), and each ring read
// through the reversed slot order, so that every cell still takes its taps in row-major order.
template <int S, int R, int V, int SHAPE, int TB, int D, bool EDGE, bool VEC, int XBC, bool UP = false,
          bool SHARE = false>
__device__ __forceinline__ void march_levels(const MarchView& a, const float* w, int lane, int64_t y0, int64_t y1,
                                             int64_t X0, const SharedRows& sh = SharedRows{nullptr, 0, 0},
                                             int lo = -1, int hi = -1) {
    constexpr int N = 2 * R + 1;
    static_assert(D % N == 0, "the FIFO length must be a multiple of the ring length");
    constexpr int U = D > 0 ? D : N;  // unroll
    constexpr int H = halo_lanes(R, TB, V);
    constexpr bool SIDES = SHAPE != SHAPE_STAR;  // ring rows carry side columns
    const int64_t rows = a.rows, cols = a.cols;
    const int64_t gx = X0 + V * lane;
    const ColMask<V> cm = col_mask<V, VEC>(gx, cols);
    // lanes [lo, hi) store (default [H, 64 - H)); a band that starts or ends at the grid's side with
    // a zero halo also stores its lanes there, see sweep_march_body
    const bool writer = lane >= (lo < 0 ? H : lo) && lane < (hi < 0 ? 64 - H : hi) && (!EDGE || cm.any);
    Row<R, V> lv[TB][N];  // lv[0]: input rows; lv[l]: level l < TB (the output level is stored directly)
    RawT<S, V, VEC> fifo[D > 0 ? D : 1];
    // input row j lives in ring slot |j - j0| % N, FIFO slot |j - j0| % D
    constexpr int64_t SG = UP ? -1 : 1;  // row step of the march
    const int64_t j0 = UP ? y1 - 1 + R * TB : y0 - R * TB;
    const int64_t need_lo = y0 - R * TB, need_hi = y1 - 1 + R * TB;  // within the grid unless EDGE
    const RowSpan sp{EDGE && need_lo < 0 ? 0 : need_lo, EDGE && need_hi > rows - 1 ? rows - 1 : need_hi};
    using RawR = RawT<S, V, VEC>;
    auto fetch = [&](int64_t j) -> RawR {
        if constexpr (SHARE) {
            static_assert(sizeof(RawR) == sizeof(float4), "shared rows hold one 16-byte vector per lane");
            // (read through an LDS-qualified pointer: a generic one would let the compiler merge this
            // read and the global one below into a flat load, which waits on both counters)
            using LdsVec = __attribute__((address_space(3))) const float4;
            if (sh.lds && !negative(j - sh.o0) && negative(j - sh.o1))
                return __builtin_bit_cast(RawR, ((LdsVec*)sh.lds)[(j - sh.o0) * 64 + lane]);
        }
        return fetch_raw<S, V, VEC, EDGE, XBC, UP>(a, j, gx, cm, X0, sp);
    };
    // a row loaded and widened at once (the ring's first rows, and the one-row lead when D = 0)
    auto load_row = [&](int64_t j) -> Cells<V> {
        if constexpr (SHARE) return cells_of<S, R, V, EDGE, XBC>(a, fetch(j), j, gx, cm);
        return load_now<S, R, V, VEC, EDGE, XBC, UP>(a, j, gx, cm, X0, sp);
    };
    constexpr int FIRST = D > 0 ? 2 * R : N;  // rows loaded straight into the ring
#pragma unroll
    for (int t = 0; t < FIRST; ++t) set_own<R, V>(lv[0][t], load_row(j0 + SG * t));
    if constexpr (D > 0) {
#pragma unroll
        for (int t = 0; t < D; ++t) {
            // issued in the order the loop consumes them (the scheduler would otherwise reorder
            // these independent loads, and the first row needed could be the last to arrive)
            fifo[(2 * R + t) % D] = fetch(j0 + SG * (2 * R + t));
            __builtin_amdgcn_sched_barrier(0);
        }
        // one wait for the whole prologue (ring rows and FIFO, loaded together): the loop's entry
        // then carries no pending load, so each iteration waits only for the FIFO row it consumes
        __builtin_amdgcn_s_waitcnt(0);
    }
    if constexpr (SIDES) {  // after all the loads
#pragma unroll
        for (int t = 0; t < 2 * R; ++t) fill_sides<R, V>(lv[0][t]);
    }
    // The loop runs whole groups of U iterations: the last group may run up to U - 1 iterations past
    // the segment, on rows whose loads are clamped (or take their outside value) and whose outputs
    // are not stored.  No exit from inside a group keeps the FIFO registers fixed across the loop's
    // back edge, so the loads in flight there are not waited for.  (A task spans at most 2^31 + 2R(TB
    // - 1) iterations, so the counter fits 32 bits, whose compares are scalar instructions.)
    const uint32_t iters = uint32_t((y1 - y0) + 2 * R * (TB - 1));
    // One group of U iterations.  WARM: the group may start before every level has 2R+1 rows of the
    // level below (i < 2R(TB-1)), so each level checks.  One-column bands, whose levels are a few
    // instructions each, run the groups after the warm-up from a second copy without the checks (a
    // compare and a branch per level and row); wider bands keep one copy (their registers).
    // (the iteration index is 64-bit, so that the row and address arithmetic derived from it is
    // strength-reduced; the compares use its low 32 bits, which are scalar instructions)
    auto group = [&](int64_t i0, auto warm) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u;
            const uint32_t ic = uint32_t(i);
            Row<R, V>& in = lv[0][(u + 2 * R) % N];  // input row j0 +- (i + 2R) enters the window
            if constexpr (D > 0) {
                const int f = (u + 2 * R) % D;
                const int64_t j = j0 + SG * (i + 2 * R);
                Cells<V> q = cells_of<S, R, V, EDGE, XBC>(a, fifo[f], j, gx, cm);
                if constexpr (S == ST_F32) pin_copy<V>(q);
                set_own<R, V>(in, q);
                fifo[f] = fetch(j + SG * D);
            }
            if (SIDES) fill_sides<R, V>(in);
#pragma unroll
            for (int l = 1; l <= TB; ++l) {
                if constexpr (decltype(warm)::value)
                    if (ic < uint32_t(2 * R * (l - 1))) break;  // level l - 1 does not have 2R+1 rows yet
                // row of level l
                const int64_t m = UP ? y1 - 1 + R * (TB - 1) - i + int64_t(l - 1) * R
                                     : y0 - R * (TB - 1) + i - int64_t(l - 1) * R;
                Cells<V> q = apply<R, V, SHAPE, N, UP>(lv[l - 1], u + l - 1, w);
                if (l == TB) {
                    // (the row against the segment's far end in 32-bit scalar compares: downwards
                    // m >= y0 here and m - y0 < 2^32; upwards the sign of m - y0)
                    const int64_t mr = m - y0;
                    const bool in_seg = UP ? int32_t(uint32_t(uint64_t(mr) >> 32)) >= 0
                                           : uint32_t(mr) < uint32_t(y1 - y0);
                    if (writer && in_seg)
                        store_row<S, V, VEC, EDGE>(a.dst, m * cols, gx, q, cm, X0);
                } else {
                    Row<R, V>& x = lv[l][(u + l - 1) % N];
                    // every level is rounded to the storage type; cells outside the grid keep their
                    // outside value (a periodic grid computes them like the cells they wrap to)
                    round_cells<S, V>(q);
                    if (EDGE && !periodic<XBC>(a)) {
                        const bool row_in = m >= 0 && m < rows;
#pragma unroll
                        for (int c = 0; c < V; ++c)
                            q.c[c] = row_in && cm.ok[c] ? q.c[c] : outside_value<S, XBC>(a, R, m, gx + c);
                    }
                    set_own<R, V>(x, q);
                    if (SIDES) fill_sides<R, V>(x);
                }
                if (D == 0 && l == 1) {  // input row m1 -+ R is no longer needed: fetch the row N further on
                    set_own<R, V>(lv[0][u % N], load_row(j0 + SG * (i + N)));
                }
            }
        }
    };
    constexpr uint32_t WARM = 2 * R * (TB - 1);  // the first iteration at which every level computes
    int64_t i0 = 0;
    if constexpr (V == 1 && TB > 1) {
        for (; uint32_t(i0) < iters && uint32_t(i0) < WARM; i0 += U) group(i0, std::true_type{});
        for (; uint32_t(i0) < iters; i0 += U) group(i0, std::false_type{});
    } else {
        // Wave priority falls with progress (3 until 40 % of the iterations, then 2, 1 from 70 %, 0
        // from 90 %).  A SIMD issues the oldest of its equally prioritised wavefronts first, so
        // without this its two or three tasks finish one after another and the last runs alone,
        // with nothing to hide its latencies; this way a task that gets ahead yields to the others
        // and they finish close together (Star-2D9P +5 %, BF16 storage +9 %, Box-2D49P +3 %).
        // (Grids of one-column bands are latency-bound with a wavefront or two per SIMD: no gain.)
        const uint32_t p1 = uint32_t(uint64_t(iters) * 40 / 100), p2 = uint32_t(uint64_t(iters) * 70 / 100),
                       p3 = uint32_t(uint64_t(iters) * 90 / 100);
        __builtin_amdgcn_s_setprio(3);
        for (; uint32_t(i0) < iters; i0 += U) {
            const uint32_t ic = uint32_t(i0);
            if (ic >= p3) __builtin_amdgcn_s_setprio(0);
            else if (ic >= p2) __builtin_amdgcn_s_setprio(1);
            else if (ic >= p1) __builtin_amdgcn_s_setprio(2);
            group(i0, std::bool_constant<(TB > 1)>{});
        }
        __builtin_amdgcn_s_setprio(0);
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
        // (a star's centre-row side weights feed the DPP FMAs of star_centre.h, whose second
        // operand must be a vector register)
        const bool star_side = SHAPE == SHAPE_STAR && V >= 4 && q / K == R && q % K != R;
        if ((V == 1 && SHAPE == SHAPE_BOX && R >= 3) || star_side) {
            const float sw = w[q];
            asm volatile("v_mov_b32 %0, %1" : "=v"(wv[q]) : "s"(sw));
        } else {
            wv[q] = w[q];
        }
    }
}

// A task reads or writes outside the grid, or near enough to need the edge checks.
template <int R, int TB>
__device__ __forceinline__ bool task_edge(const MarchView& a, int64_t y0, int64_t y1, int64_t X0, int V) {
    return y0 - R * TB < 0 || y1 + R * TB > a.rows || X0 < 0 || X0 + 64 * V > a.cols;
}

// One task: output rows [y0, y1) of the band whose first loaded column is X0, TB levels, input rows
// loaded D iterations ahead (0: one); VEC selects vector or element accesses (see RawT); XBC: the
// boundary rule of the edge tasks (XBC_PERIODIC, XBC_FRAME, else the constant halo b).
template <int S, int R, int V, int SHAPE, int TB, int D, bool VEC = true, int XBC = XBC_CONST>
__device__ __forceinline__ void march_task(const MarchView& a, const float* w, int lane, int64_t y0, int64_t y1,
                                           int64_t X0, int lo = -1, int hi = -1) {
    const bool edge = task_edge<R, TB>(a, y0, y1, X0, V);
    float wv[(2 * R + 1) * (2 * R + 1)];
    load_weights<R, V, SHAPE>(w, wv);
    const SharedRows none{nullptr, 0, 0};
    if (edge) march_levels<S, R, V, SHAPE, TB, D, true, VEC, XBC>(a, wv, lane, y0, y1, X0, none, lo, hi);
    else march_levels<S, R, V, SHAPE, TB, D, false, VEC, XBC_CONST>(a, wv, lane, y0, y1, X0, none, lo, hi);
}

// The same task marched upwards when `up` is set (constant halo), taking the input rows `sh` from LDS.
// Upward tasks take the general (edge) form only, which keeps the kernel's code to one more copy of
// the loop.
template <int S, int R, int V, int SHAPE, int TB, int D, bool VEC = true>
__device__ __forceinline__ void march_task_dir(const MarchView& a, const float* w, int lane, int64_t y0, int64_t y1,
                                               int64_t X0, bool up, const SharedRows& sh) {
    float wv[(2 * R + 1) * (2 * R + 1)];
    load_weights<R, V, SHAPE>(w, wv);
    if (up) march_levels<S, R, V, SHAPE, TB, D, true, VEC, XBC_CONST, true, true>(a, wv, lane, y0, y1, X0, sh);
    else if (task_edge<R, TB>(a, y0, y1, X0, V))
        march_levels<S, R, V, SHAPE, TB, D, true, VEC, XBC_CONST, false, true>(a, wv, lane, y0, y1, X0, sh);
    else march_levels<S, R, V, SHAPE, TB, D, false, VEC, XBC_CONST, false, true>(a, wv, lane, y0, y1, X0, sh);
}

// Stage input rows r0 .. r0 + R TB - 1 of the task (y0, y1, X0) in LDS (`dst[(row - o0) * 64 + lane]`) as
// the task's own fetches would return them, for the neighbouring task that shares them.  All loads are
// issued before the first LDS write, so staging costs one memory latency.
template <int S, int R, int V, int TB, bool VEC = true>
__device__ __forceinline__ void stage_rows(const MarchView& a, int lane, int64_t y0, int64_t y1, int64_t X0,
                                           int64_t r0, int64_t o0, float4* dst) {
    using RawR = RawT<S, V, VEC>;
    constexpr int RT = R * TB;
    const int64_t gx = X0 + V * lane;
    const ColMask<V> cm = col_mask<V, VEC>(gx, a.cols);
    const int64_t need_lo = y0 - R * TB, need_hi = y1 - 1 + R * TB;
    RawR raw[RT];
    if (task_edge<R, TB>(a, y0, y1, X0, V)) {
        const RowSpan sp{need_lo < 0 ? 0 : need_lo, need_hi > a.rows - 1 ? a.rows - 1 : need_hi};
#pragma unroll
        for (int t = 0; t < RT; ++t) raw[t] = fetch_raw<S, V, VEC, true, XBC_CONST>(a, r0 + t, gx, cm, X0, sp);
    } else {
        const RowSpan sp{need_lo, need_hi};
#pragma unroll
        for (int t = 0; t < RT; ++t) raw[t] = fetch_raw<S, V, VEC, false, XBC_CONST>(a, r0 + t, gx, cm, X0, sp);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) dst[(r0 + t - o0) * 64 + lane] = __builtin_bit_cast(float4, raw[t]);
}

}  // namespace march
}  // namespace st
