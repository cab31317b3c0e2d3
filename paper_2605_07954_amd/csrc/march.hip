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

#include "internal.h"
#include "storage.h"

namespace st {
namespace {

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
__device__ __forceinline__ void march_one(const MarchArgs& a, const float* w, int lane, int64_t y0, int64_t y1,
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
__device__ __forceinline__ void march_levels(const MarchArgs& a, const float* w, int lane, int64_t y0, int64_t y1,
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
    const bool edge = y0 - R * TB < 0 || y1 + R * TB > a.rows || X0 < 0 || X0 + 64 * V > a.cols;
    // Weights: scalar registers (a VOP2 FMA reads one scalar operand) unless the footprint is large
    // and each weight feeds a single FMA per row (V = 1): then they would spill out of the scalar file
    // and cost a lane read per use, so they are copied into vector registers once (register moves).
    constexpr int K = 2 * R + 1;
    float wv[K * K];
#pragma unroll
    for (int q = 0; q < K * K; ++q) {
        if constexpr (V == 1 && SHAPE == SHAPE_BOX && R >= 3) {
            const float sw = a.w[q];
            asm volatile("v_mov_b32 %0, %1" : "=v"(wv[q]) : "s"(sw));
        } else {
            wv[q] = a.w[q];
        }
    }
    if constexpr (TB == 1) {
        if (edge) march_one<S, R, V, SHAPE, true>(a, wv, lane, y0, y1, X0);
        else march_one<S, R, V, SHAPE, false>(a, wv, lane, y0, y1, X0);
    } else {
        if (edge) march_levels<S, R, V, SHAPE, TB, true>(a, wv, lane, y0, y1, X0);
        else march_levels<S, R, V, SHAPE, TB, false>(a, wv, lane, y0, y1, X0);
    }
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

// Depths per radius: the rings of TB levels must fit the register file next to each other.
template <int S, int V, int SH>
MarchFn march_fn(int r, int levels) {
#define ST_MARCH(R, TB) \
    if (r == R && levels == TB) return march_kernel<S, R, V, SH, TB>();
    ST_MARCH(1, 1) ST_MARCH(1, 2) ST_MARCH(1, 3) ST_MARCH(1, 4)
    ST_MARCH(2, 1) ST_MARCH(2, 2) ST_MARCH(2, 3)
    ST_MARCH(3, 1) ST_MARCH(3, 2)
    ST_MARCH(4, 1) ST_MARCH(4, 2)
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

int march_max_tb(int radius) { return radius == 1 ? 4 : radius == 2 ? 3 : 2; }

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
