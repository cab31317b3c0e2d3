// Jacobi sweep kernels for constant-weight star and box stencils (paper Sec. II-C update,
// Sec. IV-A fixed halo, Sec. IV-E centre-first accumulation).
//
// Two kernels:
//   sweep_naive  one step per launch, one thread per cell, neighbours read straight from
//                global memory with a bounds test.  The plain GPU reference path.
//   sweep_tiled  tb steps per launch (temporal blocking).  A 256-thread workgroup owns a
//                TX x TY output tile; it loads the tile plus an r*tb halo into LDS with
//                16-byte loads (cells outside the grid get the halo value b), then runs tb
//                levels in LDS (ping-pong), each level shrinking the valid region by r,
//                and stores only the tile.  Each thread computes a 4-column x RS-row block
//                from a register ring of input rows (three 16-byte LDS reads per row), so
//                every tap is a register operand of one FMA.
// Both use the same per-cell FP32 order (centre product, then one FMA per footprint tap in
// row-major order), so their results are bitwise identical for every tb and tile.
#include <algorithm>
#include <map>
#include <mutex>

#include "internal.h"
#include "storage.h"
#include "sweep_body.h"

namespace st {

namespace {


// ---------------------------------------------------------------------------
// naive kernel
// ---------------------------------------------------------------------------
template <int S, int R, int SHAPE>
__global__ __launch_bounds__(256) void sweep_naive(SweepArgs a) {
    using F = Fmt<S>;
    using T = typename F::T;
    const int64_t n = a.rows * a.cols;
    const T* src = static_cast<const T*>(a.src);
    auto at = [&](int64_t y, int64_t x) -> float {
        return (y < 0 || y >= a.rows || x < 0 || x >= a.cols) ? a.b : F::ld(src[y * a.cols + x]);
    };
    constexpr int K = 2 * R + 1;
    // grid-stride: the grid is capped on the host, so any cell count fits one launch
    for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < n; idx += int64_t(gridDim.x) * 256) {
        const int64_t i = idx / a.cols, j = idx - i * a.cols;
        float acc = a.w[R * K + R] * at(i, j);
#pragma unroll
        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) {
                if ((dy == 0 && dx == 0) || !tap_in(SHAPE, dy, dx)) continue;
                acc = __builtin_fmaf(a.w[(dy + R) * K + dx + R], at(i + dy, j + dx), acc);
            }
        static_cast<T*>(a.dst)[idx] = F::st(acc);
    }
}

// ---------------------------------------------------------------------------
// tiled temporal-blocking kernel (body in sweep_body.h, shared with the batched kernel)
// ---------------------------------------------------------------------------
template <int S, int R, int SHAPE, int TX, int TY, int RS>
__global__ __launch_bounds__(NT) void sweep_tiled(SweepArgs a) {
    extern __shared__ float4 lds4[];
    const int64_t t = xcd_tile(blockIdx.x, a.tiles_x * a.tiles_y);
    tile_body<S, R, SHAPE, TX, TY, RS>(a.src, a.dst, a.rows, a.cols, a.b, a.tb, (t / a.tiles_x) * TY,
                                       (t % a.tiles_x) * TX, a.w, reinterpret_cast<float*>(lds4));
}

// ---------------------------------------------------------------------------
// persistent streaming kernel (FP32, cols % 4 == 0): LDS-DMA double buffering
// ---------------------------------------------------------------------------
// Each workgroup loops over tiles (stride = grid size).  While it computes tile i from one LDS
// staging buffer, the hardware copies tile i+1 into the other with global_load_lds_dwordx4 (no
// registers involved), so the load of the next tile hides behind the arithmetic of this one.
// Staging layout is dense: buffer column 0 holds global column x0 - A, every staged row is
// exactly BW = 4 * NCH floats, so 64 consecutive 16-byte chunks of one DMA instruction land
// contiguously, lane by lane.  Chunks that fall outside the grid are fetched from a clamped
// in-bounds address and then overwritten with b by the lane that fetched them.
struct SGeo {
    int H, A, bw, bh, nch, total;
};

__host__ __device__ inline SGeo sgeometry(int R, int tb, int TX, int TY) {
    SGeo g;
    g.H = R * tb;
    g.A = ((g.H + 3) & ~3) + 8;
    g.bw = (g.A + TX + g.H + 8 + 3) & ~3;
    g.bh = TY + 2 * g.H;
    g.nch = g.bw / 4;
    g.total = g.bh * g.nch;
    return g;
}

__host__ __device__ inline size_t stream_lds_bytes(int R, int tb, int TX, int TY) {
    SGeo g = sgeometry(R, tb, TX, TY);
    return (size_t(tb > 1 ? 3 : 2) * size_t(g.bw) * size_t(g.bh) + MAXK) * sizeof(float);
}

// Issue (or, with FIX, repair) this lane's share of the DMA of one tile into `buf`.
template <bool FIX>
__device__ __forceinline__ void stream_stage(const float* src, int64_t rows, int64_t cols, float b, const SGeo& g,
                                             int64_t y0, int64_t x0, float* buf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int k = 64 * wave + lane;
    int row = k / g.nch, cc = k - row * g.nch;
    const int dq = NT / g.nch, dr = NT % g.nch;
    for (int j = 0; j * NT < g.total; ++j, k += NT) {
        if (k < g.total) {
            const int64_t gy = y0 - g.H + row, gx = x0 - g.A + 4 * cc;
            const bool in = gy >= 0 && gy < rows && gx >= 0 && gx + 4 <= cols;
            if (FIX) {
                if (!in) reinterpret_cast<float4*>(buf)[k] = make_float4(b, b, b, b);
            } else {
                const float* gp = in ? src + gy * cols + gx : src;
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void*)(gp),
                    (__attribute__((address_space(3))) void*)(buf + 4 * (j * NT + 64 * wave)), 16, 0,
                    0);
            }
        }
        row += dq;
        cc += dr;
        if (cc >= g.nch) {
            cc -= g.nch;
            ++row;
        }
    }
}

template <int R, int SHAPE, int TX, int TY, int RS>
__global__ __launch_bounds__(NT) void sweep_stream(SweepArgs a) {
    constexpr int K = 2 * R + 1;
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    const int tb = a.tb;
    const SGeo g = sgeometry(R, tb, TX, TY);
    const int H = g.H, A = g.A, BW = g.bw, BH = g.bh;
    // Buffers are picked by offset arithmetic on the LDS base (an array of pointers would make the
    // compiler lose the LDS address space and fall back to flat loads).
    float* mid = lds + 2 * BH * BW;
    float* wsh = mid + (tb > 1 ? BH * BW : 0);
    const int64_t rows = a.rows, cols = a.cols;
    const float b = a.b;
    const float* src = static_cast<const float*>(a.src);
    float* dst = static_cast<float*>(a.dst);
    const int64_t ntiles = a.tiles_x * a.tiles_y;
    if (threadIdx.x < K * K) wsh[threadIdx.x] = a.w[threadIdx.x];

    int64_t t = blockIdx.x;
    if (t < ntiles) {
        const int64_t m = xcd_tile(t, ntiles);
        stream_stage<false>(src, rows, cols, b, g, (m / a.tiles_x) * TY, (m % a.tiles_x) * TX, lds);
    }
    float wreg[K * K];
    for (int it = 0; t < ntiles; ++it, t += gridDim.x) {
        const int64_t m = xcd_tile(t, ntiles);
        const int64_t y0 = (m / a.tiles_x) * TY, x0 = (m % a.tiles_x) * TX;
        float* cur = lds + (it & 1) * (BH * BW);
        // Every wave waits for its own DMA of the current tile; the barrier then orders all of
        // them before the out-of-grid repair (same chunks) and the repair before any read.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        stream_stage<true>(src, rows, cols, b, g, y0, x0, cur);
        __syncthreads();
        if (it == 0) {
#pragma unroll
            for (int q = 0; q < K * K; ++q) wreg[q] = wsh[q];
        }
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) {
            const int64_t mn = xcd_tile(tn, ntiles);
            stream_stage<false>(src, rows, cols, b, g, (mn / a.tiles_x) * TY, (mn % a.tiles_x) * TX,
                                lds + ((it + 1) & 1) * (BH * BW));
        }
        const float* sb = cur;
        for (int l = 1; l <= tb; ++l) {
            const int E = R * (tb - l);
            const bool last = (l == tb);
            float* db = (l & 1) ? mid : cur;
            const int g0 = (A - E) & ~3;
            const int g1 = (A + TX + E + 3) & ~3;
            const int ngx = (g1 - g0) >> 2;
            const int HL = TY + 2 * E;
            const int nseg = (HL + RS - 1) / RS;
            const int nitems = ngx * nseg;
            for (int item = threadIdx.x; item < nitems; item += NT) {
                const int seg = item / ngx;
                const int bc = g0 + 4 * (item - seg * ngx);
                const int r0 = H - E + seg * RS;
                const int nr = min(RS, HL - seg * RS);
                const int64_t gx0 = x0 - A + bc;
                float v[RS + 2 * R][12];
#pragma unroll
                for (int j = 0; j < RS + 2 * R; ++j) {
                    const int br = min(r0 - R + j, BH - 1);
                    const float4* p = reinterpret_cast<const float4*>(sb + br * BW + bc - 4);
                    const float4 q0 = p[0], q1 = p[1], q2 = p[2];
                    v[j][0] = q0.x; v[j][1] = q0.y; v[j][2] = q0.z; v[j][3] = q0.w;
                    v[j][4] = q1.x; v[j][5] = q1.y; v[j][6] = q1.z; v[j][7] = q1.w;
                    v[j][8] = q2.x; v[j][9] = q2.y; v[j][10] = q2.z; v[j][11] = q2.w;
                    if (j < 2 * R) continue;
                    const int kr = j - 2 * R;
                    float o[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) o[c] = wreg[R * K + R] * v[kr + R][4 + c];
#pragma unroll
                    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                        for (int dx = -R; dx <= R; ++dx) {
                            if ((dy == 0 && dx == 0) || !tap_in(SHAPE, dy, dx)) continue;
                            const float wt = wreg[(dy + R) * K + dx + R];
#pragma unroll
                            for (int c = 0; c < 4; ++c) o[c] = __builtin_fmaf(wt, v[kr + R + dy][4 + c + dx], o[c]);
                        }
                    if (kr >= nr) continue;
                    const int brow = r0 + kr;
                    const int64_t gy = y0 - H + brow;
                    if (last) {
                        if (gy >= rows) continue;
                        if (gx0 + 4 <= cols) {
                            *reinterpret_cast<float4*>(dst + gy * cols + gx0) = make_float4(o[0], o[1], o[2], o[3]);
                        } else {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                if (gx0 + c < cols) dst[gy * cols + gx0 + c] = o[c];
                        }
                    } else {
                        const bool row_in = gy >= 0 && gy < rows;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const int64_t gx = gx0 + c;
                            o[c] = (row_in && gx >= 0 && gx < cols) ? o[c] : b;
                        }
                        *reinterpret_cast<float4*>(db + brow * BW + bc) = make_float4(o[0], o[1], o[2], o[3]);
                    }
                }
            }
            __syncthreads();
            sb = db;
        }
    }
}

// ---------------------------------------------------------------------------
// dispatch tables
// ---------------------------------------------------------------------------
struct TileDef {
    int tx, ty;
};
constexpr TileDef kTiles[] = {{64, 64}, {128, 32}, {128, 64}, {256, 32}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kRS = 8;

using KernelFn = void (*)(SweepArgs);

template <int S, int R, int SH>
KernelFn tiled_fn(int tile) {
    switch (tile) {
        case 0: return sweep_tiled<S, R, SH, 64, 64, kRS>;
        case 1: return sweep_tiled<S, R, SH, 128, 32, kRS>;
        case 2: return sweep_tiled<S, R, SH, 128, 64, kRS>;
        case 3: return sweep_tiled<S, R, SH, 256, 32, kRS>;
    }
    return nullptr;
}

template <int S, int SH>
KernelFn tiled_fn_r(int r, int tile) {
    switch (r) {
        case 1: return tiled_fn<S, 1, SH>(tile);
        case 2: return tiled_fn<S, 2, SH>(tile);
        case 3: return tiled_fn<S, 3, SH>(tile);
        case 4: return tiled_fn<S, 4, SH>(tile);
    }
    return nullptr;
}

KernelFn tiled_lookup(int storage, int shape, int r, int tile) {
    if (storage == ST_F32)
        return shape == SHAPE_BOX ? tiled_fn_r<ST_F32, SHAPE_BOX>(r, tile) : tiled_fn_r<ST_F32, SHAPE_STAR>(r, tile);
    if (storage == ST_BF16)
        return shape == SHAPE_BOX ? tiled_fn_r<ST_BF16, SHAPE_BOX>(r, tile) : tiled_fn_r<ST_BF16, SHAPE_STAR>(r, tile);
    if (storage == ST_F16)
        return shape == SHAPE_BOX ? tiled_fn_r<ST_F16, SHAPE_BOX>(r, tile) : tiled_fn_r<ST_F16, SHAPE_STAR>(r, tile);
    return nullptr;
}

template <int S, int SH>
KernelFn naive_fn_r(int r) {
    switch (r) {
        case 1: return sweep_naive<S, 1, SH>;
        case 2: return sweep_naive<S, 2, SH>;
        case 3: return sweep_naive<S, 3, SH>;
        case 4: return sweep_naive<S, 4, SH>;
    }
    return nullptr;
}

template <int SH>
KernelFn stream_fn_r(int r, int tile) {
#define ST_STREAM_TILES(R)                                  \
    switch (tile) {                                         \
        case 0: return sweep_stream<R, SH, 64, 64, 4>;      \
        case 1: return sweep_stream<R, SH, 128, 32, 4>;     \
        case 2: return sweep_stream<R, SH, 128, 64, 8>;     \
        case 3: return sweep_stream<R, SH, 256, 32, 8>;     \
    }                                                       \
    return nullptr;
    switch (r) {
        case 1: ST_STREAM_TILES(1)
        case 2: ST_STREAM_TILES(2)
        case 3: ST_STREAM_TILES(3)
        case 4: ST_STREAM_TILES(4)
    }
#undef ST_STREAM_TILES
    return nullptr;
}

KernelFn stream_lookup(int shape, int r, int tile) {
    return shape == SHAPE_BOX ? stream_fn_r<SHAPE_BOX>(r, tile) : stream_fn_r<SHAPE_STAR>(r, tile);
}

KernelFn naive_lookup(int storage, int shape, int r) {
    if (storage == ST_F32) return shape == SHAPE_BOX ? naive_fn_r<ST_F32, SHAPE_BOX>(r) : naive_fn_r<ST_F32, SHAPE_STAR>(r);
    if (storage == ST_BF16) return shape == SHAPE_BOX ? naive_fn_r<ST_BF16, SHAPE_BOX>(r) : naive_fn_r<ST_BF16, SHAPE_STAR>(r);
    if (storage == ST_F16) return shape == SHAPE_BOX ? naive_fn_r<ST_F16, SHAPE_BOX>(r) : naive_fn_r<ST_F16, SHAPE_STAR>(r);
    return nullptr;
}

int tile_index(int tx, int ty) {
    for (int i = 0; i < kNumTiles; ++i)
        if (kTiles[i].tx == tx && kTiles[i].ty == ty) return i;
    return -1;
}

void fill_args(const st_plan* p, const void* src, void* dst, const float* kappa, SweepArgs& a) {
    a.src = src;
    a.dst = dst;
    a.kappa = kappa;
    a.rows = p->rows;
    a.cols = p->cols;
    a.b = p->bq;
    std::memcpy(a.w, p->w, sizeof(a.w));
}

}  // namespace

bool tile_supported(int shape, int radius, int tx, int ty) {
    (void)shape;
    (void)radius;
    return tile_index(tx, ty) >= 0;
}

int supported_tiles(int* xy, int cap) {
    for (int i = 0; i < kNumTiles && i < cap; ++i) {
        xy[2 * i] = kTiles[i].tx;
        xy[2 * i + 1] = kTiles[i].ty;
    }
    return kNumTiles;
}

int max_tb(const st_plan* p, int tx, int ty) {
    int tb = 1;
    if (is_march(p->variant)) return march_max_tb(p->shape, p->radius, march_vmax(p->variant));
    if (p->variant == VARIANT_RESIDENT) return std::max(1, std::min(64, resident_max_tb(p)));
    if (p->variant == VARIANT_MFMA) return 1;
    if (p->variant == VARIANT_STREAM) {
        while (tb < 16 && stream_lds_bytes(p->radius, tb + 1, tx, ty) <= lds_limit()) ++tb;
    } else {
        while (tb < 16 && lds_bytes(p->radius, tb + 1, tx, ty) <= lds_limit()) ++tb;
    }
    return tb;
}

bool stream_usable(const st_plan* p) { return p->storage == ST_F32 && p->cols % 4 == 0; }

size_t tiled_lds_bytes(int r, int tb, int tx, int ty) { return lds_bytes(r, tb, tx, ty); }

int launch_naive(const st_plan* p, const void* src, void* dst, const float* kappa, hipStream_t s) {
    KernelFn fn = naive_lookup(p->storage, p->shape, p->radius);
    if (!fn) return fail(ST_EUNSUPPORTED, "no naive kernel for this storage/shape/radius");
    SweepArgs a;
    fill_args(p, src, dst, kappa, a);
    a.tb = 1;
    a.tiles_x = a.tiles_y = 0;
    const int64_t n = p->rows * p->cols;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, kNaiveMaxBlocks);
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(blocks)), dim3(256), 0, s, a);
    ST_LAUNCH_CHECK("sweep_naive");
    return ST_OK;
}

int launch_pass(const st_plan* p, const void* src, void* dst, const float* kappa, int levels, hipStream_t s) {
    if (p->flags & ST_FLAG_NAIVE) {
        // the reference path: one launch per step through the workspace is handled by the caller
        return fail(ST_EUNSUPPORTED, "launch_pass called on a naive plan");
    }
    const int ti = tile_index(p->tile_x, p->tile_y);
    if (p->variant == VARIANT_MFMA && levels == 1 && mfma_usable(p)) return launch_mfma(p, src, dst, s);
    if (is_march(p->variant) && march_usable(p) &&
        levels <= march_max_tb(p->shape, p->radius, march_vmax(p->variant)))
        return launch_march(p, src, dst, levels, march_vmax(p->variant), s);
    const bool aligned = (reinterpret_cast<uintptr_t>(src) % 16) == 0 && (reinterpret_cast<uintptr_t>(dst) % 16) == 0;
    if (p->variant == VARIANT_STREAM && stream_usable(p) && aligned) {
        KernelFn fn = stream_lookup(p->shape, p->radius, ti);
        if (!fn) return fail(ST_EUNSUPPORTED, "no streaming kernel for this shape/radius/tile");
        const size_t lds = stream_lds_bytes(p->radius, levels, p->tile_x, p->tile_y);
        if (int rc = prepare_lds(reinterpret_cast<const void*>(fn), lds)) return rc;
        SweepArgs a;
        fill_args(p, src, dst, kappa, a);
        a.tb = levels;
        a.tiles_x = (p->cols + p->tile_x - 1) / p->tile_x;
        a.tiles_y = (p->rows + p->tile_y - 1) / p->tile_y;
        const int64_t ntiles = a.tiles_x * a.tiles_y;
        int blocks = 0;
        if (int rc = resident_blocks(reinterpret_cast<const void*>(fn), lds, &blocks)) return rc;
        clear_stale_error();
        hipLaunchKernelGGL(fn, dim3(unsigned(std::min<int64_t>(ntiles, blocks))), dim3(NT), lds, s, a);
        ST_LAUNCH_CHECK("sweep_stream");
        return ST_OK;
    }
    KernelFn fn = tiled_lookup(p->storage, p->shape, p->radius, ti);
    if (!fn) return fail(ST_EUNSUPPORTED, "no tiled kernel for this storage/shape/radius/tile");
    const size_t lds = lds_bytes(p->radius, levels, p->tile_x, p->tile_y);
    SweepArgs a;
    fill_args(p, src, dst, kappa, a);
    a.tb = levels;
    a.tiles_x = (p->cols + p->tile_x - 1) / p->tile_x;
    a.tiles_y = (p->rows + p->tile_y - 1) / p->tile_y;
    if (int rc = prepare_lds(reinterpret_cast<const void*>(fn), lds)) return rc;
    const int64_t blocks = a.tiles_x * a.tiles_y;
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(blocks)), dim3(NT), lds, s, a);
    ST_LAUNCH_CHECK("sweep_tiled");
    return ST_OK;
}

}  // namespace st
