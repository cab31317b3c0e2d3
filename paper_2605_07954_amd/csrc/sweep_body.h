// Device body of the tiled temporal-blocking Jacobi pass (paper Sec. II-C update, Sec. IV-A
// fixed halo, Sec. IV-E centre-first accumulation), shared by the single-grid kernel and the
// batched persistent kernel.
//
// A 256-thread workgroup owns a TX x TY output tile.  It stages the tile plus an r*tb halo into
// LDS with 16-byte loads (cells outside the grid get the halo value b), runs tb levels in LDS
// (ping-pong), each level shrinking the valid region by r, and stores only the tile.  Each
// thread computes a 4-column x RS-row block from a register ring of input rows (three 16-byte
// LDS reads per row); every tap is a register operand of one FMA.  Per cell the FP32 order is
// the centre product, then one FMA per footprint tap in row-major (dy, dx) order.
#pragma once

#include "internal.h"
#include "storage.h"

namespace st {

constexpr int NT = 256;  // threads per workgroup

__device__ __forceinline__ bool tap_in(int shape, int dy, int dx) {
    return shape == SHAPE_BOX || dy == 0 || dx == 0;
}


// LDS geometry of one pass.  Buffer column bc holds global column x0 - off + bc, buffer row br
// holds global row y0 - H + br, with H = r*tb the halo depth.  off is a multiple of 8 so that
// 16-byte chunks of the buffer map to aligned 16-byte chunks of the field.
struct Geo {
    int H, off, bw, bh;
};

__host__ __device__ inline Geo geometry(int R, int tb, int TX, int TY) {
    Geo g;
    g.H = R * tb;
    g.off = ((g.H + 4 + 7) / 8) * 8;
    g.bw = ((g.off + TX + g.H + 7 + 7) / 8) * 8;
    g.bh = TY + 2 * g.H;
    return g;
}

// LDS of one pass: one or two field buffers, then the weights (kept in dynamic LDS so that
// several inlined bodies in one kernel do not each reserve their own static copy).
__host__ __device__ inline size_t lds_floats(int R, int tb, int TX, int TY) {
    Geo g = geometry(R, tb, TX, TY);
    return size_t(tb > 1 ? 2 : 1) * size_t(g.bw) * size_t(g.bh);
}

__host__ __device__ inline size_t lds_bytes(int R, int tb, int TX, int TY) {
    return (lds_floats(R, tb, TX, TY) + MAXK) * sizeof(float);
}

// Map the launch's block index to a tile so that each of the 8 XCDs (which receive blocks
// round-robin) works on a contiguous band of tiles; vertically adjacent tiles then share
// their halo rows through the same L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t ntiles) {
    const int64_t q = ntiles / 8, rem = ntiles % 8;
    const int64_t k = bid % 8, i = bid / 8;
    return k * q + (k < rem ? k : rem) + i;
}

// One tb-level pass over the output tile with origin (y0, x0).  `w` holds the dense
// (2r+1)^2 weights (kernel arguments or global memory); `lds` is the dynamic LDS block of
// lds_bytes(R, tb, TX, TY) bytes.  All NT threads of the workgroup must call it together.
template <int S, int R, int SHAPE, int TX, int TY, int RS>
__device__ __forceinline__ void tile_body(const void* srcv, void* dstv, int64_t rows, int64_t cols, float b, int tb,
                                          int64_t y0, int64_t x0, const float* w, float* lds) {
    using F = Fmt<S>;
    using T = typename F::T;
    constexpr int VEC = F::VEC;
    constexpr int K = 2 * R + 1;
    const Geo g = geometry(R, tb, TX, TY);
    const int H = g.H, OFF = g.off, BW = g.bw, BH = g.bh;
    float* buf0 = lds;
    float* buf1 = lds + BH * BW;
    const T* src = static_cast<const T*>(srcv);
    T* dst = static_cast<T*>(dstv);
    const bool vec_ok = (cols % VEC) == 0 && (reinterpret_cast<uintptr_t>(src) % 16) == 0 &&
                        (reinterpret_cast<uintptr_t>(dst) % 16) == 0;

    // Weights go through LDS into vector registers: with up to 81 taps they would not fit the
    // scalar register file next to the kernel's other uniform values, and spilled scalars cost an
    // extra instruction per use.
    float* wsh = lds + lds_floats(R, tb, TX, TY);
    if (threadIdx.x < K * K) wsh[threadIdx.x] = w[threadIdx.x];
    // ---- stage the haloed tile into LDS (16-byte chunks; out-of-grid cells = b) ----
    {
        const int c_lo = (OFF - H) & ~(VEC - 1);
        const int c_hi = (OFF + TX + H + VEC - 1) & ~(VEC - 1);
        const int nch = (c_hi - c_lo) / VEC;
        // The BH x nch chunks are dealt round-robin to the NT threads; each thread walks its
        // chunks with an incremental (row, column) update instead of a division per chunk, and
        // keeps up to U chunks in flight (raw 16-byte words first, widened into LDS after all of
        // them were issued), so the load phase costs about one memory latency.
        constexpr int U = 12;
        const int total = BH * nch;
        const int dq = NT / nch, dr = NT % nch;
        int br = int(threadIdx.x) / nch, cc = int(threadIdx.x) % nch;
        for (int k0 = threadIdx.x; k0 < total; k0 += U * NT) {
            uint4 raw[U];
            int dstoff[U];
            bool got[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                got[u] = false;
                dstoff[u] = 0;
                if (k0 + u * NT < total) {
                    const int bc = c_lo + cc * VEC;
                    const int64_t gy = y0 - H + br, gx = x0 - OFF + bc;
                    dstoff[u] = br * BW + bc;
                    float4* p = reinterpret_cast<float4*>(buf0 + dstoff[u]);
                    if (gy < 0 || gy >= rows || gx + VEC <= 0 || gx >= cols) {
#pragma unroll
                        for (int e = 0; e < VEC; e += 4) p[e / 4] = make_float4(b, b, b, b);
                    } else if (vec_ok && gx >= 0 && gx + VEC <= cols) {
                        raw[u] = *reinterpret_cast<const uint4*>(src + gy * cols + gx);
                        got[u] = true;
                    } else {
                        float v[VEC];
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const int64_t x = gx + e;
                            v[e] = (x >= 0 && x < cols) ? F::ld(src[gy * cols + x]) : b;
                        }
#pragma unroll
                        for (int e = 0; e < VEC; e += 4) p[e / 4] = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
                    }
                }
                br += dq;
                cc += dr;
                if (cc >= nch) {
                    cc -= nch;
                    ++br;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!got[u]) continue;
                float v[VEC];
                widen_chunk<S>(raw[u], v);
                float4* p = reinterpret_cast<float4*>(buf0 + dstoff[u]);
#pragma unroll
                for (int e = 0; e < VEC; e += 4) p[e / 4] = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
            }
        }
    }
    __syncthreads();

    float wreg[K * K];
#pragma unroll
    for (int q = 0; q < K * K; ++q) wreg[q] = wsh[q];

    // ---- tb levels ----
    for (int l = 1; l <= tb; ++l) {
        const int E = R * (tb - l);  // margin still needed around the tile after this level
        const float* sb = (l & 1) ? buf0 : buf1;
        float* db = (l & 1) ? buf1 : buf0;
        const bool last = (l == tb);
        const int g0 = (OFF - E) & ~3;
        const int g1 = (OFF + TX + E + 3) & ~3;
        const int ngx = (g1 - g0) >> 2;
        const int HL = TY + 2 * E;
        const int nseg = (HL + RS - 1) / RS;
        const int nitems = ngx * nseg;
        for (int it = threadIdx.x; it < nitems; it += NT) {
            const int seg = it / ngx;
            const int bc = g0 + 4 * (it - seg * ngx);
            const int r0 = H - E + seg * RS;  // buffer row of the block's first output row
            const int nr = min(RS, HL - seg * RS);
            const int64_t gx0 = x0 - OFF + bc;

            // register ring: row j of the block's input (buffer row r0 - R + j), columns bc-4 .. bc+7
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
                const int kr = j - 2 * R;  // output row of the block completed by this input row
                // per cell: centre product, then one FMA per footprint tap in row-major order; the four
                // cells of the block advance together so each weight register feeds four FMAs
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
                    if (vec_ok && gx0 + 4 <= cols) {
                        store4<S>(dst + gy * cols + gx0, o);
                    } else {
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (gx0 + c < cols) dst[gy * cols + gx0 + c] = F::st(o[c]);
                    }
                } else {
                    const bool row_in = gy >= 0 && gy < rows;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int64_t gx = gx0 + c;
                        o[c] = (row_in && gx >= 0 && gx < cols) ? F::rnd(o[c]) : b;
                    }
                    *reinterpret_cast<float4*>(db + brow * BW + bc) = make_float4(o[0], o[1], o[2], o[3]);
                }
            }
        }
        __syncthreads();
    }
}


// Whole-grid body: one workgroup keeps a small grid (plus an r-deep halo of b) resident in LDS
// for all `steps` steps, so the grid never round-trips through HBM between steps.  Buffer column
// bc holds grid column bc - 8, buffer row br holds grid row br - R.  `lds` must hold
// resident_lds_bytes(R, rows, cols) bytes.
__host__ __device__ inline int resident_bw(int64_t cols) { return int(((8 + cols + 8 + 7) / 8) * 8); }

__host__ __device__ inline size_t resident_lds_bytes(int R, int64_t rows, int64_t cols) {
    return (size_t(2) * size_t(rows + 2 * R) * size_t(resident_bw(cols)) + MAXK) * sizeof(float);
}

template <int R, int SHAPE, int RS>
__device__ __forceinline__ void resident_body(const float* src, float* dst, int rows, int cols, float b, int steps,
                                              const float* w, float* lds) {
    constexpr int K = 2 * R + 1;
    constexpr int OFF = 8;
    const int BW = resident_bw(cols), BH = rows + 2 * R;
    // buffers by offset arithmetic on the LDS base (keeps the compiler on LDS instructions)
    float* wsh = lds + 2 * BH * BW;
    if (threadIdx.x < K * K) wsh[threadIdx.x] = w[threadIdx.x];
    for (int k = threadIdx.x; k < 2 * BH * BW; k += NT) lds[k] = b;
    __syncthreads();
    for (int k = threadIdx.x; k < rows * cols; k += NT) {
        const int i = k / cols, j = k - i * cols;
        lds[(i + R) * BW + OFF + j] = src[k];
    }
    __syncthreads();
    float wreg[K * K];
#pragma unroll
    for (int q = 0; q < K * K; ++q) wreg[q] = wsh[q];
    const int ngx = (cols + 3) >> 2;
    const int nseg = (rows + RS - 1) / RS;
    for (int s = 0; s < steps; ++s) {
        const float* sb = lds + (s & 1) * (BH * BW);
        float* db = lds + ((s + 1) & 1) * (BH * BW);
        for (int it = threadIdx.x; it < ngx * nseg; it += NT) {
            const int seg = it / ngx;
            const int gx0 = 4 * (it - seg * ngx);
            const int bc = OFF + gx0;
            const int r0 = R + seg * RS;
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
                const int gy = seg * RS + kr;
                if (gy >= rows) continue;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (gx0 + c < cols) db[(gy + R) * BW + bc + c] = o[c];  // halo cells keep b
            }
        }
        __syncthreads();
    }
    const float* fin = lds + (steps & 1) * (BH * BW);
    for (int k = threadIdx.x; k < rows * cols; k += NT) {
        const int i = k / cols, j = k - i * cols;
        dst[k] = fin[(i + R) * BW + OFF + j];
    }
}

}  // namespace st
