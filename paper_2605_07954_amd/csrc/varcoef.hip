// Variable-coefficient (conservative) heat step: a 5-point Jacobi update (paper Sec. II-C)
// whose weights come from a diffusivity field kappa:
//   u'(c) = u(c) + sum_{nb in N, W, E, S} kf (u(nb) - u(c)),  kf = (kappa(c) + kappa(nb)) / 2,
// with u(nb) := b and kappa(nb) := kappa(c) across the grid edge.  FP32 order: acc = u(c), then
// acc = fma(0.5f * (kappa(c) + kappa(nb)), u(nb) - u(c), acc) for nb = N, W, E, S.
//
// varcoef_naive: one step per launch, one thread per cell.
// varcoef_tiled: tb steps per launch; u and kappa tiles with a tb-deep halo staged in LDS,
//                4-column x RS-row register blocks per thread, as in the constant-weight sweep.
#include <algorithm>

#include "internal.h"

namespace st {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ float vc_update(float uc, float kc, float un, float kn, float uw, float kw, float ue,
                                           float ke, float us, float ks) {
    float acc = uc;
    acc = __builtin_fmaf(0.5f * (kc + kn), un - uc, acc);
    acc = __builtin_fmaf(0.5f * (kc + kw), uw - uc, acc);
    acc = __builtin_fmaf(0.5f * (kc + ke), ue - uc, acc);
    acc = __builtin_fmaf(0.5f * (kc + ks), us - uc, acc);
    return acc;
}

__global__ __launch_bounds__(NT) void varcoef_naive(SweepArgs a) {
    const int64_t n = a.rows * a.cols;
    const float* u = static_cast<const float*>(a.src);
    const float* k = a.kappa;
    // grid-stride: the grid is capped on the host, so any cell count fits one launch
    for (int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x; idx < n; idx += int64_t(gridDim.x) * NT) {
        const int64_t i = idx / a.cols, j = idx - i * a.cols;
        const float uc = u[idx], kc = k[idx];
        const bool hn = i > 0, hw = j > 0, he = j + 1 < a.cols, hs = i + 1 < a.rows;
        const float un = hn ? u[idx - a.cols] : a.b, kn = hn ? k[idx - a.cols] : kc;
        const float uw = hw ? u[idx - 1] : a.b, kw = hw ? k[idx - 1] : kc;
        const float ue = he ? u[idx + 1] : a.b, ke = he ? k[idx + 1] : kc;
        const float us = hs ? u[idx + a.cols] : a.b, ks = hs ? k[idx + a.cols] : kc;
        static_cast<float*>(a.dst)[idx] = vc_update(uc, kc, un, kn, uw, kw, ue, ke, us, ks);
    }
}

struct VGeo {
    int H, off, bw, bh;
};

__host__ __device__ inline VGeo vgeometry(int tb, int TX, int TY) {
    VGeo g;
    g.H = tb;
    g.off = ((g.H + 4 + 3) / 4) * 4;
    g.bw = ((g.off + TX + g.H + 8 + 3) / 4) * 4;
    g.bh = TY + 2 * g.H;
    return g;
}

__host__ __device__ inline size_t vlds_bytes(int tb, int TX, int TY) {
    VGeo g = vgeometry(tb, TX, TY);
    return size_t(3) * size_t(g.bw) * size_t(g.bh) * sizeof(float);
}

template <int TX, int TY, int RS>
__global__ __launch_bounds__(NT) void varcoef_tiled(SweepArgs a) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    const int tb = a.tb;
    const VGeo g = vgeometry(tb, TX, TY);
    const int H = g.H, OFF = g.off, BW = g.bw, BH = g.bh;
    float* buf0 = lds;
    float* buf1 = lds + BH * BW;
    float* kap = lds + 2 * BH * BW;
    const int64_t tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int64_t y0 = ty * TY, x0 = tx * TX;
    const int64_t rows = a.rows, cols = a.cols;
    const float* src = static_cast<const float*>(a.src);
    float* dst = static_cast<float*>(a.dst);
    const float* kg = a.kappa;
    const float b = a.b;

    // stage u (out of grid: b) and kappa (out of grid: 0, never read for a live cell)
    const int c_lo = OFF - H, c_hi = OFF + TX + H;
    const int wdt = c_hi - c_lo;
    for (int k = threadIdx.x; k < BH * wdt; k += NT) {
        const int br = k / wdt, bc = c_lo + (k - br * wdt);
        const int64_t gy = y0 - H + br, gx = x0 - OFF + bc;
        const bool in = gy >= 0 && gy < rows && gx >= 0 && gx < cols;
        buf0[br * BW + bc] = in ? src[gy * cols + gx] : b;
        kap[br * BW + bc] = in ? kg[gy * cols + gx] : 0.0f;
    }
    __syncthreads();

    for (int l = 1; l <= tb; ++l) {
        const int E = tb - l;
        const float* sb = (l & 1) ? buf0 : buf1;
        float* db = (l & 1) ? buf1 : buf0;
        const bool last = (l == tb);
        const int g0 = (OFF - E) & ~3;
        const int g1 = (OFF + TX + E + 3) & ~3;
        const int ngx = (g1 - g0) >> 2;
        const int HL = TY + 2 * E;
        const int nseg = (HL + RS - 1) / RS;
        for (int it = threadIdx.x; it < ngx * nseg; it += NT) {
            const int seg = it / ngx;
            const int bc = g0 + 4 * (it - seg * ngx);
            const int r0 = H - E + seg * RS;
            const int nr = min(RS, HL - seg * RS);
            const int64_t gx0 = x0 - OFF + bc;
            bool col_in[6];  // columns bc-1 .. bc+4 inside the grid
#pragma unroll
            for (int c = 0; c < 6; ++c) col_in[c] = (gx0 - 1 + c) >= 0 && (gx0 - 1 + c) < cols;
            float uv[RS + 2][6], kv[RS + 2][6];
#pragma unroll
            for (int j = 0; j < RS + 2; ++j) {
                const int br = min(r0 - 1 + j, BH - 1);
                const float* pu = sb + br * BW + bc;
                const float* pk = kap + br * BW + bc;
                const float4 u1 = *reinterpret_cast<const float4*>(pu);
                const float4 k1 = *reinterpret_cast<const float4*>(pk);
                uv[j][0] = pu[-1]; uv[j][1] = u1.x; uv[j][2] = u1.y; uv[j][3] = u1.z; uv[j][4] = u1.w; uv[j][5] = pu[4];
                kv[j][0] = pk[-1]; kv[j][1] = k1.x; kv[j][2] = k1.y; kv[j][3] = k1.z; kv[j][4] = k1.w; kv[j][5] = pk[4];
                if (j < 2) continue;
                const int kr = j - 2;
                if (kr >= nr) continue;
                const int brow = r0 + kr;
                const int64_t gy = y0 - H + brow;
                const bool row_in = gy >= 0 && gy < rows;
                const bool n_in = gy - 1 >= 0, s_in = gy + 1 < rows;
                float o[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float uc = uv[kr + 1][c + 1], kc = kv[kr + 1][c + 1];
                    const float kn = n_in ? kv[kr][c + 1] : kc;
                    const float ks = s_in ? kv[kr + 2][c + 1] : kc;
                    const float kw = col_in[c] ? kv[kr + 1][c] : kc;
                    const float ke = col_in[c + 2] ? kv[kr + 1][c + 2] : kc;
                    const float v = vc_update(uc, kc, uv[kr][c + 1], kn, uv[kr + 1][c], kw, uv[kr + 1][c + 2], ke,
                                              uv[kr + 2][c + 1], ks);
                    o[c] = (row_in && col_in[c + 1]) ? v : b;
                }
                if (last) {
                    if (!row_in) continue;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (col_in[c + 1]) dst[gy * cols + gx0 + c] = o[c];
                } else {
                    *reinterpret_cast<float4*>(db + brow * BW + bc) = make_float4(o[0], o[1], o[2], o[3]);
                }
            }
        }
        __syncthreads();
    }
}

constexpr int VRS = 8;

using VcFn = void (*)(SweepArgs);

// The tiles of the constant-weight sweep's set: small ones give a small grid enough workgroups.
VcFn varcoef_lookup(int tx, int ty) {
    if (tx == 64 && ty == 64) return varcoef_tiled<64, 64, VRS>;
    if (tx == 128 && ty == 32) return varcoef_tiled<128, 32, VRS>;
    if (tx == 128 && ty == 64) return varcoef_tiled<128, 64, VRS>;
    if (tx == 256 && ty == 32) return varcoef_tiled<256, 32, VRS>;
    return nullptr;
}

}  // namespace

size_t varcoef_lds_bytes(int tb, int tx, int ty) { return vlds_bytes(tb, tx, ty); }

int varcoef_launch(const st_plan* p, const float* src, float* dst, const float* kappa, int levels, hipStream_t s) {
    SweepArgs a;
    a.src = src;
    a.dst = dst;
    a.kappa = kappa;
    a.rows = p->rows;
    a.cols = p->cols;
    a.b = p->bq;
    if (levels <= 0) {  // naive reference path
        a.tb = 1;
        const int64_t n = p->rows * p->cols;
        clear_stale_error();
        hipLaunchKernelGGL(varcoef_naive, dim3(unsigned(std::min<int64_t>((n + NT - 1) / NT, kNaiveMaxBlocks))),
                           dim3(NT), 0, s, a);
        ST_LAUNCH_CHECK("varcoef_naive");
        return ST_OK;
    }
    const int tx = p->tile_x, ty = p->tile_y;
    VcFn fn = varcoef_lookup(tx, ty);
    if (!fn) return fail(ST_EUNSUPPORTED, "no varcoef kernel for this tile");
    const size_t lds = vlds_bytes(levels, tx, ty);
    a.tb = levels;
    a.tiles_x = (p->cols + tx - 1) / tx;
    a.tiles_y = (p->rows + ty - 1) / ty;
    if (int rc = prepare_lds(reinterpret_cast<const void*>(fn), lds)) return rc;
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(a.tiles_x * a.tiles_y)), dim3(NT), lds, s, a);
    ST_LAUNCH_CHECK("varcoef_tiled");
    return ST_OK;
}

}  // namespace st
