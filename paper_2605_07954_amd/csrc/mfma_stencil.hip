// The Jacobi update (Sec. II-C, constant halo of Sec. IV-A) as a dense contraction on the matrix
// cores -- the family of the paper's tensor-core baseline (Sec. V: the stencil rewritten so that a
// matrix unit does the multiply-adds), built for gfx950's BF16 MFMA with split operands.
//
// For one output row block (16 rows i0.., 16 columns x0..) and one footprint row dy:
//   out[i0+m][x0+n] += sum_k U[m][k] * T[k][n],
//   U[m][k] = u[i0 + m + dy - r][x0 - 8 + k]          (k in [0, 32): a 32-column input window)
//   T[k][n] = W[dy][k - 8 - n + r] if |k - 8 - n| <= r, else 0  (a banded Toeplitz block)
// (the window starts 8 columns left of the block, so that it is 16-byte aligned in LDS and in the
// field; the band sits inside K = 32 for every r <= 8)
// -- one v_mfma_f32_16x16x32_bf16 per (dy, operand-part pair).  U is the A operand and T the B
// operand; T depends on the weights only, so its fragments are built once per workgroup and kept
// in registers.  Every FP32 value enters as three BF16 parts, x = x0 + x1 + x2 exactly (each part
// is the nearest BF16 of what the previous parts leave; 3 x 8 significant bits cover FP32's 24),
// and the six products whose weight is at least 2^-16 relative -- u0w0, u0w1, u1w0, u0w2, u1w1,
// u2w0 -- are accumulated in FP32 by the MFMA (the leading one and the five others in separate
// accumulators, summed at the end); the three dropped ones are below 2^-24 relative, FP32's own
// rounding.  The result is therefore not the canonical FMA order bit for
// bit but within FP32 rounding of it (rel-L2 against FP64 is the gate).  Redundancy: a 32-wide K
// for 2r + 1 useful taps per row, i.e. 32 / (2r + 1) times the useful multiply-adds, six times over.
//
// A workgroup (4 wavefronts) computes a 64 x 64 output tile: its (64 + 2r) x 80 input window
// (columns x0 - 8 .. x0 + 71) is loaded once with 16-byte loads, split, and staged in LDS as three
// BF16 planes (8-byte stores); wavefront w owns the 16-column strip
// w and its four 16-row blocks, which it advances together (four independent accumulators).  One
// level per pass.
#include <algorithm>

#include "internal.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_m;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_m;

namespace st {

namespace {

constexpr int MT = 64;            // output tile side
constexpr int LW = 80;            // staged columns: x0 - 8 .. x0 + 71 (the last strip's 32-wide window)
constexpr int LS = 88;            // LDS row stride in BF16 elements (176 bytes: staggers the 16 rows of a read)
constexpr int NTM = 256;

struct MfmaArgs {
    const float* src;
    float* dst;
    int64_t rows, cols;
    int64_t tiles_x;
    int vec;  // rows are 16-byte aligned (cols % 4 == 0, aligned field): 16-byte loads
    float b;
    float w[MAXK];
};

__device__ __forceinline__ void split3(float x, __bf16& p0, __bf16& p1, __bf16& p2) {
    p0 = (__bf16)x;
    const float r1 = x - float(p0);  // exact: x and its nearest BF16 share all but the low 16 bits
    p1 = (__bf16)r1;
    const float r2 = r1 - float(p1);  // exact, at most 8 significant bits: fits p2
    p2 = (__bf16)r2;
}

template <int R, int SHAPE>
__global__ __launch_bounds__(NTM) void sweep_mfma(MfmaArgs a) {
    constexpr int K = 2 * R + 1;
    constexpr int LR = MT + 2 * R;  // staged rows
    __shared__ __attribute__((aligned(16))) __bf16 plane[3][LR * LS];
    const int64_t tile = blockIdx.x;
    const int64_t y0 = (tile / a.tiles_x) * MT, x0 = (tile % a.tiles_x) * MT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, n = lane & 15;

    // B fragments: lane holds T[8q + t][n] for t = 0..7, per footprint row and weight part
    bf16x8_m bw[K][3];
#pragma unroll
    for (int dy = 0; dy < K; ++dy) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int d = 8 * q + t - 8 - n + R;  // dx + r
            float wv = 0.0f;
            if (d >= 0 && d < K && (SHAPE == SHAPE_BOX || dy == R || d == R)) wv = a.w[dy * K + d];
            __bf16 p0, p1, p2;
            split3(wv, p0, p1, p2);
            bw[dy][0][t] = p0;
            bw[dy][1][t] = p1;
            bw[dy][2][t] = p2;
        }
    }
    // stage the input window as three BF16 planes (out-of-grid cells hold b), four cells at a time
    for (int e = threadIdx.x; e < LR * (LW / 4); e += NTM) {
        const int r = e / (LW / 4), c = 4 * (e % (LW / 4));
        const int64_t gy = y0 - R + r, gx = x0 - 8 + c;
        float v[4];
        if (a.vec && gy >= 0 && gy < a.rows && gx >= 0 && gx + 4 <= a.cols) {
            const float4 f = *reinterpret_cast<const float4*>(a.src + gy * a.cols + gx);
            v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                v[t] = (gy >= 0 && gy < a.rows && gx + t >= 0 && gx + t < a.cols) ? a.src[gy * a.cols + gx + t] : a.b;
        }
        typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_m;
        bf16x4_m h0, h1, h2;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            __bf16 p0, p1, p2;
            split3(v[t], p0, p1, p2);
            h0[t] = p0;
            h1[t] = p1;
            h2[t] = p2;
        }
        *reinterpret_cast<bf16x4_m*>(&plane[0][r * LS + c]) = h0;
        *reinterpret_cast<bf16x4_m*>(&plane[1][r * LS + c]) = h1;
        *reinterpret_cast<bf16x4_m*>(&plane[2][r * LS + c]) = h2;
    }
    __syncthreads();
    // two accumulators per block: the leading products u0 w0, and the five smaller ones (about 2^-8
    // of the total, so their FP32 accumulation rounds 2^-8 as coarsely), added once at the end
    f32x4_m acc[4], low[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = low[rb] = f32x4_m{0.0f, 0.0f, 0.0f, 0.0f};
    const int col = wave * 16 + 8 * q;  // first staged column of this lane's A chunk
#pragma unroll
    for (int dy = 0; dy < K; ++dy) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int row = rb * 16 + n + dy;  // A row m = n (lane & 15) of block rb, footprint row dy
            const bf16x8_m a0 = *reinterpret_cast<const bf16x8_m*>(&plane[0][row * LS + col]);
            const bf16x8_m a1 = *reinterpret_cast<const bf16x8_m*>(&plane[1][row * LS + col]);
            const bf16x8_m a2 = *reinterpret_cast<const bf16x8_m*>(&plane[2][row * LS + col]);
            low[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bw[dy][0], low[rb], 0, 0, 0);
            low[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bw[dy][1], low[rb], 0, 0, 0);
            low[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bw[dy][2], low[rb], 0, 0, 0);
            low[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bw[dy][0], low[rb], 0, 0, 0);
            low[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bw[dy][1], low[rb], 0, 0, 0);
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bw[dy][0], acc[rb], 0, 0, 0);
        }
    }
    // C: lane holds rows 4q + v of column n of each block
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t gy = y0 + rb * 16 + 4 * q + v, gx = x0 + wave * 16 + n;
            if (gy < a.rows && gx < a.cols) a.dst[gy * a.cols + gx] = acc[rb][v] + low[rb][v];
        }
}

using FnM = void (*)(MfmaArgs);

FnM lookup_mfma(int shape, int r) {
    const bool box = shape == SHAPE_BOX;
    switch (r) {
        case 1: return box ? sweep_mfma<1, SHAPE_BOX> : sweep_mfma<1, SHAPE_STAR>;
        case 2: return box ? sweep_mfma<2, SHAPE_BOX> : sweep_mfma<2, SHAPE_STAR>;
        case 3: return box ? sweep_mfma<3, SHAPE_BOX> : sweep_mfma<3, SHAPE_STAR>;
        case 4: return box ? sweep_mfma<4, SHAPE_BOX> : sweep_mfma<4, SHAPE_STAR>;
    }
    return nullptr;
}

}  // namespace

bool mfma_usable(const st_plan* p) { return p->kind == KIND_CONST && p->storage == ST_F32 && p->bc == ST_BC_CONST; }

int launch_mfma(const st_plan* p, const void* src, void* dst, hipStream_t s) {
    FnM fn = lookup_mfma(p->shape, p->radius);
    if (!fn || !mfma_usable(p)) return fail(ST_EUNSUPPORTED, "no matrix-core kernel for this plan");
    MfmaArgs a;
    a.src = static_cast<const float*>(src);
    a.dst = static_cast<float*>(dst);
    a.rows = p->rows;
    a.cols = p->cols;
    a.tiles_x = (p->cols + MT - 1) / MT;
    a.vec = p->cols % 4 == 0 && reinterpret_cast<uintptr_t>(src) % 16 == 0;
    const int64_t tiles = a.tiles_x * ((p->rows + MT - 1) / MT);
    if (tiles > (int64_t(1) << 31) - 1) return fail(ST_EUNSUPPORTED, "grid too large for one launch");
    a.b = p->bq;
    std::memcpy(a.w, p->w, sizeof(a.w));
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(tiles)), dim3(NTM), 0, s, a);
    ST_LAUNCH_CHECK("sweep_mfma");
    return ST_OK;
}

}  // namespace st
