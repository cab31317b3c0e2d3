// FP64 reductions of a field: residual^2, energy, mass and the mass of the next step (the
// quantities behind the paper's periodic host-side convergence check, Sec. IV).  Two stages with
// a fixed assignment of cells to threads and fixed-shape trees, so the sums are bitwise
// reproducible run to run.
#include "internal.h"
#include "storage.h"

namespace st {

namespace {

constexpr int NT = 256;
constexpr int NBLK = 1024;  // stage-1 blocks (fixed: part of the summation order)

struct NormArgs {
    const void* u;
    const void* up;
    double* partial;  // [NBLK][4]
    double* out4;
    const int* stop;  // nullable: a nonzero value skips the reduction
    int64_t rows, cols;
    int r;
    double b;
    double wsum;
    // 2D prefix sums of the FP64 weights: P[y][x] = sum of W[y'][x'] over y' < y, x' < x
    // (y, x in [0, 2r + 1], row stride 2r + 2)
    double P[(2 * ST_MAX_RADIUS + 2) * (2 * ST_MAX_RADIUS + 2)];
};

constexpr int PMAX = (2 * ST_MAX_RADIUS + 2) * (2 * ST_MAX_RADIUS + 2);

// Support sum S of cell (i, j): the sum of the weights W[dy][dx] whose source cell (i - dy, j - dx)
// lies in the grid -- wsum at least r from every edge, else the rectangle dy in [max(-r, i - rows
// + 1), min(r, i)], dx likewise, from four prefix sums.  O(1) per cell, so the threads whose cells
// lie on an edge cost no more than the rest.
__device__ __forceinline__ double support(const NormArgs& a, const double* P, int64_t i, int64_t j) {
    const int r = a.r;
    if (i >= r && i < a.rows - r && j >= r && j < a.cols - r) return a.wsum;
    const int64_t stride = 2 * r + 2;
    const int64_t y0 = (i - a.rows + 1 > -r ? i - a.rows + 1 : -r) + r, y1 = (i < r ? i : r) + r + 1;
    const int64_t x0 = (j - a.cols + 1 > -r ? j - a.cols + 1 : -r) + r, x1 = (j < r ? j : r) + r + 1;
    return P[y1 * stride + x1] - P[y0 * stride + x1] - P[y1 * stride + x0] + P[y0 * stride + x0];
}

__device__ __forceinline__ void accumulate(const NormArgs& a, const double* P, float xf, const float* xpf, int64_t i,
                                           int64_t j, double& s0, double& s1, double& s2, double& s3) {
    const double x = double(xf);
    if (xpf) {
        const double d = x - double(*xpf);
        s0 += d * d;
    }
    s1 += x * x;
    s2 += x;
    s3 += (x - a.b) * support(a, P, i, j);
}

// Stage 1: thread t of block g takes the cells (or, with VEC, the groups of four cells, which then
// never straddle a row) t + NT g, + NT NBLK, ... in that order; the row and column of each are
// stepped forward, not divided out per cell.
template <int S, bool VEC>
__global__ __launch_bounds__(NT) void norms_stage1(NormArgs a) {
    using F = Fmt<S>;
    using T = typename F::T;
    const T* u = static_cast<const T*>(a.u);
    const T* up = static_cast<const T*>(a.up);
    if (a.stop && __hip_atomic_load(a.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    __shared__ double P[PMAX];
    for (int t = threadIdx.x; t < PMAX; t += NT) P[t] = a.P[t];
    __syncthreads();
    constexpr int G = VEC ? 4 : 1;  // cells per item
    const int64_t items = (a.rows * a.cols) / G;  // VEC: cols % 4 == 0, so no partial item
    const int64_t stride = int64_t(NBLK) * NT;
    int64_t it = int64_t(blockIdx.x) * NT + threadIdx.x;
    // (i, j) of the item's first cell, and the row/column step of one stride
    int64_t i = (it * G) / a.cols, j = it * G - i * a.cols;
    const int64_t di = (stride * G) / a.cols, dj = stride * G - di * a.cols;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (; it < items; it += stride) {
        float x[G], xp[G];
        if constexpr (VEC) {
            if constexpr (S == ST_F32) {
                const float4 q = reinterpret_cast<const float4*>(u)[it];
                x[0] = q.x; x[1] = q.y; x[2] = q.z; x[3] = q.w;
                if (up) {
                    const float4 p = reinterpret_cast<const float4*>(up)[it];
                    xp[0] = p.x; xp[1] = p.y; xp[2] = p.z; xp[3] = p.w;
                }
            } else {
                const uint2 q = reinterpret_cast<const uint2*>(u)[it];
                x[0] = F::ld(T(q.x & 0xffffu)); x[1] = F::ld(T(q.x >> 16));
                x[2] = F::ld(T(q.y & 0xffffu)); x[3] = F::ld(T(q.y >> 16));
                if (up) {
                    const uint2 p = reinterpret_cast<const uint2*>(up)[it];
                    xp[0] = F::ld(T(p.x & 0xffffu)); xp[1] = F::ld(T(p.x >> 16));
                    xp[2] = F::ld(T(p.y & 0xffffu)); xp[3] = F::ld(T(p.y >> 16));
                }
            }
        } else {
            x[0] = F::ld(u[it]);
            if (up) xp[0] = F::ld(up[it]);
        }
#pragma unroll
        for (int e = 0; e < G; ++e) accumulate(a, P, x[e], up ? &xp[e] : nullptr, i, j + e, s0, s1, s2, s3);
        i += di;
        j += dj;
        if (j >= a.cols) {
            j -= a.cols;
            ++i;
        }
    }
    __shared__ double red[4][NT];
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    red[3][threadIdx.x] = s3;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) a.partial[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(NT) void norms_stage2(NormArgs a) {
    if (a.stop && __hip_atomic_load(a.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    __shared__ double red[4][NT];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double s = 0;
        for (int k = threadIdx.x; k < NBLK; k += NT) s += a.partial[k * 4 + q];
        red[q][threadIdx.x] = s;
    }
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.out4[0] = red[0][0];
        a.out4[1] = red[1][0];
        a.out4[2] = red[2][0];
        a.out4[3] = red[3][0] + a.b * double(a.rows * a.cols) * a.wsum;
    }
}

}  // namespace

}  // namespace st

using namespace st;

extern "C" int stencil_norms_ws_bytes(const st_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(ST_EINVAL, "NULL argument");
    *bytes = size_t(NBLK) * 4 * sizeof(double);
    return ST_OK;
}

extern "C" int stencil_norms(const st_plan* plan, const void* u_prev, const void* u, double* out4, void* workspace,
                             size_t ws_bytes, void* stream) {
    return launch_norms(plan, u_prev, u, out4, workspace, ws_bytes, nullptr, static_cast<hipStream_t>(stream));
}

int st::launch_norms(const st_plan* plan, const void* u_prev, const void* u, double* out4, void* workspace,
                     size_t ws_bytes, const int* stop, hipStream_t s) {
    if (!plan || !u || !out4) return fail(ST_EINVAL, "NULL argument");
    if (!workspace || ws_bytes < size_t(NBLK) * 4 * sizeof(double)) return fail(ST_ENOWS, "workspace too small");
    NormArgs a;
    a.stop = stop;
    a.u = u;
    a.up = u_prev;
    a.partial = static_cast<double*>(workspace);
    a.out4 = out4;
    a.rows = plan->rows;
    a.cols = plan->cols;
    a.r = plan->radius;
    a.b = double(plan->bq);
    a.wsum = plan->wsum;
    double w[MAXK] = {};
    const int k = 2 * plan->radius + 1;
    for (int t = 0; t < k * k; ++t) w[t] = double(plan->w[t]);
    if (plan->kind == KIND_3D) {
        // the first three sums over all cells (rows taken as planes * rows); no next-step mass
        a.rows = plan->planes * plan->rows;
        a.wsum = std::nan("");
        a.b = 0.0;
    }
    if (plan->bc == ST_BC_PERIODIC) {
        // every cell keeps the whole weight sum on a torus: next mass = sum(W) * sum(u)
        a.r = 0;
        a.b = 0.0;
    } else if (plan->bc == ST_BC_FRAME) {
        a.wsum = std::nan("");  // depends on the frame: reported as NaN
        a.b = 0.0;
    }
    if (plan->kind == KIND_VARCOEF) {
        // the next-step mass of the varcoef update depends on kappa; report the first three only
        a.r = 1;
        a.wsum = 1.0;
        std::fill(w, w + MAXK, 0.0);
        w[4] = 1.0;
    }
    const int kk = 2 * a.r + 1;
    std::fill(a.P, a.P + PMAX, 0.0);
    for (int y = 0; y < kk; ++y)
        for (int x = 0; x < kk; ++x)
            a.P[(y + 1) * (kk + 1) + x + 1] =
                w[y * kk + x] + a.P[y * (kk + 1) + x + 1] + a.P[(y + 1) * (kk + 1) + x] - a.P[y * (kk + 1) + x];
    // groups of four cells with one vector load each when rows hold whole groups and both fields
    // start on a group boundary (16 bytes for FP32, 8 for 16-bit storage)
    const size_t gbytes = plan->storage == ST_F32 ? 16 : 8;
    const bool vec = plan->cols % 4 == 0 && reinterpret_cast<uintptr_t>(u) % gbytes == 0 &&
                     reinterpret_cast<uintptr_t>(u_prev) % gbytes == 0;
    clear_stale_error();
#define ST_NORMS1(S)                                                                          \
    if (vec)                                                                                  \
        hipLaunchKernelGGL((norms_stage1<S, true>), dim3(NBLK), dim3(NT), 0, s, a);           \
    else                                                                                      \
        hipLaunchKernelGGL((norms_stage1<S, false>), dim3(NBLK), dim3(NT), 0, s, a);
    switch (plan->storage) {
        case ST_F32: ST_NORMS1(ST_F32) break;
        case ST_BF16: ST_NORMS1(ST_BF16) break;
        case ST_F16: ST_NORMS1(ST_F16) break;
        default: return fail(ST_EINVAL, "bad storage");
    }
#undef ST_NORMS1
    ST_LAUNCH_CHECK("norms_stage1");
    hipLaunchKernelGGL(norms_stage2, dim3(1), dim3(NT), 0, s, a);
    ST_LAUNCH_CHECK("norms_stage2");
    return ST_OK;
}
