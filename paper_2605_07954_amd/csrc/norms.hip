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
    int64_t rows, cols;
    int r;
    double b;
    double wsum;
    float w[MAXK];
};

template <int S>
__global__ __launch_bounds__(NT) void norms_stage1(NormArgs a) {
    using F = Fmt<S>;
    using T = typename F::T;
    const T* u = static_cast<const T*>(a.u);
    const T* up = static_cast<const T*>(a.up);
    const int64_t n = a.rows * a.cols;
    const int r = a.r, k = 2 * r + 1;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int64_t idx = int64_t(blockIdx.x) * NT + threadIdx.x; idx < n; idx += int64_t(NBLK) * NT) {
        const double x = double(F::ld(u[idx]));
        if (up) {
            const double d = x - double(F::ld(up[idx]));
            s0 += d * d;
        }
        s1 += x * x;
        s2 += x;
        const int64_t i = idx / a.cols, j = idx - i * a.cols;
        double sup;
        if (i >= r && i < a.rows - r && j >= r && j < a.cols - r) {
            sup = a.wsum;
        } else {
            // S_j = sum of the weights W_d whose source cell j - d lies in the grid, in row-major tap order
            sup = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    const float w = a.w[(dy + r) * k + dx + r];
                    if (w == 0.0f) continue;
                    const int64_t si = i - dy, sj = j - dx;
                    if (si >= 0 && si < a.rows && sj >= 0 && sj < a.cols) sup += double(w);
                }
        }
        s3 += (x - a.b) * sup;
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
    if (!plan || !u || !out4) return fail(ST_EINVAL, "NULL argument");
    if (!workspace || ws_bytes < size_t(NBLK) * 4 * sizeof(double)) return fail(ST_ENOWS, "workspace too small");
    NormArgs a;
    a.u = u;
    a.up = u_prev;
    a.partial = static_cast<double*>(workspace);
    a.out4 = out4;
    a.rows = plan->rows;
    a.cols = plan->cols;
    a.r = plan->radius;
    a.b = double(plan->bq);
    a.wsum = plan->wsum;
    std::memcpy(a.w, plan->w, sizeof(a.w));
    if (plan->kind == KIND_VARCOEF) {
        // the next-step mass of the varcoef update depends on kappa; report the first three only
        a.r = 1;
        a.wsum = 1.0;
        std::memset(a.w, 0, sizeof(a.w));
        a.w[4] = 1.0f;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    clear_stale_error();
    switch (plan->storage) {
        case ST_F32: hipLaunchKernelGGL(norms_stage1<ST_F32>, dim3(NBLK), dim3(NT), 0, s, a); break;
        case ST_BF16: hipLaunchKernelGGL(norms_stage1<ST_BF16>, dim3(NBLK), dim3(NT), 0, s, a); break;
        case ST_F16: hipLaunchKernelGGL(norms_stage1<ST_F16>, dim3(NBLK), dim3(NT), 0, s, a); break;
        default: return fail(ST_EINVAL, "bad storage");
    }
    ST_LAUNCH_CHECK("norms_stage1");
    hipLaunchKernelGGL(norms_stage2, dim3(1), dim3(NT), 0, s, a);
    ST_LAUNCH_CHECK("norms_stage2");
    return ST_OK;
}
