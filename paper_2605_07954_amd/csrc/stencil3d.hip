// 3D Jacobi stencil (the update of Sec. II-C on a planes x rows x cols grid, the constant halo of
// Sec. IV-A, the centre-first FP32 order of Sec. IV-E extended to (dz, dy, dx)):
//   u'(k, i, j) = sum_{dz, dy, dx in [-r, r]} W[dz+r][dy+r][dx+r] ~u(k+dz, i+dy, j+dx),
// per cell acc = W_c u_c, then one FMA per footprint tap in row-major (dz, dy, dx) order (star:
// the taps on the three axes; box: all of them).
//
// One workgroup owns a TY x TX column of the grid and marches along z over a segment of planes:
// the 2r + 1 input planes of the current output plane sit in an LDS ring, each with its r-deep
// (y, x) halo; every iteration stores a plane fetched earlier into the slot the oldest plane leaves,
// starts fetching the plane after next into registers (two register sets, so two planes are in
// flight), and computes its cells of the output plane from the ring meanwhile.  A wavefront covers one row of the
// tile (64 consecutive columns), so loads and stores are coalesced and LDS reads of one tap hit 64
// consecutive words.  One level per pass (no temporal blocking): HBM-bound for the 7-point star
// (8 bytes and 13 FLOP per update), LDS-bound for large boxes.
#include <algorithm>

#include "internal.h"
#include "storage.h"

namespace st {

namespace {

constexpr int TX = 64, TY = 32, NT3 = 256;
constexpr int ROWS_PER_THREAD = TY / (NT3 / TX);  // 8

struct Args3 {
    const void* src;
    void* dst;
    int64_t planes, rows, cols;
    int64_t tiles_x, tiles_y, zseg;  // tile grid and planes per segment
    float b;
    float w[MAXK3];
};

// One plane of the tile with its r-deep (y, x) halo, in the storage type's FP32 values: fetched into
// registers (PER values per thread) while the previous plane computes, stored into LDS afterwards.
template <int R>
struct PlaneRegs {
    static constexpr int PW = TX + 2 * R, PH = TY + 2 * R, PS = PW * PH;
    static constexpr int PER = (PS + NT3 - 1) / NT3;
    float v[PER];
};

template <int S, int R>
__device__ __forceinline__ void fetch_plane(const Args3& a, PlaneRegs<R>& p, int64_t z, int64_t y0, int64_t x0) {
    using T = typename Fmt<S>::T;
    using P = PlaneRegs<R>;
    const T* src = static_cast<const T*>(a.src);
    const bool zin = z >= 0 && z < a.planes;
#pragma unroll
    for (int j = 0; j < P::PER; ++j) {
        const int k = int(threadIdx.x) + NT3 * j;
        const int py = k / P::PW, px = k % P::PW;
        const int64_t y = y0 - R + py, x = x0 - R + px;
        float v = a.b;
        if (k < P::PS && zin && y >= 0 && y < a.rows && x >= 0 && x < a.cols) v = Fmt<S>::ld(src[(z * a.rows + y) * a.cols + x]);
        p.v[j] = v;
    }
}

template <int R>
__device__ __forceinline__ void store_plane(float* slot, const PlaneRegs<R>& p) {
    using P = PlaneRegs<R>;
#pragma unroll
    for (int j = 0; j < P::PER; ++j) {
        const int k = int(threadIdx.x) + NT3 * j;
        if (k < P::PS) slot[k] = p.v[j];
    }
}

template <int S, int R, int SHAPE>
__global__ __launch_bounds__(NT3) void sweep3d(Args3 a) {
    constexpr int K = 2 * R + 1;
    using P = PlaneRegs<R>;
    constexpr int PW = P::PW, PS = P::PS;
    __shared__ float ring[K][PS];
    const int64_t t = blockIdx.x;
    const int64_t tile = t % (a.tiles_x * a.tiles_y), seg = t / (a.tiles_x * a.tiles_y);
    const int64_t y0 = (tile / a.tiles_x) * TY, x0 = (tile % a.tiles_x) * TX;
    const int64_t z0 = seg * a.zseg, z1 = z0 + a.zseg < a.planes ? z0 + a.zseg : a.planes;
    const int tx = threadIdx.x % TX, ty0 = threadIdx.x / TX;
    using T = typename Fmt<S>::T;
    T* dst = static_cast<T*>(a.dst);
    // planes z0 - R .. z0 + R - 1 into slots; plane z lives in slot (z - z0 + R) mod K
    P pre;
    for (int q = 0; q < 2 * R; ++q) {
        fetch_plane<S, R>(a, pre, z0 - R + q, y0, x0);
        store_plane<R>(ring[q], pre);
    }
    // planes fetched two ahead (two register sets, the loop unrolled by two): twice the bytes in
    // flight per workgroup while a plane computes
    P pre2;
    fetch_plane<S, R>(a, pre, z0 + R, y0, x0);
    if (z0 + 1 < z1) fetch_plane<S, R>(a, pre2, z0 + 1 + R, y0, x0);
    auto compute = [&](int64_t z) {
        const int c_slot = int((z - z0 + R) % K);
#pragma unroll
        for (int rr = 0; rr < ROWS_PER_THREAD; ++rr) {
            const int ty = ty0 + rr * (NT3 / TX);
            const int o = (ty + R) * PW + tx + R;  // the cell's offset within a plane tile
            float acc = a.w[(R * K + R) * K + R] * ring[c_slot][o];
#pragma unroll
            for (int dz = -R; dz <= R; ++dz) {
                const float* pl = ring[(c_slot + dz + K) % K];
#pragma unroll
                for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        const int nz = (dz != 0) + (dy != 0) + (dx != 0);
                        if (nz == 0 || (SHAPE == SHAPE_STAR && nz > 1)) continue;
                        acc = __builtin_fmaf(a.w[((dz + R) * K + dy + R) * K + dx + R], pl[o + dy * PW + dx], acc);
                    }
            }
            const int64_t y = y0 + ty, x = x0 + tx;
            if (y < a.rows && x < a.cols) dst[(z * a.rows + y) * a.cols + x] = Fmt<S>::st(acc);
        }
    };
    for (int64_t z = z0; z < z1; z += 2) {
        store_plane<R>(ring[int((z - z0 + 2 * R) % K)], pre);  // plane z + R
        __syncthreads();
        if (z + 2 < z1) fetch_plane<S, R>(a, pre, z + 2 + R, y0, x0);
        compute(z);
        __syncthreads();  // every thread is done with the slot the next store overwrites
        if (z + 1 >= z1) break;
        store_plane<R>(ring[int((z + 1 - z0 + 2 * R) % K)], pre2);  // plane z + 1 + R
        __syncthreads();
        if (z + 3 < z1) fetch_plane<S, R>(a, pre2, z + 3 + R, y0, x0);
        compute(z + 1);
        __syncthreads();
    }
}

using Fn3 = void (*)(Args3);

template <int S, int SH>
Fn3 lookup3(int r) {
    if (r == 1) return sweep3d<S, 1, SH>;
    if (r == 2) return sweep3d<S, 2, SH>;
    return nullptr;
}

Fn3 lookup3(int storage, int shape, int r) {
    const bool box = shape == SHAPE_BOX;
    if (storage == ST_F32) return box ? lookup3<ST_F32, SHAPE_BOX>(r) : lookup3<ST_F32, SHAPE_STAR>(r);
    if (storage == ST_BF16) return box ? lookup3<ST_BF16, SHAPE_BOX>(r) : lookup3<ST_BF16, SHAPE_STAR>(r);
    if (storage == ST_F16) return box ? lookup3<ST_F16, SHAPE_BOX>(r) : lookup3<ST_F16, SHAPE_STAR>(r);
    return nullptr;
}

}  // namespace

int launch_3d(const st_plan* p, const void* src, void* dst, hipStream_t s) {
    Fn3 fn = lookup3(p->storage, p->shape, p->radius);
    if (!fn) return fail(ST_EUNSUPPORTED, "no 3D kernel for this storage/shape/radius");
    Args3 a;
    a.src = src;
    a.dst = dst;
    a.planes = p->planes;
    a.rows = p->rows;
    a.cols = p->cols;
    a.b = p->bq;
    std::memcpy(a.w, p->w3, sizeof(a.w));
    a.tiles_x = (p->cols + TX - 1) / TX;
    a.tiles_y = (p->rows + TY - 1) / TY;
    int blocks = 0;
    if (int rc = resident_blocks(reinterpret_cast<const void*>(fn), 0, &blocks)) return rc;
    // z segments so that the launch about fills the device once; each segment reloads 2r planes
    const int64_t tiles = a.tiles_x * a.tiles_y;
    const int64_t segs = std::max<int64_t>(1, std::min<int64_t>(p->planes, (blocks + tiles - 1) / tiles));
    a.zseg = (p->planes + segs - 1) / segs;
    const int64_t nseg = (p->planes + a.zseg - 1) / a.zseg;
    const int64_t grid = tiles * nseg;
    if (grid > (int64_t(1) << 31) - 1) return fail(ST_EUNSUPPORTED, "3D grid too large for one launch");
    clear_stale_error();
    hipLaunchKernelGGL(fn, dim3(unsigned(grid)), dim3(NT3), 0, s, a);
    ST_LAUNCH_CHECK("sweep3d");
    return ST_OK;
}

}  // namespace st
