// LDS-resident multi-workgroup sweep: the paper's mapping of one tile per processing element, kept
// in on-chip memory for every step, with a halo swap gated by completion counters (Sec. IV-B and
// IV-C), transplanted to one cooperative launch.  Each workgroup owns one tile of the grid for the
// whole run, in LDS; every tb steps ("epoch") it publishes its tile to a global exchange field,
// raises its counter, waits until its eight neighbours raised theirs, reads the r*tb-deep halo
// ring from the exchange field, and advances its tile tb levels in LDS (the region shrinking by r
// per level, as in the tiled passes).  The per-cell FP32 order is the canonical one (centre product,
// then one FMA per footprint tap in row-major order), so results equal every other kernel's bit for
// bit.
//
// Exchange fields alternate between the workspace and `out`, arranged so that the last epoch
// exchanges through the workspace and the final tiles go to `out` (which no neighbour reads any
// more by then).  A workgroup writes exchange field e+2 only after it saw its neighbours publish
// epoch e+1, which they do only after they finished reading field e: two fields suffice.
//
// Ordering: the tile's stores and the neighbours' halo loads are device-scope relaxed atomics
// (coherent across the XCDs' L2 caches); a workgroup waits for its stores to complete before its
// thread 0 raises the counter, and a reader issues its halo loads only after its counter poll
// returned the new value.
//
// Every wait is bounded: thread 0 polls a neighbour's counter at most spin_limit times (in total
// per epoch), checks a shared give-up flag every 64 polls, and on running out raises the flag and
// records (workgroup, epoch, neighbour); every workgroup that sees the flag leaves its epoch loop,
// so the kernel always ends.  The host reads the record with stencil_resident_status.  The launch
// is cooperative, so either every workgroup is resident at once or the launch fails.
#include <algorithm>

#include "internal.h"
#include "storage.h"

namespace st {

namespace {

constexpr int NTR = 256;

struct ResArgs {
    const void* in;
    void* out;
    void* ws;
    int* flags;   // [gy * gx] epochs published, zeroed before the launch
    int* status;  // [4]: give-up flag, workgroup, epoch, neighbour
    int64_t rows, cols;
    int gy, gx;   // workgroup grid
    int TY, TX;   // largest tile (the LDS buffers' interior)
    int H;        // halo depth r * tb
    int tb, steps;
    int64_t spin_limit;
    float b;
    float w[MAXK];
};

__device__ __forceinline__ int64_t part_lo(int i, int n, int64_t len) { return (len * i) / n; }

template <int S>
__device__ __forceinline__ typename Fmt<S>::T* as_field(void* p) {
    return static_cast<typename Fmt<S>::T*>(p);
}

// Exchange-field accesses as device-scope relaxed atomics: coherent across the chip's L2 caches
// without the whole-cache write-back and invalidate of a device-scope fence (which cost ~40 us
// per swap with one fence pair per workgroup and epoch).
template <typename T>
__device__ __forceinline__ void xstore(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xload(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every neighbour of workgroup (ty, tx) published epoch `want`.  Returns true when the
// run must stop (this wait gave up, or another workgroup did).
__device__ bool wait_neighbours(const ResArgs& a, int ty, int tx, int want, int wg) {
    int64_t spins = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int ny = ty + dy, nx = tx + dx;
            if ((dy == 0 && dx == 0) || ny < 0 || ny >= a.gy || nx < 0 || nx >= a.gx) continue;
            const int nb = ny * a.gx + nx;
            while (__hip_atomic_load(a.flags + nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
                ++spins;
                if ((spins & 63) == 0 &&
                    __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                    return true;
                if (spins > a.spin_limit) {
                    if (atomicCAS(a.status, 0, 1) == 0) {
                        __hip_atomic_store(a.status + 1, wg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(a.status + 2, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(a.status + 3, nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    return true;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    return false;
}

template <int S, int R, int SHAPE>
__global__ __launch_bounds__(NTR) void sweep_resident(ResArgs a) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    __shared__ int quit;
    constexpr int K = 2 * R + 1;
    const int H = a.H;
    const int BW = a.TX + 2 * H, BH = a.TY + 2 * H;
    float* bufs[2] = {lds, lds + BH * BW};
    const int wg = blockIdx.x;
    const int ty = wg / a.gx, tx = wg % a.gx;
    const int64_t y0 = part_lo(ty, a.gy, a.rows), y1 = part_lo(ty + 1, a.gy, a.rows);
    const int64_t x0 = part_lo(tx, a.gx, a.cols), x1 = part_lo(tx + 1, a.gx, a.cols);
    const int th = int(y1 - y0), tw = int(x1 - x0);
    using T = typename Fmt<S>::T;
    const T* in = static_cast<const T*>(a.in);
    float wv[K * K];
#pragma unroll
    for (int q = 0; q < K * K; ++q) wv[q] = a.w[q];
    // the tile's initial state; buffer cell (y, x) holds grid cell (y0 + y - H, x0 + x - H)
    int cur = 0;
    for (int k = threadIdx.x; k < th * tw; k += NTR) {
        const int y = k / tw, x = k % tw;
        bufs[0][(y + H) * BW + x + H] = Fmt<S>::ld(in[(y0 + y) * a.cols + x0 + x]);
    }
    const int E = (a.steps + a.tb - 1) / a.tb;
    bool stopped = false;
    for (int e = 0; e < E; ++e) {
        T* xg = as_field<S>(((E - 1 - e) % 2 == 0) ? a.ws : a.out);  // exchange field of epoch e
        __syncthreads();  // the tile's state is complete in bufs[cur]
        for (int k = threadIdx.x; k < th * tw; k += NTR) {
            const int y = k / tw, x = k % tw;
            xstore(xg + (y0 + y) * a.cols + x0 + x, Fmt<S>::st(bufs[cur][(y + H) * BW + x + H]));
        }
        // every store of the tile has completed (reached the device's coherence point) before the
        // counter is raised; the readers load the field at that point too, after seeing the counter
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(a.flags + wg, e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            quit = wait_neighbours(a, ty, tx, e + 1, wg) ? 1 : 0;
        }
        __syncthreads();
        if (quit) {
            stopped = true;
            break;
        }
        // the halo ring: the H-deep band around the tile, from the exchange field (b outside the grid)
        float* cb = bufs[cur];
        const int RW = tw + 2 * H, RH = th + 2 * H;
        for (int k = threadIdx.x; k < RW * RH; k += NTR) {
            const int y = k / RW, x = k % RW;  // buffer coordinates
            if (y >= H && y < H + th && x >= H && x < H + tw) continue;
            const int64_t gyy = y0 + y - H, gxx = x0 + x - H;
            float v = a.b;
            if (gyy >= 0 && gyy < a.rows && gxx >= 0 && gxx < a.cols) v = Fmt<S>::ld(xload(xg + gyy * a.cols + gxx));
            cb[y * BW + x] = v;
        }
        __syncthreads();
        const int levels = min(a.tb, a.steps - e * a.tb);
        for (int l = 1; l <= levels; ++l) {
            const float* sb = bufs[cur];
            float* db = bufs[cur ^ 1];
            const int lo = l * R;  // level l is exact on buffer rows/cols [lo, extent - lo)
            const int ch = RH - 2 * lo, cw = RW - 2 * lo;
            for (int k = threadIdx.x; k < ch * cw; k += NTR) {
                const int y = lo + k / cw, x = lo + k % cw;
                const int64_t gyy = y0 + y - H, gxx = x0 + x - H;
                float o = a.b;
                if (gyy >= 0 && gyy < a.rows && gxx >= 0 && gxx < a.cols) {
                    const float* c = sb + y * BW + x;
                    o = wv[R * K + R] * c[0];
#pragma unroll
                    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                        for (int dx = -R; dx <= R; ++dx) {
                            if ((dy == 0 && dx == 0) || (SHAPE == SHAPE_STAR && dy != 0 && dx != 0)) continue;
                            o = __builtin_fmaf(wv[(dy + R) * K + dx + R], c[dy * BW + dx], o);
                        }
                    o = Fmt<S>::rnd(o);
                }
                db[y * BW + x] = o;
            }
            cur ^= 1;
            __syncthreads();
        }
    }
    if (stopped) return;
    T* out = as_field<S>(a.out);
    for (int k = threadIdx.x; k < th * tw; k += NTR) {
        const int y = k / tw, x = k % tw;
        out[(y0 + y) * a.cols + x0 + x] = Fmt<S>::st(bufs[cur][(y + H) * BW + x + H]);
    }
}

__global__ void resident_reset(int* flags, int n, int* status) {
    const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = 0;
    if (i < 4) status[i] = 0;
}

using FnR = void (*)(ResArgs);

template <int S, int SH>
FnR lookup_res(int r) {
    switch (r) {
        case 1: return sweep_resident<S, 1, SH>;
        case 2: return sweep_resident<S, 2, SH>;
        case 3: return sweep_resident<S, 3, SH>;
        case 4: return sweep_resident<S, 4, SH>;
    }
    return nullptr;
}

FnR lookup_res(int storage, int shape, int r) {
    const bool box = shape == SHAPE_BOX;
    if (storage == ST_F32) return box ? lookup_res<ST_F32, SHAPE_BOX>(r) : lookup_res<ST_F32, SHAPE_STAR>(r);
    if (storage == ST_BF16) return box ? lookup_res<ST_BF16, SHAPE_BOX>(r) : lookup_res<ST_BF16, SHAPE_STAR>(r);
    if (storage == ST_F16) return box ? lookup_res<ST_F16, SHAPE_BOX>(r) : lookup_res<ST_F16, SHAPE_STAR>(r);
    return nullptr;
}

// Workgroup grid of a plan: the most square gy x gx with gy * gx <= the device's compute units
// (one workgroup per unit), every tile at least r * tb cells on each side (so that a halo comes
// from the eight direct neighbours only) and the largest tile's two LDS buffers within the limit.
struct ResGeo {
    int gy, gx, TY, TX;
    size_t lds;
};

bool res_geometry(const st_plan* p, int tb, int cus, ResGeo* g) {
    const int H = p->radius * tb;
    bool found = false;
    int64_t best = 0;
    for (int gy = 1; gy <= cus; ++gy) {
        const int gx = cus / gy;
        if (gy > p->rows || gx > p->cols) continue;
        const int64_t tymin = p->rows / gy, txmin = p->cols / gx;
        if (tymin < H || txmin < H) continue;
        const int TY = int((p->rows + gy - 1) / gy), TX = int((p->cols + gx - 1) / gx);
        const size_t lds = size_t(2) * size_t(TY + 2 * H) * size_t(TX + 2 * H) * sizeof(float);
        if (lds > lds_limit()) continue;
        // prefer more workgroups, then squarer tiles (less halo per cell)
        const int64_t score = int64_t(gy) * gx * 1000000 - int64_t(TY + TX);
        if (!found || score > best) {
            found = true;
            best = score;
            *g = ResGeo{gy, gx, TY, TX, lds};
        }
    }
    return found;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return cus;
}

}  // namespace

size_t resident_ws_tail() { return 64 * 1024; }

bool resident_usable(const st_plan* p, int tb) {
    if (p->kind != KIND_CONST || p->bc != ST_BC_CONST) return false;
    const int cus = device_cus();
    if (cus <= 0) return false;
    ResGeo g;
    return res_geometry(p, tb, std::min(cus, int(resident_ws_tail() / sizeof(int)) - 16), &g);
}

int resident_max_tb(const st_plan* p) {
    int tb = 0;
    for (int t = 1; t <= 64; ++t)
        if (resident_usable(p, t)) tb = t;
    return tb;
}

int launch_resident(const st_plan* p, const void* in, void* out, void* ws, int64_t steps, hipStream_t s) {
    const int cus = device_cus();
    ResGeo g;
    if (cus <= 0 || !res_geometry(p, p->tb, std::min(cus, int(resident_ws_tail() / sizeof(int)) - 16), &g))
        return fail(ST_EUNSUPPORTED, "grid does not fit the resident variant at this depth");
    FnR fn = lookup_res(p->storage, p->shape, p->radius);
    if (!fn) return fail(ST_EUNSUPPORTED, "no resident kernel for this storage/shape/radius");
    if (int rc = prepare_lds(reinterpret_cast<const void*>(fn), g.lds)) return rc;
    const size_t field = (size_t(field_cells(p)) * elem_size(p->storage) + 255) & ~size_t(255);
    ResArgs a;
    a.in = in;
    a.out = out;
    a.ws = ws;
    a.flags = reinterpret_cast<int*>(static_cast<char*>(ws) + field);
    a.status = a.flags + (resident_ws_tail() / sizeof(int) - 16);
    a.rows = p->rows;
    a.cols = p->cols;
    a.gy = g.gy;
    a.gx = g.gx;
    a.TY = g.TY;
    a.TX = g.TX;
    a.H = p->radius * p->tb;
    a.tb = p->tb;
    a.steps = int(steps);
    a.spin_limit = p->spin_limit;
    a.b = p->bq;
    std::memcpy(a.w, p->w, sizeof(a.w));
    const int n = g.gy * g.gx;
    clear_stale_error();
    hipLaunchKernelGGL(resident_reset, dim3((n + 255) / 256), dim3(256), 0, s, a.flags, n, a.status);
    ST_LAUNCH_CHECK("resident_reset");
    void* args[] = {&a};
    ST_HIP_CHECK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(fn), dim3(n), dim3(NTR), args,
                                            unsigned(g.lds), s));
    return ST_OK;
}

int read_resident_status(const st_plan* p, const void* ws, int* status4, hipStream_t s) {
    const size_t field = (size_t(field_cells(p)) * elem_size(p->storage) + 255) & ~size_t(255);
    const int* st = reinterpret_cast<const int*>(static_cast<const char*>(ws) + field) +
                    (resident_ws_tail() / sizeof(int) - 16);
    ST_HIP_CHECK(hipMemcpyAsync(status4, st, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    ST_HIP_CHECK(hipStreamSynchronize(s));
    return ST_OK;
}

}  // namespace st
