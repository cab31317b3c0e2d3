// Batched persistent kernel: many independent grids of uneven size and mixed stencil shape in
// one launch.
//
// Work items are (grid, tile, pass).  Items are handed out by one atomic queue head in an
// order where every item's dependencies come earlier: first the whole-grid items (small grids
// that stay resident in LDS for all their steps), then the tiled items pass by pass.  Before a
// tiled item of pass p starts, the tiles around it must have finished pass p-1; each tile has a
// completion counter that its owner bumps after storing (the per-tile counterpart of the
// send/receive counters that gate the paper's halo swap, Sec. IV-C).  Because an item only ever
// waits on items handed out before it, which are held by running workgroups, the queue cannot
// deadlock; a spin limit still ends every wait so that a bug cannot hang the device (the
// timeout flag in the workspace header records it).
//
// Producer: stores -> __threadfence() (agent-scope release, makes the tile visible to other
// XCDs) -> barrier -> counter store.  Consumer: counter load -> __threadfence() (agent-scope
// acquire) -> barrier -> loads.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "sweep_body.h"

namespace st {

namespace {

struct BatchDesc {
    const float* in;
    float* out;
    float* ws;
    int64_t rows, cols;
    int64_t tiles_x, tiles_y;
    int64_t cnt_off;
    int r, shape, tile_id, tb, steps, passes, resident, pad;
    float b;
    float w[MAXK];
};

struct BatchArgs {
    unsigned long long* head;
    int* timeout_flag;
    int* counters;
    const BatchDesc* desc;
    const int64_t* pass_start;   // [max_passes + 1] item offsets of the tiled passes (after the resident items)
    const int64_t* tile_prefix;  // [n_tiled + 1] tile offsets within one pass, in queue order
    const int* order;            // [n]: resident grids first, then tiled grids by pass count, descending
    int64_t total;
    int n_res, n_tiled, max_passes;
    int64_t spin_limit;
};

constexpr int kBatchTiles[][2] = {{64, 64}, {128, 32}, {128, 64}, {256, 32}};
constexpr int kRS = 8;

template <int R, int SH>
__device__ __forceinline__ void run_tile(const BatchDesc& d, const float* src, float* dst, int levels, int64_t y0,
                                         int64_t x0, float* lds) {
    switch (d.tile_id) {
        case 0: tile_body<ST_F32, R, SH, 64, 64, kRS>(src, dst, d.rows, d.cols, d.b, levels, y0, x0, d.w, lds); break;
        case 1: tile_body<ST_F32, R, SH, 128, 32, kRS>(src, dst, d.rows, d.cols, d.b, levels, y0, x0, d.w, lds); break;
        case 2: tile_body<ST_F32, R, SH, 128, 64, kRS>(src, dst, d.rows, d.cols, d.b, levels, y0, x0, d.w, lds); break;
        default: tile_body<ST_F32, R, SH, 256, 32, kRS>(src, dst, d.rows, d.cols, d.b, levels, y0, x0, d.w, lds); break;
    }
}

__device__ __forceinline__ void dispatch_tile(const BatchDesc& d, const float* src, float* dst, int levels, int64_t y0,
                                              int64_t x0, float* lds) {
    if (d.shape == SHAPE_BOX) {
        switch (d.r) {
            case 1: run_tile<1, SHAPE_BOX>(d, src, dst, levels, y0, x0, lds); break;
            case 2: run_tile<2, SHAPE_BOX>(d, src, dst, levels, y0, x0, lds); break;
            default: run_tile<3, SHAPE_BOX>(d, src, dst, levels, y0, x0, lds); break;
        }
    } else {
        switch (d.r) {
            case 1: run_tile<1, SHAPE_STAR>(d, src, dst, levels, y0, x0, lds); break;
            case 2: run_tile<2, SHAPE_STAR>(d, src, dst, levels, y0, x0, lds); break;
            default: run_tile<3, SHAPE_STAR>(d, src, dst, levels, y0, x0, lds); break;
        }
    }
}

__device__ __forceinline__ void dispatch_resident(const BatchDesc& d, float* lds) {
    const int rows = int(d.rows), cols = int(d.cols);
    if (d.shape == SHAPE_BOX) {
        switch (d.r) {
            case 1: resident_body<1, SHAPE_BOX, kRS>(d.in, d.out, rows, cols, d.b, d.steps, d.w, lds); break;
            case 2: resident_body<2, SHAPE_BOX, kRS>(d.in, d.out, rows, cols, d.b, d.steps, d.w, lds); break;
            default: resident_body<3, SHAPE_BOX, kRS>(d.in, d.out, rows, cols, d.b, d.steps, d.w, lds); break;
        }
    } else {
        switch (d.r) {
            case 1: resident_body<1, SHAPE_STAR, kRS>(d.in, d.out, rows, cols, d.b, d.steps, d.w, lds); break;
            case 2: resident_body<2, SHAPE_STAR, kRS>(d.in, d.out, rows, cols, d.b, d.steps, d.w, lds); break;
            default: resident_body<3, SHAPE_STAR, kRS>(d.in, d.out, rows, cols, d.b, d.steps, d.w, lds); break;
        }
    }
}

// largest index i in [0, n) with a[i] <= x (a ascending, a[0] <= x)
__device__ __forceinline__ int upper_index(const int64_t* a, int n, int64_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(NT) void batched_persistent(BatchArgs a) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    __shared__ long long item_sh;
    for (;;) {
        if (threadIdx.x == 0) item_sh = (long long)atomicAdd(a.head, 1ull);
        __syncthreads();
        const long long item = item_sh;
        __syncthreads();
        if (item >= a.total) break;
        if (item < a.n_res) {
            const BatchDesc& d = a.desc[a.order[item]];
            dispatch_resident(d, lds);
            __syncthreads();
            continue;
        }
        const int64_t i = item - a.n_res;
        const int p = upper_index(a.pass_start, a.max_passes + 1, i);
        const int64_t o = i - a.pass_start[p];
        const int k = upper_index(a.tile_prefix, a.n_tiled + 1, o);
        const int g = a.order[a.n_res + k];
        const BatchDesc& d = a.desc[g];
        const int64_t t = o - a.tile_prefix[k];
        const int64_t ty = t / d.tiles_x, tx = t - ty * d.tiles_x;
        const int TX = kBatchTiles[d.tile_id][0], TY = kBatchTiles[d.tile_id][1];
        int* cnt = a.counters + d.cnt_off;
        if (p > 0 && threadIdx.x == 0) {
            // wait until every tile within reach of this tile's halo has finished pass p-1
            const int H = d.r * d.tb;
            const int ry = (H + TY - 1) / TY, rx = (H + TX - 1) / TX;
            int64_t spins = 0;
            for (int64_t yy = max<int64_t>(0, ty - ry); yy <= min<int64_t>(d.tiles_y - 1, ty + ry); ++yy)
                for (int64_t xx = max<int64_t>(0, tx - rx); xx <= min<int64_t>(d.tiles_x - 1, tx + rx); ++xx) {
                    const int* c = cnt + yy * d.tiles_x + xx;
                    int seen;
                    while ((seen = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < p) {
                        if (++spins > a.spin_limit) {
                            // first timeout wins the diagnostic record: item, grid, tile, pass,
                            // waited-on tile and the counter value it showed
                            if (atomicCAS(a.timeout_flag, 0, 1) == 0) {
                                long long* rec = reinterpret_cast<long long*>(a.timeout_flag) + 1;
                                rec[0] = item;
                                rec[1] = g;
                                rec[2] = t;
                                rec[3] = p;
                                rec[4] = yy * d.tiles_x + xx;
                                rec[5] = seen;
                            }
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            __threadfence();
        }
        __syncthreads();
        const int P = d.passes;
        const float* src = p == 0 ? d.in : (((P - p) % 2 == 0) ? d.out : d.ws);  // buffer written by pass p-1
        float* dst = ((P - 1 - p) % 2 == 0) ? d.out : d.ws;
        const int levels = min(d.tb, d.steps - p * d.tb);
        dispatch_tile(d, src, dst, levels, ty * TY, tx * TX, lds);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(cnt + t, p + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void batch_reset(unsigned long long* head, int* timeout_flag, int* counters, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) {
        *head = 0ull;
        *timeout_flag = 0;
    }
    if (i < 6) reinterpret_cast<long long*>(timeout_flag)[1 + i] = -1;
    for (int64_t k = i; k < n; k += int64_t(gridDim.x) * blockDim.x) counters[k] = 0;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int batch_tile_id(int tx, int ty) {
    for (int i = 0; i < 4; ++i)
        if (kBatchTiles[i][0] == tx && kBatchTiles[i][1] == ty) return i;
    return -1;
}

}  // namespace

}  // namespace st

using namespace st;

struct st_batch {
    int n;
    uint32_t flags;
    std::vector<BatchDesc> desc;
    std::vector<int64_t> pass_start, tile_prefix;
    std::vector<int> order;
    int n_res, n_tiled, max_passes;
    int64_t total_items, total_tiles;
    size_t off_cnt, off_desc, off_pstart, off_tprefix, off_order, off_fields, ws_bytes;
    std::vector<size_t> field_off;  // per grid: workspace offset of its ping-pong field (0 = none)
    std::vector<int> zero_steps;    // grids with steps == 0 (copied, not queued)
    int64_t spin_limit;             // polls before a dependency wait gives up
    size_t lds;
    int blocks;
    // staging + graph
    void* pinned;
    size_t pinned_bytes;
    hipEvent_t staged;
    bool staged_valid;
    std::vector<const void*> last_in;
    std::vector<void*> last_out;
    void* last_ws;
    hipGraphExec_t exec;
    void* g_ws;
    void* g_stream;
};

namespace {

// LDS budget per workgroup of the persistent kernel: two workgroups per CU when the device
// allows 80 KiB per workgroup.
size_t batch_lds_budget() { return std::min<size_t>(80 * 1024, lds_limit()); }

size_t tile_lds(int r, int tb, int tid) {
    return tiled_lds_bytes(r, tb, kBatchTiles[tid][0], kBatchTiles[tid][1]);
}

}  // namespace

extern "C" int stencil_batch_create(st_batch** out, int n, st_plan* const* plans, const int64_t* steps,
                                    uint32_t flags) {
    if (!out) return fail(ST_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !plans || !steps) return fail(ST_EINVAL, "need n >= 1 plans and steps");
    if (flags & ~ST_FLAG_GRAPH) return fail(ST_EINVAL, "unknown batch flag bits");
    st_batch* B = new (std::nothrow) st_batch();
    if (!B) return fail(ST_ENOMEM, "batch allocation failed");
    B->n = n;
    B->flags = flags;
    B->desc.resize(n);
    B->field_off.assign(n, 0);
    std::vector<int> res, tiled;
    int64_t cnt_total = 0;
    size_t lds_max = 0;
    for (int g = 0; g < n; ++g) {
        const st_plan* p = plans[g];
        if (!p || p->kind != KIND_CONST || p->storage != ST_F32 || p->radius > 3 || steps[g] < 0 ||
            steps[g] > (int64_t(1) << 30)) {
            delete B;
            return fail(p ? ST_EUNSUPPORTED : ST_EINVAL, "batched grids must be FP32 constant-weight plans, r <= 3");
        }
        BatchDesc& d = B->desc[g];
        std::memset(&d, 0, sizeof(d));
        d.rows = p->rows;
        d.cols = p->cols;
        d.r = p->radius;
        d.shape = p->shape;
        d.b = p->bq;
        d.steps = int(steps[g]);
        std::memcpy(d.w, p->w, sizeof(d.w));
        if (steps[g] == 0) {  // plain copy in -> out, enqueued by stencil_run_batched
            d.passes = 0;
            d.tiles_x = d.tiles_y = 1;
            B->zero_steps.push_back(g);
            continue;
        }
        const size_t rl = resident_lds_bytes(p->radius, p->rows, p->cols);
        if (rl <= batch_lds_budget()) {
            d.resident = 1;
            d.passes = 1;
            d.tb = d.steps;
            d.tiles_x = d.tiles_y = 1;
            lds_max = std::max(lds_max, rl);
            res.push_back(g);
            continue;
        }
        int tid = batch_tile_id(p->tile_x, p->tile_y);
        if (tid < 0) tid = 2;
        int tb = std::max(1, p->tb);
        while (tb > 1 && tile_lds(p->radius, tb, tid) > batch_lds_budget()) --tb;
        d.tile_id = tid;
        d.tb = tb;
        d.tiles_x = (p->cols + kBatchTiles[tid][0] - 1) / kBatchTiles[tid][0];
        d.tiles_y = (p->rows + kBatchTiles[tid][1] - 1) / kBatchTiles[tid][1];
        d.passes = d.steps == 0 ? 0 : (d.steps + tb - 1) / tb;
        d.cnt_off = cnt_total;
        cnt_total += d.tiles_x * d.tiles_y;
        lds_max = std::max(lds_max, tile_lds(p->radius, tb, tid));
        tiled.push_back(g);
    }
    std::stable_sort(tiled.begin(), tiled.end(),
                     [&](int a, int b) { return B->desc[a].passes > B->desc[b].passes; });
    B->n_res = int(res.size());
    B->n_tiled = int(tiled.size());
    B->order = res;
    B->order.insert(B->order.end(), tiled.begin(), tiled.end());
    B->tile_prefix.assign(1, 0);
    for (int g : tiled) B->tile_prefix.push_back(B->tile_prefix.back() + B->desc[g].tiles_x * B->desc[g].tiles_y);
    B->max_passes = tiled.empty() ? 0 : B->desc[tiled[0]].passes;
    B->pass_start.assign(1, 0);
    for (int p = 0; p < B->max_passes; ++p) {
        int active = 0;  // grids still running at pass p form a prefix of the tiled order (passes descending)
        while (active < B->n_tiled && B->desc[tiled[active]].passes > p) ++active;
        B->pass_start.push_back(B->pass_start.back() + B->tile_prefix[active]);
    }
    for (size_t k = 1; k < B->pass_start.size(); ++k)
        if (B->pass_start[k] <= B->pass_start[k - 1]) {  // every pass below max_passes has at least one tile
            delete B;
            return fail(ST_EINVAL, "internal: empty pass in the batch queue");
        }
    if (B->pass_start.size() < 2) B->pass_start.push_back(0);
    B->total_tiles = cnt_total;
    B->total_items = B->n_res + B->pass_start[B->max_passes];
    // workspace layout
    size_t off = 256;  // header: queue head (8 B), timeout flag (4 B), first-timeout record (6 x 8 B at 16)
    B->off_cnt = off;
    off = align256(off + size_t(std::max<int64_t>(cnt_total, 1)) * sizeof(int));
    B->off_desc = off;
    off = align256(off + size_t(n) * sizeof(BatchDesc));
    B->off_pstart = off;
    off = align256(off + B->pass_start.size() * sizeof(int64_t));
    B->off_tprefix = off;
    off = align256(off + B->tile_prefix.size() * sizeof(int64_t));
    B->off_order = off;
    off = align256(off + size_t(n) * sizeof(int));
    B->off_fields = off;
    for (int g : tiled) {
        if (B->desc[g].passes >= 2) {
            B->field_off[g] = off;
            off = align256(off + size_t(B->desc[g].rows * B->desc[g].cols) * sizeof(float));
        }
    }
    B->ws_bytes = off;
    B->lds = std::max<size_t>(lds_max, 16);
    B->pinned = nullptr;
    B->pinned_bytes = B->off_fields - B->off_desc;
    B->staged = nullptr;
    B->staged_valid = false;
    B->last_ws = nullptr;
    B->exec = nullptr;
    B->g_ws = nullptr;
    B->g_stream = nullptr;
    B->blocks = 0;
    // ~1 s of polling by default: far above any legitimate wait, and it ends a wait that a bug
    // would make endless.  MI355STENCIL_BATCH_SPIN overrides it (tests use a short limit).
    B->spin_limit = int64_t(1) << 20;
    if (const char* e = std::getenv("MI355STENCIL_BATCH_SPIN")) B->spin_limit = std::max<int64_t>(1, std::atoll(e));
    *out = B;
    return ST_OK;
}

extern "C" int stencil_batch_workspace_bytes(const st_batch* batch, size_t* bytes) {
    if (!batch || !bytes) return fail(ST_EINVAL, "NULL argument");
    *bytes = batch->ws_bytes;
    return ST_OK;
}

extern "C" int stencil_batch_destroy(st_batch* batch) {
    if (!batch) return ST_OK;
    if (batch->staged) {
        (void)hipEventSynchronize(batch->staged);
        (void)hipEventDestroy(batch->staged);
    }
    if (batch->pinned) (void)hipHostFree(batch->pinned);
    if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
    delete batch;
    return ST_OK;
}

static int enqueue_batch(st_batch* B, char* ws, hipStream_t s) {
    BatchArgs a;
    a.head = reinterpret_cast<unsigned long long*>(ws);
    a.timeout_flag = reinterpret_cast<int*>(ws + 8);
    a.counters = reinterpret_cast<int*>(ws + B->off_cnt);
    a.desc = reinterpret_cast<const BatchDesc*>(ws + B->off_desc);
    a.pass_start = reinterpret_cast<const int64_t*>(ws + B->off_pstart);
    a.tile_prefix = reinterpret_cast<const int64_t*>(ws + B->off_tprefix);
    a.order = reinterpret_cast<const int*>(ws + B->off_order);
    a.total = B->total_items;
    a.n_res = B->n_res;
    a.n_tiled = B->n_tiled;
    a.max_passes = B->max_passes;
    a.spin_limit = B->spin_limit;
    clear_stale_error();
    hipLaunchKernelGGL(batch_reset, dim3(64), dim3(256), 0, s, a.head, a.timeout_flag, a.counters,
                       std::max<int64_t>(B->total_tiles, 1));
    ST_LAUNCH_CHECK("batch_reset");
    hipLaunchKernelGGL(batched_persistent, dim3(B->blocks), dim3(NT), B->lds, s, a);
    ST_LAUNCH_CHECK("batched_persistent");
    return ST_OK;
}

extern "C" int stencil_run_batched(st_batch* B, const void* const* ins, void* const* outs, void* workspace,
                                   size_t ws_bytes, void* stream) {
    if (!B || !ins || !outs) return fail(ST_EINVAL, "NULL argument");
    if (!workspace || ws_bytes < B->ws_bytes) return fail(ST_ENOWS, "workspace too small");
    for (int g = 0; g < B->n; ++g) {
        if (!ins[g] || !outs[g]) return fail(ST_EINVAL, "NULL grid pointer");
        const size_t bytes = size_t(B->desc[g].rows * B->desc[g].cols) * sizeof(float);
        const char* x = static_cast<const char*>(ins[g]);
        const char* y = static_cast<const char*>(outs[g]);
        if (x < y + bytes && y < x + bytes) return fail(ST_EALIAS, "in and out overlap");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    if (!B->blocks) {
        if (int rc = prepare_lds(reinterpret_cast<const void*>(batched_persistent), B->lds)) return rc;
        int dev = 0, cus = 0, occ = 0;
        ST_HIP_CHECK(hipGetDevice(&dev));
        ST_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        ST_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batched_persistent, NT, B->lds));
        B->blocks = std::max(1, cus * std::max(occ, 1));
    }
    // stage the descriptor tables when any pointer changed since the last run
    bool changed = !B->staged_valid || B->last_ws != workspace;
    for (int g = 0; g < B->n && !changed; ++g) changed = B->last_in[g] != ins[g] || B->last_out[g] != outs[g];
    if (changed) {
        if (!B->pinned) {
            ST_HIP_CHECK(hipHostMalloc(&B->pinned, B->pinned_bytes, hipHostMallocDefault));
            ST_HIP_CHECK(hipEventCreateWithFlags(&B->staged, hipEventDisableTiming));
        } else {
            ST_HIP_CHECK(hipEventSynchronize(B->staged));  // the previous copy out of the staging buffer is done
        }
        char* h = static_cast<char*>(B->pinned);
        for (int g = 0; g < B->n; ++g) {
            BatchDesc d = B->desc[g];
            d.in = static_cast<const float*>(ins[g]);
            d.out = static_cast<float*>(outs[g]);
            d.ws = B->field_off[g] ? reinterpret_cast<float*>(ws + B->field_off[g]) : nullptr;
            std::memcpy(h + g * sizeof(BatchDesc), &d, sizeof(d));
        }
        std::memcpy(h + (B->off_pstart - B->off_desc), B->pass_start.data(), B->pass_start.size() * sizeof(int64_t));
        std::memcpy(h + (B->off_tprefix - B->off_desc), B->tile_prefix.data(),
                    B->tile_prefix.size() * sizeof(int64_t));
        std::memcpy(h + (B->off_order - B->off_desc), B->order.data(), B->order.size() * sizeof(int));
        ST_HIP_CHECK(hipMemcpyAsync(ws + B->off_desc, h, B->pinned_bytes, hipMemcpyHostToDevice, s));
        ST_HIP_CHECK(hipEventRecord(B->staged, s));
        B->staged_valid = true;
        B->last_in.assign(ins, ins + B->n);
        B->last_out.assign(outs, outs + B->n);
        B->last_ws = workspace;
    }
    for (int g : B->zero_steps)
        ST_HIP_CHECK(hipMemcpyAsync(outs[g], ins[g], size_t(B->desc[g].rows * B->desc[g].cols) * sizeof(float),
                                    hipMemcpyDeviceToDevice, s));
    if (B->total_items == 0) return ST_OK;
    if (!(B->flags & ST_FLAG_GRAPH)) return enqueue_batch(B, ws, s);
    if (!(B->exec && B->g_ws == workspace)) {
        if (B->exec) {
            (void)hipGraphExecDestroy(B->exec);
            B->exec = nullptr;
        }
        hipStream_t cap;
        ST_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return fail(ST_EHIP, "hipStreamBeginCapture failed");
        }
        const int rc = enqueue_batch(B, ws, cap);
        const hipError_t e = hipStreamEndCapture(cap, &graph);
        (void)hipStreamDestroy(cap);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(ST_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) return fail(ST_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
        B->g_ws = workspace;
    }
    ST_HIP_CHECK(hipGraphLaunch(B->exec, s));
    return ST_OK;
}

extern "C" int stencil_batch_status(const st_batch* batch, const void* workspace, int* timed_out, void* stream) {
    if (!batch || !workspace || !timed_out) return fail(ST_EINVAL, "NULL argument");
    int flag = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    ST_HIP_CHECK(hipMemcpyAsync(&flag, static_cast<const char*>(workspace) + 8, sizeof(int), hipMemcpyDeviceToHost, s));
    ST_HIP_CHECK(hipStreamSynchronize(s));
    *timed_out = flag;
    return ST_OK;
}
