// Batched sweep: many independent grids of uneven size and mixed stencil shape, run by one
// hipGraph launch.
//
// Small grids that fit a workgroup's LDS (with their halo and a ping-pong copy) are resident:
// one workgroup keeps the grid in LDS for all of its steps, so it never round-trips through HBM.
// The other grids are tiled; pass p of every tiled grid (tb steps each, as in the single-grid
// sweep) is one multi-grid kernel whose workgroups each take one (grid, tile) of that pass, so a
// pass of all grids costs one launch instead of one per grid.  Passes follow each other inside
// the graph, so the dependency of a tile on its neighbours' previous pass (the halo exchange of
// the paper's tiles, Sec. IV-B/C) is carried by the kernel boundary; the resident grids run on a
// parallel branch of the same graph.
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
    int r, shape, tb, steps, passes, resident;
    float b;
    float w[MAXK];
};

struct PassArgs {
    const BatchDesc* desc;
    const int* order;            // tiled grids by pass count, descending
    const int64_t* tile_prefix;  // [n_tiled + 1] tile offsets in that order
    int n_active;                // grids with more than p passes (a prefix of the order)
    int p;                       // pass index
};

// One tile shape for every tiled grid of a batch keeps the kernel's register use at the level of a
// single sweep body (each extra shape multiplies the inlined code).
constexpr int kTX = 128, kTY = 64, kRS = 8;

template <int R, int SH>
__device__ __forceinline__ void run_tile(const BatchDesc& d, const float* src, float* dst, int levels, int64_t y0,
                                         int64_t x0, float* lds) {
    tile_body<ST_F32, R, SH, kTX, kTY, kRS>(src, dst, d.rows, d.cols, d.b, levels, y0, x0, d.w, lds);
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

// One pass level of all tiled grids: workgroup o -> (grid, tile) through the tile prefix sums of
// the grids still active at this pass (a prefix of the queue order).
__global__ __launch_bounds__(NT) void batched_pass(PassArgs a) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    const int64_t o = blockIdx.x;
    const int k = upper_index(a.tile_prefix, a.n_active + 1, o);
    const BatchDesc& d = a.desc[a.order[k]];
    const int64_t t = o - a.tile_prefix[k];
    const int64_t ty = t / d.tiles_x, tx = t - ty * d.tiles_x;
    const int p = a.p, P = d.passes;
    const float* src = p == 0 ? d.in : (((P - p) % 2 == 0) ? d.out : d.ws);  // written by pass p-1
    float* dst = ((P - 1 - p) % 2 == 0) ? d.out : d.ws;
    const int levels = min(d.tb, d.steps - p * d.tb);
    dispatch_tile(d, src, dst, levels, ty * kTY, tx * kTX, lds);
}

// The LDS-resident grids: one workgroup per grid for all of its steps.
__global__ __launch_bounds__(NT) void batched_resident(const BatchDesc* desc, const int* res) {
    extern __shared__ float4 lds4[];
    dispatch_resident(desc[res[blockIdx.x]], reinterpret_cast<float*>(lds4));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }


}  // namespace

}  // namespace st

using namespace st;

struct st_batch {
    int n;
    uint32_t flags;
    std::vector<BatchDesc> desc;
    std::vector<int64_t> tile_prefix;  // over `order`
    std::vector<int> order;            // tiled grids by pass count, descending
    std::vector<int> res;              // LDS-resident grids
    std::vector<int> zero_steps;       // grids with steps == 0 (copied, not computed)
    std::vector<int> active;           // active[p]: tiled grids with more than p passes
    std::vector<int> tiled;            // tiled grids, in input order
    std::vector<int> tb_max;           // per grid: deepest pass the batch tile's LDS budget allows
    int max_passes;
    size_t off_desc, off_tprefix, off_order, off_res, off_fields, ws_bytes;
    std::vector<size_t> field_off;     // per grid: workspace offset of its ping-pong field (0 = none)
    size_t lds_pass, lds_res;
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
};

namespace {

// LDS budget per workgroup of the batched kernels: two workgroups per CU when the device allows
// 80 KiB per workgroup.
size_t batch_lds_budget() { return std::min<size_t>(80 * 1024, lds_limit()); }

}  // namespace

// Pass structure of the tiled grids from their current depths: passes per grid, the queue order
// (by pass count, descending, so that the grids still active at pass p are a prefix), the tile
// prefix sums over that order and the LDS of the deepest pass.
static void build_passes(st_batch* B) {
    std::vector<int> order = B->tiled;
    size_t lds = 0;
    for (int g : order) {
        BatchDesc& d = B->desc[g];
        d.passes = (d.steps + d.tb - 1) / d.tb;
        lds = std::max(lds, tiled_lds_bytes(d.r, d.tb, kTX, kTY));
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return B->desc[a].passes > B->desc[b].passes; });
    B->order = order;
    B->tile_prefix.assign(1, 0);
    for (int g : order) B->tile_prefix.push_back(B->tile_prefix.back() + B->desc[g].tiles_x * B->desc[g].tiles_y);
    B->max_passes = order.empty() ? 0 : B->desc[order[0]].passes;
    B->active.clear();
    for (int p = 0; p < B->max_passes; ++p) {
        int a = 0;
        while (a < int(order.size()) && B->desc[order[a]].passes > p) ++a;
        B->active.push_back(a);
    }
    B->lds_pass = lds;
}

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
    B->tb_max.assign(n, 0);
    std::vector<int> tiled;
    size_t lds_res = 0;
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
            B->zero_steps.push_back(g);
            continue;
        }
        const size_t rl = resident_lds_bytes(p->radius, p->rows, p->cols);
        if (rl <= batch_lds_budget()) {
            d.resident = 1;
            d.passes = 1;
            d.tb = d.steps;
            lds_res = std::max(lds_res, rl);
            B->res.push_back(g);
            continue;
        }
        // deepest pass the batch tile allows; the plan's depth, capped by it, is the starting point
        int tbm = 16;
        while (tbm > 1 && tiled_lds_bytes(p->radius, tbm, kTX, kTY) > batch_lds_budget()) --tbm;
        B->tb_max[g] = tbm;
        d.tb = std::min(std::max(1, p->tb), tbm);
        d.tiles_x = (p->cols + kTX - 1) / kTX;
        d.tiles_y = (p->rows + kTY - 1) / kTY;
        tiled.push_back(g);
    }
    B->tiled = tiled;
    build_passes(B);
    // workspace: descriptor table, queue tables, one ping-pong field per tiled grid with two or more
    // steps (any depth the autotuner may pick below the step count needs it)
    size_t off = 0;
    B->off_desc = off;
    off = align256(off + size_t(n) * sizeof(BatchDesc));
    B->off_tprefix = off;
    off = align256(off + B->tile_prefix.size() * sizeof(int64_t));
    B->off_order = off;
    off = align256(off + std::max<size_t>(B->order.size(), 1) * sizeof(int));
    B->off_res = off;
    off = align256(off + std::max<size_t>(B->res.size(), 1) * sizeof(int));
    B->off_fields = off;
    for (int g : tiled) {
        if (B->desc[g].steps >= 2) {
            B->field_off[g] = off;
            off = align256(off + size_t(B->desc[g].rows * B->desc[g].cols) * sizeof(float));
        }
    }
    B->ws_bytes = std::max<size_t>(off, 256);
    B->lds_res = lds_res;
    B->pinned = nullptr;
    B->pinned_bytes = B->off_fields - B->off_desc;
    B->staged = nullptr;
    B->staged_valid = false;
    B->last_ws = nullptr;
    B->exec = nullptr;
    B->g_ws = nullptr;
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

// Enqueue the batch's kernels: the resident grids on `side` (joined back into `s` at the end when
// side != s), the pass levels of the tiled grids on `s`.
static int enqueue_batch(st_batch* B, char* ws, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
    const BatchDesc* desc = reinterpret_cast<const BatchDesc*>(ws + B->off_desc);
    const bool branch = side != s;
    if (!B->res.empty()) {
        if (int rc = prepare_lds(reinterpret_cast<const void*>(batched_resident), B->lds_res)) return rc;
        if (branch) {
            ST_HIP_CHECK(hipEventRecord(fork, s));
            ST_HIP_CHECK(hipStreamWaitEvent(side, fork, 0));
        }
        clear_stale_error();
        hipLaunchKernelGGL(batched_resident, dim3(unsigned(B->res.size())), dim3(NT), B->lds_res, side, desc,
                           reinterpret_cast<const int*>(ws + B->off_res));
        ST_LAUNCH_CHECK("batched_resident");
    }
    if (B->max_passes > 0) {
        if (int rc = prepare_lds(reinterpret_cast<const void*>(batched_pass), B->lds_pass)) return rc;
        for (int p = 0; p < B->max_passes; ++p) {
            PassArgs a;
            a.desc = desc;
            a.order = reinterpret_cast<const int*>(ws + B->off_order);
            a.tile_prefix = reinterpret_cast<const int64_t*>(ws + B->off_tprefix);
            a.n_active = B->active[p];
            a.p = p;
            const int64_t blocks = B->tile_prefix[B->active[p]];
            clear_stale_error();
            hipLaunchKernelGGL(batched_pass, dim3(unsigned(blocks)), dim3(NT), B->lds_pass, s, a);
            ST_LAUNCH_CHECK("batched_pass");
        }
    }
    if (branch && !B->res.empty()) {
        ST_HIP_CHECK(hipEventRecord(join, side));
        ST_HIP_CHECK(hipStreamWaitEvent(s, join, 0));
    }
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
        std::memcpy(h + (B->off_tprefix - B->off_desc), B->tile_prefix.data(), B->tile_prefix.size() * sizeof(int64_t));
        if (!B->order.empty())
            std::memcpy(h + (B->off_order - B->off_desc), B->order.data(), B->order.size() * sizeof(int));
        if (!B->res.empty()) std::memcpy(h + (B->off_res - B->off_desc), B->res.data(), B->res.size() * sizeof(int));
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
    if (B->res.empty() && B->max_passes == 0) return ST_OK;
    if (!(B->flags & ST_FLAG_GRAPH)) return enqueue_batch(B, ws, s, s, nullptr, nullptr);
    if (!(B->exec && B->g_ws == workspace)) {
        if (B->exec) {
            (void)hipGraphExecDestroy(B->exec);
            B->exec = nullptr;
        }
        // capture: the resident grids on a side branch forked from and joined back into the main one
        hipStream_t cap = nullptr, side = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
        int rc = ST_OK;
        hipGraph_t graph = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
            rc = fail(ST_EHIP, "stream/event creation for graph capture failed");
        } else if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(ST_EHIP, "hipStreamBeginCapture failed");
        } else {
            rc = enqueue_batch(B, ws, cap, side, fork, join);
            const hipError_t e = hipStreamEndCapture(cap, &graph);
            if (!rc && e != hipSuccess) rc = fail(ST_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        }
        if (!rc) {
            const hipError_t e2 = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
            if (e2 != hipSuccess) rc = fail(ST_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (side) (void)hipStreamDestroy(side);
        if (cap) (void)hipStreamDestroy(cap);
        (void)hipGetLastError();
        if (rc) return rc;
        B->g_ws = workspace;
    }
    ST_HIP_CHECK(hipGraphLaunch(B->exec, s));
    return ST_OK;
}

// Coordinate descent over the stencil classes (shape, radius) of the tiled grids: for each class
// in turn, time the whole batch (direct launches) with the class's depth capped at each candidate,
// keep the fastest, then move to the next class.
extern "C" int stencil_batch_autotune(st_batch* B, const void* const* ins, void* const* outs, void* workspace,
                                      size_t ws_bytes, int* tb_out, void* stream) {
    if (!B || !ins || !outs) return fail(ST_EINVAL, "NULL argument");
    if (!workspace || ws_bytes < B->ws_bytes) return fail(ST_ENOWS, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (tb_out) std::fill(tb_out, tb_out + 6, 0);
    const uint32_t flags = B->flags;
    B->flags &= ~ST_FLAG_GRAPH;
    std::vector<int> classes;  // shape * 8 + r
    for (int g : B->tiled) {
        const int c = B->desc[g].shape * 8 + B->desc[g].r;
        if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ST_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(ST_EHIP, "hipEventCreate");
    static const int kCaps[] = {1, 2, 3, 4, 6, 8, 12, 16};
    auto apply = [&](int cls, int cap) {
        for (int g : B->tiled)
            if (B->desc[g].shape * 8 + B->desc[g].r == cls) B->desc[g].tb = std::min(cap, B->tb_max[g]);
        build_passes(B);
        B->staged_valid = false;  // descriptor tables changed
    };
    auto timed = [&](float* ms) -> int {
        for (int rep = 0; rep < 2; ++rep) {  // the first run warms up and stages the tables
            if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) return fail(ST_EHIP, "hipEventRecord");
            if (int r = stencil_run_batched(B, ins, outs, workspace, ws_bytes, stream)) return r;
        }
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return fail(ST_EHIP, "hipEventRecord/Synchronize");
        return hipEventElapsedTime(ms, e0, e1) == hipSuccess ? ST_OK : fail(ST_EHIP, "hipEventElapsedTime");
    };
    for (int cls : classes) {
        if (rc) break;
        int deepest = 1;
        for (int g : B->tiled)
            if (B->desc[g].shape * 8 + B->desc[g].r == cls) deepest = std::max(deepest, B->tb_max[g]);
        int best_cap = 0;
        float best = 1e30f;
        for (int cap : kCaps) {
            if (cap > deepest) break;
            apply(cls, cap);
            float ms = 0.0f;
            if ((rc = timed(&ms))) break;
            if (ms < best) {
                best = ms;
                best_cap = cap;
            }
        }
        if (!rc && best_cap) apply(cls, best_cap);
        if (tb_out && !rc) {
            // report the cap chosen for each class in class order: star r=1..3 then box r=1..3
            const int slot = (cls / 8) * 3 + (cls % 8) - 1;
            if (slot >= 0 && slot < 6) tb_out[slot] = best_cap;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    B->flags = flags;
    if (B->exec) {  // the captured graph holds the old pass structure
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    return rc;
}
