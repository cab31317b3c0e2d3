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
#include "march_body.h"
#include "sweep_body.h"

namespace st {

namespace {

struct BatchDesc {
    const float* in;
    float* out;
    float* ws;
    int64_t rows, cols;
    int64_t tiles_x, tiles_y;  // tiled engine: tiles; marching engine: bands and segments
    int64_t seg;               // marching engine: output rows per task
    int r, shape, tb, steps, passes, resident;
    int vec;  // marching engine: rows 16-byte aligned in every buffer (cols % 4 == 0): vector accesses
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

// Marching engine: one launch runs `levels` (the template TB) levels of pass p for the grids
// order[s0 .. s0+n) of one stencil class; wavefront task -> (grid, band, segment) through the class's
// task prefix sums.  Four columns per lane: one vector access per lane and row for grids whose rows
// are 16-byte aligned in every buffer, four element accesses otherwise (any width and alignment).
struct MarchPassArgs {
    const BatchDesc* desc;
    const int* order;            // the class's grids, ordered by passes then last-pass depth, descending
    const int64_t* task_prefix;  // prefix sums of tasks over `order`
    int s0, n;                   // the slice of `order` this launch covers
    int p;                       // pass index
};

constexpr int MW = 4;  // wavefronts per workgroup of the marching engine
constexpr int MV = 4;  // columns per lane of the marching engine (vector or element accesses per grid)

// LDS of a batched marching workgroup: the input rows that the two wavefronts of a pair share (2 r tb
// rows of 64 lanes x 16 bytes per pair).
constexpr size_t march_share_bytes(int r, int tb) { return size_t(MW / 2) * 2 * r * tb * 64 * sizeof(float4); }

template <int R, int SH, int TB>
__global__ __launch_bounds__(64 * MW) void batched_march(MarchPassArgs a) {
    extern __shared__ float4 shared_rows[];
    const int lane = int(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t* pre = a.task_prefix + a.s0;
    const int64_t task_in = pre[0] + int64_t(blockIdx.x) * MW + wave;
    const bool active = task_in < pre[a.n];
    // a wavefront past the launch's last task computes as that task (its setup is then a plain load
    // chain from the descriptor table, like the others') but stages nothing and stops at the barrier
    const int64_t task = active ? task_in : pre[a.n] - 1;
    // a grid's tasks go down each band in turn, so a workgroup's wavefronts take neighbouring
    // segments.  Wavefronts 0 and 2 march upwards and 1 and 3 downwards, so the pairs 0-1 and 2-3
    // meet at their start: each stages its own half of the 2 r tb input rows around the boundary in
    // LDS, and both read the whole overlap from there instead of reading it from HBM twice.
    const bool up = !(wave & 1);
    constexpr int H = march::halo_lanes(R, TB, MV);
    constexpr int64_t RT = int64_t(R) * TB;
    const int k = upper_index(pre, a.n + 1, task);
    const BatchDesc& d = a.desc[a.order[a.s0 + k]];
    const int64_t t = task - pre[k];
    const int64_t segi = t % d.tiles_y, band = t / d.tiles_y;
    const int64_t y0 = segi * d.seg;
    const int64_t y1 = y0 + d.seg < d.rows ? y0 + d.seg : d.rows;
    // the partner: the next task for an upward wavefront, the previous one for a downward one
    const int64_t pt = up ? task + 1 : task - 1;
    bool paired = false;
    if (active && pt >= pre[k] && pt < pre[k + 1] && pt < pre[a.n]) {
        const int64_t tp = pt - pre[k];
        paired = tp / d.tiles_y == band && (up ? tp % d.tiles_y == segi + 1 : tp % d.tiles_y + 1 == segi);
    }
    const int64_t yb = up ? y1 : y0;  // the pair's boundary
    const int P = d.passes, p = a.p;
    const float* src = p == 0 ? d.in : (((P - p) % 2 == 0) ? d.out : d.ws);  // written by pass p-1
    float* dst = ((P - 1 - p) % 2 == 0) ? d.out : d.ws;
    const march::MarchView v{src, dst, d.rows, d.cols, d.b, march::BC_CONST, nullptr};
    const int64_t X0 = band * (MV * (64 - 2 * H)) - MV * H;
    float4* mine = shared_rows + (wave >> 1) * (2 * RT * 64);
    if (paired) {  // each stages the rows on its own side of the boundary
        if (d.vec) march::stage_rows<ST_F32, R, MV, TB, true>(v, lane, y0, y1, X0, up ? yb - RT : yb, yb - RT, mine);
        else march::stage_rows<ST_F32, R, MV, TB, false>(v, lane, y0, y1, X0, up ? yb - RT : yb, yb - RT, mine);
    }
    __syncthreads();  // every wavefront of the workgroup reaches it once
    if (!active) return;
    const march::SharedRows sh{paired ? mine : nullptr, yb - RT, yb + RT};
    // input rows in flight: one ring length, except box r >= 3 with several levels (registers)
    constexpr int D = SH == SHAPE_STAR || R <= 2 || TB == 1 ? 2 * R + 1 : 0;
    if (d.vec) march::march_task_dir<ST_F32, R, MV, SH, TB, D, true>(v, d.w, lane, y0, y1, X0, up, sh);
    else march::march_task_dir<ST_F32, R, MV, SH, TB, D, false>(v, d.w, lane, y0, y1, X0, up, sh);
}

using MarchPassFn = void (*)(MarchPassArgs);

template <int SH>
MarchPassFn batched_march_fn(int r, int levels) {
#define ST_BMARCH(R, TB) \
    if (r == R && levels == TB) return batched_march<R, SH, TB>;
    if constexpr (SH == SHAPE_STAR) {
        ST_BMARCH(1, 1) ST_BMARCH(1, 2) ST_BMARCH(1, 3) ST_BMARCH(1, 4) ST_BMARCH(1, 5) ST_BMARCH(1, 6)
        ST_BMARCH(1, 7) ST_BMARCH(1, 8)
        ST_BMARCH(2, 1) ST_BMARCH(2, 2) ST_BMARCH(2, 3) ST_BMARCH(2, 4) ST_BMARCH(2, 5) ST_BMARCH(2, 6)
        ST_BMARCH(3, 1) ST_BMARCH(3, 2) ST_BMARCH(3, 3) ST_BMARCH(3, 4)
    } else {
        ST_BMARCH(1, 1) ST_BMARCH(1, 2) ST_BMARCH(1, 3) ST_BMARCH(1, 4) ST_BMARCH(1, 5) ST_BMARCH(1, 6)
        ST_BMARCH(2, 1) ST_BMARCH(2, 2) ST_BMARCH(2, 3)
        ST_BMARCH(3, 1) ST_BMARCH(3, 2)
    }
#undef ST_BMARCH
    return nullptr;
}

MarchPassFn batched_march_lookup(int shape, int r, int levels) {
    return shape == SHAPE_BOX ? batched_march_fn<SHAPE_BOX>(r, levels) : batched_march_fn<SHAPE_STAR>(r, levels);
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
    std::vector<int> tiled;            // grids that are neither resident nor zero-step, in input order
    std::vector<int> tb_max;           // per grid: deepest pass the batch tile's LDS budget allows
    int max_passes;
    // per stencil class (slot = shape * 3 + r - 1): engine (0 = LDS tiles, 1 = marching) and depth
    int engine[6], depth[6];
    int64_t seg_min[6];  // marching: least output rows per task (0: the tasks about fill the device once)
    struct MLaunch {
        int s0, n, p, levels;
        int64_t tasks;
    };
    struct MClass {
        int64_t seg = 0;               // output rows per task (the longest a grid's segment may be)
        std::vector<int> order;        // the class's marching grids by passes, then last-pass depth
        std::vector<int64_t> prefix;   // task prefix sums over `order`
        std::vector<MLaunch> launches; // in pass order
    } mclass[6];
    size_t off_desc, off_tprefix, off_order, off_res, off_morder[6], off_mprefix[6], off_fields, ws_bytes;
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

static int class_slot(const BatchDesc& d) { return d.shape * 3 + d.r - 1; }

// Marching engine: output rows per task for a class, so that its tasks about fill the device once
// (`waves`: the wavefronts of the class's kernel the device holds at once).
static int64_t march_segment(int64_t band_rows, int64_t waves) {
    const int64_t seg = (band_rows + waves - 1) / waves;
    return std::min<int64_t>(2048, std::max<int64_t>(8, seg));
}

// Wavefronts of the marching kernel for (shape, radius, depth) resident at once (4096 if unknown).
static int64_t march_waves(int shape, int r, int tb) {
    MarchPassFn fn = batched_march_lookup(shape, r, tb);
    int blocks = 0;
    if (!fn || resident_blocks(reinterpret_cast<const void*>(fn), march_share_bytes(r, tb), &blocks) != ST_OK ||
        blocks < 1) {
        (void)hipGetLastError();
        return 4096;
    }
    return int64_t(blocks) * MW;
}

// Pass structure from each class's engine and depth.  Tiled engine: passes per grid, the queue
// order (by pass count, descending, so that the grids still active at pass p are a prefix), the tile
// prefix sums over that order and the LDS of the deepest pass.  Marching engine, per class: bands
// and segments per grid, the order by (passes, depth of the last pass) descending, the task prefix
// sums, and the launches -- at pass p the full-depth grids are a prefix of the order and the grids
// finishing with a shallower pass follow in groups of equal depth.
static void build_passes(st_batch* B) {
    std::vector<int> order;
    size_t lds = 0;
    for (int c = 0; c < 6; ++c) B->mclass[c] = st_batch::MClass();
    for (int g : B->tiled) {
        BatchDesc& d = B->desc[g];
        const int c = class_slot(d);
        if (B->engine[c] == 0) {
            d.tb = std::min(B->depth[c] > 0 ? B->depth[c] : d.tb, B->tb_max[g]);
            d.tiles_x = (d.cols + kTX - 1) / kTX;
            d.tiles_y = (d.rows + kTY - 1) / kTY;
            d.passes = (d.steps + d.tb - 1) / d.tb;
            lds = std::max(lds, tiled_lds_bytes(d.r, d.tb, kTX, kTY));
            order.push_back(g);
        } else {
            d.tb = B->depth[c];
            d.passes = (d.steps + d.tb - 1) / d.tb;
            const int64_t band_w = MV * (64 - 2 * march::halo_lanes(d.r, d.tb, MV));
            d.tiles_x = (d.cols + band_w - 1) / band_w;  // bands
            B->mclass[c].order.push_back(g);
        }
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
    for (int c = 0; c < 6; ++c) {
        st_batch::MClass& M = B->mclass[c];
        if (M.order.empty()) continue;
        const int tb = B->depth[c];
        auto last_depth = [&](int g) { return B->desc[g].steps - (B->desc[g].passes - 1) * tb; };
        std::stable_sort(M.order.begin(), M.order.end(), [&](int a, int b) {
            const BatchDesc &da = B->desc[a], &db = B->desc[b];
            return da.passes != db.passes ? da.passes > db.passes : last_depth(a) > last_depth(b);
        });
        int64_t band_rows = 0;
        for (int g : M.order) band_rows += B->desc[g].tiles_x * B->desc[g].rows;
        const int64_t seg =
            std::max(march_segment(band_rows, march_waves(c / 3, c % 3 + 1, tb)), B->seg_min[c]);
        M.seg = seg;
        M.prefix.assign(1, 0);
        for (int g : M.order) {
            BatchDesc& d = B->desc[g];
            d.seg = std::min<int64_t>(seg, d.rows);
            d.tiles_y = (d.rows + d.seg - 1) / d.seg;  // segments
            M.prefix.push_back(M.prefix.back() + d.tiles_x * d.tiles_y);
        }
        const int P = B->desc[M.order[0]].passes;
        const int n = int(M.order.size());
        for (int p = 0; p < P; ++p) {
            // grids at pass p: passes > p (a prefix); those with passes == p + 1 run their last depth
            int a = 0;
            while (a < n && B->desc[M.order[a]].passes > p) ++a;
            int full = 0;
            while (full < a && (B->desc[M.order[full]].passes > p + 1 || last_depth(M.order[full]) == tb)) ++full;
            auto push = [&](int s0, int e, int levels) {
                if (e > s0) M.launches.push_back({s0, e - s0, p, levels, M.prefix[e] - M.prefix[s0]});
            };
            push(0, full, tb);
            for (int s0 = full; s0 < a;) {
                const int lv = last_depth(M.order[s0]);
                int e = s0;
                while (e < a && last_depth(M.order[e]) == lv) ++e;
                push(s0, e, lv);
                s0 = e;
            }
        }
    }
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
        if (!p || steps[g] < 0 || steps[g] > (int64_t(1) << 30)) {
            delete B;
            return fail(ST_EINVAL, "NULL plan, or steps outside [0, 2^30]");
        }
        if (p->kind != KIND_CONST || p->storage != ST_F32 || p->radius > 3 || p->bc != ST_BC_CONST) {
            delete B;
            return fail(ST_EUNSUPPORTED, "batched grids must be FP32 constant-weight plans with a constant halo, r <= 3");
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
    for (int c = 0; c < 6; ++c) {
        B->engine[c] = 0;
        B->depth[c] = 0;  // 0: each grid keeps its plan's depth (capped by the tile's LDS)
        B->seg_min[c] = 0;
    }
    build_passes(B);
    // workspace: descriptor table, queue tables, one ping-pong field per tiled grid with two or more
    // steps (any depth the autotuner may pick below the step count needs it)
    size_t off = 0;
    B->off_desc = off;
    off = align256(off + size_t(n) * sizeof(BatchDesc));
    B->off_tprefix = off;
    off = align256(off + (tiled.size() + 1) * sizeof(int64_t));
    B->off_order = off;
    off = align256(off + std::max<size_t>(tiled.size(), 1) * sizeof(int));
    B->off_res = off;
    off = align256(off + std::max<size_t>(B->res.size(), 1) * sizeof(int));
    for (int c = 0; c < 6; ++c) {  // room for every tiled grid in any class's marching tables
        B->off_morder[c] = off;
        off = align256(off + std::max<size_t>(tiled.size(), 1) * sizeof(int));
        B->off_mprefix[c] = off;
        off = align256(off + (tiled.size() + 1) * sizeof(int64_t));
    }
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

// The marching launches of class c, in pass order, on stream `s`.
static int enqueue_march_class(st_batch* B, int c, char* ws, hipStream_t s) {
    const st_batch::MClass& M = B->mclass[c];
    const BatchDesc& d0 = B->desc[M.order[0]];
    for (const st_batch::MLaunch& L : M.launches) {
        MarchPassFn fn = batched_march_lookup(d0.shape, d0.r, L.levels);
        if (!fn) return fail(ST_EUNSUPPORTED, "no batched marching kernel for this class/depth");
        MarchPassArgs a;
        a.desc = reinterpret_cast<const BatchDesc*>(ws + B->off_desc);
        a.order = reinterpret_cast<const int*>(ws + B->off_morder[c]);
        a.task_prefix = reinterpret_cast<const int64_t*>(ws + B->off_mprefix[c]);
        a.s0 = L.s0;
        a.n = L.n;
        a.p = L.p;
        const int64_t blocks = (L.tasks + MW - 1) / MW;
        clear_stale_error();
        hipLaunchKernelGGL(fn, dim3(unsigned(blocks)), dim3(64 * MW), march_share_bytes(d0.r, L.levels), s, a);
        ST_LAUNCH_CHECK("batched_march");
    }
    return ST_OK;
}

// Enqueue the batch's kernels: the resident grids on `side`, the marching classes on `mside[c]`
// (each joined back into `s` at the end when it differs from s), the pass levels of the tiled grids
// on `s`.
static int enqueue_batch(st_batch* B, char* ws, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join,
                         const hipStream_t* mside, const hipEvent_t* mjoin) {
    const BatchDesc* desc = reinterpret_cast<const BatchDesc*>(ws + B->off_desc);
    const bool branch = side != s;
    if (branch) {
        ST_HIP_CHECK(hipEventRecord(fork, s));
        for (int c = 0; c < 6; ++c)
            if (!B->mclass[c].order.empty()) ST_HIP_CHECK(hipStreamWaitEvent(mside[c], fork, 0));
    }
    for (int c = 0; c < 6; ++c) {
        if (B->mclass[c].order.empty()) continue;
        if (int rc = enqueue_march_class(B, c, ws, branch ? mside[c] : s)) return rc;
        if (branch) {
            ST_HIP_CHECK(hipEventRecord(mjoin[c], mside[c]));
        }
    }
    if (!B->res.empty()) {
        if (int rc = prepare_lds(reinterpret_cast<const void*>(batched_resident), B->lds_res)) return rc;
        if (branch) {
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
    if (branch)
        for (int c = 0; c < 6; ++c)
            if (!B->mclass[c].order.empty()) ST_HIP_CHECK(hipStreamWaitEvent(s, mjoin[c], 0));
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
            auto a16 = [](const void* q) { return reinterpret_cast<uintptr_t>(q) % 16 == 0; };
            d.vec = d.cols % MV == 0 && a16(d.in) && a16(d.out) && (!d.ws || a16(d.ws));
            std::memcpy(h + g * sizeof(BatchDesc), &d, sizeof(d));
        }
        std::memcpy(h + (B->off_tprefix - B->off_desc), B->tile_prefix.data(), B->tile_prefix.size() * sizeof(int64_t));
        if (!B->order.empty())
            std::memcpy(h + (B->off_order - B->off_desc), B->order.data(), B->order.size() * sizeof(int));
        if (!B->res.empty()) std::memcpy(h + (B->off_res - B->off_desc), B->res.data(), B->res.size() * sizeof(int));
        for (int c = 0; c < 6; ++c) {
            const st_batch::MClass& M = B->mclass[c];
            if (M.order.empty()) continue;
            std::memcpy(h + (B->off_morder[c] - B->off_desc), M.order.data(), M.order.size() * sizeof(int));
            std::memcpy(h + (B->off_mprefix[c] - B->off_desc), M.prefix.data(), M.prefix.size() * sizeof(int64_t));
        }
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
    bool any_march = false;
    for (int c = 0; c < 6; ++c) any_march = any_march || !B->mclass[c].order.empty();
    if (B->res.empty() && B->max_passes == 0 && !any_march) return ST_OK;
    if (!(B->flags & ST_FLAG_GRAPH)) return enqueue_batch(B, ws, s, s, nullptr, nullptr, nullptr, nullptr);
    if (!(B->exec && B->g_ws == workspace)) {
        if (B->exec) {
            (void)hipGraphExecDestroy(B->exec);
            B->exec = nullptr;
        }
        // capture: the resident grids on a side branch forked from and joined back into the main one
        hipStream_t cap = nullptr, side = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
        hipStream_t mside[6] = {};
        hipEvent_t mjoin[6] = {};
        int rc = ST_OK;
        hipGraph_t graph = nullptr;
        bool made = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess &&
                    hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess &&
                    hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess &&
                    hipEventCreateWithFlags(&join, hipEventDisableTiming) == hipSuccess;
        for (int c = 0; c < 6 && made; ++c)
            made = hipStreamCreateWithFlags(&mside[c], hipStreamNonBlocking) == hipSuccess &&
                   hipEventCreateWithFlags(&mjoin[c], hipEventDisableTiming) == hipSuccess;
        if (!made) {
            rc = fail(ST_EHIP, "stream/event creation for graph capture failed");
        } else if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(ST_EHIP, "hipStreamBeginCapture failed");
        } else {
            rc = enqueue_batch(B, ws, cap, side, fork, join, mside, mjoin);
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
        for (int c = 0; c < 6; ++c) {
            if (mjoin[c]) (void)hipEventDestroy(mjoin[c]);
            if (mside[c]) (void)hipStreamDestroy(mside[c]);
        }
        if (cap) (void)hipStreamDestroy(cap);
        (void)hipGetLastError();
        if (rc) return rc;
        B->g_ws = workspace;
    }
    ST_HIP_CHECK(hipGraphLaunch(B->exec, s));
    return ST_OK;
}

extern "C" int stencil_batch_set_class(st_batch* B, int shape, int radius, int engine, int depth) {
    if (!B) return fail(ST_EINVAL, "batch is NULL");
    if ((shape != SHAPE_STAR && shape != SHAPE_BOX) || radius < 1 || radius > 3 || (engine != 0 && engine != 1))
        return fail(ST_EINVAL, "bad class or engine");
    if (depth < 1 || depth > 16 || (engine == 1 && depth > march_max_tb(shape, radius, 1)))
        return fail(ST_EUNSUPPORTED, "depth out of range for this engine");
    const int c = shape * 3 + radius - 1;
    B->engine[c] = engine;
    B->depth[c] = depth;
    build_passes(B);
    B->staged_valid = false;
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    return ST_OK;
}

extern "C" int stencil_batch_set_segment(st_batch* B, int shape, int radius, int64_t min_rows) {
    if (!B) return fail(ST_EINVAL, "batch is NULL");
    if ((shape != SHAPE_STAR && shape != SHAPE_BOX) || radius < 1 || radius > 3 || min_rows < 0)
        return fail(ST_EINVAL, "bad class or segment length");
    const int c = shape * 3 + radius - 1;
    B->seg_min[c] = min_rows;
    build_passes(B);
    B->staged_valid = false;
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    return ST_OK;
}

extern "C" int stencil_batch_get_segment(const st_batch* B, int shape, int radius, int64_t* rows) {
    if (!B || !rows) return fail(ST_EINVAL, "NULL argument");
    if ((shape != SHAPE_STAR && shape != SHAPE_BOX) || radius < 1 || radius > 3)
        return fail(ST_EINVAL, "bad class");
    const int c = shape * 3 + radius - 1;
    *rows = B->engine[c] == 1 && !B->mclass[c].order.empty() ? B->mclass[c].seg : 0;
    return ST_OK;
}

// Coordinate descent over the stencil classes (shape, radius) of the non-resident grids: for each
// class in turn, time the whole batch (direct launches) with every candidate engine and depth -- LDS
// tiles with the class's depth capped at 1, 2, 3, 4, 6, 8, 12 or 16, or marching with 1 .. the
// deepest its radius allows, each marching depth with the default segments and with segments 2, 4
// and 8 times as long -- keep the fastest, then move to the next class.
extern "C" int stencil_batch_autotune(st_batch* B, const void* const* ins, void* const* outs, void* workspace,
                                      size_t ws_bytes, int* tb_out, int* engine_out, void* stream) {
    if (!B || !ins || !outs) return fail(ST_EINVAL, "NULL argument");
    if (!workspace || ws_bytes < B->ws_bytes) return fail(ST_ENOWS, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (tb_out) std::fill(tb_out, tb_out + 6, 0);
    if (engine_out) std::fill(engine_out, engine_out + 6, 0);
    const uint32_t flags = B->flags;
    B->flags &= ~ST_FLAG_GRAPH;
    bool present[6] = {};
    int deepest[6] = {};
    for (int g : B->tiled) {
        const int c = class_slot(B->desc[g]);
        present[c] = true;
        deepest[c] = std::max(deepest[c], B->tb_max[g]);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ST_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(ST_EHIP, "hipEventCreate");
    auto apply = [&](int c, int engine, int depth, int seg_mult) {
        B->engine[c] = engine;
        B->depth[c] = depth;
        B->seg_min[c] = 0;
        build_passes(B);
        if (engine == 1 && seg_mult > 1) {  // longer than the default segment of this depth
            B->seg_min[c] = seg_mult * B->mclass[c].seg;
            build_passes(B);
        }
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
    static const int kCaps[] = {1, 2, 3, 4, 6, 8, 12, 16};
    for (int c = 0; c < 6 && rc == ST_OK; ++c) {
        if (!present[c]) continue;
        const int r = c % 3 + 1;
        struct Cand {
            int engine, depth, seg_mult;
        };
        std::vector<Cand> cands;
        for (int cap : kCaps)
            if (cap <= deepest[c]) cands.push_back({0, cap, 1});
        for (int t = 1; t <= march_max_tb(c / 3, r, 1); ++t)
            for (int m : {1, 2, 4, 8}) cands.push_back({1, t, m});
        Cand best = cands[0];
        float best_ms = 1e30f;
        for (const Cand& cd : cands) {
            apply(c, cd.engine, cd.depth, cd.seg_mult);
            float ms = 0.0f;
            if ((rc = timed(&ms))) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = cd;
            }
        }
        if (rc) break;
        apply(c, best.engine, best.depth, best.seg_mult);
        if (tb_out) tb_out[c] = best.depth;
        if (engine_out) engine_out[c] = best.engine;
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
