// Host side of the C ABI: plans, validation, pass scheduling, graphs, autotuning, errors.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "internal.h"

namespace st {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

size_t elem_size(int storage) { return storage == ST_F32 ? 4 : 2; }

size_t lds_limit() {
    static std::mutex mu;
    static size_t cached = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (!cached) {
        int dev = 0, optin = 0, plain = 0, count = 0;
        if (hipGetDeviceCount(&count) == hipSuccess && count > 0 && hipGetDevice(&dev) == hipSuccess) {
            if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
            if (hipDeviceGetAttribute(&plain, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) plain = 0;
        }
        (void)hipGetLastError();
        cached = size_t(std::max({optin, plain, 65536}));
    }
    return cached;
}

int resident_blocks(const void* fn, size_t lds, int* blocks) {
    static std::mutex mu;
    static std::map<std::pair<const void*, size_t>, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({fn, lds});
    if (it == cache.end()) {
        int dev = 0, cus = 0, occ = 0;
        ST_HIP_CHECK(hipGetDevice(&dev));
        ST_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        ST_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 256, lds));
        it = cache.emplace(std::make_pair(fn, lds), std::max(1, cus * std::max(occ, 1))).first;
    }
    *blocks = it->second;
    return ST_OK;
}

int prepare_lds(const void* fn, size_t bytes) {
    if (bytes > lds_limit()) return fail(ST_EUNSUPPORTED, "kernel needs more LDS than a workgroup may have");
    if (bytes > 65536) ST_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
    return ST_OK;
}

// Round b to the storage type on the host (nearest even), widened back to float.  The host
// copy of the conversion is only used for this one plan constant.
static float round_to_storage(double b, int storage) {
    float f = float(b);
    if (storage == ST_F32) return f;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if (storage == ST_BF16) {
        uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
        float o;
        std::memcpy(&o, &r, 4);
        return o;
    }
    _Float16 h = (_Float16)f;  // host compiler's IEEE conversion, round to nearest even
    return (float)h;
}

static int classify_shape(int r, const float* w) {
    const int k = 2 * r + 1;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
            if (dy != 0 && dx != 0 && w[(dy + r) * k + dx + r] != 0.0f) return SHAPE_BOX;
    return SHAPE_STAR;
}

// default blocking: deeper temporal blocks for cheap stencils, where HBM dominates
static void default_blocking(st_plan* p) {
    p->tile_x = 128;
    p->tile_y = 64;
    const int taps = p->shape == SHAPE_BOX ? (2 * p->radius + 1) * (2 * p->radius + 1) : 4 * p->radius + 1;
    int tb = taps >= 40 ? 2 : (taps >= 13 ? 4 : 6);
    tb = std::min(tb, max_tb(p, p->tile_x, p->tile_y));
    p->tb = std::max(tb, 1);
}

static void init_plan(st_plan* p) {
    std::memset(p, 0, sizeof(*p));
    p->planes = 1;
    p->spin_limit = int64_t(1) << 22;
}

static int check_flags(uint32_t flags) {
    if (flags & ~(ST_FLAG_NAIVE | ST_FLAG_GRAPH | ST_FLAG_ALLOW_MFMA)) return fail(ST_EINVAL, "unknown flag bits");
    return ST_OK;
}

// --------------------------------------------------------------------------
// graphs
// --------------------------------------------------------------------------
static void drop_graph(st_plan* p) {
    if (p->graph_exec) {
        (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(p->graph_exec));
        p->graph_exec = nullptr;
    }
}

}  // namespace st

using namespace st;

extern "C" {

const char* stencil_strerror(int code) {
    switch (code) {
        case ST_OK: return "success";
        case ST_EINVAL: return "invalid argument";
        case ST_EALIAS: return "input and output overlap";
        case ST_EUNSUPPORTED: return "unsupported configuration";
        case ST_EHIP: return "HIP runtime error";
        case ST_ENOWS: return "workspace missing or too small";
        case ST_ENOMEM: return "host allocation failed";
        case ST_ESTATE: return "invalid object state";
    }
    return "unknown status code";
}

const char* stencil_last_error(void) { return g_last_error.c_str(); }

int stencil_plan(st_plan** out, int64_t rows, int64_t cols, int radius, const float* weights, double boundary,
                 int storage, uint32_t flags) {
    if (!out) return fail(ST_EINVAL, "out is NULL");
    *out = nullptr;
    if (rows < 1 || cols < 1) return fail(ST_EINVAL, "rows and cols must be >= 1");
    if (rows > (int64_t(1) << 31) || cols > (int64_t(1) << 31)) return fail(ST_EINVAL, "grid side too large");
    if (rows * cols > (int64_t(1) << 46)) return fail(ST_EINVAL, "grid has more cells than device memory can hold");
    if (radius < 1 || radius > ST_MAX_RADIUS) return fail(ST_EINVAL, "radius must be in [1, 4]");
    if (!weights) return fail(ST_EINVAL, "weights is NULL");
    if (storage != ST_F32 && storage != ST_BF16 && storage != ST_F16) return fail(ST_EINVAL, "unknown storage type");
    if (!std::isfinite(boundary)) return fail(ST_EINVAL, "boundary value must be finite");
    if (int rc = check_flags(flags)) return rc;
    const int k = 2 * radius + 1;
    for (int i = 0; i < k * k; ++i)
        if (!std::isfinite(weights[i])) return fail(ST_EINVAL, "weights must be finite");
    st_plan* p = new (std::nothrow) st_plan;
    if (!p) return fail(ST_ENOMEM, "plan allocation failed");
    init_plan(p);
    p->kind = KIND_CONST;
    p->rows = rows;
    p->cols = cols;
    p->radius = radius;
    p->storage = storage;
    p->flags = flags;
    for (int i = 0; i < k * k; ++i) p->w[i] = weights[i];
    p->shape = classify_shape(radius, weights);
    p->b = boundary;
    p->bq = round_to_storage(boundary, storage);
    double s = 0.0;
    for (int i = 0; i < k * k; ++i) s += double(weights[i]);
    p->wsum = s;
    default_blocking(p);
    *out = p;
    return ST_OK;
}

int stencil_plan3d(st_plan** out, int64_t planes, int64_t rows, int64_t cols, int radius, const float* weights,
                   double boundary, int storage, uint32_t flags) {
    if (!out) return fail(ST_EINVAL, "out is NULL");
    *out = nullptr;
    if (planes < 1 || rows < 1 || cols < 1) return fail(ST_EINVAL, "planes, rows and cols must be >= 1");
    if (planes > (int64_t(1) << 31) || rows > (int64_t(1) << 31) || cols > (int64_t(1) << 31))
        return fail(ST_EINVAL, "grid side too large");
    if (rows * cols > (int64_t(1) << 46) || planes > (int64_t(1) << 46) / (rows * cols))
        return fail(ST_EINVAL, "grid has more cells than device memory can hold");
    if (radius < 1 || radius > ST_MAX_RADIUS_3D) return fail(ST_EINVAL, "3D radius must be in [1, 2]");
    if (!weights) return fail(ST_EINVAL, "weights is NULL");
    if (storage != ST_F32 && storage != ST_BF16 && storage != ST_F16) return fail(ST_EINVAL, "unknown storage type");
    if (!std::isfinite(boundary)) return fail(ST_EINVAL, "boundary value must be finite");
    if (flags & ~ST_FLAG_GRAPH) return fail(ST_EINVAL, "3D plans take ST_FLAG_GRAPH only");
    const int k = 2 * radius + 1;
    for (int i = 0; i < k * k * k; ++i)
        if (!std::isfinite(weights[i])) return fail(ST_EINVAL, "weights must be finite");
    st_plan* p = new (std::nothrow) st_plan;
    if (!p) return fail(ST_ENOMEM, "plan allocation failed");
    init_plan(p);
    p->kind = KIND_3D;
    p->planes = planes;
    p->rows = rows;
    p->cols = cols;
    p->radius = radius;
    p->storage = storage;
    p->flags = flags;
    double s = 0.0;
    bool box = false;
    for (int dz = -radius; dz <= radius; ++dz)
        for (int dy = -radius; dy <= radius; ++dy)
            for (int dx = -radius; dx <= radius; ++dx) {
                const int q = ((dz + radius) * k + dy + radius) * k + dx + radius;
                p->w3[q] = weights[q];
                s += double(weights[q]);
                if (((dz != 0) + (dy != 0) + (dx != 0)) > 1 && weights[q] != 0.0f) box = true;
            }
    p->shape = box ? SHAPE_BOX : SHAPE_STAR;
    p->wsum = s;
    p->b = boundary;
    p->bq = round_to_storage(boundary, storage);
    p->tb = 1;
    *out = p;
    return ST_OK;
}

int stencil_get_planes(const st_plan* plan, int64_t* planes) {
    if (!plan || !planes) return fail(ST_EINVAL, "NULL argument");
    *planes = plan->planes;
    return ST_OK;
}

int stencil_plan_varcoef(st_plan** out, int64_t rows, int64_t cols, double boundary, uint32_t flags) {
    if (!out) return fail(ST_EINVAL, "out is NULL");
    *out = nullptr;
    if (rows < 1 || cols < 1) return fail(ST_EINVAL, "rows and cols must be >= 1");
    if (rows > (int64_t(1) << 31) || cols > (int64_t(1) << 31)) return fail(ST_EINVAL, "grid side too large");
    if (rows * cols > (int64_t(1) << 46)) return fail(ST_EINVAL, "grid has more cells than device memory can hold");
    if (!std::isfinite(boundary)) return fail(ST_EINVAL, "boundary value must be finite");
    if (int rc = check_flags(flags)) return rc;
    st_plan* p = new (std::nothrow) st_plan;
    if (!p) return fail(ST_ENOMEM, "plan allocation failed");
    init_plan(p);
    p->kind = KIND_VARCOEF;
    p->rows = rows;
    p->cols = cols;
    p->radius = 1;
    p->shape = SHAPE_STAR;
    p->storage = ST_F32;
    p->flags = flags;
    p->b = boundary;
    p->bq = float(boundary);
    p->tile_x = 128;
    p->tile_y = 64;
    p->tb = 4;
    while (p->tb > 1 && varcoef_lds_bytes(p->tb, p->tile_x, p->tile_y) > lds_limit()) --p->tb;
    *out = p;
    return ST_OK;
}

int stencil_destroy(st_plan* plan) {
    if (!plan) return ST_OK;
    drop_graph(plan);
    delete plan;
    return ST_OK;
}

int stencil_tiles(int* xy, int cap, int* n) {
    if (!n || (cap > 0 && !xy) || cap < 0) return fail(ST_EINVAL, "bad arguments");
    *n = supported_tiles(xy, cap);
    return ST_OK;
}

int stencil_set_blocking(st_plan* plan, int tb, int tile_x, int tile_y) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind == KIND_3D) return fail(ST_EUNSUPPORTED, "3D plans have one blocking");
    if (tb < 0 || tb > (plan->variant == VARIANT_RESIDENT ? 64 : 16) || tile_x < 0 || tile_y < 0)
        return fail(ST_EINVAL, "blocking out of range");
    const int tx = tile_x ? tile_x : plan->tile_x;
    const int ty = tile_y ? tile_y : plan->tile_y;
    if (!tile_supported(plan->shape, plan->radius, tx, ty)) return fail(ST_EUNSUPPORTED, "tile not instantiated");
    const int t = tb ? tb : plan->tb;
    if (plan->kind == KIND_CONST && t > max_tb(plan, tx, ty))
        return fail(ST_EUNSUPPORTED, "temporal block too deep for this tile's LDS budget");
    if (plan->kind == KIND_VARCOEF && varcoef_lds_bytes(t, tx, ty) > lds_limit())
        return fail(ST_EUNSUPPORTED, "temporal block too deep for the LDS budget");
    plan->tb = t;
    plan->tile_x = tx;
    plan->tile_y = ty;
    drop_graph(plan);
    return ST_OK;
}

int stencil_set_variant(st_plan* plan, int variant) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind == KIND_3D) return fail(ST_EUNSUPPORTED, "3D plans have one kernel");
    if (variant != ST_VARIANT_TILED && variant != ST_VARIANT_STREAM && variant != ST_VARIANT_MARCH &&
        variant != ST_VARIANT_MARCH8 && variant != ST_VARIANT_MARCH1 && variant != ST_VARIANT_RESIDENT &&
        variant != ST_VARIANT_MFMA)
        return fail(ST_EINVAL, "unknown variant");
    if (variant == ST_VARIANT_MFMA && !mfma_usable(plan))
        return fail(ST_EUNSUPPORTED, "the matrix-core variant takes FP32 constant-weight plans with a constant halo");
    if (variant == ST_VARIANT_RESIDENT && (plan->kind != KIND_CONST || plan->bc != ST_BC_CONST))
        return fail(ST_EUNSUPPORTED, "the resident variant takes constant-weight plans with a constant halo");
    if (variant == ST_VARIANT_STREAM && (plan->kind != KIND_CONST || !stream_usable(plan)))
        return fail(ST_EUNSUPPORTED, "streaming needs an FP32 constant-weight plan with cols % 4 == 0");
    if ((variant == ST_VARIANT_MARCH || variant == ST_VARIANT_MARCH8 || variant == ST_VARIANT_MARCH1) &&
        !march_usable(plan))
        return fail(ST_EUNSUPPORTED, "marching needs a constant-weight plan");
    if (plan->bc != ST_BC_CONST && !is_march(variant))
        return fail(ST_EUNSUPPORTED, "periodic and framed boundaries run on the marching variants only");
    const int old = plan->variant;
    plan->variant = variant;
    if (plan->tb > max_tb(plan, plan->tile_x, plan->tile_y)) {  // keep the plan launchable
        plan->variant = old;
        return fail(ST_EUNSUPPORTED, "current temporal block too deep for this variant; lower it first");
    }
    drop_graph(plan);
    return ST_OK;
}

int stencil_set_boundary(st_plan* plan, int kind, const void* frame) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind == KIND_3D) return fail(ST_EUNSUPPORTED, "3D plans take a constant halo only");
    if (plan->kind != KIND_CONST) return fail(ST_EINVAL, "boundary rules apply to constant-weight plans");
    if (kind != ST_BC_CONST && kind != ST_BC_PERIODIC && kind != ST_BC_FRAME) return fail(ST_EINVAL, "unknown boundary");
    if ((kind == ST_BC_FRAME) != (frame != nullptr)) return fail(ST_EINVAL, "a frame is given exactly with ST_BC_FRAME");
    if (kind != ST_BC_CONST && (plan->flags & ST_FLAG_NAIVE))
        return fail(ST_EUNSUPPORTED, "the naive reference path takes a constant halo only");
    if (kind != ST_BC_CONST && !is_march(plan->variant)) {
        plan->variant = VARIANT_MARCH;
        plan->tb = std::min(plan->tb, march_max_tb(plan->shape, plan->radius, 4));
    }
    plan->bc = kind;
    plan->frame = frame;
    drop_graph(plan);
    return ST_OK;
}

int stencil_get_boundary(const st_plan* plan, int* kind) {
    if (!plan || !kind) return fail(ST_EINVAL, "NULL argument");
    *kind = plan->bc;
    return ST_OK;
}

int stencil_frame_elems(const st_plan* plan, int64_t* elems) {
    if (!plan || !elems) return fail(ST_EINVAL, "NULL argument");
    *elems = 2 * int64_t(plan->radius) * (plan->cols + 2 * plan->radius) + 2 * int64_t(plan->radius) * plan->rows;
    return ST_OK;
}

int stencil_set_march_segment(st_plan* plan, int64_t min_rows) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (min_rows < 0) return fail(ST_EINVAL, "min_rows must be >= 0");
    plan->seg_min = min_rows;
    drop_graph(plan);
    return ST_OK;
}

int stencil_get_march_segment(const st_plan* plan, int64_t* min_rows) {
    if (!plan || !min_rows) return fail(ST_EINVAL, "NULL argument");
    *min_rows = plan->seg_min;
    return ST_OK;
}

int stencil_get_variant(const st_plan* plan, int* variant) {
    if (!plan || !variant) return fail(ST_EINVAL, "NULL argument");
    *variant = plan->variant;
    return ST_OK;
}

int stencil_get_dims(const st_plan* plan, int64_t* rows, int64_t* cols, int* storage) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (rows) *rows = plan->rows;
    if (cols) *cols = plan->cols;
    if (storage) *storage = plan->storage;
    return ST_OK;
}

int stencil_get_blocking(const st_plan* plan, int* tb, int* tile_x, int* tile_y) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (tb) *tb = plan->tb;
    if (tile_x) *tile_x = plan->tile_x;
    if (tile_y) *tile_y = plan->tile_y;
    return ST_OK;
}

int stencil_set_spin_limit(st_plan* plan, int64_t polls) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (polls < 1) return fail(ST_EINVAL, "polls must be >= 1");
    plan->spin_limit = polls;
    drop_graph(plan);
    return ST_OK;
}

static bool resident_run(const st_plan* p) {
    return p->variant == VARIANT_RESIDENT && p->kind == KIND_CONST && !(p->flags & ST_FLAG_NAIVE);
}

static int64_t n_passes(const st_plan* p, int64_t steps) {
    if (steps <= 0) return 0;
    const int64_t tb = (p->flags & ST_FLAG_NAIVE) ? 1 : p->tb;
    return (steps + tb - 1) / tb;
}

int stencil_workspace_bytes(const st_plan* plan, int64_t steps, size_t* bytes) {
    if (!plan || !bytes) return fail(ST_EINVAL, "NULL argument");
    if (steps < 0) return fail(ST_EINVAL, "steps must be >= 0");
    if (resident_run(plan)) {
        *bytes = steps >= 1 ? ((size_t(field_cells(plan)) * elem_size(plan->storage) + 255) & ~size_t(255)) +
                                  resident_ws_tail()
                            : 0;
        return ST_OK;
    }
    *bytes = n_passes(plan, steps) >= 2 ? size_t(field_cells(plan)) * elem_size(plan->storage) : 0;
    return ST_OK;
}

static bool overlap(const void* a, const void* b, size_t n) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + n && y < x + n;
}

// Enqueue all passes of a run on `s`.
static int enqueue_run(st_plan* p, const void* in, void* out, const float* kappa, int64_t steps, void* ws,
                       hipStream_t s) {
    const size_t bytes = size_t(field_cells(p)) * elem_size(p->storage);
    if (steps == 0) {
        ST_HIP_CHECK(hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s));
        return ST_OK;
    }
    if (resident_run(p)) return launch_resident(p, in, out, ws, steps, s);
    const bool naive = p->flags & ST_FLAG_NAIVE;
    const int64_t tb = naive ? 1 : p->tb;
    const int64_t P = n_passes(p, steps);
    const void* src = in;
    for (int64_t k = 0; k < P; ++k) {
        void* dst = ((P - 1 - k) % 2 == 0) ? out : ws;
        const int levels = int(std::min<int64_t>(tb, steps - k * tb));
        int rc;
        if (p->kind == KIND_3D)
            rc = launch_3d(p, src, dst, s);
        else if (p->kind == KIND_VARCOEF)
            rc = varcoef_launch(p, static_cast<const float*>(src), static_cast<float*>(dst), kappa, naive ? 0 : levels, s);
        else if (naive)
            rc = launch_naive(p, src, dst, kappa, s);
        else
            rc = launch_pass(p, src, dst, kappa, levels, s);
        if (rc) return rc;
        src = dst;
    }
    return ST_OK;
}

static int run_common(st_plan* plan, const void* in, void* out, const float* kappa, int64_t steps, void* workspace,
                      size_t ws_bytes, void* stream) {
    if (!in || !out) return fail(ST_EINVAL, "in/out is NULL");
    if (steps < 0) return fail(ST_EINVAL, "steps must be >= 0");
    const size_t bytes = size_t(field_cells(plan)) * elem_size(plan->storage);
    if (overlap(in, out, bytes)) return fail(ST_EALIAS, "in and out overlap");
    size_t need = 0;
    stencil_workspace_bytes(plan, steps, &need);
    if (need) {
        if (!workspace || ws_bytes < need) return fail(ST_ENOWS, "workspace too small");
        if (overlap(workspace, in, bytes) || overlap(workspace, out, bytes))
            return fail(ST_EALIAS, "workspace overlaps in/out");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // (the resident variant is one cooperative launch: it is not captured)
    if (!(plan->flags & ST_FLAG_GRAPH) || steps == 0 || resident_run(plan))
        return enqueue_run(plan, in, out, kappa, steps, workspace, s);

    // graph path: capture the passes once per (in, kappa, out, workspace, steps, stream)
    if (!(plan->graph_exec && plan->g_in == in && plan->g_kappa == kappa && plan->g_out == out &&
          plan->g_ws == workspace && plan->g_steps == steps && plan->g_stream == stream)) {
        drop_graph(plan);
        hipStream_t cap;
        ST_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return fail(ST_EHIP, "hipStreamBeginCapture failed");
        }
        int rc = enqueue_run(plan, in, out, kappa, steps, workspace, cap);
        hipError_t e = hipStreamEndCapture(cap, &graph);
        (void)hipStreamDestroy(cap);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(ST_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(ST_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        plan->graph_exec = exec;
        plan->g_in = in;
        plan->g_kappa = kappa;
        plan->g_out = out;
        plan->g_ws = workspace;
        plan->g_steps = steps;
        plan->g_stream = stream;
    }
    ST_HIP_CHECK(hipGraphLaunch(static_cast<hipGraphExec_t>(plan->graph_exec), s));
    return ST_OK;
}

int stencil_run(st_plan* plan, const void* in, void* out, int64_t steps, void* workspace, size_t ws_bytes,
                void* stream) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind == KIND_VARCOEF) return fail(ST_EINVAL, "varcoef plans run through stencil_run_varcoef");
    return run_common(plan, in, out, nullptr, steps, workspace, ws_bytes, stream);
}

int stencil_resident_status(const st_plan* plan, const void* workspace, size_t ws_bytes, int* status4, void* stream) {
    if (!plan || !workspace || !status4) return fail(ST_EINVAL, "NULL argument");
    if (plan->kind != KIND_CONST) return fail(ST_EINVAL, "not a constant-weight plan");
    const size_t need = ((size_t(field_cells(plan)) * elem_size(plan->storage) + 255) & ~size_t(255)) + resident_ws_tail();
    if (ws_bytes < need) return fail(ST_ENOWS, "workspace smaller than a resident run's");
    return read_resident_status(plan, workspace, status4, static_cast<hipStream_t>(stream));
}

int stencil_run_varcoef(st_plan* plan, const float* in, const float* kappa, float* out, int64_t steps,
                        void* workspace, size_t ws_bytes, void* stream) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind != KIND_VARCOEF) return fail(ST_EINVAL, "not a varcoef plan");
    if (!kappa) return fail(ST_EINVAL, "kappa is NULL");
    const size_t bytes = size_t(field_cells(plan)) * 4;
    if (overlap(kappa, out, bytes)) return fail(ST_EALIAS, "kappa and out overlap");
    return run_common(plan, in, out, kappa, steps, workspace, ws_bytes, stream);
}

}  // extern "C"

// Times every candidate blocking of `plan` on the caller's buffers (kappa: varcoef plans only) and
// keeps the fastest; see stencil_autotune.
static int autotune_impl(st_plan* plan, const void* in, const float* kappa, void* out, void* workspace,
                         size_t ws_bytes, int64_t sample_steps, int* tb_out, int* tile_x_out, int* tile_y_out,
                         void* stream) {
    if (plan->flags & ST_FLAG_NAIVE) return fail(ST_ESTATE, "naive plans have nothing to tune");
    if (sample_steps < 1) return fail(ST_EINVAL, "sample_steps must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t saved_flags = plan->flags;
    plan->flags &= ~ST_FLAG_GRAPH;
    int best_tb = plan->tb, best_tx = plan->tile_x, best_ty = plan->tile_y, best_var = plan->variant;
    int64_t best_seg = plan->seg_min;
    float best_ms = 1e30f;
    int tiles[32];
    const int nt = supported_tiles(tiles, 16);
    static const int kTb[] = {1, 2, 3, 4, 6, 8};
    hipEvent_t e0, e1;
    ST_HIP_CHECK(hipEventCreate(&e0));
    ST_HIP_CHECK(hipEventCreate(&e1));
    int rc = ST_OK;
    const int nvar = plan->kind == KIND_CONST ? 7 : 1;
    for (int var = 0; var < nvar && rc == ST_OK; ++var)
    for (int ti = 0; ti < nt && rc == ST_OK; ++ti) {
        if (var == VARIANT_STREAM && !stream_usable(plan)) break;
        if (plan->bc != ST_BC_CONST && !is_march(var)) break;  // other boundaries: marching only
        if (var == VARIANT_RESIDENT && (ti > 0 || plan->bc != ST_BC_CONST)) break;  // no tile either
        if (var == VARIANT_MFMA && (ti > 0 || !(saved_flags & ST_FLAG_ALLOW_MFMA) || !mfma_usable(plan))) break;
        if (is_march(var) && (ti > 0 || !march_usable(plan))) break;  // marching has no tile
        if (var == VARIANT_MARCH8 && plan->cols % 8 != 0) break;  // would run the four-column kernels
        const int tx = tiles[2 * ti], ty = tiles[2 * ti + 1];
        plan->variant = var;
        // LDS tiles: the depths of kTb; marching: every depth it offers
        int cands[16], nc = 0;
        if (var == VARIANT_MFMA) {
            cands[nc++] = 1;
        } else if (var == VARIANT_RESIDENT) {
            static const int kRes[] = {1, 2, 4, 8, 12, 16, 24, 32, 48};
            for (int tb : kRes)
                if (resident_usable(plan, tb) && nc < 16) cands[nc++] = tb;
        } else if (is_march(var)) {
            for (int tb = 1; tb <= max_tb(plan, tx, ty) && nc < 16; ++tb) cands[nc++] = tb;
        } else {
            for (int tb : kTb) cands[nc++] = tb;
        }
        for (int k = 0; k < nc && rc == ST_OK; ++k) {
            const int tb = cands[k];
            if (plan->kind == KIND_CONST && tb > max_tb(plan, tx, ty)) continue;
            if (plan->kind == KIND_VARCOEF && varcoef_lds_bytes(tb, tx, ty) > lds_limit()) continue;
            if (tb > sample_steps) continue;
            plan->tb = tb;
            plan->tile_x = tx;
            plan->tile_y = ty;
            size_t need = 0;
            stencil_workspace_bytes(plan, sample_steps, &need);
            if (need > ws_bytes) continue;
            // marching with several levels: also segments of at least 1/2, 1, 2, 4, 8 x r (tb - 1) rows
            int64_t segs[6] = {0}, ns = 1;
            if (is_march(var) && tb > 1) {
                const int64_t unit = int64_t(plan->radius) * (tb - 1);
                if (unit >= 4 && unit / 2 < plan->rows) segs[ns++] = unit / 2;
                for (int64_t f = 1; f <= 8; f *= 2)
                    if (f * unit < plan->rows) segs[ns++] = f * unit;
            }
            for (int64_t si = 0; si < ns && rc == ST_OK; ++si) {
                plan->seg_min = segs[si];
                if ((rc = run_common(plan, in, out, kappa, sample_steps, workspace, ws_bytes, stream))) break;  // warm-up
                float ms = 1e30f;  // the better of two timed runs
                for (int rep = 0; rep < 2 && rc == ST_OK; ++rep) {
                    if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(ST_EHIP, "hipEventRecord"); break; }
                    if ((rc = run_common(plan, in, out, kappa, sample_steps, workspace, ws_bytes, stream))) break;
                    if (hipEventRecord(e1, s) != hipSuccess) { rc = fail(ST_EHIP, "hipEventRecord"); break; }
                    if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(ST_EHIP, "hipEventSynchronize"); break; }
                    float t = 0;
                    (void)hipEventElapsedTime(&t, e0, e1);
                    ms = std::min(ms, t);
                }
                if (rc) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best_tb = tb;
                    best_tx = tx;
                    best_ty = ty;
                    best_var = var;
                    best_seg = segs[si];
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->flags = saved_flags;
    plan->variant = best_var;
    plan->tb = best_tb;
    plan->tile_x = best_tx;
    plan->tile_y = best_ty;
    plan->seg_min = best_seg;
    drop_graph(plan);
    if (rc) return rc;
    if (tb_out) *tb_out = best_tb;
    if (tile_x_out) *tile_x_out = best_tx;
    if (tile_y_out) *tile_y_out = best_ty;
    return ST_OK;
}

extern "C" {

int stencil_autotune(st_plan* plan, const void* in, void* out, void* workspace, size_t ws_bytes,
                     int64_t sample_steps, int* tb_out, int* tile_x_out, int* tile_y_out, void* stream) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind == KIND_3D) return fail(ST_EUNSUPPORTED, "3D plans have nothing to tune");
    if (plan->kind != KIND_CONST) return fail(ST_EINVAL, "varcoef plans are tuned by stencil_autotune_varcoef");
    return autotune_impl(plan, in, nullptr, out, workspace, ws_bytes, sample_steps, tb_out, tile_x_out, tile_y_out,
                         stream);
}

int stencil_autotune_varcoef(st_plan* plan, const float* in, const float* kappa, float* out, void* workspace,
                             size_t ws_bytes, int64_t sample_steps, int* tb_out, int* tile_x_out, int* tile_y_out,
                             void* stream) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind != KIND_VARCOEF) return fail(ST_EINVAL, "not a varcoef plan");
    if (!kappa) return fail(ST_EINVAL, "kappa is NULL");
    if (!in || !out) return fail(ST_EINVAL, "in/out is NULL");
    const size_t bytes = size_t(field_cells(plan)) * 4;
    if (overlap(kappa, out, bytes)) return fail(ST_EALIAS, "kappa and out overlap");
    return autotune_impl(plan, in, kappa, out, workspace, ws_bytes, sample_steps, tb_out, tile_x_out, tile_y_out,
                         stream);
}

}  // extern "C"

extern "C" {

int stencil_solve_ws_bytes(const st_plan* plan, int64_t check_every, size_t* bytes) {
    if (!plan || !bytes) return fail(ST_EINVAL, "NULL argument");
    if (check_every < 1) return fail(ST_EINVAL, "check_every must be >= 1");
    size_t nb = 0, run_ws = 0;
    if (int rc = stencil_norms_ws_bytes(plan, &nb)) return rc;
    if (int rc = stencil_workspace_bytes(plan, check_every, &run_ws)) return rc;
    const size_t field = (size_t(field_cells(plan)) * elem_size(plan->storage) + 255) & ~size_t(255);
    *bytes = field + std::max(run_ws, field) + ((nb + 255) & ~size_t(255)) + 256 + 256;
    return ST_OK;
}

}  // extern "C"

namespace st {
namespace {

// Solve bookkeeping on the device: rec = {stop flag, pad, steps done (int64), relative residual}.
struct SolveRec {
    int stop;
    int pad;
    int64_t steps;
    double rel;
};

__global__ void solve_reset(SolveRec* r) {
    r->stop = 0;
    r->steps = 0;
    r->rel = 0.0;
}

// After an interval: the relative residual of its last step; raise the stop flag at convergence
// or at the last interval, and record where the run stopped.
__global__ void solve_check(const double* sums, double tol, int64_t steps_after, int last, SolveRec* r) {
    if (r->stop) return;
    const double rel = sums[1] > 0.0 ? sqrt(sums[0] / sums[1]) : sqrt(sums[0]);
    r->rel = rel;
    r->steps = steps_after;
    if (rel <= tol || last) r->stop = 1;
}

}  // namespace
}  // namespace st

extern "C" {

int stencil_solve(st_plan* plan, const void* in, void* out, int64_t max_steps, int64_t check_every, double tol,
                  int64_t* steps_done, double* rel_residual, void* workspace, size_t ws_bytes, void* stream) {
    if (!plan || !in || !out || !steps_done || !rel_residual) return fail(ST_EINVAL, "NULL argument");
    if (plan->kind == KIND_VARCOEF) return fail(ST_EINVAL, "stencil_solve takes a constant-weight plan");
    if (max_steps < 1 || check_every < 1 || !(tol >= 0.0)) return fail(ST_EINVAL, "bad max_steps/check_every/tol");
    size_t need = 0;
    if (int rc = stencil_solve_ws_bytes(plan, check_every, &need)) return rc;
    if (!workspace || ws_bytes < need) return fail(ST_ENOWS, "workspace too small");
    const size_t bytes = size_t(field_cells(plan)) * elem_size(plan->storage);
    if (overlap(in, out, bytes)) return fail(ST_EALIAS, "in and out overlap");
    const size_t field = (bytes + 255) & ~size_t(255);
    size_t run_ws = 0, nb = 0;
    stencil_workspace_bytes(plan, check_every, &run_ws);
    stencil_norms_ws_bytes(plan, &nb);
    char* ws = static_cast<char*>(workspace);
    void* prev = ws;                                   // the iterate one step before `out`
    void* scratch = ws + field;                        // stencil_run's own ping-pong field
    const size_t scratch_bytes = std::max(run_ws, field);
    void* nscr = ws + field + scratch_bytes;           // norms partial sums
    double* sums = reinterpret_cast<double*>(static_cast<char*>(nscr) + ((nb + 255) & ~size_t(255)));
    SolveRec* rec = reinterpret_cast<SolveRec*>(reinterpret_cast<char*>(sums) + 256);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the two runs per check differ in their buffers and step counts, so a cached graph would be
    // captured again on every call: enqueue directly for the duration of the solve
    struct Guard {
        st_plan* p;
        uint32_t saved;
        ~Guard() {
            p->flags = saved;
            p->stop = nullptr;
        }
    } guard{plan, plan->flags};
    plan->flags &= ~ST_FLAG_GRAPH;
    // Marching plans: the convergence test runs on the device, where it raises a flag that turns
    // the remaining passes and reductions into no-ops, so the host enqueues checks in growing
    // chunks (1, 2, 4, ... 64) and synchronises once per chunk, not once per check.  Other
    // variants read the residual back at every check.
    const bool on_device = plan->kind == KIND_CONST && !(plan->flags & ST_FLAG_NAIVE) && is_march(plan->variant) &&
                           march_usable(plan) &&
                           plan->tb <= march_max_tb(plan->shape, plan->radius, march_vmax(plan->variant));
    if (on_device) {
        clear_stale_error();
        hipLaunchKernelGGL(solve_reset, dim3(1), dim3(1), 0, s, rec);
        ST_LAUNCH_CHECK("solve_reset");
        plan->stop = &rec->stop;
        const void* cur = in;
        int64_t enq = 0;
        for (int64_t chunk = 1; enq < max_steps; chunk = std::min<int64_t>(chunk * 2, 64)) {
            for (int64_t c = 0; c < chunk && enq < max_steps; ++c) {
                const int64_t k = std::min(check_every, max_steps - enq);
                if (int rc = stencil_run(plan, cur, prev, k - 1, scratch, scratch_bytes, stream)) return rc;
                if (int rc = stencil_run(plan, prev, out, 1, scratch, scratch_bytes, stream)) return rc;
                enq += k;
                if (int rc = launch_norms(plan, prev, out, sums, nscr, nb, &rec->stop, s)) return rc;
                hipLaunchKernelGGL(solve_check, dim3(1), dim3(1), 0, s, sums, tol, enq, enq == max_steps ? 1 : 0, rec);
                ST_LAUNCH_CHECK("solve_check");
                cur = out;
            }
            SolveRec h;
            ST_HIP_CHECK(hipMemcpyAsync(&h, rec, sizeof(h), hipMemcpyDeviceToHost, s));
            ST_HIP_CHECK(hipStreamSynchronize(s));
            if (h.stop) {
                *steps_done = h.steps;
                *rel_residual = h.rel;
                return ST_OK;
            }
        }
        return fail(ST_ESTATE, "internal: the solve ended without its stop record");
    }
    const void* cur = in;
    int64_t done = 0;
    double rel = 0.0;
    while (done < max_steps) {
        const int64_t k = std::min(check_every, max_steps - done);
        // k - 1 steps into `prev`, then the last step into `out`: the residual compares them
        if (int rc = stencil_run(plan, cur, prev, k - 1, scratch, scratch_bytes, stream)) return rc;
        if (int rc = stencil_run(plan, prev, out, 1, scratch, scratch_bytes, stream)) return rc;
        done += k;
        if (int rc = stencil_norms(plan, prev, out, sums, nscr, nb, stream)) return rc;
        double h[4];
        ST_HIP_CHECK(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s));
        ST_HIP_CHECK(hipStreamSynchronize(s));
        rel = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
        if (rel <= tol) break;
        cur = out;
    }
    *steps_done = done;
    *rel_residual = rel;
    return ST_OK;
}

}  // extern "C"

// --------------------------------------------------------------------------
// stencil_run_noalloc: stencil_run with its ping-pong field in a static device array
// --------------------------------------------------------------------------
namespace st {
namespace {

constexpr size_t kNoallocBytes = size_t(64) << 20;  // 16 Mi FP32 or 32 Mi 16-bit cells
constexpr int kMaxDevices = 64;

// The library's own ping-pong field for stencil_run_noalloc.  Each device holds its copy from the
// time the library's code object is loaded on it until the process ends.  Host code never uses
// this name as an address: the per-device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** ptr) {
    int dev = 0;
    ST_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ST_EUNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(ST_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return ST_OK;
}

}  // namespace
}  // namespace st

extern "C" {

int stencil_noalloc_max_bytes(size_t* bytes) {
    if (!bytes) return fail(ST_EINVAL, "bytes is NULL");
    *bytes = kNoallocBytes;
    return ST_OK;
}

int stencil_run_noalloc(st_plan* plan, const void* in, void* out, int64_t steps, void* stream) {
    if (!plan) return fail(ST_EINVAL, "plan is NULL");
    if (plan->kind == KIND_VARCOEF) return fail(ST_EINVAL, "stencil_run_noalloc takes a constant-weight plan");
    if (!in || !out) return fail(ST_EINVAL, "in/out is NULL");
    if (steps < 0) return fail(ST_EINVAL, "steps must be >= 0");
    const size_t bytes = size_t(field_cells(plan)) * elem_size(plan->storage);
    if (overlap(in, out, bytes)) return fail(ST_EALIAS, "in and out overlap");
    size_t need = 0;
    stencil_workspace_bytes(plan, steps, &need);
    if (need > kNoallocBytes)
        return fail(ST_EUNSUPPORTED, "grid larger than the static ping-pong field (64 MiB: 16 Mi FP32 or 32 Mi "
                                     "16-bit cells); use stencil_run with a workspace");
    void* ws = nullptr;
    if (int rc = scratch_address(&ws)) return rc;
    if (overlap(ws, in, bytes) || overlap(ws, out, bytes)) return fail(ST_EALIAS, "in/out overlap the static field");
    // always enqueued directly (never through the plan's cached graph, whose capture creates a
    // stream and instantiates a graph), so that a caller may capture this call itself
    return enqueue_run(plan, in, out, nullptr, steps, ws, static_cast<hipStream_t>(stream));
}

}  // extern "C"
