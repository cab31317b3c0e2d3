// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/mi355stencil.h"

namespace st {

// thread-local error detail, set by fail()
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// On failure the runtime's sticky last-error is consumed as well, so that it cannot be
// mistaken later for the status of an unrelated launch (ours or the caller's).
#define ST_HIP_CHECK(expr)                                                             \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (void)hipGetLastError();                                                   \
            return ::st::fail(ST_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)

#define ST_LAUNCH_CHECK(what)                                                          \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return ::st::fail(ST_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

enum Shape { SHAPE_STAR = 0, SHAPE_BOX = 1 };
enum Kind { KIND_CONST = 0, KIND_VARCOEF = 1, KIND_3D = 2 };
enum Variant {
    VARIANT_TILED = ST_VARIANT_TILED,
    VARIANT_STREAM = ST_VARIANT_STREAM,
    VARIANT_MARCH = ST_VARIANT_MARCH,
    VARIANT_MARCH8 = ST_VARIANT_MARCH8,
    VARIANT_MARCH1 = ST_VARIANT_MARCH1,
    VARIANT_RESIDENT = ST_VARIANT_RESIDENT,
    VARIANT_MFMA = ST_VARIANT_MFMA
};

constexpr int MAXK = (2 * ST_MAX_RADIUS + 1) * (2 * ST_MAX_RADIUS + 1);  // 81
constexpr int MAXK3 = (2 * ST_MAX_RADIUS_3D + 1) * (2 * ST_MAX_RADIUS_3D + 1) * (2 * ST_MAX_RADIUS_3D + 1);  // 125

// Workgroups of a one-cell-per-thread reference launch; beyond it the kernels stride over the grid
// (a launch may hold at most 2^32 threads).
constexpr int64_t kNaiveMaxBlocks = int64_t(1) << 20;

// Kernel argument block of one sweep pass (passed by value; weights live in kernargs).
struct SweepArgs {
    const void* src;
    void* dst;
    const float* kappa;  // varcoef only
    int64_t rows, cols;
    int64_t tiles_x, tiles_y;  // tile grid of this launch
    float b;                   // halo value, already rounded to the storage type
    int tb;                    // levels (steps) in this pass
    float w[MAXK];             // dense (2r+1)^2 row-major weights
};

}  // namespace st

struct st_plan {
    int kind;         // st::Kind
    int64_t rows, cols;
    int64_t planes;   // 3D plans: planes along z (1 for 2D plans)
    float w3[st::MAXK3];  // 3D plans: dense (2r+1)^3 weights
    int radius;
    int shape;        // st::Shape
    int storage;      // ST_F32 / ST_BF16 / ST_F16
    uint32_t flags;
    float w[st::MAXK];
    double b;         // as given
    float bq;         // b rounded to storage, widened to float
    double wsum;      // sum of the FP32 weights in FP64
    int tb, tile_x, tile_y;
    int variant;      // st::Variant (FP32 grids with cols % 4 == 0 may stream)
    int64_t seg_min;  // marching: least output rows per task (0: one task per resident wavefront)
    int bc;             // ST_BC_CONST (halo b), ST_BC_PERIODIC or ST_BC_FRAME (marching variants only)
    int64_t spin_limit; // resident variant: polls before a neighbour wait gives up
    const int* stop;    // while a solve runs: device flag that turns its marching passes into no-ops
    const void* frame;  // ST_BC_FRAME: caller-owned device frame (storage type)
    // cached hipGraph of a full run (ST_FLAG_GRAPH)
    void* graph_exec;
    const void* g_in;
    const float* g_kappa;  // varcoef plans: the diffusivity field the graph reads
    void* g_out;
    void* g_ws;
    int64_t g_steps;
    void* g_stream;
};

namespace st {

size_t elem_size(int storage);

// launchers (sweep.hip / varcoef.hip); return ST_OK or an error code
int launch_pass(const st_plan* p, const void* src, void* dst, const float* kappa, int levels, hipStream_t s);
int launch_naive(const st_plan* p, const void* src, void* dst, const float* kappa, hipStream_t s);
bool tile_supported(int shape, int radius, int tx, int ty);
int supported_tiles(int* xy, int cap);
int max_tb(const st_plan* p, int tx, int ty);
int varcoef_launch(const st_plan* p, const float* src, float* dst, const float* kappa, int levels, hipStream_t s);
size_t tiled_lds_bytes(int r, int tb, int tx, int ty);
size_t varcoef_lds_bytes(int tb, int tile_x, int tile_y);

// Largest dynamic LDS allocation one workgroup may request on the current device (bytes);
// 64 KiB when no device is visible.
size_t lds_limit();
// Allow `fn` to launch with `bytes` of dynamic LDS (ST_EUNSUPPORTED above lds_limit()).
int prepare_lds(const void* fn, size_t bytes);
// Workgroups of NT threads with `lds` bytes of dynamic LDS that fit the device at once.
int resident_blocks(const void* fn, size_t lds, int* blocks);
bool stream_usable(const st_plan* p);
// FP64 norms (norms.hip) with an optional device stop flag (NULL: always run).
int launch_norms(const st_plan* plan, const void* u_prev, const void* u, double* out4, void* workspace, size_t ws_bytes,
                 const int* stop, hipStream_t s);
// Cells of one field of the plan (planes * rows * cols).
inline int64_t field_cells(const st_plan* p) { return p->planes * p->rows * p->cols; }
// LDS-resident cooperative sweep (resident.hip): the whole run in one launch; workspace = one field
// + resident_ws_tail() bytes of counters and status.
size_t resident_ws_tail();
bool resident_usable(const st_plan* p, int tb);
int resident_max_tb(const st_plan* p);
int launch_resident(const st_plan* p, const void* in, void* out, void* ws, int64_t steps, hipStream_t s);
int read_resident_status(const st_plan* p, const void* ws, int* status4, hipStream_t s);
// Matrix-core pass (mfma_stencil.hip): one level, FP32 storage, constant halo; not the canonical
// FMA order bit for bit (within FP32 rounding of it).
bool mfma_usable(const st_plan* p);
int launch_mfma(const st_plan* p, const void* src, void* dst, hipStream_t s);
// 3D pass (stencil3d.hip): one step of a 3D plan.
int launch_3d(const st_plan* p, const void* src, void* dst, hipStream_t s);
// Row-marching pass (march.hip): constant-weight plans of any storage, width and alignment, up to
// vmax (1, 4 or 8) columns per lane; up to march_max_tb(shape, radius, vmax) levels per pass (vmax 4:
// star 8 / 6 / 4 / 3 for r = 1 / 2 / 3 / 4, box 6 / 3 / 2 / 2; vmax 8: star 8 / 4 / 3 / 2, box
// 3 / 2 / 2 / 1).
int march_max_tb(int shape, int radius, int vmax);
bool march_usable(const st_plan* p);
int launch_march(const st_plan* p, const void* src, void* dst, int levels, int vmax, hipStream_t s);
inline bool is_march(int variant) {
    return variant == VARIANT_MARCH || variant == VARIANT_MARCH8 || variant == VARIANT_MARCH1;
}
inline int march_vmax(int variant) { return variant == VARIANT_MARCH8 ? 8 : variant == VARIANT_MARCH1 ? 1 : 4; }
// Drop a stale runtime error left by earlier API calls so that the check after our next
// launch reports that launch only.
inline void clear_stale_error() { (void)hipGetLastError(); }

}  // namespace st
