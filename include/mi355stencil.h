/*
 * mi355stencil.h -- C ABI of the MI355X (gfx950) library for iterated 2D
 * Jacobi stencils with fixed halos, its batched form, 16-bit storage, FP64
 * norms, and the CNN surrogate that advances a variable-coefficient heat
 * field K steps at once.
 *
 * Conventions for every entry point
 *   - Returns an int status: ST_OK (0) or a negative ST_E* code.  Never throws.
 *     stencil_last_error() gives a thread-local message for the last failure.
 *   - Device pointers are plain HIP device addresses owned by the caller
 *     (for example torch tensors' data_ptr()).  The library never allocates
 *     device memory behind the caller's back: scratch space is a caller-owned
 *     "workspace" whose minimum size is queried first.  Plans, batches and
 *     models own host memory only (the batched entry point also owns one
 *     pinned host staging table and one hipGraph).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued on it, asynchronously.  Only the entry
 *     points marked "synchronises" wait for the device.
 *   - Fields are row-major with pitch = cols elements: element (i, j) lives at
 *     base[i * cols + j], i = row in [0, rows), j = column in [0, cols).
 *   - Launch errors are checked right after each launch (ST_EHIP); faults
 *     inside a kernel surface at the caller's next synchronisation.
 *   - One device per process: occupancy and LDS limits are queried once, on
 *     the device current at the first call, and cached.  A plan or batch may
 *     be used from one host thread at a time (it caches graphs and tables).
 */
#ifndef MI355STENCIL_H
#define MI355STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ST_OK            0
#define ST_EINVAL       (-1)  /* bad shape, radius, weights, pointer or count */
#define ST_EALIAS       (-2)  /* input and output buffers overlap              */
#define ST_EUNSUPPORTED (-3)  /* no kernel for this combination                */
#define ST_EHIP         (-4)  /* a HIP runtime call or kernel launch failed     */
#define ST_ENOWS        (-5)  /* workspace missing or smaller than required    */
#define ST_ENOMEM       (-6)  /* host allocation failed                        */
#define ST_ESTATE       (-7)  /* object used in a state that does not allow it */

/* ---- storage types ----------------------------------------------------- */
#define ST_F32   0   /* IEEE binary32                                     */
#define ST_BF16  1   /* bfloat16 (upper half of binary32), raw uint16 bits */
#define ST_F16   2   /* IEEE binary16, raw uint16 bits                     */

/* ---- plan flags -------------------------------------------------------- */
#define ST_FLAG_NAIVE  0x1u  /* one step per launch, no LDS tiling: the plain GPU reference path */
#define ST_FLAG_GRAPH  0x2u  /* stencil_run replays its passes from a cached hipGraph            */
#define ST_FLAG_ALLOW_MFMA 0x4u /* stencil_autotune may pick ST_VARIANT_MFMA, whose results are
                                   within FP32 rounding of the canonical order, not bit for bit */

#define ST_MAX_RADIUS 4
#define ST_MAX_RADIUS_3D 2

typedef struct st_plan st_plan;
typedef struct st_batch st_batch;
typedef struct sg_model sg_model;

/* stencil_plan -- describe one iterated 2D Jacobi stencil.
 *
 * Operation (paper Sec. II-C, Jacobi update equation; Sec. IV-A, zero padding
 * and halo of depth r; Sec. IV-E, centre-first accumulation):
 *   for every cell (i, j) of a rows x cols grid,
 *     u'(i,j) = sum_{dy,dx in [-r, r]} W[dy+r][dx+r] * ~u(i+dy, j+dx),
 *   where ~u equals u on the grid and the fixed halo value `boundary` outside
 *   it; the halo is never updated, and every step reads only the previous one.
 *
 *   weights   host pointer to (2r+1)^2 floats, row-major; W[dy+r][dx+r]
 *             multiplies the value dy rows below and dx columns right (a
 *             correlation).  Copied into the plan.  Must be finite.
 *   radius    1 <= r <= ST_MAX_RADIUS.
 *   boundary  fixed halo value b; rounded to the storage type.  Finite.
 *   storage   ST_F32, ST_BF16 or ST_F16.  Arithmetic is FP32 in every case;
 *             16-bit fields are rounded (nearest-even) after every step.
 *   flags     ST_FLAG_* bits.
 * Per-cell FP32 order: acc = W_c * u_c, then acc = fma(W_k, u_k, acc) over the
 * footprint taps in row-major (dy, dx) order (star footprint when every weight
 * off the two axes is zero, else the full box).
 * Errors: ST_EINVAL (rows or cols < 1 or > 2^31, more than 2^46 cells, bad
 * radius, non-finite weight or b, NULL out/weights, unknown storage or flag
 * bits), ST_ENOMEM. */
int stencil_plan(st_plan** out, int64_t rows, int64_t cols, int radius, const float* weights,
                 double boundary, int storage, uint32_t flags);

/* stencil_plan3d -- the same Jacobi update on a 3D grid of planes x rows x cols cells (element
 * (k, i, j) at base[(k * rows + i) * cols + j]):
 *   u'(k,i,j) = sum_{dz,dy,dx in [-r, r]} W[dz+r][dy+r][dx+r] * ~u(k+dz, i+dy, j+dx),
 * ~u = u in the grid and the constant `boundary` outside (the paper's fixed halo, Sec. IV-A, in
 * three dimensions); weights: (2r+1)^3 floats, row-major in (dz, dy, dx).  Per-cell FP32 order: the
 * centre product, then one FMA per footprint tap in row-major (dz, dy, dx) order (star footprint --
 * the taps on the three axes -- when every other weight is zero, else the full box).
 * 1 <= r <= ST_MAX_RADIUS_3D; storage ST_F32 / ST_BF16 / ST_F16 (FP32 arithmetic, rounded every
 * step); flags: ST_FLAG_GRAPH only.  A 3D plan runs one step per pass (stencil_run, stencil_run_noalloc,
 * stencil_workspace_bytes and stencil_norms take it; the blocking, variant, boundary, autotune and
 * batch calls refuse it with ST_EUNSUPPORTED, and its norms' next-step mass is NaN).  Errors: as
 * stencil_plan, and planes < 1. */
int stencil_plan3d(st_plan** out, int64_t planes, int64_t rows, int64_t cols, int radius, const float* weights,
                   double boundary, int storage, uint32_t flags);
/* stencil_get_planes -- planes of a 3D plan (1 for a 2D plan): a field holds planes * rows * cols cells. */
int stencil_get_planes(const st_plan* plan, int64_t* planes);

/* stencil_plan_varcoef -- variable-coefficient (conservative) heat step, a
 * Jacobi update (Sec. II-C) whose five weights vary with position:
 *   u'(c) = u(c) + sum_{nb in N, W, E, S} kf * (u(nb) - u(c)),
 *   kf = (kappa(c) + kappa(nb)) / 2; at the grid edge kappa(nb) := kappa(c)
 *   and u(nb) := b.  FP32 order: acc = u(c); for nb in N, W, E, S:
 *   acc = fma(0.5f * (kappa(c) + kappa(nb)), u(nb) - u(c), acc).
 * FP32 storage only.  Errors as stencil_plan. */
int stencil_plan_varcoef(st_plan** out, int64_t rows, int64_t cols, double boundary, uint32_t flags);

/* stencil_destroy -- free a plan (host memory and any cached graph).  NULL is a no-op. */
int stencil_destroy(st_plan* plan);

/* stencil_set_blocking -- choose the temporal-blocking depth tb (steps per HBM
 * round trip, 1..16; up to 64 steps per halo swap for ST_VARIANT_RESIDENT) and the output tile (tile_x, tile_y) of the tiled
 * kernel; 0 keeps the current value.  The result is bitwise independent of
 * these choices.  Errors: ST_EINVAL (value out of range), ST_EUNSUPPORTED
 * (tile not instantiated; the supported set is listed by stencil_tiles()). */
int stencil_set_blocking(st_plan* plan, int tb, int tile_x, int tile_y);

/* kernel variants of the constant-weight sweep */
#define ST_VARIANT_TILED   0  /* one launch per pass, one tile per workgroup                    */
#define ST_VARIANT_STREAM  1  /* persistent workgroups; the next tile is copied into LDS by DMA
                                 while the current one computes (FP32, cols % 4 == 0)          */
#define ST_VARIANT_MARCH   2  /* each wavefront walks a column band down the grid, rows in a
                                 register ring, side columns by lane shifts; tb up to 8 / 6 /
                                 4 / 3 (star, r = 1 / 2 / 3 / 4) or 6 / 3 / 2 / 2 (box); the
                                 tile is ignored; any storage, width and alignment (four
                                 columns per lane: one vector access per lane and row when
                                 cols % 4 == 0 and the buffers are 16-byte aligned, else one
                                 element access per column)                                     */
#define ST_VARIANT_MARCH8  3  /* the same marching pass with eight columns per lane when
                                 cols % 8 == 0 and the buffers are 16-byte aligned (else as
                                 ST_VARIANT_MARCH); tb up to 8 / 4 / 3 / 2 (star) or
                                 3 / 2 / 2 / 1 (box)                                            */
#define ST_VARIANT_MARCH1  4  /* the marching pass with one column per lane (more, shorter
                                 tasks: for small grids); depths as ST_VARIANT_MARCH            */
#define ST_VARIANT_RESIDENT 5 /* the whole run in one cooperative launch: one workgroup per compute
                                 unit keeps its tile in LDS for every step and swaps an r*tb-deep
                                 halo with its eight neighbours every tb steps through global
                                 memory, gated by per-tile counters with bounded waits (the paper's
                                 PE-resident tiles and counter-gated halo swap, Sec. IV-B/C).  For
                                 grids whose tiles fit LDS (about 2048^2 and below at r = 1); tb
                                 up to what the tiles allow (each tile at least r*tb cells per
                                 side); constant halo only.  Synchronises nothing; a wait that runs
                                 out of polls ends the run early and is reported by
                                 stencil_resident_status                                         */

/* stencil_set_variant -- choose the kernel variant (bitwise the same results).  Errors:
 * ST_EINVAL (unknown value), ST_EUNSUPPORTED (streaming needs FP32 storage and cols % 4 == 0;
 * both need a constant-weight plan; or the current tb is deeper than the variant
 * allows: its LDS budget when streaming, the depths listed above when marching -- lower tb
 * first).  A streaming run whose buffers are not 16-byte aligned falls back to the tiled
 * kernels. */
int stencil_set_variant(st_plan* plan, int variant);
int stencil_get_variant(const st_plan* plan, int* variant);

#define ST_VARIANT_MFMA    6  /* the update as a dense contraction on the matrix cores: per 16 x 16
                                 output block and footprint row, a 16 x 32 window of the field times
                                 a banded 32 x 16 Toeplitz block of the weights
                                 (v_mfma_f32_16x16x32_bf16), every FP32 operand split exactly into
                                 three BF16 parts and the six products above 2^-24 relative summed
                                 in FP32.  One level per pass (tb = 1); FP32 storage, constant halo.
                                 NOT bitwise the canonical order: within FP32 rounding of it (the
                                 paper's tensor-core family, Sec. V, for MI355X).  The autotuner
                                 considers it only for plans created with ST_FLAG_ALLOW_MFMA     */

/* stencil_set_spin_limit -- resident variant: polls of a neighbour's counter (in total per tile
 * and epoch) before a wait gives up (default 2^22, seconds).  A give-up raises a flag that ends
 * every workgroup's run at its next wait, so the launch always completes; the output is then
 * unspecified and stencil_resident_status reports it.  Errors: ST_EINVAL (NULL plan, polls < 1). */
int stencil_set_spin_limit(st_plan* plan, int64_t polls);

/* stencil_resident_status -- after a resident run on `workspace`: status4[0] = 1 if a wait gave up
 * (else 0), then the workgroup, the epoch it waited for and the neighbour it waited on.
 * Synchronises `stream`.  Errors: ST_EINVAL, ST_ENOWS (workspace smaller than the run's), ST_EHIP. */
int stencil_resident_status(const st_plan* plan, const void* workspace, size_t ws_bytes, int* status4, void* stream);

/* stencil_set_march_segment -- marching variants: each wavefront computes about
 * `min_rows` output rows of its column band at least (0, the default: as many
 * (band, segment) tasks as the device holds wavefronts at once).  A segment
 * recomputes r (tb - 1) rows of the lower levels at either end, which on
 * small grids costs more than the idle SIMDs of fewer, longer tasks.  The
 * launch then lengthens the segment by fewer than 2r + 1 rows so that its row
 * loop fills whole unrolled groups.  The tasks that take the grid's edge checks
 * (the outer bands, and the segments within r tb rows of the top and bottom)
 * get proportionally shorter segments, so that every task takes about the same
 * time; a segment raised by min_rows keeps one length per band, except that
 * with a halo of +0 (whose side bands take no column checks) the top and
 * bottom rows still go to short segments.  Bitwise the same results; values
 * above rows act as rows.
 * stencil_autotune sets it.
 * Errors: ST_EINVAL (NULL plan, negative min_rows). */
int stencil_set_march_segment(st_plan* plan, int64_t min_rows);
int stencil_get_march_segment(const st_plan* plan, int64_t* min_rows);

/* ---- boundary rules --------------------------------------------------- */
#define ST_BC_CONST    0  /* the fixed halo value b of stencil_plan (the paper's zero halo, Sec. IV-A) */
#define ST_BC_PERIODIC 1  /* periodic: the cell outside the grid at (i, j) is u(i mod rows, j mod cols) */
#define ST_BC_FRAME    2  /* a fixed halo given by the caller, never updated                          */

/* stencil_set_boundary -- choose how the cells outside the grid are defined in every step of
 * the Jacobi update (Sec. II-C), beyond the paper's constant halo:
 *   ST_BC_CONST     the plan's halo value b (the default); `frame` must be NULL;
 *   ST_BC_PERIODIC  the grid wraps in both directions (a torus); `frame` must be NULL;
 *   ST_BC_FRAME     the r-deep ring around the grid holds the values of the device array
 *                   `frame` (storage type of the plan; caller-owned, read by every run, so it
 *                   must stay valid and unchanged while runs are enqueued).  Layout, in elements:
 *                   top strip r x (cols + 2r) (rows -r .. -1, columns -r .. cols+r-1), bottom strip
 *                   r x (cols + 2r) (rows rows .. rows+r-1), left strip rows x r (columns -r .. -1),
 *                   right strip rows x r (columns cols .. cols+r-1), each row-major, one after
 *                   the other: stencil_frame_elems() elements in all.
 * Periodic and framed plans run on the row-marching kernels only: the plan switches to
 * ST_VARIANT_MARCH unless it already uses a marching variant (with tb lowered to that variant's
 * limit), stencil_set_variant refuses the tiled and streaming variants, and the autotuner tries
 * marching candidates only.  Batches (stencil_batch_create) and the naive flag take constant
 * halos only.  stencil_norms' next-step mass is sum(W) * sum(u) on a periodic grid and NaN with a
 * frame.  Host-only.  Errors: ST_EINVAL (NULL plan, unknown kind, frame missing or given
 * wrongly, varcoef plan), ST_EUNSUPPORTED (a naive plan). */
int stencil_set_boundary(st_plan* plan, int kind, const void* frame);
int stencil_get_boundary(const st_plan* plan, int* kind);
/* stencil_frame_elems -- elements of the frame of ST_BC_FRAME: 2r (cols + 2r) + 2r rows. */
int stencil_frame_elems(const st_plan* plan, int64_t* elems);

/* stencil_get_dims -- the plan's rows, cols and storage type (ST_F32 / ST_BF16 / ST_F16); NULL
 * outputs are skipped.  A field of the plan occupies rows * cols * (4 or 2) bytes.  Host-only.
 * Errors: ST_EINVAL (NULL plan). */
int stencil_get_dims(const st_plan* plan, int64_t* rows, int64_t* cols, int* storage);

/* stencil_get_blocking -- read back the current (tb, tile_x, tile_y). */
int stencil_get_blocking(const st_plan* plan, int* tb, int* tile_x, int* tile_y);

/* stencil_tiles -- write up to `cap` supported (tile_x, tile_y) pairs into
 * `xy` (2 ints each) and their count into *n.  Host-only. */
int stencil_tiles(int* xy, int cap, int* n);

/* stencil_workspace_bytes -- minimum workspace for stencil_run(plan, ..., steps):
 * one extra field (rows*cols elements of the storage type) when the run takes
 * two or more passes, else 0; the resident variant needs one field (rounded up to 256 bytes)
 * plus 64 KiB of counters whenever steps >= 1.  Host-only. */
int stencil_workspace_bytes(const st_plan* plan, int64_t steps, size_t* bytes);

/* stencil_run -- advance `steps` Jacobi steps: out = S^steps(in).
 *   in, out     device fields of the plan's storage type; `in` is only read.
 *               They must not overlap (ST_EALIAS).  steps == 0 copies in->out.
 *   workspace   device scratch of at least stencil_workspace_bytes(steps)
 *               bytes (ST_ENOWS otherwise); its contents are clobbered.
 * The passes ping-pong between workspace and out so that the last pass writes
 * out.  Asynchronous on `stream`.  Varcoef plans use stencil_run_varcoef. */
int stencil_run(st_plan* plan, const void* in, void* out, int64_t steps, void* workspace,
                size_t ws_bytes, void* stream);

/* stencil_run_noalloc -- for callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same result
 * as stencil_run(plan, in, out, steps, ...), bitwise, with the ping-pong field taken from a static
 * device array of the library instead of a workspace.  That array is 64 MiB
 * (stencil_noalloc_max_bytes), enough for a grid of 16 Mi FP32 or 32 Mi 16-bit cells; each GPU the
 * library is loaded on holds its own copy until the process ends.  This entry point allocates
 * nothing: no hipMalloc/hipFree, no stream, no graph (a plan's ST_FLAG_GRAPH is ignored here: the
 * passes are enqueued directly on `stream`, which the caller may be capturing).  Every call on one
 * GPU shares that GPU's array: calls that overlap in time on one GPU (different streams, or host
 * threads) race and give undefined results -- order them on one stream.  The array needs no
 * clearing (every pass writes every cell it later reads).  Constant-weight plans only.
 * Errors: ST_EINVAL (NULL plan/in/out, negative steps, varcoef plan), ST_EALIAS (in/out overlap),
 * ST_EUNSUPPORTED (the run needs a ping-pong field larger than the static array: use stencil_run),
 * ST_EHIP. */
int stencil_run_noalloc(st_plan* plan, const void* in, void* out, int64_t steps, void* stream);
int stencil_noalloc_max_bytes(size_t* bytes);

/* stencil_run_varcoef -- the same for a varcoef plan; kappa is a device FP32
 * rows x cols diffusivity field (only read). */
int stencil_run_varcoef(st_plan* plan, const float* in, const float* kappa, float* out, int64_t steps,
                        void* workspace, size_t ws_bytes, void* stream);

/* stencil_norms_ws_bytes -- workspace bytes stencil_norms needs (partial sums). */
int stencil_norms_ws_bytes(const st_plan* plan, size_t* bytes);

/* stencil_norms -- FP64 reductions of a field (the host's periodic
 * convergence check of Sec. IV), written as 4 doubles to the DEVICE pointer
 * out4:
 *   out4[0] = sum (u - u_prev)^2     (0 when u_prev is NULL)  -- residual^2
 *   out4[1] = sum u^2                                        -- energy
 *   out4[2] = sum u                                          -- mass
 *   out4[3] = sum_j (u_j - b) S_j + b * rows*cols * sum(W)   -- mass of the next step,
 *             S_j = sum of the weights W_d whose source cell j - d lies in the grid.
 * Values are read in the plan's storage type and widened exactly.  The order
 * of summation is fixed (two-stage tree), so results are run-to-run bitwise
 * reproducible; it depends only on the grid shape and on whether both fields
 * start on a 16-byte (FP32) or 8-byte (16-bit) boundary with cols % 4 == 0
 * (four cells per load), not on the values.  Errors: ST_EINVAL, ST_ENOWS, ST_EHIP. */
int stencil_norms(const st_plan* plan, const void* u_prev, const void* u, double* out4, void* workspace,
                  size_t ws_bytes, void* stream);

/* stencil_autotune -- time every supported (variant, tb, tile) candidate on the caller's buffers
 * for `sample_steps` steps (one warm-up run, then the better of two timed runs) and keep the
 * fastest in the plan (variant, blocking and segment length).  Candidates: LDS tiles with tb in
 * {1, 2, 3, 4, 6, 8} within their LDS budget; marching with one, four and, when cols % 8 == 0,
 * eight columns per lane at every depth each offers, each depth above 1 also with segments of
 * at least 1/2 (when that is 2 rows or more), 1, 2, 4 and 8 x r (tb - 1) rows
 * (stencil_set_march_segment); the resident variant at swap depths {1, 2, 4, 8, 12, 16, 24, 32, 48}
 * where the grid's tiles allow them; the matrix-core variant only for plans created with
 * ST_FLAG_ALLOW_MFMA (periodic and framed plans: the marching variants only).
 * Clobbers out and workspace (which must be sized for sample_steps).  Writes
 * the chosen values to *tb_out, *tile_x_out, *tile_y_out when non-NULL.
 * Synchronises the stream.  Errors: as stencil_run; ST_EINVAL for a varcoef plan (see
 * stencil_autotune_varcoef). */
int stencil_autotune(st_plan* plan, const void* in, void* out, void* workspace, size_t ws_bytes,
                     int64_t sample_steps, int* tb_out, int* tile_x_out, int* tile_y_out, void* stream);

/* stencil_autotune_varcoef -- the same for a varcoef plan (the conservative heat step with the
 * diffusivity field `kappa`, device FP32 rows x cols, only read): times its LDS-tile kernel at
 * every tile of stencil_tiles() and tb in {1, 2, 3, 4, 6, 8} within the LDS budget and keeps the
 * fastest.  Errors: as stencil_run_varcoef; ST_EINVAL for a constant-weight plan. */
int stencil_autotune_varcoef(st_plan* plan, const float* in, const float* kappa, float* out, void* workspace,
                             size_t ws_bytes, int64_t sample_steps, int* tb_out, int* tile_x_out, int* tile_y_out,
                             void* stream);

/* stencil_solve_ws_bytes -- workspace stencil_solve needs for this check interval. */
int stencil_solve_ws_bytes(const st_plan* plan, int64_t check_every, size_t* bytes);

/* stencil_solve -- iterate to convergence with a periodic check (the host-side convergence
 * check between otherwise host-free iterations, paper Sec. IV): every `check_every` steps the
 * FP64 relative residual ||u_t - u_{t-1}||_2 / ||u_t||_2 of the last step is computed on the
 * device and read back; the loop stops once it is <= tol or after max_steps steps.  `out`
 * receives the last iterate, *steps_done the number of steps taken (a multiple of check_every
 * unless max_steps cut the last interval), *rel_residual the last residual.  The result is
 * bitwise the same as stencil_run(plan, in, out, *steps_done).  With a marching variant the
 * test itself runs on the device and raises a flag that turns the passes enqueued after
 * convergence into no-ops, so the host enqueues checks in chunks of 1, 2, 4, ... 64 and
 * synchronises once per chunk; other variants synchronise at every check.  The call returns
 * with the stream idle.  The workspace (stencil_solve_ws_bytes) holds the previous iterate,
 * stencil_run's ping-pong field, the reduction's partial sums and the device-side record.
 * Errors: as stencil_run; ST_EINVAL for a varcoef plan or bad counts. */
int stencil_solve(st_plan* plan, const void* in, void* out, int64_t max_steps, int64_t check_every, double tol,
                  int64_t* steps_done, double* rel_residual, void* workspace, size_t ws_bytes, void* stream);

/* ---- batched: many independent grids, one graph launch ------------------ */

/* stencil_batch_create -- group n plans (FP32, constant weights, r <= 3; each may differ in
 * shape, radius, footprint and weights) with their own step counts into one batch.
 * Grids that fit a workgroup's LDS together with their halo and a ping-pong copy stay
 * resident in LDS for all their steps (one workgroup per grid).  The others are tiled
 * (128 x 64 tiles) with their plan's temporal depth (lowered if the batch tile would not fit
 * the LDS budget); pass p of all tiled grids is one multi-grid kernel, and the passes follow
 * each other, so each tile's dependency on its neighbours' previous pass (the tiles' halo
 * swap, paper Sec. IV-B/C) is carried by the kernel boundary.  Steps == 0 is a copy.  The
 * plans must outlive the batch.  flags: ST_FLAG_GRAPH captures the whole run (resident
 * grids on a parallel branch) in one hipGraph replayed by every run.
 * Errors: ST_EINVAL, ST_EUNSUPPORTED, ST_ENOMEM. */
int stencil_batch_create(st_batch** out, int n, st_plan* const* plans, const int64_t* steps, uint32_t flags);

/* stencil_batch_workspace_bytes -- workspace for the batch: descriptor and queue tables and
 * one ping-pong field per tiled grid with two or more steps. */
int stencil_batch_workspace_bytes(const st_batch* batch, size_t* bytes);

/* stencil_run_batched -- outs[g] = S_g^{steps[g]}(ins[g]) for every grid g.
 * ins/outs are HOST arrays of n device pointers; no in/out pair may overlap (ST_EALIAS for a
 * grid's own pair; fields of different grids and the workspace must not overlap either).
 * Results are bitwise those of stencil_run on each grid.  Asynchronous on `stream`.
 * The descriptor tables are copied into the workspace (from a pinned host buffer the batch owns)
 * only when a pointer differs from the previous call's, and are reused as they are otherwise: the
 * workspace must keep its contents between calls of the same batch, or be passed at a different
 * address. */
int stencil_run_batched(st_batch* batch, const void* const* ins, void* const* outs, void* workspace,
                        size_t ws_bytes, void* stream);

/* stencil_batch_set_class -- set the engine (0 = LDS tiles, 1 = marching) and pass depth of one
 * stencil class (shape 0 = star, 1 = box; radius 1..3) of the batch by hand; results are bitwise
 * the same for every choice.  Tiles: depth 1..16, further capped per grid by what its tile fits
 * in LDS.  Marching: depth up to 8 / 6 / 4 (star, r = 1 / 2 / 3) or 6 / 3 / 2 (box).  Errors: ST_EINVAL,
 * ST_EUNSUPPORTED (depth out of range). */
int stencil_batch_set_class(st_batch* batch, int shape, int radius, int engine, int depth);

/* stencil_batch_set_segment -- marching engine: each wavefront of the class (shape, radius)
 * computes at least `min_rows` output rows of its band (0, the default: segments sized so that
 * the class's tasks about fill the device once, and at least 8 rows).  As for a single plan
 * (stencil_set_march_segment), longer segments recompute fewer rows of the lower levels and
 * re-read fewer input rows.  Bitwise the same results.  stencil_batch_autotune sets it.
 * stencil_batch_get_segment reads the segment length the class's marching launches use (0 when
 * the class runs on tiles or is absent).  Errors: ST_EINVAL (bad class, negative min_rows). */
int stencil_batch_set_segment(st_batch* batch, int shape, int radius, int64_t min_rows);
int stencil_batch_get_segment(const st_batch* batch, int shape, int radius, int64_t* rows);

/* stencil_batch_autotune -- pick, for each stencil class (shape, radius) of the grids that are
 * not LDS-resident, the engine and the depth of its passes: LDS tiles of 128 x 64 (one multi-grid
 * launch per pass for all tiled classes) with the depth capped at 1, 2, 3, 4, 6, 8, 12 or 16
 * (and by what each grid's tile fits in LDS), or marching (one wavefront per column band, four
 * columns per lane, any width and alignment; one chain of launches per class, the classes on
 * parallel branches of the graph) with every depth it offers (up to 8 / 6 / 4 levels for star
 * r = 1 / 2 / 3, 6 / 3 / 2 for box), each with the default segments and with segments 2, 4 and 8
 * times as long (stencil_batch_set_segment).  Coordinate descent: each
 * class in turn, every candidate timed on the whole batch run twice on the caller's buffers (outs
 * are overwritten; results are bitwise those of any other choice).  Writes the chosen depth and
 * engine (0 = tiles, 1 = marching) per class to tb_out[6] / engine_out[6] when non-NULL (star
 * r = 1, 2, 3, then box r = 1, 2, 3; 0 = class absent).  Synchronises the stream.  Errors: as
 * stencil_run_batched.  A new batch starts with every class on tiles at its plans' depths. */
int stencil_batch_autotune(st_batch* batch, const void* const* ins, void* const* outs, void* workspace,
                           size_t ws_bytes, int* tb_out, int* engine_out, void* stream);

/* stencil_batch_destroy -- free the batch (graph, pinned table).  NULL is a no-op. */
int stencil_batch_destroy(st_batch* batch);

/* ---- CNN surrogate ------------------------------------------------------ */
/* Network: 6 conv3x3 layers with zero "same" padding, channels
 * 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, bias on every layer, exact-erf GELU
 * after layers 1-5, and a residual output scaled by the field:
 *   s     = RMS of u0 over the field (FP64; s = 1 for an all-zero field)
 *   inv   = fp32(1 / s),  gain = fp32(2^-11 s)
 *   u_hat = u0 + gain * f(u0 * inv, (kappa - 0.125) / 0.075)
 * (the network sees the field in units of its size and predicts the K-step update in units of
 * 2^-11 of it).  Layer 1 runs on FP32 MFMA; layers 2-5 as BF16 MFMA implicit GEMMs with FP32
 * accumulation; layer 6 on BF16 MFMA over the BF16 activations with each FP32 weight split into a
 * BF16 pair (16 significant bits).  Activations are stored as BF16.
 *
 * Parameter buffer (device, FP32, SG_PARAM_COUNT floats), per layer l = 1..6:
 *   W_l as [ky][kx][ci][co] (3 x 3 x C_in x C_out), then b_l[C_out].
 * Optimiser state: Adam m and v, SG_PARAM_COUNT floats each, m then v. */
#define SG_PARAM_COUNT 37889

/* surrogate_create -- host-side model object (layer table, step counter). */
int surrogate_create(sg_model** out, uint32_t flags);
int surrogate_destroy(sg_model* m);

/* surrogate_param_bytes -- bytes of the parameter buffer (SG_PARAM_COUNT floats) and of the Adam
 * state (2 * SG_PARAM_COUNT floats); NULL outputs are skipped.  Host-only.  Errors: ST_EINVAL. */
int surrogate_param_bytes(const sg_model* m, size_t* params, size_t* optim_state);

/* surrogate_init -- seeded initialisation on the device: He-normal weights N(0, 2 / (9 C_in)) (the
 * last layer's scaled by 0.1, so that the untrained network starts near u_hat = u0), zero biases,
 * and zero Adam state (skipped when optim_state is NULL).  Weight i of the flat layout is
 * fp32(sd_l * z_i) with z_i the Box-Muller normal sqrt(-2 ln(1 - u1)) cos(2 pi u2), computed in
 * FP64 from u = (w >> 11) 2^-53 of the first two words w of Philox4x64-10 (Salmon et al., SC 2011)
 * at counter (i, 0, 0, 0) and key (seed, 0).  Asynchronous.  Errors: ST_EINVAL, ST_EHIP. */
int surrogate_init(sg_model* m, float* params, float* optim_state, uint64_t seed, void* stream);

/* surrogate_workspace_bytes -- device workspace for a batch of `batch` fields
 * of rows x cols: activations, pre-activations, gradients and partial sums. */
int surrogate_workspace_bytes(const sg_model* m, int batch, int64_t rows, int64_t cols, size_t* bytes);

/* surrogate_infer -- u_hat[b] = surrogate(u0[b], kappa[b]) for `batch`
 * fields of rows x cols (device FP32, contiguous one after another); each field's
 * scale constants (inv, gain) come from its own RMS.  Asynchronous.  Errors: ST_EINVAL, ST_ENOWS,
 * ST_EHIP. */
int surrogate_infer(sg_model* m, const float* params, const float* u0, const float* kappa, float* u_hat,
                      int batch, int64_t rows, int64_t cols, void* workspace, size_t ws_bytes, void* stream);

/* surrogate_loss_grad -- forward, masked MSE loss against `target`, and the
 * full backward pass:  loss = (1/n) sum_{b, i, j in mask_b} (u_hat - target)^2
 * where mask_b keeps rows [lo_hi[4b], lo_hi[4b+1]) x cols [lo_hi[4b+2],
 * lo_hi[4b+3]) of field b (lo_hi: HOST array of 4*batch ints, batch <= 64)
 * and n counts the kept cells of all fields.  Writes d loss / d params to
 * `grad` (SG_PARAM_COUNT floats) and the loss to the device double *loss.
 * `scale` (device, 2 * batch floats, nullable): each field's (inv, gain) pair (see
 * surrogate_field_scale); NULL takes them from each field's own RMS.  surrogate_train passes those
 * of the whole trajectory field each crop was cut from.  Deterministic (fixed-order reductions).
 * Asynchronous. */
int surrogate_loss_grad(sg_model* m, const float* params, const float* u0, const float* kappa,
                        const float* scale, const float* target, const int* lo_hi, int batch, int64_t rows,
                        int64_t cols, float* grad, double* loss, void* workspace, size_t ws_bytes, void* stream);

/* surrogate_field_scale -- the scale constants of n fields of rows x cols (device FP32, one after
 * another): scale[2b] = inv = fp32(1 / s), scale[2b + 1] = gain = fp32(2^-11 s), s = the RMS of
 * field b in FP64 (a fixed-order two-stage sum; s = 1 for an all-zero field).  For
 * surrogate_loss_grad's `scale` argument when the fields given there are crops of larger fields.
 * Workspace: n * 256 doubles.  Asynchronous.  Errors: ST_EINVAL, ST_ENOWS, ST_EHIP. */
int surrogate_field_scale(const float* u0, int n, int64_t rows, int64_t cols, float* scale, void* workspace,
                          size_t ws_bytes, void* stream);

/* surrogate_adam -- one Adam step (Kingma & Ba, Algorithm 1, bias-corrected)
 * on params with `grad`; `t` is the 1-based step index.  optim = m then v. */
int surrogate_adam(sg_model* m, float* params, const float* grad, float* optim, int t, float lr,
                   float beta1, float beta2, float eps, void* stream);

/* surrogate_synth_fields -- training-data synthesis on the GPU: for each of
 * `n` coefficient rows (host-drawn random numbers, FP32, 4*(16+8) per row:
 * 16 sine modes (p, q, a, -) then 8 cosine modes (kx, ky, b, phase)), write
 *   u0(i,j)    = sum a sin(p pi (i+1)/(rows+1)) sin(q pi (j+1)/(cols+1))
 *   kappa(i,j) = 0.125 + 0.075 * sum b cos(2 pi (kx j/cols + ky i/rows) + phase) / sum |b|
 * to u0_out / kappa_out (n fields each, device FP32).  Asynchronous. */
int surrogate_synth_fields(const float* coef, int n, int64_t rows, int64_t cols, float* u0_out,
                           float* kappa_out, void* stream);

/* surrogate_crop -- copy n crops of h x w at per-field offsets yx (device
 * int32 pairs) from fields of rows x cols: src -> dst.  Asynchronous. */
int surrogate_crop(const float* src, float* dst, const int* yx, int n, int64_t rows, int64_t cols,
                   int64_t h, int64_t w, void* stream);

/* surrogate_train -- the whole training loop on the device: the network learns to replace K
 * plain steps of the variable-coefficient heat stencil on trajectories that stencil generates.
 * For optimiser step s = 0 .. cfg->steps-1 and trajectory b = 0 .. cfg->batch-1 (index
 * i = s*batch + b):
 *   1. (u0, kappa) of rows x cols from coefficient row coef[i] (as surrogate_synth_fields);
 *   2. the target u_K = K steps of the plain varcoef stencil from u0 (an internal varcoef plan);
 *   3. crop x crop windows of u0, kappa and u_K at crop_yx[2i], crop_yx[2i+1] (row, col);
 *   4. masked MSE loss and gradient on the crops (surrogate_loss_grad); the mask drops the 6 cells
 *      next to a crop edge that cuts the grid (the network's receptive field), keeps domain edges;
 *      the step's loss goes to losses[s] (device doubles);
 *   5. one Adam step with t = step0 + s + 1 and the cosine schedule
 *      lr_s = lr (1 + cos(pi (step0 + s) / total_steps)) / 2.
 * The random numbers (coefficients, crop offsets) are inputs, and every reduction has a fixed
 * order, so training is deterministic: steps [0, a) then [a, n) in two calls (step0 = a in the
 * second) give bitwise the same params, optim and losses as one call over [0, n).
 * coef: device FP32, steps*batch rows of 96; crop_yx: HOST int32, 2*steps*batch.  Asynchronous
 * (the host only enqueues).  Errors: ST_EINVAL (bad config or offsets), ST_ENOWS, ST_EHIP. */
typedef struct sg_train_cfg {
    int64_t rows, cols;   /* trajectory grid */
    int64_t crop;         /* square crop side, <= rows and cols */
    int batch;            /* trajectories per optimiser step, 1 .. 64 */
    int K;                /* plain steps the network replaces, >= 1 */
    int64_t steps;        /* optimiser steps in this call */
    int64_t step0;        /* global index of the first of them */
    int64_t total_steps;  /* length of the cosine schedule, >= step0 + steps */
    float lr, beta1, beta2, eps;
} sg_train_cfg;
int surrogate_train_ws_bytes(const sg_model* m, const sg_train_cfg* cfg, size_t* bytes);
int surrogate_train(sg_model* m, float* params, float* optim, const float* coef, const int* crop_yx,
                    const sg_train_cfg* cfg, double* losses, void* workspace, size_t ws_bytes, void* stream);

/* surrogate_infer_checked -- the surrogate with the plain stencil as judge and fallback:
 * computes u_hat = surrogate(u0, kappa), judges it against K plain steps of the judge plan (a
 * varcoef plan of the same shape), and measures rel = ||u_hat - u_K|| / ||u_K|| in FP64 over
 *   SG_JUDGE_FULL   every cell: the plain stencil runs on the whole field;
 *   SG_JUDGE_PATCH  a 4 x 4 lattice of patches of min(64, rows) x min(64, cols) cells whose
 *                   origins are spread evenly over the grid (row origin of lattice row a:
 *                   ((rows - p) a + 1) / 3, integer division; columns alike), the first and last
 *                   at the edges.  Each patch's window, the patch dilated by K cells (its light
 *                   cone) and clipped to the grid, is copied edge to edge into a small "mosaic"
 *                   field, and K plain steps run on the mosaic only: every patch cell is exactly
 *                   the full-field result (a wrong neighbour across a window junction travels one
 *                   cell per step), at a fraction of the cost.  When the windows would cover more
 *                   than half of the grid's cells the whole field is judged instead.
 * If rel <= tol, out = u_hat; else out = u_K (the plain K-step result on the whole field, run
 * after the decision in PATCH mode) and *used_fallback = 1.  The surrogate result is never
 * accepted unjudged here.  Synchronises (to read the error).  Workspace:
 * surrogate_checked_ws_bytes (the surrogate's for one field, 3 fields, partial sums).
 * Errors: ST_EINVAL (NULL argument, judge not a varcoef plan of this shape, K < 0, tol < 0 or
 * NaN, unknown judge mode), ST_ENOWS, ST_EHIP. */
#define SG_JUDGE_FULL  0
#define SG_JUDGE_PATCH 1
int surrogate_checked_ws_bytes(const sg_model* m, int64_t rows, int64_t cols, size_t* bytes);
int surrogate_infer_checked(sg_model* m, const float* params, const float* u0, const float* kappa, float* out,
                            int64_t rows, int64_t cols, st_plan* judge, int64_t K, double tol, int judge_mode,
                            int* used_fallback, double* rel_err, void* workspace, size_t ws_bytes, void* stream);

/* ---- errors ------------------------------------------------------------- */
const char* stencil_strerror(int code);
const char* stencil_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MI355STENCIL_H */
