/*
 * Plain CPU oracle for iterated 2D Jacobi stencils.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never links or calls it, and it shares no code with the GPU path.
 *
 * Definition followed (paper Sec. II-C, Jacobi update equation; Sec. IV-A,
 * zero-padding / halo of depth r; Sec. IV-E, scalar loop that initialises the
 * accumulator with the centre product and then adds one weighted neighbour at
 * a time):
 *
 *   Extended field  ~u  on rows [-r, rows+r) x cols [-r, cols+r):
 *       ~u = u inside the grid, ~u = b (the fixed halo value) outside.
 *   One step, for every grid cell (i, j):
 *       u'(i,j) = sum_{dy,dx in [-r,r]} W[dy+r][dx+r] * ~u(i+dy, j+dx)
 *   The halo is never updated.  Steps are out-of-place (Jacobi).
 *
 * Weight layout: W is (2r+1)x(2r+1) row-major; W[dy+r][dx+r] multiplies the
 * value dy rows below and dx columns to the right (a correlation).
 *
 * Accumulation order ("canonical"): acc = W_centre * u(i,j); then, for the
 * remaining taps with W != 0 in row-major (dy, dx) order, acc += W * u.  In the
 * FP32 mode every "+=" is a single fused multiply-add (fmaf), so the FP32
 * result is fully specified bit for bit.  The FP64 mode uses separate multiply
 * and add (the build uses -ffp-contract=off) and is the accuracy reference.
 *
 * Compile: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* tap list: centre first, then the nonzero off-centre taps in row-major order */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;          /* number of off-centre taps */
    int dy[81], dx[81];
    double w64[81];
    float w32[81];
    double c64;
    float c32;
} taps_t;

static int build_taps_f64(int r, const double *W, taps_t *t) {
    if (r < 0 || r > 4) return ORC_EINVAL;
    int k = 2 * r + 1;
    t->n = 0;
    t->c64 = W[r * k + r];
    for (int dy = -r; dy <= r; dy++)
        for (int dx = -r; dx <= r; dx++) {
            if (dy == 0 && dx == 0) continue;
            double w = W[(dy + r) * k + (dx + r)];
            if (w == 0.0) continue;
            t->dy[t->n] = dy; t->dx[t->n] = dx; t->w64[t->n] = w; t->n++;
        }
    return ORC_OK;
}

static int build_taps_f32(int r, const float *W, taps_t *t) {
    if (r < 0 || r > 4) return ORC_EINVAL;
    int k = 2 * r + 1;
    t->n = 0;
    t->c32 = W[r * k + r];
    for (int dy = -r; dy <= r; dy++)
        for (int dx = -r; dx <= r; dx++) {
            if (dy == 0 && dx == 0) continue;
            float w = W[(dy + r) * k + (dx + r)];
            if (w == 0.0f) continue;
            t->dy[t->n] = dy; t->dx[t->n] = dx; t->w32[t->n] = w; t->n++;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* FP64 mode                                                                 */
/* ------------------------------------------------------------------------ */
/* One Jacobi step on extended buffers of pitch ep = cols + 2r; (i, j) index the
 * grid, the buffer origin is the halo corner (-r, -r). */
static void step_f64(int64_t rows, int64_t cols, int r, const taps_t *t,
                     const double *src, double *dst) {
    int64_t ep = cols + 2 * r;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; i++) {
        const double *srow = src + (i + r) * ep + r;
        double *drow = dst + (i + r) * ep + r;
        for (int64_t j = 0; j < cols; j++) {
            double acc = t->c64 * srow[j];
            for (int k = 0; k < t->n; k++)
                acc += t->w64[k] * srow[(int64_t)t->dy[k] * ep + j + t->dx[k]];
            drow[j] = acc;
        }
    }
}

static void fill_halo_f64(int64_t rows, int64_t cols, int r, double b, double *e) {
    int64_t ep = cols + 2 * r;
    for (int64_t i = 0; i < rows + 2 * r; i++)
        for (int64_t j = 0; j < ep; j++)
            if (i < r || i >= rows + r || j < r || j >= cols + r) e[i * ep + j] = b;
}

int oracle_stencil_f64(int64_t rows, int64_t cols, int r, const double *W, double b,
                       int64_t steps, const double *in, double *out) {
    if (rows < 0 || cols < 0 || steps < 0 || !W || (rows > 0 && cols > 0 && (!in || !out)))
        return ORC_EINVAL;
    taps_t t;
    if (build_taps_f64(r, W, &t)) return ORC_EINVAL;
    if (rows == 0 || cols == 0) return ORC_OK;
    int64_t ep = cols + 2 * r, n = (rows + 2 * r) * ep;
    double *a = (double *)malloc(sizeof(double) * n), *c = (double *)malloc(sizeof(double) * n);
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    fill_halo_f64(rows, cols, r, b, a);
    fill_halo_f64(rows, cols, r, b, c);
    for (int64_t i = 0; i < rows; i++) memcpy(a + (i + r) * ep + r, in + i * cols, sizeof(double) * cols);
    for (int64_t s = 0; s < steps; s++) {
        step_f64(rows, cols, r, &t, a, c);
        double *tmp = a; a = c; c = tmp;
    }
    for (int64_t i = 0; i < rows; i++) memcpy(out + i * cols, a + (i + r) * ep + r, sizeof(double) * cols);
    free(a); free(c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* FP32-canonical mode                                                       */
/* ------------------------------------------------------------------------ */
static void step_f32(int64_t rows, int64_t cols, int r, const taps_t *t,
                     const float *src, float *dst) {
    int64_t ep = cols + 2 * r;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; i++) {
        const float *srow = src + (i + r) * ep + r;
        float *drow = dst + (i + r) * ep + r;
        for (int64_t j = 0; j < cols; j++) {
            float acc = t->c32 * srow[j];
            for (int k = 0; k < t->n; k++)
                acc = fmaf(t->w32[k], srow[(int64_t)t->dy[k] * ep + j + t->dx[k]], acc);
            drow[j] = acc;
        }
    }
}

static void fill_halo_f32(int64_t rows, int64_t cols, int r, float b, float *e) {
    int64_t ep = cols + 2 * r;
    for (int64_t i = 0; i < rows + 2 * r; i++)
        for (int64_t j = 0; j < ep; j++)
            if (i < r || i >= rows + r || j < r || j >= cols + r) e[i * ep + j] = b;
}

int oracle_stencil_f32(int64_t rows, int64_t cols, int r, const float *W, float b,
                       int64_t steps, const float *in, float *out) {
    if (rows < 0 || cols < 0 || steps < 0 || !W || (rows > 0 && cols > 0 && (!in || !out)))
        return ORC_EINVAL;
    taps_t t;
    if (build_taps_f32(r, W, &t)) return ORC_EINVAL;
    if (rows == 0 || cols == 0) return ORC_OK;
    int64_t ep = cols + 2 * r, n = (rows + 2 * r) * ep;
    float *a = (float *)malloc(sizeof(float) * n), *c = (float *)malloc(sizeof(float) * n);
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    fill_halo_f32(rows, cols, r, b, a);
    fill_halo_f32(rows, cols, r, b, c);
    for (int64_t i = 0; i < rows; i++) memcpy(a + (i + r) * ep + r, in + i * cols, sizeof(float) * cols);
    for (int64_t s = 0; s < steps; s++) {
        step_f32(rows, cols, r, &t, a, c);
        float *tmp = a; a = c; c = tmp;
    }
    for (int64_t i = 0; i < rows; i++) memcpy(out + i * cols, a + (i + r) * ep + r, sizeof(float) * cols);
    free(a); free(c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 16-bit storage emulation: the field is stored as BF16 or FP16 after every  */
/* step; the arithmetic is the FP32-canonical step.                          */
/* ------------------------------------------------------------------------ */
typedef union { float f; uint32_t u; } fbits;

/* BF16 = the upper 16 bits of an IEEE single; round to nearest, ties to even. */
uint16_t oracle_f32_to_bf16(float x) {
    fbits v; v.f = x;
    if ((v.u & 0x7f800000u) == 0x7f800000u && (v.u & 0x007fffffu))   /* NaN: keep quiet NaN */
        return (uint16_t)((v.u >> 16) | 0x0040u);
    uint32_t lsb = (v.u >> 16) & 1u;
    uint32_t rounded = v.u + 0x7fffu + lsb;
    return (uint16_t)(rounded >> 16);
}

float oracle_bf16_to_f32(uint16_t h) { fbits v; v.u = (uint32_t)h << 16; return v.f; }

/* IEEE binary16 (1-5-10), round to nearest even, with subnormals and overflow
 * to infinity.  Written from the format definition: value = (-1)^s 2^(e-15)
 * (1 + m/1024) for 1 <= e <= 30, 2^-14 (m/1024) for e = 0. */
uint16_t oracle_f32_to_f16(float x) {
    fbits v; v.f = x;
    uint32_t sign = (v.u >> 16) & 0x8000u;
    uint32_t ax = v.u & 0x7fffffffu;
    if (ax >= 0x7f800000u) /* inf or NaN */
        return (uint16_t)(sign | 0x7c00u | (ax > 0x7f800000u ? 0x200u : 0u));
    if (ax < 0x00800000u)  /* FP32 subnormal: |x| < 2^-126, far below half the FP16 quantum */
        return (uint16_t)sign;
    int e = (int)(ax >> 23) - 127;               /* x = mant * 2^(e-23) */
    uint32_t mant = (ax & 0x7fffffu) | 0x800000u;
    if (e > 15) return (uint16_t)(sign | 0x7c00u);   /* overflow */
    /* FP16 quantum (value of one unit in the last place): 2^(e-10) for a
     * normal result (e >= -14), 2^-24 for a subnormal one.  shift = number of
     * low significand bits that fall below the quantum. */
    int shift = (e >= -14) ? 13 : (-1 - e);
    if (shift > 25) return (uint16_t)sign;       /* below a quarter quantum */
    uint32_t kept = mant >> shift;
    uint32_t rem = mant & ((1u << shift) - 1u);
    uint32_t half = 1u << (shift - 1);
    if (rem > half || (rem == half && (kept & 1u))) kept++;
    uint32_t res;
    if (e >= -14) {
        /* biased exponent e+15 and fraction kept-1024; kept == 2048 carries into the exponent */
        res = ((uint32_t)(e + 15) << 10) + kept - 0x400u;
        if (res >= 0x7c00u) return (uint16_t)(sign | 0x7c00u);
    } else {
        res = kept;  /* subnormal; kept == 1024 is exactly the smallest normal's encoding */
    }
    return (uint16_t)(sign | res);
}

float oracle_f16_to_f32(uint16_t h) {
    uint32_t sign = (h & 0x8000u) ? 1u : 0u;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    float v;
    if (e == 0) v = ldexpf((float)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexpf((float)(m + 1024), e - 25);
    return sign ? -v : v;
}

static float lowp_load(int dtype, uint16_t h) {
    return dtype == 1 ? oracle_bf16_to_f32(h) : oracle_f16_to_f32(h);
}
static uint16_t lowp_store(int dtype, float x) {
    return dtype == 1 ? oracle_f32_to_bf16(x) : oracle_f32_to_f16(x);
}

/* dtype: 1 = BF16, 2 = FP16.  b is rounded to the storage type like any stored value. */
int oracle_stencil_lowp(int dtype, int64_t rows, int64_t cols, int r, const float *W, float b,
                        int64_t steps, const uint16_t *in, uint16_t *out) {
    if ((dtype != 1 && dtype != 2) || rows < 0 || cols < 0 || steps < 0 || !W ||
        (rows > 0 && cols > 0 && (!in || !out)))
        return ORC_EINVAL;
    taps_t t;
    if (build_taps_f32(r, W, &t)) return ORC_EINVAL;
    if (rows == 0 || cols == 0) return ORC_OK;
    float bq = lowp_load(dtype, lowp_store(dtype, b));
    int64_t ep = cols + 2 * r, n = (rows + 2 * r) * ep;
    float *a = (float *)malloc(sizeof(float) * n), *c = (float *)malloc(sizeof(float) * n);
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    fill_halo_f32(rows, cols, r, bq, a);
    fill_halo_f32(rows, cols, r, bq, c);
    for (int64_t i = 0; i < rows; i++)
        for (int64_t j = 0; j < cols; j++) a[(i + r) * ep + r + j] = lowp_load(dtype, in[i * cols + j]);
    for (int64_t s = 0; s < steps; s++) {
        step_f32(rows, cols, r, &t, a, c);
        /* store to the 16-bit format and read back: the value every later step sees */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < rows; i++)
            for (int64_t j = 0; j < cols; j++) {
                float *p = c + (i + r) * ep + r + j;
                *p = lowp_load(dtype, lowp_store(dtype, *p));
            }
        float *tmp = a; a = c; c = tmp;
    }
    for (int64_t i = 0; i < rows; i++)
        for (int64_t j = 0; j < cols; j++) out[i * cols + j] = lowp_store(dtype, a[(i + r) * ep + r + j]);
    free(a); free(c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Light-cone patch (FP64): the exact result on a sub-rectangle after T steps */
/* of a full-size grid, computing only the cells the patch depends on.       */
/* ------------------------------------------------------------------------ */
/* After T steps, patch cells depend only on inputs within r*T of the patch
 * (Jacobi dependency cone).  Working window = patch dilated by r*T, clipped to
 * the grid.  Step s (0-based) updates the patch dilated by r*(T-1-s), clipped;
 * every in-grid cell outside the current update region is poisoned with NaN,
 * so any read the cone argument says cannot happen would show up as NaN. */
int oracle_stencil_patch_f64(int64_t rows, int64_t cols, int r, const double *W, double b,
                             int64_t steps, const float *in_full,
                             int64_t py0, int64_t px0, int64_t ph, int64_t pw, double *out) {
    if (rows <= 0 || cols <= 0 || steps < 0 || !W || !in_full || !out || ph <= 0 || pw <= 0 ||
        py0 < 0 || px0 < 0 || py0 + ph > rows || px0 + pw > cols)
        return ORC_EINVAL;
    taps_t t;
    if (build_taps_f64(r, W, &t)) return ORC_EINVAL;
    int64_t reach = (int64_t)r * steps;
    int64_t wy0 = py0 - reach < 0 ? 0 : py0 - reach;
    int64_t wx0 = px0 - reach < 0 ? 0 : px0 - reach;
    int64_t wy1 = py0 + ph + reach > rows ? rows : py0 + ph + reach;
    int64_t wx1 = px0 + pw + reach > cols ? cols : px0 + pw + reach;
    int64_t wh = wy1 - wy0, ww = wx1 - wx0;
    int64_t ep = ww + 2 * r, n = (wh + 2 * r) * ep;
    double *a = (double *)malloc(sizeof(double) * n), *c = (double *)malloc(sizeof(double) * n);
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    /* extended window: grid coordinates (wy0 - r + ei, wx0 - r + ej) */
    for (int64_t ei = 0; ei < wh + 2 * r; ei++)
        for (int64_t ej = 0; ej < ep; ej++) {
            int64_t gi = wy0 - r + ei, gj = wx0 - r + ej;
            double v;
            if (gi < 0 || gi >= rows || gj < 0 || gj >= cols) v = b;          /* true halo */
            else if (ei < r || ei >= wh + r || ej < r || ej >= ww + r) v = NAN; /* outside the cone */
            else v = (double)in_full[gi * cols + gj];
            a[ei * ep + ej] = v;
            c[ei * ep + ej] = (gi < 0 || gi >= rows || gj < 0 || gj >= cols) ? b : NAN;
        }
    /* Step s is computed on the cone region R_s (the patch grown by r*(steps-1-s), clipped to the
     * grid).  The destination buffer was last written two steps earlier over R_{s-2}, which is R_s
     * grown by 2r: that band is first poisoned with NaN, so a read that leaves the cone shows up.
     * Per cell the order is the centre product, then one add per tap in row-major order. */
    for (int64_t s = 0; s < steps; s++) {
        int64_t m = (int64_t)r * (steps - 1 - s), q = m + 2 * (int64_t)r;
        int64_t ry0 = py0 - m < 0 ? 0 : py0 - m, rx0 = px0 - m < 0 ? 0 : px0 - m;
        int64_t ry1 = py0 + ph + m > rows ? rows : py0 + ph + m;
        int64_t rx1 = px0 + pw + m > cols ? cols : px0 + pw + m;
        int64_t zy0 = py0 - q < wy0 ? wy0 : py0 - q, zx0 = px0 - q < wx0 ? wx0 : px0 - q;
        int64_t zy1 = py0 + ph + q > wy1 ? wy1 : py0 + ph + q;
        int64_t zx1 = px0 + pw + q > wx1 ? wx1 : px0 + pw + q;
#pragma omp parallel for schedule(static)
        for (int64_t gi = zy0; gi < zy1; gi++) {
            double *drow = c + (gi - wy0 + r) * ep + r - wx0;
            const double *srow = a + (gi - wy0 + r) * ep + r - wx0;
            for (int64_t gj = zx0; gj < zx1; gj++) drow[gj] = NAN;
            if (gi < ry0 || gi >= ry1) continue;
            for (int64_t gj = rx0; gj < rx1; gj++) drow[gj] = t.c64 * srow[gj];
            for (int k = 0; k < t.n; k++) {
                const double w = t.w64[k];
                const double *tap = srow + (int64_t)t.dy[k] * ep + t.dx[k];
                for (int64_t gj = rx0; gj < rx1; gj++) drow[gj] += w * tap[gj];
            }
        }
        double *tmp = a; a = c; c = tmp;
    }
    for (int64_t i = 0; i < ph; i++)
        for (int64_t j = 0; j < pw; j++)
            out[i * pw + j] = a[(py0 + i - wy0 + r) * ep + (px0 + j - wx0 + r)];
    free(a); free(c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Variable-coefficient (conservative) heat step.                            */
/*   u'(c) = u(c) + sum_{nb in N, W, E, S} kf * (u(nb) - u(c)),              */
/*   kf = (kappa(c) + kappa(nb)) / 2;  at a face on the grid edge            */
/*   kappa(nb) := kappa(c) and u(nb) := b.                                   */
/* A Jacobi update (Sec. II-C) whose 5 weights vary with position.  FP32     */
/* order: start from u(c); for nb in N, W, E, S (row-major order of the      */
/* offsets): d = u(nb) - u(c); kf = 0.5f * (kappa(c) + kappa(nb));           */
/* acc = fmaf(kf, d, acc).                                                   */
/* ------------------------------------------------------------------------ */
int oracle_varcoef_f64(int64_t rows, int64_t cols, double b, int64_t steps,
                       const double *kappa, const double *in, double *out) {
    if (rows < 0 || cols < 0 || steps < 0 || (rows > 0 && cols > 0 && (!kappa || !in || !out))) return ORC_EINVAL;
    if (rows == 0 || cols == 0) return ORC_OK;
    int64_t n = rows * cols;
    double *a = (double *)malloc(sizeof(double) * n), *c = (double *)malloc(sizeof(double) * n);
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    memcpy(a, in, sizeof(double) * n);
    static const int DY[4] = {-1, 0, 0, 1}, DX[4] = {0, -1, 1, 0};
    for (int64_t s = 0; s < steps; s++) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < rows; i++)
            for (int64_t j = 0; j < cols; j++) {
                double uc = a[i * cols + j], kc = kappa[i * cols + j], acc = uc;
                for (int k = 0; k < 4; k++) {
                    int64_t ni = i + DY[k], nj = j + DX[k];
                    int inside = ni >= 0 && ni < rows && nj >= 0 && nj < cols;
                    double un = inside ? a[ni * cols + nj] : b;
                    double kn = inside ? kappa[ni * cols + nj] : kc;
                    acc += 0.5 * (kc + kn) * (un - uc);
                }
                c[i * cols + j] = acc;
            }
        double *tmp = a; a = c; c = tmp;
    }
    memcpy(out, a, sizeof(double) * n);
    free(a); free(c);
    return ORC_OK;
}

int oracle_varcoef_f32(int64_t rows, int64_t cols, float b, int64_t steps,
                       const float *kappa, const float *in, float *out) {
    if (rows < 0 || cols < 0 || steps < 0 || (rows > 0 && cols > 0 && (!kappa || !in || !out))) return ORC_EINVAL;
    if (rows == 0 || cols == 0) return ORC_OK;
    int64_t n = rows * cols;
    float *a = (float *)malloc(sizeof(float) * n), *c = (float *)malloc(sizeof(float) * n);
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    memcpy(a, in, sizeof(float) * n);
    static const int DY[4] = {-1, 0, 0, 1}, DX[4] = {0, -1, 1, 0};
    for (int64_t s = 0; s < steps; s++) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < rows; i++)
            for (int64_t j = 0; j < cols; j++) {
                float uc = a[i * cols + j], kc = kappa[i * cols + j], acc = uc;
                for (int k = 0; k < 4; k++) {
                    int64_t ni = i + DY[k], nj = j + DX[k];
                    int inside = ni >= 0 && ni < rows && nj >= 0 && nj < cols;
                    float un = inside ? a[ni * cols + nj] : b;
                    float kn = inside ? kappa[ni * cols + nj] : kc;
                    float kf = 0.5f * (kc + kn);
                    acc = fmaf(kf, un - uc, acc);
                }
                c[i * cols + j] = acc;
            }
        float *tmp = a; a = c; c = tmp;
    }
    memcpy(out, a, sizeof(float) * n);
    free(a); free(c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* array forms of the 16-bit conversions (for tests and input preparation)   */
/* ------------------------------------------------------------------------ */
void oracle_f32_to_bf16_array(int64_t n, const float *in, uint16_t *out) {
    for (int64_t i = 0; i < n; i++) out[i] = oracle_f32_to_bf16(in[i]);
}
void oracle_bf16_to_f32_array(int64_t n, const uint16_t *in, float *out) {
    for (int64_t i = 0; i < n; i++) out[i] = oracle_bf16_to_f32(in[i]);
}
void oracle_f32_to_f16_array(int64_t n, const float *in, uint16_t *out) {
    for (int64_t i = 0; i < n; i++) out[i] = oracle_f32_to_f16(in[i]);
}
void oracle_f16_to_f32_array(int64_t n, const uint16_t *in, float *out) {
    for (int64_t i = 0; i < n; i++) out[i] = oracle_f16_to_f32(in[i]);
}

/* ------------------------------------------------------------------------ */
/* Other boundary rules for the extended field ~u (the paper uses the zero    */
/* halo of Sec. IV-A only; these are the library's further boundary modes):   */
/*   bc = 1  periodic: ~u(i, j) = u(i mod rows, j mod cols) -- the halo is    */
/*           refreshed from the grid before every step;                      */
/*   bc = 2  fixed halo frame: the r-deep ring around the grid holds values   */
/*           given by the caller and is never updated.  Frame layout, in      */
/*           elements: top strip r x (cols + 2r) (rows -r..-1, columns        */
/*           -r..cols+r-1), bottom strip r x (cols + 2r) (rows rows..rows+r-1),*/
/*           left strip rows x r (columns -r..-1), right strip rows x r        */
/*           (columns cols..cols+r-1), each row-major, one after another.     */
/* ------------------------------------------------------------------------ */
static int64_t wrap_idx(int64_t i, int64_t n) { int64_t m = i % n; return m < 0 ? m + n : m; }

/* index into the frame of the out-of-grid cell (i, j), |i|, |j| within r of the grid */
static int64_t frame_index(int64_t rows, int64_t cols, int r, int64_t i, int64_t j) {
    const int64_t wf = cols + 2 * r;
    if (i < 0) return (i + r) * wf + (j + r);
    if (i >= rows) return (int64_t)r * wf + (i - rows) * wf + (j + r);
    if (j < 0) return 2 * (int64_t)r * wf + i * r + (j + r);
    return 2 * (int64_t)r * wf + rows * r + i * r + (j - cols);
}

int64_t oracle_frame_elems(int64_t rows, int64_t cols, int r) {
    return 2 * (int64_t)r * (cols + 2 * r) + 2 * (int64_t)r * rows;
}

#define ORC_BC_FILL(T)                                                                          \
    static void bc_fill_##T(int bc, int64_t rows, int64_t cols, int r, const T *frame, T *e) {   \
        int64_t ep = cols + 2 * r;                                                                \
        for (int64_t i = -r; i < rows + r; i++)                                                   \
            for (int64_t j = -r; j < cols + r; j++) {                                             \
                if (i >= 0 && i < rows && j >= 0 && j < cols) continue;                           \
                T v = bc == 1 ? e[(wrap_idx(i, rows) + r) * ep + wrap_idx(j, cols) + r]            \
                              : frame[frame_index(rows, cols, r, i, j)];                          \
                e[(i + r) * ep + (j + r)] = v;                                                    \
            }                                                                                     \
    }
ORC_BC_FILL(double)
ORC_BC_FILL(float)

int oracle_stencil_bc_f64(int bc, int64_t rows, int64_t cols, int r, const double *W, const double *frame,
                          int64_t steps, const double *in, double *out) {
    if ((bc != 1 && bc != 2) || rows < 1 || cols < 1 || steps < 0 || !W || !in || !out || (bc == 2 && !frame))
        return ORC_EINVAL;
    taps_t t;
    if (build_taps_f64(r, W, &t)) return ORC_EINVAL;
    int64_t ep = cols + 2 * r, n = (rows + 2 * r) * ep;
    double *a = (double *)calloc(n, sizeof(double)), *c = (double *)calloc(n, sizeof(double));
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    for (int64_t i = 0; i < rows; i++) memcpy(a + (i + r) * ep + r, in + i * cols, sizeof(double) * cols);
    if (bc == 2) { bc_fill_double(2, rows, cols, r, frame, a); bc_fill_double(2, rows, cols, r, frame, c); }
    for (int64_t s = 0; s < steps; s++) {
        if (bc == 1) bc_fill_double(1, rows, cols, r, frame, a);
        step_f64(rows, cols, r, &t, a, c);
        double *tmp = a; a = c; c = tmp;
    }
    for (int64_t i = 0; i < rows; i++) memcpy(out + i * cols, a + (i + r) * ep + r, sizeof(double) * cols);
    free(a); free(c);
    return ORC_OK;
}

int oracle_stencil_bc_f32(int bc, int64_t rows, int64_t cols, int r, const float *W, const float *frame,
                          int64_t steps, const float *in, float *out) {
    if ((bc != 1 && bc != 2) || rows < 1 || cols < 1 || steps < 0 || !W || !in || !out || (bc == 2 && !frame))
        return ORC_EINVAL;
    taps_t t;
    if (build_taps_f32(r, W, &t)) return ORC_EINVAL;
    int64_t ep = cols + 2 * r, n = (rows + 2 * r) * ep;
    float *a = (float *)calloc(n, sizeof(float)), *c = (float *)calloc(n, sizeof(float));
    if (!a || !c) { free(a); free(c); return ORC_ENOMEM; }
    for (int64_t i = 0; i < rows; i++) memcpy(a + (i + r) * ep + r, in + i * cols, sizeof(float) * cols);
    if (bc == 2) { bc_fill_float(2, rows, cols, r, frame, a); bc_fill_float(2, rows, cols, r, frame, c); }
    for (int64_t s = 0; s < steps; s++) {
        if (bc == 1) bc_fill_float(1, rows, cols, r, frame, a);
        step_f32(rows, cols, r, &t, a, c);
        float *tmp = a; a = c; c = tmp;
    }
    for (int64_t i = 0; i < rows; i++) memcpy(out + i * cols, a + (i + r) * ep + r, sizeof(float) * cols);
    free(a); free(c);
    return ORC_OK;
}

/* 16-bit storage with a periodic or framed boundary; the frame holds 16-bit values */
int oracle_stencil_bc_lowp(int dtype, int bc, int64_t rows, int64_t cols, int r, const float *W,
                           const uint16_t *frame, int64_t steps, const uint16_t *in, uint16_t *out) {
    if ((dtype != 1 && dtype != 2) || (bc != 1 && bc != 2) || rows < 1 || cols < 1 || steps < 0 || !W || !in ||
        !out || (bc == 2 && !frame))
        return ORC_EINVAL;
    taps_t t;
    if (build_taps_f32(r, W, &t)) return ORC_EINVAL;
    int64_t ep = cols + 2 * r, n = (rows + 2 * r) * ep, nf = oracle_frame_elems(rows, cols, r);
    float *a = (float *)calloc(n, sizeof(float)), *c = (float *)calloc(n, sizeof(float));
    float *fr = (float *)calloc(nf > 0 ? nf : 1, sizeof(float));
    if (!a || !c || !fr) { free(a); free(c); free(fr); return ORC_ENOMEM; }
    if (bc == 2)
        for (int64_t k = 0; k < nf; k++) fr[k] = lowp_load(dtype, frame[k]);
    for (int64_t i = 0; i < rows; i++)
        for (int64_t j = 0; j < cols; j++) a[(i + r) * ep + r + j] = lowp_load(dtype, in[i * cols + j]);
    if (bc == 2) { bc_fill_float(2, rows, cols, r, fr, a); bc_fill_float(2, rows, cols, r, fr, c); }
    for (int64_t s = 0; s < steps; s++) {
        if (bc == 1) bc_fill_float(1, rows, cols, r, fr, a);
        step_f32(rows, cols, r, &t, a, c);
        for (int64_t i = 0; i < rows; i++)
            for (int64_t j = 0; j < cols; j++) {
                float *p = c + (i + r) * ep + r + j;
                *p = lowp_load(dtype, lowp_store(dtype, *p));
            }
        float *tmp = a; a = c; c = tmp;
    }
    for (int64_t i = 0; i < rows; i++)
        for (int64_t j = 0; j < cols; j++) out[i * cols + j] = lowp_store(dtype, a[(i + r) * ep + r + j]);
    free(a); free(c); free(fr);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 3D: the same Jacobi update on a planes x rows x cols grid with a constant */
/* halo b of depth r:                                                        */
/*   u'(k,i,j) = sum_{dz,dy,dx in [-r,r]} W[dz+r][dy+r][dx+r] ~u(k+dz,i+dy,j+dx) */
/* Canonical FP32 order: the centre product, then one fmaf per nonzero tap in */
/* row-major (dz, dy, dx) order.                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;                       /* off-centre taps with a nonzero weight */
    int dz[729], dy[729], dx[729];
    int q[729];                  /* index of each tap's weight in W */
    int centre;
} taps3_t;

static int build_taps3(int r, const double *W, taps3_t *t) {
    if (r < 1 || r > 4) return ORC_EINVAL;
    int k = 2 * r + 1;
    t->n = 0;
    t->centre = (r * k + r) * k + r;
    for (int dz = -r; dz <= r; dz++)
        for (int dy = -r; dy <= r; dy++)
            for (int dx = -r; dx <= r; dx++) {
                int q = ((dz + r) * k + (dy + r)) * k + (dx + r);
                if ((dz == 0 && dy == 0 && dx == 0) || W[q] == 0.0) continue;
                t->dz[t->n] = dz; t->dy[t->n] = dy; t->dx[t->n] = dx; t->q[t->n] = q;
                t->n++;
            }
    return ORC_OK;
}

/* FP64: weights promoted from the FP32 ones the caller passes as doubles; separate mul and add */
int oracle_stencil3d_f64(int64_t planes, int64_t rows, int64_t cols, int r, const double *W, double b,
                         int64_t steps, const double *in, double *out) {
    if (planes < 1 || rows < 1 || cols < 1 || steps < 0 || !W || !in || !out) return ORC_EINVAL;
    taps3_t *t = (taps3_t *)malloc(sizeof(taps3_t));
    if (!t) return ORC_ENOMEM;
    if (build_taps3(r, W, t)) { free(t); return ORC_EINVAL; }
    int64_t ep = cols + 2 * r, eq = (rows + 2 * r) * ep, n = (planes + 2 * r) * eq;
    double *a = (double *)malloc(sizeof(double) * n), *c = (double *)malloc(sizeof(double) * n);
    if (!a || !c) { free(a); free(c); free(t); return ORC_ENOMEM; }
    for (int64_t q = 0; q < n; q++) a[q] = c[q] = b;
    for (int64_t k = 0; k < planes; k++)
        for (int64_t i = 0; i < rows; i++)
            memcpy(a + (k + r) * eq + (i + r) * ep + r, in + (k * rows + i) * cols, sizeof(double) * cols);
    for (int64_t s = 0; s < steps; s++) {
#pragma omp parallel for schedule(static)
        for (int64_t ki = 0; ki < planes * rows; ki++) {
            int64_t k = ki / rows, i = ki % rows;
            const double *src = a + (k + r) * eq + (i + r) * ep + r;
            double *dst = c + (k + r) * eq + (i + r) * ep + r;
            for (int64_t j = 0; j < cols; j++) {
                double acc = W[t->centre] * src[j];
                for (int q = 0; q < t->n; q++)
                    acc += W[t->q[q]] * src[(int64_t)t->dz[q] * eq + (int64_t)t->dy[q] * ep + j + t->dx[q]];
                dst[j] = acc;
            }
        }
        double *tmp = a; a = c; c = tmp;
    }
    for (int64_t k = 0; k < planes; k++)
        for (int64_t i = 0; i < rows; i++)
            memcpy(out + (k * rows + i) * cols, a + (k + r) * eq + (i + r) * ep + r, sizeof(double) * cols);
    free(a); free(c); free(t);
    return ORC_OK;
}

/* FP32-canonical: the centre product, then fmaf per nonzero tap in row-major (dz, dy, dx) order */
int oracle_stencil3d_f32(int64_t planes, int64_t rows, int64_t cols, int r, const float *W, float b,
                         int64_t steps, const float *in, float *out) {
    if (planes < 1 || rows < 1 || cols < 1 || steps < 0 || !W || !in || !out || r < 1 || r > 4) return ORC_EINVAL;
    int kk = 2 * r + 1;
    double W64[729];
    for (int q = 0; q < kk * kk * kk; q++) W64[q] = W[q];
    taps3_t *t = (taps3_t *)malloc(sizeof(taps3_t));
    if (!t) return ORC_ENOMEM;
    if (build_taps3(r, W64, t)) { free(t); return ORC_EINVAL; }
    int64_t ep = cols + 2 * r, eq = (rows + 2 * r) * ep, n = (planes + 2 * r) * eq;
    float *a = (float *)malloc(sizeof(float) * n), *c = (float *)malloc(sizeof(float) * n);
    if (!a || !c) { free(a); free(c); free(t); return ORC_ENOMEM; }
    for (int64_t q = 0; q < n; q++) a[q] = c[q] = b;
    for (int64_t k = 0; k < planes; k++)
        for (int64_t i = 0; i < rows; i++)
            memcpy(a + (k + r) * eq + (i + r) * ep + r, in + (k * rows + i) * cols, sizeof(float) * cols);
    for (int64_t s = 0; s < steps; s++) {
#pragma omp parallel for schedule(static)
        for (int64_t ki = 0; ki < planes * rows; ki++) {
            int64_t k = ki / rows, i = ki % rows;
            const float *src = a + (k + r) * eq + (i + r) * ep + r;
            float *dst = c + (k + r) * eq + (i + r) * ep + r;
            for (int64_t j = 0; j < cols; j++) {
                float acc = W[t->centre] * src[j];
                for (int q = 0; q < t->n; q++)
                    acc = fmaf(W[t->q[q]], src[(int64_t)t->dz[q] * eq + (int64_t)t->dy[q] * ep + j + t->dx[q]], acc);
                dst[j] = acc;
            }
        }
        float *tmp = a; a = c; c = tmp;
    }
    for (int64_t k = 0; k < planes; k++)
        for (int64_t i = 0; i < rows; i++)
            memcpy(out + (k * rows + i) * cols, a + (k + r) * eq + (i + r) * ep + r, sizeof(float) * cols);
    free(a); free(c); free(t);
    return ORC_OK;
}
