// CNN surrogate of the variable-coefficient heat step: six 3x3 convolutions (zero "same"
// padding), channels 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, bias everywhere, exact-erf GELU after
// layers 1-5, residual output u_hat = u0 + gain * f(u0 * inv, (kappa - 0.125) / 0.075), where
// inv = fp32(1 / s) and gain = fp32(2^-11 s) come from the RMS s of the field (s = 1 for a zero
// field): the network sees the field in units of its size and predicts the K-step update in
// units of 2^-11 of it, so that its last layer works with values of order one.
//
//   layer 1 (2 -> 32)   FP32 MFMA (v_mfma_f32_16x16x4_f32), K = 9 taps x 2 inputs
//   layers 2-5 (32->32) BF16 MFMA implicit GEMM (v_mfma_f32_16x16x32_bf16), FP32 accumulate:
//                       M = 16 output channels, N = 16 consecutive pixels of a row, K = the 32
//                       input channels of one tap; 9 taps x 2 M-halves per 16 pixels
//   layer 6 (32 -> 1)   BF16 MFMA over the BF16 activations with each FP32 weight split into a
//                       BF16 pair (high + low part, 16 significant bits), FP32 accumulate
// Backward: dA = the same MFMA convolution with the taps flipped and the channel roles swapped,
// times GELU'(Z) in the epilogue; dW of layers 2-5 is an MFMA GEMM whose reduction runs over
// pixels (activation and gradient tiles are staged channel-major in LDS so that 8 consecutive
// pixels form one 16-byte operand); every weight/bias gradient is reduced from per-block partial
// sums in a fixed order, so training is deterministic.
//
// Activations are NHWC BF16 (32 channels = 64 bytes per pixel); pre-activations Z are FP32.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "internal.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

namespace st {

namespace {

constexpr int C = 32;
constexpr int NL = 6;
// parameter offsets (floats): W_l [ky][kx][ci][co] then b_l[co]
constexpr int CI[NL] = {2, 32, 32, 32, 32, 32};
constexpr int CO[NL] = {32, 32, 32, 32, 32, 1};
constexpr int woff(int l) {
    int o = 0;
    for (int k = 0; k < l; ++k) o += 9 * CI[k] * CO[k] + CO[k];
    return o;
}
constexpr int boff(int l) { return woff(l) + 9 * CI[l] * CO[l]; }
static_assert(woff(NL) == SG_PARAM_COUNT, "parameter count");

constexpr float KMID = 0.125f, KHALF = 0.075f;
constexpr double UPDATE_SCALE = 1.0 / 2048.0;  // 2^-11: the unit of the predicted update, per unit of field RMS

// bf16 <-> f32
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ __forceinline__ uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// GELU(z) = z Phi(z) with the normal CDF Phi(z) = erfc(-z / sqrt 2) / 2, and GELU'(z) = Phi(z) +
// z phi(z).  erfc comes from the Chebyshev-fitted formula of Press, Teukolsky, Vetterling and
// Flannery, Numerical Recipes (2nd ed.), Sec. 6.2: for x >= 0, erfc(x) = t exp(-x^2 + c0 + t (c1 +
// t (c2 + ... + t c9))) with t = 1 / (1 + x / 2), fractional error below 1.2e-7 everywhere -- so
// Phi(z) keeps its relative accuracy far into the negative tail, where GELU is small and its BF16
// rounding is still done relative to its own size.
//
// Evaluated as a power of two: with L = log2(e) and s = x sqrt(L) = |z| sqrt(L / 2),
//   tail = erfc(x) / 2 = 1 - Phi(|z|) = t 2^(-s^2 + (L c0 - 1) + t (L c1 + t (L c2 + ...))),
//   t = 1 / (1 + s / (2 sqrt L)),   phi(z) = 2^(-s^2 + log2(1 / sqrt(2 pi))),
// so the scale factors fold into the constants, and GELU(z) = max(z, 0) - |z| tail for either sign.
struct ErfcTail {
    float s;     // |z| sqrt(L / 2)
    float tail;  // 1 - Phi(|z|)
};

__device__ __forceinline__ ErfcTail erfc_tail(float z) {
    constexpr float KS = 0.849321782588958740f;  // sqrt(L / 2)
    constexpr float KT = 0.416277319192886353f;  // 1 / (2 sqrt L)
    constexpr float D0 = -2.82574820518493652f, D1 = 1.44272923469543457f, D2 = 0.539700627326965332f,
                    D3 = 0.139630049467086792f, D4 = -0.268756866455078125f, D5 = 0.402321577072143555f,
                    D6 = -1.63775312900543213f, D7 = 2.14747452735900879f, D8 = -1.18611490726470947f,
                    D9 = 0.246517300605773926f;  // L c_k, and L c0 - 1
    ErfcTail r;
    r.s = fabsf(z) * KS;
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(KT, r.s, 1.0f));
    float p = __builtin_fmaf(D9, t, D8);
    p = __builtin_fmaf(p, t, D7);
    p = __builtin_fmaf(p, t, D6);
    p = __builtin_fmaf(p, t, D5);
    p = __builtin_fmaf(p, t, D4);
    p = __builtin_fmaf(p, t, D3);
    p = __builtin_fmaf(p, t, D2);
    p = __builtin_fmaf(p, t, D1);
    p = __builtin_fmaf(p, t, D0);
    r.tail = t * __builtin_amdgcn_exp2f(__builtin_fmaf(-r.s, r.s, p));
    return r;
}

// max(z, 0) in one integer max on the bit pattern: a negative float (or -0) is a negative integer
// (fmaxf would first quiet a signalling NaN: two instructions)
__device__ __forceinline__ float relu(float z) { return __int_as_float(max(__float_as_int(z), 0)); }

__device__ __forceinline__ float gelu(float z) { return __builtin_fmaf(-fabsf(z), erfc_tail(z).tail, relu(z)); }

__device__ __forceinline__ float gelu_grad(float z) {
    constexpr float LOG2_INV_SQRT_2PI = -1.32574808597564697f;
    const ErfcTail e = erfc_tail(z);
    const float cdf = z >= 0.0f ? 1.0f - e.tail : e.tail;
    const float pdf = __builtin_amdgcn_exp2f(__builtin_fmaf(-e.s, e.s, LOG2_INV_SQRT_2PI));
    return __builtin_fmaf(z, pdf, cdf);
}

// ---------------------------------------------------------------------------
// weight preparation: FP32 master -> BF16 MFMA A-operand fragments
// frag[tap][nt][lane][8]: lane holds W'[tap][k = 8*(lane/16) + i][n = 16*nt + lane%16], i.e. the
// 16 x 32 (output channel x input channel) A operand with row n - 16 nt = lane % 16
// forward:   W'[tap][ci][co]  = W[tap][ci][co]
// backward:  W'[tap][co][ci]  = W[8 - tap][ci][co]   (flipped taps, swapped channel roles)
// ---------------------------------------------------------------------------
constexpr int FRAG = 9 * 2 * 64 * 8;  // bf16 per layer and direction
// Layer 6 (32 -> 1, forward): frag6[tap][lane][8] is the A operand whose row 0 holds bf16(W6) and
// row 1 bf16(W6 - bf16(W6)), every other row zero: one MFMA per tap yields both partial sums,
// which together carry 16 significant bits of every FP32 weight (relative error <= 2^-18).
constexpr int FRAG6 = 9 * 64 * 8;
constexpr int NFRAG = 4 * 2 * FRAG + FRAG6;  // bf16 in the fragment area

__global__ void prep_frags(const float* params, uint16_t* frags) {
    // frags: [4 layers][2 directions][FRAG], then [FRAG6]
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NFRAG) return;
    if (idx >= 4 * 2 * FRAG) {
        const int r = idx - 4 * 2 * FRAG;
        const int tap = r / (64 * 8), lane = (r / 8) % 64, i = r % 8;
        const int m = lane % 16, k = 8 * (lane / 16) + i;
        const float w = params[woff(5) + tap * C + k];
        const uint16_t hi = f2bf(w);
        frags[idx] = m == 0 ? hi : m == 1 ? f2bf(w - bf2f(hi)) : uint16_t(0);
        return;
    }
    const int l = idx / (2 * FRAG), dir = (idx / FRAG) % 2, r = idx % FRAG;
    const int tap = r / (2 * 64 * 8), nt = (r / (64 * 8)) % 2, lane = (r / 8) % 64, i = r % 8;
    const int k = 8 * (lane / 16) + i, n = 16 * nt + lane % 16;
    const float* W = params + woff(l + 1);
    float v;
    if (dir == 0) v = W[(tap * C + k) * C + n];
    else v = W[((8 - tap) * C + n) * C + k];
    frags[idx] = f2bf(v);
}

// ---------------------------------------------------------------------------
// Tiles of TH x TW output pixels; their input is the haloed (TH+2) x (TW+2) patch of NHWC BF16
// activations (4 chunks of 8 channels per pixel).  The persistent kernels below walk tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...: the next tile's patch is loaded into registers while
// the current one computes from LDS (two LDS buffers, one barrier per tile).
// ---------------------------------------------------------------------------
constexpr int TH = 8, TW = 32;
constexpr int TPIX = (TH + 2) * (TW + 2);      // haloed patch pixels
constexpr int TCHUNK = TPIX * 4;               // 16-byte chunks in the patch
constexpr int SPT = (TCHUNK + 255) / 256;      // chunks per thread

// LDS slot of chunk c of patch pixel p: pixels are 5 slots apart (one 16-byte slot of padding), so
// the same chunk of 8 or 16 consecutive pixels falls in distinct 16-byte bank groups (5 is odd),
// and an operand's address is a per-lane base plus a compile-time offset.
constexpr int PSTRIDE = 5;
constexpr int PSLOTS = TPIX * PSTRIDE;  // uint4 slots per patch buffer
__device__ __forceinline__ int slot(int p, int c) { return p * PSTRIDE + c; }

struct Tile {
    int b, y0, x0;
};

__device__ __forceinline__ Tile tile_at(int64_t t, int H, int W) {
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int64_t per = int64_t(tiles_x) * tiles_y;
    const int r = int(t % per);
    return Tile{int(t / per), (r / tiles_x) * TH, (r % tiles_x) * TW};
}

__host__ __device__ inline int64_t tile_count(int nb, int H, int W) {
    return int64_t(nb) * ((H + TH - 1) / TH) * ((W + TW - 1) / TW);
}

// Global loads of a tile's patch (zero outside the field) into registers.  Offsets within the
// patch are 32-bit (9 rows of W * C < 2^31 elements); a tile whose patch lies inside the field
// loads without per-pixel checks.
__device__ __forceinline__ void patch_fetch(const uint16_t* X, Tile tc, int H, int W, uint4 (&r)[SPT]) {
    const int64_t base = ((int64_t(tc.b) * H + (tc.y0 - 1)) * W + (tc.x0 - 1)) * C;  // patch pixel (0, 0)
    const bool inside = tc.y0 >= 1 && tc.y0 + TH + 1 <= H && tc.x0 >= 1 && tc.x0 + TW + 1 <= W;
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int k = int(threadIdx.x) + 256 * j;
        const int pix = k >> 2, ch = k & 3;
        const int py = pix / (TW + 2), px = pix % (TW + 2);
        const int yy = tc.y0 - 1 + py, xx = tc.x0 - 1 + px;
        r[j] = make_uint4(0, 0, 0, 0);
        if (k < TCHUNK && (inside || (yy >= 0 && yy < H && xx >= 0 && xx < W)))
            r[j] = *reinterpret_cast<const uint4*>(X + (base + ((py * W + px) * C + ch * 8)));
    }
}

__device__ __forceinline__ void patch_store(uint4* lds, const uint4 (&r)[SPT]) {
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int k = int(threadIdx.x) + 256 * j;
        if (k < TCHUNK) lds[slot(k >> 2, k & 3)] = r[j];
    }
}

// ---------------------------------------------------------------------------
// 32 -> 32 MFMA convolution (forward, or backward-data with flipped fragments).  Each wave owns
// TH/4 rows x TW pixels of a tile.  The weights are the A operand (M = 16 output channels, K = 32
// input channels of one tap) and the activations the B operand (N = 16 pixels), so a lane's result
// is 4 consecutive channels of one pixel and the epilogue writes 8- or 16-byte vectors.
// ---------------------------------------------------------------------------
enum Epi { EPI_FWD = 0, EPI_BWD_BF16 = 1, EPI_BWD_F32 = 2 };

struct ConvArgs {
    const uint16_t* X;      // input activations (fwd) or dZ (bwd), NHWC bf16
    const uint16_t* frags;  // 9 x 2 x 64 x 8 bf16
    const float* bias;      // fwd only
    const float* Zprev;     // bwd: pre-activations whose GELU' scales the result
    float* Zout;            // fwd: pre-activation out (nullable)
    uint16_t* Aout;         // fwd: GELU(Z) bf16; bwd: dZ bf16
    float* Fout;            // bwd: dZ fp32 (layer-1 target)
    int nb, H, W;
};

// Two values rounded to BF16 (nearest even) and packed low-first: one v_cvt_pk_bf16_f32.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

template <int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv_mfma(ConvArgs a) {
    __shared__ uint4 patch[2][PSLOTS];
    const int64_t ntiles = tile_count(a.nb, a.H, a.W);
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // A fragments of all taps, loaded once per workgroup
    bf16x8_t wf[9][2];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
            wf[k][nt] = *reinterpret_cast<const bf16x8_t*>(a.frags + ((k * 2 + nt) * 64 + lane) * 8);
    const int lane_px = lane & 15, ch0 = 4 * (lane >> 4);  // result: channels 16 nt + ch0 + i of pixel lane_px
    f32x4_t bias4[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias4[nt][i] = EPI == EPI_FWD ? a.bias[16 * nt + ch0 + i] : 0.0f;
    constexpr int ROWS = TH / 4;  // rows per wave
    constexpr int MT = TW / 16;   // 16-pixel groups per row
    uint4 pre[SPT];
    patch_fetch(a.X, tile_at(t, a.H, a.W), a.H, a.W, pre);
    for (int buf = 0; t < ntiles; t += gridDim.x, buf ^= 1) {
        const Tile tc = tile_at(t, a.H, a.W);
        uint4* lds = patch[buf];
        patch_store(lds, pre);
        __syncthreads();
        if (t + gridDim.x < ntiles) patch_fetch(a.X, tile_at(t + gridDim.x, a.H, a.W), a.H, a.W, pre);
        // the first tap's MFMAs start from the bias (forward) or zero, read straight from `bias4`; the
        // taps run in the outer loop so that consecutive MFMAs feed independent accumulators
        f32x4_t acc[ROWS][MT][2];
        const uint4* opnd = lds + slot((wave * ROWS) * (TW + 2) + lane_px, lane >> 4);
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const bf16x8_t xv =
                        __builtin_bit_cast(bf16x8_t, opnd[PSTRIDE * ((r + k / 3) * (TW + 2) + m * 16 + k % 3)]);
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        acc[r][m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[k][nt], xv,
                                                                                k == 0 ? bias4[nt] : acc[r][m][nt], 0, 0, 0);
                }
        // epilogue; offsets inside a row are 32-bit (W * C < 2^31 is checked on the host)
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = tc.y0 + wave * ROWS + r;
            if (y >= a.H) continue;
            const int64_t row = (int64_t(tc.b) * a.H + y) * a.W * C;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int x = tc.x0 + m * 16 + lane_px;
                if (x >= a.W) continue;
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const int64_t o = row + (x * C + 16 * nt + ch0);
                    float v[4];
                    if (EPI == EPI_FWD) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) v[i] = acc[r][m][nt][i];
                        if (a.Zout) *reinterpret_cast<float4*>(a.Zout + o) = make_float4(v[0], v[1], v[2], v[3]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) v[i] = gelu(v[i]);
                    } else {
                        const float4 z = *reinterpret_cast<const float4*>(a.Zprev + o);
                        v[0] = acc[r][m][nt][0] * gelu_grad(z.x);
                        v[1] = acc[r][m][nt][1] * gelu_grad(z.y);
                        v[2] = acc[r][m][nt][2] * gelu_grad(z.z);
                        v[3] = acc[r][m][nt][3] * gelu_grad(z.w);
                    }
                    if (EPI == EPI_BWD_F32)
                        *reinterpret_cast<float4*>(a.Fout + o) = make_float4(v[0], v[1], v[2], v[3]);
                    else
                        *reinterpret_cast<uint2*>(a.Aout + o) = make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// layer 1: 2 -> 32 in FP32 on MFMA (v_mfma_f32_16x16x4_f32): M = 16 output channels, N = 16 pixels
// of a row, K = the 18 (tap, input channel) pairs k = 2 tap + c, padded to 20.  The patch holds
// (u0, (kappa - 0.125) / 0.075) per pixel in FP32, normalised once per patch pixel.
// ---------------------------------------------------------------------------
constexpr int SPT1 = (TPIX + 255) / 256;  // patch pixels per thread

__device__ __forceinline__ void input_fetch(const float* u0, const float* kappa, Tile tc, int H, int W,
                                            float2 (&r)[SPT1]) {
    const int64_t base = (int64_t(tc.b) * H + (tc.y0 - 1)) * W + (tc.x0 - 1);  // patch pixel (0, 0)
    const bool inside = tc.y0 >= 1 && tc.y0 + TH + 1 <= H && tc.x0 >= 1 && tc.x0 + TW + 1 <= W;
#pragma unroll
    for (int j = 0; j < SPT1; ++j) {
        const int k = int(threadIdx.x) + 256 * j;
        const int py = k / (TW + 2), px = k % (TW + 2);
        const int yy = tc.y0 - 1 + py, xx = tc.x0 - 1 + px;
        r[j] = make_float2(0.0f, KMID);  // zero padding of both input channels
        if (k < TPIX && (inside || (yy >= 0 && yy < H && xx >= 0 && xx < W))) {
            const int64_t q = base + (py * W + px);
            r[j] = make_float2(u0[q], kappa[q]);
        }
    }
}

__device__ __forceinline__ void input_store(float* lds, const float2 (&r)[SPT1], float inv) {
#pragma unroll
    for (int j = 0; j < SPT1; ++j) {
        const int k = int(threadIdx.x) + 256 * j;
        if (k < TPIX) {
            lds[2 * k] = r[j].x * inv;
            lds[2 * k + 1] = (r[j].y - KMID) / KHALF;
        }
    }
}

// scale: per field (inv, gain); the u0 channel enters as u0 * inv
__global__ __launch_bounds__(256) void l1_fwd(const float* params, const float* u0, const float* kappa,
                                              const float* scale, int nb, int H, int W, float* Z, uint16_t* A) {
    __shared__ float patch[2][2 * TPIX];
    const int64_t ntiles = tile_count(nb, H, W);
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lane_px = lane & 15, ch0 = 4 * (lane >> 4);
    // per K step s this lane supplies k = 4 s + lane / 16: weight W1[k][co] (A) and the patch value
    // at tap k / 2, channel k % 2 (B), found at `koff[s]` floats from its pixel's first channel
    float wa[5][2];
    int koff[5];
#pragma unroll
    for (int s5 = 0; s5 < 5; ++s5) {
        const int k = 4 * s5 + (lane >> 4);
        const int tap = k >> 1;
        koff[s5] = k < 18 ? 2 * ((tap / 3) * (TW + 2) + tap % 3) + (k & 1) : -1;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) wa[s5][mt] = k < 18 ? params[k * C + 16 * mt + lane_px] : 0.0f;
    }
    float bias[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias[mt][i] = params[9 * 2 * C + 16 * mt + ch0 + i];
    constexpr int ROWS = TH / 4, MT = TW / 16;
    float2 pre[SPT1];
    input_fetch(u0, kappa, tile_at(t, H, W), H, W, pre);
    for (int buf = 0; t < ntiles; t += gridDim.x, buf ^= 1) {
        const Tile tc = tile_at(t, H, W);
        float* lds = patch[buf];
        input_store(lds, pre, scale[2 * tc.b]);
        __syncthreads();
        if (t + gridDim.x < ntiles) input_fetch(u0, kappa, tile_at(t + gridDim.x, H, W), H, W, pre);
        // accumulators start from the bias; K steps outermost so that consecutive MFMAs feed
        // independent accumulators
        f32x4_t acc[ROWS][MT][2];
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
                    acc[r][m][mt] = f32x4_t{bias[mt][0], bias[mt][1], bias[mt][2], bias[mt][3]};
        const float* opnd = lds + 2 * ((wave * ROWS) * (TW + 2) + lane_px);
#pragma unroll
        for (int s5 = 0; s5 < 5; ++s5)
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const float bv = koff[s5] >= 0 ? opnd[2 * (r * (TW + 2) + m * 16) + koff[s5]] : 0.0f;
                    acc[r][m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[s5][0], bv, acc[r][m][0], 0, 0, 0);
                    acc[r][m][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[s5][1], bv, acc[r][m][1], 0, 0, 0);
                }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int y = tc.y0 + wave * ROWS + r;
            if (y >= H) continue;
            const int64_t row = (int64_t(tc.b) * H + y) * W * C;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int x = tc.x0 + m * 16 + lane_px;
                if (x >= W) continue;
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const int64_t o = row + (x * C + 16 * mt + ch0);
                    float v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = acc[r][m][mt][i];
                    if (Z) *reinterpret_cast<float4*>(Z + o) = make_float4(v[0], v[1], v[2], v[3]);
                    *reinterpret_cast<uint2*>(A + o) =
                        make_uint2(pack_bf16(gelu(v[0]), gelu(v[1])), pack_bf16(gelu(v[2]), gelu(v[3])));
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// layer 6: 32 -> 1 with the residual, on MFMA with the split weights of frag6 (M row 0: high
// parts, row 1: low parts), N = 16 pixels, K = 32 channels of one tap; the bias starts row 0.
// Lanes 0-15 hold rows 0-3 of their pixel: f = row 0 + row 1.  Its arithmetic per tile is short,
// so it runs one patch buffer (two barriers per tile) to fit three workgroups per CU and keep
// more loads in flight.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void l6_fwd(
    const float* params, const uint16_t* frag6, const uint16_t* A5, const float* u0, const float* scale, int nb, int H,
    int W, float* uhat) {
    __shared__ uint4 patch[PSLOTS];  // one buffer (two barriers per tile): three workgroups per CU
    const int64_t ntiles = tile_count(nb, H, W);
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lane_px = lane & 15;
    bf16x8_t wf[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) wf[k] = *reinterpret_cast<const bf16x8_t*>(frag6 + (k * 64 + lane) * 8);
    const float b0 = lane < 16 ? params[woff(5) + 9 * C] : 0.0f;
    constexpr int ROWS = TH / 4, MT = TW / 16;
    uint4 pre[SPT];
    patch_fetch(A5, tile_at(t, H, W), H, W, pre);
    for (; t < ntiles; t += gridDim.x) {
        const Tile tc = tile_at(t, H, W);
        uint4* lds = patch;
        __syncthreads();  // every wave is done reading the previous tile
        patch_store(lds, pre);
        __syncthreads();
        if (t + gridDim.x < ntiles) patch_fetch(A5, tile_at(t + gridDim.x, H, W), H, W, pre);
        f32x4_t acc[ROWS][MT];
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[r][m] = f32x4_t{b0, 0, 0, 0};
        const uint4* opnd = lds + slot((wave * ROWS) * (TW + 2) + lane_px, lane >> 4);
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const bf16x8_t xv =
                        __builtin_bit_cast(bf16x8_t, opnd[PSTRIDE * ((r + k / 3) * (TW + 2) + m * 16 + k % 3)]);
                    acc[r][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[k], xv, acc[r][m], 0, 0, 0);
                }
        if (lane < 16) {
            const float gain = scale[2 * tc.b + 1];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int y = tc.y0 + wave * ROWS + r;
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const int x = tc.x0 + m * 16 + lane_px;
                    if (y < H && x < W) {
                        const int64_t o = (int64_t(tc.b) * H + y) * W + x;
                        uhat[o] = __builtin_fmaf(gain, acc[r][m][0] + acc[r][m][1], u0[o]);
                    }
                }
            }
        }
    }
}

constexpr int MAXB = 64;  // largest training batch (per-sample loss masks travel in the kernel arguments)
struct MaskArgs {
    int lohi[4 * MAXB];  // per sample: rows [lohi[0], lohi[1]) x cols [lohi[2], lohi[3])
};

// dF = d loss / d f = (2/n) gain (u_hat - target) on the mask; per-block FP64 partial sums of the
// squared error
__global__ __launch_bounds__(256) void loss_grad(const float* uhat, const float* target, const float* scale, int nb,
                                                 int H, int W, MaskArgs mk, double inv_n, float* dF, double* partial) {
    __shared__ double red[256];
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double e2 = 0.0;
    if (p < int64_t(nb) * H * W) {
        const int b = int(p / (int64_t(H) * W));
        const int y = int((p / W) % H), x = int(p % W);
        const int* m = mk.lohi + 4 * b;
        const bool in = y >= m[0] && y < m[1] && x >= m[2] && x < m[3];
        const float d = in ? uhat[p] - target[p] : 0.0f;
        dF[p] = float(2.0 * inv_n * double(scale[2 * b + 1])) * d;
        e2 = double(d) * double(d);
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_finish(const double* partial, int n, double inv_n, double* loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) s += partial[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * inv_n;
}

// dZ5[p][ci] = GELU'(Z5[p][ci]) * sum_t W6[t][ci] dF[p - t + (1,1)]   (bf16)
__global__ __launch_bounds__(256) void l6_bwd_data(const float* params, const float* dF, const float* Z5, int nb,
                                                   int H, int W, uint16_t* dZ5) {
    __shared__ float w[9 * C];
    for (int k = threadIdx.x; k < 9 * C; k += 256) w[k] = params[woff(5) + k];
    __syncthreads();
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= int64_t(nb) * H * W) return;
    const int64_t b = p / (int64_t(H) * W);
    const int y = int((p / W) % H), x = int(p % W);
    float g[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y - (t / 3 - 1), xx = x - (t % 3 - 1);
        g[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? dF[(b * H + yy) * W + xx] : 0.0f;
    }
    uint32_t packed[C / 2];
#pragma unroll
    for (int ci = 0; ci < C; ++ci) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc = __builtin_fmaf(w[t * C + ci], g[t], acc);
        const uint32_t h = f2bf(acc * gelu_grad(Z5[p * C + ci]));
        if (ci & 1) packed[ci / 2] |= h << 16; else packed[ci / 2] = h;
    }
    uint4* dst = reinterpret_cast<uint4*>(dZ5 + p * C);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
}

// ---------------------------------------------------------------------------
// weight gradients: per-block partials over a 32 x 32 pixel region, reduced later in fixed order
// ---------------------------------------------------------------------------
constexpr int RH = 32, RW = 32;  // pixels per partial block

// Layers 1 and 6 take their region in chunks of WCH rows staged in LDS (the chunk's gradient rows
// and its input rows with a one-pixel halo, zero outside the grid), so that each output's sum over
// the region reads LDS instead of waiting on a global load per pixel.  Pixels are visited row by row
// as before; a zero-padded input or gradient adds an exact zero.
constexpr int WCH = 8;  // rows per staged chunk

// layer 1: dW1[t][ci][co] = sum_p X0[p + t][ci] dZ1[p][co], db1[co] = sum_p dZ1[p][co]  (all FP32)
// one thread per (t, ci, co) output (576) plus 32 bias threads.
__global__ __launch_bounds__(640) void l1_bwd_weight(const float* u0, const float* kappa, const float* scale,
                                                     const float* dZ1, int nb, int H, int W, float* partial) {
    __shared__ float gz[WCH][RW][C];           // dZ1 of the chunk
    __shared__ float xin[WCH + 2][RW + 2][2];  // X0 (scaled u0, centred kappa) with halo
    const int rx = (W + RW - 1) / RW, ry = (H + RH - 1) / RH;
    const int blk = blockIdx.x;
    const int b = blk / (rx * ry), r = blk % (rx * ry);
    const int y0 = (r / rx) * RH, x0 = (r % rx) * RW;
    const int j = threadIdx.x;
    const float inv = scale[2 * b];
    const int t = j / (2 * C), ci = (j / C) % 2, co = j % C;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    float acc = 0.0f;
    for (int c0 = y0; c0 < y0 + RH; c0 += WCH) {
        __syncthreads();  // the previous chunk is no longer read
        for (int e = j; e < WCH * RW * C; e += 640) {
            const int k = e % C, x = (e / C) % RW, y = e / (C * RW);
            const int gy = c0 + y, gx = x0 + x;
            gz[y][x][k] = (gy < H && gx < W) ? dZ1[((int64_t(b) * H + gy) * W + gx) * C + k] : 0.0f;
        }
        for (int e = j; e < (WCH + 2) * (RW + 2); e += 640) {
            const int x = e % (RW + 2), y = e / (RW + 2);
            const int gy = c0 + y - 1, gx = x0 + x - 1;
            const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
            const int64_t q = (int64_t(b) * H + gy) * W + gx;
            xin[y][x][0] = in ? u0[q] * inv : 0.0f;
            xin[y][x][1] = in ? (kappa[q] - KMID) / KHALF : 0.0f;
        }
        __syncthreads();
        if (j < 9 * 2 * C) {
            for (int y = 0; y < WCH; ++y)
#pragma unroll 8
                for (int x = 0; x < RW; ++x) acc = __builtin_fmaf(xin[y + 1 + dy][x + 1 + dx][ci], gz[y][x][co], acc);
        } else if (j < 9 * 2 * C + C) {
            const int cb = j - 9 * 2 * C;
            for (int y = 0; y < WCH; ++y)
#pragma unroll 8
                for (int x = 0; x < RW; ++x) acc += gz[y][x][cb];
        }
    }
    if (j < 9 * 2 * C + C) partial[int64_t(blk) * (9 * 2 * C + C) + j] = acc;
}

// layer 6: dW6[t][ci] = sum_p A5[p + t][ci] dF[p], db6 = sum_p dF[p]
__global__ __launch_bounds__(320) void l6_bwd_weight(const uint16_t* A5, const float* dF, int nb, int H, int W,
                                                     float* partial) {
    __shared__ float at[WCH + 2][RW + 2][C + 1];  // A5 with halo (padded: lanes of one row differ in ci)
    __shared__ float gf[WCH][RW];
    const int rx = (W + RW - 1) / RW, ry = (H + RH - 1) / RH;
    const int blk = blockIdx.x;
    const int b = blk / (rx * ry), r = blk % (rx * ry);
    const int y0 = (r / rx) * RH, x0 = (r % rx) * RW;
    const int j = threadIdx.x;
    const int t = j / C, ci = j % C;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    float acc = 0.0f;
    for (int c0 = y0; c0 < y0 + RH; c0 += WCH) {
        __syncthreads();
        for (int e = j; e < (WCH + 2) * (RW + 2) * C; e += 320) {
            const int k = e % C, x = (e / C) % (RW + 2), y = e / (C * (RW + 2));
            const int gy = c0 + y - 1, gx = x0 + x - 1;
            at[y][x][k] = (gy >= 0 && gy < H && gx >= 0 && gx < W)
                              ? bf2f(A5[((int64_t(b) * H + gy) * W + gx) * C + k]) : 0.0f;
        }
        for (int e = j; e < WCH * RW; e += 320) {
            const int x = e % RW, y = e / RW;
            const int gy = c0 + y, gx = x0 + x;
            gf[y][x] = (gy < H && gx < W) ? dF[(int64_t(b) * H + gy) * W + gx] : 0.0f;
        }
        __syncthreads();
        if (j < 9 * C) {
            for (int y = 0; y < WCH; ++y)
#pragma unroll 8
                for (int x = 0; x < RW; ++x) acc = __builtin_fmaf(at[y + 1 + dy][x + 1 + dx][ci], gf[y][x], acc);
        } else if (j == 9 * C) {
            for (int y = 0; y < WCH; ++y)
                for (int x = 0; x < RW; ++x) acc += gf[y][x];
        }
    }
    if (j < 9 * C + 1) partial[int64_t(blk) * (9 * C + 1) + j] = acc;
}

// layers 2-5: dW[t][ci][co] = sum_p A[p + t][ci] dZ[p][co] on MFMA.  The region is processed in
// 8-row chunks; per chunk the activation tile (with halo) is staged channel-major three times,
// shifted by 0, 1, 2 pixels in x, and the gradient tile channel-major, so that each MFMA
// operand (8 consecutive pixels of one channel) is one aligned 16-byte LDS read.
// Wave w owns the output quarter (ci half w/2, co half w%2) for all 9 taps.
// db[co] = sum_p dZ[p][co] is accumulated from the staged gradient tile.
constexpr int CH = 8;  // rows per chunk
__global__ __launch_bounds__(256) void mfma_bwd_weight(const uint16_t* A, const uint16_t* dZ, int nb, int H, int W,
                                                       float* partial) {
    __shared__ uint16_t at[3][C][CH + 2][RW];  // [shift][ci][row][x]: A at (row-1, x+shift-1) of the chunk
    __shared__ uint16_t gt[C][CH][RW];         // [co][row][x]
    __shared__ float bsum[4][C];
    const int rx = (W + RW - 1) / RW, ry = (H + RH - 1) / RH;
    const int blk = blockIdx.x;
    const int b = blk / (rx * ry), r = blk % (rx * ry);
    const int y0 = (r / rx) * RH, x0 = (r % rx) * RW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mh = wave >> 1, nh = wave & 1;
    f32x4_t acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4_t{0, 0, 0, 0};
    float bacc = 0.0f;  // thread c < 32: running bias sum of channel c... computed below
    if (threadIdx.x < 4 * C) bsum[threadIdx.x / C][threadIdx.x % C] = 0.0f;
    for (int c0 = 0; c0 < RH; c0 += CH) {
        const int cy0 = y0 + c0;
        __syncthreads();
        // stage A: rows cy0-1 .. cy0+CH, cols x0-1 .. x0+RW (34 pixels), 4 chunks of 8 channels each
        for (int k = threadIdx.x; k < (CH + 2) * (RW + 2) * 4; k += 256) {
            const int pix = k >> 2, cq = k & 3;
            const int row = pix / (RW + 2), col = pix % (RW + 2);
            const int yy = cy0 - 1 + row, xx = x0 - 1 + col;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                v = reinterpret_cast<const uint4*>(A + ((int64_t(b) * H + yy) * W + xx) * C)[cq];
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint16_t h = uint16_t(e & 1 ? wd[e >> 1] >> 16 : wd[e >> 1] & 0xffffu);
                const int ci = cq * 8 + e;
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    const int x = col - s;  // tile column col holds A(x0-1+col); copy s at x holds A(x0-1+x+s)
                    if (x >= 0 && x < RW) at[s][ci][row][x] = h;
                }
            }
        }
        // stage dZ: rows cy0 .. cy0+CH-1, cols x0 .. x0+RW-1 (zero outside the field)
        for (int k = threadIdx.x; k < CH * RW * 4; k += 256) {
            const int pix = k >> 2, cq = k & 3;
            const int row = pix / RW, col = pix % RW;
            const int yy = cy0 + row, xx = x0 + col;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (yy < H && xx < W) v = reinterpret_cast<const uint4*>(dZ + ((int64_t(b) * H + yy) * W + xx) * C)[cq];
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
                gt[cq * 8 + e][row][col] = uint16_t(e & 1 ? wd[e >> 1] >> 16 : wd[e >> 1] & 0xffffu);
        }
        __syncthreads();
        // bias partial: thread j < 128 sums channel j%32 over a quarter of the chunk's pixels
        if (threadIdx.x < 4 * C) {
            const int co = threadIdx.x % C, q = threadIdx.x / C;
            float s = 0.0f;
            for (int rr = q * (CH / 4); rr < (q + 1) * (CH / 4); ++rr)
                for (int x = 0; x < RW; ++x) s += bf2f(gt[co][rr][x]);
            bsum[q][co] += s;
        }
        // MFMA over the chunk: K = 32 pixels of one row per instruction
#pragma unroll
        for (int rr = 0; rr < CH; ++rr) {
            const bf16x8_t bv = *reinterpret_cast<const bf16x8_t*>(&gt[nh * 16 + (lane & 15)][rr][8 * (lane >> 4)]);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int ky = t / 3, kx = t % 3;
                const bf16x8_t av =
                    *reinterpret_cast<const bf16x8_t*>(&at[kx][mh * 16 + (lane & 15)][rr + ky][8 * (lane >> 4)]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
            }
        }
    }
    __syncthreads();
    // D layout: lane holds D[ci = 16*mh + 4*(lane/16) + i][co = 16*nh + lane%16]
    float* out = partial + int64_t(blk) * (9 * C * C + C);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ci = 16 * mh + 4 * (lane >> 4) + i, co = 16 * nh + (lane & 15);
            out[(t * C + ci) * C + co] = acc[t][i];
        }
    if (threadIdx.x < C) out[9 * C * C + threadIdx.x] = ((bsum[0][threadIdx.x] + bsum[1][threadIdx.x]) +
                                                          bsum[2][threadIdx.x]) + bsum[3][threadIdx.x];
    (void)bacc;
}

// grad[off + j] = sum_{blk} partial[blk][j] in block order (FP64 accumulation)
// Block g sums outputs j = 64 g .. 64 g + 63 over the nblk partials: wave q takes the partials
// k = q, q + 16, ... (one coalesced 256-byte row segment per load), and the sixteen FP64 sums are
// added in wave order.  A fixed order, so the gradient is reproducible run to run.
constexpr int RP_WAVES = 16;
__global__ __launch_bounds__(64 * RP_WAVES) void reduce_partials(const float* partial, int nblk, int len, float* grad) {
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (j < len)
#pragma unroll 4
        for (int k = q; k < nblk; k += RP_WAVES) s += double(partial[int64_t(k) * len + j]);
    __shared__ double red[RP_WAVES][64];
    red[q][lane] = s;
    __syncthreads();
    if (q == 0 && j < len) {
        double t = red[0][lane];
#pragma unroll
        for (int w = 1; w < RP_WAVES; ++w) t += red[w][lane];
        grad[j] = float(t);
    }
}

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba, Algorithm 1) with bias correction
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mhat = mi / c1, vhat = vi / c2;
    p[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

// ---------------------------------------------------------------------------
// training-data synthesis and crops
// ---------------------------------------------------------------------------
constexpr int NU = 16, NK = 8;
constexpr int SY = 16, SX = 64;  // cells per synthesis block (4 per thread)

// Both fields are separable per mode: sin(a i) sin(b j) for u0, and
// cos(A_j + B_i) = cos A_j cos B_i - sin A_j sin B_i for kappa.  Each block evaluates the
// per-row and per-column factors of its 16 x 64 cells once (FP64 trigonometry, rounded to FP32)
// and combines them with FMAs.
__global__ __launch_bounds__(256) void synth_kernel(const float* coef, int n, int rows, int cols, float* u0,
                                                    float* kappa) {
    __shared__ float su[NU][SY], tu[NU][SX], cb[NK][SY], sb[NK][SY], ca[NK][SX], sa[NK][SX];
    __shared__ float amp[NU], bamp[NK], binv;
    const int bx = (cols + SX - 1) / SX, by = (rows + SY - 1) / SY;
    const int t = blockIdx.x / (bx * by), r = blockIdx.x % (bx * by);
    const int i0 = (r / bx) * SY, j0 = (r % bx) * SX;
    const float* c = coef + int64_t(t) * 4 * (NU + NK);
    const double pi = 3.14159265358979323846;
    for (int k = threadIdx.x; k < NU * (SY + SX); k += 256) {
        const int m = k / (SY + SX), q = k % (SY + SX);
        if (q < SY) su[m][q] = float(sin(double(c[4 * m]) * pi * (i0 + q + 1) / (rows + 1)));
        else tu[m][q - SY] = float(sin(double(c[4 * m + 1]) * pi * (j0 + q - SY + 1) / (cols + 1)));
    }
    for (int k = threadIdx.x; k < NK * (SY + SX); k += 256) {
        const int m = k / (SY + SX), q = k % (SY + SX);
        const float* cm = c + 4 * (NU + m);
        if (q < SY) {
            const double B = 2.0 * pi * double(cm[1]) * double(i0 + q) / rows;
            cb[m][q] = float(cos(B));
            sb[m][q] = float(sin(B));
        } else {
            const double A = 2.0 * pi * double(cm[0]) * double(j0 + q - SY) / cols + double(cm[3]);
            ca[m][q - SY] = float(cos(A));
            sa[m][q - SY] = float(sin(A));
        }
    }
    if (threadIdx.x < NU) amp[threadIdx.x] = c[4 * threadIdx.x + 2];
    if (threadIdx.x < NK) bamp[threadIdx.x] = c[4 * (NU + threadIdx.x) + 2];
    if (threadIdx.x == 0) {
        double nrm = 0.0;
        for (int m = 0; m < NK; ++m) nrm += fabs(double(c[4 * (NU + m) + 2]));
        binv = float(0.075 / fmax(nrm, 1e-30));
    }
    __syncthreads();
    for (int k = threadIdx.x; k < SY * SX; k += 256) {
        const int q = k / SX, e = k % SX;
        const int i = i0 + q, j = j0 + e;
        if (i >= rows || j >= cols) continue;
        float u = 0.0f, g = 0.0f;
#pragma unroll
        for (int m = 0; m < NU; ++m) u = __builtin_fmaf(amp[m] * su[m][q], tu[m][e], u);
#pragma unroll
        for (int m = 0; m < NK; ++m) g = __builtin_fmaf(bamp[m], ca[m][e] * cb[m][q] - sa[m][e] * sb[m][q], g);
        const int64_t o = (int64_t(t) * rows + i) * cols + j;
        u0[o] = u;
        kappa[o] = 0.125f + g * binv;
    }
}

__global__ void crop_kernel(const float* src, float* dst, const int* yx, int n, int rows, int cols, int h, int w) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(n) * h * w) return;
    const int t = int(idx / (int64_t(h) * w));
    const int i = int((idx / w) % h), j = int(idx % w);
    const int y = yx[2 * t] + i, x = yx[2 * t + 1] + j;
    dst[idx] = (y >= 0 && y < rows && x >= 0 && x < cols) ? src[(int64_t(t) * rows + y) * cols + x] : 0.0f;
}

// FP64 sums of (a - b)^2 and b^2 (judge error), two-stage fixed order
__global__ void diff_norms(const float* a, const float* b, int64_t n, double* partial) {
    __shared__ double r0[256], r1[256];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256) {
        const double d = double(a[k]) - double(b[k]);
        s0 += d * d;
        s1 += double(b[k]) * double(b[k]);
    }
    r0[threadIdx.x] = s0;
    r1[threadIdx.x] = s1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            r0[threadIdx.x] += r0[threadIdx.x + h];
            r1[threadIdx.x] += r1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r0[0];
        partial[2 * blockIdx.x + 1] = r1[0];
    }
}

__global__ void diff_norms_finish(const double* partial, int nblk, double* out2) {
    if (threadIdx.x != 0) return;
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < nblk; ++k) {
        s0 += partial[2 * k];
        s1 += partial[2 * k + 1];
    }
    out2[0] = s0;
    out2[1] = s1;
}

// Scale constants of each field: s = RMS of the field's cells (FP64, fixed-order two-stage sum;
// s = 1 for an all-zero field), scale[2b] = fp32(1 / s), scale[2b + 1] = fp32(2^-11 s).
constexpr int SCB = 256;  // stage-1 blocks per field
__global__ __launch_bounds__(256) void field_scale_partial(const float* u, int64_t n, double* partial) {
    __shared__ double red[256];
    const int b = blockIdx.y;
    const float* f = u + int64_t(b) * n;
    double acc = 0.0;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(SCB) * 256) {
        const double x = double(f[k]);
        acc += x * x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[int64_t(b) * SCB + blockIdx.x] = red[0];
}

__global__ void field_scale_finish(const double* partial, int nb, int64_t n, float* scale) {
    const int b = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double acc = 0.0;
    for (int k = 0; k < SCB; ++k) acc += partial[int64_t(b) * SCB + k];
    double s = sqrt(acc / double(n));
    if (!(s > 0.0)) s = 1.0;
    scale[2 * b] = float(1.0 / s);
    scale[2 * b + 1] = float(UPDATE_SCALE * s);
}

// ---- the light-cone patch judge -------------------------------------------------------------
// An n x n lattice of patches; window (a, c) = patch (a, c) dilated by K cells and clipped to the
// grid.  The windows are packed edge to edge into a "mosaic" field in lattice order, so that the
// mosaic's outer edges are the grid's edges wherever a window touches them; K plain steps on the
// mosaic are exact on every patch (a wrong neighbour across an inner junction moves one cell per
// step and stays K or more cells away from the patch).
constexpr int PLAT = 4;    // lattice points per axis
constexpr int PSIDE = 64;  // patch side (capped by the grid)
struct MosaicArgs {
    int n;                                  // lattice points per axis
    int py, px;                             // patch side in rows / columns
    int y[PLAT], x[PLAT];                   // patch origins in the grid
    int wy[PLAT], wx[PLAT];                 // window origins in the grid
    int my[PLAT + 1], mx[PLAT + 1];         // window origins in the mosaic (prefix sums)
    int rows, cols;                         // grid
};

__device__ __forceinline__ int lattice_of(const int* m, int n, int v) {
    int a = 0;
    while (a + 1 < n && v >= m[a + 1]) ++a;
    return a;
}

// mosaic cell -> grid cell copy of u0 and kappa
__global__ __launch_bounds__(256) void gather_mosaic(const float* u0, const float* kappa, MosaicArgs g, float* mu,
                                                     float* mk) {
    const int MR = g.my[g.n], MC = g.mx[g.n];
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= int64_t(MR) * MC) return;
    const int i = int(idx / MC), j = int(idx % MC);
    const int a = lattice_of(g.my, g.n, i), c = lattice_of(g.mx, g.n, j);
    const int64_t q = int64_t(g.wy[a] + (i - g.my[a])) * g.cols + (g.wx[c] + (j - g.mx[c]));
    mu[idx] = u0[q];
    mk[idx] = kappa[q];
}

// FP64 sums over the patch cells of (u_hat - judge)^2 and judge^2: one block per patch, fixed order
__global__ __launch_bounds__(256) void patch_norms(const float* uhat, const float* mjudge, MosaicArgs g,
                                                   double* partial) {
    __shared__ double r0[256], r1[256];
    const int a = blockIdx.x / g.n, c = blockIdx.x % g.n;
    const int MC = g.mx[g.n];
    double s0 = 0.0, s1 = 0.0;
    for (int k = threadIdx.x; k < g.py * g.px; k += 256) {
        const int dy = k / g.px, dx = k % g.px;
        const int gy = g.y[a] + dy, gx = g.x[c] + dx;
        const double v = double(mjudge[int64_t(g.my[a] + gy - g.wy[a]) * MC + (g.mx[c] + gx - g.wx[c])]);
        const double d = double(uhat[int64_t(gy) * g.cols + gx]) - v;
        s0 += d * d;
        s1 += v * v;
    }
    r0[threadIdx.x] = s0;
    r1[threadIdx.x] = s1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            r0[threadIdx.x] += r0[threadIdx.x + h];
            r1[threadIdx.x] += r1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r0[0];
        partial[2 * blockIdx.x + 1] = r1[0];
    }
}

// ---- seeded initialisation ------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of two 64 x 64 -> 128-bit
// products of words 0 and 2, whose halves are mixed with words 1 and 3 and the key; the key is
// bumped by two Weyl constants per round.
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// He-normal weights N(0, 2 / (9 C_in)) (layer 6 scaled by 0.1), zero biases, zero Adam state.
// Parameter i draws the first two words of Philox4x64-10 at counter (i, 0, 0, 0), key (seed, 0),
// u = (word >> 11) 2^-53, and takes the Box-Muller normal sqrt(-2 ln(1 - u1)) cos(2 pi u2) in FP64.
__global__ __launch_bounds__(256) void init_params_kernel(float* params, float* optim, uint64_t seed) {
    const int i = int(blockIdx.x) * 256 + threadIdx.x;
    if (i >= SG_PARAM_COUNT) return;
    if (optim) {
        optim[i] = 0.0f;
        optim[SG_PARAM_COUNT + i] = 0.0f;
    }
    int l = 0;
    while (i >= woff(l + 1)) ++l;
    if (i >= boff(l)) {
        params[i] = 0.0f;
        return;
    }
    uint64_t c[4] = {uint64_t(i), 0, 0, 0};
    philox4x64_10(c, seed, 0);
    const double u1 = double(c[0] >> 11) * 0x1p-53, u2 = double(c[1] >> 11) * 0x1p-53;
    const double z = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
    const double sd = sqrt(2.0 / (9.0 * CI[l])) * (l == NL - 1 ? 0.1 : 1.0);
    params[i] = float(sd * z);
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Lattice, windows and mosaic of the patch judge for a rows x cols grid and K steps.
MosaicArgs mosaic_layout(int64_t rows, int64_t cols, int64_t K) {
    MosaicArgs g;
    std::memset(&g, 0, sizeof(g));
    g.n = PLAT;
    g.rows = int(rows);
    g.cols = int(cols);
    g.py = int(std::min<int64_t>(PSIDE, rows));
    g.px = int(std::min<int64_t>(PSIDE, cols));
    g.my[0] = g.mx[0] = 0;
    for (int a = 0; a < PLAT; ++a) {
        // patch origins spread evenly, the first at the top/left edge and the last at the bottom/right
        g.y[a] = int(((rows - g.py) * a + (PLAT - 1) / 2) / (PLAT - 1));
        g.x[a] = int(((cols - g.px) * a + (PLAT - 1) / 2) / (PLAT - 1));
        const int64_t y0 = std::max<int64_t>(0, g.y[a] - K), y1 = std::min<int64_t>(rows, g.y[a] + g.py + K);
        const int64_t x0 = std::max<int64_t>(0, g.x[a] - K), x1 = std::min<int64_t>(cols, g.x[a] + g.px + K);
        g.wy[a] = int(y0);
        g.wx[a] = int(x0);
        g.my[a + 1] = int(g.my[a] + (y1 - y0));
        g.mx[a + 1] = int(g.mx[a] + (x1 - x0));
    }
    return g;
}

// workspace layout for a batch of nb fields of H x W
struct WsLayout {
    size_t frags, scale, scalep, act[5], z[5], dzb[2], dz1, dF, partial, lossp, total;
    int64_t npix;
    int nblk_px, nblk_rg;
};

WsLayout layout(int nb, int64_t H, int64_t W, bool train) {
    WsLayout L;
    L.npix = int64_t(nb) * H * W;
    L.nblk_px = int((L.npix + 255) / 256);
    L.nblk_rg = int(nb * ((H + RH - 1) / RH) * ((W + RW - 1) / RW));
    size_t off = 0;
    L.frags = off;
    off = a256(off + size_t(NFRAG) * 2);
    L.scale = off;
    off = a256(off + size_t(nb) * 2 * 4);
    L.scalep = off;
    off = a256(off + size_t(nb) * SCB * 8);
    const size_t actb = size_t(L.npix) * C * 2, zb = size_t(L.npix) * C * 4;
    for (int l = 0; l < 5; ++l) {
        if (train || l < 2) {
            L.act[l] = off;
            off = a256(off + actb);
        } else {
            L.act[l] = L.act[l % 2];  // inference ping-pongs two activation buffers
        }
    }
    for (int l = 0; l < 5; ++l) {
        if (train) {
            L.z[l] = off;
            off = a256(off + zb);
        } else {
            L.z[l] = 0;
        }
    }
    if (train) {
        L.dzb[0] = off;
        off = a256(off + actb);
        L.dzb[1] = off;
        off = a256(off + actb);
        L.dz1 = off;
        off = a256(off + zb);
        L.dF = off;
        off = a256(off + size_t(L.npix) * 4);
        L.partial = off;
        off = a256(off + size_t(L.nblk_rg) * (9 * C * C + C) * 4);
        L.lossp = off;
        off = a256(off + size_t(L.nblk_px) * 8);
    } else {
        L.dzb[0] = L.dzb[1] = L.dz1 = L.dF = L.partial = L.lossp = 0;
    }
    L.total = off;
    return L;
}

int check_dims(int nb, int64_t H, int64_t W) {
    if (nb < 1 || H < 1 || W < 1 || H > 32768 || W > 32768 || int64_t(nb) * H * W > (int64_t(1) << 31))
        return fail(ST_EINVAL, "bad surrogate batch/shape");
    return ST_OK;
}

// Grid of a persistent tile kernel: one workgroup per resident slot, at most one per tile.
int tile_grid(const void* fn, int nb, int H, int W, unsigned* grid) {
    int blocks = 0;
    if (int rc = resident_blocks(fn, 0, &blocks)) return rc;
    *grid = unsigned(std::min<int64_t>(tile_count(nb, H, W), blocks));
    return ST_OK;
}

template <int EPI>
int launch_conv(const ConvArgs& a, hipStream_t s) {
    unsigned grid = 0;
    if (int rc = tile_grid(reinterpret_cast<const void*>(conv_mfma<EPI>), a.nb, a.H, a.W, &grid)) return rc;
    hipLaunchKernelGGL(conv_mfma<EPI>, dim3(grid), dim3(256), 0, s, a);
    ST_LAUNCH_CHECK("conv_mfma");
    return ST_OK;
}

// The scale constants of nb fields of H x W (see field_scale_finish) into `scale`.
int compute_scale(const float* u0, int nb, int H, int W, double* partial, float* scale, hipStream_t s) {
    clear_stale_error();
    hipLaunchKernelGGL(field_scale_partial, dim3(SCB, nb), dim3(256), 0, s, u0, int64_t(H) * W, partial);
    ST_LAUNCH_CHECK("field_scale_partial");
    hipLaunchKernelGGL(field_scale_finish, dim3((nb + 63) / 64), dim3(64), 0, s, partial, nb, int64_t(H) * W, scale);
    ST_LAUNCH_CHECK("field_scale_finish");
    return ST_OK;
}

// Forward pass; `scale` holds the (inv, gain) pair of each field (device).
int forward_impl(const float* params, const float* u0, const float* kappa, const float* scale, float* uhat, int nb,
                 int H, int W, char* ws, const WsLayout& L, bool train, hipStream_t s) {
    uint16_t* frags = reinterpret_cast<uint16_t*>(ws + L.frags);
    clear_stale_error();
    hipLaunchKernelGGL(prep_frags, dim3((NFRAG + 255) / 256), dim3(256), 0, s, params, frags);
    ST_LAUNCH_CHECK("prep_frags");
    auto act = [&](int l) { return reinterpret_cast<uint16_t*>(ws + L.act[l]); };
    auto zz = [&](int l) { return train ? reinterpret_cast<float*>(ws + L.z[l]) : nullptr; };
    unsigned g1 = 0;
    if (int rc = tile_grid(reinterpret_cast<const void*>(l1_fwd), nb, H, W, &g1)) return rc;
    hipLaunchKernelGGL(l1_fwd, dim3(g1), dim3(256), 0, s, params, u0, kappa, scale, nb, H, W, zz(0), act(0));
    ST_LAUNCH_CHECK("l1_fwd");
    for (int l = 1; l <= 4; ++l) {
        ConvArgs a;
        a.X = act(l - 1);
        a.frags = frags + size_t(l - 1) * 2 * FRAG;
        a.bias = params + boff(l);
        a.Zprev = nullptr;
        a.Zout = zz(l);
        a.Aout = act(l);
        a.Fout = nullptr;
        a.nb = nb;
        a.H = H;
        a.W = W;
        if (int rc = launch_conv<EPI_FWD>(a, s)) return rc;
    }
    unsigned g6 = 0;
    if (int rc = tile_grid(reinterpret_cast<const void*>(l6_fwd), nb, H, W, &g6)) return rc;
    hipLaunchKernelGGL(l6_fwd, dim3(g6), dim3(256), 0, s, params, frags + 4 * 2 * FRAG, act(4), u0, scale, nb, H, W,
                       uhat);
    ST_LAUNCH_CHECK("l6_fwd");
    return ST_OK;
}

}  // namespace

}  // namespace st

using namespace st;

struct sg_model {
    uint32_t flags;
};

extern "C" {

int surrogate_create(sg_model** out, uint32_t flags) {
    if (!out) return fail(ST_EINVAL, "out is NULL");
    if (flags) return fail(ST_EINVAL, "no surrogate flags are defined");
    sg_model* m = new (std::nothrow) sg_model;
    if (!m) return fail(ST_ENOMEM, "model allocation failed");
    m->flags = flags;
    *out = m;
    return ST_OK;
}

int surrogate_destroy(sg_model* m) {
    delete m;
    return ST_OK;
}

int surrogate_param_bytes(const sg_model* m, size_t* params, size_t* optim_state) {
    if (!m) return fail(ST_EINVAL, "model is NULL");
    if (params) *params = size_t(SG_PARAM_COUNT) * sizeof(float);
    if (optim_state) *optim_state = size_t(2) * SG_PARAM_COUNT * sizeof(float);
    return ST_OK;
}

int surrogate_init(sg_model* m, float* params, float* optim_state, uint64_t seed, void* stream) {
    if (!m || !params) return fail(ST_EINVAL, "NULL argument");
    clear_stale_error();
    hipLaunchKernelGGL(init_params_kernel, dim3((SG_PARAM_COUNT + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), params, optim_state, seed);
    ST_LAUNCH_CHECK("init_params");
    return ST_OK;
}

int surrogate_workspace_bytes(const sg_model* m, int batch, int64_t rows, int64_t cols, size_t* bytes) {
    if (!m || !bytes) return fail(ST_EINVAL, "NULL argument");
    if (int rc = check_dims(batch, rows, cols)) return rc;
    *bytes = layout(batch, rows, cols, true).total;
    return ST_OK;
}

int surrogate_infer(sg_model* m, const float* params, const float* u0, const float* kappa, float* u_hat, int batch,
                      int64_t rows, int64_t cols, void* workspace, size_t ws_bytes, void* stream) {
    if (!m || !params || !u0 || !kappa || !u_hat) return fail(ST_EINVAL, "NULL argument");
    if (int rc = check_dims(batch, rows, cols)) return rc;
    const WsLayout L = layout(batch, rows, cols, false);
    if (!workspace || ws_bytes < L.total) return fail(ST_ENOWS, "workspace too small");
    char* ws = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* scale = reinterpret_cast<float*>(ws + L.scale);
    if (int rc = compute_scale(u0, batch, int(rows), int(cols), reinterpret_cast<double*>(ws + L.scalep), scale, s))
        return rc;
    return forward_impl(params, u0, kappa, scale, u_hat, batch, int(rows), int(cols), ws, L, false, s);
}

// Loss and gradient; `scale_in` = the (inv, gain) pair of each field (device), or NULL to take them
// from the fields given (their own RMS).
static int loss_grad_impl(const float* params, const float* u0, const float* kappa, const float* scale_in,
                          const float* target, const int* lo_hi, int batch, int64_t rows, int64_t cols, float* grad,
                          double* loss, void* workspace, size_t ws_bytes, void* stream) {
    if (int rc = check_dims(batch, rows, cols)) return rc;
    if (batch > MAXB) return fail(ST_EINVAL, "training batch larger than 64");
    MaskArgs mk;
    std::memset(&mk, 0, sizeof(mk));
    double n = 0.0;
    for (int b = 0; b < batch; ++b) {
        const int* m = lo_hi + 4 * b;
        mk.lohi[4 * b] = std::max(0, m[0]);
        mk.lohi[4 * b + 1] = std::min<int>(int(rows), m[1]);
        mk.lohi[4 * b + 2] = std::max(0, m[2]);
        mk.lohi[4 * b + 3] = std::min<int>(int(cols), m[3]);
        n += double(std::max(0, mk.lohi[4 * b + 1] - mk.lohi[4 * b])) *
             double(std::max(0, mk.lohi[4 * b + 3] - mk.lohi[4 * b + 2]));
    }
    if (n <= 0.0) return fail(ST_EINVAL, "empty loss mask");
    const WsLayout L = layout(batch, rows, cols, true);
    if (!workspace || ws_bytes < L.total) return fail(ST_ENOWS, "workspace too small");
    char* ws = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int H = int(rows), W = int(cols), nb = batch;
    const float* scale = scale_in;
    if (!scale) {
        float* sc = reinterpret_cast<float*>(ws + L.scale);
        if (int rc = compute_scale(u0, nb, H, W, reinterpret_cast<double*>(ws + L.scalep), sc, s)) return rc;
        scale = sc;
    }
    float* uhat = reinterpret_cast<float*>(ws + L.dz1);  // scratch: dz1 is not needed until layer-2 backward
    if (int rc = forward_impl(params, u0, kappa, scale, uhat, nb, H, W, ws, L, true, s)) return rc;
    float* dF = reinterpret_cast<float*>(ws + L.dF);
    double* lossp = reinterpret_cast<double*>(ws + L.lossp);
    const unsigned gpx = unsigned(L.nblk_px);
    hipLaunchKernelGGL(loss_grad, dim3(gpx), dim3(256), 0, s, uhat, target, scale, nb, H, W, mk, 1.0 / n, dF, lossp);
    ST_LAUNCH_CHECK("loss_grad");
    hipLaunchKernelGGL(loss_finish, dim3(1), dim3(256), 0, s, lossp, L.nblk_px, 1.0 / n, loss);
    ST_LAUNCH_CHECK("loss_finish");
    auto act = [&](int l) { return reinterpret_cast<uint16_t*>(ws + L.act[l]); };
    auto zz = [&](int l) { return reinterpret_cast<float*>(ws + L.z[l]); };
    float* partial = reinterpret_cast<float*>(ws + L.partial);
    const unsigned grg = unsigned(L.nblk_rg);
    // layer 6
    hipLaunchKernelGGL(l6_bwd_weight, dim3(grg), dim3(320), 0, s, act(4), dF, nb, H, W, partial);
    ST_LAUNCH_CHECK("l6_bwd_weight");
    hipLaunchKernelGGL(reduce_partials, dim3((9 * C + 1 + 63) / 64), dim3(64 * RP_WAVES), 0, s, partial, L.nblk_rg, 9 * C + 1,
                       grad + woff(5));
    ST_LAUNCH_CHECK("reduce l6");
    uint16_t* dzb[2] = {reinterpret_cast<uint16_t*>(ws + L.dzb[0]), reinterpret_cast<uint16_t*>(ws + L.dzb[1])};
    hipLaunchKernelGGL(l6_bwd_data, dim3(gpx), dim3(256), 0, s, params, dF, zz(4), nb, H, W, dzb[0]);
    ST_LAUNCH_CHECK("l6_bwd_data");
    // layers 5 .. 2 (index l = 4 .. 1): dZ_l in dzb[cur]
    const uint16_t* frags = reinterpret_cast<const uint16_t*>(ws + L.frags);
    int cur = 0;
    float* dz1 = reinterpret_cast<float*>(ws + L.dz1);
    for (int l = 4; l >= 1; --l) {
        hipLaunchKernelGGL(mfma_bwd_weight, dim3(grg), dim3(256), 0, s, act(l - 1), dzb[cur], nb, H, W, partial);
        ST_LAUNCH_CHECK("mfma_bwd_weight");
        hipLaunchKernelGGL(reduce_partials, dim3((9 * C * C + C + 63) / 64), dim3(64 * RP_WAVES), 0, s, partial, L.nblk_rg,
                           9 * C * C + C, grad + woff(l));
        ST_LAUNCH_CHECK("reduce mfma layer");
        ConvArgs a;
        a.X = dzb[cur];
        a.frags = frags + size_t(l - 1) * 2 * FRAG + FRAG;
        a.bias = nullptr;
        a.Zprev = zz(l - 1);
        a.Zout = nullptr;
        a.Aout = l > 1 ? dzb[cur ^ 1] : nullptr;
        a.Fout = l > 1 ? nullptr : dz1;
        a.nb = nb;
        a.H = H;
        a.W = W;
        if (int rc = l > 1 ? launch_conv<EPI_BWD_BF16>(a, s) : launch_conv<EPI_BWD_F32>(a, s)) return rc;
        cur ^= 1;
    }
    // layer 1
    hipLaunchKernelGGL(l1_bwd_weight, dim3(grg), dim3(640), 0, s, u0, kappa, scale, dz1, nb, H, W, partial);
    ST_LAUNCH_CHECK("l1_bwd_weight");
    hipLaunchKernelGGL(reduce_partials, dim3((9 * 2 * C + C + 63) / 64), dim3(64 * RP_WAVES), 0, s, partial, L.nblk_rg,
                       9 * 2 * C + C, grad + woff(0));
    ST_LAUNCH_CHECK("reduce l1");
    return ST_OK;
}

int surrogate_loss_grad(sg_model* m, const float* params, const float* u0, const float* kappa, const float* scale,
                        const float* target, const int* lo_hi, int batch, int64_t rows, int64_t cols, float* grad,
                        double* loss, void* workspace, size_t ws_bytes, void* stream) {
    if (!m || !params || !u0 || !kappa || !target || !lo_hi || !grad || !loss) return fail(ST_EINVAL, "NULL argument");
    return loss_grad_impl(params, u0, kappa, scale, target, lo_hi, batch, rows, cols, grad, loss, workspace, ws_bytes,
                          stream);
}

int surrogate_field_scale(const float* u0, int n, int64_t rows, int64_t cols, float* scale, void* workspace,
                          size_t ws_bytes, void* stream) {
    if (!u0 || !scale) return fail(ST_EINVAL, "NULL argument");
    if (int rc = check_dims(n, rows, cols)) return rc;
    if (!workspace || ws_bytes < size_t(n) * SCB * sizeof(double)) return fail(ST_ENOWS, "workspace too small");
    return compute_scale(u0, n, int(rows), int(cols), static_cast<double*>(workspace), scale,
                         static_cast<hipStream_t>(stream));
}

int surrogate_adam(sg_model* m, float* params, const float* grad, float* optim, int t, float lr, float beta1,
                   float beta2, float eps, void* stream) {
    if (!m || !params || !grad || !optim) return fail(ST_EINVAL, "NULL argument");
    if (t < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(ST_EINVAL, "bad Adam hyper-parameters");
    const float c1 = float(1.0 - std::pow(double(beta1), t)), c2 = float(1.0 - std::pow(double(beta2), t));
    clear_stale_error();
    hipLaunchKernelGGL(adam_kernel, dim3((SG_PARAM_COUNT + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       params, grad, optim, optim + SG_PARAM_COUNT, SG_PARAM_COUNT, lr, beta1, beta2, eps, c1, c2);
    ST_LAUNCH_CHECK("adam");
    return ST_OK;
}

int surrogate_synth_fields(const float* coef, int n, int64_t rows, int64_t cols, float* u0_out, float* kappa_out,
                           void* stream) {
    if (!coef || !u0_out || !kappa_out) return fail(ST_EINVAL, "NULL argument");
    if (n < 1 || rows < 1 || cols < 1 || int64_t(n) * rows * cols > (int64_t(1) << 33)) return fail(ST_EINVAL, "bad sizes");
    const int64_t blocks = int64_t(n) * ((rows + SY - 1) / SY) * ((cols + SX - 1) / SX);
    clear_stale_error();
    hipLaunchKernelGGL(synth_kernel, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream), coef, n,
                       int(rows), int(cols), u0_out, kappa_out);
    ST_LAUNCH_CHECK("synth");
    return ST_OK;
}

int surrogate_crop(const float* src, float* dst, const int* yx, int n, int64_t rows, int64_t cols, int64_t h, int64_t w,
                   void* stream) {
    if (!src || !dst || !yx) return fail(ST_EINVAL, "NULL argument");
    if (n < 1 || h < 1 || w < 1 || rows < 1 || cols < 1) return fail(ST_EINVAL, "bad sizes");
    const int64_t total = int64_t(n) * h * w;
    clear_stale_error();
    hipLaunchKernelGGL(crop_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       src, dst, yx, n, int(rows), int(cols), int(h), int(w));
    ST_LAUNCH_CHECK("crop");
    return ST_OK;
}

int surrogate_checked_ws_bytes(const sg_model* m, int64_t rows, int64_t cols, size_t* bytes) {
    if (!m || !bytes) return fail(ST_EINVAL, "NULL argument");
    if (int rc = check_dims(1, rows, cols)) return rc;
    const size_t field = a256(size_t(rows * cols) * 4);
    *bytes = layout(1, rows, cols, false).total + 3 * field + a256(1024 * 16) + 256;
    return ST_OK;
}

}  // extern "C"

namespace {

constexpr int COEF_ROW = 4 * (16 + 8);  // floats per trajectory's coefficient row
constexpr int RFIELD = 6;               // receptive-field radius of six 3x3 layers

struct TrainWs {
    size_t u0, kp, uk, cu0, ckp, cuk, grad, jws, yx, scale, scalep, sg, total;
    size_t field, crop, jws_bytes;
};

int train_layout(const sg_train_cfg* c, TrainWs* T) {
    if (!c) return fail(ST_EINVAL, "cfg is NULL");
    if (c->rows < 1 || c->cols < 1 || c->crop < 1 || c->crop > c->rows || c->crop > c->cols || c->batch < 1 ||
        c->batch > MAXB || c->K < 1 || c->steps < 0 || c->step0 < 0 || c->total_steps < c->step0 + c->steps ||
        !(c->lr >= 0.0f) || !(c->beta1 >= 0.0f && c->beta1 < 1.0f) || !(c->beta2 >= 0.0f && c->beta2 < 1.0f) ||
        !(c->eps > 0.0f))
        return fail(ST_EINVAL, "bad training configuration");
    if (int rc = check_dims(c->batch, c->rows, c->cols)) return rc;
    const int64_t B = c->batch;
    T->field = a256(size_t(B * c->rows * c->cols) * 4);
    T->crop = a256(size_t(B * c->crop * c->crop) * 4);
    T->jws_bytes = a256(size_t(c->rows * c->cols) * 4);
    size_t off = 0;
    T->u0 = off; off += T->field;
    T->kp = off; off += T->field;
    T->uk = off; off += T->field;
    T->cu0 = off; off += T->crop;
    T->ckp = off; off += T->crop;
    T->cuk = off; off += T->crop;
    T->grad = off; off += a256(size_t(SG_PARAM_COUNT) * 4);
    T->jws = off; off += T->jws_bytes;
    T->yx = off; off += a256(size_t(std::max<int64_t>(c->steps, 1) * B) * 8);
    T->scale = off; off += a256(size_t(B) * 2 * 4);
    T->scalep = off; off += a256(size_t(B) * SCB * 8);
    T->sg = off; off += layout(c->batch, c->crop, c->crop, true).total;
    T->total = off;
    return ST_OK;
}

}  // namespace

extern "C" {

int surrogate_train_ws_bytes(const sg_model* m, const sg_train_cfg* cfg, size_t* bytes) {
    if (!m || !bytes) return fail(ST_EINVAL, "NULL argument");
    TrainWs T;
    if (int rc = train_layout(cfg, &T)) return rc;
    *bytes = T.total;
    return ST_OK;
}

int surrogate_train(sg_model* m, float* params, float* optim, const float* coef, const int* crop_yx,
                    const sg_train_cfg* cfg, double* losses, void* workspace, size_t ws_bytes, void* stream) {
    if (!m || !params || !optim || !coef || !crop_yx || !losses) return fail(ST_EINVAL, "NULL argument");
    TrainWs T;
    if (int rc = train_layout(cfg, &T)) return rc;
    if (!workspace || ws_bytes < T.total) return fail(ST_ENOWS, "workspace too small");
    const sg_train_cfg c = *cfg;
    const int B = c.batch;
    const int64_t n = c.steps * B;
    for (int64_t i = 0; i < n; ++i) {
        const int y = crop_yx[2 * i], x = crop_yx[2 * i + 1];
        if (y < 0 || x < 0 || y + c.crop > c.rows || x + c.crop > c.cols) return fail(ST_EINVAL, "crop outside the grid");
    }
    if (c.steps == 0) return ST_OK;
    char* ws = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* U0 = reinterpret_cast<float*>(ws + T.u0);
    float* KP = reinterpret_cast<float*>(ws + T.kp);
    float* UK = reinterpret_cast<float*>(ws + T.uk);
    float* cu0 = reinterpret_cast<float*>(ws + T.cu0);
    float* ckp = reinterpret_cast<float*>(ws + T.ckp);
    float* cuk = reinterpret_cast<float*>(ws + T.cuk);
    float* grad = reinterpret_cast<float*>(ws + T.grad);
    int* yx = reinterpret_cast<int*>(ws + T.yx);
    ST_HIP_CHECK(hipMemcpyAsync(yx, crop_yx, size_t(n) * 8, hipMemcpyHostToDevice, s));
    // the judge: the plain stencil, as deep per pass as this device's LDS allows, on 128 x 32 tiles
    // (the fastest tile of the set for 1024^2 fields at depth 8; the result does not depend on it)
    st_plan* judge = nullptr;
    if (int rc = stencil_plan_varcoef(&judge, c.rows, c.cols, 0.0, 0)) return rc;
    for (int tb : {8, 4, 2, 1})
        if (stencil_set_blocking(judge, tb, 128, 32) == ST_OK) break;
    int rc = ST_OK;
    const int64_t field = c.rows * c.cols;
    for (int64_t st = 0; st < c.steps && rc == ST_OK; ++st) {
        if ((rc = surrogate_synth_fields(coef + st * B * COEF_ROW, B, c.rows, c.cols, U0, KP, stream))) break;
        for (int b = 0; b < B && rc == ST_OK; ++b)
            rc = stencil_run_varcoef(judge, U0 + b * field, KP + b * field, UK + b * field, c.K, ws + T.jws,
                                     T.jws_bytes, stream);
        if (rc) break;
        // the network's scale constants come from the whole trajectory field, as at inference
        float* scale = reinterpret_cast<float*>(ws + T.scale);
        if ((rc = compute_scale(U0, B, int(c.rows), int(c.cols), reinterpret_cast<double*>(ws + T.scalep), scale, s)))
            break;
        const int* yx_s = yx + 2 * st * B;
        if ((rc = surrogate_crop(U0, cu0, yx_s, B, c.rows, c.cols, c.crop, c.crop, stream))) break;
        if ((rc = surrogate_crop(KP, ckp, yx_s, B, c.rows, c.cols, c.crop, c.crop, stream))) break;
        if ((rc = surrogate_crop(UK, cuk, yx_s, B, c.rows, c.cols, c.crop, c.crop, stream))) break;
        int lohi[4 * MAXB];
        for (int b = 0; b < B; ++b) {
            const int y = crop_yx[2 * (st * B + b)], x = crop_yx[2 * (st * B + b) + 1];
            lohi[4 * b] = y > 0 ? RFIELD : 0;
            lohi[4 * b + 1] = int(c.crop) - (y + c.crop < c.rows ? RFIELD : 0);
            lohi[4 * b + 2] = x > 0 ? RFIELD : 0;
            lohi[4 * b + 3] = int(c.crop) - (x + c.crop < c.cols ? RFIELD : 0);
        }
        if ((rc = loss_grad_impl(params, cu0, ckp, scale, cuk, lohi, B, c.crop, c.crop, grad, losses + st, ws + T.sg,
                                 ws_bytes - T.sg, stream)))
            break;
        const int64_t g = c.step0 + st;
        const double lr = double(c.lr) * 0.5 * (1.0 + std::cos(3.14159265358979323846 * double(g) / double(c.total_steps)));
        rc = surrogate_adam(m, params, grad, optim, int(g + 1), float(lr), c.beta1, c.beta2, c.eps, stream);
    }
    // the judge's kernels are enqueued: destroying the host-side plan does not wait for them
    stencil_destroy(judge);
    return rc;
}

int surrogate_infer_checked(sg_model* m, const float* params, const float* u0, const float* kappa, float* out,
                            int64_t rows, int64_t cols, st_plan* judge, int64_t K, double tol, int judge_mode,
                            int* used_fallback, double* rel_err, void* workspace, size_t ws_bytes, void* stream) {
    if (!m || !params || !u0 || !kappa || !out || !judge || !used_fallback || !rel_err)
        return fail(ST_EINVAL, "NULL argument");
    if (judge->kind != KIND_VARCOEF || judge->rows != rows || judge->cols != cols)
        return fail(ST_EINVAL, "judge must be a varcoef plan of the same shape");
    if (K < 0 || !(tol >= 0.0)) return fail(ST_EINVAL, "bad K or tol");
    if (judge_mode != SG_JUDGE_FULL && judge_mode != SG_JUDGE_PATCH) return fail(ST_EINVAL, "unknown judge mode");
    size_t need = 0;
    if (int rc = surrogate_checked_ws_bytes(m, rows, cols, &need)) return rc;
    if (!workspace || ws_bytes < need) return fail(ST_ENOWS, "workspace too small");
    char* ws = static_cast<char*>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const WsLayout L = layout(1, rows, cols, false);
    const size_t field = a256(size_t(rows * cols) * 4);
    float* uhat = reinterpret_cast<float*>(ws + L.total);
    float* b1 = reinterpret_cast<float*>(ws + L.total + field);
    float* b2 = reinterpret_cast<float*>(ws + L.total + 2 * field);
    double* part = reinterpret_cast<double*>(ws + L.total + 3 * field);
    double* sums = reinterpret_cast<double*>(ws + L.total + 3 * field + a256(1024 * 16));
    float* scale = reinterpret_cast<float*>(ws + L.scale);
    if (int rc = compute_scale(u0, 1, int(rows), int(cols), reinterpret_cast<double*>(ws + L.scalep), scale, s))
        return rc;
    if (int rc = forward_impl(params, u0, kappa, scale, uhat, 1, int(rows), int(cols), ws, L, false, s)) return rc;
    const int64_t n = rows * cols;
    // the patch judge needs its four mosaic fields in the two spare fields (else judge the whole field)
    const MosaicArgs g = mosaic_layout(rows, cols, K);
    const int64_t mcells = int64_t(g.my[g.n]) * g.mx[g.n];
    const bool patch = judge_mode == SG_JUDGE_PATCH && 2 * a256(size_t(mcells) * 4) <= field;
    bool full_done = false;
    if (patch) {
        const size_t mf = a256(size_t(mcells) * 4);
        float* mu = b1;
        float* mk = reinterpret_cast<float*>(reinterpret_cast<char*>(b1) + mf);
        float* mo = b2;
        float* mw = reinterpret_cast<float*>(reinterpret_cast<char*>(b2) + mf);
        clear_stale_error();
        hipLaunchKernelGGL(gather_mosaic, dim3(unsigned((mcells + 255) / 256)), dim3(256), 0, s, u0, kappa, g, mu, mk);
        ST_LAUNCH_CHECK("gather_mosaic");
        st_plan* mp = nullptr;
        if (int rc = stencil_plan_varcoef(&mp, g.my[g.n], g.mx[g.n], judge->b, 0)) return rc;
        int tb = judge->tb, tx = judge->tile_x, ty = judge->tile_y;
        while (tb > 1 && stencil_set_blocking(mp, tb, tx, ty) != ST_OK) --tb;
        int rc = stencil_run_varcoef(mp, mu, mk, mo, K, mw, mf, stream);
        stencil_destroy(mp);  // host-side only: the enqueued kernels keep their arguments
        if (rc) return rc;
        hipLaunchKernelGGL(patch_norms, dim3(g.n * g.n), dim3(256), 0, s, uhat, mo, g, part);
        ST_LAUNCH_CHECK("patch_norms");
        hipLaunchKernelGGL(diff_norms_finish, dim3(1), dim3(64), 0, s, part, g.n * g.n, sums);
        ST_LAUNCH_CHECK("diff_norms_finish");
    } else {
        // the whole field: K plain steps
        if (int rc = stencil_run_varcoef(judge, u0, kappa, b1, K, b2, field, stream)) return rc;
        full_done = true;
        const int nblk = int(std::min<int64_t>(1024, (n + 255) / 256));
        clear_stale_error();
        hipLaunchKernelGGL(diff_norms, dim3(nblk), dim3(256), 0, s, uhat, b1, n, part);
        ST_LAUNCH_CHECK("diff_norms");
        hipLaunchKernelGGL(diff_norms_finish, dim3(1), dim3(64), 0, s, part, nblk, sums);
        ST_LAUNCH_CHECK("diff_norms_finish");
    }
    double h[2] = {0, 0};
    ST_HIP_CHECK(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s));
    ST_HIP_CHECK(hipStreamSynchronize(s));
    const int64_t judged = patch ? int64_t(g.n) * g.n * g.py * g.px : n;
    const double rel = h[1] > 1e-60 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0] / double(judged));
    *rel_err = rel;
    const bool fallback = !(rel <= tol);
    *used_fallback = fallback ? 1 : 0;
    if (!fallback) {
        ST_HIP_CHECK(hipMemcpyAsync(out, uhat, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
    } else if (full_done) {
        ST_HIP_CHECK(hipMemcpyAsync(out, b1, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
    } else {
        if (int rc = stencil_run_varcoef(judge, u0, kappa, out, K, b1, field, stream)) return rc;
    }
    return ST_OK;
}

}  // extern "C"
