// Storage formats of a field and their exact widening to / rounding from FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/mi355stencil.h"

namespace st {

template <int S>
struct Fmt;

template <>
struct Fmt<ST_F32> {
    using T = float;
    static constexpr int VEC = 4;  // elements per 16-byte chunk
    __device__ __forceinline__ static float ld(T v) { return v; }
    __device__ __forceinline__ static T st(float x) { return x; }
    __device__ __forceinline__ static float rnd(float x) { return x; }
};

// Storing a 16-bit cell rounds the finished FP32 value (round to nearest even), i.e. two roundings
// when the value is the result of an FMA.  Left alone, the compiler may fuse that last FMA with the
// FP16 conversion into one mixed-precision FMA that rounds once, straight to FP16, which differs in
// about one cell per thousand; the empty register constraint below keeps the FP32 value as written.
__device__ __forceinline__ float as_fp32(float x) {
    asm volatile("" : "+v"(x));
    return x;
}

typedef float F32x2 __attribute__((ext_vector_type(2)));

// bfloat16: the upper 16 bits of a binary32; widening is a shift, rounding is
// gfx950's hardware convert (round to nearest even).  Pairs convert in one
// instruction (a in the low half), the same rounding as one at a time.
template <>
struct Fmt<ST_BF16> {
    using T = uint16_t;
    static constexpr int VEC = 8;
    __device__ __forceinline__ static float ld(T v) { return __uint_as_float(uint32_t(v) << 16); }
    __device__ __forceinline__ static T st(float x) {
        __bf16 h = (__bf16)as_fp32(x);
        return __builtin_bit_cast(uint16_t, h);
    }
    __device__ __forceinline__ static float rnd(float x) { return ld(st(x)); }
    __device__ __forceinline__ static uint32_t st2(float a, float b) {
        typedef __bf16 B2 __attribute__((ext_vector_type(2)));
        const F32x2 v = {as_fp32(a), as_fp32(b)};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, B2));
    }
    __device__ __forceinline__ static void rnd2(float& a, float& b) {
        const uint32_t p = st2(a, b);
        a = __uint_as_float(p << 16);
        b = __uint_as_float(p & 0xffff0000u);
    }
};

// IEEE binary16 with subnormals; hardware convert, round to nearest even.  Pairs
// convert in one instruction (a in the low half), the same rounding.
template <>
struct Fmt<ST_F16> {
    using T = uint16_t;
    static constexpr int VEC = 8;
    // (the widened value is kept as an FP32 register: left alone, the compiler folds the widening
    // into mixed-precision FMAs, which measured slower on gfx950 and save no instruction: the row is
    // widened for the later rows' taps anyway)
    __device__ __forceinline__ static float ld(T v) {
        float x = (float)__builtin_bit_cast(_Float16, v);
        asm("" : "+v"(x));
        return x;
    }
    __device__ __forceinline__ static T st(float x) {
        _Float16 h = (_Float16)as_fp32(x);
        return __builtin_bit_cast(uint16_t, h);
    }
    __device__ __forceinline__ static float rnd(float x) { return ld(st(x)); }
    __device__ __forceinline__ static uint32_t st2(float a, float b) {
        typedef _Float16 H2 __attribute__((ext_vector_type(2)));
        const F32x2 v = {as_fp32(a), as_fp32(b)};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, H2));
    }
    __device__ __forceinline__ static void rnd2(float& a, float& b) {
        const uint32_t p = st2(a, b);
        a = ld(uint16_t(p & 0xffffu));
        b = ld(uint16_t(p >> 16));
    }
};

// Load one 16-byte chunk (VEC elements) and widen to FP32.
template <int S>
__device__ __forceinline__ void load_chunk(const typename Fmt<S>::T* p, float* v);

template <>
__device__ __forceinline__ void load_chunk<ST_F32>(const float* p, float* v) {
    float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}

template <int S>
__device__ __forceinline__ void load_chunk16(const uint16_t* p, float* v) {
    uint4 q = *reinterpret_cast<const uint4*>(p);
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = Fmt<S>::ld(uint16_t(w[k] & 0xffffu));
        v[2 * k + 1] = Fmt<S>::ld(uint16_t(w[k] >> 16));
    }
}

template <>
__device__ __forceinline__ void load_chunk<ST_BF16>(const uint16_t* p, float* v) { load_chunk16<ST_BF16>(p, v); }
template <>
__device__ __forceinline__ void load_chunk<ST_F16>(const uint16_t* p, float* v) { load_chunk16<ST_F16>(p, v); }

// Widen one raw 16-byte chunk (VEC elements) to FP32.
template <int S>
__device__ __forceinline__ void widen_chunk(uint4 q, float* v);

template <>
__device__ __forceinline__ void widen_chunk<ST_F32>(uint4 q, float* v) {
    v[0] = __uint_as_float(q.x); v[1] = __uint_as_float(q.y); v[2] = __uint_as_float(q.z); v[3] = __uint_as_float(q.w);
}

template <int S>
__device__ __forceinline__ void widen_chunk16(uint4 q, float* v) {
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = Fmt<S>::ld(uint16_t(w[k] & 0xffffu));
        v[2 * k + 1] = Fmt<S>::ld(uint16_t(w[k] >> 16));
    }
}
template <>
__device__ __forceinline__ void widen_chunk<ST_BF16>(uint4 q, float* v) { widen_chunk16<ST_BF16>(q, v); }
template <>
__device__ __forceinline__ void widen_chunk<ST_F16>(uint4 q, float* v) { widen_chunk16<ST_F16>(q, v); }

// Store 4 consecutive FP32 values (rounded to the storage type) with one vector store.
template <int S>
__device__ __forceinline__ void store4(typename Fmt<S>::T* p, const float* v);

template <>
__device__ __forceinline__ void store4<ST_F32>(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}

template <int S>
__device__ __forceinline__ void store4_16(uint16_t* p, const float* v) {
    uint32_t a = uint32_t(Fmt<S>::st(v[0])) | (uint32_t(Fmt<S>::st(v[1])) << 16);
    uint32_t b = uint32_t(Fmt<S>::st(v[2])) | (uint32_t(Fmt<S>::st(v[3])) << 16);
    *reinterpret_cast<uint2*>(p) = make_uint2(a, b);
}
template <>
__device__ __forceinline__ void store4<ST_BF16>(uint16_t* p, const float* v) { store4_16<ST_BF16>(p, v); }
template <>
__device__ __forceinline__ void store4<ST_F16>(uint16_t* p, const float* v) { store4_16<ST_F16>(p, v); }

}  // namespace st
