// Storage formats of the SRJ device kernels and their load/store conversions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace srj {

struct bf16_t {
    uint16_t v;
};

template <class S> struct Tr;
template <> struct Tr<double> {
    using C = double;
    static __device__ __forceinline__ double ld(double x) { return x; }
    static __device__ __forceinline__ double st(double x) { return x; }
    static __device__ __forceinline__ double from64(double x) { return x; }
};
template <> struct Tr<float> {
    using C = float;
    static __device__ __forceinline__ float ld(float x) { return x; }
    static __device__ __forceinline__ float st(float x) { return x; }
    static __device__ __forceinline__ float from64(double x) { return (float)x; }
};
template <> struct Tr<bf16_t> {
    using C = float;
    static __device__ __forceinline__ float ld(bf16_t x) { return __uint_as_float((uint32_t)x.v << 16); }
    static __device__ __forceinline__ bf16_t st(float f)
    {
        // round to nearest, ties to even (gfx950 converts in one instruction, subnormals
        // kept); NaN stays a NaN
        bf16_t r;
        r.v = __builtin_bit_cast(uint16_t, (__bf16)f);
        return r;
    }
    static __device__ __forceinline__ bf16_t from64(double x) { return st((float)x); }
};

template <class S> __device__ __forceinline__ S zero_of();
template <> __device__ __forceinline__ double zero_of<double>() { return 0.0; }
template <> __device__ __forceinline__ float zero_of<float>() { return 0.0f; }
template <> __device__ __forceinline__ bf16_t zero_of<bf16_t>() { return bf16_t{0}; }


#define SRJ_DISPATCH(f, KCALL)                               \
    switch (f) {                                             \
    case FMT_F64: { using S = double; KCALL; break; }        \
    case FMT_F32: { using S = float; KCALL; break; }         \
    default: { using S = bf16_t; KCALL; break; }             \
    }

}  // namespace srj
