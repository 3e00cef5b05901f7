// Storage codecs for the population array.
//
// The array holds h_a = f_a - w_a (deviation from the rest-state weights) in
// one of four formats; arithmetic runs in FP64 for the FP64 store and in FP32
// for the others.  Narrowing conversions round to nearest, ties to even.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmwf {

enum StoreKind { kStoreF64 = 0, kStoreF32 = 1, kStoreF16 = 2, kStoreBF16 = 3 };

struct StoreF64 {
    using T = double;
    using R = double;
    static constexpr int kind = kStoreF64;
    __device__ __forceinline__ static R load(const T* p) { return *p; }
    __device__ __forceinline__ static void store(T* p, R v) { *p = v; }
    __device__ __forceinline__ static T from_double(double v) { return v; }
    __device__ __forceinline__ static double to_double(T v) { return v; }
};

struct StoreF32 {
    using T = float;
    using R = float;
    static constexpr int kind = kStoreF32;
    __device__ __forceinline__ static R load(const T* p) { return *p; }
    __device__ __forceinline__ static void store(T* p, R v) { *p = v; }
    __device__ __forceinline__ static T from_double(double v) { return (float)v; }
    __device__ __forceinline__ static double to_double(T v) { return (double)v; }
};

struct StoreF16 {
    using T = _Float16;
    using R = float;
    static constexpr int kind = kStoreF16;
    __device__ __forceinline__ static R load(const T* p) { return (float)*p; }
    __device__ __forceinline__ static void store(T* p, R v) { *p = (_Float16)v; }
    __device__ __forceinline__ static T from_double(double v) { return (_Float16)v; }
    __device__ __forceinline__ static double to_double(T v) { return (double)(float)v; }
};

// bfloat16 kept as raw bits: the upper half of an IEEE binary32.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

struct StoreBF16 {
    using T = uint16_t;
    using R = float;
    static constexpr int kind = kStoreBF16;
    __device__ __forceinline__ static R load(const T* p) { return bf16_to_f32(*p); }
    __device__ __forceinline__ static void store(T* p, R v) { *p = f32_to_bf16_rne(v); }
    __device__ __forceinline__ static T from_double(double v) { return f32_to_bf16_rne((float)v); }
    __device__ __forceinline__ static double to_double(T v) { return (double)bf16_to_f32(v); }
};

inline int store_bytes(int kind) { return kind == kStoreF64 ? 8 : kind == kStoreF32 ? 4 : 2; }

}  // namespace lbmwf
