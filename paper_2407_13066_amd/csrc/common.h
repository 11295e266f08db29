// Device-side helpers shared by the btoep HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace btoep {

constexpr int kWave = 64;

// Complex value with real type T (float or double).  Plain POD so that arrays
// of it have the interleaved (re, im) layout of the stored operator.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

// BF16 complex: low 16 bits = real part, high 16 bits = imaginary part.
struct alignas(4) bf16c {
    uint32_t bits;
};

template <typename T>
__device__ __forceinline__ cx<T> cmake(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return cx<T>{a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return cx<T>{a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return cx<T>{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return cx<T>{a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return cx<T>{a.re * s, a.im * s}; }
// multiply by +i (sgn > 0) or -i (sgn < 0)
template <int SGN, typename T>
__device__ __forceinline__ cx<T> cmul_i(cx<T> a) {
    return SGN > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}
// acc += a * b
template <typename T>
__device__ __forceinline__ void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cfmac(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}

__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }

// float -> bf16 bits, round to nearest even (finite inputs; NaN kept quiet).
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// Conversions of a complex value into each storage type.
template <typename S>
struct Store;
template <>
struct Store<cx<double>> {
    __device__ static cx<double> from(cx<double> v) { return v; }
};
template <>
struct Store<cx<float>> {
    __device__ static cx<float> from(cx<double> v) { return cx<float>{(float)v.re, (float)v.im}; }
};
template <>
struct Store<bf16c> {
    // Round a double to the nearest bf16 (8 significant bits), ties to even, in one step:
    // round the 52-bit double mantissa to 7 stored bits, then the result is exact in float.
    __device__ static uint32_t one(double x) {
        uint64_t u = (uint64_t)__double_as_longlong(x);
        if (((u >> 52) & 0x7ffu) == 0x7ffu) return f32_to_bf16_rne((float)x);  // inf / nan
        u += (1ull << 44) - 1ull + ((u >> 45) & 1ull);
        u &= ~((1ull << 45) - 1ull);
        return __float_as_uint((float)__longlong_as_double((long long)u)) >> 16;
    }
    __device__ static bf16c from(cx<double> v) { return bf16c{one(v.re) | (one(v.im) << 16)}; }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace btoep
