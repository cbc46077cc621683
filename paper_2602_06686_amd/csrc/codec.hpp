// Storage types of the shifted populations h_i = f_i - w_i and their
// conversion to the compute type.  FP16 and BF16 round to nearest even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptrt {

using bf16_t = __bf16;

template <class S>
struct Codec;

template <>
struct Codec<double> {
    using compute = double;
    static constexpr int bytes = 8;
    __device__ __forceinline__ static double load(const double *p) { return *p; }
    __device__ __forceinline__ static double to_double(double v) { return v; }
    template <bool NT = false>
    __device__ __forceinline__ static void store(double *p, double v)
    {
        if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
    }
};

template <>
struct Codec<float> {
    using compute = float;
    static constexpr int bytes = 4;
    __device__ __forceinline__ static float load(const float *p) { return *p; }
    template <bool NT = false>
    __device__ __forceinline__ static void store(float *p, float v)
    {
        if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
    }
};

template <>
struct Codec<_Float16> {
    using compute = float;
    static constexpr int bytes = 2;
    __device__ __forceinline__ static float load(const _Float16 *p) { return (float)*p; }
    template <bool NT = false>
    __device__ __forceinline__ static void store(_Float16 *p, float v)
    {
        const _Float16 hv = (_Float16)v;
        if constexpr (NT) __builtin_nontemporal_store(hv, p); else *p = hv;
    }
};

template <>
struct Codec<bf16_t> {
    using compute = float;
    static constexpr int bytes = 2;
    __device__ __forceinline__ static float load(const bf16_t *p) { return (float)*p; }
    // the conversion compiles to the gfx950 float -> bf16 instruction, which
    // rounds to nearest even and keeps NaN a NaN
    template <bool NT = false>
    __device__ __forceinline__ static void store(bf16_t *p, float v)
    {
        const bf16_t b = (bf16_t)v;
        if constexpr (NT) __builtin_nontemporal_store(b, p); else *p = b;
    }
};

// FP64 read of a stored value (gathers and diagnostics report in FP64).
template <class S>
__device__ __forceinline__ double load_f64(const S *p)
{
    return (double)Codec<S>::load(p);
}

// Store of an FP64 value: rounded once, directly from FP64, for FP64 and
// FP32 storage; FP16/BF16 go through FP32 first.
template <class S>
__device__ __forceinline__ void store_f64(S *p, double v)
{
    if constexpr (sizeof(S) >= 4)
        *p = (S)v;
    else
        Codec<S>::template store<false>(p, (float)v);
}

} // namespace ptrt
