// Storage types of the shifted populations h_i = f_i - w_i and their
// conversion to the compute type.  FP16 and BF16 round to nearest even;
// their stochastic-rounding variants (f16sr_t, bf16sr_t: the same bits in
// memory) round each store up or down with the probability given by its
// distance to the two neighbours.  fast_recip: the collision takes 1 / rho
// from the refined hardware reciprocal (FP32 storage, whose two-step passes
// are bound by instruction issue); the 16-bit types keep the correctly
// rounded division (their one-step kernels are bound by HBM, and their
// rounding stays as measured for the precision form).
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
    static constexpr bool fast_recip = false;
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
    static constexpr bool fast_recip = true;
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
    static constexpr bool fast_recip = false;
    static constexpr int bytes = 2;
    __device__ __forceinline__ static float load(const _Float16 *p) { return (float)*p; }
    template <bool NT = false>
    __device__ __forceinline__ static void store(_Float16 *p, float v)
    {
        const _Float16 hv = (_Float16)v;
        if constexpr (NT) __builtin_nontemporal_store(hv, p); else *p = hv;
    }
    __device__ __forceinline__ static void store_nearest(_Float16 *p, float v) { *p = (_Float16)v; }
};

template <>
struct Codec<bf16_t> {
    using compute = float;
    static constexpr bool fast_recip = false;
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
    __device__ __forceinline__ static void store_nearest(bf16_t *p, float v) { *p = (bf16_t)v; }
};

// Stochastic rounding to a 16-bit format: a value between two neighbours
// of the target rounds to the upper one (in magnitude) with probability
// equal to its distance from the lower one in units of their gap.  Random
// bits are added to the FP32 bit pattern below the target's last mantissa
// bit and those bits are then cut off, so the carry into the kept bits
// (and across a binade) happens with exactly that probability; the result
// then converts exactly.  The random bits come from the value's own bits
// (sr_bits): deterministic (the same value always rounds the same way),
// while a value that changes from one step to the next draws new ones.
// No branches: the stores of a step are not held up by divergent lanes.

// Random bits: the value's bits times an odd constant, modulo 2^32
// (multiplicative hashing), read from the top: for a fixed pattern of the
// bits to be cut off, the top bits vary uniformly with the kept bits, so
// over the values of a lattice the round-up frequency of each pattern is
// its distance from the lower neighbour (unbiased); an exactly
// representable value has nothing to cut and stays as it is.
__device__ __forceinline__ unsigned sr_bits(unsigned b)
{
    return b * 0x9E3779B1u;
}

// FP16 (10 mantissa bits, normal from 2^-14): 13 bits cut off in the
// normal range; below 2^-14 the gap is 2^-24 throughout, so a uniform
// dither of one gap before the round to nearest does the same there.
// Non-finite values pass unchanged; finite ones beyond the FP16 range
// become infinite in the conversion.
__device__ __forceinline__ float sr_to_f16_grid(float v)
{
    const unsigned b = __float_as_uint(v), a = b & 0x7FFFFFFFu, h = sr_bits(b);
    const float cut = __uint_as_float((b + (h >> 19)) & ~0x1FFFu);
    const float dith = fmaf((float)(h >> 8) * 0x1p-24f - 0.5f, 0x1p-24f, v);
    return a >= 0x7F800000u ? v : (a >= 0x38800000u ? cut : dith);
}

// BF16 (the FP32 exponent range, 7 mantissa bits): 16 bits cut off for
// every finite value, subnormals included.
__device__ __forceinline__ float sr_to_bf16_grid(float v)
{
    const unsigned b = __float_as_uint(v);
    const float cut = __uint_as_float((b + (sr_bits(b) >> 16)) & 0xFFFF0000u);
    return (b & 0x7FFFFFFFu) >= 0x7F800000u ? v : cut;
}

struct f16sr_t {
    _Float16 v;
};
struct bf16sr_t {
    bf16_t v;
};

template <>
struct Codec<f16sr_t> {
    using compute = float;
    static constexpr bool fast_recip = false;
    static constexpr int bytes = 2;
    __device__ __forceinline__ static float load(const f16sr_t *p) { return (float)p->v; }
    template <bool NT = false>
    __device__ __forceinline__ static void store(f16sr_t *p, float v)
    {
        const _Float16 hv = (_Float16)sr_to_f16_grid(v);
        if constexpr (NT) __builtin_nontemporal_store(hv, &p->v); else p->v = hv;
    }
    __device__ __forceinline__ static void store_nearest(f16sr_t *p, float v) { p->v = (_Float16)v; }
};

template <>
struct Codec<bf16sr_t> {
    using compute = float;
    static constexpr bool fast_recip = false;
    static constexpr int bytes = 2;
    __device__ __forceinline__ static float load(const bf16sr_t *p) { return (float)p->v; }
    template <bool NT = false>
    __device__ __forceinline__ static void store(bf16sr_t *p, float v)
    {
        const bf16_t b = (bf16_t)sr_to_bf16_grid(v);
        if constexpr (NT) __builtin_nontemporal_store(b, &p->v); else p->v = b;
    }
    __device__ __forceinline__ static void store_nearest(bf16sr_t *p, float v) { p->v = (bf16_t)v; }
};

// FP64 read of a stored value (gathers and diagnostics report in FP64).
template <class S>
__device__ __forceinline__ double load_f64(const S *p)
{
    return (double)Codec<S>::load(p);
}

// Store of an FP64 value (initial state, checkpoint): rounded once,
// directly from FP64, for FP64 and FP32 storage; FP16/BF16 go through FP32
// first and round to nearest in every variant.
template <class S>
__device__ __forceinline__ void store_f64(S *p, double v)
{
    if constexpr (sizeof(S) >= 4)
        *p = (S)v;
    else
        Codec<S>::store_nearest(p, (float)v);
}

} // namespace ptrt
