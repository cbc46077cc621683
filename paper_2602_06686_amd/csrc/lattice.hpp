// Velocity sets of the P-TRT kernels, in the population order of the C
// interface (include/ptrt.h).  Everything here is a compile-time constant so
// that the fully unrolled per-direction code folds every e_i, w_i and
// opposite index into immediates.
#pragma once

#include <utility>

namespace ptrt {

// Call f(std::integral_constant<int, I>{}) for I = 0 .. N-1 at compile time.
template <class F, int... I>
__host__ __device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(static_cast<F &&>(f), std::make_integer_sequence<int, N>{});
}

// The coefficients c_i = 3 w_i of the first-order equilibrium term
// (3 w_i rho e_i.u) in a compute type C.  Rounded one by one, the c_i would
// give sum_i c_i e_ia e_ib = delta_ab (1 + d) with a rounding residue d, so
// the equilibrium's first moment would be rho u (1 + d) and every collision
// would rescale the momentum by a fixed factor: a bias that accumulates
// linearly and, in FP32 with tau+ near 1/2, dominates the velocity error
// (64^3 vortex at Re = 1600, 500 steps, against FP64: 8.1e-6 with
// independently rounded weights, 2.4e-6 with these, on the GPU; a CPU
// model of the same update with FP64 arithmetic and FP32 storage: 7e-8).
// So one class of c_i is rounded and the other is solved from the identity
// sum_i c_i e_ix^2 = 1 with operations that are exact in C (a subtraction of
// two numbers within a factor two of each other, products and quotients by
// powers of two); the identity then holds exactly for the rounded values.
template <class C>
__host__ __device__ constexpr C round_to_bits(double v, int bits)
{
    // v in (0, 1), rounded to `bits` significant bits
    double s = 1.0;
    while (v * s < (double)(1LL << (bits - 1))) s *= 2.0;
    return C((double)(long long)(v * s + 0.5) / s);
}

template <class C>
__host__ __device__ constexpr int mantissa_bits()
{
    return sizeof(C) == 8 ? 53 : 24;
}

// D2Q9, Eq. D2Q9 of the paper in its printed order.  Inversion pairs are
// listed by their first member (the one with the larger e.(1, 1/2)); the
// second member is opp(first).  Pair classes: 0 = axial, 1 = diagonal.
struct D2Q9 {
    static constexpr int Q = 9, D = 2, NP = 4;
    __host__ __device__ static constexpr int ex(int i)
    {
        constexpr int t[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i)
    {
        constexpr int t[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr int opp(int i)
    {
        constexpr int t[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        return t[i];
    }
    __host__ __device__ static constexpr int pair_first(int p)
    {
        constexpr int t[4] = {1, 2, 5, 6};
        return t[p];
    }
    __host__ __device__ static constexpr int pair_class(int p) { return p < 2 ? 0 : 1; }
    __host__ __device__ static constexpr double w(int i)
    {
        return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    // 3 w: axial 1/3 rounded, diagonal (1 - 2 c_axial) / 4, so 2 c_a + 4 c_d = 1
    template <class C>
    __host__ __device__ static constexpr C c1(int i)
    {
        constexpr C ca = C(1.0 / 3.0);
        constexpr C cd = (C(1) - C(2) * ca) / C(4);
        return i == 0 ? C(0) : (i <= 4 ? ca : cd);
    }
};

// D3Q19 (App. A.2): rest; +x -x +y -y +z -z; the four diagonals of the xy,
// xz and yz planes, each followed by its opposite.  Weights 1/3, 1/18, 1/36.
struct D3Q19 {
    static constexpr int Q = 19, D = 3, NP = 9;
    __host__ __device__ static constexpr int ex(int i)
    {
        constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i)
    {
        constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int i)
    {
        constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr int opp(int i)
    {
        return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
    }
    __host__ __device__ static constexpr int pair_first(int p) { return 2 * p + 1; }
    __host__ __device__ static constexpr int pair_class(int p) { return p < 3 ? 0 : 1; }
    __host__ __device__ static constexpr double w(int i)
    {
        return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    // 3 w: diagonal 1/12 rounded, axial (1 - 8 c_d) / 2, so 2 c_a + 8 c_d = 1
    template <class C>
    __host__ __device__ static constexpr C c1(int i)
    {
        constexpr C cd = C(1.0 / 12.0);
        constexpr C ca = (C(1) - C(8) * cd) / C(2);
        return i == 0 ? C(0) : (i <= 6 ? ca : cd);
    }
};

// D3Q27 (App. A.3): the D3Q19 set followed by the eight body diagonals
// (1,1,1) (-1,-1,-1) (1,1,-1) (-1,-1,1) (1,-1,1) (-1,1,-1) (-1,1,1) (1,-1,-1).
// Weights 8/27, 2/27, 1/54, 1/216.  Pair classes: 0 axial, 1 face, 2 body.
struct D3Q27 {
    static constexpr int Q = 27, D = 3, NP = 13;
    __host__ __device__ static constexpr int ex(int i)
    {
        constexpr int t[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                               1, -1, 1, -1, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i)
    {
        constexpr int t[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                               1, -1, 1, -1, -1, 1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int i)
    {
        constexpr int t[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                               1, -1, -1, 1, 1, -1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int opp(int i)
    {
        return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
    }
    __host__ __device__ static constexpr int pair_first(int p) { return 2 * p + 1; }
    __host__ __device__ static constexpr int pair_class(int p) { return p < 3 ? 0 : (p < 9 ? 1 : 2); }
    __host__ __device__ static constexpr double w(int i)
    {
        return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
    }
    // 3 w: face 1/18 rounded to three bits fewer than the type holds, body
    // c_f / 4, axial (1 - (8 c_f + 8 c_b)) / 2 (8 c_f + 2 c_f is then exact),
    // so 2 c_a + 8 c_f + 8 c_b = 1
    template <class C>
    __host__ __device__ static constexpr C c1(int i)
    {
        constexpr C cf = round_to_bits<C>(1.0 / 18.0, mantissa_bits<C>() - 3);
        constexpr C cb = cf / C(4);
        constexpr C ca = (C(1) - (C(8) * cf + C(8) * cb)) / C(2);
        return i == 0 ? C(0) : (i <= 6 ? ca : (i <= 18 ? cf : cb));
    }
};

// The first-moment identity of the rounded coefficients (exact: each sum
// below is of values representable in double, so double arithmetic does not
// round it).
static_assert(2.0 * (double)D2Q9::c1<float>(1) + 4.0 * (double)D2Q9::c1<float>(5) == 1.0, "D2Q9 c1");
static_assert(2.0 * (double)D3Q19::c1<float>(1) + 8.0 * (double)D3Q19::c1<float>(7) == 1.0,
              "D3Q19 c1");
static_assert(2.0 * (double)D3Q27::c1<float>(1) + 8.0 * (double)D3Q27::c1<float>(7) +
                      8.0 * (double)D3Q27::c1<float>(19) ==
                  1.0,
              "D3Q27 c1");

} // namespace ptrt
