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
};

} // namespace ptrt
