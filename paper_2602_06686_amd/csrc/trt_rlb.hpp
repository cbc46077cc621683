// TRT-RLB collision (arXiv 2602.06686, Sec. 2.2, Eq. TRT-RLB) evaluated the
// way the paper describes its cost: explicit Hermite projection of the
// non-equilibrium part (Eq. projection) and reconstruction (Eq.
// R2R3_hermite).  It is the comparison model for the P-TRT kernels: the
// paper's equivalence theorems make its post-collision state equal to
// P-TRT's (Remark on exactness), and its efficiency table compares the two.
//
//   h*_i = heq_i + (1 - 1/tau+) (R2_i + P1_i) + (1 - 1/tau-) R3_i + S_i
//   R2_i = w_i H2_i : A2 / (2 c_s^4),  A2_ab = sum_j H2_j,ab fneq_j
//   P1_i = w_i e_i . (sum_j e_j fneq_j) / c_s^2   (first order relaxed with tau+)
//   S_i  = (1 - 1/(2 tau+)) w_i e_i.F / c_s^2     (Scheme II without G_i)
//   R3_i : D2Q9, the printed contraction w_i H3_i : A3 / (6 c_s^6), which is
//          the orthogonal projection on that lattice; D3Q19, the orthogonal
//          projection onto the span of the third-order modes (the printed
//          contraction is not a projection there: <H_xxy, H_yzz>_w = -c_s^6),
//          i.e. per pair (H_a, H_b) of overlapping modes the Gram inverse
//          9 [[2, 1], [1, 2]] (c_s^6 = 1/27); D3Q27, the printed contraction
//          (seven mutually orthogonal modes on this tensor-product lattice,
//          H_xyz counted with its six orderings).
#pragma once

#include "collide.hpp"

namespace ptrt {

template <class L, int I>
struct Herm {
    static constexpr double ex = L::ex(I), ey = L::ey(I), ez = L::ez(I);
    static constexpr double third = 1.0 / 3.0;
    // second order
    static constexpr double xx = ex * ex - third, yy = ey * ey - third, zz = ez * ez - third;
    static constexpr double xy = ex * ey, xz = ex * ez, yz = ey * ez;
    // independent third-order modes
    static constexpr double xxy = ey * (ex * ex - third), xyy = ex * (ey * ey - third);
    static constexpr double xxz = ez * (ex * ex - third), yyz = ez * (ey * ey - third);
    static constexpr double xzz = ex * (ez * ez - third), yzz = ey * (ez * ez - third);
    static constexpr double xyz = ex * ey * ez;
};

template <class L, class C, bool FAST = false>
__device__ __forceinline__ void collide_trt_rlb(C (&h)[L::Q], const Coef<L, C> &r, C &rho_o,
                                                C &ux_o, C &uy_o, C &uz_o)
{
    C drho, jx, jy, jz;
    shifted_moments<L>(h, drho, jx, jy, jz);
    const C rho = C(1) + drho;
    const C inv = recip<FAST>(rho);
    const C ux = jx * inv + r.hgx;
    const C uy = jy * inv + r.hgy;
    const C uz = jz * inv + r.hgz;
    const C uu = ux * ux + uy * uy + uz * uz;

    // equilibrium (Eq. feq) and non-equilibrium part of every direction
    C heq[L::Q], fneq[L::Q];
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const C eu = edot<L, i>(ux, uy, uz);
        const C poly = C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu + C(4.5) * eu * (eu * eu - uu);
        heq[i] = C(L::w(i)) * (drho + rho * poly);
        fneq[i] = h[i] - heq[i];
    });

    // Hermite moments of the non-equilibrium part (Eq. projection).  Terms
    // whose Hermite coefficient vanishes for a direction are left out at
    // compile time (IEEE arithmetic does not drop a product by zero), so the
    // model pays only for its nonzero terms, as in the paper's cost count.
    C Axx = 0, Ayy = 0, Azz = 0, Axy = 0, Axz = 0, Ayz = 0;
    C Bxxy = 0, Bxyy = 0, Bxxz = 0, Byyz = 0, Bxzz = 0, Byzz = 0, Bxyz = 0;
    C Jx = 0, Jy = 0, Jz = 0;
#define PTRT_ACC(acc, coef)                                                                       \
    if constexpr ((coef) != 0.0) acc += C(coef) * f
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using H = Herm<L, i>;
        const C f = fneq[i];
        PTRT_ACC(Axx, H::xx);
        PTRT_ACC(Ayy, H::yy);
        PTRT_ACC(Axy, H::xy);
        PTRT_ACC(Bxxy, H::xxy);
        PTRT_ACC(Bxyy, H::xyy);
        PTRT_ACC(Jx, H::ex);
        PTRT_ACC(Jy, H::ey);
        if constexpr (L::D == 3) {
            PTRT_ACC(Azz, H::zz);
            PTRT_ACC(Axz, H::xz);
            PTRT_ACC(Ayz, H::yz);
            PTRT_ACC(Bxxz, H::xxz);
            PTRT_ACC(Byyz, H::yyz);
            PTRT_ACC(Bxzz, H::xzz);
            PTRT_ACC(Byzz, H::yzz);
            PTRT_ACC(Jz, H::ez);
            if constexpr (L::Q == 27) PTRT_ACC(Bxyz, H::xyz);
        }
    });

    // reconstruction (Eq. R2R3_hermite) and update (Eq. TRT-RLB); the
    // diagonal second-order coefficients never vanish (2/3 or -1/3)
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using H = Herm<L, i>;
        const C w = C(L::w(i));
        C r2 = C(H::xx) * Axx + C(H::yy) * Ayy;
        if constexpr (L::D == 3) r2 += C(H::zz) * Azz;
        C p1 = C(0), r3 = C(0);
        {
#define PTRT_TERM(acc, coef, val)                                                                 \
    if constexpr ((coef) != 0.0) acc += C(coef) * (val)
            PTRT_TERM(r2, 2.0 * H::xy, Axy);
            PTRT_TERM(p1, H::ex, Jx);
            PTRT_TERM(p1, H::ey, Jy);
            if constexpr (L::D == 3) {
                PTRT_TERM(r2, 2.0 * H::xz, Axz);
                PTRT_TERM(r2, 2.0 * H::yz, Ayz);
                PTRT_TERM(p1, H::ez, Jz);
            }
            if constexpr (L::Q == 27) {
                PTRT_TERM(r3, 13.5 * H::xxy, Bxxy);
                PTRT_TERM(r3, 13.5 * H::xyy, Bxyy);
                PTRT_TERM(r3, 13.5 * H::xxz, Bxxz);
                PTRT_TERM(r3, 13.5 * H::yyz, Byyz);
                PTRT_TERM(r3, 13.5 * H::xzz, Bxzz);
                PTRT_TERM(r3, 13.5 * H::yzz, Byzz);
                PTRT_TERM(r3, 27.0 * H::xyz, Bxyz);
            } else if constexpr (L::D == 3) {
                // Gram-inverse projection per overlapping pair (xxy, yzz),
                // (xxz, yyz), (xyy, xzz)
                PTRT_TERM(r3, 9.0 * H::xxy, C(2) * Bxxy + Byzz);
                PTRT_TERM(r3, 9.0 * H::yzz, Bxxy + C(2) * Byzz);
                PTRT_TERM(r3, 9.0 * H::xxz, C(2) * Bxxz + Byyz);
                PTRT_TERM(r3, 9.0 * H::yyz, Bxxz + C(2) * Byyz);
                PTRT_TERM(r3, 9.0 * H::xyy, C(2) * Bxyy + Bxzz);
                PTRT_TERM(r3, 9.0 * H::xzz, Bxyy + C(2) * Bxzz);
            } else {
                PTRT_TERM(r3, 13.5 * H::xxy, Bxxy);
                PTRT_TERM(r3, 13.5 * H::xyy, Bxyy);
            }
#undef PTRT_TERM
        }
        const C R2 = w * C(4.5) * r2;
        const C P1 = w * C(3) * p1;
        const C R3 = w * r3;
        C src = C(0);
        // source: +K2 for the first member of a pair, -K2 for the second
        static_for<L::NP>([&](auto pc) {
            constexpr int q = decltype(pc)::value;
            if constexpr (L::pair_first(q) == i) src = rho * r.K2[q];
            if constexpr (L::opp(L::pair_first(q)) == i) src = -(rho * r.K2[q]);
        });
        h[i] = heq[i] + r.ap * (R2 + P1) + r.am * R3 + src;
    });
#undef PTRT_ACC
    rho_o = rho;
    ux_o = ux;
    uy_o = uy;
    uz_o = uz;
}

} // namespace ptrt
