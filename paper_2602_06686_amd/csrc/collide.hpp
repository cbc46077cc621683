// Per-node P-TRT collision (arXiv 2602.06686, Eq. PTRT) on shifted
// populations h_i = f_i - w_i held in registers.
//
// Arithmetic, per node:
//   drho = sum h_i, rho = 1 + drho, j = sum e_i h_i             (Eq. macro)
//   F = rho g, u = (j + F/2) / rho
//   equilibrium (Eq. feq) split by parity: with eu = e_i.u and uu = |u|^2,
//     heq+_i = w_i (drho + rho (9/2 eu^2 - 3/2 uu))
//     heq-_i = w_i rho eu (3 + 9/2 (eu^2 - uu))
//   (the third-order Hermite term reduces to (9/2) eu (eu^2 - uu) on lattices
//   whose velocity components are 0 or +-1)
//   per inversion pair: neq+ = (h_i + h_ibar)/2 - heq+, neq- = (h_i - h_ibar)/2 - heq-
//                                                                  (Eq. fneq_parity)
//   ghost projection P_G from the pair sums (Theorem 2, Eq. ghost_proj)
//   R2 = neq+ - P_G, R3 = neq- + (3/2) w_i e_i.F                  (Eq. R3_force)
//   h*_i = heq_i + (1 - 1/tau+) R2 + (1 - 1/tau-) R3 + (3/2) w_i e_i.F
// The last term is the net force source (1/2) w_i e_i.F / c_s^2: the
// first-order part of f^neq is relaxed with tau+ as in TRT-RLB (sentence
// after Eq. TRT-RLB) and Scheme II adds (1 - 1/(2 tau+)) w_i e_i.F / c_s^2.
//
// Ghost projections, derived once from Eq. ghost_proj with an orthogonal
// basis of the ghost subspace (the subspace the paper's fourth-order
// products span once their mass and stress components are removed):
//   D2Q9 (App. A.1): S = (n_0 - 2 sum_axial n + 4 sum_diag n) / 9,
//     P_G = S at rest, -S/2 on axial, S/4 on diagonal directions.
//   D3Q19: with A_a the neq sum over the two axial directions along a,
//     D_c the neq sum over the four diagonals of the plane normal to c,
//     X_a = A_a + D_a and Xm the mean of X:
//     S = n_0 - 2 (A_x + A_y + A_z) + (D_x + D_y + D_z)    (isotropic mode)
//     P_G = S/6 at rest, -S/18 + (X_a - Xm)/4 on axial a,
//           S/72 + (X_c - Xm)/8 on a diagonal in the plane normal to c.
#pragma once

#include "lattice.hpp"

namespace ptrt {

template <class C>
struct Relax {
    C ap, am;      // 1 - 1/tau+, 1 - 1/tau-
    C gx, gy, gz;  // body acceleration
};

template <class L>
struct Ghost;

template <>
struct Ghost<D2Q9> {
    // np: neq+ per pair (axial pairs 0,1; diagonal pairs 2,3)
    template <class C>
    __device__ __forceinline__ static void project(C n0, const C (&np)[4], C &pg0, C (&pg)[4])
    {
        const C S = (n0 + C(-4) * (np[0] + np[1]) + C(8) * (np[2] + np[3])) * C(1.0 / 9.0);
        pg0 = S;
        pg[0] = pg[1] = C(-0.5) * S;
        pg[2] = pg[3] = C(0.25) * S;
    }
};

template <>
struct Ghost<D3Q19> {
    // pairs: 0..2 axial x,y,z; 3,4 xy plane (normal z); 5,6 xz plane
    // (normal y); 7,8 yz plane (normal x)
    template <class C>
    __device__ __forceinline__ static void project(C n0, const C (&np)[9], C &pg0, C (&pg)[9])
    {
        const C Ax = C(2) * np[0], Ay = C(2) * np[1], Az = C(2) * np[2];
        const C Dz = C(2) * (np[3] + np[4]);
        const C Dy = C(2) * (np[5] + np[6]);
        const C Dx = C(2) * (np[7] + np[8]);
        const C S = n0 - C(2) * (Ax + Ay + Az) + (Dx + Dy + Dz);
        const C Xx = Ax + Dx, Xy = Ay + Dy, Xz = Az + Dz;
        const C Xm = (Xx + Xy + Xz) * C(1.0 / 3.0);
        const C sa = S * C(-1.0 / 18.0), sd = S * C(1.0 / 72.0);
        pg0 = S * C(1.0 / 6.0);
        pg[0] = sa + C(0.25) * (Xx - Xm);
        pg[1] = sa + C(0.25) * (Xy - Xm);
        pg[2] = sa + C(0.25) * (Xz - Xm);
        pg[3] = pg[4] = sd + C(0.125) * (Xz - Xm);
        pg[5] = pg[6] = sd + C(0.125) * (Xy - Xm);
        pg[7] = pg[8] = sd + C(0.125) * (Xx - Xm);
    }
};

// e.v for a compile-time velocity, written as adds/subtracts.
template <class L, int I, class C>
__device__ __forceinline__ C edot(C vx, C vy, C vz)
{
    C r = C(0);
    if constexpr (L::ex(I) == 1) r += vx;
    if constexpr (L::ex(I) == -1) r -= vx;
    if constexpr (L::ey(I) == 1) r += vy;
    if constexpr (L::ey(I) == -1) r -= vy;
    if constexpr (L::ez(I) == 1) r += vz;
    if constexpr (L::ez(I) == -1) r -= vz;
    return r;
}

// Density deviation and momentum of shifted populations.
template <class L, class C>
__device__ __forceinline__ void shifted_moments(const C (&h)[L::Q], C &drho, C &jx, C &jy, C &jz)
{
    drho = C(0);
    jx = C(0);
    jy = C(0);
    jz = C(0);
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        drho += h[i];
        if constexpr (L::ex(i) == 1) jx += h[i];
        if constexpr (L::ex(i) == -1) jx -= h[i];
        if constexpr (L::ey(i) == 1) jy += h[i];
        if constexpr (L::ey(i) == -1) jy -= h[i];
        if constexpr (L::ez(i) == 1) jz += h[i];
        if constexpr (L::ez(i) == -1) jz -= h[i];
    });
}

// In-place collision of one node.  Returns rho and u through the
// references (used by the fused diagnostics).
template <class L, class C>
__device__ __forceinline__ void collide(C (&h)[L::Q], const Relax<C> &r, C &rho_o, C &ux_o,
                                        C &uy_o, C &uz_o)
{
    C drho, jx, jy, jz;
    shifted_moments<L>(h, drho, jx, jy, jz);
    const C rho = C(1) + drho;
    const C Fx = rho * r.gx, Fy = rho * r.gy, Fz = rho * r.gz;
    const C inv = C(1) / rho;
    const C ux = (jx + C(0.5) * Fx) * inv;
    const C uy = (jy + C(0.5) * Fy) * inv;
    const C uz = (jz + C(0.5) * Fz) * inv;
    const C uu = ux * ux + uy * uy + uz * uz;

    const C w0 = C(L::w(0));
    const C eq0 = w0 * (drho - C(1.5) * rho * uu);
    const C n0 = h[0] - eq0;

    C eqp[L::NP], eqm[L::NP], np[L::NP], nm[L::NP];
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p), j = L::opp(i);
        const C w = C(L::w(i));
        const C eu = edot<L, i>(ux, uy, uz);
        const C eu2 = eu * eu;
        eqp[p] = w * (drho + rho * (C(4.5) * eu2 - C(1.5) * uu));
        eqm[p] = w * rho * eu * (C(3) + C(4.5) * (eu2 - uu));
        np[p] = C(0.5) * (h[i] + h[j]) - eqp[p];
        nm[p] = C(0.5) * (h[i] - h[j]) - eqm[p];
    });

    C pg0, pg[L::NP];
    Ghost<L>::project(n0, np, pg0, pg);

    h[0] = eq0 + r.ap * (n0 - pg0);
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p), j = L::opp(i);
        const C src = C(1.5 * L::w(i)) * edot<L, i>(Fx, Fy, Fz);
        const C sym = eqp[p] + r.ap * (np[p] - pg[p]);
        const C anti = eqm[p] + r.am * (nm[p] + src) + src;
        h[i] = sym + anti;
        h[j] = sym - anti;
    });
    rho_o = rho;
    ux_o = ux;
    uy_o = uy;
    uz_o = uz;
}

} // namespace ptrt
