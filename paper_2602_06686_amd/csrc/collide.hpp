// Per-node P-TRT collision (arXiv 2602.06686, Eq. PTRT) on shifted
// populations h_i = f_i - w_i held in registers.
//
// What is computed, per node (the paper's steps):
//   drho = sum h_i, rho = 1 + drho, j = sum e_i h_i, F = rho g,
//   u = (j + F/2) / rho = j / rho + g/2                           (Eq. macro)
//   f^eq from Eq. feq; with eu = e_i.u and uu = |u|^2 its parity halves are
//     heq+_i = w_i (drho + rho (9/2 eu^2 - 3/2 uu)) = (w_i rho)(9/2 eu^2 - 3/2 uu) + w_i drho
//     heq-_i = w_i rho eu (3 + 9/2 (eu^2 - uu)) = c_i rho eu (3/2 eu^2 + (1 - 3/2 uu)),
//   c_i = 3 w_i rounded so that the first moment is exact (lattice.hpp)
//   (the third-order Hermite term is (9/2) eu (eu^2 - uu) on lattices whose
//   velocity components are 0 or +-1)
//   neq+-_i = (h_i +- h_ibar)/2 - heq+-_i                      (Eq. fneq_parity)
//   R2 = neq+ - P_G neq,  R3 = neq- + (3/2) w_i e_i.F   (Theorem 2, Eq. R3_force)
//   h*_i = heq_i + (1 - 1/tau+) R2 + (1 - 1/tau-) R3 + (3/2) w_i e_i.F
// The last term is the net force source (1/2) w_i e_i.F / c_s^2: the
// first-order part of f^neq relaxes with tau+ as in TRT-RLB (sentence after
// Eq. TRT-RLB) and Scheme II adds (1 - 1/(2 tau+)) w_i e_i.F / c_s^2.
//
// How it is evaluated (same values, fewer operations):
// * per inversion pair p = (i, ibar): s = h_i + h_ibar, d = h_i - h_ibar;
//   the moments come from s and d;
// * the ghost moments are taken from the populations themselves: f^eq and
//   the shift w_i lie in the span of w_i times Hermite polynomials of order
//   <= 3, which is orthogonal to every ghost mode (ghosts are symmetric and
//   weighted-orthogonal to the mass and stress modes), so
//   sum_j G_j neq_j = sum_j G_j h_j;
// * with a+ = 1 - 1/tau+, a- = 1 - 1/tau-, sym = (h*_i + h*_ibar)/2 and
//   anti = (h*_i - h*_ibar)/2:
//     sym  = heq+ + a+ (s/2 - heq+ - P_G)
//     anti = heq- + a- (d/2 - heq-) + (1 + a-) (3/2) w_i rho e_i.g
//   and h*_i = sym + anti, h*_ibar = sym - anti.  The relaxation is kept in
//   the form eq + a (raw - eq): written as (1 - a) eq + a raw with the two
//   coefficients rounded separately, FP32 would no longer conserve mass and
//   momentum to round-off (the rounded coefficients do not sum to one), a
//   drift that reaches 1e-5 in velocity over 1000 steps.
//
// Ghost projections, derived once from Eq. ghost_proj with an orthogonal
// basis of the ghost subspace (the subspace the paper's fourth-order
// products span once their mass and stress components are removed):
//   D2Q9 (App. A.1): S = (h_0 - 2 (s_x + s_y) + 4 (s_d1 + s_d2)) / 9,
//     P_G = S at rest, -S/2 on axial, S/4 on diagonal directions.
//   D3Q19: with A_a = s of the axial pair along a, D_c = sum of s over the
//     two diagonal pairs in the plane normal to c, X_a = A_a + D_a and Xm
//     the mean of X:
//     S = h_0 - 2 (A_x + A_y + A_z) + (D_x + D_y + D_z)    (isotropic mode)
//     P_G = S/6 at rest, -S/18 + (X_a - Xm)/4 on axial a,
//           S/72 + (X_c - Xm)/8 on a diagonal in the plane normal to c.
#pragma once

#include "lattice.hpp"

namespace ptrt {

// Per-lattice constants of the update, computed once on the host in FP64
// and rounded to the compute type (they are uniform across every wave, so
// the kernels read them as scalar operands instead of recomputing them).
template <class L, class C>
struct Coef {
    C ap, am;           // a+ = 1 - 1/tau+, a- = 1 - 1/tau-
    C hgx, hgy, hgz;    // g / 2
    C K[L::NP];         // (1 + a-) (3/2) w_i e_i.g of the first member of each pair
    C K2[L::NP];        // 3 (1 - 1/(2 tau+)) w_i e_i.g (Scheme II source, TRT-RLB form)
    C bp6;              // 6 (1 - 1/(2 tau+)): Scheme I, 3 b+ u.g = bp6 (u . g/2)
    C G9[L::NP];        // 9 (1 - 1/(2 tau+)) w_i e_i.g: Scheme I, first member of each pair
    C gphi;             // -(9/4) (1 - 1/(2 tau+)): G_i per unit Phi difference across 2 nodes
};

// Forcing schemes (Sec. 2.1).  FORCE_II: Scheme II without G_i, net source
// (1/2) w_i e_i.F / c_s^2 (the default).  FORCE_II_G: plus the cubic
// correction of Eq. Gi, G_i = -(9/2)(1 - 1/(2 tau+)) w_i sum_a (e_ia^2 - 1/3)
// d_a(rho u_a^3), the derivative a central difference of a Phi field written
// by a separate pass.  FORCE_GUO: Scheme I (Eq. source_guo) with its -u.F
// part moved under the tau+ factor (the printed split does not conserve
// mass); its antisymmetric part equals the default's, so it adds the
// symmetric source (1 - 1/(2 tau+)) w_i rho (9 (e_i.u)(e_i.g) - 3 u.g).
enum { FORCE_II = 0, FORCE_II_G = 1, FORCE_GUO = 2 };

// Per-node symmetric source of the forcing schemes: dX are the scaled Phi
// differences gphi (Phi(x + e_X) - Phi(x - e_X)) (FORCE_II_G), ug3 =
// 3 (1 - 1/(2 tau+)) u.g (FORCE_GUO).
template <class C>
struct Src {
    C dx, dy, dz, ug3;
};

template <class L, int FORCING, int I, class C>
__device__ __forceinline__ C sym_source(const Src<C> &s, const Coef<L, C> &r, int p, C rho, C eu)
{
    constexpr double third = 1.0 / 3.0;
    constexpr double w = L::w(I);
    if constexpr (FORCING == FORCE_II_G) {
        constexpr double cx = L::ex(I) * L::ex(I) - third, cy = L::ey(I) * L::ey(I) - third,
                         cz = L::ez(I) * L::ez(I) - third;
        C t = C(w * cx) * s.dx + C(w * cy) * s.dy;
        if constexpr (L::D == 3) t += C(w * cz) * s.dz;
        return t;
    } else if constexpr (FORCING == FORCE_GUO) {
        if constexpr (I == 0)
            return -(C(w) * rho) * s.ug3;
        else
            return rho * (r.G9[p] * eu - C(w) * s.ug3);
    } else {
        return C(0);
    }
}

template <class L, class C>
inline Coef<L, C> make_coef(double tau_plus, double Lambda, const double g[3])
{
    const double tau_minus = 0.5 + Lambda / (tau_plus - 0.5);
    const double ap = 1.0 - 1.0 / tau_plus, am = 1.0 - 1.0 / tau_minus;
    Coef<L, C> c{};
    c.ap = (C)ap;
    c.am = (C)am;
    c.hgx = (C)(0.5 * g[0]);
    c.hgy = (C)(0.5 * g[1]);
    c.hgz = (C)(0.5 * g[2]);
    for (int p = 0; p < L::NP; ++p) {
        const int i = L::pair_first(p);
        const double eg = L::ex(i) * g[0] + L::ey(i) * g[1] + L::ez(i) * g[2];
        c.K[p] = (C)((1.0 + am) * 1.5 * L::w(i) * eg);
        c.K2[p] = (C)(3.0 * (1.0 - 0.5 / tau_plus) * L::w(i) * eg);
        c.G9[p] = (C)(9.0 * (1.0 - 0.5 / tau_plus) * L::w(i) * eg);
    }
    c.bp6 = (C)(6.0 * (1.0 - 0.5 / tau_plus));
    c.gphi = (C)(-2.25 * (1.0 - 0.5 / tau_plus));
    return c;
}

template <class L>
struct Ghost;

template <>
struct Ghost<D2Q9> {
    // sp: pair sums (axial pairs 0,1; diagonal pairs 2,3)
    template <class C>
    __device__ __forceinline__ static void project(C h0, const C (&sp)[4], C &pg0, C (&pg)[4])
    {
        const C S = (h0 + C(-2) * (sp[0] + sp[1]) + C(4) * (sp[2] + sp[3])) * C(1.0 / 9.0);
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
    __device__ __forceinline__ static void project(C h0, const C (&sp)[9], C &pg0, C (&pg)[9])
    {
        const C Ax = sp[0], Ay = sp[1], Az = sp[2];
        const C Dz = sp[3] + sp[4];
        const C Dy = sp[5] + sp[6];
        const C Dx = sp[7] + sp[8];
        const C S = h0 - C(2) * (Ax + Ay + Az) + (Dx + Dy + Dz);
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

// e.v for a compile-time velocity, written as adds/subtracts.  The sum
// starts from -0, which the first add or subtract folds away (-0 + v = v
// for every v, +0 + v is not when v = -0), so e.v costs one instruction
// per nonzero component after the first.
template <class L, int I, class C>
__device__ __forceinline__ C edot(C vx, C vy, C vz)
{
    C r = C(-0.0);
    if constexpr (L::ex(I) == 1) r += vx;
    if constexpr (L::ex(I) == -1) r -= vx;
    if constexpr (L::ey(I) == 1) r += vy;
    if constexpr (L::ey(I) == -1) r -= vy;
    if constexpr (L::ez(I) == 1) r += vz;
    if constexpr (L::ez(I) == -1) r -= vz;
    return r;
}

// 1 / rho.  FAST (chosen for FP32 storage): the hardware reciprocal refined
// by one Newton step, within one unit in the last place, 3 instructions
// instead of the correctly rounded division's 9 (measured +0.6-1 % on the
// issue-bound two-step passes).  Otherwise, and always in FP64, the
// division.
template <bool FAST, class C>
__device__ __forceinline__ C recip(C x)
{
    if constexpr (FAST && sizeof(C) == 4) {
        const float r0 = __builtin_amdgcn_rcpf(x);
        const float e = __builtin_fmaf(-x, r0, 1.0f);
        return __builtin_fmaf(e, r0, r0);
    } else {
        return C(1) / x;
    }
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

// The first pair whose first direction has a nonzero component on axis a
// (0, 1, 2 = x, y, z), -1 if none.
template <class L>
__host__ __device__ constexpr int first_pair_on(int a)
{
    for (int p = 0; p < L::NP; ++p) {
        const int i = L::pair_first(p);
        if ((a == 0 ? L::ex(i) : (a == 1 ? L::ey(i) : L::ez(i))) != 0) return p;
    }
    return -1;
}

// In-place collision of one node.  Returns rho and u through the
// references (used by the fused diagnostics).
// GHOST = false gives standard TRT (Eq. collision_TRT: the ghost modes
// relax with tau+ like the stress modes); same force treatment.
template <class L, class C, bool GHOST = true, int FORCING = FORCE_II, bool FAST = false>
__device__ __forceinline__ void collide(C (&h)[L::Q], const Coef<L, C> &r, C &rho_o, C &ux_o,
                                        C &uy_o, C &uz_o, Src<C> src = Src<C>{})
{
    C sp[L::NP], dp[L::NP];
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p), j = L::opp(i);
        sp[p] = h[i] + h[j];
        dp[p] = h[i] - h[j];
    });
    // each momentum sum starts from its first term (not from 0 + term,
    // which only differs in the sign of a zero sum; no result changes)
    C drho = h[0], jx = C(0), jy = C(0), jz = C(0);
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p);
        drho += sp[p];
        if constexpr (L::ex(i) != 0) {
            if constexpr (first_pair_on<L>(0) == p) jx = L::ex(i) == 1 ? dp[p] : -dp[p];
            else if constexpr (L::ex(i) == 1) jx += dp[p];
            else jx -= dp[p];
        }
        if constexpr (L::ey(i) != 0) {
            if constexpr (first_pair_on<L>(1) == p) jy = L::ey(i) == 1 ? dp[p] : -dp[p];
            else if constexpr (L::ey(i) == 1) jy += dp[p];
            else jy -= dp[p];
        }
        if constexpr (L::ez(i) != 0) {
            if constexpr (first_pair_on<L>(2) == p) jz = L::ez(i) == 1 ? dp[p] : -dp[p];
            else if constexpr (L::ez(i) == 1) jz += dp[p];
            else jz -= dp[p];
        }
    });
    const C rho = C(1) + drho;
    const C inv = recip<FAST>(rho);
    const C ux = jx * inv + r.hgx;
    const C uy = jy * inv + r.hgy;
    // 2D: u_z = 0 exactly (no z momentum, no z force)
    const C uz = L::D == 3 ? jz * inv + r.hgz : C(0);
    C uu = ux * ux + uy * uy;
    if constexpr (L::D == 3) uu = uu + uz * uz;
    const C m15uu = C(-1.5) * uu;

    C pg0 = C(0), pg[L::NP];
    if constexpr (GHOST) {
        Ghost<L>::project(h[0], sp, pg0, pg);
    } else {
        for (int p = 0; p < L::NP; ++p) pg[p] = C(0);
    }

    if constexpr (FORCING == FORCE_GUO)
        src.ug3 = r.bp6 * (ux * r.hgx + uy * r.hgy + uz * r.hgz);
    const C eq0 = C(L::w(0)) * (drho + rho * m15uu);
    h[0] = eq0 + r.ap * ((h[0] - eq0) - pg0);
    if constexpr (FORCING != FORCE_II) h[0] += sym_source<L, FORCING, 0>(src, r, 0, rho, C(0));
    // shared by the pairs: 1 - (3/2) uu, and per weight class w drho and
    // w rho, so that each pair's equilibrium halves cost one multiply-add
    // less each (the same values up to rounding; measured +1.3 % on the
    // two-step D3Q19 pass, which is bound by instruction issue)
    const C q15 = C(1) - C(1.5) * uu;
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p), j = L::opp(i);
        const C w = C(L::w(i));
        const C eu = edot<L, i>(ux, uy, uz);
        const C eu2 = eu * eu;
        const C eqp = (w * rho) * (C(4.5) * eu2 + m15uu) + w * drho;
        C sym = eqp + r.ap * ((C(0.5) * sp[p] - eqp) - pg[p]);
        if constexpr (FORCING != FORCE_II) sym += sym_source<L, FORCING, i>(src, r, p, rho, eu);
        // w rho eu (3 + (9/2)(eu^2 - uu)) with c_i = 3 w_i as L::c1 (first
        // moment exact)
        const C eqm = (L::template c1<C>(i) * rho) * (eu * (C(1.5) * eu2 + q15));
        const C anti = eqm + r.am * (C(0.5) * dp[p] - eqm) + rho * r.K[p];
        h[i] = sym + anti;
        h[j] = sym - anti;
    });
    rho_o = rho;
    ux_o = ux;
    uy_o = uy;
    uz_o = uz;
}

// Hybrid P-TRT on D3Q27 (Eq. PTRT_D3Q27, App. A.3): there are more ghost
// modes (7) than stress modes (6), so R2 is the Hermite stress projection
// itself, R2_i = w_i H2_i : A2 / (2 c_s^4) with A2_ab = sum_j H2_j,ab fneq_j;
// R3 = f^neq,- + (3/2) w_i e_i.F.  With EXACT the three fifth-order
// antisymmetric modes psi_a = e_a (e_b^2 - c_s^2)(e_c^2 - c_s^2) are
// projected out of f^neq,- first (weighted norm 4/243 each), which makes the
// update equal to TRT-RLB on this lattice.
template <class C, bool EXACT, int FORCING = FORCE_II, bool FAST = false>
__device__ __forceinline__ void collide_d3q27(C (&h)[27], const Coef<D3Q27, C> &r, C &rho_o,
                                              C &ux_o, C &uy_o, C &uz_o, Src<C> src = Src<C>{})
{
    using L = D3Q27;
    C sp[L::NP], dp[L::NP];
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p), j = L::opp(i);
        sp[p] = h[i] + h[j];
        dp[p] = h[i] - h[j];
    });
    C drho = h[0], jx = C(0), jy = C(0), jz = C(0);
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p);
        drho += sp[p];
        if constexpr (L::ex(i) == 1) jx += dp[p];
        if constexpr (L::ex(i) == -1) jx -= dp[p];
        if constexpr (L::ey(i) == 1) jy += dp[p];
        if constexpr (L::ey(i) == -1) jy -= dp[p];
        if constexpr (L::ez(i) == 1) jz += dp[p];
        if constexpr (L::ez(i) == -1) jz -= dp[p];
    });
    const C rho = C(1) + drho;
    const C inv = recip<FAST>(rho);
    const C ux = jx * inv + r.hgx;
    const C uy = jy * inv + r.hgy;
    const C uz = jz * inv + r.hgz;
    const C uu = ux * ux + uy * uy + uz * uz;
    const C m15uu = C(-1.5) * uu;

    // parity halves of the equilibrium and of the non-equilibrium part
    C eqp[L::NP], eqm[L::NP], np[L::NP], nm[L::NP];
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p);
        const C w = C(L::w(i));
        const C eu = edot<L, i>(ux, uy, uz);
        const C eu2 = eu * eu;
        eqp[p] = w * (drho + rho * (C(4.5) * eu2 + m15uu));
        eqm[p] = (L::template c1<C>(i) * rho) * (eu * (C(1) + C(1.5) * (eu2 - uu)));
        np[p] = C(0.5) * sp[p] - eqp[p];
        nm[p] = C(0.5) * dp[p] - eqm[p];
    });
    const C eq0 = C(L::w(0)) * (drho + rho * m15uu);
    const C n0 = h[0] - eq0;

    // second-order Hermite moments of f^neq (only the symmetric part counts)
    constexpr double third = 1.0 / 3.0;
    C Axx = C(-third) * n0, Ayy = C(-third) * n0, Azz = C(-third) * n0;
    C Axy = C(0), Axz = C(0), Ayz = C(0);
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p);
        constexpr double ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
        const C t = C(2) * np[p];
        Axx += C(ex * ex - third) * t;
        Ayy += C(ey * ey - third) * t;
        Azz += C(ez * ez - third) * t;
        if constexpr (ex * ey != 0) Axy += C(ex * ey) * t;
        if constexpr (ex * ez != 0) Axz += C(ex * ez) * t;
        if constexpr (ey * ez != 0) Ayz += C(ey * ez) * t;
    });

    // fifth-order antisymmetric moments (EXACT only)
    C S5x = C(0), S5y = C(0), S5z = C(0);
    if constexpr (EXACT) {
        static_for<L::NP>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int i = L::pair_first(p);
            constexpr double ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
            constexpr double px = ex * (ey * ey - third) * (ez * ez - third);
            constexpr double py = ey * (ez * ez - third) * (ex * ex - third);
            constexpr double pz = ez * (ex * ex - third) * (ey * ey - third);
            const C t = C(2) * nm[p];
            if constexpr (px != 0) S5x += C(px) * t;
            if constexpr (py != 0) S5y += C(py) * t;
            if constexpr (pz != 0) S5z += C(pz) * t;
        });
        const C inv_norm = C(243.0 / 4.0);
        S5x *= inv_norm;
        S5y *= inv_norm;
        S5z *= inv_norm;
    }

    if constexpr (FORCING == FORCE_GUO)
        src.ug3 = r.bp6 * (ux * r.hgx + uy * r.hgy + uz * r.hgz);
    h[0] = eq0 + r.ap * (C(L::w(0) * 4.5 * -third) * (Axx + Ayy + Azz));
    if constexpr (FORCING != FORCE_II) h[0] += sym_source<L, FORCING, 0>(src, r, 0, rho, C(0));
    static_for<L::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = L::pair_first(p), j = L::opp(i);
        constexpr double ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
        constexpr double w = L::w(i);
        // R2 = w (9/2) H2 : A2, off-diagonal components counted twice
        C r2 = C(ex * ex - third) * Axx + C(ey * ey - third) * Ayy + C(ez * ez - third) * Azz;
        if constexpr (ex * ey != 0) r2 += C(2 * ex * ey) * Axy;
        if constexpr (ex * ez != 0) r2 += C(2 * ex * ez) * Axz;
        if constexpr (ey * ez != 0) r2 += C(2 * ey * ez) * Ayz;
        const C R2 = C(4.5 * w) * r2;
        C R3 = nm[p];
        if constexpr (EXACT) {
            constexpr double px = ex * (ey * ey - third) * (ez * ez - third);
            constexpr double py = ey * (ez * ez - third) * (ex * ex - third);
            constexpr double pz = ez * (ex * ex - third) * (ey * ey - third);
            C p5 = C(0);
            if constexpr (px != 0) p5 += C(w * px) * S5x;
            if constexpr (py != 0) p5 += C(w * py) * S5y;
            if constexpr (pz != 0) p5 += C(w * pz) * S5z;
            R3 = R3 - p5;
        }
        C sym = eqp[p] + r.ap * R2;
        if constexpr (FORCING != FORCE_II)
            sym += sym_source<L, FORCING, i>(src, r, p, rho, edot<L, i>(ux, uy, uz));
        const C anti = eqm[p] + r.am * R3 + rho * r.K[p];
        h[i] = sym + anti;
        h[j] = sym - anti;
    });
    rho_o = rho;
    ux_o = ux;
    uy_o = uy;
    uz_o = uz;
}

} // namespace ptrt
