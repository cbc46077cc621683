/*
 * Reference (oracle) implementation of the Purified two-relaxation-time
 * (P-TRT) lattice Boltzmann update, plain C, FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct CPU
 * definition that the GPU kernels are checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product library never links, loads or calls it, and it shares no code,
 * header or table with the GPU sources.
 *
 * Every function follows one equation of the paper (arXiv 2602.06686,
 * "Purified Two-Relaxation-Time Lattice Boltzmann Method") in the paper's
 * order and notation, with no fusion or reordering beyond what the equation
 * states.  Readings taken where the paper is silent or inconsistent:
 *
 *  R1 (force terms of Eq. PTRT).  The first-order part of the
 *     non-equilibrium population is relaxed with tau_{s,1} (Sec. 2.2, the
 *     sentence after Eq. TRT-RLB, and the order-epsilon Chapman-Enskog
 *     equation).  Combining that term with the Scheme II source
 *     (1 - 1/(2 tau_{s,1})) w_i e_i.F / c_s^2 gives a net source of
 *     (1/2) w_i e_i.F / c_s^2, so the update is
 *       f* = f^eq + (1-1/tau+) R2 + (1-1/tau-) R3 + (1/2) w_i e_i.F / c_s^2
 *     with R3 from Eq. R3_force.  This keeps sum_i e_i f*_i = sum_i e_i f_i + F.
 *  R2 (cubic correction G_i of Eq. Gi).  The default update omits it; the
 *     forcing FORCING_II_G adds it.  Phi_aaa = rho u_a^3 (u from Eq.
 *     macro) for a = x, y and, in 3D, z (the printed list names x and y for
 *     the 2D lattice); the derivative is the central difference
 *     (Phi(x + e_a) - Phi(x - e_a)) / 2 with periodic wrap, and Phi = 0 at
 *     solid nodes (the wall velocity is zero).
 *  R18 (open boundaries, Sec. 3.4; D2Q9 only).  The inlet x = -1/2 is a
 *     halfway bounce-back wall moving with u_w = (u_in, 0) and density
 *     rho_0 = 1: a population leaving node x = 0 through it returns as
 *     f_ibar = f*_i - 2 w_i rho_0 e_i.u_w / c_s^2.  The outlet x = nx - 1 is
 *     a Zou-He pressure node (rho = rho_out, u_y = 0): populations leaving
 *     through it are lost, the three entering ones are
 *     f_3 = f_1 - (2/3) rho u_x, f_7 = f_5 + (f_2 - f_4)/2 - rho u_x / 6,
 *     f_6 = f_8 - (f_2 - f_4)/2 - rho u_x / 6, with
 *     u_x = (f_0 + f_2 + f_4 + 2 (f_1 + f_5 + f_8)) / rho_out - 1.
 *     The outlet condition holds at every time, so it is also applied to
 *     the initial state.  y stays periodic.  Momentum exchange (Eq. Fx): on a halfway
 *     bounce-back wall the population re-entering the fluid equals the one
 *     that left, so F = sum over fluid-solid links of 2 e_i f*_i(x_f).
 *  R17 (Scheme I, Eq. source_guo).  As printed, the -u.F/c_s^2 part sits
 *     under the tau- factor, so sum_i S_i = (u.F/c_s^2)(1/(2 tau-) -
 *     1/(2 tau+)) and mass is not conserved unless tau+ = tau-.  The
 *     oracle moves that part under the tau+ factor (the usual TRT split:
 *     symmetric part w_i (1 - 1/(2 tau+)) H2_i : uF / c_s^4, antisymmetric
 *     part w_i (1 - 1/(2 tau-)) e_i.F / c_s^2), and with Scheme I the tau-
 *     bracket holds f^{neq,-} alone: f* = f^eq + (1-1/tau+) R2 +
 *     (1-1/tau-) f^{neq,-} + S^I.  This gives a momentum gain of exactly F;
 *     the half-force correction inside the tau- bracket of Eq. PTRT belongs
 *     to Scheme II (R1).
 *  R3 (D3Q19 ghost basis).  The three products (e_a^2-c_s^2)(e_b^2-c_s^2)
 *     of Appendix A.2 are neither orthogonal to one another nor to the
 *     stress modes under the weighted inner product.  The ghost subspace of
 *     Eq. S_decomp is therefore spanned by those products after
 *     Gram-Schmidt against the mass mode, the stress modes and each other
 *     (weighted inner product sum_i w_i a_i b_i).  On D2Q9 the single
 *     product is already orthogonal and is left unchanged.
 *  R6 (force) F = rho g with g a constant acceleration (Sec. 3.3).
 *  Standard TRT (Eq. collision_TRT), used only as a comparison model, is
 *     the same update without the ghost subtraction.
 *  R7 (time step) collide, then stream (left side of Eq. PTRT); halfway
 *     bounce-back sends a population whose target node is solid back into
 *     the opposite direction of its source node (Sec. 3.3).
 *  R14 (D3Q27, App. A.3).  P-TRT on D3Q27 is the hybrid of Eq. PTRT_D3Q27:
 *     R2 is the Hermite stress projection w_i H2_i : A2 / (2 c_s^4) of
 *     f^neq, R3 is f^{neq,-} plus the force correction; the "exact" variant
 *     also subtracts the projections onto the three fifth-order modes
 *     psi^(5,k).  The appendix states that those modes are non-zero only on
 *     the body diagonals; they are also non-zero on the axial and on some
 *     face-diagonal velocities (psi^(5,x) = 1/9 at e = (1,0,0), -2/9 at
 *     (1,1,0)), so the projection here sums over every velocity.  The seven
 *     printed ghost modes are mutually orthogonal and orthogonal to the
 *     stress modes on D3Q27; they are kept for the Eq. PTRT form of the
 *     collision (ghost subtraction on D3Q27), which Theorem 2 makes equal to
 *     the hybrid's R2 and which the tests use as a pin.
 *
 * Population layout used by this file: f[node * Q + i], node = (z*ny+y)*nx+x.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 27
#define NGMAX 7

typedef struct {
    int D, Q;
    int e[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
    double cs2;
    int NG;
    double phi[NGMAX][QMAX]; /* orthogonal ghost basis, Eq. ghost_proj */
    double Nphi[NGMAX];      /* weighted norms of the basis */
} Lattice;

/* ---------------------------------------------------------------- lattices */

/* D2Q9 velocities and weights in the printed order, Eq. D2Q9. */
static void lattice_d2q9(Lattice *L)
{
    static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    L->D = 2;
    L->Q = 9;
    for (int i = 0; i < 9; ++i) {
        L->e[i][0] = ex[i];
        L->e[i][1] = ey[i];
        L->e[i][2] = 0;
        L->w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
}

/* D3Q19: one rest, six axial and twelve face-diagonal velocities (App. A.2).
 * The paper prints neither weights nor order; the textbook weights 1/3,
 * 1/18, 1/36 are used, in the order: rest, +x,-x,+y,-y,+z,-z, then the
 * diagonals of the xy, xz and yz planes, each followed by its opposite. */
static void lattice_d3q19(Lattice *L)
{
    static const int ev[19][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    L->D = 3;
    L->Q = 19;
    for (int i = 0; i < 19; ++i) {
        int n2 = 0;
        for (int a = 0; a < 3; ++a) {
            L->e[i][a] = ev[i][a];
            n2 += ev[i][a] * ev[i][a];
        }
        L->w[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
}

/* D3Q27: the D3Q19 set plus the eight body diagonals (App. A.3), weights
 * 8/27, 2/27, 1/54, 1/216 (tensor product of the 1D weights 2/3, 1/6). The
 * first nineteen velocities are in the D3Q19 order; the diagonals follow,
 * each followed by its opposite. */
static void lattice_d3q27(Lattice *L)
{
    static const int diag[8][3] = {{1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
                                   {1, -1, 1}, {-1, 1, -1},  {-1, 1, 1}, {1, -1, -1}};
    lattice_d3q19(L);
    L->Q = 27;
    for (int k = 0; k < 8; ++k)
        for (int a = 0; a < 3; ++a) L->e[19 + k][a] = diag[k][a];
    for (int i = 0; i < 27; ++i) {
        double w = 1.0;
        for (int a = 0; a < 3; ++a) w *= L->e[i][a] == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
        L->w[i] = w;
    }
}

/* Opposite index: e_{ibar} = -e_i (text after Eq. D2Q9), found by search. */
static void find_opposites(Lattice *L)
{
    for (int i = 0; i < L->Q; ++i) {
        L->opp[i] = -1;
        for (int j = 0; j < L->Q; ++j)
            if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] &&
                L->e[j][2] == -L->e[i][2])
                L->opp[i] = j;
    }
}

/* Weighted inner product sum_i w_i a_i b_i used throughout Sec. 2.3. */
static double wdot(const Lattice *L, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < L->Q; ++i) s += L->w[i] * a[i] * b[i];
    return s;
}

/* ---------------------------------------------------- Hermite, Eq. Hermite */

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

static double hermite2(const Lattice *L, int i, int a, int b)
{
    return L->e[i][a] * L->e[i][b] - L->cs2 * kd(a, b);
}

static double hermite3(const Lattice *L, int i, int a, int b, int c)
{
    const int *e = L->e[i];
    return (double)e[a] * e[b] * e[c] -
           L->cs2 * (e[a] * kd(b, c) + e[b] * kd(c, a) + e[c] * kd(a, b));
}

/* ------------------------------------------------------- ghost basis (R3) */

/* Ghost products (e_a^2 - c_s^2)(e_b^2 - c_s^2): Eq. ghost_D2Q9 and App. A.2,
 * orthogonalised (Gram-Schmidt, weighted inner product) against the mass
 * mode, the D(D+1)/2 stress modes H^(2)_{ab} and each other; reading R3. */
static void build_ghost_basis(Lattice *L)
{
    double basis[1 + 6 + NGMAX][QMAX];
    int nb = 0;
    int Q = L->Q, D = L->D;

    /* hydrodynamic symmetric modes: 1 and H^(2)_{ab}, a <= b (Eq. S_decomp) */
    for (int i = 0; i < Q; ++i) basis[nb][i] = 1.0;
    nb++;
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b) {
            for (int i = 0; i < Q; ++i) basis[nb][i] = hermite2(L, i, a, b);
            nb++;
        }
    int nhydro = nb;

    /* ghost products in the paper's order: (x,y), then (y,z), (z,x); on
     * D3Q27 then the sixth-order product / c_s^2 and the shear-energy modes
     * e_x e_y (e_z^2-c_s^2), e_y e_z (e_x^2-c_s^2), e_z e_x (e_y^2-c_s^2) */
    static const int pairs[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    L->NG = (D == 2) ? 1 : (Q == 19 ? 3 : 7);
    for (int k = 0; k < L->NG; ++k) {
        for (int i = 0; i < Q; ++i) {
            const int *e = L->e[i];
            double hx = e[0] * e[0] - L->cs2, hy = e[1] * e[1] - L->cs2, hz = e[2] * e[2] - L->cs2;
            double v;
            if (k < 3) {
                int a = pairs[k][0], b = pairs[k][1];
                v = (e[a] * e[a] - L->cs2) * (e[b] * e[b] - L->cs2);
            } else if (k == 3) {
                v = hx * hy * hz / L->cs2;
            } else if (k == 4) {
                v = e[0] * e[1] * hz;
            } else if (k == 5) {
                v = e[1] * e[2] * hx;
            } else {
                v = e[2] * e[0] * hy;
            }
            basis[nb][i] = v;
        }
        nb++;
    }

    /* classical Gram-Schmidt with re-orthogonalisation, done twice */
    for (int m = 0; m < nb; ++m) {
        for (int pass = 0; pass < 2; ++pass)
            for (int n = 0; n < m; ++n) {
                double c = wdot(L, basis[m], basis[n]) / wdot(L, basis[n], basis[n]);
                for (int i = 0; i < Q; ++i) basis[m][i] -= c * basis[n][i];
            }
    }
    for (int k = 0; k < L->NG; ++k) {
        for (int i = 0; i < Q; ++i) L->phi[k][i] = basis[nhydro + k][i];
        L->Nphi[k] = wdot(L, L->phi[k], L->phi[k]);
    }
}

static int make_lattice(int id, Lattice *L)
{
    memset(L, 0, sizeof(*L));
    if (id == 0)
        lattice_d2q9(L);
    else if (id == 1)
        lattice_d3q19(L);
    else if (id == 2)
        lattice_d3q27(L);
    else
        return -1;
    L->cs2 = 1.0 / 3.0;
    find_opposites(L);
    build_ghost_basis(L);
    return 0;
}

/* ------------------------------------------------------ per-node operators */

/* Eq. macro with F = rho g (R6): rho = sum f, rho u = sum e f + F/2. */
static void moments(const Lattice *L, const double *f, const double g[3],
                    double *rho, double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L->Q; ++i) {
        r += f[i];
        for (int a = 0; a < 3; ++a) j[a] += L->e[i][a] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * r * g[a]) / r;
}

/* Eq. feq: third-order Hermite equilibrium, every tensor term summed. */
static void equilibrium(const Lattice *L, double rho, const double u[3], double *feq)
{
    int D = L->D;
    double cs2 = L->cs2, cs4 = cs2 * cs2, cs6 = cs4 * cs2;
    for (int i = 0; i < L->Q; ++i) {
        double t1 = 0.0, t2 = 0.0, t3 = 0.0;
        for (int a = 0; a < D; ++a) {
            t1 += L->e[i][a] * u[a];
            for (int b = 0; b < D; ++b) {
                t2 += hermite2(L, i, a, b) * u[a] * u[b];
                for (int c = 0; c < D; ++c) t3 += hermite3(L, i, a, b, c) * u[a] * u[b] * u[c];
            }
        }
        feq[i] = L->w[i] * rho * (1.0 + t1 / cs2 + t2 / (2.0 * cs4) + t3 / (6.0 * cs6));
    }
}

/* Eq. fneq_parity: symmetric and antisymmetric halves. */
static void parity_split(const Lattice *L, const double *fneq, double *plus, double *minus)
{
    for (int i = 0; i < L->Q; ++i) {
        plus[i] = 0.5 * (fneq[i] + fneq[L->opp[i]]);
        minus[i] = 0.5 * (fneq[i] - fneq[L->opp[i]]);
    }
}

/* Eq. ghost_proj: (P^G f)_i = sum_k w_i phi_ik / N_k * sum_j phi_jk f_j. */
static void ghost_projection(const Lattice *L, const double *fneq, double *pg)
{
    for (int i = 0; i < L->Q; ++i) pg[i] = 0.0;
    for (int k = 0; k < L->NG; ++k) {
        double S = 0.0; /* ghost scalar moment S_{G,k} */
        for (int j = 0; j < L->Q; ++j) S += L->phi[k][j] * fneq[j];
        for (int i = 0; i < L->Q; ++i) pg[i] += L->w[i] * L->phi[k][i] / L->Nphi[k] * S;
    }
}

/* Fifth-order antisymmetric modes of D3Q27 (App. A.3):
 * psi^(5,x)_i = e_ix (e_iy^2 - c_s^2)(e_iz^2 - c_s^2) and cyclic. */
static double psi5(const Lattice *L, int k, int i)
{
    const int *e = L->e[i];
    int a = k, b = (k + 1) % 3, c = (k + 2) % 3;
    return e[a] * (e[b] * e[b] - L->cs2) * (e[c] * e[c] - L->cs2);
}

/* Collision models of the oracle. */
enum {
    MODEL_PTRT = 0,       /* Eq. PTRT; on D3Q27 the hybrid Eq. PTRT_D3Q27 */
    MODEL_TRT = 2,        /* Eq. collision_TRT: no ghost subtraction */
    MODEL_PTRT_EXACT = 3, /* D3Q27 hybrid with the fifth-order projection removed */
    MODEL_PTRT_GHOST = 4  /* Eq. PTRT (ghost subtraction) on every lattice */
};

/* R2 by the Hermite stress projection, w_i H2_i : A2 / (2 c_s^4) with
 * A2_ab = sum_j H2_j,ab fneq_j (Eq. projection, Eq. R2R3_hermite). */
static void stress_projection(const Lattice *L, const double *fneq, double *r2)
{
    double A[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            A[a][b] = 0.0;
            for (int j = 0; j < L->Q; ++j) A[a][b] += hermite2(L, j, a, b) * fneq[j];
        }
    for (int i = 0; i < L->Q; ++i) {
        double c = 0.0;
        for (int a = 0; a < L->D; ++a)
            for (int b = 0; b < L->D; ++b) c += hermite2(L, i, a, b) * A[a][b];
        r2[i] = L->w[i] * c / (2.0 * L->cs2 * L->cs2);
    }
}

/* Sum over k of (P^(5,k) f)_i = w_i psi5_ki / N5_k * sum_j psi5_kj f_j. */
static void fifth_order_projection(const Lattice *L, const double *fneq, double *p5)
{
    for (int i = 0; i < L->Q; ++i) p5[i] = 0.0;
    for (int k = 0; k < 3; ++k) {
        double S = 0.0, N = 0.0;
        for (int j = 0; j < L->Q; ++j) {
            S += psi5(L, k, j) * fneq[j];
            N += L->w[j] * psi5(L, k, j) * psi5(L, k, j);
        }
        for (int i = 0; i < L->Q; ++i) p5[i] += L->w[i] * psi5(L, k, i) / N * S;
    }
}

/* One collision f -> f*, Eq. PTRT with R1 (Eq. PTRT_D3Q27 on D3Q27, R14).
 * MODEL_TRT skips the ghost subtraction, which is standard TRT (Eq.
 * collision_TRT: the ghost modes relax with tau+ like the stress modes). */
/* Forcing schemes (Sec. 2.1). */
enum {
    FORCING_II = 0,   /* Scheme II without G_i, net source of R1 */
    FORCING_II_G = 1, /* Scheme II with the cubic correction G_i (Eq. Gi, R2) */
    FORCING_GUO = 2   /* Scheme I, Eq. source_guo with the split of R17 */
};

/* Eq. Gi: G_i = -w_i H2_i,ab / (6 c_s^6) (1 - 1/(2 tau+)) d_c Phi_abc, with
 * Phi_abc non-zero only for a = b = c; dphi[a] = d_a Phi_aaa. */
static double cubic_correction(const Lattice *L, int i, double tau_p, const double dphi[3])
{
    double c = 0.0;
    for (int a = 0; a < L->D; ++a) c += hermite2(L, i, a, a) * dphi[a];
    double cs6 = L->cs2 * L->cs2 * L->cs2;
    return -L->w[i] * c / (6.0 * cs6) * (1.0 - 1.0 / (2.0 * tau_p));
}

/* Eq. source_guo with the split of R17. */
static double guo_source(const Lattice *L, int i, double tau_p, double tau_m, const double u[3],
                         const double F[3])
{
    double eu = 0.0, eF = 0.0, uF = 0.0;
    for (int a = 0; a < 3; ++a) {
        eu += L->e[i][a] * u[a];
        eF += L->e[i][a] * F[a];
        uF += u[a] * F[a];
    }
    double cs2 = L->cs2, cs4 = cs2 * cs2;
    return L->w[i] * ((1.0 - 1.0 / (2.0 * tau_p)) * (eu * eF / cs4 - uF / cs2) +
                      (1.0 - 1.0 / (2.0 * tau_m)) * eF / cs2);
}

static void collide_full(const Lattice *L, const double *f, const double g[3], double tau_p,
                         double tau_m, int model, int forcing, const double dphi[3],
                         double *fstar)
{
    double rho, u[3], feq[QMAX], fneq[QMAX], plus[QMAX], minus[QMAX], pg[QMAX];
    double R2[QMAX], p5[QMAX];
    int q27 = L->Q == 27;
    moments(L, f, g, &rho, u);
    equilibrium(L, rho, u, feq);
    for (int i = 0; i < L->Q; ++i) fneq[i] = f[i] - feq[i];
    parity_split(L, fneq, plus, minus);
    if (q27 && (model == MODEL_PTRT || model == MODEL_PTRT_EXACT)) {
        stress_projection(L, fneq, R2); /* Eq. PTRT_D3Q27 */
    } else {
        if (model == MODEL_TRT)
            for (int i = 0; i < L->Q; ++i) pg[i] = 0.0;
        else
            ghost_projection(L, fneq, pg);
        for (int i = 0; i < L->Q; ++i) R2[i] = plus[i] - pg[i]; /* Theorem 2, Eq. R2_D2Q9 */
    }
    if (q27 && model == MODEL_PTRT_EXACT)
        fifth_order_projection(L, fneq, p5);
    else
        for (int i = 0; i < L->Q; ++i) p5[i] = 0.0;
    double F[3] = {rho * g[0], rho * g[1], rho * g[2]};
    for (int i = 0; i < L->Q; ++i) {
        if (forcing == FORCING_GUO) {
            double R3 = minus[i] - p5[i];
            fstar[i] = feq[i] + (1.0 - 1.0 / tau_p) * R2[i] + (1.0 - 1.0 / tau_m) * R3 +
                       guo_source(L, i, tau_p, tau_m, u, F);
            continue;
        }
        double eF = L->e[i][0] * F[0] + L->e[i][1] * F[1] + L->e[i][2] * F[2];
        double half_force = 0.5 * L->w[i] * eF / L->cs2;
        double R3 = minus[i] - p5[i] + half_force; /* Eq. R3_force */
        fstar[i] = feq[i] + (1.0 - 1.0 / tau_p) * R2[i] + (1.0 - 1.0 / tau_m) * R3 + half_force;
        if (forcing == FORCING_II_G) fstar[i] += cubic_correction(L, i, tau_p, dphi);
    }
}

static void collide_model(const Lattice *L, const double *f, const double g[3],
                          double tau_p, double tau_m, int model, double *fstar)
{
    collide_full(L, f, g, tau_p, tau_m, model, FORCING_II, NULL, fstar);
}

/* Phi_aaa = rho u_a^3 at every node (0 at solid nodes), [N][3] (R2). */
static void phi_field(const Lattice *L, size_t N, const double *f, const double g[3],
                      const uint8_t *solid, double *phi)
{
#pragma omp parallel for schedule(static)
    for (long long m = 0; m < (long long)N; ++m) {
        double rho, u[3];
        for (int a = 0; a < 3; ++a) phi[3 * m + a] = 0.0;
        if (solid && solid[m]) continue;
        moments(L, f + m * L->Q, g, &rho, u);
        for (int a = 0; a < L->D; ++a) phi[3 * m + a] = rho * u[a] * u[a] * u[a];
    }
}

static void collide(const Lattice *L, const double *f, const double g[3], double tau_p,
                    double tau_m, double *fstar)
{
    collide_model(L, f, g, tau_p, tau_m, MODEL_PTRT, fstar);
}

/* tau_{s,2} from the magic parameter Lambda = (tau+ - 1/2)(tau- - 1/2). */
static double tau_minus_from_lambda(double tau_p, double Lambda)
{
    return 0.5 + Lambda / (tau_p - 0.5);
}

/* ------------------------------------------------------------ public API */

int ptrt_oracle_lattice(int id, int *e_out, double *w_out, int *opp_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    for (int i = 0; i < L.Q; ++i) {
        for (int a = 0; a < 3; ++a) e_out[3 * i + a] = L.e[i][a];
        w_out[i] = L.w[i];
        opp_out[i] = L.opp[i];
    }
    return L.Q;
}

/* Orthogonal ghost basis [NG][Q] and its weighted norms; returns NG. */
int ptrt_oracle_ghost_basis(int id, double *phi_out, double *norm_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    for (int k = 0; k < L.NG; ++k) {
        for (int i = 0; i < L.Q; ++i) phi_out[k * L.Q + i] = L.phi[k][i];
        norm_out[k] = L.Nphi[k];
    }
    return L.NG;
}

int ptrt_oracle_equilibrium(int id, int n, const double *rho, const double *u3,
                            double *feq_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (int m = 0; m < n; ++m) equilibrium(&L, rho[m], u3 + 3 * m, feq_out + (size_t)m * L.Q);
    return 0;
}

/* Collide n independent nodes (f_in [n][Q]) -> f_out [n][Q]. */
int ptrt_oracle_collide(int id, int n, const double *f_in, const double g[3],
                        double tau_plus, double Lambda, double *f_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    double tau_m = tau_minus_from_lambda(tau_plus, Lambda);
    for (int m = 0; m < n; ++m)
        collide(&L, f_in + (size_t)m * L.Q, g, tau_plus, tau_m, f_out + (size_t)m * L.Q);
    return 0;
}

/* Same with tau_{s,2} given directly (used where Lambda is not the input). */
int ptrt_oracle_collide_tau(int id, int n, const double *f_in, const double g[3],
                            double tau_plus, double tau_minus, double *f_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    for (int m = 0; m < n; ++m)
        collide(&L, f_in + (size_t)m * L.Q, g, tau_plus, tau_minus, f_out + (size_t)m * L.Q);
    return 0;
}

/* Moments of every node: rho [N], u [N][3] (Eq. macro). */
int ptrt_oracle_moments(int id, int n, const double *f, const double g[3],
                        double *rho, double *u3)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (int m = 0; m < n; ++m) moments(&L, f + (size_t)m * L.Q, g, rho + m, u3 + 3 * m);
    return 0;
}

static size_t node_index(int x, int y, int z, int nx, int ny)
{
    return ((size_t)z * ny + y) * nx + x;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Central difference d_a Phi_aaa at node m with periodic wrap (R2). */
static void phi_gradient(const Lattice *L, int nx, int ny, int nz, const double *phi, size_t m,
                         double dphi[3])
{
    int x = (int)(m % nx), y = (int)((m / nx) % ny), z = (int)(m / ((size_t)nx * ny));
    int c[3] = {x, y, z}, n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        dphi[a] = 0.0;
        if (a >= L->D) continue;
        int p[3] = {x, y, z}, q[3] = {x, y, z};
        p[a] = wrap(c[a] + 1, n[a]);
        q[a] = wrap(c[a] - 1, n[a]);
        dphi[a] = 0.5 * (phi[3 * node_index(p[0], p[1], p[2], nx, ny) + a] -
                         phi[3 * node_index(q[0], q[1], q[2], nx, ny) + a]);
    }
}

/*
 * Advance f [N][Q] (pre-collision populations at time t) by nsteps steps:
 * collide every fluid node (Eq. PTRT, R1; the forcing scheme as selected),
 * then stream with periodic wrap and halfway bounce-back at solid
 * neighbours (R7).  Populations stored at solid nodes are not touched.
 * tau_minus <= 0 means "derive from Lambda".
 */
/* Zou-He pressure node on the east side of a D2Q9 lattice (R18): fills the
 * populations 3, 6, 7 (entering from outside) from the known ones. */
static void zou_he_outlet(double *f, double rho_out)
{
    double ux = (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8])) / rho_out - 1.0;
    f[3] = f[1] - 2.0 / 3.0 * rho_out * ux;
    f[7] = f[5] + 0.5 * (f[2] - f[4]) - rho_out * ux / 6.0;
    f[6] = f[8] - 0.5 * (f[2] - f[4]) - rho_out * ux / 6.0;
}

/* Collide every fluid node of f into fstar (the forcing scheme's Phi field
 * computed from f first when needed). */
static void collide_all(const Lattice *L, int model, int forcing, int nx, int ny, int nz,
                        double tau_plus, double tau_m, const double g[3], const uint8_t *solid,
                        const double *f, double *fstar, double *phi)
{
    size_t N = (size_t)nx * ny * nz;
    int Q = L->Q;
    if (phi) phi_field(L, N, f, g, solid, phi);
#pragma omp parallel for schedule(static)
    for (long long m = 0; m < (long long)N; ++m) {
        if (solid && solid[m]) continue;
        double dphi[3] = {0.0, 0.0, 0.0};
        if (phi) phi_gradient(L, nx, ny, nz, phi, (size_t)m, dphi);
        collide_full(L, f + m * Q, g, tau_plus, tau_m, model, forcing, dphi, fstar + m * Q);
    }
}

static int check_run_args(int id, int model, int forcing, int nz, const double *open)
{
    if (id == 0 && nz != 1) return -2;
    if (model != MODEL_PTRT && model != MODEL_TRT && model != MODEL_PTRT_EXACT &&
        model != MODEL_PTRT_GHOST)
        return -4;
    if (forcing != FORCING_II && forcing != FORCING_II_G && forcing != FORCING_GUO) return -5;
    if (open && (id != 0 || forcing == FORCING_II_G || !(open[1] > 0.0))) return -6;
    return 0;
}

/*
 * Advance f [N][Q] (pre-collision populations at time t) by nsteps steps:
 * collide every fluid node (Eq. PTRT, R1; the forcing scheme as selected),
 * then stream with periodic wrap and halfway bounce-back at solid
 * neighbours (R7).  Populations stored at solid nodes are not touched.
 * tau_minus <= 0 means "derive from Lambda".  open = {u_in, rho_out}
 * replaces the x-periodicity by the inlet and outlet of R18 (D2Q9), NULL
 * keeps every direction periodic.
 */
static int run_impl(int id, int model, int forcing, int nx, int ny, int nz, double tau_plus,
                    double Lambda, double tau_minus, const double g[3], const uint8_t *solid,
                    double *f, int nsteps, int nthreads, const double *open)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    int rc = check_run_args(id, model, forcing, nz, open);
    if (rc) return rc;
    double tau_m = tau_minus > 0.0 ? tau_minus : tau_minus_from_lambda(tau_plus, Lambda);
    int Q = L.Q;
    size_t N = (size_t)nx * ny * nz;
    double *fstar = (double *)malloc(N * Q * sizeof(double));
    double *phi = forcing == FORCING_II_G ? (double *)malloc(N * 3 * sizeof(double)) : NULL;
    if (!fstar || (forcing == FORCING_II_G && !phi)) {
        free(fstar);
        free(phi);
        return -3;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const double rho_w = 1.0; /* rho_0 of the moving inlet wall (R18) */
    for (int step = 0; step < nsteps; ++step) {
        collide_all(&L, model, forcing, nx, ny, nz, tau_plus, tau_m, g, solid, f, fstar, phi);
        /* streaming, left side of Eq. PTRT, with halfway bounce-back */
#pragma omp parallel for schedule(static)
        for (long long m = 0; m < (long long)N; ++m) {
            if (solid && solid[m]) continue;
            int x = (int)(m % nx), y = (int)((m / nx) % ny), z = (int)(m / ((size_t)nx * ny));
            for (int i = 0; i < Q; ++i) {
                double fs = fstar[(size_t)m * Q + i];
                if (open && x + L.e[i][0] < 0) { /* through the moving inlet wall */
                    double eu = L.e[i][0] * open[0];
                    f[(size_t)m * Q + L.opp[i]] = fs - 2.0 * L.w[i] * rho_w * eu / L.cs2;
                    continue;
                }
                if (open && x + L.e[i][0] >= nx) continue; /* leaves through the outlet */
                int xn = wrap(x + L.e[i][0], nx), yn = wrap(y + L.e[i][1], ny),
                    zn = wrap(z + L.e[i][2], nz);
                size_t t = node_index(xn, yn, zn, nx, ny);
                if (solid && solid[t])
                    f[(size_t)m * Q + L.opp[i]] = fs;
                else
                    f[t * Q + i] = fs;
            }
        }
        if (open)
            for (int y = 0; y < ny; ++y) {
                size_t m = node_index(nx - 1, y, 0, nx, ny);
                if (!(solid && solid[m])) zou_he_outlet(f + m * Q, open[1]);
            }
    }
    free(fstar);
    free(phi);
    return 0;
}

int ptrt_oracle_run_ex(int id, int model, int forcing, int nx, int ny, int nz, double tau_plus,
                       double Lambda, double tau_minus, const double g[3], const uint8_t *solid,
                       double *f, int nsteps, int nthreads)
{
    return run_impl(id, model, forcing, nx, ny, nz, tau_plus, Lambda, tau_minus, g, solid, f,
                    nsteps, nthreads, NULL);
}

/* Apply the outlet condition of R18 to a state f [N][Q] (the outlet holds it
 * at every time, the initial state included). */
int ptrt_oracle_apply_outlet(int id, int nx, int ny, int nz, const uint8_t *solid, double *f,
                             double rho_out)
{
    if (id != 0 || nz != 1 || !(rho_out > 0.0)) return -6;
    for (int y = 0; y < ny; ++y) {
        size_t m = node_index(nx - 1, y, 0, nx, ny);
        if (!(solid && solid[m])) zou_he_outlet(f + m * 9, rho_out);
    }
    return 0;
}

/* The same with the open boundaries of R18 (D2Q9): open = {u_in, rho_out}. */
int ptrt_oracle_run_open(int id, int model, int forcing, int nx, int ny, int nz, double tau_plus,
                         double Lambda, double tau_minus, const double g[3],
                         const uint8_t *solid, double *f, int nsteps, int nthreads,
                         const double *open)
{
    if (!open) return -6;
    return run_impl(id, model, forcing, nx, ny, nz, tau_plus, Lambda, tau_minus, g, solid, f,
                    nsteps, nthreads, open);
}

/* Momentum-exchange force on the solid nodes at time t (Eq. Fx, R18):
 * collide the pre-collision state f at t, then F = sum over fluid nodes x_f
 * and directions i with x_f + e_i solid of 2 e_i f*_i(x_f).  open != NULL:
 * links through the inlet and outlet are not solid links. */
int ptrt_oracle_momentum_exchange(int id, int model, int forcing, int nx, int ny, int nz,
                                  double tau_plus, double Lambda, double tau_minus,
                                  const double g[3], const uint8_t *solid, const double *f,
                                  const double *open, double F[3])
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    int rc = check_run_args(id, model, forcing, nz, open);
    if (rc) return rc;
    double tau_m = tau_minus > 0.0 ? tau_minus : tau_minus_from_lambda(tau_plus, Lambda);
    int Q = L.Q;
    size_t N = (size_t)nx * ny * nz;
    double *fstar = (double *)malloc(N * Q * sizeof(double));
    double *phi = forcing == FORCING_II_G ? (double *)malloc(N * 3 * sizeof(double)) : NULL;
    if (!fstar || (forcing == FORCING_II_G && !phi)) {
        free(fstar);
        free(phi);
        return -3;
    }
    collide_all(&L, model, forcing, nx, ny, nz, tau_plus, tau_m, g, solid, f, fstar, phi);
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    for (size_t m = 0; m < N; ++m) {
        if (!solid || solid[m]) continue;
        int x = (int)(m % nx), y = (int)((m / nx) % ny), z = (int)(m / ((size_t)nx * ny));
        for (int i = 1; i < Q; ++i) {
            if (open && (x + L.e[i][0] < 0 || x + L.e[i][0] >= nx)) continue;
            size_t t = node_index(wrap(x + L.e[i][0], nx), wrap(y + L.e[i][1], ny),
                                  wrap(z + L.e[i][2], nz), nx, ny);
            if (!solid[t]) continue;
            double fs = fstar[m * Q + i];
            Fx += 2.0 * L.e[i][0] * fs;
            Fy += 2.0 * L.e[i][1] * fs;
            Fz += 2.0 * L.e[i][2] * fs;
        }
    }
    F[0] = Fx;
    F[1] = Fy;
    F[2] = Fz;
    free(fstar);
    free(phi);
    return 0;
}

int ptrt_oracle_run_model(int id, int model, int nx, int ny, int nz, double tau_plus,
                          double Lambda, double tau_minus, const double g[3],
                          const uint8_t *solid, double *f, int nsteps, int nthreads)
{
    return ptrt_oracle_run_ex(id, model, FORCING_II, nx, ny, nz, tau_plus, Lambda, tau_minus, g,
                              solid, f, nsteps, nthreads);
}

/* d_a Phi_aaa at every node of the state f [N][Q] -> dphi [N][3] (R2). */
int ptrt_oracle_phi_gradient(int id, int nx, int ny, int nz, const double g[3],
                             const uint8_t *solid, const double *f, double *dphi)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    size_t N = (size_t)nx * ny * nz;
    double *phi = (double *)malloc(N * 3 * sizeof(double));
    if (!phi) return -3;
    phi_field(&L, N, f, g, solid, phi);
    for (size_t m = 0; m < N; ++m) phi_gradient(&L, nx, ny, nz, phi, m, dphi + 3 * m);
    free(phi);
    return 0;
}

/* Collision of n independent nodes with a model and a forcing scheme; dphi
 * [n][3] holds d_a Phi_aaa per node (used by FORCING_II_G, may be NULL
 * otherwise). */
int ptrt_oracle_collide_ex(int id, int model, int forcing, int n, const double *f_in,
                           const double g[3], const double *dphi, double tau_plus,
                           double tau_minus, double *f_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    if (model != MODEL_PTRT && model != MODEL_TRT && model != MODEL_PTRT_EXACT &&
        model != MODEL_PTRT_GHOST)
        return -4;
    if (forcing != FORCING_II && forcing != FORCING_II_G && forcing != FORCING_GUO) return -5;
    if (forcing == FORCING_II_G && !dphi) return -5;
    static const double zero[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < n; ++m)
        collide_full(&L, f_in + (size_t)m * L.Q, g, tau_plus, tau_minus, model, forcing,
                     dphi ? dphi + 3 * (size_t)m : zero, f_out + (size_t)m * L.Q);
    return 0;
}

/* P-TRT (Eq. PTRT, Eq. PTRT_D3Q27 on D3Q27). */
int ptrt_oracle_run(int id, int nx, int ny, int nz, double tau_plus, double Lambda,
                    double tau_minus, const double g[3], const uint8_t *solid,
                    double *f, int nsteps, int nthreads)
{
    return ptrt_oracle_run_model(id, 0, nx, ny, nz, tau_plus, Lambda, tau_minus, g, solid, f,
                                 nsteps, nthreads);
}

/* Standard TRT collision of n independent nodes (no ghost subtraction). */
int ptrt_oracle_collide_trt(int id, int n, const double *f_in, const double g[3],
                            double tau_plus, double tau_minus, double *f_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    for (int m = 0; m < n; ++m)
        collide_model(&L, f_in + (size_t)m * L.Q, g, tau_plus, tau_minus, MODEL_TRT,
                      f_out + (size_t)m * L.Q);
    return 0;
}

/* Collision of n independent nodes with any oracle model (0 P-TRT, 2 TRT,
 * 3 P-TRT with the fifth-order projection removed, 4 Eq. PTRT ghost form). */
int ptrt_oracle_collide_model(int id, int model, int n, const double *f_in, const double g[3],
                              double tau_plus, double tau_minus, double *f_out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    if (model != MODEL_PTRT && model != MODEL_TRT && model != MODEL_PTRT_EXACT &&
        model != MODEL_PTRT_GHOST)
        return -4;
    for (int m = 0; m < n; ++m)
        collide_model(&L, f_in + (size_t)m * L.Q, g, tau_plus, tau_minus, model,
                      f_out + (size_t)m * L.Q);
    return 0;
}

/* Fifth-order modes psi^(5,k) of D3Q27 [3][27]; returns 3 (or -1). */
int ptrt_oracle_fifth_modes(int id, double *psi_out)
{
    Lattice L;
    if (make_lattice(id, &L) || L.Q != 27) return -1;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < L.Q; ++i) psi_out[k * L.Q + i] = psi5(&L, k, i);
    return 3;
}

/*
 * One step evaluated only at the listed nodes: out[s][i] = f_i(x_s, t+1)
 * for the pre-collision state f at time t.  Each sampled population is
 * obtained from the collision at its source node x_s - e_i, or at x_s itself
 * with the opposite direction when that source is solid (R7).  Used to check
 * lattices too large for a whole-lattice oracle run.
 */
int ptrt_oracle_step_sampled(int id, int nx, int ny, int nz, double tau_plus,
                             double Lambda, const double g[3], const uint8_t *solid,
                             const double *f, int nsample, const long long *nodes,
                             double *out)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    double tau_m = tau_minus_from_lambda(tau_plus, Lambda);
    int Q = L.Q;
#pragma omp parallel for schedule(static)
    for (int s = 0; s < nsample; ++s) {
        long long m = nodes[s];
        int x = (int)(m % nx), y = (int)((m / nx) % ny), z = (int)(m / ((long long)nx * ny));
        double fs[QMAX];
        for (int i = 0; i < Q; ++i) {
            int xs = wrap(x - L.e[i][0], nx), ys = wrap(y - L.e[i][1], ny),
                zs = wrap(z - L.e[i][2], nz);
            size_t src = node_index(xs, ys, zs, nx, ny);
            if (solid && solid[src]) {
                collide(&L, f + (size_t)m * Q, g, tau_plus, tau_m, fs);
                out[(size_t)s * Q + i] = fs[L.opp[i]];
            } else {
                collide(&L, f + src * Q, g, tau_plus, tau_m, fs);
                out[(size_t)s * Q + i] = fs[i];
            }
        }
    }
    return 0;
}

/* Mass and kinetic energy over fluid nodes: sum rho, (1/2) sum rho |u|^2. */
int ptrt_oracle_diagnostics(int id, int n, const double *f, const double g[3],
                            const uint8_t *solid, double *mass, double *kinetic)
{
    Lattice L;
    if (make_lattice(id, &L)) return -1;
    double M = 0.0, K = 0.0;
    for (int m = 0; m < n; ++m) {
        if (solid && solid[m]) continue;
        double rho, u[3];
        moments(&L, f + (size_t)m * L.Q, g, &rho, u);
        M += rho;
        K += 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    }
    *mass = M;
    *kinetic = K;
    return 0;
}

int ptrt_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
