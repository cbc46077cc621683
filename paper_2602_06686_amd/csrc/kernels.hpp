// HIP kernels of the P-TRT path: the fused stream-and-collide step, the
// state scatter used by initialisation and restore, the gather used by
// moments / populations / diagnostics, and the FP64 reductions.
//
// Layout (one lattice): rows of nx nodes (row = z * ny + y, x fastest),
// stored with a pitch of nx rounded up to whole 128-byte lines, are grouped
// into tiles of R = 2^lr rows; a tile stores direction 0 of its R rows, then
// direction 1, ..., then direction Q-1, each as a contiguous chunk of
// plane = R * pitch shifted populations h_i = f_i - w_i.  Element
// (i, row, x) sits at  (row >> lr) * Q * plane + i * plane
// + (row & (R-1)) * pitch + x.  With R large enough to hold every row this is
// the plain direction-major (SoA) layout; with chunks of a few KB the Q
// streams of a step stay inside one tile, which keeps the HBM pages that a
// wave touches close together.
//
// A step pulls: population i of node x comes from node x - e_i of the
// previous post-collision state (periodic wrap), or, when that node is
// solid, from direction opp(i) of x itself (halfway bounce-back).  The
// stored state is therefore "post-collision at t-1, not yet streamed":
// pulling it gives the pre-collision populations at time t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "codec.hpp"
#include "collide.hpp"
#include "lattice.hpp"
#include "trt_rlb.hpp"

namespace ptrt {

struct Geom {
    int nx, ny, nz;
    int pitch;       // elements per stored row (nx rounded up to whole 128-byte lines)
    int lr;          // log2 of rows per tile
    long long plane; // elements of one direction inside a tile: pitch << lr
    long long tile;  // elements of a tile: Q * plane
    // Open boundaries in x (D2Q9, kernels with OPEN = true only): inlet wall
    // at x = -1/2 moving with (uin, 0), pressure outlet rho = 1 + drhoout at
    // x = nx - 1.
    double uin = 0.0, drhoout = 0.0;
};

// Offset of the first element of direction q of a row; element (q, row, x)
// is at row_base(g, q, row) + x.  Kept apart from x so that, when the row is
// uniform across a wave, the base is computed on the scalar unit and the
// loads use a scalar base with a 32-bit per-lane offset.
// The part inside a tile (direction chunk and row within the tile) is
// computed in 32 bits: a tile holds Q * nx << lr < 2^32 elements.
__device__ __forceinline__ long long row_base(const Geom &g, int q, unsigned row)
{
    const unsigned in_tile =
        (unsigned)q * (unsigned)g.plane + (row & ((1u << g.lr) - 1u)) * (unsigned)g.pitch;
    return (long long)(row >> g.lr) * g.tile + (long long)in_tile;
}

// The x part is added as a 32-bit byte offset, so that with a row-uniform
// base the access can use a scalar 64-bit base plus a 32-bit lane offset
// (no 64-bit address arithmetic per lane).
template <class S>
__device__ __forceinline__ S *at(S *base, const Geom &g, int q, unsigned row, int x)
{
    using B = typename std::conditional<std::is_const<S>::value, const char, char>::type;
    return reinterpret_cast<S *>(reinterpret_cast<B *>(base + row_base(g, q, row)) +
                                 (unsigned)x * (unsigned)sizeof(S));
}

// Source of population I pulled into (x, y, z): x coordinate and row of
// node (x, y, z) - e_I with periodic wrap.
struct Nbr {
    int xm, xp, ym, yp, zm, zp;
    __device__ __forceinline__ Nbr(const Geom &g, int x, int y, int z)
    {
        xm = x == 0 ? g.nx - 1 : x - 1;
        xp = x == g.nx - 1 ? 0 : x + 1;
        ym = y == 0 ? g.ny - 1 : y - 1;
        yp = y == g.ny - 1 ? 0 : y + 1;
        zm = z == 0 ? g.nz - 1 : z - 1;
        zp = z == g.nz - 1 ? 0 : z + 1;
    }
};

template <class L, int I>
__device__ __forceinline__ void source_of(const Geom &g, const Nbr &n, int x, int y, int z, int &sx,
                                          unsigned &srow)
{
    sx = L::ex(I) == 1 ? n.xm : (L::ex(I) == -1 ? n.xp : x);
    const int sy = L::ey(I) == 1 ? n.ym : (L::ey(I) == -1 ? n.yp : y);
    const int sz = L::ez(I) == 1 ? n.zm : (L::ez(I) == -1 ? n.zp : z);
    srow = (unsigned)sz * (unsigned)g.ny + (unsigned)sy;
}

// Zou-He pressure node on the east side of D2Q9 (x = nx - 1, u_y = 0), in
// shifted populations: the three populations entering from outside
// (3: (-1,0), 6: (-1,1), 7: (-1,-1)) from the six known ones and
// rho_out = 1 + drho_out:
//   rho_out u_x = h0 + h2 + h4 + 2 (h1 + h5 + h8) - drho_out,
//   h3 = h1 - (2/3) rho_out u_x,
//   h7 = h5 + (h2 - h4)/2 - rho_out u_x / 6,  h6 = h8 - (h2 - h4)/2 - rho_out u_x / 6
// (the shifts w_i cancel pairwise and sum to 1 in the first line).
template <class T>
__device__ __forceinline__ void zou_he_east(T (&h)[9], T drho_out)
{
    static_assert(D2Q9::ex(1) == 1 && D2Q9::ex(3) == -1 && D2Q9::ey(2) == 1 && D2Q9::ey(4) == -1 &&
                      D2Q9::ex(5) == 1 && D2Q9::ey(5) == 1 && D2Q9::ex(6) == -1 &&
                      D2Q9::ey(6) == 1 && D2Q9::ex(7) == -1 && D2Q9::ey(7) == -1 &&
                      D2Q9::ex(8) == 1 && D2Q9::ey(8) == -1,
                  "D2Q9 velocity order");
    const T ru = (h[0] + h[2] + h[4] + T(2) * (h[1] + h[5] + h[8])) - drho_out;
    const T d = T(0.5) * (h[2] - h[4]);
    h[3] = h[1] - T(2.0 / 3.0) * ru;
    h[7] = h[5] + d - T(1.0 / 6.0) * ru;
    h[6] = h[8] - d - T(1.0 / 6.0) * ru;
}

// Pull the Q populations of fluid node (x, y, z) into registers (type T).
// OPEN (D2Q9): x is not periodic; at x = 0 the populations entering through
// the inlet wall are the node's own outgoing ones plus 2 w_i e_i.u_w / c_s^2
// (moving halfway bounce-back, rho_0 = 1); at x = nx - 1 the populations
// entering through the outlet come from zou_he_east.  The periodic loads
// of those populations stay in bounds and are overwritten.
template <class L, class S, bool MASK, bool OPEN = false, class T, class LoadF>
__device__ __forceinline__ void pull(const S *__restrict__ src, const uint8_t *__restrict__ mask,
                                     const Geom &g, int x, int y, int z, T (&h)[L::Q], LoadF load)
{
    const Nbr n(g, x, y, z);
    const unsigned row = (unsigned)z * (unsigned)g.ny + (unsigned)y;
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i == 0) {
            h[0] = load(at(src, g, 0, row, x));
        } else {
            int sx;
            unsigned srow;
            source_of<L, i>(g, n, x, y, z, sx, srow);
            if constexpr (MASK) {
                if (mask[srow * (unsigned)g.nx + (unsigned)sx])
                    h[i] = load(at(src, g, L::opp(i), row, x));
                else
                    h[i] = load(at(src, g, i, srow, sx));
            } else {
                h[i] = load(at(src, g, i, srow, sx));
            }
        }
    });
    if constexpr (OPEN) {
        static_assert(L::D == 2 && L::Q == 9, "open boundaries are built for D2Q9");
        if (x == 0) {
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (L::ex(i) == 1)
                    h[i] = load(at(src, g, L::opp(i), row, x)) + T(6.0 * L::w(i)) * T(g.uin);
            });
        }
        if (x == g.nx - 1) zou_he_east(h, T(g.drhoout));
    }
}

// Write the pre-collision populations hv (shifted, FP64) of a fluid node into
// the slots its next pull reads: the inverse of pull().
// OPEN: the inlet slots take hv minus the wall-velocity term; the outlet's
// entering populations are computed by every pull and are not stored.
template <class L, class S, bool MASK, bool OPEN = false>
__device__ __forceinline__ void scatter(S *__restrict__ dst, const uint8_t *__restrict__ mask,
                                        const Geom &g, int x, int y, int z, const double (&hv)[L::Q])
{
    const Nbr n(g, x, y, z);
    const unsigned row = (unsigned)z * (unsigned)g.ny + (unsigned)y;
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i == 0) {
            store_f64(at(dst, g, 0, row, x), hv[0]);
        } else if (OPEN && L::ex(i) == 1 && x == 0) {
            store_f64(at(dst, g, L::opp(i), row, x), hv[i] - 6.0 * L::w(i) * g.uin);
        } else if (OPEN && L::ex(i) == -1 && x == g.nx - 1) {
            // filled by the outlet condition on every pull
        } else {
            int sx;
            unsigned srow;
            source_of<L, i>(g, n, x, y, z, sx, srow);
            if (MASK && mask[srow * (unsigned)g.nx + (unsigned)sx])
                store_f64(at(dst, g, L::opp(i), row, x), hv[i]);
            else
                store_f64(at(dst, g, i, srow, sx), hv[i]);
        }
    });
}

// Sum (a, b) over a workgroup of up to 1024 threads; the result is valid in
// thread 0.  Every thread of the block must call it.
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    __shared__ double sa[16], sb[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wid = tid >> 6, nw = (nthreads + 63) >> 6;
    if (lane == 0) {
        sa[wid] = a;
        sb[wid] = b;
    }
    __syncthreads();
    if (wid == 0) {
        a = lane < nw ? sa[lane] : 0.0;
        b = lane < nw ? sb[lane] : 0.0;
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
        }
    }
}

__device__ __forceinline__ unsigned flat_block()
{
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// XCD-aware block order: the hardware hands workgroup ids round-robin to the
// 8 XCDs, so id P runs on XCD P mod 8; renumbering P = 8 q + r to
// r (G8 / 8) + q gives each XCD a contiguous range of blocks (neighbouring
// rows and planes, whose shared lines then meet in that XCD's L2).  A
// bijection on [0, G8), G8 = the grid size rounded down to a multiple of 8;
// the remaining ids are kept.  Returns the block coordinates to work on.
// (Measured: a gain for the two-step kernel, whose columns share halo lines;
// a loss for the one-step kernels, which keep the hardware order.)
__device__ __forceinline__ void xcd_block(int &bx, int &by, int &bz)
{
    const unsigned G = gridDim.x * gridDim.y * gridDim.z;
    const unsigned P = flat_block();
    const unsigned G8 = G & ~7u;
    const unsigned Lb = P < G8 ? (P & 7u) * (G8 >> 3) + (P >> 3) : P;
    bx = (int)(Lb % gridDim.x);
    by = (int)((Lb / gridDim.x) % gridDim.y);
    bz = (int)(Lb / (gridDim.x * gridDim.y));
}

// Collision models: P-TRT (the method), and for comparison TRT-RLB (Hermite
// projection, Eq. TRT-RLB) and standard TRT (ghost modes kept).
// MODEL_PTRT_EXACT differs from MODEL_PTRT only on D3Q27 (fifth-order
// antisymmetric modes projected out, App. A.3).
enum { MODEL_PTRT = 0, MODEL_TRT_RLB = 1, MODEL_TRT = 2, MODEL_PTRT_EXACT = 3 };

// ---------------------------------------------------------------------------
// Phi field of the cubic correction (Eq. Gi): Phi_a = rho u_a^3 of every
// node at the current time, component-major [D][nz][ny][nx] in the compute
// type, 0 at solid nodes.
template <class C>
__device__ __forceinline__ size_t phi_index(const Geom &g, int a, unsigned row, int x)
{
    return (size_t)a * ((size_t)g.ny * (size_t)g.nz * (size_t)g.nx) + (size_t)row * (unsigned)g.nx +
           (unsigned)x;
}

// Scaled central differences of Phi at (x, y, z) with periodic wrap.
template <class L, class C>
__device__ __forceinline__ Src<C> phi_differences(const C *__restrict__ phi, const Geom &g,
                                                  const Coef<L, C> &r, int x, int y, int z,
                                                  unsigned row)
{
    const Nbr n(g, x, y, z);
    Src<C> s{};
    s.dx = r.gphi * (phi[phi_index<C>(g, 0, row, n.xp)] - phi[phi_index<C>(g, 0, row, n.xm)]);
    const unsigned rym = (unsigned)z * (unsigned)g.ny + (unsigned)n.ym;
    const unsigned ryp = (unsigned)z * (unsigned)g.ny + (unsigned)n.yp;
    s.dy = r.gphi * (phi[phi_index<C>(g, 1, ryp, x)] - phi[phi_index<C>(g, 1, rym, x)]);
    if constexpr (L::D == 3) {
        const unsigned rzm = (unsigned)n.zm * (unsigned)g.ny + (unsigned)y;
        const unsigned rzp = (unsigned)n.zp * (unsigned)g.ny + (unsigned)y;
        s.dz = r.gphi * (phi[phi_index<C>(g, 2, rzp, x)] - phi[phi_index<C>(g, 2, rzm, x)]);
    }
    return s;
}

// ---------------------------------------------------------------------------
// One node update: pull, moments, equilibrium, parity split, ghost removal,
// two-rate relaxation, force; store to the node's own slots of dst.
template <class L, class S, bool MASK, bool NT, int MODEL = MODEL_PTRT, int FORCING = FORCE_II,
          bool OPEN = false>
__device__ __forceinline__ void node_update(const S *__restrict__ src, S *__restrict__ dst,
                                            const uint8_t *__restrict__ mask, const Geom &g,
                                            const Coef<L, typename Codec<S>::compute> &r, int x,
                                            int y, int z, unsigned row, double &m, double &k,
                                            const typename Codec<S>::compute *__restrict__ phi =
                                                nullptr)
{
    using C = typename Codec<S>::compute;
    static_assert(MODEL != MODEL_TRT_RLB || FORCING == FORCE_II,
                  "the TRT-RLB comparison kernel uses Scheme II only");
    C h[L::Q];
    pull<L, S, MASK, OPEN>(src, mask, g, x, y, z, h, [](const S *p) { return Codec<S>::load(p); });
    Src<C> sc{};
    if constexpr (FORCING == FORCE_II_G) sc = phi_differences<L, C>(phi, g, r, x, y, z, row);
    C rho, ux, uy, uz;
    constexpr bool FR = Codec<S>::fast_recip;
    if constexpr (MODEL == MODEL_TRT_RLB)
        collide_trt_rlb<L, C, FR>(h, r, rho, ux, uy, uz);
    else if constexpr (MODEL == MODEL_TRT)
        collide<L, C, false, FORCING, FR>(h, r, rho, ux, uy, uz, sc);
    else if constexpr (L::Q == 27)
        collide_d3q27<C, MODEL == MODEL_PTRT_EXACT, FORCING, FR>(h, r, rho, ux, uy, uz, sc);
    else
        collide<L, C, true, FORCING, FR>(h, r, rho, ux, uy, uz, sc);
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        Codec<S>::template store<NT>(at(dst, g, i, row, x), h[i]);
    });
    m = (double)rho;
    k = 0.5 * (double)rho * ((double)ux * ux + (double)uy * uy + (double)uz * uz);
}

// Phi pass of the cubic correction: pull, moments (Eq. macro), Phi_a =
// rho u_a^3; solid nodes write 0.  Same workgroup shapes as k_step.
template <class L, class S, bool MASK, bool ROW>
__global__ void __launch_bounds__(1024)
k_phi(const S *__restrict__ src, const uint8_t *__restrict__ mask, const uint8_t *__restrict__ near,
      Geom g, Coef<L, typename Codec<S>::compute> r, typename Codec<S>::compute *__restrict__ phi)
{
    using C = typename Codec<S>::compute;
    int x, y, z;
    if constexpr (ROW) {
        x = blockIdx.x * blockDim.x + threadIdx.x;
        y = blockIdx.y;
        z = blockIdx.z;
    } else {
        x = blockIdx.x * blockDim.x + threadIdx.x;
        y = blockIdx.y * blockDim.y + threadIdx.y;
        z = blockIdx.z;
    }
    if (x >= g.nx || (!ROW && y >= g.ny)) return;
    const unsigned row = (unsigned)z * (unsigned)g.ny + (unsigned)y;
    C h[L::Q];
    bool solid = false;
    auto ld = [](const S *p) { return Codec<S>::load(p); };
    if constexpr (MASK) {
        solid = mask[row * (unsigned)g.nx + (unsigned)x] != 0;
        if (!solid) {
            if (near[row])
                pull<L, S, true>(src, mask, g, x, y, z, h, ld);
            else
                pull<L, S, false>(src, mask, g, x, y, z, h, ld);
        }
    } else {
        pull<L, S, false>(src, mask, g, x, y, z, h, ld);
    }
    C px = C(0), py = C(0), pz = C(0);
    if (!solid) {
        C drho, jx, jy, jz;
        shifted_moments<L>(h, drho, jx, jy, jz);
        const C rho = C(1) + drho;
        const C inv = C(1) / rho;
        const C ux = jx * inv + r.hgx, uy = jy * inv + r.hgy, uz = jz * inv + r.hgz;
        px = rho * (ux * ux * ux);
        py = rho * (uy * uy * uy);
        pz = rho * (uz * uz * uz);
    }
    phi[phi_index<C>(g, 0, row, x)] = px;
    phi[phi_index<C>(g, 1, row, x)] = py;
    if constexpr (L::D == 3) phi[phi_index<C>(g, 2, row, x)] = pz;
}

// Fused step kernel.
// ROW: 1D workgroups inside one row (grid (ceil(nx / blockDim.x), ny, nz)),
// so y, z and every row and tile offset are uniform across the wave and
// computed on the scalar unit; otherwise 2D workgroups over (x, y) and
// grid.z = nz (used when ny exceeds the grid's y limit).
// MASK: the lattice has solid nodes.  near[row] != 0 marks rows that hold a
// solid node or pull from one (computed on the host); only those rows read
// the mask, every other row takes the mask-free code (a uniform branch in
// ROW mode).
// NT: non-temporal stores (the state is far larger than the caches).
// DIAG: also reduce mass and kinetic energy of the pulled (pre-collision)
// state into per-block FP64 partials.
// Workgroups: at most 1024 threads (batch per-lattice launches), except
// D3Q27 in FP64, launched with at most 256 (row workgroups of 1 KB per
// direction, or the 64 x 4 fallback): the smaller bound lifts the register
// cap from 128 to 512 so that its 27 FP64 populations do not spill.
template <class L, class S, bool MASK, bool ROW, bool NT, bool DIAG, int MODEL = MODEL_PTRT,
          int FORCING = FORCE_II, bool OPEN = false>
__global__ void __launch_bounds__((L::Q == 27 && sizeof(S) == 8) ? 256 : 1024)
k_step(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask,
       const uint8_t *__restrict__ near, Geom g, Coef<L, typename Codec<S>::compute> r,
       double2 *__restrict__ partials,
       const typename Codec<S>::compute *__restrict__ phi = nullptr)
{
    int x, y, z;
    if constexpr (ROW) {
        x = blockIdx.x * blockDim.x + threadIdx.x;
        y = blockIdx.y;
        z = blockIdx.z;
    } else {
        x = blockIdx.x * blockDim.x + threadIdx.x;
        y = blockIdx.y * blockDim.y + threadIdx.y;
        z = blockIdx.z;
    }
    const bool inside = x < g.nx && (ROW || y < g.ny);
    const unsigned row = (unsigned)z * (unsigned)g.ny + (unsigned)y;
    double m = 0.0, k = 0.0;
    if constexpr (MASK) {
        if (inside || ROW) {
            if (near[row]) {
                if (inside && mask[row * (unsigned)g.nx + (unsigned)x] == 0)
                    node_update<L, S, true, NT, MODEL, FORCING, OPEN>(src, dst, mask, g, r, x, y,
                                                                      z, row, m, k, phi);
            } else if (inside) {
                node_update<L, S, false, NT, MODEL, FORCING, OPEN>(src, dst, mask, g, r, x, y, z,
                                                                   row, m, k, phi);
            }
        }
    } else if (inside) {
        node_update<L, S, false, NT, MODEL, FORCING, OPEN>(src, dst, mask, g, r, x, y, z, row, m,
                                                           k, phi);
    }
    if constexpr (DIAG) {
        block_sum2(m, k);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[flat_block()] = make_double2(m, k);
    }
}

// ---------------------------------------------------------------------------
// Scatter a full FP64 state f[Q][N] (unshifted) into dst (pre-collision at t).
template <class L, class S, bool MASK, bool OPEN = false>
__global__ void __launch_bounds__(256)
k_set_state(S *__restrict__ dst, const uint8_t *__restrict__ mask, Geom g, int z0,
            const double *__restrict__ f, long long fstride)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z + z0;
    if (x >= g.nx || y >= g.ny) return;
    const unsigned node = ((unsigned)z * (unsigned)g.ny + (unsigned)y) * (unsigned)g.nx + (unsigned)x;
    const unsigned in = node - (unsigned)z0 * (unsigned)g.ny * (unsigned)g.nx;
    if (MASK && mask[node]) return;
    double hv[L::Q];
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        hv[i] = f[(long long)i * fstride + in] - L::w(i);
    });
    scatter<L, S, MASK, OPEN>(dst, mask, g, x, y, z, hv);
}

// Equilibrium initialisation (Eq. feq) in FP64 from rho[N] and u[3][N]
// (either may be null: rho = 1, u = 0), scattered into dst.
template <class L, class S, bool MASK, bool OPEN = false>
__global__ void __launch_bounds__(256)
k_init_eq(S *__restrict__ dst, const uint8_t *__restrict__ mask, Geom g, int z0,
          const double *__restrict__ rho_in, const double *__restrict__ u_in, long long ustride)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z + z0;
    if (x >= g.nx || y >= g.ny) return;
    const unsigned node = ((unsigned)z * (unsigned)g.ny + (unsigned)y) * (unsigned)g.nx + (unsigned)x;
    const unsigned in = node - (unsigned)z0 * (unsigned)g.ny * (unsigned)g.nx;
    if (MASK && mask[node]) return;
    const double rho = rho_in ? rho_in[in] : 1.0;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (u_in) {
        ux = u_in[in];
        uy = u_in[ustride + in];
        if (L::D == 3) uz = u_in[2 * ustride + in];
    }
    const double uu = ux * ux + uy * uy + uz * uz;
    double hv[L::Q];
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const double eu = edot<L, i>(ux, uy, uz);
        const double poly = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu + 4.5 * eu * (eu * eu - uu);
        hv[i] = L::w(i) * ((rho - 1.0) + rho * poly);
    });
    scatter<L, S, MASK, OPEN>(dst, mask, g, x, y, z, hv);
}

// ---------------------------------------------------------------------------
// Gather the pre-collision state at t: any of rho[N], u[3][N], f[Q][N]
// (unshifted) and per-block (mass, kinetic energy) partials.  Solid nodes
// report zeros and contribute nothing.
template <class L, class S, bool MASK, bool OPEN = false>
__global__ void __launch_bounds__(256)
k_gather(const S *__restrict__ src, const uint8_t *__restrict__ mask, Geom g, int z0, double gx,
         double gy, double gz, double *__restrict__ rho_out, double *__restrict__ u_out,
         double *__restrict__ f_out, long long ostride, double2 *__restrict__ partials)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z + z0;
    const bool inside = x < g.nx && y < g.ny;
    const unsigned node = ((unsigned)z * (unsigned)g.ny + (unsigned)y) * (unsigned)g.nx + (unsigned)x;
    const unsigned on = node - (unsigned)z0 * (unsigned)g.ny * (unsigned)g.nx;
    const bool fluid = inside && !(MASK && mask[node]);
    double m = 0.0, k = 0.0;
    if (fluid) {
        double h[L::Q];
        pull<L, S, MASK, OPEN>(src, mask, g, x, y, z, h, [](const S *p) { return load_f64(p); });
        double drho, jx, jy, jz;
        shifted_moments<L>(h, drho, jx, jy, jz);
        const double rho = 1.0 + drho;
        const double ux = (jx + 0.5 * rho * gx) / rho;
        const double uy = (jy + 0.5 * rho * gy) / rho;
        const double uz = (jz + 0.5 * rho * gz) / rho;
        if (rho_out) rho_out[on] = rho;
        if (u_out) {
            u_out[on] = ux;
            u_out[ostride + on] = uy;
            u_out[2 * ostride + on] = uz;
        }
        if (f_out) {
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                f_out[(long long)i * ostride + on] = h[i] + L::w(i);
            });
        }
        m = rho;
        k = 0.5 * rho * (ux * ux + uy * uy + uz * uz);
    } else if (inside) {
        if (rho_out) rho_out[on] = 0.0;
        if (u_out) {
            u_out[on] = 0.0;
            u_out[ostride + on] = 0.0;
            u_out[2 * ostride + on] = 0.0;
        }
        if (f_out) {
            for (int i = 0; i < L::Q; ++i) f_out[(long long)i * ostride + on] = 0.0;
        }
    }
    if (partials) {
        block_sum2(m, k);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[flat_block()] = make_double2(m, k);
    }
}

// Sum nparts partials in a fixed order (deterministic) into out[0..1].
// (A template only so that every translation unit may instantiate it.)
template <int BLOCK = 1024>
__global__ void __launch_bounds__(BLOCK)
k_finalize(const double2 *__restrict__ partials, int nparts, double *__restrict__ out)
{
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a += partials[i].x;
        b += partials[i].y;
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// Sum (a, b, c) over a workgroup of up to 1024 threads; valid in thread 0.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c)
{
    __shared__ double sc[16];
    block_sum2(a, b);
    __syncthreads();
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wid = tid >> 6, nw = (nthreads + 63) >> 6;
    if (lane == 0) sc[wid] = c;
    __syncthreads();
    if (wid == 0) {
        c = lane < nw ? sc[lane] : 0.0;
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    }
}

// Momentum-exchange force on the solid nodes (Eq. Fx) from the stored
// post-collision state of the last step: sum over fluid nodes x_f and
// directions i with x_f + e_i solid of 2 e_i f*_i(x_f) (on a halfway
// bounce-back wall the population re-entering the fluid equals the one that
// left).  Rows without solid neighbours are skipped.  Per-block partials
// [nblocks][3]; OPEN: links through the inlet and outlet are not wall links.
template <class L, class S, bool OPEN>
__global__ void __launch_bounds__(256)
k_momentum_exchange(const S *__restrict__ src, const uint8_t *__restrict__ mask,
                    const uint8_t *__restrict__ near, Geom g, double *__restrict__ partials)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (x < g.nx && y < g.ny) {
        const unsigned row = (unsigned)z * (unsigned)g.ny + (unsigned)y;
        if (near[row] && !mask[row * (unsigned)g.nx + (unsigned)x]) {
            const Nbr n(g, x, y, z);
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (i != 0) {
                    const bool outside = OPEN && ((L::ex(i) == -1 && x == 0) ||
                                                  (L::ex(i) == 1 && x == g.nx - 1));
                    const int tx = L::ex(i) == 1 ? n.xp : (L::ex(i) == -1 ? n.xm : x);
                    const int ty = L::ey(i) == 1 ? n.yp : (L::ey(i) == -1 ? n.ym : y);
                    const int tz = L::ez(i) == 1 ? n.zp : (L::ez(i) == -1 ? n.zm : z);
                    const unsigned trow = (unsigned)tz * (unsigned)g.ny + (unsigned)ty;
                    if (!outside && mask[trow * (unsigned)g.nx + (unsigned)tx]) {
                        const double f = load_f64(at(src, g, i, row, x)) + L::w(i);
                        fx += 2.0 * L::ex(i) * f;
                        fy += 2.0 * L::ey(i) * f;
                        fz += 2.0 * L::ez(i) * f;
                    }
                }
            });
        }
    }
    block_sum3(fx, fy, fz);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const unsigned b = flat_block();
        partials[3 * (size_t)b] = fx;
        partials[3 * (size_t)b + 1] = fy;
        partials[3 * (size_t)b + 2] = fz;
    }
}

template <int BLOCK = 1024>
__global__ void __launch_bounds__(BLOCK)
k_finalize3(const double *__restrict__ partials, int nparts, double *__restrict__ out)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a += partials[3 * (size_t)i];
        b += partials[3 * (size_t)i + 1];
        c += partials[3 * (size_t)i + 2];
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
        out[2] = c;
    }
}

// ---------------------------------------------------------------------------
// Divergence check: scan a whole population buffer (padding and solid slots
// hold zeros) for NaN or infinity, 16 bytes per load, and record the
// earliest step at which one was seen: bad = min(bad, t).  The exponent
// field of a non-finite value is all ones in each storage type.
template <class S>
struct NonFiniteBits;
template <>
struct NonFiniteBits<double> {
    using W = unsigned long long;
    static constexpr W mask = 0x7FF0000000000000ull;
};
template <>
struct NonFiniteBits<float> {
    using W = unsigned int;
    static constexpr W mask = 0x7F800000u;
};
template <>
struct NonFiniteBits<_Float16> {
    using W = unsigned short;
    static constexpr W mask = 0x7C00u;
};
template <>
struct NonFiniteBits<bf16_t> {
    using W = unsigned short;
    static constexpr W mask = 0x7F80u;
};
template <>
struct NonFiniteBits<f16sr_t> : NonFiniteBits<_Float16> {};
template <>
struct NonFiniteBits<bf16sr_t> : NonFiniteBits<bf16_t> {};

template <class S>
__global__ void __launch_bounds__(256)
k_check_finite(const uint4 *__restrict__ buf, long long nvec, long long t,
               unsigned long long *__restrict__ bad)
{
    using B = NonFiniteBits<S>;
    using W = typename B::W;
    constexpr int per = (int)(sizeof(uint4) / sizeof(W));
    bool found = false;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += stride) {
        const uint4 q = buf[v];
        W w[per];
        __builtin_memcpy(w, &q, sizeof(q));
#pragma unroll
        for (int k = 0; k < per; ++k) found |= (w[k] & B::mask) == B::mask;
    }
    if (__any(found) && (threadIdx.x & 63) == 0)
        atomicMin(bad, (unsigned long long)t);
}

} // namespace ptrt
