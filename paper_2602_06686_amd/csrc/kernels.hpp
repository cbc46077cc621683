// HIP kernels of the P-TRT path: the fused stream-and-collide step, the
// state scatter used by initialisation and restore, the gather used by
// moments / populations / diagnostics, and the FP64 reductions.
//
// Layout (one lattice): direction-major planes of shifted populations,
// h[i * qs + node], node = (z * ny + y) * nx + x, x fastest.  qs >= N is the
// plane stride.  A step pulls: population i of node x comes from node
// x - e_i of the previous post-collision state (periodic wrap), or, when that
// node is solid, from direction opp(i) of x itself (halfway bounce-back).
// The stored state is therefore "post-collision at t-1, not yet streamed":
// pulling it gives the pre-collision populations at time t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.hpp"
#include "collide.hpp"
#include "lattice.hpp"

namespace ptrt {

struct Geom {
    int nx, ny, nz;
    long long qs; // plane stride in elements
};

// Source node of population i pulled into (x, y, z), periodic wrap.
template <class L, int I>
__device__ __forceinline__ unsigned source_node(const Geom &g, int x, int y, int z, int xm,
                                                int xp, int ym, int yp, int zm, int zp)
{
    const int sx = L::ex(I) == 1 ? xm : (L::ex(I) == -1 ? xp : x);
    const int sy = L::ey(I) == 1 ? ym : (L::ey(I) == -1 ? yp : y);
    const int sz = L::ez(I) == 1 ? zm : (L::ez(I) == -1 ? zp : z);
    return ((unsigned)sz * (unsigned)g.ny + (unsigned)sy) * (unsigned)g.nx + (unsigned)sx;
}

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

// Pull the Q populations of a fluid node into registers (type T).
template <class L, class S, bool MASK, class T, class LoadF>
__device__ __forceinline__ void pull(const S *__restrict__ src, const uint8_t *__restrict__ mask,
                                     const Geom &g, int x, int y, int z, unsigned node,
                                     T (&h)[L::Q], LoadF load)
{
    const Nbr n(g, x, y, z);
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const S *plane = src + (long long)i * g.qs;
        if constexpr (i == 0) {
            h[0] = load(plane + node);
        } else {
            const unsigned s = source_node<L, i>(g, x, y, z, n.xm, n.xp, n.ym, n.yp, n.zm, n.zp);
            if constexpr (MASK) {
                if (mask[s])
                    h[i] = load(src + (long long)L::opp(i) * g.qs + node);
                else
                    h[i] = load(plane + s);
            } else {
                h[i] = load(plane + s);
            }
        }
    });
}

// Write the pre-collision populations hv (shifted, FP64) of a fluid node into
// the slots its next pull reads: the inverse of pull().
template <class L, class S, bool MASK>
__device__ __forceinline__ void scatter(S *__restrict__ dst, const uint8_t *__restrict__ mask,
                                        const Geom &g, int x, int y, int z, unsigned node,
                                        const double (&hv)[L::Q])
{
    const Nbr n(g, x, y, z);
    static_for<L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i == 0) {
            store_f64(dst + node, hv[0]);
        } else {
            const unsigned s = source_node<L, i>(g, x, y, z, n.xm, n.xp, n.ym, n.yp, n.zm, n.zp);
            if (MASK && mask[s])
                store_f64(dst + (long long)L::opp(i) * g.qs + node, hv[i]);
            else
                store_f64(dst + (long long)i * g.qs + s, hv[i]);
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

// ---------------------------------------------------------------------------
// Fused step: pull, moments, equilibrium, parity split, ghost removal,
// two-rate relaxation, force; store to the node's own slots of dst.
// With DIAG, also reduce mass and kinetic energy of the pulled (pre-collision)
// state into per-block FP64 partials.
template <class L, class S, bool MASK, bool DIAG>
__global__ void __launch_bounds__(256)
k_step(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask, Geom g,
       Relax<typename Codec<S>::compute> r, double2 *__restrict__ partials)
{
    using C = typename Codec<S>::compute;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    bool active = x < g.nx && y < g.ny;
    const unsigned node = ((unsigned)z * (unsigned)g.ny + (unsigned)y) * (unsigned)g.nx + (unsigned)x;
    if (MASK && active) active = mask[node] == 0;
    double m = 0.0, k = 0.0;
    if (active) {
        C h[L::Q];
        pull<L, S, MASK>(src, mask, g, x, y, z, node, h,
                         [](const S *p) { return Codec<S>::load(p); });
        C rho, ux, uy, uz;
        collide<L, C>(h, r, rho, ux, uy, uz);
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            Codec<S>::store(dst + (long long)i * g.qs + node, h[i]);
        });
        if constexpr (DIAG) {
            m = (double)rho;
            k = 0.5 * (double)rho * ((double)ux * ux + (double)uy * uy + (double)uz * uz);
        }
    }
    if constexpr (DIAG) {
        block_sum2(m, k);
        if (threadIdx.x == 0 && threadIdx.y == 0) partials[flat_block()] = make_double2(m, k);
    }
}

// ---------------------------------------------------------------------------
// Scatter a full FP64 state f[Q][N] (unshifted) into dst (pre-collision at t).
template <class L, class S, bool MASK>
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
    scatter<L, S, MASK>(dst, mask, g, x, y, z, node, hv);
}

// Equilibrium initialisation (Eq. feq) in FP64 from rho[N] and u[3][N]
// (either may be null: rho = 1, u = 0), scattered into dst.
template <class L, class S, bool MASK>
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
    scatter<L, S, MASK>(dst, mask, g, x, y, z, node, hv);
}

// ---------------------------------------------------------------------------
// Gather the pre-collision state at t: any of rho[N], u[3][N], f[Q][N]
// (unshifted) and per-block (mass, kinetic energy) partials.  Solid nodes
// report zeros and contribute nothing.
template <class L, class S, bool MASK>
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
        pull<L, S, MASK>(src, mask, g, x, y, z, node, h,
                         [](const S *p) { return load_f64(p); });
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
template <int BLOCK = 256>
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

} // namespace ptrt
