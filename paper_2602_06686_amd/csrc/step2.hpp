// Two fused steps per pass over the populations (temporal blocking) for 3D
// lattices without solids, P-TRT with the default forcing.
//
// A workgroup owns a column of BX = 64 by BY nodes in (x, y) and a chunk of
// ZC planes in z, and marches upwards through its planes.  For each plane k
// it first computes the post-collision state of the first step (A) on the
// column plus a one-node halo in x and y, pulling from HBM, and keeps it in
// LDS in the storage type; it then computes the second step (B) for plane
// k - 1 of the column, pulling the first step's results from LDS, and
// stores those to HBM.  Population i of a B node comes from the A node
// (x, y, z) - e_i: from plane k when e_iz = -1, k - 1 when e_iz = 0 and
// k - 2 when e_iz = +1, so LDS holds the e_z = -1 directions of one plane,
// the e_z = 0 directions of two planes and the e_z = +1 directions of three
// (38 direction planes of 66 x (BY + 2) nodes on D3Q19).  The loads of the
// next plane's first step are issued before the current plane's second
// step, so their latency overlaps it.  The A values pass
// through the storage type exactly as they would through HBM, so two steps
// of this kernel equal two steps of k_step bit for bit.  A chunk recomputes
// the A planes just below and above it (ZC + 2 A planes for ZC B planes).
#pragma once

#include "kernels.hpp"

namespace ptrt {

template <class L>
struct Step2Classes {
    // class of a direction: 0 (e_z = -1), 1 (e_z = 0), 2 (e_z = +1)
    __host__ __device__ static constexpr int cls(int i) { return L::ez(i) + 1; }
    __host__ __device__ static constexpr int count(int c)
    {
        int n = 0;
        for (int i = 0; i < L::Q; ++i) n += cls(i) == c;
        return n;
    }
    __host__ __device__ static constexpr int index(int i)
    {
        int n = 0;
        for (int j = 0; j < i; ++j) n += cls(j) == cls(i);
        return n;
    }
    // slots kept per class: plane k (e_z = -1), k - 1 and k (e_z = 0),
    // k - 2 ... k (e_z = +1)
    __host__ __device__ static constexpr int slots(int c) { return c + 1; }
    __host__ __device__ static constexpr int region(int c)
    {
        int off = 0;
        for (int d = 0; d < c; ++d) off += slots(d) * count(d);
        return off;
    }
    static constexpr int planes = count(0) * slots(0) + count(1) * slots(1) + count(2) * slots(2);
};

// Workgroup rows for the storage type (LDS stays within 64 KB).
template <class L, class S>
struct Step2Shape {
    static constexpr int BX = 64;
    // measured: a gain for D3Q19 in FP32 only; in FP16 / BF16 (and on D3Q27)
    // the one-step kernel is already near its instruction-issue limit and
    // the halo's extra collisions outweigh the halved traffic
    static constexpr int BY = (sizeof(S) == 4 && L::Q == 19) ? 4 : 0;
    static constexpr int AX = BX + 2, AY = BY + 2, AP = AX * AY;
    // one wave per interior row; the A tasks (AY rows and the halo columns)
    // are shared out over them
    static constexpr int WAVES = BY;
    static constexpr size_t lds_bytes = (size_t)Step2Classes<L>::planes * AP * sizeof(S);
    static constexpr bool available = BY > 0 && sizeof(S) <= 4 && lds_bytes <= 163840;
};

// P-TRT collision of the lattice (the hybrid of Eq. PTRT_D3Q27 on D3Q27).
template <class L, class C>
__device__ __forceinline__ void collide_ptrt(C (&h)[L::Q], const Coef<L, C> &r, C &rho, C &ux,
                                             C &uy, C &uz)
{
    if constexpr (L::Q == 27)
        collide_d3q27<C, false>(h, r, rho, ux, uy, uz);
    else
        collide<L, C, true>(h, r, rho, ux, uy, uz);
}

template <class L, class S, bool NT>
__global__ void __launch_bounds__((64 * Step2Shape<L, S>::WAVES))
k_step2(const S *__restrict__ src, S *__restrict__ dst, Geom g,
        Coef<L, typename Codec<S>::compute> r, int zc)
{
    using C = typename Codec<S>::compute;
    using K = Step2Classes<L>;
    using SH = Step2Shape<L, S>;
    constexpr int BX = SH::BX, BY = SH::BY, AX = SH::AX, AY = SH::AY, AP = SH::AP;
    __shared__ S lds[K::planes * AP];

    int bx, by, bz;
    xcd_block(bx, by, bz);
    const int x0 = bx * BX, y0 = by * BY;
    const int zs = bz * zc;
    const int ze = min(zs + zc, g.nz);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    auto wrapc = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    auto ld = [](const S *p) { return Codec<S>::load(p); };

    // LDS element of direction i, slot s, A node a
    auto lds_at = [](int i_cls, int i_idx, int slot, int a) {
        return (K::region(i_cls) + slot * K::count(i_cls) + i_idx) * AP + a;
    };

    // A nodes of a task: rows 0 .. AY-1 at ax = 1 .. 64 (one wave per row,
    // the row uniform across the wave), then task AY: the two halo columns
    // ax = 0 and ax = AX-1 of every row (2 AY lanes of one wave)
    auto a_node = [&](int task, int &ax, int &ay) -> bool {
        if (task < AY) {
            ax = lane + 1;
            ay = task;
            return true;
        }
        ax = lane < AY ? 0 : AX - 1;
        ay = lane < AY ? lane : lane - AY;
        return lane < 2 * AY;
    };
    // first step, part 1: pull the stored values of A node `task` of plane k
    auto load_a = [&](int task, int k, S (&raw)[L::Q]) {
        int ax, ay;
        if (!a_node(task, ax, ay)) return;
        const int gx = wrapc(x0 - 1 + ax, g.nx);
        const int gy = wrapc(y0 - 1 + ay, g.ny);
        const int gz = wrapc(k, g.nz);
        pull<L, S, false>(src, nullptr, g, gx, gy, gz, raw, [](const S *p) { return *p; });
    };
    // part 2: collide and keep the result in the class slots of iteration it
    auto finish_a = [&](int task, int it, const S (&raw)[L::Q]) {
        int ax, ay;
        if (!a_node(task, ax, ay)) return;
        C h[L::Q];
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            h[i] = Codec<S>::load(&raw[i]);
        });
        C rho, ux, uy, uz;
        collide_ptrt<L, C>(h, r, rho, ux, uy, uz);
        const int a = ay * AX + ax;
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int c = K::cls(i);
            const int slot = it % K::slots(c);
            Codec<S>::template store<false>(&lds[lds_at(c, K::index(i), slot, a)], h[i]);
        });
    };

    // each wave owns A tasks w and w + BY (the second when <= AY); the loads
    // of the next plane are issued before the second step of the current
    // one, so that their latency overlaps it
    const int t0 = w, t1 = w + BY;
    const bool has1 = t1 <= AY;
    S raw0[L::Q], raw1[L::Q];
    load_a(t0, zs - 1, raw0);
    if (has1) load_a(t1, zs - 1, raw1);
    for (int k = zs - 1, it = 0; k <= ze; ++k, ++it) {
        finish_a(t0, it, raw0);
        if (has1) finish_a(t1, it, raw1);
        if (k < ze) {
            load_a(t0, k + 1, raw0);
            if (has1) load_a(t1, k + 1, raw1);
        }
        __syncthreads();
        if (k >= zs + 1) {
            // B: second step at interior node (x0 + lane, y0 + w, k - 1)
            const int ax = lane + 1, ay = w + 1;
            C h[L::Q];
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int c = K::cls(i);
                // plane of the source: k (c = 0), k - 1 (c = 1), k - 2 (c = 2)
                const int src_it = it - c;
                const int slot = src_it % K::slots(c);
                const int a = (ay - L::ey(i)) * AX + (ax - L::ex(i));
                h[i] = Codec<S>::load(&lds[lds_at(c, K::index(i), slot, a)]);
            });
            C rho, ux, uy, uz;
            collide_ptrt<L, C>(h, r, rho, ux, uy, uz);
            const int gz = wrapc(k - 1, g.nz);
            const unsigned row = (unsigned)gz * (unsigned)g.ny + (unsigned)(y0 + w);
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                Codec<S>::template store<NT>(at(dst, g, i, row, x0 + lane), h[i]);
            });
        }
        __syncthreads();
    }
}

} // namespace ptrt
