// Two fused steps per pass over the populations (temporal blocking), P-TRT
// with the default forcing: 3D (k_step2 over a grid, k_step2_list over
// task lists with solids) and 2D (k_step2_2d, below).
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
// (38 direction planes of 66 x (BY + 2) nodes on D3Q19).  The workgroup
// barriers order LDS only: they do not wait for global loads (in the FP32
// pass the compiled loop still waits for the next plane's loads before its
// first barrier, which measured faster than keeping them in flight across
// it: loads issued further ahead evict halo lines from L2 before the
// neighbouring columns read them).  The A values pass through the storage type exactly as they
// would through HBM, so two steps of this kernel equal two steps of k_step
// bit for bit.  A chunk recomputes the A planes just below and above it
// (ZC + 2 A planes for ZC B planes).  Measured alternatives that lost:
// forcing the next plane's loads ahead of the second step; BY = 8, 10 or
// 12; a second copy of the halo task on the wave without a second task;
// writing the e_z >= 0 classes to LDS after the second step (24 instead of
// 38 direction planes, three or four workgroups per CU); separate code
// paths for the row and halo tasks; keeping in LDS only the 64 x 4 values
// per direction that the second step reads (three workgroups per CU);
// buffer loads and stores through per-plane descriptors.
#pragma once

#include "kernels.hpp"

namespace ptrt {

// Direction classes along the marching axis (z in 3D, y in 2D).  BB: the
// second step also reads the first step's values of its own node (halfway
// bounce-back), so the e_y = -1 class keeps the plane below too.
template <class L, int AXIS = L::D - 1, bool BB = false>
struct Step2Classes {
    // class of a direction: 0 (e_z = -1), 1 (e_z = 0), 2 (e_z = +1)
    __host__ __device__ static constexpr int cls(int i)
    {
        return (AXIS == 2 ? L::ez(i) : L::ey(i)) + 1;
    }
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
    __host__ __device__ static constexpr int slots(int c) { return BB && c == 0 ? 2 : c + 1; }
    __host__ __device__ static constexpr int region(int c)
    {
        int off = 0;
        for (int d = 0; d < c; ++d) off += slots(d) * count(d);
        return off;
    }
    static constexpr int planes = count(0) * slots(0) + count(1) * slots(1) + count(2) * slots(2);
};

// Workgroup rows for the storage type.
template <class L, class S, bool MASK = false>
struct Step2Shape {
    static constexpr int BX = 64;
    // measured: a gain for D3Q19 in FP32 and FP64 (one workgroup per CU,
    // +18 % at 256^3); in FP16 / BF16 and on D3Q27 the one-step kernel is
    // already near its instruction-issue limit and the halo's extra
    // collisions outweigh the halved traffic
    static constexpr int BY = ((sizeof(S) == 4 || sizeof(S) == 8) && L::Q == 19) ? 4 : 0;
    static constexpr int AX = BX + 2, AY = BY + 2, AP = AX * AY;
    // one wave per interior row; the AY + 1 first-step tasks (AY rows and
    // the halo columns) are shared out over them, at most two per wave
    static constexpr int WAVES = BY;
    // MASK: the e_z = -1 class keeps the plane below too (bounce-back reads
    // the node's own first-step values of the previous plane)
    using K = Step2Classes<L, L::D - 1, MASK>;
    static constexpr size_t lds_bytes = (size_t)K::planes * AP * sizeof(S);
    static constexpr bool available =
        BY >= 3 && lds_bytes <= 163840 && AY + 1 <= 2 * WAVES;
};

// Workgroup barrier that orders the LDS accesses only: the global loads in
// flight (the next plane's first-step pulls) stay in flight across it,
// where __syncthreads() would wait for them.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Collision of a pass: P-TRT (the hybrid of Eq. PTRT_D3Q27 on D3Q27), or
// for the efficiency comparison TRT-RLB (Eq. TRT-RLB) or standard TRT, the
// same functions as in the one-step kernel (default forcing).
template <class L, class S, int MODEL = MODEL_PTRT, class C = typename Codec<S>::compute>
__device__ __forceinline__ void collide_pass(C (&h)[L::Q], const Coef<L, C> &r, C &rho, C &ux,
                                             C &uy, C &uz)
{
    constexpr bool FR = Codec<S>::fast_recip;
    if constexpr (MODEL == MODEL_TRT_RLB)
        collide_trt_rlb<L, C, FR>(h, r, rho, ux, uy, uz);
    else if constexpr (MODEL == MODEL_TRT)
        collide<L, C, false, FORCE_II, FR>(h, r, rho, ux, uy, uz);
    else if constexpr (L::Q == 27)
        collide_d3q27<C, false, FORCE_II, FR>(h, r, rho, ux, uy, uz);
    else
        collide<L, C, true, FORCE_II, FR>(h, r, rho, ux, uy, uz);
}

// One column chunk of the pass, run by the workgroup: second steps for
// planes zs ... ze - 1 (ze > zs) of the column x0 ... x0 + BX - 1, y0 ...
// y0 + BY - 1, first steps in lds.  MASK: halfway bounce-back in both
// steps (the first step pulls through pull<L, S, true>; the second takes
// the node's own first-step value of the opposite direction where the
// source node is solid, and solid nodes are not stored).
template <class L, class S, bool NT, bool MASK, int MODEL = MODEL_PTRT, bool ZOFF = false>
__device__ __forceinline__ void
step2_3d_task(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask,
              const Geom &g, const Coef<L, typename Codec<S>::compute> &r, S *lds, int x0, int y0,
              int zs, int ze)
{
    using C = typename Codec<S>::compute;
    using SH = Step2Shape<L, S, MASK>;
    using K = typename SH::K;
    constexpr int BY = SH::BY, AX = SH::AX, AY = SH::AY, AP = SH::AP;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    auto wrapc = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };

    // LDS element of direction i, slot s, A node a
    auto lds_at = [](int i_cls, int i_idx, int slot, int a) {
        return (K::region(i_cls) + slot * K::count(i_cls) + i_idx) * AP + a;
    };

    // A nodes of a task: rows 0 .. AY-1 at ax = 1 .. 64 (one wave per row,
    // the row uniform across the wave), then task AY: the two halo columns
    // ax = 0 and ax = AX-1 of every row (2 AY lanes of one wave; the other
    // lanes load and compute the last node again and keep nothing)
    auto a_node = [&](int task, int &ax, int &ay) -> bool {
        if (task < AY) {
            ax = lane + 1;
            ay = task;
            return true;
        }
        ax = lane < AY ? 0 : AX - 1;
        ay = lane < AY ? lane : min(lane - AY, AY - 1);
        return lane < 2 * AY;
    };
    // first step, part 1: pull the stored values of A node `task` of plane k
    // (every lane loads, so that no load sits in a branch)
    auto load_a = [&](int task, int k, S (&raw)[L::Q]) {
        int ax, ay;
        a_node(task, ax, ay);
        const int gx = wrapc(x0 - 1 + ax, g.nx);
        const int gy = wrapc(y0 - 1 + ay, g.ny);
        const int gz = wrapc(k, g.nz);
        pull<L, S, MASK>(src, mask, g, gx, gy, gz, raw, [](const S *p) { return *p; });
    };
    // the same for a row task (ay < AY): the nine source rows are uniform
    // across the wave (scalar offsets, each computed once), the lane's three
    // source columns fixed for the workgroup (nx is a multiple of BX, so
    // x0 + lane needs no wrap)
    const int rx = x0 + lane;
    const int rxm = rx == 0 ? g.nx - 1 : rx - 1, rxp = rx == g.nx - 1 ? 0 : rx + 1;
    const unsigned rmask = (1u << g.lr) - 1u;
    const unsigned xb = (unsigned)rx * sizeof(S), xbm = (unsigned)rxm * sizeof(S),
                   xbp = (unsigned)rxp * sizeof(S);
    auto load_row = [&](int ay, int k, S (&raw)[L::Q]) {
        const int gy = wrapc(y0 - 1 + ay, g.ny);
        const int gz = wrapc(k, g.nz);
        const int ys3[3] = {gy == 0 ? g.ny - 1 : gy - 1, gy, gy == g.ny - 1 ? 0 : gy + 1};
        const int zs3[3] = {gz == 0 ? g.nz - 1 : gz - 1, gz, gz == g.nz - 1 ? 0 : gz + 1};
        // byte offsets of the source rows (index 1 - e: the row of node
        // (y, z) - e), each computed once
        long long ro[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const unsigned row = (unsigned)zs3[a] * (unsigned)g.ny + (unsigned)ys3[b];
                ro[a][b] = ((long long)(row >> g.lr) * g.tile +
                            (long long)((row & rmask) * (unsigned)g.pitch)) *
                           (long long)sizeof(S);
            }
        const char *sb = reinterpret_cast<const char *>(src);
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const unsigned xo = L::ex(i) == 1 ? xbm : (L::ex(i) == -1 ? xbp : xb);
            const char *p = sb + ro[1 - L::ez(i)][1 - L::ey(i)] +
                            (long long)i * (long long)g.plane * (long long)sizeof(S) + xo;
            raw[i] = *reinterpret_cast<const S *>(p);
        });
    };
    // ZOFF: the source offsets of a task's pulls inside a z plane stay the
    // same all the way up the column (the lane's node moves in z only), so
    // they are formed once; a pull is then the scalar base of its source
    // plane plus that 32-bit lane offset (step2_zoff_ok: a z plane is a
    // whole number of row tiles, below 2^32 bytes).  Measured in FP32:
    // 1017 -> 790 VALU instructions per plane and wave, +3-6 % at 256^3 -
    // 512^3.  FP64 keeps load_row (its registers are all in use).
    static_assert(!ZOFF || (sizeof(S) == 4 && !MASK), "source offsets: FP32 without solids");
    const long long zstride = (long long)(g.ny >> g.lr) * g.tile * (long long)sizeof(S);
    auto make_off = [&](int task, auto &off) {
        int ax, ay;
        a_node(task, ax, ay);
        const int gx = wrapc(x0 - 1 + ax, g.nx), gy = wrapc(y0 - 1 + ay, g.ny);
        const unsigned m = (1u << g.lr) - 1u;
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const int sx = wrapc(gx - L::ex(i), g.nx), sy = wrapc(gy - L::ey(i), g.ny);
            off[i] = ((unsigned)(sy >> g.lr) * (unsigned)g.tile + (unsigned)i * (unsigned)g.plane +
                      ((unsigned)sy & m) * (unsigned)g.pitch + (unsigned)sx) *
                     (unsigned)sizeof(S);
        });
    };
    auto load_off = [&](const auto &off, int k, S (&raw)[L::Q]) {
        const int gz = wrapc(k, g.nz);
        const int zm = gz == 0 ? g.nz - 1 : gz - 1, zp = gz == g.nz - 1 ? 0 : gz + 1;
        const char *sb = reinterpret_cast<const char *>(src);
        const char *base[3] = {sb + (long long)zm * zstride, sb + (long long)gz * zstride,
                               sb + (long long)zp * zstride};
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            raw[i] = *reinterpret_cast<const S *>(base[1 - L::ez(i)] + off[i]);
        });
    };
    // part 2: collide and keep the result in the class slots of plane `it`
    auto finish_a = [&](int task, int it, const S (&raw)[L::Q]) {
        int ax, ay;
        const bool valid = a_node(task, ax, ay);
        C h[L::Q];
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            h[i] = Codec<S>::load(&raw[i]);
        });
        C rho, ux, uy, uz;
        collide_pass<L, S, MODEL>(h, r, rho, ux, uy, uz);
        if (!valid) return;
        const int a = ay * AX + ax;
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int c = K::cls(i);
            Codec<S>::template store<false>(&lds[lds_at(c, K::index(i), it % K::slots(c), a)],
                                            h[i]);
        });
    };

    // each wave owns A tasks w and w + BY (the second when <= AY); the
    // optional task's loads go first, so that the wait for the other task's
    // loads never has to count them
    const int t0 = w, t1 = w + BY;
    const bool has1 = t1 <= AY;
    S raw0[L::Q], raw1[L::Q];
    unsigned off0[ZOFF ? L::Q : 1], off1[ZOFF ? L::Q : 1];
    if constexpr (ZOFF) {
        make_off(t0, off0);
        make_off(t1, off1);
    }
    // FP64 (one workgroup per CU, so no other workgroup's work covers the
    // load latency) keeps the loads of two planes in flight, in a second
    // register set used on alternate planes (loop unrolled by two; measured
    // at 256^3: 25.0 -> 29.3 GLUPS).  FP32, with two workgroups per CU,
    // lost with the same (256^3 56.5 -> 53.4, 512^3 57.4 -> 49.8).
    constexpr bool DEEP = sizeof(S) == 8;
    S rawb0[DEEP ? L::Q : 1], rawb1[DEEP ? L::Q : 1];
    // row tasks in FP64 take load_row (measured at 256^3: FP64 +5.6 %;
    // FP32 +1 % at 256^3 and -1.7 % at 512^3, so FP32 keeps load_a)
    auto load_both = [&](int k) {
        if constexpr (sizeof(S) == 8 && !MASK) {
            if (has1) {
                if (t1 < AY)
                    load_row(t1, k, raw1);
                else
                    load_a(t1, k, raw1);
            }
            load_row(t0, k, raw0);
        } else if constexpr (ZOFF) {
            if (has1) load_off(off1, k, raw1);
            load_off(off0, k, raw0);
        } else {
            if (has1) load_a(t1, k, raw1);
            load_a(t0, k, raw0);
        }
    };
    auto finish_both = [&](int it) {
        if (has1) finish_a(t1, it, raw1);
        finish_a(t0, it, raw0);
    };
    // the same for the second register set (FP64 only; generic lambdas, so
    // that they are instantiated only where called)
    auto load_second_set = [&](auto k) {
        if constexpr (!MASK) {
            if (has1) {
                if (t1 < AY)
                    load_row(t1, k, rawb1);
                else
                    load_a(t1, k, rawb1);
            }
            load_row(t0, k, rawb0);
        } else {
            if (has1) load_a(t1, k, rawb1);
            load_a(t0, k, rawb0);
        }
    };
    auto finish_second_set = [&](auto it) {
        if (has1) finish_a(t1, it, rawb1);
        finish_a(t0, it, rawb0);
    };
    // first-step planes zs - 1, zs and zs + 1 (ze >= zs + 1), then for
    // k = zs + 1 ... ze the second step of plane k - 1 followed by the first
    // step of plane k + 1 (past the chunk the last plane is loaded again,
    // so that the loop has no load or store under a branch).  Measured: the
    // compiler's placement of the next plane's loads (after the second
    // step, in the same block as their collisions) beats forcing them ahead
    // of the second step.
    load_both(zs - 1);
    finish_both(0);
    load_both(zs);
    finish_both(1);
    load_both(zs + 1);
    finish_both(2);
    // the second step of plane k - 1, iteration it (first-step planes up to
    // k in lds)
    auto second = [&](int k, int it) __attribute__((always_inline)) {
        {
            // B: second step at interior node (x0 + lane, y0 + w, k - 1)
            const int ax = lane + 1, ay = w + 1;
            // past ny (the last workgroup row when BY does not divide ny)
            // the wrapped row is computed again: the same values as its
            // own workgroup writes
            const int gz = wrapc(k - 1, g.nz);
            const int gy = wrapc(y0 + w, g.ny);
            const unsigned row = (unsigned)gz * (unsigned)g.ny + (unsigned)gy;
            bool store = true;
            if constexpr (MASK) store = !mask[row * (unsigned)g.nx + (unsigned)(x0 + lane)];
            C h[L::Q];
            if constexpr (MASK) {
                const Nbr n(g, x0 + lane, gy, gz);
                static_for<L::Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int c = K::cls(i);
                    const int slot = (it - c) % K::slots(c);
                    int at_i = lds_at(c, K::index(i), slot, (ay - L::ey(i)) * AX + (ax - L::ex(i)));
                    if constexpr (i != 0) {
                        // solid source: the node's own first-step value of
                        // the opposite direction, plane k - 1 (iteration it - 1)
                        int sx;
                        unsigned srow;
                        source_of<L, i>(g, n, x0 + lane, gy, gz, sx, srow);
                        constexpr int io = L::opp(i), co = K::cls(io);
                        if (mask[srow * (unsigned)g.nx + (unsigned)sx])
                            at_i = lds_at(co, K::index(io), (it - 1) % K::slots(co), ay * AX + ax);
                    }
                    h[i] = Codec<S>::load(&lds[at_i]);
                });
            } else {
                static_for<L::Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int c = K::cls(i);
                    // plane of the source: k (c = 0), k - 1 (c = 1), k - 2 (c = 2)
                    const int slot = (it - c) % K::slots(c);
                    const int a = (ay - L::ey(i)) * AX + (ax - L::ex(i));
                    h[i] = Codec<S>::load(&lds[lds_at(c, K::index(i), slot, a)]);
                });
            }
            C rho, ux, uy, uz;
            collide_pass<L, S, MODEL>(h, r, rho, ux, uy, uz);
            if (store) {
                static_for<L::Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    Codec<S>::template store<NT>(at(dst, g, i, row, x0 + lane), h[i]);
                });
            }
        }
    };
    load_both(min(zs + 2, ze));
    if constexpr (DEEP) {
        // two planes in flight: the first step of plane k + 1 takes the set
        // loaded two iterations before, which then loads plane k + 3
        load_second_set(min(zs + 3, ze));
        for (int k = zs + 1, it = 2;; k += 2, it += 2) {
            lds_barrier();
            second(k, it);
            lds_barrier();
            if (k == ze) break;
            finish_both(it + 1);
            load_both(min(k + 3, ze));
            lds_barrier();
            second(k + 1, it + 1);
            lds_barrier();
            if (k + 1 == ze) break;
            finish_second_set(it + 2);
            load_second_set(min(k + 4, ze));
        }
    } else {
        for (int k = zs + 1, it = 2;; ++k, ++it) {
            lds_barrier();
            second(k, it);
            lds_barrier();
            if (k == ze) break;
            finish_both(it + 1);
            load_both(min(k + 2, ze));
        }
    }
}

// Per-task source offsets of the first step's pulls (ZOFF in
// step2_3d_task): FP32, a z plane a whole number of row tiles (ny a
// multiple of 2^lr, so that a node's row offset splits into a z part and a
// y part) and below 2^32 bytes (the offsets are 32-bit).
template <class S>
inline bool step2_zoff_ok(const Geom &g)
{
    if (sizeof(S) != 4 || g.ny % (1 << g.lr) != 0) return false;
    return (double)(g.ny >> g.lr) * (double)g.tile * (double)sizeof(S) < 4294967296.0;
}

// Grid (x blocks, y blocks, z chunks of zc planes), without solids; the
// launch covers workgroup rows by0 ... by0 + gridDim.y - 1.
template <class L, class S, bool NT, int MODEL = MODEL_PTRT, bool ZOFF = false>
__global__ void __launch_bounds__((64 * Step2Shape<L, S>::WAVES))
k_step2(const S *__restrict__ src, S *__restrict__ dst, Geom g,
        Coef<L, typename Codec<S>::compute> r, int zc, int by0)
{
    using SH = Step2Shape<L, S>;
    __shared__ S lds[SH::K::planes * SH::AP];
    int bx, by, bz;
    xcd_block(bx, by, bz);
    const int zs = bz * zc;
    step2_3d_task<L, S, NT, false, MODEL, ZOFF>(src, dst, nullptr, g, r, lds, bx * SH::BX,
                                                (by0 + by) * SH::BY, zs, min(zs + zc, g.nz));
}

// Task list (with solids): workgroup t runs tasks[t] = {x0, y0, zs, ze}.
template <class L, class S, bool NT, bool MASK, bool ZOFF = false>
__global__ void __launch_bounds__((64 * Step2Shape<L, S, MASK>::WAVES))
k_step2_list(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask,
             Geom g, Coef<L, typename Codec<S>::compute> r, const int4 *__restrict__ tasks,
             int ntasks)
{
    using SH = Step2Shape<L, S, MASK>;
    __shared__ S lds[SH::K::planes * SH::AP];
    int t, unused_y, unused_z;
    xcd_block(t, unused_y, unused_z);
    if (t >= ntasks) return;
    const int4 tk = tasks[t];
    step2_3d_task<L, S, NT, MASK, MODEL_PTRT, ZOFF>(src, dst, mask, g, r, lds, tk.x, tk.y, tk.z,
                                                   tk.w);
}

// Two fused steps per pass for D2Q9 without solids (the 2D counterpart of
// k_step2): each wave of a workgroup owns a strip of 62 columns and a
// chunk of rows and marches up through its rows, on its own.  For row k the wave
// computes the first step (A) on 64 nodes, columns x0 - 1 ... x0 + 62 (the
// strip plus a one-column halo on each side), pulling from HBM, and keeps
// the results in LDS in the storage type; lanes 1 ... 62 then compute the
// second step (B) for row k - 1 from LDS and store it; the loads of rows
// k + 1 and k + 2 are in flight meanwhile.  Population i of a B
// node comes from the A node (x, y) - e_i: row k when e_iy = -1, k - 1 when
// e_iy = 0, k - 2 when e_iy = +1 (1 + 2 + 3 slots of three directions,
// 18 rows of 64 values).  Bit-identical to two one-step launches.
template <class S, bool MASK = false>
struct Step2Shape2D {
    static constexpr int W = 64;     // A nodes per row (one wave)
    static constexpr int BX = W - 2; // interior columns per strip
    // waves (independent strips) per workgroup: measured best at 2048^2 and
    // 4096^2 in FP32 and FP64 (rows per chunk: chosen per lattice)
    static constexpr int NW = 4;
    using K = Step2Classes<D2Q9, 1, MASK>;
    static constexpr size_t lds_bytes = (size_t)K::planes * W * sizeof(S);
};

// Order of the LDS accesses of one wave (its lanes exchange values only
// with each other).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One task of the two-step pass, run by one wave: second steps for rows ys
// ... ye - 1 (ye > ys) of the strip of columns x0 ... x0 + BX - 1 (those
// inside the lattice), first steps kept in the wave's K::planes rows of W
// values at lds.  MASK: the task reads the mask (halfway bounce-back; a
// task whose rows ys - 1 ... ye hold no solid within one row may run with
// MASK = false): the first step pulls the node's own opposite population
// where the source is solid, the second step likewise from the first
// step's values of its own node, and solid second-step nodes are not
// stored (as in the one-step kernel).  OPEN: x is not periodic (velocity
// inlet at x = 0, Zou-He outlet at x = nx - 1, as pull<..., OPEN>): in
// both steps the populations entering the inlet node are its own outgoing
// ones plus 6 w_i u_in (the second step reads them from its own node's
// first-step values, like bounce-back), and the outlet node's entering
// ones come from zou_he_east; the first-step values across the x seam are
// then never read.
template <class S, bool NT, bool MASK, bool OPEN = false, int MODEL = MODEL_PTRT>
__device__ __forceinline__ void
step2_2d_task(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask,
              const Geom &g, const Coef<D2Q9, typename Codec<S>::compute> &r, S *lds, int x0,
              int ys, int ye)
{
    using L = D2Q9;
    using C = typename Codec<S>::compute;
    using SH = Step2Shape2D<S, MASK || OPEN>;
    using K = typename SH::K;
    constexpr int W = SH::W, BX = SH::BX;
    const int lane = (int)(threadIdx.x & 63);
    auto wrapc = [](int v, int n) {
        v %= n;
        return v < 0 ? v + n : v;
    };
    const int ax = wrapc(x0 - 1 + lane, g.nx); // this lane's A column
    const int axm = wrapc(ax - 1, g.nx), axp = wrapc(ax + 1, g.nx);
    auto lds_at = [](int c, int idx, int slot, int a) {
        return (K::region(c) + slot * K::count(c) + idx) * W + a;
    };
    auto wrapr = [&](int v) { return ((v % g.ny) + g.ny) % g.ny; };

    // Addresses: the rows in use (k - 2 ... k + 3 while the march is at row
    // k) sit in a window, o[j] their byte offsets and rw[j] their indices,
    // that advances by one row per step (one new row offset per row, with
    // a wrap test); each population adds its direction's fixed offset, and
    // the lane's x offsets are fixed for the task: little scalar work per
    // row.
    const unsigned rmask = (1u << g.lr) - 1u;
    auto row_off_w = [&](int u) -> size_t { // u in [0, ny)
        return ((size_t)((unsigned)u >> g.lr) * (size_t)g.tile +
                (size_t)(((unsigned)u & rmask) * (unsigned)g.pitch)) *
               sizeof(S);
    };
    const size_t dir_bytes = (size_t)g.plane * sizeof(S);
    const unsigned xo_m = (unsigned)axm * (unsigned)sizeof(S);
    const unsigned xo_0 = (unsigned)ax * (unsigned)sizeof(S);
    const unsigned xo_p = (unsigned)axp * (unsigned)sizeof(S);
    size_t o[6];
    int rw[6];
    auto shift = [&]() {
        static_for<5>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            o[j] = o[j + 1];
            rw[j] = rw[j + 1];
        });
        rw[5] = rw[4] + 1 == g.ny ? 0 : rw[4] + 1;
        o[5] = row_off_w(rw[5]);
    };
    // solid flag of node (column of lane + dx, window row j)
    auto solid = [&](int j, int dx) -> bool {
        const int x = dx < 0 ? axm : (dx > 0 ? axp : ax);
        return mask[(size_t)rw[j] * (unsigned)g.nx + (unsigned)x] != 0;
    };
    // first-step pull of window row J: population i of (x, y) comes from
    // (x, y) - e_i, or from the node's own opposite population when that
    // source is solid
    auto load_a = [&](auto jc, S (&raw)[L::Q]) {
        constexpr int J = decltype(jc)::value;
        const char *sb = reinterpret_cast<const char *>(src);
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int js = J - L::ey(i);
            const unsigned xo = L::ex(i) == 1 ? xo_m : (L::ex(i) == -1 ? xo_p : xo_0);
            const char *p = sb + o[js] + (size_t)i * dir_bytes + xo;
            if constexpr (MASK && i != 0) {
                if (solid(js, -L::ex(i)))
                    p = sb + o[J] + (size_t)L::opp(i) * dir_bytes + xo_0;
            }
            if constexpr (OPEN && L::ex(i) == 1) {
                if (ax == 0) p = sb + o[J] + (size_t)L::opp(i) * dir_bytes + xo_0;
            }
            raw[i] = *reinterpret_cast<const S *>(p);
        });
    };
    // open x: the inlet term on the populations entering node x = 0 (their
    // values are already the node's own outgoing ones), Zou-He at nx - 1
    auto open_fix = [&](C(&h)[L::Q], int x) {
        if (x == 0) {
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (L::ex(i) == 1) h[i] = h[i] + C(6.0 * L::w(i)) * C(g.uin);
            });
        }
        if (x == g.nx - 1) zou_he_east(h, C(g.drhoout));
    };
    auto finish_a = [&](int it, const S (&raw)[L::Q]) {
        C h[L::Q];
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            h[i] = Codec<S>::load(&raw[i]);
        });
        if constexpr (OPEN) open_fix(h, ax);
        C rho, ux, uy, uz;
        collide_pass<L, S, MODEL>(h, r, rho, ux, uy, uz);
        static_for<L::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int c = K::cls(i);
            Codec<S>::template store<false>(&lds[lds_at(c, K::index(i), it % K::slots(c), lane)], h[i]);
        });
    };

    // B lanes: 1 ... BX, inside the lattice (the last strip may be partial)
    const int bxg = x0 - 1 + lane;
    const bool b_lane = lane >= 1 && lane <= BX && bxg < g.nx;
    // one row of the march: finish A of row k from raw, refill raw with the
    // loads of row k + 2 (two rows in flight; past the chunk they are not
    // used), B of row k - 1 (window row 1).  Every wave issues the same
    // loads and stores on every row, so the wait before a row's first-step
    // collision covers only that row's loads, not the stores and the loads
    // issued after them.
    auto row_step = [&](int it, S (&raw)[L::Q]) {
        finish_a(it, raw);
        load_a(std::integral_constant<int, 4>{}, raw);
        wave_lds_sync();
        bool store = b_lane;
        if constexpr (MASK) store = store && !solid(1, 0);
        if (store) {
            C h[L::Q];
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int c = K::cls(i);
                const int slot = (it - c) % K::slots(c);
                int at_i = lds_at(c, K::index(i), slot, lane - L::ex(i));
                if constexpr (MASK && i != 0) {
                    // own node's first-step value of the opposite direction,
                    // row k - 1 (iteration it - 1)
                    constexpr int io = L::opp(i), co = K::cls(io);
                    if (solid(1 - L::ey(i), -L::ex(i)))
                        at_i = lds_at(co, K::index(io), (it - 1) % K::slots(co), lane);
                }
                if constexpr (OPEN && L::ex(i) == 1) {
                    constexpr int io = L::opp(i), co = K::cls(io);
                    if (bxg == 0) at_i = lds_at(co, K::index(io), (it - 1) % K::slots(co), lane);
                }
                h[i] = Codec<S>::load(&lds[at_i]);
            });
            if constexpr (OPEN) open_fix(h, bxg);
            C rho, ux, uy, uz;
            collide_pass<L, S, MODEL>(h, r, rho, ux, uy, uz);
            char *db = reinterpret_cast<char *>(dst) + o[1];
            static_for<L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                Codec<S>::template store<NT>(
                    reinterpret_cast<S *>(db + (size_t)i * dir_bytes + xo_0), h[i]);
            });
        }
        wave_lds_sync();
        shift();
    };
    // window at rows ys - 2 ... ys + 3: A rows ys - 1 and ys (no B yet, ye >=
    // ys + 1), then rows ys + 1 ... ye with B, alternating between two
    // register sets
    for (int j = 0; j < 6; ++j) {
        rw[j] = wrapr(ys - 2 + j);
        o[j] = row_off_w(rw[j]);
    }
    S raw0[L::Q], raw1[L::Q];
    load_a(std::integral_constant<int, 1>{}, raw0);
    load_a(std::integral_constant<int, 2>{}, raw1);
    finish_a(0, raw0);
    load_a(std::integral_constant<int, 3>{}, raw0);
    finish_a(1, raw1);
    load_a(std::integral_constant<int, 4>{}, raw1);
    shift(); // window at rows ys - 1 ... ys + 4 = k - 2 ... k + 3, k = ys + 1
    // pairs of rows with one exit test, so that the back edge is the only
    // path into the loop head
    const int nb = ye - ys;
    int it = 2;
    for (int p = 0; p < (nb >> 1); ++p, it += 2) {
        row_step(it, raw0);
        row_step(it + 1, raw1);
    }
    if (nb & 1) row_step(it, raw0);
}

// Task t of the launch: task_list[t] = {unused, x0, ys, ye}, or without a
// list (strip, chunk) = (t % strips, t / strips) with chunks of yc rows,
// the last partial.  The NW waves of a workgroup run independent tasks
// (neighbouring strips of one chunk).  Eight waves per SIMD: FP32 fits in
// 64 VGPRs (measured +1.5 % at 4096^2).
template <class S, bool NT, int NW, bool MASK, bool OPEN, int MODEL = MODEL_PTRT>
__global__ void __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(8, 8)))
k_step2_2d(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask,
           const int4 *__restrict__ task_list, Geom g, Coef<D2Q9, typename Codec<S>::compute> r,
           int yc, int strips, int tasks)
{
    using SH = Step2Shape2D<S, MASK || OPEN>;
    __shared__ S lds_all[NW * SH::K::planes * SH::W];
    int wg, unused_y, unused_z;
    xcd_block(wg, unused_y, unused_z);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int t = wg * NW + w;
    if (t >= tasks) return;
    int x0, ys, ye;
    if (task_list) {
        const int4 tk = task_list[t];
        x0 = tk.y;
        ys = tk.z;
        ye = tk.w;
    } else {
        const int bx = t % strips, by = t / strips;
        x0 = bx * SH::BX;
        ys = by * yc;
        ye = min(ys + yc, g.ny);
    }
    step2_2d_task<S, NT, MASK, OPEN, MODEL>(src, dst, mask, g, r,
                                            lds_all + w * (SH::K::planes * SH::W), x0, ys, ye);
}

} // namespace ptrt
