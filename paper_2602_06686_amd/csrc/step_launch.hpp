// Launch of one fused step of a single lattice (and, for Scheme II with the
// cubic correction, the Phi pass before it).  The template is instantiated
// once per lattice in step_d2q9.hip, step_d3q19.hip and step_d3q27.hip, so
// the three lattices' kernels compile as separate translation units.
#pragma once

#include <algorithm>
#include <vector>

#include "host_common.hpp"
#include "step2.hpp"

namespace ptrt {

struct StepLaunch {
    const void *src = nullptr; // stored state (post-collision at t-1)
    void *dst = nullptr;       // next state
    const uint8_t *mask = nullptr, *near = nullptr;
    Geom g{};
    double tau_plus = 0, Lambda = 0, force[3] = {0, 0, 0};
    int storage = PTRT_F32;
    bool has_mask = false;
    bool row = true;  // row workgroups of row_bx threads, else 64 x 4 tiles
    int row_bx = 256;
    bool nt = false;  // non-temporal stores
    int model = MODEL_PTRT, forcing = FORCE_II;
    void *phi = nullptr; // Phi field in the compute type (FORCE_II_G)
    bool open = false;   // D2Q9 inlet / outlet in x (values in g)
    hipStream_t stream = nullptr;
    // D2Q9 with solids or open x, two steps per pass: the tasks {unused,
    // x0, ys, ye} for the mask-free periodic kernel and the special ones
    // (a solid within one row of their rows, or a strip at an open x
    // boundary), and the rows of the chunks near solids
    const int4 *tasks_plain = nullptr, *tasks_special = nullptr;
    int n_plain = 0, n_special = 0;
    long long masked_rows = 0;
};

void launch_step_d2q9(const StepLaunch &a);
void launch_step_d3q19(const StepLaunch &a);
void launch_step_d3q27(const StepLaunch &a);

// Two steps in one pass (step2.hpp) when the configuration allows it:
// returns false (nothing launched) otherwise.
// *pass_bytes: the algorithmic HBM bytes of the pass (the state read once
// and written once).
bool launch_step2_d2q9(const StepLaunch &a, double *pass_bytes);
bool launch_step2_d3q19(const StepLaunch &a, double *pass_bytes);
bool launch_step2_d3q27(const StepLaunch &a, double *pass_bytes);

// Rows per chunk of the D2Q9 two-step kernel for an nx x ny lattice.  A
// wave computes the first step on yc + 2 rows to finish yc, so short chunks
// repeat first-step work but give more tasks to spread over the chip;
// measured (64^2 ... 4096^2, FP32 and FP64) best near 1600 tasks in FP32
// and 800 in FP64 (a fifth of the waves the chip holds at once, 32 and 16
// per CU as LDS allows), at most 9 rows (7 from 2^22 nodes on, 2 - 3 %
// faster there), and never 4 or 8, which measured 5 - 15 % slower than 5
// and 9 at 724^2 - 1024^2.
// strip_rows: strips x rows summed over the lattices of the launch, nodes:
// their nodes; scale multiplies the task target.
inline int step2_2d_rows_for(int storage, long long strip_rows, long long nodes, int scale = 1)
{
    const long long target = (storage == PTRT_F64 ? 800 : 1600) * (long long)scale;
    const long long cap = nodes >= (1LL << 22) ? 7 : 9;
    long long yc = std::min(cap, std::max(1LL, (strip_rows + target - 1) / target));
    if (yc == 4 || yc == 8) ++yc;
    return (int)yc;
}

inline int step2_2d_rows(int storage, int nx, int ny)
{
    const long long strips = (nx + Step2Shape2D<float>::BX - 1) / Step2Shape2D<float>::BX;
    return step2_2d_rows_for(storage, strips * ny, (long long)nx * ny);
}

// Workgroups of the 3D two-step pass resident at once on the device
// (per CU, from the occupancy query, times the CUs).
template <class L, class S>
int step2_3d_resident()
{
    using SH = Step2Shape<L, S>;
    // queried once per process (one device type), by a thread-safe static
    // initialisation: handles used from several threads may get here at once
    static const int resident = [] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(&k_step2<L, S, true>),
                64 * SH::WAVES, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            per_cu <= 0 || cus <= 0)
            return 512;
        return per_cu * cus;
    }();
    return resident;
}

// Planes per z chunk of the 3D two-step pass (grid or task list).
template <class L, class S>
int step2_3d_zc(const Geom &g)
{
    using SH = Step2Shape<L, S>;
    // z chunks: the workgroups run in rounds of R = (workgroups
    // resident per CU) x CUs, and a workgroup's time grows with
    // its zc + 2 first-step planes, so zc minimises
    // ceil(cols * ceil(nz / zc) / R) * (zc + 2) (measured at
    // 384^3: 576 workgroups of the whole depth, 1.1 rounds,
    // 34.9 GLUPS)
    const int rows = (g.ny + SH::BY - 1) / SH::BY;
    const long long cols = (long long)(g.nx / SH::BX) * rows;
    const int resident = step2_3d_resident<L, S>();
    // candidates: zc = ceil(nz / c) for c = 1, 2, ... chunks, down
    // to 8 planes or until the last round is under 1/16 of the
    // work (more chunks then only add halo planes)
    int zc = g.nz;
    double best = -1.0;
    for (int c = 1;; ++c) {
        const int z = (g.nz + c - 1) / c;
        const long long wgs = cols * ((g.nz + z - 1) / z);
        const double cost = (double)((wgs + resident - 1) / resident) * (z + 2);
        if (best < 0 || cost < best) {
            best = cost;
            zc = z;
        }
        if (z <= 8 || wgs >= 16LL * resident) break;
    }
    return zc;
}

// Task lists of the 3D two-step pass with solids: the column chunks {x0,
// y0, zs, ze} of the grid launch (zc planes) none of whose first-step rows
// y0 - 1 ... y0 + BY, zs - 1 ... ze has a solid within one row (near, per
// row z ny + y) go to the mask-free list; the others, split into chunks of
// ZM planes, to the masked list (short chunks: the masked code is slower,
// and with few such columns their time is latency).  false when the pass
// does not apply, below 2^24 nodes or with more than 5 % of the chunks
// masked (measured, one step -> two, GLUPS FP32 / FP64: channel 256^3,
// 3 % masked, 40.0 -> 45.2 / 19.5 -> 22.6; a cube over 1/8 of each axis
// at 256^3, 16 % masked, 39.7 -> 36.4 / 19.6 -> 17.7; channel 128^3, 6 %
// masked, 36.2 -> 25.4 / 19.1 -> 15.0).
template <class L, class S>
bool step2_3d_task_lists(const Geom &g, const uint8_t *near, std::vector<int4> &plain,
                         std::vector<int4> &special)
{
    using SH = Step2Shape<L, S>;
    constexpr int ZM = 8;
    if constexpr (!SH::available) {
        return false;
    } else {
        if (g.nx % SH::BX != 0 || g.ny < SH::BY) return false;
        if ((long long)g.nx * g.ny * g.nz < (1LL << 24)) return false;
        const int zc = step2_3d_zc<L, S>(g);
        const int rows = (g.ny + SH::BY - 1) / SH::BY, xb = g.nx / SH::BX;
        auto wrap = [](int v, int n) { return ((v % n) + n) % n; };
        long long chunks = 0, masked = 0;
        std::vector<int4> spec;
        for (int zs = 0; zs < g.nz; zs += zc) {
            const int ze = std::min(zs + zc, g.nz);
            for (int by = 0; by < rows; ++by) {
                const int y0 = by * SH::BY;
                bool nr = false;
                for (int z = zs - 1; z <= ze && !nr; ++z)
                    for (int y = y0 - 1; y <= y0 + SH::BY && !nr; ++y)
                        nr = near[(size_t)wrap(z, g.nz) * g.ny + wrap(y, g.ny)] != 0;
                ++chunks;
                masked += nr;
                for (int bx = 0; bx < xb; ++bx) {
                    if (!nr) {
                        plain.push_back(make_int4(bx * SH::BX, y0, zs, ze));
                    } else {
                        for (int z = zs; z < ze; z += ZM)
                            spec.push_back(make_int4(bx * SH::BX, y0, z, std::min(z + ZM, ze)));
                    }
                }
            }
        }
        if (masked * 20 > chunks) return false;
        special = spec;
        return true;
    }
}

template <class L>
bool launch_step2_lattice(const StepLaunch &a, double *pass_bytes)
{
    if ((a.open && L::D != 2) || !a.row || a.forcing != FORCE_II) return false;
    // the comparison models (TRT-RLB, TRT) run the same passes without
    // solids or open boundaries, for the efficiency comparison where the
    // pass is bound by instruction issue
    if (a.model != MODEL_PTRT &&
        (a.model == MODEL_PTRT_EXACT || a.has_mask || a.open))
        return false;
    if constexpr (L::D == 2) {
        // measured against one step per pass: a gain at every size in FP32
        // and FP64 (64^2 ... 4096^2, 8 - 30 %); none in FP16 / BF16, whose
        // one-step kernel moves half the bytes for the same arithmetic
        if (storage_bytes(a.storage) == 2) return false;
        // with solids: the rows near solids take the masked kernel in a
        // second launch, slower per node than one step per pass, so the
        // pass is used from 2^20 nodes on while they are at most 30 % of
        // the rows (measured, one step -> two, GLUPS: FP32 channel 1024^2
        // 75.4 -> 89.0, 2048^2 81.8 -> 100.7, 4096^2 86.1 -> 102.2, an
        // obstacle over 1/8 of the rows 4096^2 85.8 -> 101.1; FP64 channel
        // 1024^2 41.8 -> 58.3, 4096^2 42.2 -> 64.0; at 512^2 both lost 10 %)
        // with open x (inlet / outlet strips in the special launch), the
        // same floor (measured on the 1050^2 square cylinder, below)
        if (a.has_mask || a.open) {
            if ((long long)a.g.nx * a.g.ny < (1LL << 20)) return false;
            if (!a.tasks_plain || !a.tasks_special || a.n_plain + a.n_special == 0) return false;
            if (a.masked_rows > 0.3 * a.g.ny) return false;
        }
        dispatch_storage(a.storage, false, [&](auto st, auto) -> int {
            using S = typename decltype(st)::type;
            using C = typename Codec<S>::compute;
            using SH = Step2Shape2D<S>;
            if constexpr (sizeof(S) != 2) { // FP16 / BF16: not used (above)
                // strips of BX columns (the last may be partial), chunks of
                // yc rows (the last may be partial), NW single-strip waves per
                // workgroup
                const int yc = step2_2d_rows(a.storage, a.g.nx, a.g.ny);
                constexpr int NW = SH::NW;
                const int strips = (a.g.nx + SH::BX - 1) / SH::BX;
                const int tasks = strips * ((a.g.ny + yc - 1) / yc);
                // the state read once and written once (plus the mask bytes)
                if (pass_bytes)
                    *pass_bytes = (2.0 * L::Q * sizeof(S) + (a.has_mask ? 1.0 : 0.0)) *
                                  a.g.nx * a.g.ny;
                const Coef<L, C> r = make_coef<L, C>(a.tau_plus, a.Lambda, a.force);
                auto go = [&](auto mc, auto oc, const int4 *list, int n, auto modc) {
                    constexpr bool M = decltype(mc)::value, O = decltype(oc)::value;
                    constexpr int MD = decltype(modc)::value;
                    if (n == 0) return;
                    const dim3 grid((n + NW - 1) / NW, 1, 1);
                    if (a.nt)
                        hipLaunchKernelGGL((k_step2_2d<S, true, NW, M, O, MD>), grid,
                                           dim3(SH::W * NW), 0, a.stream, (const S *)a.src,
                                           (S *)a.dst, a.mask, list, a.g, r, yc, strips, n);
                    else
                        hipLaunchKernelGGL((k_step2_2d<S, false, NW, M, O, MD>), grid,
                                           dim3(SH::W * NW), 0, a.stream, (const S *)a.src,
                                           (S *)a.dst, a.mask, list, a.g, r, yc, strips, n);
                };
                using F = std::false_type;
                using T = std::true_type;
                using PT = std::integral_constant<int, MODEL_PTRT>;
                if (a.has_mask || a.open) {
                    go(F{}, F{}, a.tasks_plain, a.n_plain, PT{});
                    if (a.has_mask && a.open)
                        go(T{}, T{}, a.tasks_special, a.n_special, PT{});
                    else if (a.has_mask)
                        go(T{}, F{}, a.tasks_special, a.n_special, PT{});
                    else
                        go(F{}, T{}, a.tasks_special, a.n_special, PT{});
                } else if (a.model == MODEL_TRT_RLB) {
                    go(F{}, F{}, nullptr, tasks, std::integral_constant<int, MODEL_TRT_RLB>{});
                } else if (a.model == MODEL_TRT) {
                    go(F{}, F{}, nullptr, tasks, std::integral_constant<int, MODEL_TRT>{});
                } else {
                    go(F{}, F{}, nullptr, tasks, PT{});
                }
            }
            return PTRT_OK;
        });
        return true;
    } else {
        if (a.has_mask && (!a.tasks_plain || !a.tasks_special)) return false;
        bool launched = false;
        dispatch_storage(a.storage, false, [&](auto st, auto) -> int {
            using S = typename decltype(st)::type;
            using C = typename Codec<S>::compute;
            using SH = Step2Shape<L, S>;
            if constexpr (SH::available) {
                if (a.g.nx % SH::BX != 0 || a.g.ny < SH::BY) return PTRT_OK;
                const int rows = (a.g.ny + SH::BY - 1) / SH::BY;
                const int zc = step2_3d_zc<L, S>(a.g);
                const dim3 grid(a.g.nx / SH::BX, rows, (a.g.nz + zc - 1) / zc);
                const dim3 block(64 * SH::WAVES, 1, 1);
                // the state read once and written once: the first step's
                // halo re-reads are mostly L2 traffic when neighbouring
                // columns run on one XCD (the counters give the HBM reads)
                if (pass_bytes) *pass_bytes = 2.0 * a.g.nx * a.g.ny * a.g.nz * L::Q * sizeof(S);
                const Coef<L, C> r = make_coef<L, C>(a.tau_plus, a.Lambda, a.force);
                // per-task source offsets where the layout allows (FP32)
                const bool zoff = step2_zoff_ok<S>(a.g);
                auto with_zoff = [&](auto f) {
                    if constexpr (sizeof(S) == 4) {
                        if (zoff) {
                            f(std::true_type{});
                            return;
                        }
                    }
                    f(std::false_type{});
                };
                if (a.has_mask) {
                    // the mask-free column chunks, then the masked ones
                    if (pass_bytes) *pass_bytes += (double)a.g.nx * a.g.ny * a.g.nz;
                    auto go = [&](auto mc, auto zc_, const int4 *list, int n) {
                        constexpr bool M = decltype(mc)::value;
                        constexpr bool Z = decltype(zc_)::value && !M;
                        if (n == 0) return;
                        const dim3 lblock(64 * Step2Shape<L, S, M>::WAVES, 1, 1);
                        if (a.nt)
                            hipLaunchKernelGGL((k_step2_list<L, S, true, M, Z>), dim3(n), lblock,
                                               0, a.stream, (const S *)a.src, (S *)a.dst, a.mask,
                                               a.g, r, list, n);
                        else
                            hipLaunchKernelGGL((k_step2_list<L, S, false, M, Z>), dim3(n), lblock,
                                               0, a.stream, (const S *)a.src, (S *)a.dst, a.mask,
                                               a.g, r, list, n);
                    };
                    with_zoff([&](auto zc_) {
                        go(std::false_type{}, zc_, a.tasks_plain, a.n_plain);
                    });
                    go(std::true_type{}, std::false_type{}, a.tasks_special, a.n_special);
                } else {
                    // whole-depth columns that need more than one round of
                    // resident workgroups: one launch per round's worth of
                    // workgroup rows, so that every workgroup of a launch
                    // starts at once and neighbouring columns stay near
                    // the same plane (their shared halo lines then meet in
                    // L2; a second round started as slots free up drifts)
                    const int xb = a.g.nx / SH::BX;
                    int slice = rows;
                    const int resident = step2_3d_resident<L, S>();
                    if (grid.z == 1 && (long long)xb * rows > resident)
                        slice = std::max(1, resident / xb);
                    auto grid_pass = [&](auto modc, auto zc_) {
                        constexpr int MD = decltype(modc)::value;
                        constexpr bool Z = decltype(zc_)::value;
                        for (int by0 = 0; by0 < rows; by0 += slice) {
                            const dim3 gs(grid.x, std::min(slice, rows - by0), grid.z);
                            if (a.nt)
                                hipLaunchKernelGGL((k_step2<L, S, true, MD, Z>), gs, block, 0,
                                                   a.stream, (const S *)a.src, (S *)a.dst, a.g,
                                                   r, zc, by0);
                            else
                                hipLaunchKernelGGL((k_step2<L, S, false, MD, Z>), gs, block, 0,
                                                   a.stream, (const S *)a.src, (S *)a.dst, a.g,
                                                   r, zc, by0);
                        }
                    };
                    with_zoff([&](auto zc_) {
                        if (a.model == MODEL_TRT_RLB)
                            grid_pass(std::integral_constant<int, MODEL_TRT_RLB>{}, zc_);
                        else if (a.model == MODEL_TRT)
                            grid_pass(std::integral_constant<int, MODEL_TRT>{}, zc_);
                        else
                            grid_pass(std::integral_constant<int, MODEL_PTRT>{}, zc_);
                    });
                }
                launched = true;
            }
            return PTRT_OK;
        });
        return launched;
    }
}

// Model and forcing combinations that have kernels: the comparison models
// (TRT-RLB, TRT) use Scheme II without G_i; the forcing variants and the
// open boundaries (D2Q9, not with G_i) need row workgroups.
template <class L>
void launch_step_lattice(const StepLaunch &a)
{
    const dim3 block = a.row ? dim3(a.row_bx, 1, 1) : dim3(64, 4, 1);
    const dim3 grid = a.row ? dim3((a.g.nx + a.row_bx - 1) / a.row_bx, a.g.ny, a.g.nz)
                            : dim3((a.g.nx + 63) / 64, (a.g.ny + 3) / 4, a.g.nz);
    dispatch_storage(a.storage, a.has_mask, [&](auto st, auto mk) -> int {
        using S = typename decltype(st)::type;
        using C = typename Codec<S>::compute;
        constexpr bool M = decltype(mk)::value;
        const Coef<L, C> r = make_coef<L, C>(a.tau_plus, a.Lambda, a.force);
        const S *src = (const S *)a.src;
        S *dst = (S *)a.dst;
        C *phi = (C *)a.phi;
        auto go = [&](auto rowc, auto ntc, auto mc, auto fc, auto oc) {
            constexpr bool RW = decltype(rowc)::value, NT = decltype(ntc)::value;
            constexpr int MD = decltype(mc)::value, FC = decltype(fc)::value;
            constexpr bool OP = decltype(oc)::value;
            if constexpr (FC == FORCE_II_G)
                hipLaunchKernelGGL((k_phi<L, S, M, RW>), grid, block, 0, a.stream, src, a.mask,
                                   a.near, a.g, r, phi);
            hipLaunchKernelGGL((k_step<L, S, M, RW, NT, false, MD, FC, OP>), grid, block, 0,
                               a.stream, src, dst, a.mask, a.near, a.g, r, (double2 *)nullptr,
                               (const C *)phi);
        };
        using P0 = std::integral_constant<int, MODEL_PTRT>;
        using P1 = std::integral_constant<int, MODEL_TRT_RLB>;
        using P2 = std::integral_constant<int, MODEL_TRT>;
        using P3 = std::integral_constant<int, MODEL_PTRT_EXACT>;
        using F0 = std::integral_constant<int, FORCE_II>;
        using F1 = std::integral_constant<int, FORCE_II_G>;
        using F2 = std::integral_constant<int, FORCE_GUO>;
        auto run = [&](auto oc) {
            constexpr bool OP = decltype(oc)::value;
            auto with_nt = [&](auto rowc, auto mc, auto fc) {
                if (a.nt) go(rowc, std::true_type{}, mc, fc, oc);
                else go(rowc, std::false_type{}, mc, fc, oc);
            };
            auto with_forcing = [&](auto mc) {
                if (a.forcing == FORCE_GUO) {
                    with_nt(std::true_type{}, mc, F2{});
                } else if (a.forcing == FORCE_II_G) {
                    if constexpr (!OP) with_nt(std::true_type{}, mc, F1{});
                } else {
                    with_nt(std::true_type{}, mc, F0{});
                }
            };
            if (!a.row) {
                // other models, forcings and boundaries need row workgroups
                if constexpr (!OP) with_nt(std::false_type{}, P0{}, F0{});
            } else if (a.model == MODEL_TRT_RLB) {
                with_nt(std::true_type{}, P1{}, F0{});
            } else if (a.model == MODEL_TRT) {
                with_nt(std::true_type{}, P2{}, F0{});
            } else if (a.model == MODEL_PTRT_EXACT) {
                // the fifth-order modes exist on D3Q27 only; elsewhere it is P-TRT
                if constexpr (L::Q == 27) with_forcing(P3{});
                else with_forcing(P0{});
            } else {
                with_forcing(P0{});
            }
        };
        if constexpr (L::Q == 9) {
            if (a.open) run(std::true_type{});
            else run(std::false_type{});
        } else {
            run(std::false_type{});
        }
        return PTRT_OK;
    });
}

} // namespace ptrt
