// Host-side helpers shared by the single-lattice and batched entry points:
// type dispatch over (lattice, storage, mask) and launch geometry.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "ptrt.h"

namespace ptrt {

template <class T>
struct Tag {
    using type = T;
};

// Call f(Tag<S>, bool_constant<MASK>) for the runtime storage and mask.
template <class F>
inline int dispatch_storage(int storage, bool mask, F &&f)
{
    auto with_mask = [&](auto st) -> int {
        if (mask) return f(st, std::true_type{});
        return f(st, std::false_type{});
    };
    switch (storage) {
    case PTRT_F64: return with_mask(Tag<double>{});
    case PTRT_F32: return with_mask(Tag<float>{});
    case PTRT_F16: return with_mask(Tag<_Float16>{});
    case PTRT_BF16: return with_mask(Tag<bf16_t>{});
    case PTRT_F16_SR: return with_mask(Tag<f16sr_t>{});
    case PTRT_BF16_SR: return with_mask(Tag<bf16sr_t>{});
    default: return PTRT_EINVAL;
    }
}

// Call f(Tag<L>, Tag<S>, bool_constant<MASK>) for the runtime choice.
template <class F>
inline int dispatch(int lattice, int storage, bool mask, F &&f)
{
    auto with_lat = [&](auto lt) -> int {
        auto with_mask = [&](auto st) -> int {
            if (mask) return f(lt, st, std::true_type{});
            return f(lt, st, std::false_type{});
        };
        switch (storage) {
        case PTRT_F64: return with_mask(Tag<double>{});
        case PTRT_F32: return with_mask(Tag<float>{});
        case PTRT_F16: return with_mask(Tag<_Float16>{});
        case PTRT_BF16: return with_mask(Tag<bf16_t>{});
        case PTRT_F16_SR: return with_mask(Tag<f16sr_t>{});
        case PTRT_BF16_SR: return with_mask(Tag<bf16sr_t>{});
        default: return PTRT_EINVAL;
        }
    };
    if (lattice == PTRT_D2Q9) return with_lat(Tag<D2Q9>{});
    if (lattice == PTRT_D3Q19) return with_lat(Tag<D3Q19>{});
    if (lattice == PTRT_D3Q27) return with_lat(Tag<D3Q27>{});
    return PTRT_EINVAL;
}

inline size_t storage_bytes(int storage)
{
    switch (storage) {
    case PTRT_F64: return 8;
    case PTRT_F32: return 4;
    case PTRT_F16:
    case PTRT_BF16:
    case PTRT_F16_SR:
    case PTRT_BF16_SR: return 2;
    default: return 0;
    }
}

inline int lattice_q(int lattice)
{
    return lattice == PTRT_D2Q9 ? 9 : (lattice == PTRT_D3Q19 ? 19 : (lattice == PTRT_D3Q27 ? 27 : 0));
}

inline bool finite(double v) { return std::isfinite(v); }

// Checks shared by ptrt_create and the batch descriptors; returns a status
// and fills msg on failure.
inline int check_params(int lattice, int nx, int ny, int nz, double tau_plus, double Lambda,
                        const double *force, std::string &msg)
{
    if (lattice != PTRT_D2Q9 && lattice != PTRT_D3Q19 && lattice != PTRT_D3Q27) {
        msg = "unknown lattice id " + std::to_string(lattice);
        return PTRT_EINVAL;
    }
    if (nx <= 0 || ny <= 0 || nz <= 0) {
        msg = "lattice sizes must be positive";
        return PTRT_EINVAL;
    }
    if (lattice == PTRT_D2Q9 && nz != 1) {
        msg = "D2Q9 needs nz == 1";
        return PTRT_EINVAL;
    }
    if ((double)nx * ny * nz >= 2147483648.0) {
        msg = "lattice has 2^31 nodes or more";
        return PTRT_EINVAL;
    }
    if (ny > 262140 || nz > 65535) {
        msg = "ny must be <= 262140 and nz <= 65535 (launch grid limits)";
        return PTRT_EINVAL;
    }
    if (!finite(tau_plus) || !finite(Lambda) || !(tau_plus > 0.5) || !(Lambda > 0.0)) {
        msg = "need finite tau_plus > 1/2 and Lambda > 0";
        return PTRT_ETAU;
    }
    if (force)
        for (int a = 0; a < 3; ++a)
            if (!finite(force[a])) {
                msg = "force must be finite";
                return PTRT_ETAU;
            }
    return PTRT_OK;
}

// Rows (row = z * ny + y) that hold a solid node or pull from one: a row is
// marked when any row within one step in y and z (periodic) has a solid.
inline std::vector<uint8_t> near_solid_rows(const uint8_t *mask, int nx, int ny, int nz)
{
    const long long rows = (long long)ny * nz;
    std::vector<uint8_t> solid_row(rows, 0), near(rows, 0);
    for (long long r = 0; r < rows; ++r)
        for (int x = 0; x < nx; ++x)
            if (mask[r * nx + x]) {
                solid_row[r] = 1;
                break;
            }
    const int dz_lo = nz > 1 ? -1 : 0, dz_hi = nz > 1 ? 1 : 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            uint8_t f = 0;
            for (int dz = dz_lo; dz <= dz_hi && !f; ++dz)
                for (int dy = -1; dy <= 1 && !f; ++dy) {
                    const int zz = (z + dz + nz) % nz, yy = (y + dy + ny) % ny;
                    f = solid_row[(long long)zz * ny + yy];
                }
            near[(long long)z * ny + y] = f;
        }
    return near;
}

// Tiled layout of a lattice (see kernels.hpp): rows padded to a pitch of a
// whole number of 128-byte lines (a wave's row segment then starts on a
// line boundary, so no line is written partly by two waves), rows per tile
// chosen so one direction chunk of a tile is about 8 KB.  Returns the
// element count of a population buffer and fills g.
inline long long make_layout(int Q, int nx, int ny, int nz, size_t elem, Geom &g)
{
    const long long line = (long long)(128 / elem);
    const int pitch = (int)(((long long)nx + line - 1) / line * line);
    int lr = 0;
    while (((long long)pitch << (lr + 1)) * (long long)elem <= 8192) ++lr;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.pitch = pitch;
    g.lr = lr;
    g.plane = (long long)pitch << lr;
    g.tile = (long long)Q * g.plane;
    const long long rows = (long long)ny * nz;
    const long long ntiles = (rows + (1LL << lr) - 1) >> lr;
    return ntiles * g.tile;
}

// The kernels form two parts of every population address in 32 bits: the
// offset inside a tile (direction chunk plus row inside the tile, below
// Q * plane elements) and the x part in bytes (below pitch * elem).  A
// layout where either can reach 2^32 would wrap, so it is rejected here,
// before anything is allocated or launched.
inline int check_layout(int Q, int nx, int ny, int nz, size_t elem, std::string &msg)
{
    Geom g{};
    make_layout(Q, nx, ny, nz, elem, g);
    const double lim = 4294967296.0;
    if ((double)g.tile >= lim) {
        msg = "rows too long: a tile of " + std::to_string(Q) + " directions x " +
              std::to_string(g.plane) + " elements reaches 2^32 elements (32-bit offsets)";
        return PTRT_EINVAL;
    }
    if ((double)g.pitch * (double)elem >= lim) {
        msg = "rows too long: " + std::to_string(g.pitch) + " elements of " + std::to_string(elem) +
              " bytes reach 2^32 bytes (32-bit offsets)";
        return PTRT_EINVAL;
    }
    return PTRT_OK;
}


} // namespace ptrt
