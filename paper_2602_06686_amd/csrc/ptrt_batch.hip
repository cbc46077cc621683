// Batched form of libptrt (declared in include/ptrt.h): many independent
// D2Q9 lattices of different sizes advanced by one launch per step.
//
// Device layout: every instance owns a tiled population block (the layout of
// kernels.hpp, with its own rows per tile) at element offset off_k of each
// of the two population buffers, and nx_k * ny_k mask
// bytes at offset moff_k of one shared mask array (zeros for instances
// without solids).  A tile table lists (instance, x0, y0) for every
// tile_x * tile_y tile of every instance; workgroup b handles tiles
// b, b + G, b + 2G, ... of the table (G = grid size).  Each node runs the
// same pull() and collide() as the single-lattice kernel, so an instance
// evolves bit for bit like a single lattice with the same parameters.
// Two steps per pass (FP32 / FP64): a task table lists (instance, strip,
// chunk of rows) for the single-lattice two-step pass (step2.hpp); one wave
// runs one task on its instance's block of the state, mask and constants.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "step_launch.hpp"

using namespace ptrt;

namespace {

template <class C>
struct BInst {
    long long off, moff, noff; // populations, mask and near-solid row flags
    Geom g;
    Coef<D2Q9, C> r;
};

// Tile table entries are int4 {instance, x0, y0, (nrows << 16) | wpr}.
// ONEROW (blockDim.y == 1, blockDim.x a multiple of 64): wave w of the
// workgroup takes row y0 + w / wpr, columns x0 + (w % wpr) * 64 + lane, for
// w / wpr < nrows.  wpr is either the workgroup's waves (a segment of one
// long row) or the instance's row width in waves (several whole short rows
// per workgroup).  Every wave stays inside one row, so the row is
// wave-uniform and the addressing runs on the scalar unit.  Otherwise
// (2D workgroups) thread (tx, ty) takes node (x0 + tx, y0 + ty).
// Rows not flagged as near a solid take the mask-free code.
template <class S, bool ONEROW>
__global__ void __launch_bounds__(1024)
k_batch_step(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask,
             const uint8_t *__restrict__ near,
             const BInst<typename Codec<S>::compute> *__restrict__ inst,
             const int4 *__restrict__ tiles, int ntiles)
{
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BInst<typename Codec<S>::compute> p = inst[tl.x];
        int x, y;
        if constexpr (ONEROW) {
            const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
            const int wpr = tl.w & 0xffff, nrows = tl.w >> 16;
            const int r = w / wpr;
            if (r >= nrows) continue;
            y = tl.z + r;
            x = tl.y + (w - r * wpr) * 64 + (int)(threadIdx.x & 63);
        } else {
            x = tl.y + threadIdx.x;
            y = tl.z + threadIdx.y;
            if (y >= p.g.ny) continue;
        }
        const bool inside = x < p.g.nx;
        const uint8_t *m = mask + p.moff;
        const S *s = src + p.off;
        S *d = dst + p.off;
        double dm, dk;
        if (near[p.noff + y]) {
            if (inside && !m[(unsigned)y * (unsigned)p.g.nx + (unsigned)x])
                node_update<D2Q9, S, true, true>(s, d, m, p.g, p.r, x, y, 0, (unsigned)y, dm, dk);
        } else if (inside) {
            node_update<D2Q9, S, false, true>(s, d, m, p.g, p.r, x, y, 0, (unsigned)y, dm, dk);
        }
    }
}

// Two steps per pass: wave task t is tasks[t] = {instance, x0, ys, ye}, a
// strip of columns x0 ... x0 + BX - 1 and rows ys ... ye - 1 of the
// instance; MASK as in step2_2d_task (tasks with no solid within one row of
// rows ys - 1 ... ye run with MASK = false).  Wave w of workgroup g takes
// tasks g NW + w, g NW + w + G NW, ... (G workgroups): one task per wave
// when G NW covers the table, else a persistent grid.
template <class S, bool NT, int NW, bool MASK>
__global__ void __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(8, 8)))
k_batch_step2(const S *__restrict__ src, S *__restrict__ dst, const uint8_t *__restrict__ mask,
              const BInst<typename Codec<S>::compute> *__restrict__ inst,
              const int4 *__restrict__ tasks, int ntasks)
{
    using SH = Step2Shape2D<S, MASK>;
    __shared__ S lds_all[NW * SH::K::planes * SH::W];
    int wg, unused_y, unused_z;
    xcd_block(wg, unused_y, unused_z);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int stride = (int)gridDim.x * NW;
    for (int t = wg * NW + w; t < ntasks; t += stride) {
        const int4 tk = tasks[t];
        const BInst<typename Codec<S>::compute> p = inst[tk.x];
        step2_2d_task<S, NT, MASK>(src + p.off, dst + p.off, mask + p.moff, p.g, p.r,
                                   lds_all + w * (SH::K::planes * SH::W), tk.y, tk.z, tk.w);
    }
}

thread_local std::string g_batch_create_error = "no error";
// steps per captured graph; the buffer parity change of a replay is
// recorded at capture (odd with two-step passes)
constexpr int GRAPH_STEPS = 10;
constexpr int BLK_X = 64, BLK_Y = 4;

struct HostInst {
    int nx, ny;
    double tau_plus, Lambda, force[3];
    bool has_mask;
    long long off, moff, noff, N, elems;
    Geom g;
};

} // namespace

struct ptrt_batch {
    int count = 0, storage = PTRT_F32;
    std::vector<HostInst> inst;
    long long total_elems = 0, total_nodes = 0, mask_bytes = 0;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t *d_mask = nullptr, *d_near = nullptr;
    void *d_inst = nullptr;
    int4 *d_tiles = nullptr;
    int ntiles = 0;
    int tile_x = 64, tile_y = 4, blocks = 0, xcd_order = 0;
    double2 *d_partials = nullptr;
    int max_parts = 0;
    double *d_red = nullptr;
    hipStream_t stream = nullptr, capture_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_flip[2] = {0, 0}; // buffer parity change of a replay
    // two steps per pass: steps per pass asked for; the plan (rows per
    // chunk of the tasks without solids near, rows per chunk of the masked
    // ones, waves per workgroup, workgroups (0 = one wave per task), the
    // masked launch on a second stream); the task table (tasks without
    // solids near, then the others); stores
    int spp = 2, yc2 = 0, ym2 = 0, nw2 = 4, blocks2 = 0, conc2 = 0;
    std::vector<uint8_t> h_near;
    int4 *d_tasks2 = nullptr;
    int n_plain2 = 0, n_masked2 = 0;
    hipStream_t side_stream = nullptr;
    hipEvent_t fork_event = nullptr, join_event = nullptr;
    bool nt = false;
    int last_steps = 0;
    std::string err = "no error";
};

namespace {

int bfail(ptrt_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

// A failed HIP call (see fail_hip of the single-lattice handle): its error
// is also taken off the thread's last-error slot.
int bfail_hip(ptrt_batch *b, int code, const std::string &msg)
{
    (void)hipGetLastError();
    return bfail(b, code, msg);
}

#define BHIPCHK(b, expr)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return bfail_hip((b), PTRT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void drop_graphs(ptrt_batch *b)
{
    for (auto &g : b->graph)
        if (g) {
            hipGraphExecDestroy(g);
            g = nullptr;
        }
}

bool valid_plan(int tx, int ty)
{
    const int n = tx * ty;
    return tx >= 32 && ty >= 1 && tx % 32 == 0 && (ty > 1 || tx % 64 == 0) &&
           (n == 64 || n == 128 || n == 256 || n == 512 || n == 1024);
}

// A task or tile table in a new device allocation (*out; nothing is
// allocated on failure), so that the table in use is replaced only once
// its successor is complete.
int upload_table(ptrt_batch *b, const std::vector<int4> &table, int4 **out)
{
    *out = nullptr;
    int4 *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(int4) * std::max<size_t>(1, table.size()));
    if (e != hipSuccess) return bfail_hip(b, PTRT_ENOMEM, std::string("hipMalloc of a task table: ") + hipGetErrorString(e));
    if (!table.empty()) e = hipMemcpy(d, table.data(), sizeof(int4) * table.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return bfail_hip(b, PTRT_EDEVICE, std::string("task table upload: ") + hipGetErrorString(e));
    }
    *out = d;
    return PTRT_OK;
}

int build_tiles(ptrt_batch *b)
{
    std::vector<int4> spatial;
    for (int k = 0; k < b->count; ++k) {
        const HostInst &h = b->inst[k];
        if (b->tile_y > 1) {
            for (int y0 = 0; y0 < h.ny; y0 += b->tile_y)
                for (int x0 = 0; x0 < h.nx; x0 += b->tile_x) spatial.push_back(make_int4(k, x0, y0, 0));
            continue;
        }
        const int waves = b->tile_x / 64, row_waves = (h.nx + 63) / 64;
        if (row_waves >= waves) {
            // segments of tile_x nodes of one row
            for (int y = 0; y < h.ny; ++y)
                for (int x0 = 0; x0 < h.nx; x0 += b->tile_x)
                    spatial.push_back(make_int4(k, x0, y, (1 << 16) | waves));
        } else {
            // several whole rows per workgroup
            const int rows = waves / row_waves;
            for (int y0 = 0; y0 < h.ny; y0 += rows)
                spatial.push_back(make_int4(k, 0, y0, (std::min(rows, h.ny - y0) << 16) | row_waves));
        }
    }
    const int n = (int)spatial.size();
    std::vector<int4> table(n);
    if (b->xcd_order) {
        // table[8m + j] = spatial[j * chunk + m]: with round-robin dispatch of
        // workgroups over the 8 XCDs, die j walks the j-th contiguous chunk.
        const int chunk = (n + 7) / 8;
        std::vector<int4> out;
        out.reserve(n);
        for (int m = 0; m < chunk; ++m)
            for (int j = 0; j < 8; ++j) {
                const long long src = (long long)j * chunk + m;
                if (src < n) out.push_back(spatial[src]);
            }
        table = out;
    } else {
        table = spatial;
    }
    int4 *fresh = nullptr;
    const int rc = upload_table(b, table, &fresh);
    if (rc != PTRT_OK) return rc; // the previous table stays in use
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_tiles = fresh;
    b->ntiles = n;
    drop_graphs(b);
    return PTRT_OK;
}

template <class S>
void launch_fused(ptrt_batch *b, hipStream_t s)
{
    using C = typename Codec<S>::compute;
    const int grid = b->blocks > 0 ? std::min(b->blocks, b->ntiles) : b->ntiles;
    if (b->tile_y == 1)
        hipLaunchKernelGGL((k_batch_step<S, true>), dim3(grid), dim3(b->tile_x, 1, 1), 0, s,
                           (const S *)b->buf[b->cur], (S *)b->buf[b->cur ^ 1], b->d_mask, b->d_near,
                           (const BInst<C> *)b->d_inst, b->d_tiles, b->ntiles);
    else
        hipLaunchKernelGGL((k_batch_step<S, false>), dim3(grid), dim3(b->tile_x, b->tile_y, 1), 0, s,
                           (const S *)b->buf[b->cur], (S *)b->buf[b->cur ^ 1], b->d_mask, b->d_near,
                           (const BInst<C> *)b->d_inst, b->d_tiles, b->ntiles);
    b->cur ^= 1;
}

int launch_fused_any(ptrt_batch *b, hipStream_t s)
{
    b->last_steps = 1;
    return dispatch(PTRT_D2Q9, b->storage, false, [&](auto, auto st, auto) -> int {
        using S = typename decltype(st)::type;
        launch_fused<S>(b, s);
        return PTRT_OK;
    });
}

bool two_step(const ptrt_batch *b) { return b->spp == 2 && b->d_tasks2 != nullptr; }

// One pass of two steps: the tasks without solids near and the others, in
// two launches, one after the other on s, or (conc2) the masked ones on a
// second stream forked from s and joined back (in a captured graph: two
// branches), so that they overlap with the rest.  The two launches read the
// same state and write disjoint nodes.
void launch_pass2_any(ptrt_batch *b, hipStream_t s)
{
    b->last_steps = 2;
    dispatch(PTRT_D2Q9, b->storage, false, [&](auto, auto st, auto) -> int {
        using S = typename decltype(st)::type;
        using C = typename Codec<S>::compute;
        if constexpr (sizeof(S) != 2) { // FP16 / BF16: no task table
            auto go = [&](auto mc, const int4 *list, int n, hipStream_t q) {
                constexpr bool M = decltype(mc)::value;
                if (n == 0) return;
                const S *src = (const S *)b->buf[b->cur];
                S *dst = (S *)b->buf[b->cur ^ 1];
                auto launch = [&](auto nwc) {
                    constexpr int NW = decltype(nwc)::value;
                    int grid = (n + NW - 1) / NW;
                    if (b->blocks2 > 0) grid = std::min(grid, b->blocks2);
                    if (b->nt)
                        hipLaunchKernelGGL((k_batch_step2<S, true, NW, M>), dim3(grid),
                                           dim3(64 * NW), 0, q, src, dst, b->d_mask,
                                           (const BInst<C> *)b->d_inst, list, n);
                    else
                        hipLaunchKernelGGL((k_batch_step2<S, false, NW, M>), dim3(grid),
                                           dim3(64 * NW), 0, q, src, dst, b->d_mask,
                                           (const BInst<C> *)b->d_inst, list, n);
                };
                if (b->nw2 == 2) launch(std::integral_constant<int, 2>{});
                else if (b->nw2 == 8) launch(std::integral_constant<int, 8>{});
                else launch(std::integral_constant<int, 4>{});
            };
            const int4 *plain = b->d_tasks2, *masked = b->d_tasks2 + b->n_plain2;
            if (b->conc2 && b->n_plain2 > 0 && b->n_masked2 > 0) {
                (void)hipEventRecord(b->fork_event, s);
                (void)hipStreamWaitEvent(b->side_stream, b->fork_event, 0);
                go(std::true_type{}, masked, b->n_masked2, b->side_stream);
                go(std::false_type{}, plain, b->n_plain2, s);
                (void)hipEventRecord(b->join_event, b->side_stream);
                (void)hipStreamWaitEvent(s, b->join_event, 0);
            } else {
                go(std::false_type{}, plain, b->n_plain2, s);
                go(std::true_type{}, masked, b->n_masked2, s);
            }
        }
        return PTRT_OK;
    });
    b->cur ^= 1;
}

// n steps on stream s: two-step passes while two steps remain (where
// allowed), the rest one launch per step.
void advance(ptrt_batch *b, hipStream_t s, int n)
{
    if (two_step(b))
        for (; n >= 2; n -= 2) launch_pass2_any(b, s);
    for (; n > 0; --n) launch_fused_any(b, s);
}

// Rows per chunk of the two-step tasks by default: the single-lattice rule,
// at most 3 rows (on the 512-lattice benchmark batch, 38M nodes, 3 rows
// measured best with the masked chunks as long as the others, FP32 and
// FP64, with or without solids: FP32 GLUPS for 1, 2, 3, 4, 5, 7, 9, 12
// rows: 92.5, 85.9, 95.0, 92.5, 93.1, 90.1, 86.4, 83.3; one step per pass
// 81.1).  ptrt_batch_autotune searches the plan around it.
int default_rows2(const ptrt_batch *b)
{
    constexpr int BX = Step2Shape2D<float>::BX;
    long long strip_rows = 0;
    for (const HostInst &h : b->inst) strip_rows += (long long)((h.nx + BX - 1) / BX) * h.ny;
    return std::min(3, step2_2d_rows_for(b->storage, strip_rows, b->total_nodes));
}

// The two-step task table (FP32 / FP64): per instance, strips of BX
// columns (the last may be partial) times chunks of yc2 rows (the last may
// be partial); a chunk with a solid within one row of its rows ys - 1 ...
// ye (near, per instance at noff) takes the masked code, its rows split
// into chunks of ym2 rows.
int build_tasks2(ptrt_batch *b)
{
    if (b->storage != PTRT_F32 && b->storage != PTRT_F64) return PTRT_OK;
    constexpr int BX = Step2Shape2D<float>::BX;
    if (b->yc2 <= 0) b->yc2 = default_rows2(b);
    if (b->ym2 <= 0) b->ym2 = b->yc2;
    std::vector<int4> plain, masked;
    for (int k = 0; k < b->count; ++k) {
        const HostInst &h = b->inst[k];
        const int strips = (h.nx + BX - 1) / BX;
        for (int ys = 0; ys < h.ny; ys += b->yc2) {
            const int ye = std::min(ys + b->yc2, h.ny);
            bool nr = false;
            for (int y = ys - 1; y <= ye && !nr; ++y)
                nr = b->h_near[(size_t)(h.noff + ((y % h.ny) + h.ny) % h.ny)] != 0;
            if (!nr) {
                for (int bx = 0; bx < strips; ++bx) plain.push_back(make_int4(k, bx * BX, ys, ye));
            } else {
                for (int y = ys; y < ye; y += b->ym2)
                    for (int bx = 0; bx < strips; ++bx)
                        masked.push_back(make_int4(k, bx * BX, y, std::min(y + b->ym2, ye)));
            }
        }
    }
    const int n_plain = (int)plain.size(), n_masked = (int)masked.size();
    plain.insert(plain.end(), masked.begin(), masked.end());
    int4 *fresh = nullptr;
    const int rc = upload_table(b, plain, &fresh);
    if (rc != PTRT_OK) return rc; // the previous table stays in use
    if (b->d_tasks2) (void)hipFree(b->d_tasks2);
    b->d_tasks2 = fresh;
    b->n_plain2 = n_plain;
    b->n_masked2 = n_masked;
    // non-temporal stores once the two state buffers exceed the 256 MB
    // last-level cache (as for a single lattice)
    b->nt = 2.0 * (double)b->total_elems * (double)storage_bytes(b->storage) > 256.0 * 1024 * 1024;
    drop_graphs(b);
    return PTRT_OK;
}

int capture_graph(ptrt_batch *b, int parity)
{
    const int saved = b->cur;
    b->cur = parity;
    hipGraph_t g = nullptr;
    BHIPCHK(b, hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
    advance(b, b->capture_stream, GRAPH_STEPS);
    hipError_t e = hipStreamEndCapture(b->capture_stream, &g);
    b->graph_flip[parity] = b->cur ^ parity;
    b->cur = saved;
    if (e != hipSuccess) return bfail_hip(b, PTRT_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph[parity], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph[parity] = nullptr;
        return bfail_hip(b, PTRT_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return PTRT_OK;
}

Geom inst_geom(const HostInst &h) { return h.g; }

int check_instance(ptrt_batch *b, int k)
{
    if (!b) return PTRT_EINVAL;
    if (k < 0 || k >= b->count) return bfail(b, PTRT_EINVAL, "instance index out of range");
    return PTRT_OK;
}

// Workgroups of the two-step kernel (mask-free variant) that the device
// holds at once with nw waves each: the persistent grid of a plan.
int resident_blocks2(const ptrt_batch *b, int nw)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus <= 0) return 0;
    dispatch(PTRT_D2Q9, b->storage, false, [&](auto, auto st, auto) -> int {
        using S = typename decltype(st)::type;
        if constexpr (sizeof(S) != 2) {
            auto q = [&](auto nwc) {
                constexpr int NW = decltype(nwc)::value;
                (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, reinterpret_cast<const void *>(&k_batch_step2<S, true, NW, false>),
                    64 * NW, 0);
            };
            if (nw == 2) q(std::integral_constant<int, 2>{});
            else if (nw == 8) q(std::integral_constant<int, 8>{});
            else q(std::integral_constant<int, 4>{});
        }
        return PTRT_OK;
    });
    return per_cu > 0 ? per_cu * cus : 0;
}

// Device time of `passes` two-step passes after two untimed ones (ms).
float time_passes2(ptrt_batch *b, hipEvent_t e0, hipEvent_t e1, int passes)
{
    for (int k = 0; k < 2; ++k) launch_pass2_any(b, b->stream);
    (void)hipEventRecord(e0, b->stream);
    for (int k = 0; k < passes; ++k) launch_pass2_any(b, b->stream);
    (void)hipEventRecord(e1, b->stream);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0f;
    float ms = -1.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
    return ms;
}

// Search the two-step plan on the current state (the caller saves and
// restores it): every combination of rows {1, 2, 3, 5, 7}, masked rows
// {1, 2, 3, rows}, waves {2, 4, 8}, one wave per task or the resident grid,
// masked launch after or beside the others; each timed over 10 passes, the
// five fastest timed again three times and the best median kept.
int autotune2(ptrt_batch *b, hipEvent_t e0, hipEvent_t e1)
{
    struct Plan {
        int yc, ym, nw, blocks, conc;
        float ms;
    };
    std::vector<Plan> tried;
    static const int rows[] = {1, 2, 3, 5, 7};
    static const int nws[] = {2, 4, 8};
    for (int yc : rows) {
        std::vector<int> yms = {1, 2, 3};
        if (yc > 3) yms.push_back(yc);
        for (int ym : yms) {
            b->yc2 = yc;
            b->ym2 = ym;
            int rc = build_tasks2(b);
            if (rc != PTRT_OK) return rc;
            for (int nw : nws)
                for (int pers = 0; pers < 2; ++pers)
                    for (int conc = 0; conc < 2; ++conc) {
                        if (conc && b->n_masked2 == 0) continue;
                        b->nw2 = nw;
                        b->blocks2 = pers ? resident_blocks2(b, nw) : 0;
                        if (pers && b->blocks2 == 0) continue;
                        b->conc2 = conc;
                        const float ms = time_passes2(b, e0, e1, 10);
                        if (ms < 0) return bfail_hip(b, PTRT_EDEVICE, "two-step autotune timing failed");
                        tried.push_back({yc, ym, nw, b->blocks2, conc, ms});
                    }
        }
    }
    if (tried.empty()) return PTRT_OK;
    std::sort(tried.begin(), tried.end(), [](const Plan &x, const Plan &y) { return x.ms < y.ms; });
    const size_t top = std::min<size_t>(5, tried.size());
    Plan best = tried[0];
    float best_med = 1e30f;
    for (size_t i = 0; i < top; ++i) {
        const Plan &pl = tried[i];
        b->yc2 = pl.yc;
        b->ym2 = pl.ym;
        int rc = build_tasks2(b);
        if (rc != PTRT_OK) return rc;
        b->nw2 = pl.nw;
        b->blocks2 = pl.blocks;
        b->conc2 = pl.conc;
        float t[3];
        for (float &x : t) {
            x = time_passes2(b, e0, e1, 10);
            if (x < 0) return bfail_hip(b, PTRT_EDEVICE, "two-step autotune timing failed");
        }
        std::sort(t, t + 3);
        if (t[1] < best_med) {
            best_med = t[1];
            best = pl;
        }
    }
    b->yc2 = best.yc;
    b->ym2 = best.ym;
    b->nw2 = best.nw;
    b->blocks2 = best.blocks;
    b->conc2 = best.conc;
    return build_tasks2(b);
}

} // namespace

extern "C" {

int ptrt_batch_create(int count, const ptrt_instance_desc *desc, int storage, ptrt_batch **out)
{
    if (!out || !desc || count <= 0) {
        g_batch_create_error = "need count > 0 and non-NULL desc / out";
        return PTRT_EINVAL;
    }
    *out = nullptr;
    if (storage_bytes(storage) == 0) {
        g_batch_create_error = "unknown storage type";
        return PTRT_EINVAL;
    }
    ptrt_batch *b = new (std::nothrow) ptrt_batch();
    if (!b) return PTRT_ENOMEM;
    b->count = count;
    b->storage = storage;
    b->inst.resize(count);
    const size_t elem = storage_bytes(storage);
    std::vector<uint8_t> mask, near;
    long long off = 0, moff = 0, noff = 0;
    for (int k = 0; k < count; ++k) {
        const ptrt_instance_desc &d = desc[k];
        std::string msg;
        int rc = check_params(PTRT_D2Q9, d.nx, d.ny, 1, d.tau_plus, d.Lambda, d.force, msg);
        if (rc == PTRT_OK) rc = check_layout(9, d.nx, d.ny, 1, elem, msg);
        if (rc != PTRT_OK) {
            g_batch_create_error = "instance " + std::to_string(k) + ": " + msg;
            delete b;
            return rc;
        }
        HostInst &h = b->inst[k];
        h.nx = d.nx;
        h.ny = d.ny;
        h.N = (long long)d.nx * d.ny;
        h.tau_plus = d.tau_plus;
        h.Lambda = d.Lambda;
        for (int a = 0; a < 3; ++a) h.force[a] = d.force ? d.force[a] : 0.0;
        h.force[2] = 0.0;
        h.has_mask = false;
        mask.resize((size_t)(moff + h.N), 0);
        if (d.solid_mask)
            for (long long n = 0; n < h.N; ++n)
                if (d.solid_mask[n]) {
                    mask[(size_t)(moff + n)] = 1;
                    h.has_mask = true;
                }
        // every instance in the tiled layout, starting on a 256-byte boundary
        h.elems = make_layout(9, h.nx, h.ny, 1, elem, h.g);
        const long long align = 256 / (long long)elem;
        h.off = off;
        h.moff = moff;
        h.noff = noff;
        off += ((h.elems + align - 1) / align) * align;
        moff += h.N;
        const std::vector<uint8_t> nr = near_solid_rows(mask.data() + h.moff, h.nx, h.ny, 1);
        near.insert(near.end(), nr.begin(), nr.end());
        noff += h.ny;
        b->total_nodes += h.N;
    }
    b->total_elems = off;
    b->mask_bytes = moff;

    auto cleanup = [&](int code, const std::string &msg) {
        (void)hipGetLastError(); // reported here (see bfail_hip)
        g_batch_create_error = msg;
        ptrt_batch_destroy(b);
        return code;
    };
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMalloc(&b->buf[k], (size_t)b->total_elems * elem);
        if (e != hipSuccess) {
            b->buf[k] = nullptr;
            return cleanup(PTRT_ENOMEM, std::string("hipMalloc of populations: ") + hipGetErrorString(e));
        }
        if (hipMemset(b->buf[k], 0, (size_t)b->total_elems * elem) != hipSuccess)
            return cleanup(PTRT_EDEVICE, "hipMemset failed");
    }
    if (hipMalloc(&b->d_mask, (size_t)moff) != hipSuccess ||
        hipMemcpy(b->d_mask, mask.data(), (size_t)moff, hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&b->d_near, (size_t)noff) != hipSuccess ||
        hipMemcpy(b->d_near, near.data(), (size_t)noff, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(PTRT_EDEVICE, "mask upload failed");
    // instance table in the compute type of the storage
    int rc = dispatch(PTRT_D2Q9, storage, false, [&](auto, auto st, auto) -> int {
        using S = typename decltype(st)::type;
        using C = typename Codec<S>::compute;
        std::vector<BInst<C>> t(count);
        for (int k = 0; k < count; ++k) {
            const HostInst &h = b->inst[k];
            t[k] = BInst<C>{h.off, h.moff, h.noff, h.g,
                            make_coef<D2Q9, C>(h.tau_plus, h.Lambda, h.force)};
        }
        if (hipMalloc(&b->d_inst, sizeof(BInst<C>) * count) != hipSuccess) return PTRT_EDEVICE;
        if (hipMemcpy(b->d_inst, t.data(), sizeof(BInst<C>) * count, hipMemcpyHostToDevice) != hipSuccess)
            return PTRT_EDEVICE;
        return PTRT_OK;
    });
    if (rc != PTRT_OK) return cleanup(rc, "instance table upload failed");
    for (const auto &h : b->inst)
        b->max_parts = std::max(b->max_parts, ((h.nx + BLK_X - 1) / BLK_X) * ((h.ny + BLK_Y - 1) / BLK_Y));
    if (hipMalloc(&b->d_partials, sizeof(double2) * (size_t)b->max_parts) != hipSuccess ||
        hipMalloc(&b->d_red, 2 * sizeof(double) * (size_t)count) != hipSuccess)
        return cleanup(PTRT_ENOMEM, "reduction buffers");
    if (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess)
        return cleanup(PTRT_EDEVICE, "capture stream");
    if (build_tiles(b) != PTRT_OK) return cleanup(PTRT_EDEVICE, b->err);
    if (hipStreamCreateWithFlags(&b->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork_event, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join_event, hipEventDisableTiming) != hipSuccess)
        return cleanup(PTRT_EDEVICE, "side stream / events");
    b->h_near = std::move(near);
    if (build_tasks2(b) != PTRT_OK) return cleanup(PTRT_EDEVICE, b->err);
    for (int k = 0; k < count; ++k) {
        rc = ptrt_batch_init_equilibrium(b, k, nullptr, nullptr);
        if (rc != PTRT_OK) return cleanup(rc, b->err);
    }
    *out = b;
    return PTRT_OK;
}

int ptrt_batch_set_stream(ptrt_batch *b, void *s)
{
    if (!b) return PTRT_EINVAL;
    b->stream = (hipStream_t)s;
    return PTRT_OK;
}

int ptrt_batch_init_equilibrium(ptrt_batch *b, int k, const double *rho, const double *u)
{
    int rc = check_instance(b, k);
    if (rc != PTRT_OK) return rc;
    const HostInst &h = b->inst[k];
    double *d_in = nullptr;
    BHIPCHK(b, hipMalloc(&d_in, sizeof(double) * 3 * (size_t)h.N));
    hipError_t e = hipSuccess;
    if (rho) e = hipMemcpyAsync(d_in, rho, sizeof(double) * h.N, hipMemcpyHostToDevice, b->stream);
    if (u && e == hipSuccess)
        e = hipMemcpyAsync(d_in + h.N, u, sizeof(double) * 2 * h.N, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) {
        // both buffers hold the same state so that either parity is valid
        const Geom g = inst_geom(h);
        for (int k2 = 0; k2 < 2; ++k2) {
            void *dst = b->buf[b->cur ^ k2];
            dispatch(PTRT_D2Q9, b->storage, h.has_mask, [&](auto lt, auto st, auto mk) -> int {
                using L = typename decltype(lt)::type;
                using S = typename decltype(st)::type;
                constexpr bool M = decltype(mk)::value;
                hipLaunchKernelGGL((k_init_eq<L, S, M>), dim3((h.nx + BLK_X - 1) / BLK_X, (h.ny + BLK_Y - 1) / BLK_Y, 1),
                                   dim3(BLK_X, BLK_Y, 1), 0, b->stream, (S *)dst + h.off, b->d_mask + h.moff, g,
                                   0, rho ? d_in : nullptr, u ? d_in + h.N : nullptr, h.N);
                return PTRT_OK;
            });
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    hipFree(d_in);
    if (e != hipSuccess) return bfail_hip(b, PTRT_EDEVICE, std::string("init: ") + hipGetErrorString(e));
    return PTRT_OK;
}

int ptrt_batch_set_plan(ptrt_batch *b, int tile_x, int tile_y, int blocks, int xcd_order)
{
    if (!b) return PTRT_EINVAL;
    if (!valid_plan(tile_x, tile_y) || blocks < 0) return bfail(b, PTRT_EINVAL, "invalid tile plan");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    const int old[4] = {b->tile_x, b->tile_y, b->blocks, b->xcd_order};
    b->tile_x = tile_x;
    b->tile_y = tile_y;
    b->blocks = blocks;
    b->xcd_order = xcd_order ? 1 : 0;
    const int rc = build_tiles(b);
    if (rc != PTRT_OK) { // the previous plan and its table stay
        b->tile_x = old[0];
        b->tile_y = old[1];
        b->blocks = old[2];
        b->xcd_order = old[3];
    }
    return rc;
}

int ptrt_batch_step(ptrt_batch *b, int n)
{
    if (!b) return PTRT_EINVAL;
    if (n < 0) return bfail(b, PTRT_EINVAL, "negative step count");
    while (n >= GRAPH_STEPS) {
        if (!b->graph[b->cur]) {
            int rc = capture_graph(b, b->cur);
            if (rc != PTRT_OK) return rc;
        }
        BHIPCHK(b, hipGraphLaunch(b->graph[b->cur], b->stream));
        b->last_steps = two_step(b) ? 2 : 1;
        b->cur ^= b->graph_flip[b->cur];
        n -= GRAPH_STEPS;
    }
    advance(b, b->stream, n);
    BHIPCHK(b, hipGetLastError());
    return PTRT_OK;
}

int ptrt_batch_set_steps_per_pass(ptrt_batch *b, int steps)
{
    if (!b) return PTRT_EINVAL;
    if (steps != 1 && steps != 2) return bfail(b, PTRT_EINVAL, "steps per pass must be 1 or 2");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->spp = steps;
    drop_graphs(b);
    return PTRT_OK;
}

int ptrt_batch_last_pass(const ptrt_batch *b, int *steps, double *bytes)
{
    if (!b || !steps || !bytes) return PTRT_EINVAL;
    *steps = b->last_steps;
    *bytes = b->last_steps ? ptrt_batch_bytes_per_step(b) : 0.0;
    return PTRT_OK;
}

int ptrt_batch_step_separate(ptrt_batch *b, int n)
{
    if (!b) return PTRT_EINVAL;
    if (n < 0) return bfail(b, PTRT_EINVAL, "negative step count");
    for (int s = 0; s < n; ++s) {
        for (int k = 0; k < b->count; ++k) {
            const HostInst &h = b->inst[k];
            const Geom g = inst_geom(h);
            const int bx = 64, by = 4;
            const dim3 grid((h.nx + bx - 1) / bx, (h.ny + by - 1) / by, 1);
            dispatch(PTRT_D2Q9, b->storage, h.has_mask, [&](auto lt, auto st, auto mk) -> int {
                using L = typename decltype(lt)::type;
                using S = typename decltype(st)::type;
                using C = typename Codec<S>::compute;
                constexpr bool M = decltype(mk)::value;
                const Coef<L, C> r = make_coef<L, C>(h.tau_plus, h.Lambda, h.force);
                hipLaunchKernelGGL((k_step<L, S, M, false, true, false>), grid, dim3(bx, by, 1), 0, b->stream,
                                   (const S *)b->buf[b->cur] + h.off, (S *)b->buf[b->cur ^ 1] + h.off,
                                   b->d_mask + h.moff, b->d_near + h.noff, g, r, (double2 *)nullptr);
                return PTRT_OK;
            });
        }
        b->cur ^= 1;
    }
    BHIPCHK(b, hipGetLastError());
    return PTRT_OK;
}

int ptrt_batch_set_plan2(ptrt_batch *b, int rows, int masked_rows, int waves, int blocks,
                         int concurrent)
{
    if (!b) return PTRT_EINVAL;
    if (rows < 1 || rows > 64 || masked_rows < 1 || masked_rows > 64 ||
        (waves != 2 && waves != 4 && waves != 8) || blocks < 0)
        return bfail(b, PTRT_EINVAL, "invalid two-step plan");
    if (b->storage != PTRT_F32 && b->storage != PTRT_F64)
        return bfail(b, PTRT_ESTATE, "the two-step pass runs in FP32 and FP64 storage only");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    const int old[5] = {b->yc2, b->ym2, b->nw2, b->blocks2, b->conc2};
    b->yc2 = rows;
    b->ym2 = masked_rows;
    b->nw2 = waves;
    b->blocks2 = blocks;
    b->conc2 = concurrent ? 1 : 0;
    const int rc = build_tasks2(b);
    if (rc != PTRT_OK) { // the previous plan and its table stay
        b->yc2 = old[0];
        b->ym2 = old[1];
        b->nw2 = old[2];
        b->blocks2 = old[3];
        b->conc2 = old[4];
    }
    return rc;
}

int ptrt_batch_get_plan2(const ptrt_batch *b, int plan_out[5])
{
    if (!b || !plan_out) return PTRT_EINVAL;
    plan_out[0] = b->yc2;
    plan_out[1] = b->ym2;
    plan_out[2] = b->nw2;
    plan_out[3] = b->blocks2;
    plan_out[4] = b->conc2;
    return PTRT_OK;
}

int ptrt_batch_autotune(ptrt_batch *b, int *tx_o, int *ty_o, int *blocks_o, int *xcd_o)
{
    if (!b) return PTRT_EINVAL;
    static const int shapes[][2] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}, {1024, 1},
                                    {64, 2}, {64, 4}, {128, 2}, {32, 8}, {64, 8}};
    static const int grids[] = {0, 2048, 4096};
    const size_t bytes = (size_t)b->total_elems * storage_bytes(b->storage);
    // the trials run on a copy of the state, which is put back afterwards
    void *saved = nullptr;
    BHIPCHK(b, hipMalloc(&saved, bytes));
    const int cur0 = b->cur;
    hipError_t e = hipMemcpyAsync(saved, b->buf[cur0], bytes, hipMemcpyDeviceToDevice, b->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    int bt[4] = {b->tile_x, b->tile_y, b->blocks, b->xcd_order};
    int rc = e == hipSuccess ? PTRT_OK : bfail_hip(b, PTRT_EDEVICE, "autotune setup failed");
    for (const auto &sh : shapes) {
        if (rc != PTRT_OK) break;
        for (int gsz : grids)
            for (int xo = 0; xo < 2 && rc == PTRT_OK; ++xo) {
                rc = ptrt_batch_set_plan(b, sh[0], sh[1], gsz, xo);
                if (rc != PTRT_OK) break;
                for (int k = 0; k < 2; ++k) launch_fused_any(b, b->stream);
                hipEventRecord(e0, b->stream);
                for (int k = 0; k < 14; ++k) launch_fused_any(b, b->stream);
                hipEventRecord(e1, b->stream);
                if (hipEventSynchronize(e1) != hipSuccess) {
                    rc = bfail_hip(b, PTRT_EDEVICE, "autotune timing failed");
                    break;
                }
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    bt[0] = sh[0];
                    bt[1] = sh[1];
                    bt[2] = gsz;
                    bt[3] = xo;
                }
            }
    }
    // the two-step plan, on the same saved state
    if (rc == PTRT_OK && b->d_tasks2) rc = autotune2(b, e0, e1);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    // restore the state into buffer cur0 (the trials may end on either)
    b->cur = cur0;
    e = hipMemcpyAsync(b->buf[cur0], saved, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    hipFree(saved);
    if (rc != PTRT_OK) return rc;
    if (e != hipSuccess) return bfail_hip(b, PTRT_EDEVICE, std::string("autotune restore: ") + hipGetErrorString(e));
    rc = ptrt_batch_set_plan(b, bt[0], bt[1], bt[2], bt[3]);
    if (tx_o) *tx_o = bt[0];
    if (ty_o) *ty_o = bt[1];
    if (blocks_o) *blocks_o = bt[2];
    if (xcd_o) *xcd_o = bt[3];
    return rc;
}

static int batch_download(ptrt_batch *b, int k, double *rho, double *u, double *f)
{
    int rc = check_instance(b, k);
    if (rc != PTRT_OK) return rc;
    const HostInst &h = b->inst[k];
    const int per = (rho ? 1 : 0) + (u ? 3 : 0) + (f ? 9 : 0);
    if (per == 0) return PTRT_OK;
    double *d_out = nullptr;
    BHIPCHK(b, hipMalloc(&d_out, sizeof(double) * per * (size_t)h.N));
    double *d_rho = rho ? d_out : nullptr;
    double *d_u = u ? d_out + (rho ? h.N : 0) : nullptr;
    double *d_f = f ? d_out + ((rho ? 1 : 0) + (u ? 3 : 0)) * h.N : nullptr;
    const Geom g = inst_geom(h);
    dispatch(PTRT_D2Q9, b->storage, h.has_mask, [&](auto lt, auto st, auto mk) -> int {
        using L = typename decltype(lt)::type;
        using S = typename decltype(st)::type;
        constexpr bool M = decltype(mk)::value;
        hipLaunchKernelGGL((k_gather<L, S, M>), dim3((h.nx + BLK_X - 1) / BLK_X, (h.ny + BLK_Y - 1) / BLK_Y, 1),
                           dim3(BLK_X, BLK_Y, 1), 0, b->stream, (const S *)b->buf[b->cur] + h.off,
                           b->d_mask + h.moff, g, 0, h.force[0], h.force[1], 0.0, d_rho, d_u, d_f, h.N,
                           (double2 *)nullptr);
        return PTRT_OK;
    });
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && rho)
        e = hipMemcpyAsync(rho, d_rho, sizeof(double) * h.N, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && u)
        e = hipMemcpyAsync(u, d_u, sizeof(double) * 2 * h.N, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && f)
        e = hipMemcpyAsync(f, d_f, sizeof(double) * 9 * h.N, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    hipFree(d_out);
    if (e != hipSuccess) return bfail_hip(b, PTRT_EDEVICE, std::string("download: ") + hipGetErrorString(e));
    if (u) std::memset(u + 2 * h.N, 0, sizeof(double) * h.N);
    return PTRT_OK;
}

int ptrt_batch_moments(ptrt_batch *b, int k, double *rho, double *u)
{
    return batch_download(b, k, rho, u, nullptr);
}

int ptrt_batch_get_populations(ptrt_batch *b, int k, double *f)
{
    if (!f) return bfail(b, PTRT_EINVAL, "NULL argument");
    return batch_download(b, k, nullptr, nullptr, f);
}

int ptrt_batch_diagnostics(ptrt_batch *b, double *mass, double *ke)
{
    if (!b) return PTRT_EINVAL;
    for (int k = 0; k < b->count; ++k) {
        const HostInst &h = b->inst[k];
        const Geom g = inst_geom(h);
        const dim3 grid((h.nx + BLK_X - 1) / BLK_X, (h.ny + BLK_Y - 1) / BLK_Y, 1);
        dispatch(PTRT_D2Q9, b->storage, h.has_mask, [&](auto lt, auto st, auto mk) -> int {
            using L = typename decltype(lt)::type;
            using S = typename decltype(st)::type;
            constexpr bool M = decltype(mk)::value;
            hipLaunchKernelGGL((k_gather<L, S, M>), grid, dim3(BLK_X, BLK_Y, 1), 0, b->stream,
                               (const S *)b->buf[b->cur] + h.off, b->d_mask + h.moff, g, 0, h.force[0],
                               h.force[1], 0.0, (double *)nullptr, (double *)nullptr, (double *)nullptr,
                               0LL, b->d_partials);
            return PTRT_OK;
        });
        hipLaunchKernelGGL(k_finalize<1024>, dim3(1), dim3(1024), 0, b->stream, b->d_partials,
                           (int)(grid.x * grid.y), b->d_red + 2 * k);
    }
    BHIPCHK(b, hipGetLastError());
    std::vector<double> r(2 * (size_t)b->count);
    BHIPCHK(b, hipMemcpyAsync(r.data(), b->d_red, sizeof(double) * r.size(), hipMemcpyDeviceToHost, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    bool ok = true;
    for (int k = 0; k < b->count; ++k) {
        if (mass) mass[k] = r[2 * k];
        if (ke) ke[k] = r[2 * k + 1];
        ok = ok && std::isfinite(r[2 * k]) && std::isfinite(r[2 * k + 1]);
    }
    if (!ok) return bfail(b, PTRT_EDIVERGED, "non-finite mass or kinetic energy");
    return PTRT_OK;
}

long long ptrt_batch_nodes(const ptrt_batch *b) { return b ? b->total_nodes : 0; }

double ptrt_batch_bytes_per_step(const ptrt_batch *b)
{
    if (!b) return 0.0;
    return (2.0 * 9 * (double)storage_bytes(b->storage) + 1.0) * (double)b->total_nodes;
}

const char *ptrt_batch_last_error(const ptrt_batch *b)
{
    return b ? b->err.c_str() : g_batch_create_error.c_str();
}

int ptrt_batch_destroy(ptrt_batch *b)
{
    if (!b) return PTRT_OK;
    hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (int k = 0; k < 2; ++k)
        if (b->buf[k]) hipFree(b->buf[k]);
    if (b->d_mask) hipFree(b->d_mask);
    if (b->d_near) hipFree(b->d_near);
    if (b->d_inst) hipFree(b->d_inst);
    if (b->d_tiles) hipFree(b->d_tiles);
    if (b->d_tasks2) hipFree(b->d_tasks2);
    if (b->d_partials) hipFree(b->d_partials);
    if (b->d_red) hipFree(b->d_red);
    if (b->capture_stream) hipStreamDestroy(b->capture_stream);
    if (b->side_stream) (void)hipStreamDestroy(b->side_stream);
    if (b->fork_event) (void)hipEventDestroy(b->fork_event);
    if (b->join_event) (void)hipEventDestroy(b->join_event);
    delete b;
    return PTRT_OK;
}

} // extern "C"
