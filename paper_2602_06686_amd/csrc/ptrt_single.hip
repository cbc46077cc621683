// Single-lattice entry points of libptrt (declared in include/ptrt.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "step_launch.hpp"

using namespace ptrt;

static_assert(FORCE_II == PTRT_FORCING_SCHEME2 && FORCE_II_G == PTRT_FORCING_SCHEME2_G &&
                  FORCE_GUO == PTRT_FORCING_GUO,
              "forcing ids of the kernels and of the C interface");
static_assert(MODEL_PTRT == PTRT_MODEL_PTRT && MODEL_TRT_RLB == PTRT_MODEL_TRT_RLB &&
                  MODEL_TRT == PTRT_MODEL_TRT && MODEL_PTRT_EXACT == PTRT_MODEL_PTRT_EXACT,
              "model ids of the kernels and of the C interface");

// Device scratch of ptrt_momentum_exchange_noalloc (see noalloc_scratch).
static __device__ __align__(256) char scratch[16u << 20];

namespace {

thread_local std::string g_create_error = "no error";

constexpr int BLK_X = 64, BLK_Y = 4; // gather / scatter workgroup shape
constexpr int GRAPH_STEPS = 20;      // even, so a replay keeps the buffer parity

} // namespace

struct ptrt_ctx {
    int lattice = 0, Q = 0;
    int nx = 0, ny = 0, nz = 0;
    long long N = 0, elems = 0;
    Geom geo{};
    double tau_plus = 0, Lambda = 0, g[3] = {0, 0, 0};
    int storage = PTRT_F32;
    bool has_mask = false;
    std::vector<uint8_t> h_mask, h_near;
    uint8_t *d_mask = nullptr, *d_near = nullptr;
    // D2Q9 with solids: two-step tasks without / with solids near their rows
    int4 *d_tasks = nullptr; // plain tasks, then special (masked / open) ones
    int n_plain = 0, n_special = 0;
    long long masked_rows = 0;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    double2 *d_partials = nullptr;
    int nparts = 0;
    double *d_red = nullptr;
    hipStream_t stream = nullptr;
    bool allocated = false, initialized = false;
    long long t = 0;
    bool row_kernel = false, nt_store = false;
    int row_bx = 256;
    int model = MODEL_PTRT;
    int forcing = FORCE_II;
    void *d_phi = nullptr; // Phi field of the cubic correction (compute type)
    bool open = false;     // D2Q9 velocity inlet / pressure outlet in x
    int steps_per_pass = 2; // up to two fused steps per pass where allowed
    int last_pass_steps = 0;      // steps covered by the most recent pass
    double last_pass_bytes = 0.0; // its algorithmic HBM bytes
    double *d_force_parts = nullptr, *d_force = nullptr; // momentum exchange
    // small lattices: steps replayed from captured graphs of GRAPH_STEPS launches
    bool use_graph = false;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    // divergence check after every check_every-th step (0 = off): the
    // earliest step at which the state held a NaN or infinity, on the
    // device, copied to pinned host memory after each check
    int check_every = 0;
    unsigned long long *d_bad = nullptr, *h_bad = nullptr;
    hipEvent_t bad_event = nullptr;
    bool bad_pending = false;
    long long diverged_at = -1;
    std::string err = "no error";
};

namespace {

int fail(ptrt_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

// A failed HIP call, reported here: its error is also taken off the
// thread's last-error slot, so that a later launch check (hipGetLastError)
// does not report it a second time as its own.
int fail_hip(ptrt_ctx *c, int code, const std::string &msg)
{
    (void)hipGetLastError();
    return fail(c, code, msg);
}

#define HIPCHK(c, expr)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail_hip((c), PTRT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// f(bool_constant<OPEN>) for the handle's x boundaries (open ones exist on
// D2Q9 only).
template <class L, class F>
void with_open(const ptrt_ctx *c, F &&f)
{
    if constexpr (L::Q == 9) {
        if (c->open) {
            f(std::true_type{});
            return;
        }
    }
    f(std::false_type{});
}

dim3 gather_grid(const ptrt_ctx *c, int nzs)
{
    return dim3((c->nx + BLK_X - 1) / BLK_X, (c->ny + BLK_Y - 1) / BLK_Y, nzs);
}

// z-slab height so that a [Q][slab] FP64 host transfer stays under ~512 MB
int slab_planes(const ptrt_ctx *c, int per_node_doubles)
{
    const double plane = (double)c->nx * c->ny * per_node_doubles * 8.0;
    int s = (int)std::max(1.0, 512.0 * 1024 * 1024 / plane);
    return std::min(s, c->nz);
}

int ensure_phi(ptrt_ctx *c, int forcing);

// Free what allocate_device has allocated (after a failure part way, so
// that the next attempt starts from nothing).
void release_device(ptrt_ctx *c)
{
    for (void *&p : c->buf)
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
    void **owned[] = {(void **)&c->d_mask, (void **)&c->d_near, (void **)&c->d_tasks,
                      (void **)&c->d_partials, (void **)&c->d_red};
    for (void **p : owned)
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    c->n_plain = c->n_special = 0;
}

int allocate_device(ptrt_ctx *c);

int ensure_allocated(ptrt_ctx *c)
{
    if (c->allocated) return PTRT_OK;
    const int rc = allocate_device(c);
    if (rc != PTRT_OK) {
        release_device(c);
        return rc;
    }
    c->allocated = true;
    return ensure_phi(c, c->forcing);
}

int allocate_device(ptrt_ctx *c)
{
    const size_t elem = storage_bytes(c->storage);
    c->elems = make_layout(c->Q, c->nx, c->ny, c->nz, elem, c->geo);
    const size_t bytes = (size_t)c->elems * elem;
    // Row workgroups covering 1 KB of each direction's row (measured best on
    // MI355X for every storage type); non-temporal stores once the two
    // population buffers are larger than the 256 MB last-level cache.
    c->row_bx = std::min<int>(1024 / (int)elem, ((c->nx + 63) / 64) * 64);
    c->nt_store = 2.0 * (double)bytes > 256.0 * 1024 * 1024;
    // below ~32 MB per step a launch costs about as much as its work
    c->use_graph = 2.0 * (double)bytes < 32.0 * 1024 * 1024;
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMalloc(&c->buf[k], bytes);
        if (e != hipSuccess) {
            c->buf[k] = nullptr;
            return fail_hip(c, PTRT_ENOMEM, std::string("hipMalloc of populations: ") + hipGetErrorString(e));
        }
        HIPCHK(c, hipMemset(c->buf[k], 0, bytes));
    }
    if (c->has_mask) {
        HIPCHK(c, hipMalloc(&c->d_mask, (size_t)c->N));
        HIPCHK(c, hipMemcpy(c->d_mask, c->h_mask.data(), (size_t)c->N, hipMemcpyHostToDevice));
        c->h_near = near_solid_rows(c->h_mask.data(), c->nx, c->ny, c->nz);
        HIPCHK(c, hipMalloc(&c->d_near, c->h_near.size()));
        HIPCHK(c, hipMemcpy(c->d_near, c->h_near.data(), c->h_near.size(), hipMemcpyHostToDevice));
    }
    if (c->lattice == PTRT_D3Q19 && c->has_mask) {
        // the 3D two-step pass with solids: mask-free and masked column
        // chunks (none when the pass does not apply)
        std::vector<int4> plain, special;
        bool ok = false;
        if (c->storage == PTRT_F32)
            ok = step2_3d_task_lists<D3Q19, float>(c->geo, c->h_near.data(), plain, special);
        else if (c->storage == PTRT_F64)
            ok = step2_3d_task_lists<D3Q19, double>(c->geo, c->h_near.data(), plain, special);
        if (ok && (!plain.empty() || !special.empty())) {
            c->n_plain = (int)plain.size();
            c->n_special = (int)special.size();
            plain.insert(plain.end(), special.begin(), special.end());
            HIPCHK(c, hipMalloc(&c->d_tasks, sizeof(int4) * plain.size()));
            HIPCHK(c, hipMemcpy(c->d_tasks, plain.data(), sizeof(int4) * plain.size(), hipMemcpyHostToDevice));
        }
    }
    if (c->lattice == PTRT_D2Q9 && (c->has_mask || c->open)) {
        // the two-step kernel's tasks {0, x0, ys, ye}: strips of BX columns
        // times chunks of yc rows with no solid within one row of rows
        // ys - 1 ... ye (plain); the rows of the other chunks, and with open
        // x every row of the first and last strip, in chunks of ym rows
        // (special: the masked / open kernel), ym by the same rule over
        // those rows alone with twice the task target (the masked code
        // waits for the mask before its pulls; a few rows near solids give
        // short special tasks, whose time is latency).  Measured, GLUPS
        // with the masked rows in chunks of ym = yc, then by this rule:
        // FP32 channel 1024^2 50.5 -> 89.2, 2048^2 84.7 -> 101.0; FP32
        // obstacle 1024^2 49.2 -> 81.6, 2048^2 84.4 -> 96.2; FP64 channel
        // 1024^2 43.1 -> 57.9 (target x1, x2, x4, x8: obstacle 2048^2
        // FP32 85.6 / 96.2 / 94.9 / 91.5)
        using SH = Step2Shape2D<float>;
        const int strips = (c->nx + SH::BX - 1) / SH::BX;
        const int yc = step2_2d_rows(c->storage, c->nx, c->ny);
        std::vector<int4> plain, special;
        struct Chunk {
            int ys, ye;
            std::vector<int> bxs; // strips whose tasks are special
        };
        std::vector<Chunk> spec;
        long long masked_rows = 0, spec_strip_rows = 0;
        for (int ys = 0; ys < c->ny; ys += yc) {
            const int ye = std::min(ys + yc, c->ny);
            bool near = false;
            if (c->has_mask)
                for (int y = ys - 1; y <= ye && !near; ++y)
                    near = c->h_near[(size_t)(((y % c->ny) + c->ny) % c->ny)] != 0;
            if (near) masked_rows += ye - ys;
            Chunk ch{ys, ye, {}};
            for (int bx = 0; bx < strips; ++bx) {
                const bool edge = c->open && (bx == 0 || bx == strips - 1);
                if (near || edge)
                    ch.bxs.push_back(bx);
                else
                    plain.push_back(make_int4(0, bx * SH::BX, ys, ye));
            }
            if (!ch.bxs.empty()) {
                spec_strip_rows += (long long)ch.bxs.size() * (ye - ys);
                spec.push_back(std::move(ch));
            }
        }
        const int ym = step2_2d_rows_for(c->storage, spec_strip_rows, (long long)SH::BX * spec_strip_rows, 2);
        for (const Chunk &ch : spec)
            for (int ys = ch.ys; ys < ch.ye; ys += ym)
                for (int bx : ch.bxs)
                    special.push_back(make_int4(0, bx * SH::BX, ys, std::min(ys + ym, ch.ye)));
        c->n_plain = (int)plain.size();
        c->n_special = (int)special.size();
        c->masked_rows = masked_rows;
        plain.insert(plain.end(), special.begin(), special.end());
        HIPCHK(c, hipMalloc(&c->d_tasks, sizeof(int4) * plain.size()));
        HIPCHK(c, hipMemcpy(c->d_tasks, plain.data(), sizeof(int4) * plain.size(), hipMemcpyHostToDevice));
    }
    const dim3 gg = gather_grid(c, c->nz);
    c->nparts = gg.x * gg.y * gg.z;
    HIPCHK(c, hipMalloc(&c->d_partials, sizeof(double2) * (size_t)c->nparts));
    HIPCHK(c, hipMalloc(&c->d_red, 2 * sizeof(double)));
    return PTRT_OK;
}

Geom geom(const ptrt_ctx *c) { return c->geo; }

// Scatter host data (equilibrium from rho/u, or populations f) into the
// current buffer, slab by slab.
int upload_state(ptrt_ctx *c, const double *rho, const double *u, const double *f)
{
    const bool pops = f != nullptr;
    const int per_node = pops ? c->Q : 4;
    const int slab = slab_planes(c, per_node);
    const long long plane = (long long)c->nx * c->ny;
    double *d_in = nullptr;
    const size_t in_elems = (size_t)per_node * slab * plane;
    HIPCHK(c, hipMalloc(&d_in, in_elems * sizeof(double)));
    int rc = PTRT_OK;
    for (int z0 = 0; z0 < c->nz && rc == PTRT_OK; z0 += slab) {
        const int nzs = std::min(slab, c->nz - z0);
        const long long cnt = nzs * plane;
        const double *d_rho = nullptr, *d_u = nullptr;
        hipError_t e = hipSuccess;
        if (pops) {
            for (int i = 0; i < c->Q && e == hipSuccess; ++i)
                e = hipMemcpyAsync(d_in + (size_t)i * cnt, f + (size_t)i * c->N + z0 * plane,
                                   cnt * sizeof(double), hipMemcpyHostToDevice, c->stream);
        } else {
            if (rho) {
                e = hipMemcpyAsync(d_in, rho + z0 * plane, cnt * sizeof(double),
                                   hipMemcpyHostToDevice, c->stream);
                d_rho = d_in;
            }
            if (u && e == hipSuccess) {
                const int D = c->lattice == PTRT_D2Q9 ? 2 : 3;
                for (int a = 0; a < D && e == hipSuccess; ++a)
                    e = hipMemcpyAsync(d_in + (size_t)(1 + a) * cnt, u + (size_t)a * c->N + z0 * plane,
                                       cnt * sizeof(double), hipMemcpyHostToDevice, c->stream);
                d_u = d_in + cnt;
            }
        }
        if (e != hipSuccess) {
            rc = fail_hip(c, PTRT_EDEVICE, std::string("host to device copy: ") + hipGetErrorString(e));
            break;
        }
        const Geom g = geom(c);
        void *dst = c->buf[c->cur];
        const dim3 grid = gather_grid(c, nzs), block(BLK_X, BLK_Y, 1);
        dispatch(c->lattice, c->storage, c->has_mask, [&](auto lt, auto st, auto mk) -> int {
            using L = typename decltype(lt)::type;
            using S = typename decltype(st)::type;
            constexpr bool M = decltype(mk)::value;
            with_open<L>(c, [&](auto oc) {
                constexpr bool O = decltype(oc)::value;
                if (pops)
                    hipLaunchKernelGGL((k_set_state<L, S, M, O>), grid, block, 0, c->stream,
                                       (S *)dst, c->d_mask, g, z0, d_in, cnt);
                else
                    hipLaunchKernelGGL((k_init_eq<L, S, M, O>), grid, block, 0, c->stream,
                                       (S *)dst, c->d_mask, g, z0, d_rho, d_u, cnt);
            });
            return PTRT_OK;
        });
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = fail_hip(c, PTRT_EDEVICE, std::string("state upload: ") + hipGetErrorString(e));
    }
    (void)hipFree(d_in);
    return rc;
}

// Gather rho/u/f (any may be null) of the state at t to host arrays.
int download_state(ptrt_ctx *c, double *rho, double *u, double *f)
{
    const int per_node = (f ? c->Q : 0) + (rho ? 1 : 0) + (u ? 3 : 0);
    if (per_node == 0) return PTRT_OK;
    const int slab = slab_planes(c, per_node);
    const long long plane = (long long)c->nx * c->ny;
    double *d_out = nullptr;
    HIPCHK(c, hipMalloc(&d_out, (size_t)per_node * slab * plane * sizeof(double)));
    int rc = PTRT_OK;
    for (int z0 = 0; z0 < c->nz; z0 += slab) {
        const int nzs = std::min(slab, c->nz - z0);
        const long long cnt = nzs * plane;
        double *d_rho = rho ? d_out : nullptr;
        double *d_u = u ? d_out + (rho ? cnt : 0) : nullptr;
        double *d_f = f ? d_out + ((rho ? 1 : 0) + (u ? 3 : 0)) * cnt : nullptr;
        const Geom g = geom(c);
        const void *src = c->buf[c->cur];
        const dim3 grid = gather_grid(c, nzs), block(BLK_X, BLK_Y, 1);
        dispatch(c->lattice, c->storage, c->has_mask, [&](auto lt, auto st, auto mk) -> int {
            using L = typename decltype(lt)::type;
            using S = typename decltype(st)::type;
            constexpr bool M = decltype(mk)::value;
            with_open<L>(c, [&](auto oc) {
                constexpr bool O = decltype(oc)::value;
                hipLaunchKernelGGL((k_gather<L, S, M, O>), grid, block, 0, c->stream,
                                   (const S *)src, c->d_mask, g, z0, c->g[0], c->g[1], c->g[2],
                                   d_rho, d_u, d_f, cnt, (double2 *)nullptr);
            });
            return PTRT_OK;
        });
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && rho)
            e = hipMemcpyAsync(rho + z0 * plane, d_rho, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (u) {
            const int D = c->lattice == PTRT_D2Q9 ? 2 : 3;
            for (int a = 0; a < 3 && e == hipSuccess; ++a) {
                if (a < D)
                    e = hipMemcpyAsync(u + (size_t)a * c->N + z0 * plane, d_u + (size_t)a * cnt,
                                       cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            }
        }
        if (f)
            for (int i = 0; i < c->Q && e == hipSuccess; ++i)
                e = hipMemcpyAsync(f + (size_t)i * c->N + z0 * plane, d_f + (size_t)i * cnt,
                                   cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            rc = fail_hip(c, PTRT_EDEVICE, std::string("state download: ") + hipGetErrorString(e));
            break;
        }
    }
    if (u && c->lattice == PTRT_D2Q9) std::memset(u + 2 * (size_t)c->N, 0, (size_t)c->N * sizeof(double));
    (void)hipFree(d_out);
    return rc;
}

StepLaunch step_args(const ptrt_ctx *c, hipStream_t s);

// Enqueue one fused step on stream s (buffer cur -> cur ^ 1).
void launch_step(ptrt_ctx *c, hipStream_t s)
{
    const StepLaunch a = step_args(c, s);
    c->last_pass_steps = 1;
    c->last_pass_bytes = (double)c->N * (2.0 * c->Q * storage_bytes(c->storage) + (c->has_mask ? 1.0 : 0.0));
    if (c->lattice == PTRT_D2Q9) launch_step_d2q9(a);
    else if (c->lattice == PTRT_D3Q19) launch_step_d3q19(a);
    else launch_step_d3q27(a);
    c->cur ^= 1;
}

// Enqueue n steps: pairs in one pass where the configuration allows it.
void launch_steps(ptrt_ctx *c, hipStream_t s, int n)
{
    while (n >= 2 && c->steps_per_pass == 2) {
        const StepLaunch a = step_args(c, s);
        bool two = false;
        double bytes = 0.0;
        if (c->lattice == PTRT_D2Q9) two = launch_step2_d2q9(a, &bytes);
        else if (c->lattice == PTRT_D3Q19) two = launch_step2_d3q19(a, &bytes);
        else if (c->lattice == PTRT_D3Q27) two = launch_step2_d3q27(a, &bytes);
        if (!two) break;
        c->cur ^= 1;
        c->last_pass_steps = 2;
        c->last_pass_bytes = bytes;
        n -= 2;
    }
    for (; n > 0; --n) launch_step(c, s);
}

StepLaunch step_args(const ptrt_ctx *c, hipStream_t s)
{
    StepLaunch a;
    a.src = c->buf[c->cur];
    a.dst = c->buf[c->cur ^ 1];
    a.mask = c->d_mask;
    a.near = c->d_near;
    if (c->d_tasks) {
        a.tasks_plain = c->d_tasks;
        a.tasks_special = c->d_tasks + c->n_plain;
        a.n_plain = c->n_plain;
        a.n_special = c->n_special;
        a.masked_rows = c->masked_rows;
    }
    a.g = geom(c);
    a.tau_plus = c->tau_plus;
    a.Lambda = c->Lambda;
    for (int k = 0; k < 3; ++k) a.force[k] = c->g[k];
    a.storage = c->storage;
    a.has_mask = c->has_mask;
    a.row = c->row_kernel;
    a.row_bx = c->row_bx;
    a.nt = c->nt_store;
    a.model = c->model;
    a.forcing = c->forcing;
    a.phi = c->d_phi;
    a.open = c->open;
    a.stream = s;
    return a;
}

// Bytes of the Phi field: D components per node in the compute type.
size_t phi_bytes(const ptrt_ctx *c)
{
    const size_t comp = c->storage == PTRT_F64 ? 8 : 4;
    const size_t D = c->lattice == PTRT_D2Q9 ? 2 : 3;
    return D * (size_t)c->N * comp;
}

// Allocate the Phi field once the populations are allocated and the cubic
// correction is (or is about to be) selected.
int ensure_phi(ptrt_ctx *c, int forcing)
{
    if (forcing != FORCE_II_G || c->d_phi || !c->allocated) return PTRT_OK;
    hipError_t e = hipMalloc(&c->d_phi, phi_bytes(c));
    if (e != hipSuccess) {
        c->d_phi = nullptr;
        return fail_hip(c, PTRT_ENOMEM, std::string("hipMalloc of the Phi field: ") + hipGetErrorString(e));
    }
    return PTRT_OK;
}

void drop_graphs(ptrt_ctx *c)
{
    for (auto &gx : c->graph)
        if (gx) {
            (void)hipGraphExecDestroy(gx);
            gx = nullptr;
        }
}

// Capture GRAPH_STEPS steps starting from buffer `parity` into graph[parity].
int capture_graph(ptrt_ctx *c, int parity)
{
    if (!c->capture_stream)
        HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    const int saved = c->cur;
    c->cur = parity;
    hipGraph_t gr = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    launch_steps(c, c->capture_stream, GRAPH_STEPS);
    hipError_t e = hipStreamEndCapture(c->capture_stream, &gr);
    c->cur = saved;
    if (e != hipSuccess) return fail_hip(c, PTRT_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph[parity], gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
        c->graph[parity] = nullptr;
        return fail_hip(c, PTRT_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return PTRT_OK;
}

constexpr unsigned long long NO_STEP = ~0ull;

// Momentum exchange: per-block partials (three per 64 x 4 gather block)
// reduced in a fixed order into out[3], copied to force_out; synchronous.
size_t momentum_parts(const ptrt_ctx *c)
{
    const dim3 grid = gather_grid(c, c->nz);
    return (size_t)grid.x * grid.y * grid.z;
}

int momentum_exchange_with(ptrt_ctx *c, double *parts, double *out, double force_out[3])
{
    const dim3 grid = gather_grid(c, c->nz), block(BLK_X, BLK_Y, 1);
    const int nparts = (int)momentum_parts(c);
    const Geom g = geom(c);
    const void *src = c->buf[c->cur];
    dispatch(c->lattice, c->storage, false, [&](auto lt, auto st, auto) -> int {
        using L = typename decltype(lt)::type;
        using S = typename decltype(st)::type;
        with_open<L>(c, [&](auto oc) {
            constexpr bool O = decltype(oc)::value;
            hipLaunchKernelGGL((k_momentum_exchange<L, S, O>), grid, block, 0, c->stream,
                               (const S *)src, c->d_mask, c->d_near, g, parts);
        });
        return PTRT_OK;
    });
    hipLaunchKernelGGL(k_finalize3<1024>, dim3(1), dim3(1024), 0, c->stream, parts, nparts, out);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(force_out, out, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PTRT_OK;
}

// Fixed device scratch of ptrt_momentum_exchange_noalloc: the three result
// values at offset 0, the per-block partials from NOALLOC_PARTS_OFFSET on.
// In host code `scratch` only names the symbol; its device address (one per
// GPU) comes from hipGetSymbolAddress on the first call on that GPU.
constexpr size_t NOALLOC_SCRATCH_BYTES = 16u << 20;
constexpr size_t NOALLOC_PARTS_OFFSET = 256;
static_assert(sizeof(scratch) == NOALLOC_SCRATCH_BYTES, "scratch size");
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
char *g_scratch_ptr[MAX_DEVICES] = {};

int noalloc_scratch(ptrt_ctx *c, char **out)
{
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(c, PTRT_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(c, PTRT_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return PTRT_OK;
}

// Forget earlier check results (a new state was set); waits for the stream.
int reset_check(ptrt_ctx *c)
{
    c->bad_pending = false;
    c->diverged_at = -1;
    if (!c->d_bad || !c->h_bad || !c->bad_event) return PTRT_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemset(c->d_bad, 0xFF, sizeof(unsigned long long)));
    *c->h_bad = NO_STEP;
    return PTRT_OK;
}

// Pick up what the copies that have run so far brought back (no wait): the
// host runs ahead of the device, so the latest check is rarely finished,
// but every finished copy carries the minimum over all checks before it.
// A value is taken only if it is a step already enqueued (a copy in flight
// cannot then be mistaken for a result).
void poll_check(ptrt_ctx *c)
{
    if (!c->bad_pending) return;
    const unsigned long long v = *(volatile unsigned long long *)c->h_bad;
    if (v != NO_STEP && (long long)v <= c->t && v % (unsigned long long)c->check_every == 0)
        c->diverged_at = (long long)v;
    if (hipEventQuery(c->bad_event) == hipSuccess) c->bad_pending = false;
}

// Enqueue the check of the current state (step c->t) and the copy of its
// result to the host.
int launch_check(ptrt_ctx *c)
{
    const long long nvec = c->elems * (long long)storage_bytes(c->storage) / 16;
    const int blocks = (int)std::min<long long>((nvec + 255) / 256, 4096);
    dispatch_storage(c->storage, false, [&](auto st, auto) -> int {
        using S = typename decltype(st)::type;
        hipLaunchKernelGGL((k_check_finite<S>), dim3(blocks), dim3(256), 0, c->stream,
                           (const uint4 *)c->buf[c->cur], nvec, c->t, c->d_bad);
        return PTRT_OK;
    });
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->h_bad, c->d_bad, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipEventRecord(c->bad_event, c->stream));
    c->bad_pending = true;
    return PTRT_OK;
}

// Enqueue n steps: graph replays where captured, else launches.
int advance(ptrt_ctx *c, int n)
{
    if (c->use_graph)
        while (n >= GRAPH_STEPS) {
            if (!c->graph[c->cur]) {
                int rc = capture_graph(c, c->cur);
                if (rc != PTRT_OK) return rc;
            }
            HIPCHK(c, hipGraphLaunch(c->graph[c->cur], c->stream));
            n -= GRAPH_STEPS;
        }
    launch_steps(c, c->stream, n);
    return PTRT_OK;
}

} // namespace

extern "C" {

int ptrt_create(int lattice, int nx, int ny, int nz, double tau_plus, double Lambda,
                const double *force, const uint8_t *solid_mask, ptrt_ctx **out)
{
    if (!out) {
        g_create_error = "out is NULL";
        return PTRT_EINVAL;
    }
    *out = nullptr;
    std::string msg;
    int rc = check_params(lattice, nx, ny, nz, tau_plus, Lambda, force, msg);
    if (rc == PTRT_OK) rc = check_layout(lattice_q(lattice), nx, ny, nz, storage_bytes(PTRT_F32), msg);
    if (rc != PTRT_OK) {
        g_create_error = msg;
        return rc;
    }
    ptrt_ctx *c = new (std::nothrow) ptrt_ctx();
    if (!c) {
        g_create_error = "out of host memory";
        return PTRT_ENOMEM;
    }
    c->lattice = lattice;
    c->Q = lattice_q(lattice);
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->N = (long long)nx * ny * nz;
    c->tau_plus = tau_plus;
    c->Lambda = Lambda;
    if (force)
        for (int a = 0; a < 3; ++a) c->g[a] = force[a];
    if (lattice == PTRT_D2Q9) c->g[2] = 0.0;
    c->row_kernel = c->ny <= 65535 && c->nz <= 65535;
    if (solid_mask) {
        c->h_mask.assign(solid_mask, solid_mask + c->N);
        for (auto &v : c->h_mask) v = v ? 1 : 0;
        c->has_mask = std::any_of(c->h_mask.begin(), c->h_mask.end(), [](uint8_t v) { return v; });
        if (!c->has_mask) c->h_mask.clear();
    }
    *out = c;
    return PTRT_OK;
}

int ptrt_set_storage(ptrt_ctx *c, int storage)
{
    if (!c) return PTRT_EINVAL;
    if (storage_bytes(storage) == 0) return fail(c, PTRT_EINVAL, "unknown storage type");
    if (c->allocated) return fail(c, PTRT_ESTATE, "storage can only change before the first init");
    std::string msg;
    if (check_layout(c->Q, c->nx, c->ny, c->nz, storage_bytes(storage), msg) != PTRT_OK)
        return fail(c, PTRT_EINVAL, msg);
    c->storage = storage;
    return PTRT_OK;
}

int ptrt_set_model(ptrt_ctx *c, int model)
{
    if (!c) return PTRT_EINVAL;
    if (model != MODEL_PTRT && model != MODEL_TRT_RLB && model != MODEL_TRT &&
        model != MODEL_PTRT_EXACT)
        return fail(c, PTRT_EINVAL, "unknown collision model");
    if (model != MODEL_PTRT && !c->row_kernel)
        return fail(c, PTRT_EINVAL, "comparison models need ny and nz <= 65535");
    if (c->forcing != FORCE_II && model != MODEL_PTRT && model != MODEL_PTRT_EXACT)
        return fail(c, PTRT_EINVAL, "the comparison models use the default forcing only");
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail_hip(c, PTRT_EDEVICE, "stream synchronisation failed");
    c->model = model;
    drop_graphs(c);
    return PTRT_OK;
}

int ptrt_set_open_x(ptrt_ctx *c, double u_in, double rho_out)
{
    if (!c) return PTRT_EINVAL;
    if (c->lattice != PTRT_D2Q9) return fail(c, PTRT_EINVAL, "open boundaries are built for D2Q9");
    if (c->nx < 2) return fail(c, PTRT_EINVAL, "open boundaries need nx >= 2");
    if (!c->row_kernel) return fail(c, PTRT_EINVAL, "open boundaries need ny <= 65535");
    if (!std::isfinite(u_in) || !std::isfinite(rho_out) || !(rho_out > 0.0))
        return fail(c, PTRT_EINVAL, "u_in must be finite and rho_out finite and positive");
    if (c->forcing == FORCE_II_G)
        return fail(c, PTRT_EINVAL, "the cubic correction needs periodic x");
    if (c->allocated) return fail(c, PTRT_ESTATE, "open boundaries can only be set before the first init");
    c->open = true;
    c->geo.uin = u_in;
    c->geo.drhoout = rho_out - 1.0;
    return PTRT_OK;
}

int ptrt_momentum_exchange(ptrt_ctx *c, double force_out[3])
{
    if (!c || !force_out) return PTRT_EINVAL;
    if (!c->initialized || c->t == 0)
        return fail(c, PTRT_ESTATE, "momentum exchange needs a completed step");
    for (int a = 0; a < 3; ++a) force_out[a] = 0.0;
    if (!c->has_mask) return PTRT_OK;
    if (!c->d_force_parts)
        HIPCHK(c, hipMalloc(&c->d_force_parts, 3 * sizeof(double) * momentum_parts(c)));
    if (!c->d_force) HIPCHK(c, hipMalloc(&c->d_force, 3 * sizeof(double)));
    return momentum_exchange_with(c, c->d_force_parts, c->d_force, force_out);
}

int ptrt_momentum_exchange_noalloc(ptrt_ctx *c, double force_out[3])
{
    if (!c || !force_out) return PTRT_EINVAL;
    const size_t need = NOALLOC_PARTS_OFFSET + 3 * sizeof(double) * momentum_parts(c);
    if (c->has_mask && need > NOALLOC_SCRATCH_BYTES)
        return fail(c, PTRT_EINVAL,
                    "lattice too large for the fixed scratch of ptrt_momentum_exchange_noalloc: "
                    "needs " + std::to_string(need) + " bytes, holds " +
                        std::to_string(NOALLOC_SCRATCH_BYTES) +
                        " (one 64 x 4 node block per 24 bytes); use ptrt_momentum_exchange");
    if (!c->initialized || c->t == 0)
        return fail(c, PTRT_ESTATE, "momentum exchange needs a completed step");
    for (int a = 0; a < 3; ++a) force_out[a] = 0.0;
    if (!c->has_mask) return PTRT_OK;
    char *base = nullptr;
    const int rc = noalloc_scratch(c, &base);
    if (rc != PTRT_OK) return rc;
    return momentum_exchange_with(c, reinterpret_cast<double *>(base + NOALLOC_PARTS_OFFSET),
                                  reinterpret_cast<double *>(base), force_out);
}

int ptrt_last_pass(const ptrt_ctx *c, int *steps, double *bytes)
{
    if (!c || !steps || !bytes) return PTRT_EINVAL;
    *steps = c->last_pass_steps;
    *bytes = c->last_pass_bytes;
    return PTRT_OK;
}

int ptrt_set_steps_per_pass(ptrt_ctx *c, int steps)
{
    if (!c) return PTRT_EINVAL;
    if (steps != 1 && steps != 2) return fail(c, PTRT_EINVAL, "steps per pass must be 1 or 2");
    if (c->allocated && hipStreamSynchronize(c->stream) != hipSuccess)
        return fail_hip(c, PTRT_EDEVICE, "stream synchronisation failed");
    c->steps_per_pass = steps;
    drop_graphs(c);
    return PTRT_OK;
}

int ptrt_set_forcing(ptrt_ctx *c, int forcing)
{
    if (!c) return PTRT_EINVAL;
    if (forcing != FORCE_II && forcing != FORCE_II_G && forcing != FORCE_GUO)
        return fail(c, PTRT_EINVAL, "unknown forcing scheme");
    if (forcing == FORCE_II_G && c->open)
        return fail(c, PTRT_EINVAL, "the cubic correction needs periodic x");
    if (forcing != FORCE_II && c->model != MODEL_PTRT && c->model != MODEL_PTRT_EXACT)
        return fail(c, PTRT_EINVAL, "the comparison models use the default forcing only");
    if (forcing != FORCE_II && !c->row_kernel)
        return fail(c, PTRT_EINVAL, "forcing variants need ny and nz <= 65535");
    if (c->allocated && hipStreamSynchronize(c->stream) != hipSuccess)
        return fail_hip(c, PTRT_EDEVICE, "stream synchronisation failed");
    const int rc = ensure_phi(c, forcing);
    if (rc != PTRT_OK) return rc; // scheme unchanged
    c->forcing = forcing;
    drop_graphs(c);
    return PTRT_OK;
}

int ptrt_set_stream(ptrt_ctx *c, void *s)
{
    if (!c) return PTRT_EINVAL;
    c->stream = (hipStream_t)s;
    return PTRT_OK;
}

int ptrt_init_equilibrium(ptrt_ctx *c, const double *rho, const double *u)
{
    if (!c) return PTRT_EINVAL;
    int rc = ensure_allocated(c);
    if (rc != PTRT_OK) return rc;
    rc = upload_state(c, rho, u, nullptr);
    if (rc != PTRT_OK) return rc;
    c->initialized = true;
    c->t = 0;
    return reset_check(c);
}

int ptrt_set_populations(ptrt_ctx *c, const double *f)
{
    if (!c || !f) return fail(c, PTRT_EINVAL, "NULL argument");
    int rc = ensure_allocated(c);
    if (rc != PTRT_OK) return rc;
    rc = upload_state(c, nullptr, nullptr, f);
    if (rc != PTRT_OK) return rc;
    c->initialized = true;
    return reset_check(c);
}

int ptrt_step(ptrt_ctx *c, int n)
{
    if (!c) return PTRT_EINVAL;
    if (n < 0) return fail(c, PTRT_EINVAL, "negative step count");
    if (!c->initialized) return fail(c, PTRT_ESTATE, "ptrt_step before init");
    if (c->forcing == FORCE_II_G && !c->d_phi)
        return fail(c, PTRT_ESTATE, "no Phi field for the cubic correction");
    if (c->check_every > 0) {
        poll_check(c);
        if (c->diverged_at >= 0)
            return fail(c, PTRT_EDIVERGED,
                        "the divergence check found a non-finite population at step " +
                            std::to_string(c->diverged_at) + "; no steps enqueued");
    }
    while (n > 0) {
        int m = n;
        if (c->check_every > 0)
            m = (int)std::min<long long>(n, c->check_every - c->t % c->check_every);
        int rc = advance(c, m);
        if (rc != PTRT_OK) return rc;
        c->t += m;
        n -= m;
        if (c->check_every > 0 && c->t % c->check_every == 0) {
            rc = launch_check(c);
            if (rc != PTRT_OK) return rc;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(c, PTRT_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    return PTRT_OK;
}

int ptrt_moments(ptrt_ctx *c, double *rho_out, double *u_out)
{
    if (!c) return PTRT_EINVAL;
    if (!c->initialized) return fail(c, PTRT_ESTATE, "moments before init");
    return download_state(c, rho_out, u_out, nullptr);
}

int ptrt_get_populations(ptrt_ctx *c, double *f_out)
{
    if (!c || !f_out) return fail(c, PTRT_EINVAL, "NULL argument");
    if (!c->initialized) return fail(c, PTRT_ESTATE, "get_populations before init");
    return download_state(c, nullptr, nullptr, f_out);
}

int ptrt_diagnostics(ptrt_ctx *c, double *mass, double *ke)
{
    if (!c) return PTRT_EINVAL;
    if (!c->initialized) return fail(c, PTRT_ESTATE, "diagnostics before init");
    const Geom g = geom(c);
    const void *src = c->buf[c->cur];
    const dim3 grid = gather_grid(c, c->nz), block(BLK_X, BLK_Y, 1);
    dispatch(c->lattice, c->storage, c->has_mask, [&](auto lt, auto st, auto mk) -> int {
        using L = typename decltype(lt)::type;
        using S = typename decltype(st)::type;
        constexpr bool M = decltype(mk)::value;
        with_open<L>(c, [&](auto oc) {
            constexpr bool O = decltype(oc)::value;
            hipLaunchKernelGGL((k_gather<L, S, M, O>), grid, block, 0, c->stream, (const S *)src,
                               c->d_mask, g, 0, c->g[0], c->g[1], c->g[2], (double *)nullptr,
                               (double *)nullptr, (double *)nullptr, 0LL, c->d_partials);
        });
        return PTRT_OK;
    });
    hipLaunchKernelGGL(k_finalize<1024>, dim3(1), dim3(1024), 0, c->stream, c->d_partials, c->nparts, c->d_red);
    HIPCHK(c, hipGetLastError());
    double r[2];
    HIPCHK(c, hipMemcpyAsync(r, c->d_red, sizeof(r), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (mass) *mass = r[0];
    if (ke) *ke = r[1];
    if (!std::isfinite(r[0]) || !std::isfinite(r[1]))
        return fail(c, PTRT_EDIVERGED, "non-finite mass or kinetic energy at step " + std::to_string(c->t));
    return PTRT_OK;
}

int ptrt_set_divergence_check(ptrt_ctx *c, int every)
{
    if (!c) return PTRT_EINVAL;
    if (every < 0) return fail(c, PTRT_EINVAL, "the check interval must be >= 0");
    // each part allocated once (a failed attempt leaves the others for the next)
    if (every > 0 && !c->d_bad) HIPCHK(c, hipMalloc(&c->d_bad, sizeof(unsigned long long)));
    if (every > 0 && !c->h_bad)
        HIPCHK(c, hipHostMalloc((void **)&c->h_bad, sizeof(unsigned long long), hipHostMallocDefault));
    if (every > 0 && !c->bad_event) HIPCHK(c, hipEventCreateWithFlags(&c->bad_event, hipEventDisableTiming));
    const int rc = reset_check(c);
    if (rc != PTRT_OK) return rc;
    c->check_every = every;
    return PTRT_OK;
}

int ptrt_divergence_step(ptrt_ctx *c, long long *step)
{
    if (!c || !step) return PTRT_EINVAL;
    *step = -1;
    if (!c->d_bad) return PTRT_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unsigned long long v = NO_STEP;
    HIPCHK(c, hipMemcpy(&v, c->d_bad, sizeof(v), hipMemcpyDeviceToHost));
    c->bad_pending = false;
    if (v != NO_STEP) c->diverged_at = (long long)v;
    *step = c->diverged_at;
    return PTRT_OK;
}

int ptrt_get_time(const ptrt_ctx *c, long long *t)
{
    if (!c || !t) return PTRT_EINVAL;
    *t = c->t;
    return PTRT_OK;
}

const char *ptrt_last_error(const ptrt_ctx *c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

int ptrt_destroy(ptrt_ctx *c)
{
    if (!c) return PTRT_OK;
    hipError_t e = hipSuccess;
    if (c->allocated) e = hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k)
        if (c->buf[k]) (void)hipFree(c->buf[k]);
    if (c->d_mask) (void)hipFree(c->d_mask);
    if (c->d_near) (void)hipFree(c->d_near);
    if (c->d_tasks) (void)hipFree(c->d_tasks);
    for (auto &gx : c->graph)
        if (gx) (void)hipGraphExecDestroy(gx);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_red) (void)hipFree(c->d_red);
    if (c->d_phi) (void)hipFree(c->d_phi);
    if (c->d_force_parts) (void)hipFree(c->d_force_parts);
    if (c->d_force) (void)hipFree(c->d_force);
    if (c->d_bad) (void)hipFree(c->d_bad);
    if (c->h_bad) (void)hipHostFree(c->h_bad);
    if (c->bad_event) (void)hipEventDestroy(c->bad_event);
    delete c;
    return e == hipSuccess ? PTRT_OK : PTRT_EDEVICE;
}

int ptrt_velocity_set(int lattice, int *e_out, double *w_out)
{
    auto fill = [&](auto lt) {
        using L = typename decltype(lt)::type;
        for (int i = 0; i < L::Q; ++i) {
            if (e_out) {
                e_out[3 * i] = L::ex(i);
                e_out[3 * i + 1] = L::ey(i);
                e_out[3 * i + 2] = L::ez(i);
            }
            if (w_out) w_out[i] = L::w(i);
        }
        return L::Q;
    };
    if (lattice == PTRT_D2Q9) return fill(Tag<D2Q9>{});
    if (lattice == PTRT_D3Q19) return fill(Tag<D3Q19>{});
    if (lattice == PTRT_D3Q27) return fill(Tag<D3Q27>{});
    return PTRT_EINVAL;
}

double ptrt_bytes_per_node(const ptrt_ctx *c)
{
    if (!c) return 0.0;
    return 2.0 * c->Q * (double)storage_bytes(c->storage) + (c->has_mask ? 1.0 : 0.0);
}

} // extern "C"
