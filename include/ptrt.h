/*
 * ptrt.h -- C interface of libptrt, the MI355X (gfx950) implementation of the
 * Purified two-relaxation-time (P-TRT) lattice Boltzmann update of
 * arXiv 2602.06686 ("Purified Two-Relaxation-Time Lattice Boltzmann Method:
 * Removing Ghost Modes from TRT for Enhanced Stability").
 *
 * One call of ptrt_step advances a lattice by the fused per-node update of
 * Eq. PTRT: pull-streaming with halfway bounce-back at solid links (Sec. 3.3),
 * density and half-force velocity (Eq. macro), the third-order Hermite
 * equilibrium (Eq. feq), the parity split of the non-equilibrium part
 * (Eq. fneq_parity), algebraic removal of the ghost modes (Theorem 2,
 * Eq. ghost_proj; one mode on D2Q9, three on D3Q19), and relaxation with the
 * two rates tau+ and tau- plus the body-force terms (Theorem 3, Eq. R3_force).
 * The net force source is (1/2) w_i e_i.F / c_s^2 (the first-order moment is
 * relaxed with tau+, as in the sentence after Eq. TRT-RLB), so each step adds
 * exactly F to the momentum.  The cubic correction G_i of Eq. Gi is not
 * applied.  F = rho g with a constant acceleration g (Sec. 3.3).
 *
 * Parameters: tau+ is the symmetric (viscous) relaxation time,
 * nu = (tau+ - 1/2)/3 (Eq. viscosity); tau- follows from the magic parameter
 * Lambda = (tau+ - 1/2)(tau- - 1/2) (Sec. 3.2).  Lattice units throughout
 * (dx = dt = 1, c_s^2 = 1/3).
 *
 * Conventions shared by every call
 * --------------------------------
 * Host arrays (all double, caller-owned, C order):
 *   density      rho[nz][ny][nx]
 *   velocity     u[3][nz][ny][nx]      (component-major; u[2] ignored on D2Q9)
 *   populations  f[Q][nz][ny][nx]      (direction-major, unshifted f_i)
 *   solid mask   uint8 [nz][ny][nx], 1 = solid, 0 = fluid
 * The library copies what it needs during the call and keeps no caller
 * pointer.  Device memory is owned by the library and freed by destroy.
 *
 * Velocity order (also returned by ptrt_velocity_set):
 *   D2Q9  (Eq. D2Q9, printed order): (0,0) (1,0) (0,1) (-1,0) (0,-1)
 *         (1,1) (-1,1) (-1,-1) (1,-1)
 *   D3Q19 (App. A.2; order and weights 1/3, 1/18, 1/36 chosen here):
 *         rest; +x -x +y -y +z -z; (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0);
 *         (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1); (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *   D3Q27 (App. A.3; weights 8/27, 2/27, 1/54, 1/216): the D3Q19 order, then
 *         (1,1,1) (-1,-1,-1) (1,1,-1) (-1,-1,1) (1,-1,1) (-1,1,-1) (-1,1,1) (1,-1,-1)
 *
 * Time: the state is "populations at integer time t, before collision".
 * ptrt_init_equilibrium sets f(t=0) = f^eq(rho, u) and t = 0; ptrt_step(n)
 * advances t by n; moments, diagnostics and get_populations report the state
 * at the current t.  Because u includes half the force (Eq. macro), the
 * velocity reported at t = 0 is u_init + g/2.
 *
 * Storage: populations are kept on the GPU as shifted values
 * f_i - w_i (reference density 1) in the storage type chosen with
 * ptrt_set_storage: FP64 (FP64 arithmetic), FP32, FP16 or BF16 (FP32
 * arithmetic; FP16/BF16 round to nearest even on store, or stochastically
 * in their _SR variants).
 *
 * Streams: work is enqueued on the stream given to ptrt_set_stream (default:
 * the null stream).  ptrt_step is asynchronous; the calls that return host
 * data synchronise that stream.  Work already enqueued on an earlier stream
 * is not waited for when the stream changes: the caller orders the two.
 *
 * Errors: every int-returning call returns PTRT_OK (0) or a negative code and
 * leaves a message readable with ptrt_last_error.  A handle is not
 * thread-safe; distinct handles are independent.  Sizes are limited to
 * nx*ny*nz < 2^31 nodes per lattice, and the rows to Q * pitch < 2^32
 * elements, pitch = nx rounded up to whole 128-byte lines of the storage
 * type (the kernels form offsets inside a row tile in 32 bits):
 * ptrt_create (checked for FP32), ptrt_set_storage and ptrt_batch_create
 * return PTRT_EINVAL for longer rows.
 */
#ifndef PTRT_H
#define PTRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ptrt_ctx ptrt_ctx;
typedef struct ptrt_batch ptrt_batch;

enum ptrt_lattice { PTRT_D2Q9 = 0, PTRT_D3Q19 = 1, PTRT_D3Q27 = 2 };

/* Storage of the populations as shifted values h_i = f_i - w_i (the
 * collision arithmetic is FP32 for the 16-bit types, FP64 for PTRT_F64).
 * PTRT_F16 / PTRT_BF16 round each store to nearest even.  PTRT_F16_SR /
 * PTRT_BF16_SR keep the same 16-bit formats but round each store of a step
 * stochastically (up with the probability given by the value's position
 * between its two neighbours; the random bits are a hash of the value, so
 * runs are reproducible), which keeps small per-step changes from being lost
 * systematically on fine lattices; the initial state and
 * ptrt_set_populations still round to nearest. */
enum ptrt_storage {
    PTRT_F64 = 0,
    PTRT_F32 = 1,
    PTRT_F16 = 2,
    PTRT_BF16 = 3,
    PTRT_F16_SR = 4,
    PTRT_BF16_SR = 5
};

/* Collision model of ptrt_step: P-TRT (the method, Eq. PTRT) or, for
 * comparison, TRT-RLB (Eq. TRT-RLB: Hermite projection of the
 * non-equilibrium part, Eq. R2R3_hermite, with tau+ also on the first-order
 * moment and the Scheme II source without G_i; on D3Q19 the third-order
 * reconstruction is the orthogonal projection onto the third-order modes)
 * or standard TRT (P-TRT without the ghost subtraction: the ghost modes
 * relax with tau+, Eq. collision_TRT).  All three share the state layout,
 * the streaming and the force convention.
 *
 * On D3Q27 P-TRT is the paper's hybrid (Eq. PTRT_D3Q27): R2 by the Hermite
 * stress projection, R3 by the antisymmetric part, which keeps the three
 * fifth-order antisymmetric modes; PTRT_MODEL_PTRT_EXACT projects those out
 * as well (App. A.3), which equals TRT-RLB.  On D2Q9 and D3Q19
 * PTRT_MODEL_PTRT_EXACT is the same as PTRT_MODEL_PTRT. */
/* Forcing schemes (Sec. 2.1), all with F = rho * force and the half-force
 * velocity of Eq. macro:
 *   PTRT_FORCING_SCHEME2    Scheme II (Eq. source_simple) without the cubic
 *                           correction; the first-order non-equilibrium
 *                           moment relaxes with tau+, which leaves the net
 *                           source (1/2) w_i e_i.F / c_s^2 in Eq. PTRT and a
 *                           momentum gain of exactly F per step (default);
 *   PTRT_FORCING_SCHEME2_G  the same plus G_i of Eq. Gi, with
 *                           Phi_aaa = rho u_a^3 (a = x, y and, in 3D, z),
 *                           d_a Phi_aaa by central differences with
 *                           periodic wrap, Phi = 0 at solid nodes; each step
 *                           runs a Phi pass before the fused step;
 *   PTRT_FORCING_GUO        Scheme I (Eq. source_guo) with its -u.F/c_s^2
 *                           part under the tau+ factor (as printed it sits
 *                           under the tau- factor and does not conserve
 *                           mass); the tau- bracket then holds f^neq,- alone. */
enum ptrt_forcing {
    PTRT_FORCING_SCHEME2 = 0,
    PTRT_FORCING_SCHEME2_G = 1,
    PTRT_FORCING_GUO = 2
};

enum ptrt_model {
    PTRT_MODEL_PTRT = 0,
    PTRT_MODEL_TRT_RLB = 1,
    PTRT_MODEL_TRT = 2,
    PTRT_MODEL_PTRT_EXACT = 3
};

enum ptrt_status {
    PTRT_OK = 0,
    PTRT_EINVAL = -1,    /* bad lattice id, size, pointer or argument */
    PTRT_ETAU = -2,      /* tau+ <= 1/2, Lambda <= 0, or a non-finite parameter */
    PTRT_ENOMEM = -3,    /* device allocation failed */
    PTRT_EDEVICE = -4,   /* a HIP call failed (no GPU, launch error, ...) */
    PTRT_EDIVERGED = -5, /* non-finite mass, energy or populations (diagnostics, divergence check) */
    PTRT_ESTATE = -6     /* call not valid in the handle's current state */
};

/* ------------------------------------------------------------------------
 * Single lattice
 * ------------------------------------------------------------------------ */

/* Create a lattice of nx*ny*nz nodes (nz must be 1 for D2Q9) with
 * relaxation time tau_plus > 1/2 and magic parameter Lambda > 0 (Sec. 3.2),
 * acceleration force[3] (NULL = none; force[2] ignored on D2Q9) and an
 * optional solid mask (NULL = all fluid).  Boundaries are periodic in every
 * direction; walls are made of solid nodes.  Storage defaults to FP32.
 * Device memory is allocated by ptrt_init_equilibrium / ptrt_set_populations.
 * On failure *out is NULL and the message is in ptrt_last_error(NULL). */
int ptrt_create(int lattice, int nx, int ny, int nz, double tau_plus, double Lambda,
                const double *force, const uint8_t *solid_mask, ptrt_ctx **out);

/* Choose the storage type (enum ptrt_storage).  Only before the first init
 * or set_populations; PTRT_ESTATE afterwards. */
int ptrt_set_storage(ptrt_ctx *ctx, int storage);

/* Select the collision model (enum ptrt_model) for later steps; allowed at
 * any time (waits for the handle's stream).  The comparison models need
 * ny <= 65535 and nz <= 65535, and run with PTRT_FORCING_SCHEME2 only
 * (PTRT_EINVAL otherwise).  Default PTRT_MODEL_PTRT. */
int ptrt_set_model(ptrt_ctx *ctx, int model);

/* Select the forcing scheme (enum ptrt_forcing) for later steps; allowed at
 * any time (waits for the handle's stream).  The variants other than
 * PTRT_FORCING_SCHEME2 need model PTRT_MODEL_PTRT or PTRT_MODEL_PTRT_EXACT
 * and ny, nz <= 65535 (PTRT_EINVAL otherwise).  PTRT_FORCING_SCHEME2_G
 * allocates the Phi field (D values per node in the compute type: FP64 for
 * FP64 storage, FP32 otherwise), owned by the handle; PTRT_ENOMEM if that
 * fails.  Default PTRT_FORCING_SCHEME2. */
int ptrt_set_forcing(ptrt_ctx *ctx, int forcing);

/* Steps per pass over the populations (1 or 2; default 2).  With 2, pairs
 * of steps run as one kernel that keeps the first step's results in LDS
 * (temporal blocking) where the configuration allows it and it measured
 * faster: PTRT_FORCING_SCHEME2 with PTRT_MODEL_PTRT (or, without solid
 * nodes or open x, PTRT_MODEL_TRT_RLB or PTRT_MODEL_TRT), and either D3Q19 in
 * FP32 or FP64 with nx a multiple of 64 and ny >= 4 (with solid nodes:
 * from 2^24 nodes on, while at most 5 % of the kernel's column chunks have
 * a solid within one row), or D2Q9 in FP32 or FP64 (with solid nodes or
 * open x: from 2^20 nodes on, while at most 30 % of the rows lie in row
 * chunks with a solid within one row); every other case, and an odd last
 * step, runs one step per pass.  Results are bit-identical either way.
 * Allowed at any time (waits for the handle's stream). */
int ptrt_set_steps_per_pass(ptrt_ctx *ctx, int steps);

/* The most recent kernel pass enqueued by ptrt_step: *steps = the steps it
 * covers (1 or 2; 0 before any step) and *bytes = its algorithmic HBM
 * traffic in bytes (one step: 2 Q s per node, plus one mask byte per node
 * with solids; two steps: also 2 Q s per node, the state read once by the
 * first step and written once by the second).  For bandwidth accounting;
 * no synchronisation. */
int ptrt_last_pass(const ptrt_ctx *ctx, int *steps, double *bytes);

/* Open boundaries in x instead of periodic x (Sec. 3.4, creeping flow past
 * a square cylinder; D2Q9 only).  Inlet: a halfway bounce-back wall at
 * x = -1/2 moving with velocity (u_in, 0) and density rho_0 = 1; a
 * population leaving node x = 0 through it returns as
 * f_ibar = f*_i - 2 w_i rho_0 e_i.u_w / c_s^2.  Outlet: the Zou-He pressure
 * condition at x = nx - 1 with density rho_out and u_y = 0 sets the three
 * populations entering through it; populations leaving through it are
 * dropped.  y stays periodic; solid nodes still bounce back.  Only before
 * the first init or set_populations (PTRT_ESTATE afterwards); needs nx >= 2,
 * ny <= 65535, finite u_in, finite rho_out > 0, and a forcing other than
 * PTRT_FORCING_SCHEME2_G (PTRT_EINVAL otherwise).  With open boundaries the
 * populations set at the outlet's entering slots are not stored (every
 * step computes them), so ptrt_get_populations returns the Zou-He values
 * there. */
int ptrt_set_open_x(ptrt_ctx *ctx, double u_in, double rho_out);

/* Momentum-exchange force on all solid nodes (Eq. Fx), from the
 * post-collision state of the last completed step (time t - 1):
 * force_out[3] = sum over fluid nodes x_f and directions i with x_f + e_i
 * solid of 2 e_i f*_i(x_f) (halfway bounce-back returns the population that
 * left, so f*_ibar(x_s) = f*_i(x_f)), in lattice units, FP64.  Links
 * through open boundaries are not counted.  Zeros without solid nodes.
 * PTRT_ESTATE before the first step.  Synchronises the handle's stream; the
 * first call allocates a small reduction buffer owned by the handle. */
int ptrt_momentum_exchange(ptrt_ctx *ctx, double force_out[3]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * force as ptrt_momentum_exchange, from the same kernels in the same order
 * (bit-identical results), with the per-block partials and the result in a
 * fixed 16 MiB device array of the library instead of buffers it allocates.
 * Calls no hipMalloc or hipFree.  The array holds 3 doubles per 64 x 4
 * block of nodes (nx/64 x ny/4 x nz blocks, rounded up) after 256 bytes for
 * the result: up to 699040 blocks (a 512^3 lattice needs 524288);
 * PTRT_EINVAL for larger lattices.  Every call on a GPU uses that GPU's one
 * array (held until the process ends), so calls that overlap on one GPU,
 * from any handle or thread, race; each call overwrites all it reads.
 * Synchronises the handle's stream; PTRT_ESTATE before the first step. */
int ptrt_momentum_exchange_noalloc(ptrt_ctx *ctx, double force_out[3]);

/* Stream for all later work of this handle; a hipStream_t passed as void*
 * (e.g. torch.cuda.current_stream().cuda_stream).  NULL = null stream. */
int ptrt_set_stream(ptrt_ctx *ctx, void *hip_stream);

/* f(t=0) = f^eq(rho, u) at every fluid node (Eq. feq), computed on the GPU in
 * FP64 and rounded to the storage type.  rho NULL = 1 everywhere, u NULL = 0.
 * Resets the step counter to 0.  Synchronous. */
int ptrt_init_equilibrium(ptrt_ctx *ctx, const double *rho, const double *u);

/* Enqueue n >= 0 fused P-TRT steps (Eq. PTRT).  Asynchronous. */
int ptrt_step(ptrt_ctx *ctx, int n);

/* Density and half-force velocity (Eq. macro) of the state at the current
 * time, into caller arrays rho[nz][ny][nx] and u[3][nz][ny][nx] (either may
 * be NULL).  Solid nodes report 0.  Synchronous. */
int ptrt_moments(ptrt_ctx *ctx, double *rho_out, double *u_out);

/* Mass sum(rho) and kinetic energy (1/2) sum(rho |u|^2) over fluid nodes,
 * reduced on the GPU in FP64.  Returns PTRT_EDIVERGED (with the values
 * still written) if either is not finite.  Synchronous. */
int ptrt_diagnostics(ptrt_ctx *ctx, double *mass, double *kinetic_energy);

/* Copy the populations f[Q][nz][ny][nx] at the current time to the host
 * (unshifted, FP64; solid nodes report 0).  Synchronous.  Together with
 * ptrt_set_populations and ptrt_get_time this is a checkpoint. */
int ptrt_get_populations(ptrt_ctx *ctx, double *f_out);

/* Replace the state by f[Q][nz][ny][nx] (unshifted; values at solid nodes
 * are ignored), rounded to the storage type.  Keeps the step counter.
 * Synchronous. */
int ptrt_set_populations(ptrt_ctx *ctx, const double *f_in);

/* Number of steps taken since the last init. */
int ptrt_get_time(const ptrt_ctx *ctx, long long *t_out);

/* Divergence detection (the stability criterion of Sec. 3.1: a run counts
 * as stable while it stays finite).  With every > 0, ptrt_step checks the
 * state after each step whose count t is a multiple of `every`: a kernel
 * scans the whole population buffer for NaN or infinity and keeps, on the
 * device, the earliest such t; the result is copied to pinned host memory
 * behind the steps, without a wait.  A later ptrt_step that sees a recorded
 * step returns PTRT_EDIVERGED (message with the step) and enqueues nothing.
 * The check reads the state once (half the traffic of a step); an even
 * `every` keeps two steps per pass.  every = 0 turns it off.  Enabling it
 * allocates 8 bytes of device memory and 8 of pinned host memory, owned by
 * the handle.  Resets any recorded step (waits for the handle's stream);
 * ptrt_init_equilibrium and ptrt_set_populations reset it too. */
int ptrt_set_divergence_check(ptrt_ctx *ctx, int every);

/* Earliest checked step at which the state was not finite, or -1 if none
 * (or the check was never enabled), after all enqueued work has finished.
 * Synchronises the handle's stream. */
int ptrt_divergence_step(ptrt_ctx *ctx, long long *step_out);

/* Message of the last failed call on ctx; with ctx == NULL, of the last
 * failed ptrt_create on this thread.  Never NULL. */
const char *ptrt_last_error(const ptrt_ctx *ctx);

/* Free the handle and its device memory.  NULL is a no-op. */
int ptrt_destroy(ptrt_ctx *ctx);

/* Host-only table query: writes the Q velocities e[Q][3] and weights w[Q]
 * of a lattice in the order used by every population array (either pointer
 * may be NULL) and returns Q, or PTRT_EINVAL. */
int ptrt_velocity_set(int lattice, int *e_out, double *w_out);

/* Bytes of HBM traffic one node update moves (2 Q times the storage size,
 * plus 1 for the mask when the lattice has one): the algorithmic traffic
 * used for roofline figures. */
double ptrt_bytes_per_node(const ptrt_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batched form: many independent D2Q9 lattices of different sizes, each with
 * its own tau+, Lambda, force and mask, advanced together.  Each instance
 * computes exactly what a single lattice with the same parameters computes,
 * bit for bit.
 * ------------------------------------------------------------------------ */

typedef struct {
    int nx, ny;                  /* lattice size (nz = 1) */
    double tau_plus, Lambda;     /* as for ptrt_create */
    double force[3];             /* acceleration g; force[2] ignored */
    const uint8_t *solid_mask;   /* [ny][nx] or NULL; copied during the call */
} ptrt_instance_desc;

/* Create a batch of count D2Q9 instances in one device allocation with the
 * given storage type.  Every instance starts at rest (rho = 1, u = 0). */
int ptrt_batch_create(int count, const ptrt_instance_desc *desc, int storage,
                      ptrt_batch **out);

int ptrt_batch_set_stream(ptrt_batch *b, void *hip_stream);

/* Set instance k to f^eq(rho, u) (NULL = rest); synchronous. */
int ptrt_batch_init_equilibrium(ptrt_batch *b, int instance, const double *rho,
                                 const double *u);

/* Tile plan of the fused launch: workgroups of tile_x * tile_y threads
 * (64, 128, 256, 512 or 1024 threads; tile_x a multiple of 32, and of 64
 * when tile_y == 1) walking a table of tiles; `blocks` workgroups (0 = one
 * workgroup per tile; otherwise each workgroup takes every blocks-th tile).
 * With tile_y == 1 a tile is a tile_x-node segment of one row, or, for rows
 * narrower than the workgroup, as many whole rows (each rounded up to a
 * multiple of 64 nodes) as fit; with tile_y > 1 it is a tile_x x tile_y
 * block.  xcd_order != 0 orders the tile table so that the workgroups the
 * hardware sends to one of the eight accelerator dies (XCDs, round-robin by
 * workgroup index) get neighbouring tiles, which then share that die's L2.
 * Rebuilds the tile table and drops any captured graph. */
int ptrt_batch_set_plan(ptrt_batch *b, int tile_x, int tile_y, int blocks, int xcd_order);

/* Two-step plan of ptrt_batch_step (steps per pass 2, FP32 / FP64 storage;
 * PTRT_ESTATE for FP16 / BF16, which have no two-step pass): the task
 * table cuts every instance into strips of 62 columns and chunks of `rows`
 * rows (1 ... 64); a chunk with a solid within one row of its rows takes the
 * masked code, its rows in chunks of `masked_rows` (1 ... 64).  One wave
 * runs one task; `waves` (2, 4 or 8) waves per workgroup; `blocks` = 0
 * launches one wave per task, else `blocks` workgroups whose waves take
 * every (blocks x waves)-th task (persistent).  The tasks without solids
 * near and the masked ones are two launches; `concurrent` != 0 puts the
 * masked launch on a second stream of the batch beside the other (two
 * branches of the captured graph) instead of after it.  Every plan
 * computes the same values bit for bit.  Rebuilds the task table and drops
 * captured graphs; waits for the batch's stream. */
int ptrt_batch_set_plan2(ptrt_batch *b, int rows, int masked_rows, int waves, int blocks,
                         int concurrent);

/* The current two-step plan: plan_out[5] = {rows, masked_rows, waves,
 * blocks, concurrent} as for ptrt_batch_set_plan2. */
int ptrt_batch_get_plan2(const ptrt_batch *b, int plan_out[5]);

/* Time candidate plans on the device and keep the fastest.  The one-step
 * tile plans (10 tile shapes x grids 0, 2048, 4096 x table or XCD order)
 * are written to the pointers if not NULL.  With FP32 / FP64 storage the
 * two-step plan is searched as well (rows 1, 2, 3, 5, 7 x masked rows 1,
 * 2, 3 and, above 3, = rows x waves 2, 4, 8 x one wave per task or the
 * resident grid x masked launch after or beside the other, each timed over
 * ten passes, the five fastest again three times, the best median kept;
 * read it with ptrt_batch_get_plan2).  The trial steps run on the current
 * state, which is saved beforehand and restored afterwards, so the batch
 * is left as it was.  Needs one extra state-sized device buffer for the
 * duration of the call.  Synchronous. */
int ptrt_batch_autotune(ptrt_batch *b, int *tile_x, int *tile_y, int *blocks, int *xcd_order);

/* Enqueue n steps over every instance, replayed from captured HIP graphs
 * of ten steps: pairs of steps as two-step passes (below), else one launch
 * per step over every instance with the current tile plan.  Asynchronous. */
int ptrt_batch_step(ptrt_batch *b, int n);

/* Steps per pass of ptrt_batch_step (1 or 2; default 2).  With 2 and FP32
 * or FP64 storage, pairs of steps run as passes of the two-step kernel of
 * ptrt_set_steps_per_pass (first step kept in LDS) over a task table of
 * (instance, 62-column strip, chunk of rows): one launch for the chunks
 * with no solid within one row and one for the others (halfway
 * bounce-back), as ptrt_batch_set_plan2 describes; FP16 / BF16 storage and
 * an odd last step take one step per pass.  Results are bit-identical
 * either way.  The tile plan (set_plan) applies to the one-step launches.
 * Waits for the batch's stream. */
int ptrt_batch_set_steps_per_pass(ptrt_batch *b, int steps);

/* The most recent pass enqueued by ptrt_batch_step: *steps = the steps it
 * covers (1 or 2; 0 before any) and *bytes = its algorithmic HBM traffic,
 * (2 Q s + 1) bytes per node for either kind (state read once and written
 * once, mask bytes).  PTRT_EINVAL on NULL pointers. */
int ptrt_batch_last_pass(const ptrt_batch *b, int *steps, double *bytes);

/* Enqueue n steps as one launch per instance per step (the comparison
 * baseline for the fused launch).  Asynchronous. */
int ptrt_batch_step_separate(ptrt_batch *b, int n);

/* Moments and populations of one instance, layouts as for a single lattice
 * with nz = 1.  Synchronous. */
int ptrt_batch_moments(ptrt_batch *b, int instance, double *rho_out, double *u_out);
int ptrt_batch_get_populations(ptrt_batch *b, int instance, double *f_out);

/* Mass and kinetic energy of every instance (arrays of count doubles),
 * FP64 reduction on the GPU.  Returns PTRT_EDIVERGED if any is not finite. */
int ptrt_batch_diagnostics(ptrt_batch *b, double *mass, double *kinetic_energy);

/* Total node count of the batch (solid included) and the algorithmic bytes
 * one step moves. */
long long ptrt_batch_nodes(const ptrt_batch *b);
double ptrt_batch_bytes_per_step(const ptrt_batch *b);

/* As ptrt_last_error; with b == NULL, the last failed ptrt_batch_create on
 * this thread. */
const char *ptrt_batch_last_error(const ptrt_batch *b);
int ptrt_batch_destroy(ptrt_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* PTRT_H */
