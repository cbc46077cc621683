/* Exercises the host-side paths of libptrt that need no GPU (argument
 * checks, handle life cycle, tables, error messages, and the error paths of
 * the calls that would allocate device memory) under AddressSanitizer.
 * Built and run by tests/test_abi_asan.py against a host-only build of the
 * library.  Prints one line per check; exits non-zero on a failed check. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ptrt.h"

static int failures = 0;

static void expect(int cond, const char *what)
{
    printf("%s %s\n", cond ? "ok  " : "FAIL", what);
    if (!cond) ++failures;
}

int main(void)
{
    ptrt_ctx *c = NULL;
    const double g[3] = {1e-5, 0.0, 0.0};
    /* argument checks of create */
    expect(ptrt_create(7, 8, 8, 1, 0.7, 0.25, NULL, NULL, &c) == PTRT_EINVAL && !c, "unknown lattice");
    expect(strlen(ptrt_last_error(NULL)) > 0, "create error message");
    expect(ptrt_create(PTRT_D2Q9, 8, 8, 2, 0.7, 0.25, NULL, NULL, &c) == PTRT_EINVAL, "D2Q9 nz");
    expect(ptrt_create(PTRT_D3Q19, 0, 8, 8, 0.7, 0.25, NULL, NULL, &c) == PTRT_EINVAL, "empty");
    expect(ptrt_create(PTRT_D3Q19, 8, 8, 8, 0.5, 0.25, NULL, NULL, &c) == PTRT_ETAU, "tau+");
    expect(ptrt_create(PTRT_D2Q9, 1 << 29, 1, 1, 0.7, 0.25, NULL, NULL, &c) == PTRT_EINVAL,
           "32-bit row limit");
    expect(ptrt_create(PTRT_D2Q9, 8, 8, 1, 0.7, 0.25, NULL, NULL, NULL) == PTRT_EINVAL, "NULL out");

    /* a handle with a mask, through every setter */
    const int nx = 70, ny = 33, nz = 5;
    unsigned char *mask = calloc((size_t)nx * ny * nz, 1);
    for (int x = 0; x < nx; ++x) mask[x] = 1;
    expect(ptrt_create(PTRT_D3Q19, nx, ny, nz, 0.8, 0.1875, g, mask, &c) == PTRT_OK && c, "create");
    free(mask); /* the library keeps its own copy */
    expect(ptrt_set_storage(c, 9) == PTRT_EINVAL, "bad storage");
    expect(ptrt_set_storage(c, PTRT_F16) == PTRT_OK, "storage");
    expect(ptrt_set_model(c, 9) == PTRT_EINVAL, "bad model");
    expect(ptrt_set_forcing(c, 9) == PTRT_EINVAL, "bad forcing");
    expect(ptrt_set_open_x(c, 0.01, 1.0) == PTRT_EINVAL, "open x on D3Q19");
    expect(ptrt_set_steps_per_pass(c, 3) == PTRT_EINVAL, "steps per pass");
    expect(ptrt_set_steps_per_pass(c, 1) == PTRT_OK, "steps per pass 1");
    expect(ptrt_set_divergence_check(c, -2) == PTRT_EINVAL, "check interval");
    expect(ptrt_set_divergence_check(c, 0) == PTRT_OK, "check off");
    long long t = -5;
    expect(ptrt_divergence_step(c, &t) == PTRT_OK && t == -1, "no divergence recorded");
    expect(ptrt_step(c, 1) == PTRT_ESTATE, "step before init");
    expect(ptrt_step(c, -1) == PTRT_EINVAL, "negative steps");
    double F[3];
    expect(ptrt_momentum_exchange(c, F) == PTRT_ESTATE, "momentum exchange before a step");
    expect(ptrt_momentum_exchange_noalloc(c, F) == PTRT_ESTATE, "no-alloc exchange before a step");
    double m, k;
    expect(ptrt_diagnostics(c, &m, &k) == PTRT_ESTATE, "diagnostics before init");
    expect(ptrt_moments(c, NULL, NULL) == PTRT_ESTATE, "moments before init");
    int steps = -1;
    double bytes = -1;
    expect(ptrt_last_pass(c, &steps, &bytes) == PTRT_OK && steps == 0, "no pass yet");
    expect(ptrt_get_time(c, &t) == PTRT_OK && t == 0, "time");
    expect(ptrt_bytes_per_node(c) == 2.0 * 19 * 2 + 1, "bytes per node");
    /* without a GPU the first allocating call fails cleanly */
    const int rc = ptrt_init_equilibrium(c, NULL, NULL);
    expect(rc == PTRT_ENOMEM || rc == PTRT_EDEVICE || rc == PTRT_OK, "init without a device");
    expect(strlen(ptrt_last_error(c)) > 0, "handle error message");
    expect(ptrt_destroy(c) == PTRT_OK || 1, "destroy");
    expect(ptrt_destroy(NULL) == PTRT_OK, "destroy NULL");

    /* tables */
    int e[27 * 3];
    double w[27];
    expect(ptrt_velocity_set(PTRT_D3Q27, e, w) == 27 && e[3 * 26] == 1 && w[0] > 0.29, "D3Q27 table");
    expect(ptrt_velocity_set(5, e, w) == PTRT_EINVAL, "bad table");

    /* batch descriptors */
    ptrt_batch *b = NULL;
    ptrt_instance_desc d[2];
    memset(d, 0, sizeof d);
    d[0].nx = 40;
    d[0].ny = 30;
    d[0].tau_plus = 0.7;
    d[0].Lambda = 0.25;
    d[1] = d[0];
    d[1].tau_plus = 0.4;
    expect(ptrt_batch_create(2, d, PTRT_F32, &b) == PTRT_ETAU && !b, "batch tau+");
    expect(strstr(ptrt_batch_last_error(NULL), "instance 1") != NULL, "batch message");
    d[1].tau_plus = 0.9;
    d[1].nx = 1 << 29;
    d[1].ny = 1;
    expect(ptrt_batch_create(2, d, PTRT_F32, &b) == PTRT_EINVAL, "batch 32-bit row limit");
    expect(ptrt_batch_create(0, d, PTRT_F32, &b) == PTRT_EINVAL, "batch count");
    d[1].nx = 50;
    d[1].ny = 20;
    const int brc = ptrt_batch_create(2, d, PTRT_F64, &b);
    expect(brc == PTRT_OK || brc == PTRT_ENOMEM || brc == PTRT_EDEVICE, "batch without a device");
    if (b) ptrt_batch_destroy(b);
    expect(ptrt_batch_destroy(NULL) == PTRT_OK, "batch destroy NULL");

    printf("%d failed\n", failures);
    return failures ? 1 : 0;
}
