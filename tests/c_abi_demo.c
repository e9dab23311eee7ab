/* c_abi_demo.c -- a plain C11 caller of the library: no HIP headers, no
 * device buffers.  It anneals one 6x6 Shastry-Sutherland instance (J1 = 1,
 * J2 = 0.5, h = 0, 64 chains, linear T 3.0 -> 0.1 over 300 sweeps),
 * accumulates the last 100 sweeps and prints the exact int64 sums, so a test
 * can compare them with the CPU oracle.  Usage: c_abi_demo <seed> */
#include <inttypes.h>
#include <stdio.h>
#include <stdlib.h>

#include "crbm.h"

int main(int argc, char** argv)
{
    const uint64_t seed = argc > 1 ? strtoull(argv[1], NULL, 0) : 1u;
    crbm_instance inst = {0};
    inst.L = 6;
    inst.periodic = 1;
    inst.J1 = 1.0;
    inst.J2 = 0.5;
    inst.h = 0.0;
    inst.n_chains = 64;
    inst.sched_kind = CRBM_SCHED_LINEAR;
    inst.T0 = 3.0;
    inst.T1 = 0.1;
    inst.T_explicit = NULL;
    inst.id = 2;
    crbm_config cfg = {0};
    cfg.seed = seed;
    cfg.n_sweeps = 300;
    cfg.measure_every = 1;
    cfg.burn_in = 200;
    cfg.stream = NULL;
    crbm_t* h = NULL;
    int rc = crbm_create(&inst, 1, &cfg, &h);
    if (rc != CRBM_OK) {
        fprintf(stderr, "crbm_create: %d %s\n", rc, crbm_last_error());
        return 1;
    }
    if ((rc = crbm_sample(h, 300, NULL, NULL)) != CRBM_OK) {
        fprintf(stderr, "crbm_sample: %d %s\n", rc, crbm_last_error());
        return 1;
    }
    crbm_obs o;
    if ((rc = crbm_observables(h, &o, NULL)) != CRBM_OK) {
        fprintf(stderr, "crbm_observables: %d %s\n", rc, crbm_last_error());
        return 1;
    }
    /* the same handle refuses to run past its schedule */
    const int past = crbm_sample(h, 1, NULL, NULL);
    printf("%" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64
           " %" PRId64 " %" PRId64 " %" PRId64 " %d %.12f\n",
           o.n_samples, o.sum_M, o.sum_B1, o.sum_B2, o.sum_MM, o.sum_B1B1, o.sum_B2B2, o.sum_MB1, o.sum_MB2,
           o.sum_B1B2, o.sum_absM, past, o.E_per_spin);
    crbm_destroy(h);
    return 0;
}
