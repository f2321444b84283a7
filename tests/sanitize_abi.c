/*
 * sanitize_abi.c -- the host side of the C ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_sanitizers.py
 * against a copy of the library whose host code carries the sanitizers).
 *
 * Every call below returns before any HIP call: the size queries of the state,
 * tape and adjoint buffers for lattices of every kind (their layout
 * arithmetic), the parameter validation of every entry point (invalid sizes,
 * physical parameters, rates, models, null pointers, misaligned buffers), the
 * batch plan's host checks, the two-level rule and the status strings.  Exits
 * 0 when every status is the expected one.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/lbm.h"

static int failures = 0;

#define EXPECT(call, want)                                                                         \
    do {                                                                                           \
        const int got_ = (call);                                                                   \
        if (got_ != (want)) {                                                                      \
            fprintf(stderr, "FAIL line %d: %s = %d, expected %d\n", __LINE__, #call, got_, (want)); \
            failures++;                                                                            \
        }                                                                                          \
    } while (0)

static lbm_params base(int nx, int ny, int dtype) {
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.dtype = dtype;
    p.phi_A = 1.0;
    p.phi_B = 0.0;
    p.rho_A = 10.0;
    p.rho_B = 1.0;
    p.nu_A = p.nu_B = 0.1;
    p.sigma = 0.01;
    p.W = 4.0;
    p.M_phi = 0.02;
    p.eta = 1.0;
    for (int k = 0; k < 4; k++) p.theta[k] = 1.5707963267948966;
    p.eps_n = 1e-4;
    return p;
}

int main(void) {
    void* fake = (void*)(uintptr_t)(1 << 20);   /* never dereferenced: every call returns before using it */
    size_t n = 0;
    int32_t lv = -1;

    /* size queries on lattices of every kind */
    const int shapes[][4] = {{1, 1, 0, 0}, {2, 2, 1, 1}, {64, 64, 0, 0}, {65, 7, 1, 0}, {256, 1024, 0, 1},
                             {4096, 4096, 0, 1}, {51200, 1024, 0, 0}};
    for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; i++)
        for (int dt = 0; dt < 2; dt++)
            for (int v = 0; v < 4; v++) {
                lbm_params p = base(shapes[i][0], shapes[i][1], dt);
                p.bc_x = shapes[i][2];
                p.bc_y = shapes[i][3];
                if (v == 1) p.grad_scheme = LBM_GRAD_LOCAL;
                if (v == 2) {
                    p.phase_eq = LBM_CAHN_HILLIARD;
                    p.phi_B = -1.0;
                }
                if (v == 3) p.model = LBM_MODEL_CORRECTED;
                EXPECT(lbm_state_size(&p, &n), LBM_OK);
                if (n % 256 || n < (size_t)p.nx * p.ny) {
                    fprintf(stderr, "FAIL state size %zu\n", n);
                    failures++;
                }
                EXPECT(lbm_levels_per_launch(&p, &lv), LBM_OK);
                if (v == 0) {
                    EXPECT(lbm_tape_size(&p, 3, &n), LBM_OK);
                    EXPECT(lbm_adjoint_size(&p, &n), LBM_OK);
                } else {
                    EXPECT(lbm_adjoint_size(&p, &n), LBM_E_UNSUPPORTED);
                }
            }

    /* parameter validation */
    lbm_params p = base(64, 64, LBM_F32);
    lbm_params q;
    q = p; q.nx = 0; EXPECT(lbm_state_size(&q, &n), LBM_E_SIZE);
    q = p; q.ny = -3; EXPECT(lbm_state_size(&q, &n), LBM_E_SIZE);
    q = p; q.nx = 1; q.bc_x = LBM_WALLS; EXPECT(lbm_state_size(&q, &n), LBM_E_SIZE);
    q = p; q.dtype = 7; EXPECT(lbm_state_size(&q, &n), LBM_E_DTYPE);
    q = p; q.rho_A = 0.0; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.nu_B = -1.0; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.W = 0.0; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.eta = 0.5; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.phi_A = 0.0; q.phi_B = 1.0; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.theta[0] = 0.0; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.sigma = NAN; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.s_g[0] = 2.0; EXPECT(lbm_state_size(&q, &n), LBM_E_UNSTABLE);
    q = p; q.s_f[3] = 2.5; EXPECT(lbm_state_size(&q, &n), LBM_E_UNSTABLE);
    q = p; q.model = 9; EXPECT(lbm_state_size(&q, &n), LBM_E_UNSUPPORTED);
    q = p; q.phase_eq = 9; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.grad_scheme = 9; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.reserved = 1; EXPECT(lbm_state_size(&q, &n), LBM_E_PARAM);
    q = p; q.grad_scheme = LBM_GRAD_LOCAL; q.model = LBM_MODEL_CORRECTED; EXPECT(lbm_state_size(&q, &n), LBM_E_UNSUPPORTED);

    /* null pointers, sizes and alignment of the state calls */
    EXPECT(lbm_state_size(NULL, &n), LBM_E_NULL);
    EXPECT(lbm_state_size(&p, NULL), LBM_E_NULL);
    EXPECT(lbm_init(&p, NULL, NULL, NULL, NULL, NULL), LBM_E_NULL);
    EXPECT(lbm_init(&p, (void*)(uintptr_t)300, fake, NULL, NULL, NULL), LBM_E_SIZE);
    EXPECT(lbm_step(&p, NULL, 1, NULL), LBM_E_NULL);
    EXPECT(lbm_step(&p, fake, -1, NULL), LBM_E_SIZE);
    EXPECT(lbm_moments(&p, NULL, NULL, NULL, NULL, NULL), LBM_E_NULL);
    EXPECT(lbm_diagnostics(&p, NULL, NULL, NULL), LBM_E_NULL);
    EXPECT(lbm_export_state(&p, NULL, NULL, NULL, NULL, NULL, NULL), LBM_E_NULL);
    EXPECT(lbm_import_state(&p, fake, fake, fake, NULL, 3, NULL), LBM_E_NULL);
    EXPECT(lbm_import_state(&p, fake, fake, fake, fake, -1, NULL), LBM_E_SIZE);
    EXPECT(lbm_hydrostatic_pressure(&p, NULL, fake, NULL), LBM_E_NULL);
    q = p; q.gravity[0] = 1e-6; EXPECT(lbm_hydrostatic_pressure(&q, fake, fake, NULL), LBM_E_UNSUPPORTED);
    EXPECT(lbm_levels_per_launch(NULL, &lv), LBM_E_NULL);
    EXPECT(lbm_levels_per_launch(&p, NULL), LBM_E_NULL);

    /* reverse mode: host checks */
    EXPECT(lbm_tape_size(&p, 0, &n), LBM_E_SIZE);
    EXPECT(lbm_tape_size(&p, 2, NULL), LBM_E_NULL);
    EXPECT(lbm_tape_record(&p, fake, fake, 0, NULL), LBM_E_SIZE);
    EXPECT(lbm_tape_restore(&p, fake, 0, NULL, NULL), LBM_E_NULL);
    EXPECT(lbm_tape_restore(&p, (void*)(uintptr_t)((1 << 20) + 8), 0, fake, NULL), LBM_E_SIZE);
    EXPECT(lbm_adjoint_step(&p, fake, -1, fake, NULL), LBM_E_SIZE);
    EXPECT(lbm_adjoint_run(&p, fake, 0, 2, fake, NULL), LBM_E_SIZE);
    EXPECT(lbm_adjoint_phi(&p, NULL, fake, fake, NULL), LBM_E_NULL);
    EXPECT(lbm_adjoint_phi(&p, fake, (void*)(uintptr_t)((1 << 20) + 8), fake, NULL), LBM_E_SIZE);
    EXPECT(lbm_adjoint_init(&p, NULL, fake, NULL), LBM_E_NULL);
    EXPECT(lbm_adjoint_params(&p, fake, NULL, NULL, NULL), LBM_E_NULL);
    EXPECT(lbm_adjoint_import(&p, fake, NULL, NULL, NULL, -1, NULL), LBM_E_SIZE);
    EXPECT(lbm_adjoint_export(&p, NULL, NULL, NULL, NULL, NULL), LBM_E_NULL);
    q = p; q.phase_eq = LBM_CAHN_HILLIARD; q.phi_B = -1.0;
    EXPECT(lbm_tape_record(&q, fake, fake, 1, NULL), LBM_E_UNSUPPORTED);
    EXPECT(lbm_tape_restore(&q, fake, 0, fake, NULL), LBM_E_UNSUPPORTED);
    EXPECT(lbm_adjoint_run(&q, fake, 0, 1, fake, NULL), LBM_E_UNSUPPORTED);

    /* batches: host checks (a valid plan needs a device table, so none is made) */
    lbm_batch* b = NULL;
    lbm_params two[2] = {p, p};
    EXPECT(lbm_batch_create(NULL, 1, 0, &b), LBM_E_NULL);
    EXPECT(lbm_batch_create(two, 1, 0, NULL), LBM_E_NULL);
    EXPECT(lbm_batch_create(two, 0, 0, &b), LBM_E_SIZE);
    two[1].dtype = LBM_F64;
    EXPECT(lbm_batch_create(two, 2, 0, &b), LBM_E_DTYPE);
    two[1] = p;
    two[1].W = -1.0;
    EXPECT(lbm_batch_create(two, 2, 0, &b), LBM_E_PARAM);
    two[1] = base(51200, 1024, LBM_F32);   /* a case copy of 4 GiB and more: beyond 32-bit offsets */
    EXPECT(lbm_batch_create(two, 2, 0, &b), LBM_E_SIZE);
    EXPECT(lbm_batch_state_size(NULL, &n), LBM_E_NULL);
    EXPECT(lbm_batch_step(NULL, NULL, 1, NULL), LBM_E_NULL);
    EXPECT(lbm_batch_destroy(NULL), LBM_E_NULL);
    EXPECT(lbm_batch_levels_per_launch(NULL, &lv), LBM_E_NULL);
    lbm_params* many = (lbm_params*)malloc(sizeof(lbm_params) * 257);
    for (int c = 0; c < 257; c++) many[c] = p;
    EXPECT(lbm_batch_step_noalloc(many, 257, fake, 1, NULL), LBM_E_SIZE);
    EXPECT(lbm_batch_step_noalloc(many, 1, fake, -1, NULL), LBM_E_SIZE);
    EXPECT(lbm_batch_step_noalloc(many, 1, (void*)(uintptr_t)((1 << 20) + 8), 1, NULL), LBM_E_SIZE);
    EXPECT(lbm_batch_step_noalloc(NULL, 1, fake, 1, NULL), LBM_E_NULL);
    EXPECT(lbm_batch_step_noalloc(many, 1, fake, 0, NULL), LBM_OK);
    free(many);

    /* the streaming probe */
    EXPECT(lbm_bandwidth_probe(3, fake, fake, 1 << 20, 256, 1, NULL), LBM_E_PARAM);
    EXPECT(lbm_bandwidth_probe(2, fake, fake, (1 << 20) + 8, 256, 1, NULL), LBM_E_SIZE);
    EXPECT(lbm_bandwidth_probe(2, fake, NULL, 1 << 20, 256, 1, NULL), LBM_E_NULL);

    for (int c = -9; c <= 0; c++)
        if (!lbm_status_string(c)) failures++;
    if (failures) {
        fprintf(stderr, "%d failure(s)\n", failures);
        return 1;
    }
    printf("sanitize_abi: every host check ran clean\n");
    return 0;
}
