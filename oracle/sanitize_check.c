/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A driver that calls every entry point of the oracle (lbm_oracle.h) on small
 * lattices of every kind it supports -- periodic and walled axes, wetting
 * walls, lattices one and two nodes wide, the Allen-Cahn and Cahn-Hilliard
 * phase fields, the three models and the local gradient scheme, states saved
 * and reloaded -- so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py) sees every loop and
 * index of the oracle run.  Exits 0 when every call returned its expected
 * status and every value it read back is finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

static int failures = 0;

static void expect(int cond, const char *what, int nx, int ny) {
    if (!cond) {
        fprintf(stderr, "FAIL %s (%d x %d)\n", what, nx, ny);
        failures++;
    }
}

static int all_finite(const double *a, long n) {
    for (long i = 0; i < n; i++)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static orc_params base(int nx, int ny, int wall_x, int wall_y) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.wall_x = wall_x;
    p.wall_y = wall_y;
    p.phiA = 1.0;
    p.phiB = 0.0;
    p.rhoA = 10.0;
    p.rhoB = 1.0;
    p.nuA = 0.05;
    p.nuB = 0.1;
    p.sigma = 0.01;
    p.W = 4.0;
    p.M = 0.05;
    p.eta = 1.0;
    p.gy = -1e-5;
    p.Gx = 1e-6;
    p.rho_ref = 5.0;
    p.theta[0] = 1.2;
    p.theta[1] = 1.9;
    p.theta[2] = 0.8;
    p.theta[3] = 2.2;
    p.eps = 1e-4;
    return p;
}

static void run(orc_params p, const char *name) {
    const int nx = p.nx, ny = p.ny;
    const long n = (long)nx * ny;
    double *phi0 = malloc(sizeof(double) * n), *u0 = malloc(sizeof(double) * 2 * n), *p0 = malloc(sizeof(double) * n);
    double *phi = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * 2 * n), *pr = malloc(sizeof(double) * n);
    double *f = malloc(sizeof(double) * 9 * n), *g = malloc(sizeof(double) * 9 * n), *H = malloc(sizeof(double) * 5 * n);
    double *pp = malloc(sizeof(double) * n), *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
    double *c = malloc(sizeof(double) * n), *m = malloc(sizeof(double) * 2 * n);
    const double lo = p.pf ? -1.0 : 0.0;
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            const long k = (long)y * nx + x;
            const double s = 0.5 + 0.4 * sin(0.7 * x + 0.3) * cos(0.5 * y + 0.1);
            phi0[k] = lo + (1.0 - lo) * s;
            u0[k] = 1e-3 * sin(0.9 * y);
            u0[n + k] = 1e-3 * cos(1.1 * x);
        }
    if (p.gx == 0.0) expect(orc_hydrostatic_pressure(&p, phi0, p0) == 0, "hydrostatic", nx, ny);
    else expect(orc_hydrostatic_pressure(&p, phi0, p0) == -8, "hydrostatic refuses gx", nx, ny);
    for (long k = 0; k < n; k++) p0[k] = 1e-4 * sin(0.2 * k);

    orc_sim *s = orc_create(&p);
    expect(s != NULL, name, nx, ny);
    if (!s) return;
    expect(orc_init(s, phi0, u0, p0) == 0, "init", nx, ny);
    expect(orc_step(s, 7) == 0, "step", nx, ny);
    expect(orc_moments(s, phi, u, pr) == 0 && all_finite(phi, n) && all_finite(u, 2 * n) && all_finite(pr, n),
           "moments", nx, ny);
    double out[6];
    expect(orc_diagnostics(s, out) == 0 && all_finite(out, 6), "diagnostics", nx, ny);
    expect(orc_div_fields(s, a, b) == 0 && all_finite(a, n), "div fields", nx, ny);
    expect(orc_div_fields(s, NULL, b) == 0, "div fields, one output", nx, ny);
    long step = -1;
    expect(orc_get_state(s, f, g, H, pp, &step) == 0 && step == 7 && all_finite(f, 9 * n) && all_finite(g, 9 * n),
           "get state", nx, ny);
    expect(orc_get_state(s, NULL, NULL, NULL, NULL, NULL) == 0, "get state, no outputs", nx, ny);
    double sf[9], sg[9];
    expect(orc_rates(s, sf, sg) == 0, "rates", nx, ny);
    expect(orc_grad(s, a, b) == 0 && all_finite(a, n) && all_finite(b, n), "grad", nx, ny);
    expect(orc_flux(s, a, b) == 0 && all_finite(a, n), "flux", nx, ny);
    expect(orc_fa(s, a) == 0 && all_finite(a, n), "fa", nx, ny);
    expect(orc_stencils(s, phi, a, b, c) == 0 && all_finite(c, n), "stencils", nx, ny);

    /* reload the saved state into a second simulation and continue both */
    orc_sim *t = orc_create(&p);
    if (p.grad == 1) {
        /* the local scheme needs m^phiC of the previous level: the flux of level step - 1 */
        orc_sim *r = orc_create(&p);
        orc_init(r, phi0, u0, p0);
        orc_step(r, 6);
        orc_flux(r, m, m + n);
        double *up = malloc(sizeof(double) * 2 * n), *php = malloc(sizeof(double) * n);
        orc_moments(r, php, up, NULL);
        orc_step(r, 1);
        double *fr = malloc(sizeof(double) * 9 * n), *gr = malloc(sizeof(double) * 9 * n);
        orc_get_state(r, fr, gr, NULL, NULL, NULL);
        expect(orc_set_state(t, fr, gr, php, up, 7) == -8, "set state refuses the local scheme", nx, ny);
        expect(orc_set_state_m(t, fr, gr, php, up, m, 7) == 0, "set state with m", nx, ny);
        orc_destroy(r);
        free(up);
        free(php);
        free(fr);
        free(gr);
    } else {
        orc_moments(s, phi, u, pr);
        expect(orc_set_state(t, f, g, pp, u, 7) == 0, "set state", nx, ny);
        expect(orc_set_state(t, f, g, NULL, NULL, 0) == 0, "set state at level 0", nx, ny);
        expect(orc_set_state(t, f, g, pp, u, 7) == 0, "set state again", nx, ny);
    }
    expect(orc_step(t, 3) == 0, "step after reload", nx, ny);
    expect(orc_moments(t, phi, u, NULL) == 0 && all_finite(phi, n), "moments after reload", nx, ny);
    orc_destroy(t);
    orc_destroy(s);
    free(phi0);
    free(u0);
    free(p0);
    free(phi);
    free(u);
    free(pr);
    free(f);
    free(g);
    free(H);
    free(pp);
    free(a);
    free(b);
    free(c);
    free(m);
}

int main(void) {
    orc_set_threads(2);
    const int shapes[][4] = {{1, 1, 0, 0}, {1, 7, 0, 1}, {7, 1, 1, 0}, {2, 2, 1, 1}, {2, 5, 1, 0},
                             {9, 6, 0, 0}, {9, 6, 1, 1}, {13, 11, 0, 1}};
    for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; i++) {
        orc_params p = base(shapes[i][0], shapes[i][1], shapes[i][2], shapes[i][3]);
        run(p, "present");
        orc_params q = p;
        q.model = 1;
        q.visc_law = 1;
        run(q, "original, inverse-linear viscosity");
        q = p;
        q.grad = 1;
        run(q, "local gradient");
        q = p;
        q.pf = 1;
        q.phiB = -1.0;
        run(q, "Cahn-Hilliard");
        q.model = 2;
        run(q, "corrected, Cahn-Hilliard");
        q = p;
        q.gx = 1e-6;
        for (int k = 0; k < 9; k++) q.sf[k] = q.sg[k] = 1.1;
        run(q, "general rates, gx");
    }
    int cx[9], cy[9];
    double w[9], M[81], Minv[81], meq[9], mR[9], mF[9], fo[9], S[9], fv[9], geq[9], Fi[9];
    orc_lattice(cx, cy, w, M, Minv);
    orc_params p = base(8, 8, 1, 1);
    double pw, pg;
    orc_wetting(&p, 1.0, 0.8, 0.6, &pw, &pg);
    orc_moments_f(&p, 0.4, 1e-3, -2e-3, 0.01, 0.02, 1e-5, 2e-5, meq, mR);
    for (int k = 0; k < 9; k++) {
        S[k] = 0.6 + 0.1 * k;
        fv[k] = w[k] * 0.4;
    }
    orc_collide_node(S, fv, meq, mR, fo);
    orc_moments_f_ch(&p, 0.4, 1e-3, 1e-3, -2e-3, 1e-5, 2e-5, meq, mR);
    orc_moments_g(&p, 3.0, 1e-4, 1e-3, -2e-3, 0.01, 0.02, 1e-5, 2e-5, 0.1, 0.2, 1e-6, 2e-6, 3e-6, meq, mF);
    orc_direct_g(&p, 3.0, 1e-4, 1e-3, -2e-3, 0.01, 0.02, 1e-5, 2e-5, 0.1, 0.2, 1e-6, 2e-6, 3e-6, geq, Fi);
    expect(isfinite(pw) && isfinite(pg) && all_finite(fo, 9) && all_finite(geq, 9) && all_finite(Fi, 9),
           "building blocks", 8, 8);
    expect(orc_num_threads() >= 1, "threads", 0, 0);
    if (failures) {
        fprintf(stderr, "%d failure(s)\n", failures);
        return 1;
    }
    printf("sanitize_check: every oracle entry point ran clean\n");
    return 0;
}
