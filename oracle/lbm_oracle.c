/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).
 *
 * A deliberately plain FP64 implementation: every stage of a time step runs
 * over the whole lattice and stores its result in a full field before the
 * next stage starts, the collision is done literally in moment space with the
 * matrix M1 of App. C and its numerically computed inverse, and streaming is
 * a push with half-way bounce-back.  No blocking or fusion.
 *
 * Order of one step (the paper has no algorithm box; this is the order in
 * which Sec. 3 defines the quantities):
 *   1. phi = sum_i f_i                                   (Sec. 3, macroscopic quantities)
 *   2. ghost layer: periodic wrap or wetting ghosts      (Eq. Dwetting)
 *   3. grad phi, lap phi                                 (Eqs. central1, central2)
 *   4. closure: mu_phi, rho, grad rho, n, lambda, m^phiC, F, nu
 *                                                        (Sec. 2: Eqs. for mu_phi, lambda, rho-phi,
 *                                                         linearMu / inverseNu, m^CC; Sec. 3 force F)
 *   5. u from Eq. comU                                   (F does not depend on u)
 *   6. Euler time derivatives of the history products    (App. C, explicit Euler)
 *   7. p from Eq. computP, second way of Remark 1 (H, J, K of App. C)
 *   8. f collision in moment space (Eq. evoPF, Eq. MfMRAC1)
 *   9. g collision in moment space (Remark 2, Eq. MgMF1)
 *  10. history <- current products
 *  11. streaming with half-way bounce-back (Sec. 4 preamble)
 * Options: the Cahn-Hilliard phase field replaces the AC flux by the one of
 * Eq. CHE and the f moments by Eq. MfMRCH1 (after step 4, ch_flux); the
 * corrected comparison model adds F_a = a u and solves step 5 with it
 * (ch_flux / ac_corrected_force); the local gradient scheme replaces step 3's
 * grad phi of levels >= 1 by Eq. local (local_gradient).
 *
 * Pins (tests/test_oracle_*.py): every stage above against a closed form, a
 * textbook identity or the paper's printed values, including the CH moments,
 * the corrected model's F_a (periodic closed forms) and the local gradient
 * (tanh derivative); the wall rules that the paper leaves open -- the mirror
 * of mu_phi at walls (Cahn-Hilliard) and the mirror of D with reversed normal
 * component (corrected AC model) -- by the no-flux property they stand for
 * (sum of F_a's coefficient over a walled lattice is zero); the diagnostics
 * (Sec. 4.1) by the expansion Eq. strainRate comes from (its trace on a
 * compressive wave) and by S_m = rho div u at equal densities and its
 * second-order fall for a carried, relaxing interface
 * (tests/test_oracle_diagnostics.py).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocities ordered as the columns of M1 (rows 3 and 5 of M1 are c_x and c_y). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Standard D2Q9 weights; the paper does not print them, they are the ones
 * that give cs^2 = c^2/3 (App. C). */
static const double WT[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double CS2 = 1.0 / 3.0;

/* Eq. (M1) of App. C. */
static const double M1[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

struct orc_sim {
    orc_params P;
    int nx, ny;
    long n;             /* nodes */
    long step;
    double Minv[9][9];
    double sf[9], sg[9];
    int snu_local;      /* s_g^7 = s_g^8 follow nu(phi) */
    double *f, *g;      /* [9][n] post-streaming at the current level */
    double *fs, *gs;    /* [9][n] post-collision scratch */
    double *H;          /* [5][n] history products of the previous level */
    double *phi_prev;   /* [n] */
    /* per-step scratch fields */
    double *phi, *ext, *gx, *gy, *lap;
    double *rho, *mu, *lam, *nxv, *nyv, *mx, *my, *Fx, *Fy, *snu;
    double *ux, *uy, *pr, *P5, *dP5;
    double *muext;      /* (nx+2) x (ny+2) mu with its ghost layer (Cahn-Hilliard) */
    double *fa;         /* [n] corrected model: F_a = fa u */
    double *dxv, *dyv;  /* [n] corrected AC model: D = grad phi - lambda n */
    double *dext;       /* (nx+2) x (ny+2) second extended field (corrected AC model) */
};

/* ------------------------------------------------------------------ */
/* Gauss-Jordan inverse with partial pivoting (generic, no use of the
 * orthogonality of M1). */
static int invert9(const double A[9][9], double R[9][9]) {
    double a[9][18];
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 18; j++) a[i][j] = j < 9 ? A[i][j] : (j - 9 == i ? 1.0 : 0.0);
    for (int c = 0; c < 9; c++) {
        int piv = c;
        for (int r = c + 1; r < 9; r++)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (fabs(a[piv][c]) < 1e-300) return -1;
        if (piv != c)
            for (int j = 0; j < 18; j++) {
                double t = a[c][j];
                a[c][j] = a[piv][j];
                a[piv][j] = t;
            }
        double d = a[c][c];
        for (int j = 0; j < 18; j++) a[c][j] /= d;
        for (int r = 0; r < 9; r++)
            if (r != c) {
                double m = a[r][c];
                for (int j = 0; j < 18; j++) a[r][j] -= m * a[c][j];
            }
    }
    for (int i = 0; i < 9; i++)
        for (int j = 0; j < 9; j++) R[i][j] = a[i][j + 9];
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

void orc_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}

void orc_lattice(int cx[9], int cy[9], double w[9], double M[81], double Minv[81]) {
    double R[9][9];
    invert9(M1, R);
    for (int i = 0; i < 9; i++) {
        if (cx) cx[i] = CX[i];
        if (cy) cy[i] = CY[i];
        if (w) w[i] = WT[i];
        for (int j = 0; j < 9; j++) {
            if (M) M[i * 9 + j] = M1[i][j];
            if (Minv) Minv[i * 9 + j] = R[i][j];
        }
    }
}

/* ------------------------------------------------------------------ */
static int opposite(int i) {
    for (int j = 0; j < 9; j++)
        if (CX[j] == -CX[i] && CY[j] == -CY[i]) return j;
    return -1;
}

static int check_params(const orc_params *p) {
    if (p->nx < 1 || p->ny < 1) return -2;
    if (p->wall_x && p->nx < 2) return -2;
    if (p->wall_y && p->ny < 2) return -2;
    if (!(p->phiA > p->phiB)) return -4;
    if (!(p->rhoA > 0 && p->rhoB > 0 && p->nuA > 0 && p->nuB > 0)) return -4;
    if (!(p->W > 0 && p->sigma >= 0 && p->M >= 0)) return -4;
    if (p->eta != 1.0) return -4;
    if (p->pf != 0 && p->pf != 1) return -4;
    if (p->model != 0 && p->model != 1 && p->model != 2) return -8;
    if (p->grad != 0 && p->grad != 1) return -4;
    if (p->grad == 1 && (p->pf != 0 || p->model == 2)) return -8;
    if (p->visc_law != 0 && p->visc_law != 1) return -4;
    for (int i = 0; i < 9; i++)
        if (p->sf[i] >= 2.0 || p->sg[i] >= 2.0) return -5;
    return 0;
}

orc_sim *orc_create(const orc_params *p) {
    if (!p || check_params(p) != 0) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->P = *p;
    s->nx = p->nx;
    s->ny = p->ny;
    s->n = (long)p->nx * p->ny;
    invert9(M1, s->Minv);
    /* Sec. 4 preamble: s_f^3 = s_f^5 = 1/(M/(eta cs^2) + 1/2), s_g^7 = s_g^8 =
     * 1/(nu/cs^2 + 1/2), the others 1 unless given. */
    for (int i = 0; i < 9; i++) {
        s->sf[i] = p->sf[i] > 0 ? p->sf[i] : 1.0;
        s->sg[i] = p->sg[i] > 0 ? p->sg[i] : 1.0;
    }
    double sM = 1.0 / (p->M / (p->eta * CS2) + 0.5);
    if (!(p->sf[3] > 0)) s->sf[3] = sM;
    if (!(p->sf[5] > 0)) s->sf[5] = sM;
    s->snu_local = !(p->sg[7] > 0 && p->sg[8] > 0);
    long n = s->n;
    size_t dz = sizeof(double);
    s->f = calloc(9 * n, dz);
    s->g = calloc(9 * n, dz);
    s->fs = calloc(9 * n, dz);
    s->gs = calloc(9 * n, dz);
    s->H = calloc(5 * n, dz);
    s->phi_prev = calloc(n, dz);
    s->phi = calloc(n, dz);
    s->ext = calloc((size_t)(p->nx + 2) * (p->ny + 2), dz);
    s->gx = calloc(n, dz);
    s->gy = calloc(n, dz);
    s->lap = calloc(n, dz);
    s->rho = calloc(n, dz);
    s->mu = calloc(n, dz);
    s->lam = calloc(n, dz);
    s->nxv = calloc(n, dz);
    s->nyv = calloc(n, dz);
    s->mx = calloc(n, dz);
    s->my = calloc(n, dz);
    s->Fx = calloc(n, dz);
    s->Fy = calloc(n, dz);
    s->snu = calloc(n, dz);
    s->ux = calloc(n, dz);
    s->uy = calloc(n, dz);
    s->pr = calloc(n, dz);
    s->P5 = calloc(5 * n, dz);
    s->dP5 = calloc(5 * n, dz);
    s->muext = calloc((size_t)(p->nx + 2) * (p->ny + 2), dz);
    s->fa = calloc(n, dz);
    s->dxv = calloc(n, dz);
    s->dyv = calloc(n, dz);
    s->dext = calloc((size_t)(p->nx + 2) * (p->ny + 2), dz);
    return s;
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    double *bufs[] = {s->f, s->g, s->fs, s->gs, s->H, s->phi_prev, s->phi, s->ext, s->gx, s->gy,
                      s->lap, s->rho, s->mu, s->lam, s->nxv, s->nyv, s->mx, s->my, s->Fx, s->Fy,
                      s->snu, s->ux, s->uy, s->pr, s->P5, s->dP5, s->muext, s->fa,
                      s->dxv, s->dyv, s->dext};
    for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); i++) free(bufs[i]);
    free(s);
}

int orc_rates(const orc_sim *s, double sf[9], double sg[9]) {
    for (int i = 0; i < 9; i++) {
        sf[i] = s->sf[i];
        sg[i] = s->sg[i];
    }
    if (s->snu_local) sg[7] = sg[8] = -1.0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Wetting condition, Eq. (FEwetting) discretised as Eq. (Dwetting):
 *   a phi_w^2 + b phi_w + c = 0,
 *   a = 4 cos(theta) / (W (phiA - phiB)),  b = 8/3 - a (phiA + phiB),
 *   c = a phiA phiB + phi2/3 - 3 phi1,
 * with phi1, phi2 the first and second fluid nodes (distances 1/2 and 3/2
 * from the half-way wall).  The root the paper selects, (-b + sqrt(D))/(2a),
 * is evaluated in the algebraically identical form -2c/(b + sqrt(D)), which
 * stays finite at a = 0.  The ghost node at distance -1/2 takes the value of
 * the quadratic through (0, phi_w), (1/2, phi1), (3/2, phi2) -- the same
 * quadratic from which the one-sided wall derivative above is built. */
void orc_wetting(const orc_params *p, double theta, double phi1, double phi2, double *phi_w,
                 double *phi_g) {
    double dphi = p->phiA - p->phiB;
    double a = 4.0 * cos(theta) / (p->W * dphi);
    double b = 8.0 / 3.0 - a * (p->phiA + p->phiB);
    double c = a * p->phiA * p->phiB + phi2 / 3.0 - 3.0 * phi1;
    double D = b * b - 4.0 * a * c;
    if (D < 0) D = 0;
    double pw = -2.0 * c / (b + sqrt(D));
    if (phi_w) *phi_w = pw;
    if (phi_g) *phi_g = (8.0 * pw - 6.0 * phi1 + phi2) / 3.0;
}

/* Fill s->ext ((nx+2) x (ny+2), one ghost layer) from s->phi: periodic axes
 * wrap; on wall axes the x-walls are filled first, then the y-walls across
 * the extended rows (this fixes the corner ghosts). */
static void fill_ghosts(const orc_sim *s, const double *phi, double *ext) {
    int nx = s->nx, ny = s->ny, ex = nx + 2;
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) ext[(y + 1) * ex + (x + 1)] = phi[y * nx + x];
    for (int y = 0; y < ny; y++) {
        double *row = ext + (y + 1) * ex;
        if (!s->P.wall_x) {
            row[0] = row[nx];
            row[nx + 1] = row[1];
        } else {
            orc_wetting(&s->P, s->P.theta[0], row[1], row[2], NULL, &row[0]);
            orc_wetting(&s->P, s->P.theta[1], row[nx], row[nx - 1], NULL, &row[nx + 1]);
        }
    }
    for (int X = 0; X < ex; X++) {
        if (!s->P.wall_y) {
            ext[X] = ext[ny * ex + X];
            ext[(ny + 1) * ex + X] = ext[1 * ex + X];
        } else {
            orc_wetting(&s->P, s->P.theta[2], ext[1 * ex + X], ext[2 * ex + X], NULL, &ext[X]);
            orc_wetting(&s->P, s->P.theta[3], ext[ny * ex + X], ext[(ny - 1) * ex + X], NULL,
                        &ext[(ny + 1) * ex + X]);
        }
    }
}

/* Eqs. (central1), (central2) on the extended field. */
static void stencils(const orc_sim *s, const double *ext, double *gx, double *gy, double *lap) {
    int nx = s->nx, ny = s->ny, ex = nx + 2;
#pragma omp parallel for
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            double c0 = ext[(y + 1) * ex + (x + 1)];
            double sx = 0, sy = 0, sl = 0;
            for (int i = 1; i < 9; i++) {
                double v = ext[(y + 1 + CY[i]) * ex + (x + 1 + CX[i])];
                sx += WT[i] * CX[i] * v;
                sy += WT[i] * CY[i] * v;
                sl += 2.0 * WT[i] * (v - c0);
            }
            long k = (long)y * nx + x;
            if (gx) gx[k] = sx / CS2;
            if (gy) gy[k] = sy / CS2;
            if (lap) lap[k] = sl / CS2;
        }
}

int orc_stencils(const orc_sim *cs, const double *phi, double *gx, double *gy, double *lap) {
    orc_sim *s = (orc_sim *)cs;
    if (!s || !phi) return -1;
    fill_ghosts(s, phi, s->ext);
    stencils(s, s->ext, gx, gy, lap);
    return 0;
}

/* Ghost layer of a field mirrored at walls: periodic axes wrap; an x-wall
 * ghost is sx times the first fluid node of its row, then a y-wall ghost is sy
 * times the first fluid row over the extended columns (x-walls first, as for
 * phi). */
static void fill_ghosts_signed(const orc_sim *s, const double *v, double *ext, double sx, double sy) {
    int nx = s->nx, ny = s->ny, ex = nx + 2;
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) ext[(y + 1) * ex + (x + 1)] = v[y * nx + x];
    for (int y = 0; y < ny; y++) {
        double *row = ext + (y + 1) * ex;
        if (!s->P.wall_x) {
            row[0] = row[nx];
            row[nx + 1] = row[1];
        } else {
            row[0] = sx * row[1];
            row[nx + 1] = sx * row[nx];
        }
    }
    for (int X = 0; X < ex; X++) {
        if (!s->P.wall_y) {
            ext[X] = ext[ny * ex + X];
            ext[(ny + 1) * ex + X] = ext[1 * ex + X];
        } else {
            ext[X] = sy * ext[1 * ex + X];
            ext[(ny + 1) * ex + X] = sy * ext[ny * ex + X];
        }
    }
}

/* Ghost layer of the chemical potential for the Cahn-Hilliard flux: periodic
 * axes wrap; at a wall the no-flux condition d mu / dn = 0 is imposed by
 * mirroring the first fluid node (x-walls first, then y-walls over the
 * extended rows, as for phi). */
static void fill_ghosts_mirror(const orc_sim *s, const double *v, double *ext) {
    fill_ghosts_signed(s, v, ext, 1.0, 1.0);
}

/* Sec. 2 closure for one node (AC form of D(phi)). */
typedef struct {
    double rho, drx, dry, mu_phi, lam, nx, ny, mx, my, Fx, Fy, nu, snu;
} closure_t;

static closure_t closure(const orc_sim *s, double phi, double gx, double gy, double lap) {
    const orc_params *p = &s->P;
    closure_t c;
    double dphi = p->phiA - p->phiB;
    double beta = 12.0 * p->sigma / (p->W * pow(dphi, 4));
    double kap = 1.5 * p->sigma * p->W / (dphi * dphi);
    c.mu_phi = 4.0 * beta * (phi - p->phiA) * (phi - p->phiB) * (phi - 0.5 * (p->phiA + p->phiB)) -
               kap * lap;
    double drho = (p->rhoA - p->rhoB) / dphi;
    c.rho = drho * (phi - p->phiB) + p->rhoB;
    c.drx = drho * gx;
    c.dry = drho * gy;
    double gn = sqrt(gx * gx + gy * gy + p->eps * p->eps);
    c.nx = gx / gn;
    c.ny = gy / gn;
    c.lam = (kap > 0 ? sqrt(2.0 * beta / kap) : 4.0 / (p->W * dphi)) * (p->phiA - phi) * (phi - p->phiB);
    /* m^phiC = -(drho/dphi) M D(phi), D = grad phi - lambda n */
    c.mx = -drho * p->M * (gx - c.lam * c.nx);
    c.my = -drho * p->M * (gy - c.lam * c.ny);
    if (p->model != 0) c.mx = c.my = 0.0; /* original and corrected models: mass flux rho u only */
    /* F = F_s + external: F_s = mu_phi grad phi */
    c.Fx = c.mu_phi * gx + p->Gx + (c.rho - p->rho_ref) * p->gx;
    c.Fy = c.mu_phi * gy + p->Gy + (c.rho - p->rho_ref) * p->gy;
    double t = (phi - p->phiB) / dphi;
    if (p->visc_law == 0) {
        double muA = p->rhoA * p->nuA, muB = p->rhoB * p->nuB;
        double mud = t * (muA - muB) + muB;
        c.nu = mud / c.rho;
    } else {
        double inv = t * (1.0 / p->nuA - 1.0 / p->nuB) + 1.0 / p->nuB;
        c.nu = 1.0 / inv;
    }
    c.snu = s->snu_local ? 1.0 / (c.nu / CS2 + 0.5) : s->sg[7];
    return c;
}

/* ------------------------------------------------------------------ */
/* App. C, Eq. (MfMRAC1): equilibrium and source moments of the AC model
 * (c = 1).  lam_n = lambda * n; dphiu, dphiv are explicit-Euler time
 * derivatives of phi u and phi v. */
void orc_moments_f(const orc_params *p, double phi, double u, double v, double lam_nx,
                   double lam_ny, double dphiu, double dphiv, double meq[9], double mR[9]) {
    double eta = p->eta;
    meq[0] = phi;
    meq[1] = -4.0 * phi + 2.0 * eta * phi;
    meq[2] = 4.0 * phi - 3.0 * eta * phi;
    meq[3] = phi * u;
    meq[4] = -phi * u;
    meq[5] = phi * v;
    meq[6] = -phi * v;
    meq[7] = 0.0;
    meq[8] = 0.0;
    mR[0] = mR[1] = mR[2] = 0.0;
    mR[3] = lam_nx / 3.0 + dphiu;
    mR[4] = -lam_nx / 3.0 - dphiu;
    mR[5] = lam_ny / 3.0 + dphiv;
    mR[6] = -lam_ny / 3.0 - dphiv;
    mR[7] = mR[8] = 0.0;
}

/* App. C, Eq. (MfMRCH1): the Cahn-Hilliard moments carry eta mu_phi in rows 1
 * and 2 and no lambda n source. */
void orc_moments_f_ch(const orc_params *p, double phi, double mu, double u, double v, double dphiu,
                      double dphiv, double meq[9], double mR[9]) {
    double eta = p->eta;
    meq[0] = phi;
    meq[1] = -4.0 * phi + 2.0 * eta * mu;
    meq[2] = 4.0 * phi - 3.0 * eta * mu;
    meq[3] = phi * u;
    meq[4] = -phi * u;
    meq[5] = phi * v;
    meq[6] = -phi * v;
    meq[7] = 0.0;
    meq[8] = 0.0;
    mR[0] = mR[1] = mR[2] = 0.0;
    mR[3] = dphiu;
    mR[4] = -dphiu;
    mR[5] = dphiv;
    mR[6] = -dphiv;
    mR[7] = mR[8] = 0.0;
}

/* App. C, Eq. (MgMF1) with c = 1.  dP_um_x = d_t(u m_x), dP_vm_y = d_t(v m_y),
 * dP_cross = d_t(u m_y + v m_x); F is the total force; (drx, dry) = grad rho. */
void orc_moments_g(const orc_params *p, double rho, double pr, double u, double v, double mx,
                   double my, double Fx, double Fy, double drx, double dry, double dP_um_x,
                   double dP_vm_y, double dP_cross, double meq[9], double mF[9]) {
    double r0 = p->rho0;
    double uu = u * u + v * v;
    double um = u * mx + v * my;
    double dum = dP_um_x + dP_vm_y; /* d_t(u . m) */
    double ugr = u * drx + v * dry;
    double uF = u * Fx + v * Fy;
    meq[0] = r0;
    meq[1] = -4.0 * r0 + (6.0 * pr + 3.0 * rho * uu + 3.0 * um);
    meq[2] = 4.0 * r0 - (9.0 * pr + 3.0 * rho * uu + 3.0 * um);
    meq[3] = rho * u;
    meq[4] = -rho * u;
    meq[5] = rho * v;
    meq[6] = -rho * v;
    meq[7] = u * mx - v * my + rho * (u * u - v * v);
    meq[8] = (u * my + v * mx + 2.0 * rho * u * v) / 2.0;
    mF[0] = ugr;
    mF[1] = 3.0 * dum + 6.0 * uF;
    mF[2] = -ugr - (3.0 * dum + 6.0 * uF);
    mF[3] = Fx;
    mF[4] = -Fx;
    mF[5] = Fy;
    mF[6] = -Fy;
    mF[7] = 2.0 / 3.0 * (u * drx - v * dry) + (2.0 * (u * Fx - v * Fy) + (dP_um_x - dP_vm_y));
    mF[8] = 1.0 / 3.0 * (u * dry + v * drx) + (2.0 * (u * Fy + v * Fx) + dP_cross) / 2.0;
}

/* Sec. 3: g^eq_i = alpha_i + s_i(phi, u) (Eq. geq) and
 * F_i = w_i [u.grad rho + c_i.F/cs^2 + (M_2F - cs^2 u.grad rho I):(c_i c_i - cs^2 I)/(2 cs^4)]
 * with M_2F of Eq. (M2F) in the second way of Remark 1:
 * d_t(rho uu + p I) -> uF + Fu, d_t(m u) kept (symmetric part). */
void orc_direct_g(const orc_params *p, double rho, double pr, double u, double v, double mx,
                  double my, double Fx, double Fy, double drx, double dry, double dP_um_x,
                  double dP_vm_y, double dP_cross, double geq[9], double Fi[9]) {
    double Q[2][2], M2[2][2];
    double uv[2] = {u, v}, mm[2] = {mx, my}, FF[2] = {Fx, Fy}, gr[2] = {drx, dry};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            Q[a][b] = rho * uv[a] * uv[b] + 0.5 * (mm[a] * uv[b] + mm[b] * uv[a]);
    double ugr = u * drx + v * dry;
    double dmu[2][2] = {{dP_um_x, 0.5 * dP_cross}, {0.5 * dP_cross, dP_vm_y}};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            M2[a][b] = uv[a] * FF[b] + FF[a] * uv[b] + dmu[a][b] +
                       CS2 * (uv[a] * gr[b] + uv[b] * gr[a]) + (a == b ? CS2 * ugr : 0.0);
    for (int i = 0; i < 9; i++) {
        double c[2] = {(double)CX[i], (double)CY[i]};
        double alpha = (i == 0) ? (WT[0] - 1.0) * pr / CS2 + p->rho0 : WT[i] * pr / CS2;
        double qc = 0, mc = 0;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                double t = c[a] * c[b] - (a == b ? CS2 : 0.0);
                qc += Q[a][b] * t;
                mc += (M2[a][b] - (a == b ? CS2 * ugr : 0.0)) * t;
            }
        double cru = c[0] * rho * u + c[1] * rho * v;
        geq[i] = alpha + WT[i] * (cru / CS2 + qc / (2.0 * CS2 * CS2));
        double cF = c[0] * Fx + c[1] * Fy;
        Fi[i] = WT[i] * (ugr + cF / CS2 + mc / (2.0 * CS2 * CS2));
    }
}

/* ------------------------------------------------------------------ */
static void matvec(const double A[9][9], const double *x, double *y) {
    for (int i = 0; i < 9; i++) {
        double s = 0;
        for (int j = 0; j < 9; j++) s += A[i][j] * x[j];
        y[i] = s;
    }
}

/* Cahn-Hilliard mass flux m^phiC = -(drho/dphi) M grad mu_phi (Sec. 2, D =
 * grad mu for Eq. CHE), grad mu by Eq. central1 on mu with its ghost layer;
 * zero for the original and corrected models (m = rho u).  The corrected
 * model's interface force F_a = (drho/dphi) u div(M grad mu_phi) (App. A,
 * Eq. NS2-add; Sec. 4 preamble) is kept as its coefficient fa = (drho/dphi) M lap mu_phi
 * of u, lap by Eq. central2 on the same ghost layer; zero for the others. */
static void ch_flux(orc_sim *s, const double *mu, double *mx, double *my) {
    const orc_params *p = &s->P;
    long n = s->n;
    fill_ghosts_mirror(s, mu, s->muext);
    stencils(s, s->muext, mx, my, s->fa);
    double drho = (p->rhoA - p->rhoB) / (p->phiA - p->phiB);
    for (long k = 0; k < n; k++) {
        mx[k] = p->model == 0 ? -drho * p->M * mx[k] : 0.0;
        my[k] = p->model == 0 ? -drho * p->M * my[k] : 0.0;
        s->fa[k] = p->model == 2 ? drho * p->M * s->fa[k] : 0.0;
    }
}

/* The corrected model's interface force with the AC phase field (App. A,
 * Eq. NS2-add; Sec. 4 preamble): F_a = (drho/dphi) u div(M D), D = grad phi -
 * lambda n with the closure's grad phi and n.  div D by Eq. central1 applied to
 * each component, on a ghost layer in which a wall mirrors D of the first fluid
 * node with its normal component reversed (no diffusive flux through the wall).
 * Keeps the coefficient fa = (drho/dphi) M div D of u. */
static void ac_corrected_force(orc_sim *s) {
    const orc_params *p = &s->P;
    long n = s->n;
    for (long k = 0; k < n; k++) {
        s->dxv[k] = s->gx[k] - s->lam[k] * s->nxv[k];
        s->dyv[k] = s->gy[k] - s->lam[k] * s->nyv[k];
    }
    fill_ghosts_signed(s, s->dxv, s->muext, -1.0, 1.0);
    fill_ghosts_signed(s, s->dyv, s->dext, 1.0, -1.0);
    stencils(s, s->muext, s->dxv, NULL, NULL); /* d Dx / dx */
    stencils(s, s->dext, NULL, s->dyv, NULL);  /* d Dy / dy */
    double drho = (p->rhoA - p->rhoB) / (p->phiA - p->phiB);
    for (long k = 0; k < n; k++) s->fa[k] = drho * p->M * (s->dxv[k] + s->dyv[k]);
}

/* The local scheme for grad phi of the AC model (Eq. local), levels >= 1:
 * with A = -M - cs^2/2, B = M lambda and C = sum_i c_i f_i - phi u + d_t(phi u)/2,
 * C = A grad phi + B n.  u depends on grad phi through F_s = mu_phi grad phi
 * (Eq. comU: u = u0 + mu_phi grad phi / (2 rho), u0 the velocity without F_s),
 * so with the explicit-Euler d_t(phi u) = phi u - (phi u)^{n-1}
 *   C0 = sum_i c_i f_i - phi u0 / 2 - (phi u)^{n-1} / 2 = A' grad phi + B n,
 *   A' = A + phi mu_phi / (4 rho),
 * whence |grad phi| = (|C0| + B) / (-A') (clamped at 0) and
 * grad phi = -|grad phi| C0 / |C0| (n points against C0, A' being negative).
 * Where grad phi vanishes the direction C0 / |C0| is undefined, as n is in the
 * stencil scheme; it is regularised with the same eps_n:
 * C0 / sqrt(|C0|^2 + (A' eps_n)^2), |C0| = |A'| |grad phi| in the bulk.
 * mu_phi takes lap phi from Eq. central2.  Overwrites s->gx, s->gy. */
static void local_gradient(orc_sim *s) {
    const orc_params *p = &s->P;
    long n = s->n;
    double A = -p->M - 0.5 * CS2;
#pragma omp parallel for
    for (long k = 0; k < n; k++) {
        closure_t c = closure(s, s->phi[k], 0.0, 0.0, s->lap[k]);
        double jfx = 0, jfy = 0, jgx = 0, jgy = 0;
        for (int i = 0; i < 9; i++) {
            jfx += CX[i] * s->f[i * n + k];
            jfy += CY[i] * s->f[i * n + k];
            jgx += CX[i] * s->g[i * n + k];
            jgy += CY[i] * s->g[i * n + k];
        }
        double u0 = (jgx + 0.5 * (p->Gx + (c.rho - p->rho_ref) * p->gx)) / c.rho;
        double v0 = (jgy + 0.5 * (p->Gy + (c.rho - p->rho_ref) * p->gy)) / c.rho;
        double cx = jfx - 0.5 * s->phi[k] * u0 - 0.5 * s->H[0 * n + k];
        double cy = jfy - 0.5 * s->phi[k] * v0 - 0.5 * s->H[1 * n + k];
        double Ap = A + s->phi[k] * c.mu_phi / (4.0 * c.rho);
        double B = p->M * c.lam;
        double cn = sqrt(cx * cx + cy * cy);
        double mag = (cn + B) / (-Ap);
        if (mag > 0) {
            double inv = 1.0 / sqrt(cn * cn + Ap * Ap * p->eps * p->eps);
            s->gx[k] = -mag * cx * inv;
            s->gy[k] = -mag * cy * inv;
        } else {
            s->gx[k] = 0.0;
            s->gy[k] = 0.0;
        }
    }
}

/* Stages 1-7: every macroscopic field of the current level into the scratch
 * arrays of s (phi, ext, gradients, closure, u, history derivatives, p). */
static void macroscopic(orc_sim *s) {
    long n = s->n;
    int nx = s->nx, ny = s->ny;
    const orc_params *p = &s->P;
    for (long k = 0; k < n; k++) {
        double a = 0;
        for (int i = 0; i < 9; i++) a += s->f[i * n + k];
        s->phi[k] = a;
    }
    fill_ghosts(s, s->phi, s->ext);
    stencils(s, s->ext, s->gx, s->gy, s->lap);
    if (p->grad == 1 && s->step > 0) local_gradient(s);
#pragma omp parallel for
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            long k = (long)y * nx + x;
            closure_t c = closure(s, s->phi[k], s->gx[k], s->gy[k], s->lap[k]);
            s->rho[k] = c.rho;
            s->mu[k] = c.mu_phi;
            s->lam[k] = c.lam;
            s->nxv[k] = c.nx;
            s->nyv[k] = c.ny;
            s->mx[k] = c.mx;
            s->my[k] = c.my;
            s->Fx[k] = c.Fx;
            s->Fy[k] = c.Fy;
            s->snu[k] = c.snu;
        }
    if (p->pf == 1) ch_flux(s, s->mu, s->mx, s->my);
    else if (p->model == 2) ac_corrected_force(s);
    double drho = (p->rhoA - p->rhoB) / (p->phiA - p->phiB);
#pragma omp parallel for
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            long k = (long)y * nx + x;
            double rho = s->rho[k], mx = s->mx[k], my = s->my[k], Fx = s->Fx[k], Fy = s->Fy[k];
            double drx = drho * s->gx[k], dry = drho * s->gy[k];
            /* Eq. (comU): rho u = sum_i c_i g_i + F/2 */
            double jx = 0, jy = 0;
            for (int i = 0; i < 9; i++) {
                jx += CX[i] * s->g[i * n + k];
                jy += CY[i] * s->g[i * n + k];
            }
            /* corrected model: F = F_0 + fa u in Eq. comU, solved for u exactly
             * (fa is zero for the other models) */
            double a = s->fa[k];
            double u = (jx + 0.5 * Fx) / (rho - 0.5 * a);
            double v = (jy + 0.5 * Fy) / (rho - 0.5 * a);
            Fx += a * u;
            Fy += a * v;
            s->Fx[k] = Fx;
            s->Fy[k] = Fy;
            s->ux[k] = u;
            s->uy[k] = v;
            /* history products chi and their explicit-Euler derivatives */
            double P[5] = {s->phi[k] * u, s->phi[k] * v, u * mx, v * my, u * my + v * mx};
            for (int j = 0; j < 5; j++) {
                s->P5[j * n + k] = P[j];
                s->dP5[j * n + k] = s->step > 0 ? P[j] - s->H[j * n + k] : 0.0;
            }
            /* Eq. (computP), second way of Remark 1: J d d_t p dropped,
             * d_t(rho u.u) -> 2 F.u, d_t(m.u) by explicit Euler; H and K of App. C. */
            double sg0 = s->sg[0], sg2 = s->sg[2];
            double Hc = (sg2 - sg0) / (9.0 * sg0 * sg2);
            double Kc = 1.0 / 3.0;
            double sum = 0;
            for (int i = 1; i < 9; i++) sum += s->g[i * n + k];
            double ugr = u * drx + v * dry;
            double trQ = rho * (u * u + v * v) + (u * mx + v * my);
            double s0 = WT[0] * (-CS2 * trQ) / (2.0 * CS2 * CS2); /* s_0(phi,u) of Eq. geq at c_0 = 0 */
            double dum = s->dP5[2 * n + k] + s->dP5[3 * n + k];
            double uF = u * Fx + v * Fy;
            s->pr[k] = CS2 / (1.0 - WT[0]) * (sum + (0.5 + Hc) * ugr + s0 + Kc * (2.0 * uF + dum));
        }
}

/* One node of Eq. (evoPF) -- and of Remark 2 for g -- in moment form:
 * m = M1 f; m* = m - S (m - m^eq) + (I - S/2) m_R; f* = M1^-1 m*. */
static void collide_node(const double Minv[9][9], const double S[9], const double fv[9], const double meq[9],
                         const double mR[9], double out[9]) {
    double m[9], ms[9];
    matvec(M1, fv, m);
    for (int j = 0; j < 9; j++) ms[j] = m[j] - S[j] * (m[j] - meq[j]) + (1.0 - S[j] / 2.0) * mR[j];
    matvec(Minv, ms, out);
}

void orc_collide_node(const double S[9], const double fv[9], const double meq[9], const double mR[9],
                      double out[9]) {
    double R[9][9];
    invert9(M1, R);
    collide_node(R, S, fv, meq, mR, out);
}

static void collide(orc_sim *s) {
    long n = s->n;
    int nx = s->nx, ny = s->ny;
    const orc_params *p = &s->P;
#pragma omp parallel for
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            long k = (long)y * nx + x;
            double fv[9], gv[9], meq[9], mR[9], out[9];
            for (int i = 0; i < 9; i++) {
                fv[i] = s->f[i * n + k];
                gv[i] = s->g[i * n + k];
            }
            double u = s->ux[k], v = s->uy[k];
            /* Eq. (evoPF), moment form */
            if (p->pf == 1)
                orc_moments_f_ch(p, s->phi[k], s->mu[k], u, v, s->dP5[0 * n + k], s->dP5[1 * n + k], meq, mR);
            else
                orc_moments_f(p, s->phi[k], u, v, s->lam[k] * s->nxv[k], s->lam[k] * s->nyv[k],
                              s->dP5[0 * n + k], s->dP5[1 * n + k], meq, mR);
            collide_node(s->Minv, s->sf, fv, meq, mR, out);
            for (int i = 0; i < 9; i++) s->fs[i * n + k] = out[i];
            /* Remark 2, moment form of Eq. (evoNS) */
            orc_moments_g(p, s->rho[k], s->pr[k], u, v, s->mx[k], s->my[k], s->Fx[k], s->Fy[k],
                          (p->rhoA - p->rhoB) / (p->phiA - p->phiB) * s->gx[k],
                          (p->rhoA - p->rhoB) / (p->phiA - p->phiB) * s->gy[k], s->dP5[2 * n + k],
                          s->dP5[3 * n + k], s->dP5[4 * n + k], meq, mR);
            double sg[9];
            for (int j = 0; j < 9; j++) sg[j] = s->sg[j];
            sg[7] = sg[8] = s->snu[k];
            collide_node(s->Minv, sg, gv, meq, mR, out);
            for (int i = 0; i < 9; i++) s->gs[i * n + k] = out[i];
        }
}

/* Push streaming; a population that would leave through a wall face comes
 * back to its node in the opposite direction (half-way bounce-back). */
static void stream(orc_sim *s) {
    long n = s->n;
    int nx = s->nx, ny = s->ny;
    for (int i = 0; i < 9; i++) {
        int o = opposite(i);
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long k = (long)y * nx + x;
                int tx = x + CX[i], ty = y + CY[i];
                int out = 0;
                if (tx < 0 || tx >= nx) {
                    if (s->P.wall_x) out = 1;
                    else tx = (tx + nx) % nx;
                }
                if (ty < 0 || ty >= ny) {
                    if (s->P.wall_y) out = 1;
                    else ty = (ty + ny) % ny;
                }
                if (out) {
                    s->f[o * n + k] = s->fs[i * n + k];
                    s->g[o * n + k] = s->gs[i * n + k];
                } else {
                    long t = (long)ty * nx + tx;
                    s->f[i * n + t] = s->fs[i * n + k];
                    s->g[i * n + t] = s->gs[i * n + k];
                }
            }
    }
}

int orc_step(orc_sim *s, long nsteps) {
    if (!s || nsteps < 0) return -1;
    for (long t = 0; t < nsteps; t++) {
        macroscopic(s);
        collide(s);
        memcpy(s->H, s->P5, sizeof(double) * 5 * s->n);
        memcpy(s->phi_prev, s->phi, sizeof(double) * s->n);
        stream(s);
        s->step++;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
int orc_init(orc_sim *s, const double *phi0, const double *u0, const double *p0) {
    if (!s || !phi0) return -1;
    long n = s->n;
    int nx = s->nx, ny = s->ny;
    const orc_params *p = &s->P;
    memcpy(s->phi, phi0, sizeof(double) * n);
    fill_ghosts(s, s->phi, s->ext);
    stencils(s, s->ext, s->gx, s->gy, s->lap);
    for (long k = 0; k < n; k++) {
        closure_t c = closure(s, phi0[k], s->gx[k], s->gy[k], s->lap[k]);
        s->mu[k] = c.mu_phi;
        s->mx[k] = c.mx;
        s->my[k] = c.my;
        s->rho[k] = c.rho;
    }
    if (p->pf == 1) ch_flux(s, s->mu, s->mx, s->my);
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            long k = (long)y * nx + x;
            double u = u0 ? u0[k] : 0.0, v = u0 ? u0[n + k] : 0.0, pr = p0 ? p0[k] : 0.0;
            double meq[9], mR[9], out[9];
            if (p->pf == 1)
                orc_moments_f_ch(p, phi0[k], s->mu[k], u, v, 0, 0, meq, mR);
            else
                orc_moments_f(p, phi0[k], u, v, 0, 0, 0, 0, meq, mR);
            matvec(s->Minv, meq, out);
            for (int i = 0; i < 9; i++) s->f[i * n + k] = out[i];
            orc_moments_g(p, s->rho[k], pr, u, v, s->mx[k], s->my[k], 0, 0, 0, 0, 0, 0, 0, meq, mR);
            matvec(s->Minv, meq, out);
            for (int i = 0; i < 9; i++) s->g[i * n + k] = out[i];
        }
    memset(s->H, 0, sizeof(double) * 5 * n);
    memcpy(s->phi_prev, phi0, sizeof(double) * n);
    s->step = 0;
    return 0;
}

/* Initial pressure of the two fluids at rest under gravity along y (the
 * gravity-driven set-ups of Secs. 4.4 and 4.5 do not state it; read as
 * hydrostatic): the density law of Sec. 2 at phi0 gives rho, and p follows
 * dp/dy = (rho - rho_ref) g_y down every column by the trapezoid rule from
 * p = 0 at the top row; the mean over the lattice is then subtracted. */
int orc_hydrostatic_pressure(const orc_params *p, const double *phi0, double *p0) {
    if (!p || !phi0 || !p0) return -1;
    if (p->gx != 0.0) return -8;
    int nx = p->nx, ny = p->ny;
    long n = (long)nx * ny;
    double drho = (p->rhoA - p->rhoB) / (p->phiA - p->phiB);
    double total = 0.0;
    for (int x = 0; x < nx; x++) {
        p0[(long)(ny - 1) * nx + x] = 0.0;
        for (int y = ny - 2; y >= 0; y--) {
            double rho_lo = p->rhoB + drho * (phi0[(long)y * nx + x] - p->phiB);
            double rho_hi = p->rhoB + drho * (phi0[(long)(y + 1) * nx + x] - p->phiB);
            double f_lo = (rho_lo - p->rho_ref) * p->gy, f_hi = (rho_hi - p->rho_ref) * p->gy;
            p0[(long)y * nx + x] = p0[(long)(y + 1) * nx + x] - 0.5 * (f_lo + f_hi);
        }
    }
    for (long k = 0; k < n; k++) total += p0[k];
    for (long k = 0; k < n; k++) p0[k] -= total / (double)n;
    return 0;
}

/* grad phi of the current level as the closure uses it (Eq. central1, or
 * Eq. local when selected). */
int orc_grad(const orc_sim *cs, double *gx, double *gy) {
    orc_sim *s = (orc_sim *)cs;
    if (!s || !gx || !gy) return -1;
    macroscopic(s);
    memcpy(gx, s->gx, sizeof(double) * s->n);
    memcpy(gy, s->gy, sizeof(double) * s->n);
    return 0;
}

/* m^phiC of the current level (Eq. mPhiC for the Allen-Cahn model, the
 * Cahn-Hilliard flux of Eq. CHE otherwise; zero for the original and
 * corrected models). */
int orc_flux(const orc_sim *cs, double *mx, double *my) {
    orc_sim *s = (orc_sim *)cs;
    if (!s || !mx || !my) return -1;
    macroscopic(s);
    memcpy(mx, s->mx, sizeof(double) * s->n);
    memcpy(my, s->my, sizeof(double) * s->n);
    return 0;
}

/* The corrected model's coefficient a of F_a = a u at the current level
 * (zero for the other models). */
int orc_fa(const orc_sim *cs, double *a) {
    orc_sim *s = (orc_sim *)cs;
    if (!s || !a) return -1;
    macroscopic(s);
    memcpy(a, s->fa, sizeof(double) * s->n);
    return 0;
}

int orc_moments(const orc_sim *cs, double *phi, double *u, double *p) {
    orc_sim *s = (orc_sim *)cs;
    if (!s) return -1;
    macroscopic(s);
    long n = s->n;
    for (long k = 0; k < n; k++) {
        if (phi) phi[k] = s->phi[k];
        if (u) {
            u[k] = s->ux[k];
            u[n + k] = s->uy[k];
        }
        if (p) p[k] = s->pr[k];
    }
    return 0;
}

int orc_get_state(const orc_sim *s, double *f, double *g, double *H, double *phi_prev, long *step) {
    if (!s) return -1;
    long n = s->n;
    if (f) memcpy(f, s->f, sizeof(double) * 9 * n);
    if (g) memcpy(g, s->g, sizeof(double) * 9 * n);
    if (H) memcpy(H, s->H, sizeof(double) * 5 * n);
    if (phi_prev) memcpy(phi_prev, s->phi_prev, sizeof(double) * n);
    if (step) *step = s->step;
    return 0;
}

int orc_set_state(orc_sim *s, const double *f, const double *g, const double *phi_prev,
                  const double *u_prev, long step) {
    if (s && s->P.grad == 1 && step > 0) return -8; /* the local scheme's history needs m^phiC */
    return orc_set_state_m(s, f, g, phi_prev, u_prev, NULL, step);
}

/* As orc_set_state; m_prev ([2][n], m^phiC of level n-1), when given, replaces
 * the one the closure would compute from phi_prev (the local gradient scheme
 * keeps it as history). */
int orc_set_state_m(orc_sim *s, const double *f, const double *g, const double *phi_prev,
                    const double *u_prev, const double *m_prev, long step) {
    if (!s || !f || !g || step < 0) return -1;
    if (s->P.grad == 1 && step > 0 && !m_prev) return -1;
    long n = s->n;
    memcpy(s->f, f, sizeof(double) * 9 * n);
    memcpy(s->g, g, sizeof(double) * 9 * n);
    s->step = step;
    memset(s->H, 0, sizeof(double) * 5 * n);
    if (step > 0) {
        if (!phi_prev || !u_prev) return -1;
        memcpy(s->phi_prev, phi_prev, sizeof(double) * n);
        fill_ghosts(s, phi_prev, s->ext);
        stencils(s, s->ext, s->gx, s->gy, s->lap);
        for (long k = 0; k < n; k++) {
            closure_t c = closure(s, phi_prev[k], s->gx[k], s->gy[k], s->lap[k]);
            s->mu[k] = c.mu_phi;
            s->mx[k] = c.mx;
            s->my[k] = c.my;
        }
        if (s->P.pf == 1) ch_flux(s, s->mu, s->mx, s->my);
        for (long k = 0; k < n; k++) {
            double u = u_prev[k], v = u_prev[n + k], ph = phi_prev[k];
            double mx = m_prev ? m_prev[k] : s->mx[k], my = m_prev ? m_prev[n + k] : s->my[k];
            double P[5] = {ph * u, ph * v, u * mx, v * my, u * my + v * mx};
            for (int j = 0; j < 5; j++) s->H[j * n + k] = P[j];
        }
    } else {
        long k;
        for (k = 0; k < n; k++) {
            double a = 0;
            for (int i = 0; i < 9; i++) a += f[i * n + k];
            s->phi_prev[k] = a;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-node diagnostics of the current level (Sec. 4.1), after macroscopic():
 *  div u = tr S with S from Eq. (strainRate):
 *     S = -s_2/(2 rho cs^2) [sum_i c_i c_i (g_i - g_i^eq) + M_2F/2],
 *     s_2 the node's s_nu, tr M_2F = 2 u.F + d_t(u.m) + 4 cs^2 u.grad rho
 *     (way 2 of Remark 1: d_t(rho uu + p I) -> uF + Fu),
 *  S_m = d_t rho + div(m^CC) = (rho^n - rho^{n-1}) + rho div u + u.grad rho + div m^phiC,
 *  where div m^phiC uses Eq. (central1); interior[k] = 0 (and S_m 0) at nodes
 *  that have a neighbour beyond a wall. */
static void div_fields(orc_sim *s, double *div, double *sm, unsigned char *interior) {
    const orc_params *p = &s->P;
    long n = s->n;
    int nx = s->nx, ny = s->ny;
    double drho = (p->rhoA - p->rhoB) / (p->phiA - p->phiB);
    for (long k = 0; k < n; k++) {
        double geq[9], meq[9], mF[9];
        double u = s->ux[k], v = s->uy[k];
        orc_moments_g(p, s->rho[k], s->pr[k], u, v, s->mx[k], s->my[k], s->Fx[k], s->Fy[k],
                      drho * s->gx[k], drho * s->gy[k], s->dP5[2 * n + k], s->dP5[3 * n + k],
                      s->dP5[4 * n + k], meq, mF);
        matvec(s->Minv, meq, geq);
        double acc = 0;
        for (int i = 0; i < 9; i++) {
            double c2 = CX[i] * CX[i] + CY[i] * CY[i];
            acc += c2 * (s->g[i * n + k] - geq[i]);
        }
        double ugr = u * drho * s->gx[k] + v * drho * s->gy[k];
        double trM2F = 2.0 * (u * s->Fx[k] + v * s->Fy[k]) + (s->dP5[2 * n + k] + s->dP5[3 * n + k]) +
                       2.0 * CS2 * ugr + 2.0 * CS2 * ugr;
        div[k] = -s->snu[k] / (2.0 * s->rho[k] * CS2) * (acc + 0.5 * trM2F);
    }
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            long k = (long)y * nx + x;
            int ok = 1;
            double dmx = 0, dmy = 0;
            for (int i = 1; i < 9; i++) {
                int tx = x + CX[i], ty = y + CY[i];
                if (tx < 0 || tx >= nx) {
                    if (p->wall_x) ok = 0;
                    tx = (tx + nx) % nx;
                }
                if (ty < 0 || ty >= ny) {
                    if (p->wall_y) ok = 0;
                    ty = (ty + ny) % ny;
                }
                long t = (long)ty * nx + tx;
                dmx += WT[i] * CX[i] * s->mx[t];
                dmy += WT[i] * CY[i] * s->my[t];
            }
            interior[k] = (unsigned char)ok;
            if (!ok) {
                sm[k] = 0.0;
                continue;
            }
            double divm = (dmx + dmy) / CS2;
            double rho_prev = drho * (s->phi_prev[k] - p->phiB) + p->rhoB;
            double dtr = s->step > 0 ? s->rho[k] - rho_prev : 0.0;
            double ugr = s->ux[k] * drho * s->gx[k] + s->uy[k] * drho * s->gy[k];
            sm[k] = dtr + s->rho[k] * div[k] + ugr + divm;
        }
}

/* div u (tr S) and S_m of every node of the current level, [ny][nx] each; S_m
 * is NaN at nodes with a neighbour beyond a wall.  Either pointer may be NULL. */
int orc_div_fields(const orc_sim *cs, double *div, double *sm) {
    orc_sim *s = (orc_sim *)cs;
    if (!s) return -1;
    macroscopic(s);
    long n = s->n;
    double *d = calloc(n, sizeof(double)), *m = calloc(n, sizeof(double));
    unsigned char *in = calloc(n, 1);
    div_fields(s, d, m, in);
    for (long k = 0; k < n; k++)
        if (!in[k]) m[k] = NAN;
    if (div) memcpy(div, d, sizeof(double) * n);
    if (sm) memcpy(sm, m, sizeof(double) * n);
    free(d);
    free(m);
    free(in);
    return 0;
}

/* Diagnostics of the current level (Sec. 4.1) from the per-node fields above:
 * the rms of S_m runs over the nodes whose eight neighbours are all fluid
 * nodes (all nodes when both axes are periodic); D_u^rms runs over all nodes. */
int orc_diagnostics(const orc_sim *cs, double out[6]) {
    orc_sim *s = (orc_sim *)cs;
    if (!s || !out) return -1;
    macroscopic(s);
    long n = s->n;
    double *div = calloc(n, sizeof(double)), *sm = calloc(n, sizeof(double));
    unsigned char *interior = calloc(n, 1);
    div_fields(s, div, sm, interior);
    double sum_phi = 0, maxdiv = 0, sdu = 0, umax = 0, nonfinite = 0;
    for (long k = 0; k < n; k++) {
        double u = s->ux[k], v = s->uy[k];
        sum_phi += s->phi[k];
        if (fabs(div[k]) > maxdiv) maxdiv = fabs(div[k]);
        sdu += div[k] * div[k];
        double um = sqrt(u * u + v * v);
        if (um > umax) umax = um;
        for (int i = 0; i < 9; i++)
            if (!isfinite(s->f[i * n + k]) || !isfinite(s->g[i * n + k])) nonfinite = 1;
    }
    double ssm = 0;
    long cnt = 0;
    for (long k = 0; k < n; k++) {
        if (!interior[k]) continue;
        ssm += sm[k] * sm[k];
        cnt++;
    }
    out[0] = sum_phi;
    out[1] = maxdiv;
    out[2] = sqrt(sdu / (double)n);
    out[3] = cnt > 0 ? sqrt(ssm / (double)cnt) : 0.0;
    out[4] = umax;
    out[5] = nonfinite;
    free(div);
    free(sm);
    free(interior);
    return 0;
}
