/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 CPU reference of the consistent and conservative phase-field
 * lattice Boltzmann method of Zhan, Chai & Shi (arXiv:2111.00847): the
 * conservative Allen-Cahn MRT model for the order parameter (Sec. 3,
 * Eq. evoPF with the App. C moments of Eq. MfMRAC1; or the Cahn-Hilliard
 * model with those of Eq. MfMRCH1) coupled to the
 * incompressible MRT model for the flow (Eq. evoNS, Remark 2, App. C moments
 * of Eq. MgMF1), isotropic finite differences (Eqs. central1, central2),
 * half-way bounce-back (Sec. 4 preamble) and the wetting boundary condition
 * (Eq. Dwetting).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU baseline may
 * load this library.  It shares no code with the GPU library.
 *
 * Lattice units (dx = dt = c = 1, cs^2 = 1/3).  Fields are row-major
 * [ny][nx], x fastest, y = 0 the bottom row.  Distributions are [9][ny][nx]
 * with the velocity ordering of the rows of M1 in App. C:
 * c0..c8 = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    int nx, ny;
    int wall_x, wall_y;   /* 0: periodic axis, 1: half-way bounce-back walls on both faces */
    int visc_law;         /* 0: linear dynamic viscosity (Eq. linearMu); 1: inverse-linear nu (Eq. inverseNu) */
    int model;            /* 0: present consistent model; 1: original (m = rho u); 2: corrected (m = rho u plus F_a; Cahn-Hilliard only) */
    int pf;               /* phase-field equation: 0 Allen-Cahn (D = grad phi - lambda n, Eq. ACE);
                             1 Cahn-Hilliard (D = grad mu_phi, Eq. CHE; moments of Eq. MfMRCH1) */
    int grad;             /* grad phi: 0 Eq. central1; 1 the local scheme of Eq. local (Allen-Cahn,
                             levels >= 1; level 0 and lap phi use the stencils) */
    double phiA, phiB, rhoA, rhoB, nuA, nuB;
    double sigma, W, M, eta;
    double sf[9], sg[9];  /* <= 0 selects the paper's default (Sec. 4 preamble) */
    double Gx, Gy;        /* uniform body-force density */
    double gx, gy;        /* gravity; adds (rho - rho_ref) * g */
    double rho_ref;
    double theta[4];      /* contact angle [rad] at the x-, x+, y-, y+ walls */
    double rho0;          /* constant density in g^eq (Eq. geq) */
    double eps;           /* regularisation of |grad phi| in n */
} orc_params;

typedef struct orc_sim orc_sim;

orc_sim *orc_create(const orc_params *p);
void orc_destroy(orc_sim *s);
/* f = f^eq(phi0,u0), g = g^eq(phi0,u0,p0); u0 is [2][ny][nx] or NULL, p0 [ny][nx] or NULL. */
int orc_init(orc_sim *s, const double *phi0, const double *u0, const double *p0);
int orc_step(orc_sim *s, long nsteps);
/* Hydrostatic initial pressure for gravity along y: rho from the density law
 * of Sec. 2 at phi0, dp/dy = (rho - rho_ref) g_y down every column (trapezoid
 * rule from the top row), zero mean.  phi0, p0: [ny][nx].  -8 if gx != 0. */
int orc_hydrostatic_pressure(const orc_params *p, const double *phi0, double *p0);
/* phi, p: [ny][nx]; u: [2][ny][nx]; values at the current time level (pre-collision). */
int orc_moments(const orc_sim *s, double *phi, double *u, double *p);
/* out: sum phi, max|div u|, D_u^rms, S_m^rms, max|u|, non-finite flag. */
int orc_diagnostics(const orc_sim *s, double out[6]);
/* The per-node fields behind them: div u = tr S (Eq. strainRate) and S_m
 * (Sec. 4.1), [ny][nx] each; S_m is NaN at nodes with a neighbour beyond a
 * wall.  Either pointer may be NULL. */
int orc_div_fields(const orc_sim *s, double *div, double *sm);
/* Post-streaming distributions at the current level, the five Euler-history
 * products H = (phi u, phi v, u m_x, v m_y, u m_y + v m_x) of the previous
 * level, and phi at the previous level; any pointer may be NULL. */
int orc_get_state(const orc_sim *s, double *f, double *g, double *H, double *phi_prev, long *step);
/* Load a state given post-streaming f, g at level `step` and phi, u of level
 * step-1 (ignored when step == 0); the history products are recomputed here
 * from phi_prev with this file's own stencil and closure. */
int orc_set_state(orc_sim *s, const double *f, const double *g, const double *phi_prev,
                  const double *u_prev, long step);
/* As orc_set_state, with m^phiC of level step-1 (m_prev, [2][n]) given rather
 * than recomputed: the local gradient scheme's history (required for it when
 * step > 0; orc_set_state refuses that case with -8). */
int orc_set_state_m(orc_sim *s, const double *f, const double *g, const double *phi_prev,
                    const double *u_prev, const double *m_prev, long step);
/* Resolved relaxation rates: s_f (9) and constant part of s_g (9; entries 7, 8
 * are -1 when they follow the local viscosity). */
int orc_rates(const orc_sim *s, double sf[9], double sg[9]);

/* OpenMP threads the oracle's loops use. */
int orc_num_threads(void);
void orc_set_threads(int n);   /* OpenMP threads of the following calls (n > 0) */

/* ---- building blocks exposed for the pins ---- */
/* grad phi of the current level as the step uses it (the stencil, or Eq.
 * local for the local gradient scheme at levels >= 1). */
int orc_grad(const orc_sim *s, double *gx, double *gy);
/* m^phiC of the current level (zero for the original and corrected models). */
int orc_flux(const orc_sim *s, double *mx, double *my);
/* a of the corrected model's interface force F_a = a u, current level (zero
 * for the other models). */
int orc_fa(const orc_sim *s, double *a);
/* grad phi and lap phi of an arbitrary field with this lattice's ghost rule. */
int orc_stencils(const orc_sim *s, const double *phi, double *gx, double *gy, double *lap);
void orc_lattice(int cx[9], int cy[9], double w[9], double M[81], double Minv[81]);
/* Wetting wall value and ghost value for one wall-normal line (Eq. Dwetting). */
void orc_wetting(const orc_params *p, double theta, double phi1, double phi2, double *phi_w, double *phi_g);
/* Equilibrium/source moments (App. C) for given macroscopic values. */
void orc_moments_f(const orc_params *p, double phi, double u, double v, double lam_nx, double lam_ny,
                   double dphiu, double dphiv, double meq[9], double mR[9]);
/* Cahn-Hilliard equilibrium/source moments (App. C, Eq. MfMRCH1). */
void orc_moments_f_ch(const orc_params *p, double phi, double mu, double u, double v, double dphiu,
                      double dphiv, double meq[9], double mR[9]);
void orc_moments_g(const orc_params *p, double rho, double pr, double u, double v, double mx, double my,
                   double Fx, double Fy, double drx, double dry, double dP_um_x, double dP_vm_y,
                   double dP_cross, double meq[9], double mF[9]);
/* One node of the collision in moment form (Eq. evoPF; Remark 2 for g):
 * out = M1^-1 [(I - S) M1 fv + S meq + (I - S/2) mR]. */
void orc_collide_node(const double S[9], const double fv[9], const double meq[9], const double mR[9],
                      double out[9]);
/* Direct (Sec. 3) forms: g^eq_i (Eq. geq) and F_i with M_2F in the second way of Remark 1. */
void orc_direct_g(const orc_params *p, double rho, double pr, double u, double v, double mx, double my,
                  double Fx, double Fy, double drx, double dry, double dP_um_x, double dP_vm_y,
                  double dP_cross, double geq[9], double Fi[9]);

#ifdef __cplusplus
}
#endif
#endif
