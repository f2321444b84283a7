/*
 * lbm.h -- C ABI of liblbm, an MI355X (gfx950) implementation of the
 * consistent and conservative phase-field lattice Boltzmann method of
 * Zhan, Chai & Shi, "Consistent and conservative phase-field based lattice
 * Boltzmann method for incompressible two-phase flows" (arXiv:2111.00847).
 *
 * One time step advances two D2Q9 populations:
 *   f -- conservative Allen-Cahn phase field, MRT collision in moment space
 *        (Sec. 3, Eq. evoPF; App. C, Eq. MfMRAC1),
 *   g -- incompressible flow with the consistent mass flux
 *        m^CC = rho u + m^phiC, m^phiC = -(drho/dphi) M (grad phi - lambda n)
 *        (Sec. 2; Sec. 3, Eq. evoNS, Remark 2; App. C, Eq. MgMF1),
 * with isotropic gradient / Laplacian stencils (App. C, Eqs. central1,
 * central2), explicit-Euler time derivatives (App. C), the pressure of
 * Eq. computP in the second way of Remark 1, half-way bounce-back and the
 * wetting boundary condition of Eq. Dwetting (Sec. 4.3).
 * Options (lbm_params): the Cahn-Hilliard phase field (phase_eq), the original
 * and corrected comparison models (model) and the local gradient scheme of
 * Eq. local (grad_scheme); each entry point states which it covers.
 *
 * Conventions (all entry points):
 *  - Lattice units: dx = dt = c = 1, cs^2 = 1/3.
 *  - Fields are row-major [ny][nx], x fastest, y = 0 the bottom row; vector
 *    fields are [2][ny][nx] (x component first); distributions are
 *    [9][ny][nx] with c0..c8 = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),
 *    (-1,-1),(1,-1) (the column order of M1 in App. C).
 *  - Every array argument has the element type selected by lbm_params.dtype
 *    (float or double) unless stated otherwise, and is DEVICE memory unless
 *    stated otherwise.  The caller owns every buffer; the library never
 *    allocates or frees caller memory and keeps no pointer after returning.
 *    The only library-owned objects are lbm_batch plans.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous on it unless documented as synchronising.
 *  - Validation is synchronous and returns a negative lbm_status; a failing
 *    HIP call returns LBM_E_HIP.  No C++ exception crosses the ABI.
 *  - A state buffer is opaque: its size is given by lbm_state_size, it must
 *    be 256-byte aligned, it is written only by lbm_init / lbm_import_state /
 *    lbm_step, and it holds everything a step needs (both ping-pong copies of
 *    the populations, the Euler history, the level stamps).  A device-to-
 *    device copy of it is a checkpoint; a state may only be used with the
 *    lbm_params it was initialised with.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_E_NULL = -1,        /* a required pointer is NULL */
    LBM_E_SIZE = -2,        /* grid or buffer size invalid (nx, ny < 1; < 2 across a wall axis) */
    LBM_E_DTYPE = -3,       /* dtype not LBM_F32 / LBM_F64 */
    LBM_E_PARAM = -4,       /* physical parameter invalid (rho, nu, W <= 0, phi_A <= phi_B, eta != 1, ...) */
    LBM_E_UNSTABLE = -5,    /* a relaxation rate outside (0, 2): tau <= 1/2 */
    LBM_E_HIP = -6,         /* a HIP runtime call failed */
    LBM_E_NONFINITE = -7,   /* diagnostics found a NaN or Inf in the state */
    LBM_E_UNSUPPORTED = -8  /* option not implemented (e.g. a model flag) */
} lbm_status;

typedef enum { LBM_F32 = 0, LBM_F64 = 1 } lbm_dtype;
typedef enum { LBM_PERIODIC = 0, LBM_WALLS = 1 } lbm_bc;
typedef enum {
    LBM_VISC_LINEAR_MU = 0,   /* linear dynamic viscosity, Sec. 2, Eq. linearMu (the paper's default) */
    LBM_VISC_INVERSE_NU = 1   /* inverse-linear kinematic viscosity, Sec. 2, Eq. inverseNu */
} lbm_visc;
typedef enum {
    LBM_MODEL_PRESENT = 0,    /* consistent mass flux m^CC (the paper's model) */
    LBM_MODEL_ORIGINAL = 1,   /* mass flux rho u only (m^phiC = 0 in the flow model; Sec. 4 preamble) */
    LBM_MODEL_CORRECTED = 2   /* mass flux rho u plus the interface force F_a = (drho/dphi) u div(M_phi D)
                                 (Sec. 4 preamble; App. A, Eq. NS2-add); u solves Eq. comU with
                                 F = F_0 + F_a exactly.  Cahn-Hilliard: div(M_phi D) = M_phi lap mu_phi
                                 (Eq. central2).  Allen-Cahn: div D of D = grad phi - lambda n by Eq.
                                 central1, a wall mirroring D with its normal component reversed.
                                 Not with the local gradient scheme or the reverse mode
                                 (LBM_E_UNSUPPORTED) */
} lbm_model;

typedef enum {
    LBM_ALLEN_CAHN = 0,       /* conservative Allen-Cahn: D = grad phi - lambda n (Sec. 2, Eq. ACE; Eq. MfMRAC1) */
    LBM_CAHN_HILLIARD = 1     /* Cahn-Hilliard: D = grad mu_phi (Sec. 2, Eq. CHE; Eq. MfMRCH1); mu_phi has
                                 zero normal derivative at walls; the reverse mode is AC only */
} lbm_phase_eq;

typedef enum {
    LBM_GRAD_STENCIL = 0,     /* grad phi by the isotropic central scheme (Eq. central1) */
    LBM_GRAD_LOCAL = 1        /* grad phi from the first moment of f by the local scheme of Eq. local
                                 (Allen-Cahn only; level 0 and lap phi keep the stencils).  u depends on
                                 grad phi through F_s = mu_phi grad phi, which folds into the scheme's
                                 coefficient: C0 = sum_i c_i f_i - phi u0/2 - (phi u)^{n-1}/2 = A' grad phi
                                 + B n with A' = -M_phi - cs^2/2 + phi mu_phi/(4 rho), B = M_phi lambda,
                                 u0 the velocity without F_s; |grad phi| = (|C0| + B)/(-A') clamped at 0.
                                 The history then holds m^phiC of the previous level too (22 planes per
                                 copy instead of 20).  Every call but the reverse mode (LBM_E_UNSUPPORTED);
                                 export and import carry the five history planes */
} lbm_grad;

/* Problem statement in the paper's notation (Sec. 2; Sec. 4 preamble). */
typedef struct lbm_params {
    int32_t nx, ny;                 /* lattice nodes */
    int32_t dtype;                  /* lbm_dtype: element type of state and fields */
    int32_t bc_x, bc_y;             /* lbm_bc per axis; WALLS = half-way bounce-back on both faces */
    int32_t visc_law;               /* lbm_visc */
    int32_t model;                  /* lbm_model */
    int32_t phase_eq;               /* lbm_phase_eq: phase-field equation */
    int32_t grad_scheme;            /* lbm_grad: scheme of grad phi */
    int32_t reserved;               /* must be 0 */
    double phi_A, phi_B;            /* order parameter of the two bulk phases, phi_A > phi_B */
    double rho_A, rho_B;            /* densities (Eq. rho-phi) */
    double nu_A, nu_B;              /* kinematic viscosities; mu = rho nu */
    double sigma, W, M_phi, eta;    /* surface tension, interface width, mobility; eta must be 1 */
    double s_f[9], s_g[9];          /* MRT rates; an entry <= 0 selects the paper's default:
                                       s_f^3 = s_f^5 = 1/(M_phi/(eta cs^2) + 1/2),
                                       s_g^7 = s_g^8 = 1/(nu(phi)/cs^2 + 1/2) per node,
                                       all others 1 (Sec. 4 preamble) */
    double body_force[2];           /* uniform force density G (Sec. 4.2) */
    double gravity[2];              /* adds (rho - rho_ref) * gravity to F (Secs. 4.4, 4.5) */
    double rho_ref;
    double theta[4];                /* contact angle [rad] at the x-, x+, y-, y+ walls (Sec. 4.3);
                                       pi/2 is the neutral (no-flux) wall */
    double rho0;                    /* constant density of g^eq (Eq. geq); a gauge, 0 is best for FP32 */
    double eps_n;                   /* n = grad phi / sqrt(|grad phi|^2 + eps_n^2) */
} lbm_params;

/* Human-readable name of a status code (static storage). */
const char *lbm_status_string(int status);

/* Bytes of device memory the caller must provide for one lattice's state. */
int lbm_state_size(const lbm_params *p, size_t *nbytes /* host */);

/* Initial state f = f^eq(phi0, u0), g = g^eq(phi0, u0, p0) (equilibria of
 * Eq. MfMRAC1 -- Eq. MfMRCH1 for Cahn-Hilliard -- and Eq. MgMF1 at the given
 * fields; the Euler time derivatives of the first step are zero).  phi0:
 * [ny][nx]; u0: [2][ny][nx] or NULL (zero); p0: [ny][nx] or NULL (zero).
 * Every option. */
int lbm_init(const lbm_params *p, void *state, const void *phi0, const void *u0, const void *p0,
             void *stream);

/* Initial pressure of the two fluids at rest under gravity (the gravity-driven
 * set-ups of Secs. 4.4 and 4.5 leave it unstated; read as hydrostatic): with
 * rho from the density law of Sec. 2 at phi0, p0 integrates
 * dp/dy = (rho - rho_ref) gravity[1] down every column by the trapezoid rule
 * from the top row, in FP64, then takes the mean out.  phi0, p0: [ny][nx];
 * zero gravity gives p0 = 0.  gravity[0] != 0: LBM_E_UNSUPPORTED.  Runs as one
 * workgroup (an initialisation call, not a per-step one). */
int lbm_hydrostatic_pressure(const lbm_params *p, const void *phi0, void *p0, void *stream);

/* Advance nsteps >= 0 time steps (Sec. 3): moments, closure, both MRT
 * collisions and streaming with bounce-back, fused in one kernel per step --
 * or per two steps, for the Allen-Cahn step with stencil or local gradients
 * (present and original models) on a lattice of at least 256 tiles of 64 x 8
 * nodes whose state copy is below 4 GiB, cache-resident or streamed from HBM
 * (lbm_levels_per_launch; the environment variable LBM_TWO_LEVEL = "0" or "1"
 * turns the size rule off or on for every such state): a run of n steps is
 * then n / 2 two-level launches and, for odd n, one one-level launch, with
 * results equal bit for bit to n one-level launches.  On a non-NULL stream, runs of >= 64 steps
 * replay a captured graph of 32 steps (cached per params, state and stream);
 * while the caller captures the stream itself, the kernels are launched into
 * the caller's graph instead.  Every option. */
int lbm_step(const lbm_params *p, void *state, int64_t nsteps, void *stream);

/* Time levels that one step launch of lbm_step advances for these params
 * (1 or 2; see lbm_step).  Host only, no device work. */
int lbm_levels_per_launch(const lbm_params *p, int32_t *levels /* host */);

/* Order parameter, velocity (Eq. comU) and pressure (Eq. computP) of the
 * current time level.  phi, p: [ny][nx] or NULL; u: [2][ny][nx] or NULL.
 * Every option. */
int lbm_moments(const lbm_params *p, const void *state, void *phi, void *u, void *pr,
                void *stream);

/* Diagnostics of the current level (Sec. 4.1), FP64, written to HOST out[6]:
 *   out[0] sum of phi, out[1] max |div u|, out[2] D_u^rms, out[3] S_m^rms,
 *   out[4] max |u|, out[5] 1 if any population is NaN/Inf else 0,
 * with div u = tr S of Eq. strainRate and S_m = d_t rho + div m^CC, where
 * div m^phiC uses Eq. central1 (rms over nodes whose eight neighbours are
 * fluid).  Synchronises the stream.  Returns LBM_E_NONFINITE when out[5] = 1.
 * Every option. */
int lbm_diagnostics(const lbm_params *p, const void *state, double *out /* host [6] */,
                    void *stream);

/* Post-streaming populations f^n, g^n ([9][ny][nx] each, either may be NULL),
 * phi and u of level n-1 (hist: [3][ny][nx] = phi, u, v; [5][ny][nx] with
 * m^phiC_x, m^phiC_y of level n-1 appended for the local gradient scheme; NULL
 * to skip), and the step index n (host int64, NULL to skip).  Synchronises the
 * stream when step is requested. */
int lbm_export_state(const lbm_params *p, const void *state, void *f, void *g, void *hist,
                     int64_t *step, void *stream);

/* Inverse of lbm_export_state: load post-streaming f^n, g^n and the level
 * n-1 history (same planes as lbm_export_state; ignored when n == 0) as the
 * state of step n. */
int lbm_import_state(const lbm_params *p, void *state, const void *f, const void *g,
                     const void *hist, int64_t step, void *stream);

/* ---- reverse mode: tapes and the adjoint step ------------------------------
 * The adjoint of the step map S^n -> S^{n+1} (Sec. 3, as lbm_step computes it)
 * for a loss L(phi^N): given dL/dS^{n+1}, lbm_adjoint_step forms
 * dL/dS^n = (dS^{n+1}/dS^n)^T dL/dS^{n+1} and accumulates dL/d(gravity) and
 * dL/d(theta) of that step.  The adjoint of level n holds dL/df^n, dL/dg^n
 * (post-streaming populations, [9][ny][nx] each) and dL/d(phi, u, v) of the
 * history stored at level n (the fields of level n-1, [3][ny][nx]).
 * A backward pass over levels N-1 .. 0:
 *   lbm_adjoint_phi(state at level N, dL/dphi^N)        -- starts the pass
 *   for each segment, newest first: lbm_tape_record from the segment's first
 *   level, then lbm_adjoint_step(tape, j) for j = L-1 .. 0 (or one lbm_adjoint_run)
 *   lbm_adjoint_init -> dL/dphi0; lbm_adjoint_params -> dL/dgravity, dL/dtheta.
 * Or, with memory for every level, one segment recorded by the forward pass
 * itself (levels 0 .. N, ending on lbm_tape_restore of slot N) and no
 * recomputation in the backward pass.
 * Level mismatches (a step whose tape level is not one below the adjoint's),
 * a slot j the tape does not hold and a tape recorded for another lattice or
 * dtype are detected on the device from the tape's header before any slot is
 * read; the step is skipped and lbm_adjoint_params then returns LBM_E_PARAM.
 * Adjoint and tape buffers are caller-owned device memory, 256-byte aligned,
 * in the dtype of the params.  The reverse mode is
 * that of the Allen-Cahn step with the stencil gradient and the present or
 * original model: every call below returns LBM_E_UNSUPPORTED for other
 * params (Cahn-Hilliard, the local gradient scheme, the corrected model). */

/* Bytes of a tape of `nlevels` consecutive levels. */
int lbm_tape_size(const lbm_params *p, int32_t nlevels, size_t *nbytes /* host */);
/* Record levels n .. n + nlevels - 1 into `tape`, n being the level of
 * `state` (which is not modified): a copy of its current level, then
 * nlevels - 1 ordinary steps run from tape slot to tape slot (bitwise the
 * levels lbm_step would produce). */
int lbm_tape_record(const lbm_params *p, const void *state, void *tape, int32_t nlevels, void *stream);
/* Make tape slot j the current level of `state` (level = the tape's first
 * level + j; the state's other copy is left as it is): with a tape recorded
 * for every level of a trajectory, the forward pass ends here instead of
 * stepping again.  Reads the tape's header back to the host (synchronises the
 * stream): LBM_E_SIZE when the tape holds no slot j, LBM_E_PARAM when it was
 * recorded for another lattice or dtype. */
int lbm_tape_restore(const lbm_params *p, const void *tape, int32_t j, void *state, void *stream);
/* Bytes of an adjoint buffer. */
int lbm_adjoint_size(const lbm_params *p, size_t *nbytes /* host */);
/* Start a backward pass at the level N of `state`: dL/df_i^N = dL/dphi^N for
 * all i (phi = sum_i f_i), all other adjoints and the parameter sums zero.
 * dL_dphi: [ny][nx]. */
int lbm_adjoint_phi(const lbm_params *p, const void *state, void *adj, const void *dL_dphi, void *stream);
/* One adjoint step: adj holds level n + 1 on entry and level n on return,
 * n = (first level of the tape) + j; the forward level n is tape slot j. */
int lbm_adjoint_step(const lbm_params *p, const void *tape, int32_t j, void *adj, void *stream);
/* `count` adjoint steps over tape slots j_first, j_first - 1, ..., j_first - count + 1
 * (the same as that many lbm_adjoint_step calls, launched from one call). */
int lbm_adjoint_run(const lbm_params *p, const void *tape, int32_t j_first, int32_t count, void *adj,
                    void *stream);
/* dL/dphi0 ([ny][nx]) from the adjoint of level 0, through lbm_init with
 * u0 = NULL (f^0 = w_i phi0; p0 is held fixed).  Writes NaN if the adjoint is
 * not at level 0. */
int lbm_adjoint_init(const lbm_params *p, const void *adj, void *dL_dphi0, void *stream);
/* Sums of the parameter derivatives accumulated since the pass started, to
 * HOST out[6] = dL/dgravity[0..1], dL/dtheta[0..3]; `level` (host, may be
 * NULL) receives the adjoint's level.  Synchronises the stream. */
int lbm_adjoint_params(const lbm_params *p, const void *adj, double *out /* host [6] */, int64_t *level,
                       void *stream);
/* Copy the adjoint of the current level out ([9][ny][nx], [9][ny][nx],
 * [3][ny][nx]; any may be NULL), or load one as the adjoint of `level`
 * (NULL arrays load zeros; the parameter sums restart at zero). */
int lbm_adjoint_export(const lbm_params *p, const void *adj, void *fbar, void *gbar, void *hbar, void *stream);
int lbm_adjoint_import(const lbm_params *p, void *adj, const void *fbar, const void *gbar, const void *hbar,
                       int64_t level, void *stream);

/* ---- batches: many independent lattices, one launch per time step ---------
 * (the per-step update above applied to every case).  All cases share one
 * dtype; any option; each case's state copy below 4 GiB (else LBM_E_SIZE: the
 * batch kernels address a case with 32-bit offsets).  Batches holding Cahn-Hilliard,
 * corrected Allen-Cahn or local-gradient cases run tiles of 4 or 8 rows, one
 * node per thread; those cases equal the lone runs to rounding (the tile height may
 * differ), the plain Allen-Cahn cases bitwise.  A batch whose every case runs
 * the plain Allen-Cahn step (stencil gradients, present or original model)
 * advances two levels per launch as lbm_step does (64 x 8 tiles; an odd step
 * count ends on a one-level launch) when it has at least 256 such tiles, or
 * whatever its size with LBM_TWO_LEVEL=1 in the environment when the plan is
 * made (never with LBM_TWO_LEVEL=0).  The plan is
 * library-owned (a small device table of the cases and, once lbm_batch_step
 * runs on a non-NULL stream with nsteps >= 32 that the caller is not
 * capturing, a captured hipGraph of 32 steps for that state and stream). */
typedef struct lbm_batch lbm_batch;

/* Plan a batch of `ncases` lattices (cases: host array of ncases lbm_params).
 * autotune != 0: the first lbm_batch_init times the candidate tile shapes and
 * grid sizes of the one-level batch launch (one workgroup per tile, or fewer
 * workgroups striding over the tiles) on the batch itself and keeps the
 * fastest.  LBM_BATCH_SHAPE="ty,by,grid" in the environment fixes the shape
 * of the one-level launch instead and skips the timing: tile rows ty and
 * thread rows by (4,4 8,4 8,8 16,4 16,8; 16-row tiles in FP32 only; by = ty
 * when the batch holds Cahn-Hilliard, corrected or local-gradient cases) and
 * grid workgroups (0: one per tile); another value makes this call return
 * LBM_E_PARAM. */
int lbm_batch_create(const lbm_params *cases, int32_t ncases, int32_t autotune, lbm_batch **out);
/* Bytes of the caller-allocated batch state (every case's state back to back). */
int lbm_batch_state_size(const lbm_batch *batch, size_t *nbytes /* host */);
/* Byte offset of case c's state inside the batch state: lbm_moments,
 * lbm_diagnostics, lbm_export_state accept (state + offset) with case c's params. */
int lbm_batch_case_offset(const lbm_batch *batch, int32_t c, size_t *offset /* host */);
/* Initialise every case as lbm_init does.  phi0, p0: HOST arrays of ncases
 * device pointers (p0 may be NULL, or hold NULLs).  Runs the autotuner first
 * when requested (it synchronises the stream and overwrites the state). */
int lbm_batch_init(lbm_batch *batch, void *state, const void *const *phi0, const void *const *p0,
                   void *stream);
/* Advance every case by nsteps. */
int lbm_batch_step(lbm_batch *batch, void *state, int64_t nsteps, void *stream);
/* The tuning in use: tile rows, thread rows per 64-wide workgroup, workgroups
 * per launch, work items per step (any pointer may be NULL). */
int lbm_batch_tuning(const lbm_batch *batch, int32_t *tile_rows, int32_t *thread_rows, int32_t *grid,
                     int32_t *items);
/* Levels one launch of the plan advances (1 or 2; host *levels). */
int lbm_batch_levels_per_launch(const lbm_batch *batch, int32_t *levels);
int lbm_batch_destroy(lbm_batch *batch);

/* ---- a batch step that allocates nothing ----------------------------------
 * For callers that cannot allocate: code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.  lbm_batch_step_noalloc advances
 * the cases of a batch state (the layout lbm_batch_state_size and
 * lbm_batch_case_offset give for the same cases, initialised by
 * lbm_batch_init or by lbm_init of every case at its offset) exactly as
 * lbm_batch_step does with an untuned plan of the same cases (8-row tiles,
 * one workgroup per work item, two levels per launch under the same rule,
 * LBM_TWO_LEVEL read at every call), without a plan and without allocating: the
 * case table (at most LBM_NOALLOC_MAX_CASES cases, about 140 KB) lives in a
 * fixed device array of the library that every GPU it runs on holds until
 * the process ends; the call writes it with small kernels on `stream` before
 * its steps.  Every call on one GPU shares that array and it keeps the last
 * call's table: calls that overlap on one GPU (different streams or host
 * threads) race, calls ordered on one stream do not.  No graph is captured
 * or replayed.  Errors: LBM_E_SIZE for more cases than the limit, a state
 * not 256-byte aligned or nsteps < 0; otherwise those of lbm_batch_create. */
#define LBM_NOALLOC_MAX_CASES 256
int lbm_batch_step_noalloc(const lbm_params *cases, int32_t ncases, void *state, int64_t nsteps, void *stream);

/* ---- streaming probe -------------------------------------------------------
 * Not part of the method: the HBM read, write and copy rates of the device,
 * the measured ceiling next to the nominal peak that the step kernels'
 * bandwidth is compared with.  One launch of `blocks` workgroups of 256
 * threads streaming `bytes` (a multiple of 16; 16-byte aligned buffers) with
 * 16-byte loads and stores in a grid-stride loop:
 *   kind 0: read src; dst receives one uint32 per thread (blocks * 1024 bytes);
 *   kind 1: write dst (src unused, may be NULL);
 *   kind 2: copy src to dst.
 * nt != 0: non-temporal stores.  Asynchronous on `stream`.  Errors:
 * LBM_E_PARAM (kind), LBM_E_SIZE (blocks, bytes, alignment), LBM_E_NULL. */
int lbm_bandwidth_probe(int32_t kind, void *dst, const void *src, size_t bytes, int32_t blocks, int32_t nt,
                        void *stream);

#ifdef __cplusplus
}
#endif
#endif
