// lbm_api.hip -- extern "C" entry points of liblbm (declared in include/lbm.h):
// parameter validation, resolution of the paper's parameters into kernel
// constants, state layout and dispatch to the gfx950 kernels.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_kernels.hpp"

namespace lbm {

static size_t elem_size(int dtype) { return dtype == LBM_F64 ? 8 : 4; }

// Workgroups of the diagnostics kernels (64 x 8 tiles), one partial record each.
size_t diag_blocks(const lbm_params* p) { return (size_t)((p->nx + 63) / 64) * ((p->ny + 7) / 8); }

Layout layout_of(const lbm_params* p) {
    return make_layout(p->nx, p->ny, elem_size(p->dtype), diag_blocks(p), p->grad_scheme == LBM_GRAD_LOCAL ? 5 : 3);
}

int validate(const lbm_params* p) {
    if (!p) return LBM_E_NULL;
    if (p->dtype != LBM_F32 && p->dtype != LBM_F64) return LBM_E_DTYPE;
    if (p->nx < 1 || p->ny < 1) return LBM_E_SIZE;
    if ((long long)p->nx * p->ny > (1LL << 34)) return LBM_E_SIZE;
    if (p->bc_x != LBM_PERIODIC && p->bc_x != LBM_WALLS) return LBM_E_PARAM;
    if (p->bc_y != LBM_PERIODIC && p->bc_y != LBM_WALLS) return LBM_E_PARAM;
    if (p->bc_x == LBM_WALLS && p->nx < 2) return LBM_E_SIZE;
    if (p->bc_y == LBM_WALLS && p->ny < 2) return LBM_E_SIZE;
    if (p->visc_law != LBM_VISC_LINEAR_MU && p->visc_law != LBM_VISC_INVERSE_NU) return LBM_E_PARAM;
    if (p->phase_eq != LBM_ALLEN_CAHN && p->phase_eq != LBM_CAHN_HILLIARD) return LBM_E_PARAM;
    if (p->reserved != 0) return LBM_E_PARAM;
    if (p->grad_scheme != LBM_GRAD_STENCIL && p->grad_scheme != LBM_GRAD_LOCAL) return LBM_E_PARAM;
    if (p->grad_scheme == LBM_GRAD_LOCAL && p->phase_eq != LBM_ALLEN_CAHN) return LBM_E_UNSUPPORTED;
    if (p->model != LBM_MODEL_PRESENT && p->model != LBM_MODEL_ORIGINAL && p->model != LBM_MODEL_CORRECTED)
        return LBM_E_UNSUPPORTED;
    if (p->model == LBM_MODEL_CORRECTED && p->grad_scheme == LBM_GRAD_LOCAL) return LBM_E_UNSUPPORTED;
    const double vals[] = {p->phi_A, p->phi_B, p->rho_A, p->rho_B, p->nu_A, p->nu_B, p->sigma, p->W,
                           p->M_phi, p->eta, p->body_force[0], p->body_force[1], p->gravity[0],
                           p->gravity[1], p->rho_ref, p->rho0, p->eps_n};
    for (double v : vals)
        if (!isfinite(v)) return LBM_E_PARAM;
    if (!(p->phi_A > p->phi_B)) return LBM_E_PARAM;
    if (!(p->rho_A > 0 && p->rho_B > 0 && p->nu_A > 0 && p->nu_B > 0)) return LBM_E_PARAM;
    if (!(p->W > 0 && p->sigma >= 0 && p->M_phi >= 0 && p->eps_n >= 0)) return LBM_E_PARAM;
    if (p->eta != 1.0) return LBM_E_PARAM;
    for (int i = 0; i < 9; i++) {
        if (!isfinite(p->s_f[i]) || !isfinite(p->s_g[i])) return LBM_E_PARAM;
        if (p->s_f[i] >= 2.0 || p->s_g[i] >= 2.0) return LBM_E_UNSTABLE;
    }
    for (int k = 0; k < 4; k++)
        if (!(p->theta[k] > 0 && p->theta[k] < M_PI)) return LBM_E_PARAM;
    // default rates must be stable: s = 1/(x/cs^2 + 1/2) lies in (0, 2) for x > 0
    if (!(p->s_f[3] > 0 && p->s_f[5] > 0) && !(p->M_phi > 0)) return LBM_E_UNSTABLE;
    return LBM_OK;
}

// The collision with the default rates compiled in (KParams::rates_std):
// LBM_STD_RATES = 1 for FP32 and FP64, 2 for FP32 only, 0 never.
#ifndef LBM_STD_RATES
#define LBM_STD_RATES 1
#endif
static bool std_rates_enabled(size_t esz) { return LBM_STD_RATES == 1 || (LBM_STD_RATES == 2 && esz == 4); }

template <typename T>
KParams<T> resolve(const lbm_params* p, const Layout& L) {
    KParams<T> K;
    memset(&K, 0, sizeof(K));
    K.nx = p->nx;
    K.ny = p->ny;
    K.wall_x = p->bc_x == LBM_WALLS;
    K.wall_y = p->bc_y == LBM_WALLS;
    K.visc_law = p->visc_law;
    K.model = p->model;
    K.pf = p->phase_eq;
    K.grad = p->grad_scheme;
    K.plane = L.plane;
    const double dphi = p->phi_A - p->phi_B;
    // Sec. 2: beta = 12 sigma / (W dphi^4), k = 3 sigma W / (2 dphi^2), sqrt(2 beta / k) = 4 / (W dphi)
    const double beta = 12.0 * p->sigma / (p->W * dphi * dphi * dphi * dphi);
    const double kap = 1.5 * p->sigma * p->W / (dphi * dphi);
    K.phiA = (T)p->phi_A;
    K.phiB = (T)p->phi_B;
    K.phim = (T)(0.5 * (p->phi_A + p->phi_B));
    K.beta4 = (T)(4.0 * beta);
    K.kap = (T)kap;
    K.lamc = (T)(4.0 / (p->W * dphi));
    const double drho = (p->rho_A - p->rho_B) / dphi;
    K.drho = (T)drho;
    K.rhoB = (T)p->rho_B;
    K.drhoM = (T)(drho * p->M_phi);
    K.Mphi = (T)p->M_phi;
    K.Aloc = (T)(-p->M_phi - 0.5 / 3.0);
    K.inv_dphi = (T)(1.0 / dphi);
    K.muA = (T)(p->rho_A * p->nu_A);
    K.muB = (T)(p->rho_B * p->nu_B);
    K.inv_nuA = (T)(1.0 / p->nu_A);
    K.inv_nuB = (T)(1.0 / p->nu_B);
    // Sec. 4 preamble: rates of the mobility and the viscosity, the others 1.
    const double cs2 = 1.0 / 3.0;
    double sf[9], sg[9];
    for (int i = 0; i < 9; i++) {
        sf[i] = p->s_f[i] > 0 ? p->s_f[i] : 1.0;
        sg[i] = p->s_g[i] > 0 ? p->s_g[i] : 1.0;
    }
    const double sM = 1.0 / (p->M_phi / (p->eta * cs2) + 0.5);
    if (!(p->s_f[3] > 0)) sf[3] = sM;
    if (!(p->s_f[5] > 0)) sf[5] = sM;
    K.snu_local = !(p->s_g[7] > 0 && p->s_g[8] > 0);
    for (int i = 0; i < 9; i++) {
        K.sf[i] = (T)sf[i];
        K.sg[i] = (T)sg[i];
    }
    K.rates_std = std_rates_enabled(sizeof(T)) && sf[0] == 1.0 && sf[1] == 1.0 && sf[2] == 1.0 && sf[4] == 1.0 && sf[6] == 1.0 && sf[7] == 1.0 &&
                  sf[8] == 1.0 && sg[0] == 1.0 && sg[1] == 1.0 && sg[2] == 1.0 && sg[3] == 1.0 && sg[5] == 1.0;
    K.Gx = (T)p->body_force[0];
    K.Gy = (T)p->body_force[1];
    K.gx = (T)p->gravity[0];
    K.gy = (T)p->gravity[1];
    K.rho_ref = (T)p->rho_ref;
    // Eq. (Dwetting): a = 4 cos(theta) / (W dphi), b = 8/3 - a (phiA + phiB), c = a phiA phiB + ...
    for (int k = 0; k < 4; k++) {
        const double a = 4.0 * cos(p->theta[k]) / (p->W * dphi);
        K.wa[k] = (T)a;
        K.wb[k] = (T)(8.0 / 3.0 - a * (p->phi_A + p->phi_B));
        K.wc0[k] = (T)(a * p->phi_A * p->phi_B);
        K.wda[k] = (T)(-4.0 * sin(p->theta[k]) / (p->W * dphi));
    }
    K.rho0 = (T)p->rho0;
    K.eps2 = (T)(p->eps_n * p->eps_n);
    K.Hp = (T)((sg[2] - sg[0]) / (9.0 * sg[0] * sg[2]));
    K.rest_w = p->phase_eq == LBM_CAHN_HILLIARD ? 1.0 : 4.0 / 9.0;
    return K;
}

template KParams<float> resolve<float>(const lbm_params*, const Layout&);
template KParams<double> resolve<double>(const lbm_params*, const Layout&);

// Shape of the step launch: 64 x TY tiles on workgroups of 64 x BY threads.
// Taller tiles amortise the one-node halo ring; more waves hide latency.
// Measured on MI355X (FP32): lattices of >= 2048 16-row tiles run best at
// (8, 8) (30.9 GLUPS on 4096^2, within 3.5% of every other shape; 26.1 vs 25.1
// at (16, 8) on 2048 x 1024); below that the step is latency bound and the
// tallest tile that still gives >= 4096 waves wins: (16, 8) for 1024 x 512
// (27.2 vs 21.8 at (8, 8)), (8, 8) for 256 x 1024 (27.4 vs 25.5 at (16, 8)),
// else (4, 4).  FP64 tiles stop at 8 rows
// (taller ones spill); (8, 4) measured best for FP64.
#ifndef LBM_STEP_TY
#define LBM_STEP_TY 0   // force a tile height (4, 8, 16); 0 = by lattice size
#endif
#ifndef LBM_STEP_BY
#define LBM_STEP_BY 0   // force thread rows per workgroup (4, 8); 0 = by lattice size
#endif
void step_shape(const lbm_params* p, int* ty, int* by) {
    const long long tx = (p->nx + 63) / 64;
    const long long t16 = tx * ((p->ny + 15) / 16), t8 = tx * ((p->ny + 7) / 8);
    int t, b;
    if (p->dtype == LBM_F64) {
        t = 8;
        b = 4;
    } else if (t16 >= 2048) {
        t = 8;
        b = 8;
    } else if (t16 * 8 >= 4096) {
        t = 16;
        b = 8;
    } else if (t8 * 8 >= 4096) {
        t = 8;
        b = 8;
    } else {
        t = 4;
        b = 4;
    }
    if (LBM_STEP_TY) t = LBM_STEP_TY;
    if (LBM_STEP_BY) b = LBM_STEP_BY;
    if (p->dtype == LBM_F64 && t > 8) t = 8;
    if (b > t) b = 4;
    *ty = t;
    *by = b;
}

int step_tile_rows(const lbm_params* p) {
    int t, b;
    step_shape(p, &t, &b);
    return t;
}

static thread_local char g_last_error[256];

// Captured graphs of GRAPH_K plain steps, reused while (params, state, stream,
// tile height) match; a small most-recently-used cache.
constexpr int GRAPH_K = 32;
constexpr size_t GRAPH_CACHE = 256;
struct StepGraph {
    lbm_params p;
    void* state;
    hipStream_t stream;
    int ty, by;
    int copy;             // the copy the graph's first launch expects the state in
    hipGraphExec_t exec;
};
static std::mutex g_graph_mu;
static std::vector<StepGraph> g_graphs;   // front = most recent

// The copy each state was last left in by lbm_init, lbm_import_state and
// lbm_step, as far as this library knows: the step kernel takes it as the
// guess of which copy to start loading from.  A state the record does not
// know (or knows wrongly: a device copy restored as a checkpoint, a state
// stepped through a replayed graph an odd number of launches) still steps
// correctly, only without the head start.  A small most-recently-used list.
constexpr size_t COPY_RECORDS = 1024;
static std::mutex g_copy_mu;
static std::vector<std::pair<const void*, int>> g_copies;   // front = most recent

int copy_guess(const void* state) {
    std::lock_guard<std::mutex> lock(g_copy_mu);
    for (const auto& e : g_copies)
        if (e.first == state) return e.second;
    return 0;
}

void copy_record(const void* state, int copy) {
    std::lock_guard<std::mutex> lock(g_copy_mu);
    for (size_t i = 0; i < g_copies.size(); i++)
        if (g_copies[i].first == state) {
            g_copies.erase(g_copies.begin() + i);
            break;
        }
    if (g_copies.size() == COPY_RECORDS) g_copies.pop_back();
    g_copies.insert(g_copies.begin(), std::make_pair(state, copy));
}

int hip_fail(hipError_t e) {
    snprintf(g_last_error, sizeof g_last_error, "%s", hipGetErrorString(e));
    return LBM_E_HIP;
}

}  // namespace lbm

using namespace lbm;

extern "C" {

const char* lbm_status_string(int s) {
    switch (s) {
        case LBM_OK: return "ok";
        case LBM_E_NULL: return "null pointer";
        case LBM_E_SIZE: return "invalid size";
        case LBM_E_DTYPE: return "invalid dtype";
        case LBM_E_PARAM: return "invalid parameter";
        case LBM_E_UNSTABLE: return "relaxation rate outside (0, 2)";
        case LBM_E_HIP: return g_last_error[0] ? g_last_error : "HIP runtime error";
        case LBM_E_NONFINITE: return "non-finite value in the state";
        case LBM_E_UNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

int lbm_state_size(const lbm_params* p, size_t* nbytes) {
    int rc = validate(p);
    if (rc) return rc;
    if (!nbytes) return LBM_E_NULL;
    *nbytes = layout_of(p).total;
    return LBM_OK;
}

int lbm_init(const lbm_params* p, void* state, const void* phi0, const void* u0, const void* p0,
             void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state || !phi0) return LBM_E_NULL;
    if ((uintptr_t)state % 256) return LBM_E_SIZE;
    Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (p->dtype == LBM_F32)
        e = launch_init<float>(resolve<float>(p, L), (char*)state, L, (const float*)phi0, (const float*)u0,
                               (const float*)p0, p->dtype, s);
    else
        e = launch_init<double>(resolve<double>(p, L), (char*)state, L, (const double*)phi0,
                                (const double*)u0, (const double*)p0, p->dtype, s);
    copy_record(state, 0);
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_hydrostatic_pressure(const lbm_params* p, const void* phi0, void* p0, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!phi0 || !p0) return LBM_E_NULL;
    if (p->gravity[0] != 0.0) return LBM_E_UNSUPPORTED;
    Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (p->dtype == LBM_F32)
        e = launch_hydrostatic<float>(resolve<float>(p, L), (const float*)phi0, (float*)p0, s);
    else
        e = launch_hydrostatic<double>(resolve<double>(p, L), (const double*)phi0, (double*)p0, s);
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_step(const lbm_params* p, void* state, int64_t nsteps, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state) return LBM_E_NULL;
    if (nsteps < 0) return LBM_E_SIZE;
    Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    int ty, by;
    step_shape(p, &ty, &by);
    int copy = copy_guess(state);
    auto launch = [&](int64_t n, int& c) -> hipError_t {
        if (p->dtype == LBM_F32) return launch_step<float>(resolve<float>(p, L), (char*)state, L, n, s, ty, by, c);
        return launch_step<double>(resolve<double>(p, L), (char*)state, L, n, s, ty, by, c);
    };
    hipError_t e;
    // Long runs on a non-NULL stream replay a graph of GRAPH_K steps, unless the
    // caller is capturing that stream itself (the plain launches then go into
    // the caller's graph).
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s != nullptr && nsteps >= 2 * GRAPH_K) {
        e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (s != nullptr && nsteps >= 2 * GRAPH_K && cs == hipStreamCaptureStatusNone) {
        std::lock_guard<std::mutex> lock(g_graph_mu);
        size_t hit = g_graphs.size();
        for (size_t i = 0; i < g_graphs.size(); i++)
            if (g_graphs[i].state == state && g_graphs[i].stream == s && g_graphs[i].ty == ty && g_graphs[i].by == by &&
                g_graphs[i].copy == copy && memcmp(&g_graphs[i].p, p, sizeof(lbm_params)) == 0) {
                hit = i;
                break;
            }
        if (hit == g_graphs.size()) {
            hipGraph_t g;
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e);
            int c = copy;
            hipError_t le = launch(GRAPH_K, c);
            e = hipStreamEndCapture(s, &g);
            if (le != hipSuccess) return hip_fail(le);
            if (e != hipSuccess) return hip_fail(e);
            // GRAPH_K is even and so is the launch count of every path: a replay
            // leaves the state in the copy it found it in
            if (c != copy) return hip_fail(hipErrorUnknown);
            StepGraph sg{*p, state, s, ty, by, copy, nullptr};
            e = hipGraphInstantiate(&sg.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(e);
            if (g_graphs.size() == GRAPH_CACHE) {
                (void)hipGraphExecDestroy(g_graphs.back().exec);
                g_graphs.pop_back();
            }
            g_graphs.insert(g_graphs.begin(), sg);
            hit = 0;
        } else if (hit != 0) {
            StepGraph sg = g_graphs[hit];
            g_graphs.erase(g_graphs.begin() + hit);
            g_graphs.insert(g_graphs.begin(), sg);
            hit = 0;
        }
        for (int64_t t = 0; t + GRAPH_K <= nsteps; t += GRAPH_K) {
            e = hipGraphLaunch(g_graphs[0].exec, s);
            if (e != hipSuccess) return hip_fail(e);
        }
        nsteps %= GRAPH_K;
    }
    e = launch(nsteps, copy);
    copy_record(state, copy);
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_levels_per_launch(const lbm_params* p, int32_t* levels) {
    int rc = validate(p);
    if (rc) return rc;
    if (!levels) return LBM_E_NULL;
    *levels = two_level_path(layout_of(p), p->nx, p->ny, p->phase_eq, p->model, p->grad_scheme) ? 2 : 1;
    return LBM_OK;
}

int lbm_moments(const lbm_params* p, const void* state, void* phi, void* u, void* pr, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state) return LBM_E_NULL;
    Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (p->dtype == LBM_F32)
        e = launch_moments<float>(resolve<float>(p, L), (const char*)state, L, (float*)phi, (float*)u,
                                  (float*)pr, s);
    else
        e = launch_moments<double>(resolve<double>(p, L), (const char*)state, L, (double*)phi, (double*)u,
                                   (double*)pr, s);
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_diagnostics(const lbm_params* p, const void* state, double* out, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state || !out) return LBM_E_NULL;
    Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (p->dtype == LBM_F32)
        e = launch_diagnostics<float>(resolve<float>(p, L), (const char*)state, L, out, s);
    else
        e = launch_diagnostics<double>(resolve<double>(p, L), (const char*)state, L, out, s);
    if (e != hipSuccess) return hip_fail(e);
    return out[5] != 0.0 ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_export_state(const lbm_params* p, const void* state, void* f, void* g, void* hist, int64_t* step,
                     void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state) return LBM_E_NULL;
    Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (f || g || hist) {
        if (p->dtype == LBM_F32)
            e = launch_export<float>(resolve<float>(p, L), (const char*)state, L, (float*)f, (float*)g,
                                     (float*)hist, s);
        else
            e = launch_export<double>(resolve<double>(p, L), (const char*)state, L, (double*)f, (double*)g,
                                      (double*)hist, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (step) {
        int64_t sv = 0;
        e = hipMemcpyAsync(&sv, (const char*)state + L.off_stamp, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e);
        *step = stamp_level(sv);
    }
    return LBM_OK;
}

int lbm_import_state(const lbm_params* p, void* state, const void* f, const void* g, const void* hist,
                     int64_t step, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state || !f || !g) return LBM_E_NULL;
    if (step < 0) return LBM_E_SIZE;
    if (step > 0 && !hist) return LBM_E_NULL;
    if ((uintptr_t)state % 256) return LBM_E_SIZE;
    Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (p->dtype == LBM_F32)
        e = launch_import<float>(resolve<float>(p, L), (char*)state, L, (const float*)f, (const float*)g,
                                 (const float*)hist, step, p->dtype, s);
    else
        e = launch_import<double>(resolve<double>(p, L), (char*)state, L, (const double*)f,
                                  (const double*)g, (const double*)hist, step, p->dtype, s);
    copy_record(state, (int)(step & 1));
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

}  // extern "C"
