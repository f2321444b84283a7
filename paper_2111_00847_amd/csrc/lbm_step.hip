// lbm_step.hip -- gfx950 kernels of the fused phase-field LBM time step.
//
// Memory layout (structure of arrays, x fastest): a state buffer is
//   [header | copy 0 | copy 1 | level stamps | diagnostics scratch],
// a copy being f_0 | f_1..f_8 | g_0..g_8 | hist = (phi, u, v), every
// plane padded to a multiple of 64 elements.  The copy that holds level n
// holds the post-collision populations of level n-1 -- a node obtains its
// level-n populations by pulling them from its neighbours -- and the history
// of level n-1, from which the explicit-Euler time derivatives are formed.  A
// launch reads that copy and writes the other.  The level and its copy are
// kept in per-row stamps owned by the workgroups (lbm_common.hpp), so host
// code never needs them, no workgroup waits for another, and a sequence of
// steps can be captured in a graph.
//
// The phi stencils need phi on a one-node ring around each tile.  A tile of
// 64 x TY nodes first pulls the populations of its (64+2) x (TY+2) window,
// sums them into phi in LDS (the ring's pulls hit L2: those lines are the
// neighbour tiles' own reads), fills wall ghosts, and then each thread runs
// the per-node update for its nodes (lbm_fused.hpp).
#include <cstdlib>

#include "lbm_ch_step.hpp"
#include "lbm_fused.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// Steps on states that the last-level cache holds (NT false) start their loads
// on the copy of the host's parity guess `hint` while the level stamp is read
// (step_core); LBM_PARITY_HINT=0 reads the stamp first there too.  States
// streamed from HBM always read the stamp first: a wrong guess would cost a
// whole extra copy of HBM reads (the guess is wrong after every replay of a
// captured graph of an odd number of launches, 1.5x the step time measured on
// 4096 x 4096 FP32), while the stamp read costs a tile little next to its
// stream of loads.
#ifndef LBM_PARITY_HINT
#define LBM_PARITY_HINT 1
#endif

template <typename T, int TY, int MODE, typename OFF, int NBY, bool STD, bool NT = true, bool LATE_G = false>
__global__ __launch_bounds__(TX* NBY) __attribute__((amdgpu_waves_per_eu(StepWaves<T, TY, NBY>::value)))
void k_step(KParams<T> P, char* state, size_t off0, size_t off1, size_t off_stamp, int ntx, int nty, T* out_phi,
            T* out_u, T* out_p, int hint) {
    __shared__ T sphi[TY + 2][TX + 3];
    __shared__ T sphp[TY + 2][TX + 3];
    int xt, yt;
    if (LBM_XCD_REMAP) {
        xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    } else {
        xt = blockIdx.x % ntx;
        yt = blockIdx.x / ntx;
    }
    step_tile<T, TY, MODE, OFF, NBY, STD, NT, LATE_G, MODE == 0 && LBM_PARITY_HINT && !NT>(
        P, state, off0, off1, off_stamp, xt, yt, out_phi, out_u, out_p, sphi, sphp, hint);
}

// The Cahn-Hilliard variant and the corrected comparison model with the
// Allen-Cahn phase field (ACC), both on the two-node phi window of lbm_ch.hpp:
// one 64 x TY tile per workgroup, one node per thread (64 x TY threads; 64 x 8
// for 16 rows), tiles dealt to the XCDs as for the Allen-Cahn step, the same
// state layout, level stamps and store policy.  MODE 0: one time step; MODE 1:
// phi, u, p of the current level.  Tile shape (measured on MI355X, FP32 square
// droplet, us per step): 8 rows on 64 x 8 threads 574 / 39.5 / 9.4 at 4096^2 /
// 1024^2 / 200^2, against 589 / 42.0 / 11.7 for the shapes used before (8 rows
// on 64 x 4 threads with two nodes per thread, 4 rows on 64 x 4 below 1024
// tiles); 16 rows on 64 x 8 threads 575 / 38.2 / 18.4; 16 rows on 64 x 16 656 /
// 43.2 / 14.0.  LBM_CH_TY forces 4, 8 or 16 rows.
#ifndef LBM_CH_TY
#define LBM_CH_TY 0
#endif

template <typename T, int TY, int MODE, bool ACC, bool STD, bool NT = true, int NBY = BY, typename OFF = uint64_t>
__global__ __launch_bounds__(TX* NBY) void k_step_ch(KParams<T> P, char* state, size_t off0, size_t off1,
                                                    size_t off_stamp, int ntx, int nty, T* out_phi, T* out_u,
                                                    T* out_p) {
    __shared__ ChWindow<T, TY> W;
    int xt, yt;
    if (LBM_XCD_REMAP) {
        xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    } else {
        xt = blockIdx.x % ntx;
        yt = blockIdx.x / ntx;
    }
    ch_step_tile<T, TY, MODE, ACC, STD, NT, NBY, OFF>(P, state, off0, off1, off_stamp, xt, yt, out_phi, out_u, out_p,
                                                      W);
}

// Rows of the CH tile (8 unless LBM_CH_TY) and thread rows (one node per thread).
constexpr int CH_TY = (LBM_CH_TY == 4 || LBM_CH_TY == 16) ? LBM_CH_TY : 8;
constexpr int CH_NBY = CH_TY == 4 ? 4 : 8;

template <typename T, int MODE, bool ACC, bool STD, bool NT, typename OFF>
static void launch_ch_shape(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + CH_TY - 1) / CH_TY;
    k_step_ch<T, CH_TY, MODE, ACC, STD, NT, CH_NBY, OFF><<<ntx * nty, dim3(TX, CH_NBY), 0, s>>>(
        P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, ntx, nty, phi, u, p);
}

// Steps address a copy below 4 GiB with 32-bit byte offsets from a uniform
// base, as the Allen-Cahn step does (1323 against 1960 VALU instructions in the
// FP32 kernel, 62 against 68 VGPRs; measured on MI355X, FP32 square droplet, us
// per step: 554 against 571 at 4096^2, 37.0 against 39.7 at 1024^2, 7.0 against
// 9.6 at 200^2); moments and larger copies with 64-bit ones.
template <typename T, int MODE, bool ACC, bool STD, bool NT = true>
static void launch_ch_acc_std(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p) {
    if constexpr (MODE == 0) {
        if (L.buf_bytes < (size_t(1) << 32)) {
            launch_ch_shape<T, MODE, ACC, STD, NT, uint32_t>(P, state, L, s, phi, u, p);
            return;
        }
    }
    launch_ch_shape<T, MODE, ACC, STD, NT, uint64_t>(P, state, L, s, phi, u, p);
}

// the standard rates compiled in for steps (moments do not collide); steps on
// a state that the last-level cache holds store it with ordinary stores
template <typename T, int MODE, bool ACC>
static void launch_ch_acc(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p) {
    if constexpr (MODE == 0) {
        const bool cached = cached_state(L);
        if (P.rates_std) {
            if (cached) launch_ch_acc_std<T, MODE, ACC, true, false>(P, state, L, s, phi, u, p);
            else launch_ch_acc_std<T, MODE, ACC, true>(P, state, L, s, phi, u, p);
        } else {
            if (cached) launch_ch_acc_std<T, MODE, ACC, false, false>(P, state, L, s, phi, u, p);
            else launch_ch_acc_std<T, MODE, ACC, false>(P, state, L, s, phi, u, p);
        }
    } else {
        launch_ch_acc_std<T, MODE, ACC, false>(P, state, L, s, phi, u, p);
    }
}

// CH (any model) or the corrected AC model: the two-node-window kernels.
template <typename T, int MODE>
static void launch_ch(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p) {
    if (P.pf == 1) launch_ch_acc<T, MODE, false>(P, state, L, s, phi, u, p);
    else launch_ch_acc<T, MODE, true>(P, state, L, s, phi, u, p);
}

// ---------------------------------------------------------------- init / import / export
// phi at (x, y) of a caller field, extended by the lattice's ghost rule:
// periodic axes wrap; x-wall ghosts from the row, y-wall ghosts from the
// (possibly x-ghost) column -- the same order as the LDS window.
template <typename T>
__device__ T field_at(const KParams<T>& P, const T* phi, int x, int y) {
    if (!P.wall_x && (x < 0 || x >= P.nx)) x = x < 0 ? x + P.nx : x - P.nx;
    if (!P.wall_y && (y < 0 || y >= P.ny)) y = y < 0 ? y + P.ny : y - P.ny;
    auto col = [&](int xx, int yy) -> T {
        const T* row = phi + (long long)yy * P.nx;
        if (xx < 0) return wet_ghost(P, 0, row[0], row[1]);
        if (xx >= P.nx) return wet_ghost(P, 1, row[P.nx - 1], row[P.nx - 2]);
        return row[xx];
    };
    if (y < 0) return wet_ghost(P, 2, col(x, 0), col(x, 1));
    if (y >= P.ny) return wet_ghost(P, 3, col(x, P.ny - 1), col(x, P.ny - 2));
    return col(x, y);
}

// mu_phi of a caller field at (x, y) (Sec. 2), positions beyond a wall taking
// the value of the first fluid node (x first, then y), periodic axes wrapping.
template <typename T>
__device__ T mu_at(const KParams<T>& P, const T* phi, int x, int y) {
    if (x < 0 || x >= P.nx) x = P.wall_x ? (x < 0 ? 0 : P.nx - 1) : (x < 0 ? x + P.nx : x - P.nx);
    if (y < 0 || y >= P.ny) y = P.wall_y ? (y < 0 ? 0 : P.ny - 1) : (y < 0 ? y + P.ny : y - P.ny);
    T n_[3][3];
    for (int j = 0; j < 3; j++)
        for (int i = 0; i < 3; i++) n_[j][i] = field_at(P, phi, x + i - 1, y + j - 1);
    T gx, gy, lap;
    stencil(n_[0][0], n_[0][1], n_[0][2], n_[1][0], n_[1][1], n_[1][2], n_[2][0], n_[2][1], n_[2][2], gx, gy, lap);
    return chem_pot(P, n_[1][1], lap);
}

// Equilibria at every node into `eq` (f^eq planes 0..8, g^eq planes 9..17).
template <typename T>
__global__ void k_equilibrium(KParams<T> P, const T* phi0, const T* u0, const T* p0, T* eq) {
    const long long n = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / P.nx), x = (int)(k - (long long)y * P.nx);
        T n_[3][3];
        for (int j = 0; j < 3; j++)
            for (int i = 0; i < 3; i++) n_[j][i] = field_at(P, phi0, x + i - 1, y + j - 1);
        T gx, gy, lap;
        stencil(n_[0][0], n_[0][1], n_[0][2], n_[1][0], n_[1][1], n_[1][2], n_[2][0], n_[2][1], n_[2][2],
                gx, gy, lap);
        const T phi = n_[1][1];
        const T u = u0 ? u0[k] : T(0), v = u0 ? u0[n + k] : T(0), p = p0 ? p0[k] : T(0);
        T lnx, lny, mx, my;
        if (P.pf == 1) {   // Cahn-Hilliard: grad mu of the initial field, mu mirrored at walls
            T mn[3][3];
            for (int j = 0; j < 3; j++)
                for (int i = 0; i < 3; i++) mn[j][i] = mu_at(P, phi0, x + i - 1, y + j - 1);
            T gmx, gmy, lm;
            stencil(mn[0][0], mn[0][1], mn[0][2], mn[1][0], mn[1][1], mn[1][2], mn[2][0], mn[2][1], mn[2][2], gmx,
                    gmy, lm);
            mass_flux_ch(P, gmx, gmy, mx, my);
        } else {
            mass_flux(P, phi, gx, gy, lnx, lny, mx, my);
        }
        const T rho = P.drho * (phi - P.phiB) + P.rhoB;
        T m[9], e[9];
        T mf[9] = {phi, T(-2) * phi, phi, phi * u, -phi * u, phi * v, -phi * v, T(0), T(0)};
        if (P.pf == 1) {   // Eq. MfMRCH1
            const T mu = chem_pot(P, phi, lap);
            mf[1] = T(-4) * phi + T(2) * mu;
            mf[2] = T(4) * phi - T(3) * mu;
        }
        from_moments(mf, e);
        for (int i = 0; i < Q; i++) eq[i * P.plane + k] = e[i];
        T tr = T(3) * rho * (u * u + v * v) + T(3) * (u * mx + v * my);
        m[0] = P.rho0;
        m[1] = T(-4) * P.rho0 + T(6) * p + tr;
        m[2] = T(4) * P.rho0 - T(9) * p - tr;
        m[3] = rho * u;
        m[4] = -rho * u;
        m[5] = rho * v;
        m[6] = -rho * v;
        m[7] = (u * mx - v * my) + rho * (u * u - v * v);
        m[8] = T(0.5) * ((u * my + v * mx) + T(2) * rho * u * v);
        from_moments(m, e);
        for (int i = 0; i < Q; i++) eq[(9 + i) * P.plane + k] = e[i];
    }
}

// Store post-streaming populations `post` (planes 0..17, level n) into the
// pull representation of copy `dst`: slot (i, y) holds what (y + c_i) pulls,
// or -- when y + c_i is beyond a wall -- what y itself pulls in direction
// opp(i).  `post_stride` is the plane stride of `post`.
template <typename T>
__global__ void k_to_pull(KParams<T> P, const T* post, long long post_stride, char* dst_base) {
    const Copy<T> D = copy_at<T>(dst_base, P.plane);
    const long long n = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / P.nx), x = (int)(k - (long long)y * P.nx);
        for (int h = 0; h < 2; h++) {
            const T* src = post + h * 9 * post_stride;
            for (int i = 0; i < Q; i++) {
                int tx = x + cx(i), ty = y + cy(i);
                bool wall = false;
                if (tx < 0 || tx >= P.nx) {
                    if (P.wall_x) wall = true;
                    else tx = tx < 0 ? tx + P.nx : tx - P.nx;
                }
                if (ty < 0 || ty >= P.ny) {
                    if (P.wall_y) wall = true;
                    else ty = ty < 0 ? ty + P.ny : ty - P.ny;
                }
                T val = wall ? src[opp(i) * post_stride + k] : src[i * post_stride + (long long)ty * P.nx + tx];
                if (h == 1) D.g[i * P.plane + k] = val;
                else if (i == 0) D.f0[k] = rest_encode<T>((double)val, D.h[k], P.rest_w);
                else D.f[i * P.plane + k] = val;
            }
        }
    }
}

template <typename T>
__global__ void k_export(KParams<T> P, char* state, size_t off0, size_t off1, size_t off_stamp, T* f, T* g,
                         T* hist) {
    const int cur = stamp_copy(*reinterpret_cast<const int64_t*>(state + off_stamp));
    const Copy<T> S = copy_at<T>(state + (cur ? off1 : off0), P.plane);
    const long long n = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / P.nx), x = (int)(k - (long long)y * P.nx);
        if (f) {
            f[k] = (T)rest_decode(S.f0[k], S.h[k], P.rest_w);
            for (int i = 1; i < Q; i++) f[i * n + k] = pull(S.f, P, i, x, y);
        }
        if (g)
            for (int i = 0; i < Q; i++) g[i * n + k] = pull(S.g, P, i, x, y);
        if (hist)   // phi, u, v of level n-1 (and m^phiC of level n-1 for the local gradient scheme)
            for (int j = 0; j < (P.grad == 1 ? 5 : 3); j++) hist[j * n + k] = S.h[j * P.plane + k];
    }
}

template <typename T>
__global__ void k_copy_hist(KParams<T> P, const T* hist, char* dst_base) {
    const Copy<T> D = copy_at<T>(dst_base, P.plane);
    const long long n = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        for (int j = 0; j < (P.grad == 1 ? 5 : 3); j++) D.h[j * P.plane + k] = hist ? hist[j * n + k] : T(0);
}

__global__ void k_set_header(StateHeader* H, int nx, int ny, int dtype) {
    H->magic = STATE_MAGIC;
    H->nx = nx;
    H->ny = ny;
    H->dtype = dtype;
}

__global__ void k_set_stamps(int64_t* stamp, long long n, int64_t value) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        stamp[i] = value;
}

// Hydrostatic pressure of the two fluids at rest (the initial pressure of the
// gravity-driven set-ups): rho from the density law of Sec. 2 at phi0,
// dp/dy = (rho - rho_ref) g_y integrated down every column by the trapezoid
// rule from p = 0 at the top row, then the mean taken out.  One workgroup:
// every thread walks its columns twice (FP64 sums; the second walk subtracts
// the mean that the block reduction of the first one gives).
constexpr int HYDRO_THREADS = 1024;

template <typename T>
__global__ __launch_bounds__(HYDRO_THREADS) void k_hydrostatic(KParams<T> P, const T* phi0, T* p0) {
    __shared__ double red[HYDRO_THREADS / 64];
    const int nx = P.nx, ny = P.ny;
    const double gy = (double)P.gy, drho = (double)P.drho, rhoB = (double)P.rhoB, rref = (double)P.rho_ref,
                 phiB = (double)P.phiB;
    auto force = [&](int j, int x) { return (drho * ((double)phi0[(long long)j * nx + x] - phiB) + rhoB - rref) * gy; };
    double total = 0.0;
    for (int pass = 0; pass < 2; pass++) {
        const double mean = pass == 0 ? 0.0 : total / ((double)nx * (double)ny);
        double acc = 0.0;
        for (int x = threadIdx.x; x < nx; x += HYDRO_THREADS) {
            double p = 0.0, fu = force(ny - 1, x);
            acc += p;
            if (pass == 1) p0[(long long)(ny - 1) * nx + x] = (T)(p - mean);
            for (int j = ny - 2; j >= 0; j--) {
                const double f = force(j, x);
                p -= 0.5 * (f + fu);
                fu = f;
                acc += p;
                if (pass == 1) p0[(long long)j * nx + x] = (T)(p - mean);
            }
        }
        if (pass == 0) {
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
            __syncthreads();
            double t = 0.0;
            for (int w = 0; w < HYDRO_THREADS / 64; w++) t += red[w];
            total = t;
        }
    }
}

// ---------------------------------------------------------------- launchers
static int grid1d(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// Byte size of one copy fits 32-bit offsets?
static bool small_copy(const Layout& L) { return L.buf_bytes < (size_t(1) << 32); }


template <typename T, int TY, int MODE, int NBY = BY>
static void launch_tile(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p,
                        int hint = 0) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    dim3 blk(TX, NBY);
    // the standard rates compiled in for steps (moments do not collide)
    const bool std_rates = MODE == 0 && P.rates_std;
    if (MODE == 0 && resident_state(L)) {   // the last-level cache holds both copies: g loaded late
        if (std_rates)
            k_step<T, TY, MODE, uint32_t, NBY, true, false, true><<<ntx * nty, blk, 0, s>>>(
                P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, ntx, nty, phi, u, p, hint);
        else
            k_step<T, TY, MODE, uint32_t, NBY, false, false, true><<<ntx * nty, blk, 0, s>>>(
                P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, ntx, nty, phi, u, p, hint);
    } else if (MODE == 0 && cached_state(L)) {
        if (std_rates)
            k_step<T, TY, MODE, uint32_t, NBY, true, false><<<ntx * nty, blk, 0, s>>>(
                P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, ntx, nty, phi, u, p, hint);
        else
            k_step<T, TY, MODE, uint32_t, NBY, false, false><<<ntx * nty, blk, 0, s>>>(
                P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, ntx, nty, phi, u, p, hint);
    } else if (small_copy(L)) {
        if (std_rates)
            k_step<T, TY, MODE, uint32_t, NBY, true><<<ntx * nty, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                                L.off_stamp, ntx, nty, phi, u, p, hint);
        else
            k_step<T, TY, MODE, uint32_t, NBY, false><<<ntx * nty, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                                 L.off_stamp, ntx, nty, phi, u, p, hint);
    } else {
        if (std_rates)
            k_step<T, TY, MODE, uint64_t, NBY, true><<<ntx * nty, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                                L.off_stamp, ntx, nty, phi, u, p, hint);
        else
            k_step<T, TY, MODE, uint64_t, NBY, false><<<ntx * nty, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                                 L.off_stamp, ntx, nty, phi, u, p, hint);
    }
}

// Two levels per launch for the Allen-Cahn step with either gradient scheme
// (stencils or Eq. local; present or original model; lbm_step2.hip) on
// lattices of at least one 64 x 8 tile per CU whose copy fits 32-bit offsets.
// Measured on MI355X, FP32, per level: 256 x 1024 (cache-resident) 7.2 us
// against 9.0 one-level, 1024 x 512 14.4 against 16.1, 4096 x 4096 (streamed
// from HBM, which the two-level launch crosses once per two levels) 378 against
// 521; FP64 4096 x 4096 974 against 985.  Below the size rule, where every CU
// runs at most one short tile, the longer chain of the two-level tile costs
// more than the launch it saves (256 x 128: 5.1 against 4.8 us, 64 x 8: 4.9
// against 4.7).  The environment variable LBM_TWO_LEVEL, read at every call,
// overrides the size rule: "0" never, "1" on every eligible state whatever its
// size.  The compile-time LBM_TWO_LEVEL=0 removes the path.
#ifndef LBM_TWO_LEVEL
#define LBM_TWO_LEVEL 1
#endif

bool two_level_path(const Layout& L, int nx, int ny, int pf, int model, int grad) {
    if (!LBM_TWO_LEVEL || pf != 0 || model == 2 || L.buf_bytes >= (size_t(1) << 32)) return false;
    const char* e = getenv("LBM_TWO_LEVEL");
    if (e && e[0] == '0' && e[1] == 0) return false;
    if (e && e[0] == '1' && e[1] == 0) return true;
    const long long tiles8 = (long long)((nx + TX - 1) / TX) * ((ny + 7) / 8);
    return tiles8 >= 256;
}

template <typename T>
hipError_t launch_step(const KParams<T>& P, char* state, const Layout& L, int64_t nsteps, hipStream_t s,
                       int ty, int by, int& copy) {
    constexpr int T16 = sizeof(T) == 8 ? 8 : 16;   // FP64 tiles stop at 8 rows
    if (two_level_path(L, P.nx, P.ny, P.pf, P.model, P.grad))
        for (; nsteps >= 2; nsteps -= 2) {
            launch_step2<T>(P, state, L, s);
            copy ^= 1;
        }
    for (int64_t t = 0; t < nsteps; t++) {
        const int h = copy;   // the copy this launch is expected to find the state in
        copy ^= 1;
        if (P.pf == 1 || P.model == 2) launch_ch<T, 0>(P, state, L, s, nullptr, nullptr, nullptr);
        else if (P.grad == 1) launch_local<T, 0>(P, state, L, s, nullptr, nullptr, nullptr);
        else if (ty == 4) launch_tile<T, 4, 0>(P, state, L, s, nullptr, nullptr, nullptr, h);
        else if (ty == 8 || sizeof(T) == 8) {
            if (by == 8) launch_tile<T, 8, 0, 8>(P, state, L, s, nullptr, nullptr, nullptr, h);
            else launch_tile<T, 8, 0>(P, state, L, s, nullptr, nullptr, nullptr, h);
        } else {
            if (by == 8) launch_tile<T, T16, 0, 8>(P, state, L, s, nullptr, nullptr, nullptr, h);
            else launch_tile<T, T16, 0>(P, state, L, s, nullptr, nullptr, nullptr, h);
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_moments(const KParams<T>& P, const char* state, const Layout& L, T* phi, T* u, T* p,
                          hipStream_t s) {
    if (P.pf == 1 || P.model == 2) launch_ch<T, 1>(P, const_cast<char*>(state), L, s, phi, u, p);
    else if (P.grad == 1) launch_local<T, 1>(P, const_cast<char*>(state), L, s, phi, u, p);
    else launch_tile<T, 8, 1>(P, const_cast<char*>(state), L, s, phi, u, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const KParams<T>& P, char* state, const Layout& L, const T* phi0, const T* u0,
                       const T* p0, int dtype, hipStream_t s) {
    T* scratch = reinterpret_cast<T*>(state + L.off_buf[1]);   // 18 planes of T fit in one copy
    char* dst = state + L.off_buf[0];
    int g = grid1d(L.n);
    k_equilibrium<T><<<g, 256, 0, s>>>(P, phi0, u0, p0, scratch);
    k_copy_hist<T><<<g, 256, 0, s>>>(P, nullptr, dst);   // before k_to_pull: f_0 is stored relative to it
    k_to_pull<T><<<g, 256, 0, s>>>(P, scratch, P.plane, dst);
    k_set_header<<<1, 1, 0, s>>>(reinterpret_cast<StateHeader*>(state), P.nx, P.ny, dtype);
    k_set_stamps<<<grid1d((long long)L.nstamp), 256, 0, s>>>(reinterpret_cast<int64_t*>(state + L.off_stamp),
                                                              (long long)L.nstamp, stamp_of(0, 0));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hydrostatic(const KParams<T>& P, const T* phi0, T* p0, hipStream_t s) {
    k_hydrostatic<T><<<1, HYDRO_THREADS, 0, s>>>(P, phi0, p0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_import(const KParams<T>& P, char* state, const Layout& L, const T* f, const T* g,
                         const T* hist, int64_t step, int dtype, hipStream_t s) {
    // f and g are separate caller arrays of [9][n]; stage them contiguously in
    // the other copy, which the next step overwrites anyway.
    int cur = (int)(step & 1);
    char* dst = state + L.off_buf[cur];
    T* stage = reinterpret_cast<T*>(state + L.off_buf[1 - cur]);
    size_t bytes9 = (size_t)9 * L.n * sizeof(T);
    hipError_t e = hipMemcpy2DAsync(stage, (size_t)P.plane * sizeof(T), f, (size_t)L.n * sizeof(T),
                                    (size_t)L.n * sizeof(T), 9, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpy2DAsync(stage + 9 * P.plane, (size_t)P.plane * sizeof(T), g, (size_t)L.n * sizeof(T),
                         (size_t)L.n * sizeof(T), 9, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    (void)bytes9;
    int gr = grid1d(L.n);
    k_copy_hist<T><<<gr, 256, 0, s>>>(P, step > 0 ? hist : nullptr, dst);   // before k_to_pull (f_0)
    k_to_pull<T><<<gr, 256, 0, s>>>(P, stage, P.plane, dst);
    k_set_header<<<1, 1, 0, s>>>(reinterpret_cast<StateHeader*>(state), P.nx, P.ny, dtype);
    k_set_stamps<<<grid1d((long long)L.nstamp), 256, 0, s>>>(reinterpret_cast<int64_t*>(state + L.off_stamp),
                                                              (long long)L.nstamp, stamp_of(step, cur));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_export(const KParams<T>& P, const char* state, const Layout& L, T* f, T* g, T* hist,
                         hipStream_t s) {
    k_export<T><<<grid1d(L.n), 256, 0, s>>>(P, const_cast<char*>(state), L.off_buf[0], L.off_buf[1], L.off_stamp, f,
                                             g, hist);
    return hipGetLastError();
}

#define LBM_INSTANTIATE(T)                                                                              \
    template hipError_t launch_step<T>(const KParams<T>&, char*, const Layout&, int64_t, hipStream_t, int, int, \
                                       int&);                                                            \
    template hipError_t launch_moments<T>(const KParams<T>&, const char*, const Layout&, T*, T*, T*,     \
                                          hipStream_t);                                                 \
    template hipError_t launch_init<T>(const KParams<T>&, char*, const Layout&, const T*, const T*,     \
                                       const T*, int, hipStream_t);                                     \
    template hipError_t launch_import<T>(const KParams<T>&, char*, const Layout&, const T*, const T*,   \
                                         const T*, int64_t, int, hipStream_t);                          \
    template hipError_t launch_export<T>(const KParams<T>&, const char*, const Layout&, T*, T*, T*,     \
                                         hipStream_t);                                                  \
    template hipError_t launch_hydrostatic<T>(const KParams<T>&, const T*, T*, hipStream_t);

LBM_INSTANTIATE(float)
LBM_INSTANTIATE(double)

}  // namespace lbm
