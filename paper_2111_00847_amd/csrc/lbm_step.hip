// lbm_step.hip -- gfx950 kernels of the fused phase-field LBM time step.
//
// Memory layout (structure of arrays, x fastest): a state buffer is
//   [header | copy 0: f[9] g[9] hist[3] | copy 1: same | diagnostics scratch]
// with every plane padded to a multiple of 64 elements.  Copy (n & 1) holds
// the post-collision populations of level n-1 -- a node obtains its level-n
// populations by pulling them from its neighbours -- and hist = (phi, u, v)
// of level n-1, from which the explicit-Euler time derivatives are formed.
// A step reads copy (n & 1) and writes copy (1 - n & 1).  The level n is kept
// in per-row stamps owned by the workgroups (lbm_common.hpp), so host code
// never needs the parity, no workgroup waits for another, and a sequence of
// steps can be captured in a graph.
//
// The phi stencils need phi on a one-node ring around each tile.  A tile of
// 64 x TY nodes (256 threads) first pulls the populations of its (64+2) x
// (TY+2) window, sums them into phi in LDS (the ring's pulls hit L2: those
// lines are the neighbour tiles' own reads), fills wall ghosts, and then each
// thread runs the per-node update for TY/4 nodes of its column.
#include "lbm_kernels.hpp"
#include "lbm_tile.hpp"

namespace lbm {

// Tile order: consecutive workgroup ids are dealt round-robin to the 8 XCDs,
// each with its own L2.  Remap so that XCD j gets a contiguous band of tiles,
// whose shared halo rows/columns then hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    constexpr int NX = 8;
    const int q = nb / NX, rem = nb % NX;
    const int xcd = b % NX, slot = b / NX;
    // XCDs 0..rem-1 own q+1 tiles, the others q
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

template <typename T, typename OFF>
__device__ __forceinline__ T ld(const char* base, OFF byteoff) {
    return *reinterpret_cast<const T*>(base + byteoff);
}
// Tuning knobs (compile time, measured on MI355X): non-temporal stores for
// the streamed state (+3% on a 4096^2 lattice); g loaded after the window
// barrier (prefetching it with f gained nothing and costs registers); tiles
// dealt to XCDs in bands (+11% on 256 x 1024, neutral on 4096^2).
#ifndef LBM_NT_STORES
#define LBM_NT_STORES 1
#endif
#ifndef LBM_PREFETCH_G      // load g together with f, before the window barrier
#define LBM_PREFETCH_G 0
#endif
#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 1
#endif

template <typename T, typename OFF>
__device__ __forceinline__ void st(char* base, OFF byteoff, T v) {
    if (LBM_NT_STORES) __builtin_nontemporal_store(v, reinterpret_cast<T*>(base + byteoff));
    else *reinterpret_cast<T*>(base + byteoff) = v;
}

// The fused step.  One 64 x TY tile per 256-thread workgroup; thread
// (lx, ly) owns nodes (x0 + lx, y0 + ly + 4 r), r < TY/4, keeps their pulled f
// in registers from the phi pass to the collision, and the ring of the phi
// window is pulled by spare threads.  MODE 0: one time step; MODE 1: write
// phi, u, p of the current level.  OFF: byte-offset type within one copy.
// FP32 16-row tiles keep four nodes per thread in flight; capping them at 128
// VGPRs (4 waves per SIMD) is worth +10% on a 4096^2 lattice.  FP64 tiles are
// never taller than 8 rows (the host caps them): they would spill.
template <typename T, int TY>
struct StepWaves {
    static constexpr int value = (sizeof(T) == 4 && TY >= 16) ? 4 : 1;
};

template <typename T, int TY, int MODE, typename OFF>
__global__ __launch_bounds__(TX* BY) __attribute__((amdgpu_waves_per_eu(StepWaves<T, TY>::value)))
void k_step(KParams<T> P, char* state, size_t off0, size_t off1, size_t off_stamp, int ntx,
                                                 int nty, T* out_phi, T* out_u, T* out_p) {
    constexpr int R = TY / BY;
    constexpr int WX = TX + 2, WY = TY + 2;
    constexpr OFF ES = sizeof(T);
    __shared__ T sphi[WY][TX + 3];
    __shared__ T sphp[WY][TX + 3];
    const int t = LBM_XCD_REMAP ? xcd_tile(blockIdx.x, ntx * nty) : (int)blockIdx.x;
    const int xt = t % ntx;
    const int x0 = xt * TX, y0 = (t / ntx) * TY;
    int64_t* stamp = reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0;
    const int64_t step = stamp[0];
    const bool first = step == 0;
    const int cur = (int)(step & 1);
    const char* src = state + (cur ? off1 : off0);
    char* dst = state + (cur ? off0 : off1);
    const Copy<T> S = copy_at<T>(const_cast<char*>(src), P.plane);
    const OFF pl = (OFF)P.plane;
    const OFF bF = 8 * pl;               // byte base of f_1; f_i at bF + (i - 1) pl ES
    const OFF bG = bF + 8 * pl * ES;     // g_i at bG + i pl ES
    const OFF bH = bG + 9 * pl * ES;     // hist_j at bH + j pl ES
    const OFF nx = (OFF)P.nx;

    const int lx = threadIdx.x;
    const int tid = threadIdx.y * TX + lx;
    const int x = x0 + lx;

    // column neighbours of this thread: index 0 = x-1, 1 = x, 2 = x+1
    OFF col[3];
    bool wx[3] = {false, false, false};
    col[1] = (OFF)x;
    if (x == 0) {
        wx[0] = P.wall_x;
        col[0] = (OFF)(P.nx - 1);
    } else {
        col[0] = (OFF)(x - 1);
    }
    if (x == P.nx - 1) {
        wx[2] = P.wall_x;
        col[2] = 0;
    } else {
        col[2] = (OFF)(x + 1);
    }

    T f[R][9];
    double phid[R];
    T gp[LBM_PREFETCH_G ? R : 1][9];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * BY, y = y0 + ly;
        phid[r] = 0.0;
        if (x >= P.nx || y >= P.ny) continue;
        OFF row[3];
        bool wy[3] = {false, false, false};
        row[1] = (OFF)y * nx;
        if (y == 0) {
            wy[0] = P.wall_y;
            row[0] = (OFF)(P.ny - 1) * nx;
        } else {
            row[0] = (OFF)(y - 1) * nx;
        }
        if (y == P.ny - 1) {
            wy[2] = P.wall_y;
            row[2] = 0;
        } else {
            row[2] = (OFF)(y + 1) * nx;
        }
        const OFF k = row[1] + col[1];
        const double f0 = ld<double>(src, (OFF)8 * k);
        f[r][0] = (T)f0;
#pragma unroll
        for (int i = 1; i < Q; i++) {
            const int ax = 1 - cx(i), ay = 1 - cy(i);
            const bool bb = wx[ax] || wy[ay];
            const OFF o = bb ? bF + ((OFF)(opp(i) - 1) * pl + k) * ES : bF + ((OFF)(i - 1) * pl + row[ay] + col[ax]) * ES;
            f[r][i] = ld<T>(src, o);
        }
        phid[r] = f0 + moving_sum_d(f[r]);
        sphi[ly + 1][lx + 1] = (T)phid[r];
        if (!first) sphp[ly + 1][lx + 1] = ld<T>(src, bH + k * ES);
        if (LBM_PREFETCH_G) {
#pragma unroll
            for (int i = 0; i < Q; i++) {
                const int ax = 1 - cx(i), ay = 1 - cy(i);
                const bool bb = wx[ax] || wy[ay];
                const OFF o = bb ? bG + ((OFF)opp(i) * pl + k) * ES : bG + ((OFF)i * pl + row[ay] + col[ax]) * ES;
                gp[LBM_PREFETCH_G ? r : 0][i] = ld<T>(src, o);
            }
        }
    }

    // ring of the window (and, for a ragged tile, the halo column/row inside it)
    auto fill_node = [&](int wxi, int wyi) {
        int gx = x0 - 1 + wxi, gy = y0 - 1 + wyi;
        if (gx > P.nx || gy > P.ny) return;
        if (gx < 0 || gx >= P.nx) {
            if (P.wall_x) return;
            gx = gx < 0 ? gx + P.nx : gx - P.nx;
        }
        if (gy < 0 || gy >= P.ny) {
            if (P.wall_y) return;
            gy = gy < 0 ? gy + P.ny : gy - P.ny;
        }
        T fw[9];
        sphi[wyi][wxi] = (T)node_phi(P, S, gx, gy, fw);
        if (!first) sphp[wyi][wxi] = S.h[(long long)gy * P.nx + gx];
    };
    for (int idx = tid; idx < 2 * WX + 2 * TY; idx += TX * BY) {
        if (idx < WX) fill_node(idx, 0);
        else if (idx < 2 * WX) fill_node(idx - WX, WY - 1);
        else if (idx < 2 * WX + TY) fill_node(0, 1 + idx - 2 * WX);
        else fill_node(WX - 1, 1 + idx - 2 * WX - TY);
    }
    if (x0 + TX > P.nx)
        for (int wy = tid; wy < WY; wy += TX * BY) fill_node(P.nx - x0 + 1, wy);
    if (y0 + TY > P.ny)
        for (int wxi = tid; wxi < WX; wxi += TX * BY) fill_node(wxi, P.ny - y0 + 1);
    __syncthreads();
    wall_ghosts<T, TY>(P, !first, x0, y0, sphi, sphp);

#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * BY, y = y0 + ly;
        if (x >= P.nx || y >= P.ny) continue;
        OFF row[3];
        bool wy[3] = {false, false, false};
        row[1] = (OFF)y * nx;
        if (y == 0) {
            wy[0] = P.wall_y;
            row[0] = (OFF)(P.ny - 1) * nx;
        } else {
            row[0] = (OFF)(y - 1) * nx;
        }
        if (y == P.ny - 1) {
            wy[2] = P.wall_y;
            row[2] = 0;
        } else {
            row[2] = (OFF)(y + 1) * nx;
        }
        const OFF k = row[1] + col[1];
        T g[9];
#pragma unroll
        for (int i = 0; i < Q; i++) {
            if (LBM_PREFETCH_G) {
                g[i] = gp[LBM_PREFETCH_G ? r : 0][i];
            } else {
                const int ax = 1 - cx(i), ay = 1 - cy(i);
                const bool bb = wx[ax] || wy[ay];
                const OFF o = bb ? bG + ((OFF)opp(i) * pl + k) * ES : bG + ((OFF)i * pl + row[ay] + col[ax]) * ES;
                g[i] = ld<T>(src, o);
            }
        }
        T gx, gy, lap, gxp = T(0), gyp = T(0), lp, php = T(0), up = T(0), vp = T(0);
        win_stencil<T, TY>(sphi, lx + 1, ly + 1, gx, gy, lap);
        if (!first) {
            win_stencil<T, TY>(sphp, lx + 1, ly + 1, gxp, gyp, lp);
            php = sphp[ly + 1][lx + 1];
            up = ld<T>(src, bH + (pl + k) * ES);
            vp = ld<T>(src, bH + (2 * pl + k) * ES);
        }
        Macro<T> M = macro(P, g, sphi[ly + 1][lx + 1], gx, gy, lap, first, php, gxp, gyp, up, vp);
        if (MODE == 1) {
            if (out_phi) out_phi[k] = M.phi;
            if (out_u) {
                out_u[k] = M.u;
                out_u[(long long)P.nx * P.ny + k] = M.v;
            }
            if (out_p) out_p[k] = M.p;
            continue;
        }
        const double f0n = collide_f(P, M, f[r], phid[r]);
        collide_g(P, M, g);
        st<double>(dst, (OFF)8 * k, f0n);
#pragma unroll
        for (int i = 1; i < Q; i++) st<T>(dst, bF + ((OFF)(i - 1) * pl + k) * ES, f[r][i]);
#pragma unroll
        for (int i = 0; i < Q; i++) st<T>(dst, bG + ((OFF)i * pl + k) * ES, g[i]);
        st<T>(dst, bH + k * ES, M.phi);
        st<T>(dst, bH + (pl + k) * ES, M.u);
        st<T>(dst, bH + (2 * pl + k) * ES, M.v);
    }
    // Own rows move to level n + 1.  Every wave of the workgroup consumed its
    // load of stamp[0] (it addresses all loads above) before the barriers, so
    // no wave can still be about to read it.
    if (MODE == 0 && tid < TY && y0 + tid < P.ny) stamp[tid] = step + 1;
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
        mass_flux(P, phi, gx, gy, lnx, lny, mx, my);
        const T rho = P.drho * (phi - P.phiB) + P.rhoB;
        T m[9], e[9];
        T mf[9] = {phi, T(-2) * phi, phi, phi * u, -phi * u, phi * v, -phi * v, T(0), T(0)};
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
                else if (i == 0) D.f0[k] = (double)val;
                else D.f[i * P.plane + k] = val;
            }
        }
    }
}

template <typename T>
__global__ void k_export(KParams<T> P, char* state, size_t off0, size_t off1, size_t off_stamp, T* f, T* g,
                         T* hist) {
    const int cur = (int)(*reinterpret_cast<const int64_t*>(state + off_stamp) & 1);
    const Copy<T> S = copy_at<T>(state + (cur ? off1 : off0), P.plane);
    const long long n = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / P.nx), x = (int)(k - (long long)y * P.nx);
        if (f) {
            f[k] = (T)S.f0[k];
            for (int i = 1; i < Q; i++) f[i * n + k] = pull(S.f, P, i, x, y);
        }
        if (g)
            for (int i = 0; i < Q; i++) g[i * n + k] = pull(S.g, P, i, x, y);
        if (hist)
            for (int j = 0; j < 3; j++) hist[j * n + k] = S.h[j * P.plane + k];
    }
}

template <typename T>
__global__ void k_copy_hist(KParams<T> P, const T* hist, char* dst_base) {
    const Copy<T> D = copy_at<T>(dst_base, P.plane);
    const long long n = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        for (int j = 0; j < 3; j++) D.h[j * P.plane + k] = hist ? hist[j * n + k] : T(0);
}

__global__ void k_set_header(StateHeader* H, int nx, int ny, int dtype) {
    H->magic = STATE_MAGIC;
    H->nx = nx;
    H->ny = ny;
    H->dtype = dtype;
}

__global__ void k_set_stamps(int64_t* stamp, long long n, int64_t level) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        stamp[i] = level;
}

// ---------------------------------------------------------------- launchers
static int grid1d(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// Byte size of one copy fits 32-bit offsets?
static bool small_copy(const Layout& L) { return L.buf_bytes < (size_t(1) << 32); }

template <typename T, int TY, int MODE>
static void launch_tile(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    dim3 blk(TX, BY);
    if (small_copy(L))
        k_step<T, TY, MODE, uint32_t><<<ntx * nty, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp,
                                                                 ntx, nty, phi, u, p);
    else
        k_step<T, TY, MODE, uint64_t><<<ntx * nty, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp,
                                                                 ntx, nty, phi, u, p);
}

template <typename T>
hipError_t launch_step(const KParams<T>& P, char* state, const Layout& L, int64_t nsteps, hipStream_t s,
                       int ty) {
    for (int64_t t = 0; t < nsteps; t++) {
        if (ty == 4) launch_tile<T, 4, 0>(P, state, L, s, nullptr, nullptr, nullptr);
        else if (ty == 8 || sizeof(T) == 8) launch_tile<T, 8, 0>(P, state, L, s, nullptr, nullptr, nullptr);
        else launch_tile<T, sizeof(T) == 8 ? 8 : 16, 0>(P, state, L, s, nullptr, nullptr, nullptr);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_moments(const KParams<T>& P, const char* state, const Layout& L, T* phi, T* u, T* p,
                          hipStream_t s) {
    launch_tile<T, 8, 1>(P, const_cast<char*>(state), L, s, phi, u, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const KParams<T>& P, char* state, const Layout& L, const T* phi0, const T* u0,
                       const T* p0, int dtype, hipStream_t s) {
    T* scratch = reinterpret_cast<T*>(state + L.off_buf[1]);   // 18 planes of T fit in one copy
    char* dst = state + L.off_buf[0];
    int g = grid1d(L.n);
    k_equilibrium<T><<<g, 256, 0, s>>>(P, phi0, u0, p0, scratch);
    k_to_pull<T><<<g, 256, 0, s>>>(P, scratch, P.plane, dst);
    k_copy_hist<T><<<g, 256, 0, s>>>(P, nullptr, dst);
    k_set_header<<<1, 1, 0, s>>>(reinterpret_cast<StateHeader*>(state), P.nx, P.ny, dtype);
    k_set_stamps<<<grid1d((long long)L.nstamp), 256, 0, s>>>(reinterpret_cast<int64_t*>(state + L.off_stamp),
                                                              (long long)L.nstamp, 0);
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
    k_to_pull<T><<<gr, 256, 0, s>>>(P, stage, P.plane, dst);
    k_copy_hist<T><<<gr, 256, 0, s>>>(P, step > 0 ? hist : nullptr, dst);
    k_set_header<<<1, 1, 0, s>>>(reinterpret_cast<StateHeader*>(state), P.nx, P.ny, dtype);
    k_set_stamps<<<grid1d((long long)L.nstamp), 256, 0, s>>>(reinterpret_cast<int64_t*>(state + L.off_stamp),
                                                              (long long)L.nstamp, step);
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
    template hipError_t launch_step<T>(const KParams<T>&, char*, const Layout&, int64_t, hipStream_t, int); \
    template hipError_t launch_moments<T>(const KParams<T>&, const char*, const Layout&, T*, T*, T*,     \
                                          hipStream_t);                                                 \
    template hipError_t launch_init<T>(const KParams<T>&, char*, const Layout&, const T*, const T*,     \
                                       const T*, int, hipStream_t);                                     \
    template hipError_t launch_import<T>(const KParams<T>&, char*, const Layout&, const T*, const T*,   \
                                         const T*, int64_t, int, hipStream_t);                          \
    template hipError_t launch_export<T>(const KParams<T>&, const char*, const Layout&, T*, T*, T*,     \
                                         hipStream_t);

LBM_INSTANTIATE(float)
LBM_INSTANTIATE(double)

}  // namespace lbm
