// lbm_adjoint.hip -- reverse mode of the fused step: tapes of forward levels
// and the adjoint step.
//
// Tape.  A segment of the forward trajectory, levels n0 .. n0 + L - 1, each
// one state copy (the same bytes as a ping-pong copy), recorded by running the
// ordinary step body from slot j into slot j + 1, so that its levels are
// bitwise those of the plain path.
//
// Adjoint.  The adjoint of level n holds dL/df^n and dL/dg^n of the
// post-streaming populations and dL/d(phi, u, v) of the history stored at
// level n (the level n-1 fields).  It lives in one of two copies (n & 1) of an
// adjoint buffer.  One adjoint step n+1 -> n runs three kernels:
//   A (k_adj_local, tiles)  recomputes the forward node update of level n from
//       the tape, reads the adjoint of each post-collision population where the
//       population streams to (the reverse of the pull, with bounce-back), and
//       applies node_vjp.  It writes the adjoints of the pulled populations,
//       of the previous velocity, and of the stencil inputs (gradient,
//       Laplacian, centre) to scratch planes, plus per-tile sums of the
//       gravity derivative.
//   E (k_adj_edges, one workgroup)  the adjoint of the wall ghost layer: for
//       every ghost the sum of what the neighbouring nodes' stencils took from
//       it, routed through Eq. Dwetting to its first and second fluid nodes
//       (y-wall ghosts, including the corner ghosts built on x-wall ghosts,
//       first; then x-wall ghosts), plus the contact-angle derivatives.
//   B (k_adj_gather, nodes)  the transposed stencils: the adjoint of phi at a
//       node gathers the stencil adjoints of the nodes whose windows hold it,
//       adds the wall routing of E, and is added to all nine populations
//       (phi = sum_i f_i); likewise the previous phi of the history.
// Parameter derivatives accumulate into fixed per-workgroup slots (no atomics;
// deterministic) and are summed by lbm_adjoint_params.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/lbm.h"
#include "lbm_adjoint.hpp"
#include "lbm_fused.hpp"

namespace lbm {

Layout layout_of(const lbm_params* p);
int validate(const lbm_params* p);
int hip_fail(hipError_t e);
int step_tile_rows(const lbm_params* p);
template <typename T>
KParams<T> resolve(const lbm_params* p, const Layout& L);

constexpr size_t ADJ_HDR = 256;
constexpr size_t TAPE_HDR = 256;
constexpr int ATY = BY;   // adjoint tiles: 64 x 4, one node per thread

struct TapeHeader {
    int64_t n0;
    int32_t nlevels, nx, ny, dtype;
};

struct AdjHeader {
    int64_t level;     // level of the adjoint currently held
    int32_t status;    // 0 ok; 1 an adjoint step met an adjoint of the wrong level; 2 init not at level 0
    int32_t nx, ny, dtype;
    double result[6];  // lbm_adjoint_params output
};

// Scratch planes written by A and read by E and B.
enum { S_PHIC = 0, S_GX, S_GY, S_LAP, S_PHP, S_GXP, S_GYP, S_PHI, S_COUNT };
constexpr int ADJ_PLANES = 21;   // f (9), g (9), history (3)

struct AdjLayout {
    long long plane;
    size_t esz;
    size_t off_copy[2];
    size_t off_scr;
    size_t off_edge;
    long long emax;       // edge array length per (level, wall, depth)
    size_t off_part;      // doubles: 2 per tile of A (gravity), then 4 (contact angles)
    int ntA;
    size_t total;
};

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

AdjLayout adj_layout_of(const lbm_params* p) {
    Layout L = layout_of(p);
    AdjLayout A;
    A.plane = L.plane;
    A.esz = L.esz;
    const size_t cp = (size_t)ADJ_PLANES * L.plane * L.esz;
    A.off_copy[0] = ADJ_HDR;
    A.off_copy[1] = A.off_copy[0] + cp;
    A.off_scr = A.off_copy[1] + cp;
    A.off_edge = A.off_scr + (size_t)S_COUNT * L.plane * L.esz;
    A.emax = ((long long)(p->nx > p->ny ? p->nx : p->ny) + 63) / 64 * 64;
    A.off_part = al256(A.off_edge + (size_t)16 * A.emax * L.esz);
    A.ntA = ((p->nx + TX - 1) / TX) * ((p->ny + ATY - 1) / ATY);
    A.total = al256(A.off_part + (size_t)(2 * A.ntA + 4) * sizeof(double));
    return A;
}

// Device view of an adjoint buffer.
template <typename T>
struct AdjView {
    char* base;
    long long plane;
    T* copy[2];
    T* scr;
    T* edge;
    long long emax;
    double* part;
    int ntA;
    __device__ AdjHeader* hdr() const { return reinterpret_cast<AdjHeader*>(base); }
    __device__ T* plane_of(int c, int i) const { return copy[c] + (long long)i * plane; }
    __device__ T* s(int i) const { return scr + (long long)i * plane; }
    // lev 0: current phi, 1: previous; wall 0..3 (x-, x+, y-, y+); depth 0: first fluid node
    __device__ T* e(int lev, int wall, int depth) const { return edge + ((lev * 4 + wall) * 2 + depth) * emax; }
};

template <typename T>
AdjView<T> adj_view(void* adj, const AdjLayout& A) {
    AdjView<T> V;
    V.base = (char*)adj;
    V.plane = A.plane;
    V.copy[0] = reinterpret_cast<T*>(V.base + A.off_copy[0]);
    V.copy[1] = reinterpret_cast<T*>(V.base + A.off_copy[1]);
    V.scr = reinterpret_cast<T*>(V.base + A.off_scr);
    V.edge = reinterpret_cast<T*>(V.base + A.off_edge);
    V.emax = A.emax;
    V.part = reinterpret_cast<double*>(V.base + A.off_part);
    V.ntA = A.ntA;
    return V;
}

// ---------------------------------------------------------------- tape
__global__ void k_tape_copy(const char* state, size_t off0, size_t off1, size_t off_stamp, size_t bytes,
                            char* tape, int nlevels, int nx, int ny, int dtype) {
    const int64_t n = *reinterpret_cast<const int64_t*>(state + off_stamp);
    const uint4* src = reinterpret_cast<const uint4*>(state + ((n & 1) ? off1 : off0));
    uint4* dst = reinterpret_cast<uint4*>(tape + TAPE_HDR);
    const size_t nv = bytes / sizeof(uint4);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nv; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        TapeHeader* h = reinterpret_cast<TapeHeader*>(tape);
        h->n0 = n;
        h->nlevels = nlevels;
        h->nx = nx;
        h->ny = ny;
        h->dtype = dtype;
    }
}

template <typename T, int TY, typename OFF>
__global__ __launch_bounds__(TX* BY) __attribute__((amdgpu_waves_per_eu(StepWaves<T, TY>::value)))
void k_tape_step(KParams<T> P, char* tape, size_t slot, int j, int ntx, int nty) {
    __shared__ T sphi[TY + 2][TX + 3];
    __shared__ T sphp[TY + 2][TX + 3];
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    char* src = tape + TAPE_HDR + (size_t)j * slot;
    int xt, yt;
    xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    step_core<T, TY, 0, OFF>(P, src, src + slot, n, xt, yt, nullptr, nullptr, nullptr, sphi, sphp);
}

// ---------------------------------------------------------------- adjoint step, kernel A
// Adjoint of post-collision population i of node (x, y): the population
// streams to (x, y) + c_i, or back to (x, y) as opp(i) through a wall.
template <typename T>
__device__ __forceinline__ T push_read(const T* planes, long long plane, const KParams<T>& P, int i, int x, int y) {
    int tx = x + cx(i), ty = y + cy(i);
    bool bb = false;
    if (tx < 0 || tx >= P.nx) {
        if (P.wall_x) bb = true;
        else tx = tx < 0 ? tx + P.nx : tx - P.nx;
    }
    if (ty < 0 || ty >= P.ny) {
        if (P.wall_y) bb = true;
        else ty = ty < 0 ? ty + P.ny : ty - P.ny;
    }
    if (bb) return planes[opp(i) * plane + (long long)y * P.nx + x];
    return planes[i * plane + (long long)ty * P.nx + tx];
}

template <typename T>
__global__ __launch_bounds__(TX* BY) void k_adj_local(KParams<T> P, const char* tape, size_t slot, int j,
                                                     AdjView<T> V) {
    __shared__ T sphi[ATY + 2][TX + 3];
    __shared__ T sphp[ATY + 2][TX + 3];
    __shared__ double red[2][TX * BY];
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    AdjHeader* H = V.hdr();
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (H->status != 0 || H->level != n + 1) {
        if (blockIdx.x == 0 && tid == 0 && H->level != n + 1) H->status = 1;
        return;
    }
    const bool first = n == 0;
    const Copy<T> S = copy_at<T>(const_cast<char*>(tape + TAPE_HDR + (size_t)j * slot), P.plane);
    const int ntx = (P.nx + TX - 1) / TX;
    const int x0 = (blockIdx.x % ntx) * TX, y0 = (blockIdx.x / ntx) * ATY;
    fill_window<T, ATY>(P, S, !first, x0, y0, sphi, sphp);

    const int lx = threadIdx.x, ly = threadIdx.y;
    const int x = x0 + lx, y = y0 + ly;
    double gsum_x = 0.0, gsum_y = 0.0;
    if (x < P.nx && y < P.ny) {
        const long long k = (long long)y * P.nx + x;
        T f[9], g[9];
        f[0] = (T)S.f0[k];
#pragma unroll
        for (int i = 1; i < Q; i++) f[i] = pull(S.f, P, i, x, y);
#pragma unroll
        for (int i = 0; i < Q; i++) g[i] = pull(S.g, P, i, x, y);
        T gx, gy, lap, gxp = T(0), gyp = T(0), lp, php = T(0), up = T(0), vp = T(0);
        win_stencil<T, ATY>(sphi, lx + 1, ly + 1, gx, gy, lap);
        if (!first) {
            win_stencil<T, ATY>(sphp, lx + 1, ly + 1, gxp, gyp, lp);
            php = sphp[ly + 1][lx + 1];
            up = S.h[P.plane + k];
            vp = S.h[2 * P.plane + k];
        }
        const Macro<T> M = macro(P, g, sphi[ly + 1][lx + 1], gx, gy, lap, first, php, gxp, gyp, up, vp);
        const int ci = (int)((n + 1) & 1), co = (int)(n & 1);
        T fo[9], go[9];
#pragma unroll
        for (int i = 0; i < Q; i++) {
            fo[i] = push_read(V.copy[ci], V.plane, P, i, x, y);
            go[i] = push_read(V.copy[ci] + 9 * V.plane, V.plane, P, i, x, y);
        }
        const T hphi = V.plane_of(ci, 18)[k], hu = V.plane_of(ci, 19)[k], hv = V.plane_of(ci, 20)[k];
        NodeAdj<T> A;
        node_vjp(P, M, f, g, gx, gy, lap, first, php, gxp, gyp, up, vp, fo, go, hphi, hu, hv, A);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            V.plane_of(co, i)[k] = A.f[i];
            V.plane_of(co, 9 + i)[k] = A.g[i];
        }
        V.plane_of(co, 19)[k] = first ? T(0) : A.up;
        V.plane_of(co, 20)[k] = first ? T(0) : A.vp;
        V.s(S_PHIC)[k] = A.phic;
        V.s(S_GX)[k] = A.gx;
        V.s(S_GY)[k] = A.gy;
        V.s(S_LAP)[k] = A.lap;
        V.s(S_PHP)[k] = A.php;
        V.s(S_GXP)[k] = A.gxp;
        V.s(S_GYP)[k] = A.gyp;
        V.s(S_PHI)[k] = M.phi;
        gsum_x = (double)A.grav_x;
        gsum_y = (double)A.grav_y;
    }
    // per-tile sums of the gravity derivative, accumulated over the steps of a pass
    red[0][tid] = gsum_x;
    red[1][tid] = gsum_y;
    __syncthreads();
    for (int w = TX * BY / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        V.part[2 * blockIdx.x] += red[0][0];
        V.part[2 * blockIdx.x + 1] += red[1][0];
    }
}

// ---------------------------------------------------------------- adjoint step, kernel E
// Stencil weights of window offset (ex, ey): phi(x + e) enters grad_x phi,
// grad_y phi and lap phi at x with these coefficients (App. C).
template <typename T>
__device__ __forceinline__ T wgx(int ex, int ey) {
    return ex == 0 ? T(0) : T(ex) * (ey == 0 ? T(1) / T(3) : T(1) / T(12));
}
template <typename T>
__device__ __forceinline__ T wgy(int ex, int ey) {
    return ey == 0 ? T(0) : T(ey) * (ex == 0 ? T(1) / T(3) : T(1) / T(12));
}
template <typename T>
__device__ __forceinline__ T wlap(int ex, int ey) {
    return (ex == 0 && ey == 0) ? T(-10) / T(3) : ((ex == 0 || ey == 0) ? T(2) / T(3) : T(1) / T(6));
}

// Sum of what the fluid nodes around position (X, Y) of the extended lattice
// took from it through their stencils (lev 0: current phi; 1: previous phi).
template <typename T>
__device__ T ext_adjoint(const KParams<T>& P, const AdjView<T>& V, int lev, int X, int Y) {
    const T* sgx = V.s(lev ? S_GXP : S_GX);
    const T* sgy = V.s(lev ? S_GYP : S_GY);
    const T* slp = V.s(S_LAP);
    T acc = T(0);
    for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
            int xs = X + dx, ys = Y + dy;   // a node whose window holds (X, Y) at offset (-dx, -dy)
            if (xs < 0 || xs >= P.nx) {
                if (P.wall_x) continue;
                xs = xs < 0 ? xs + P.nx : xs - P.nx;
            }
            if (ys < 0 || ys >= P.ny) {
                if (P.wall_y) continue;
                ys = ys < 0 ? ys + P.ny : ys - P.ny;
            }
            const long long k = (long long)ys * P.nx + xs;
            acc += wgx<T>(-dx, -dy) * sgx[k] + wgy<T>(-dx, -dy) * sgy[k];
            if (!lev) acc += wlap<T>(-dx, -dy) * slp[k];
        }
    return acc;
}

template <typename T>
__device__ __forceinline__ T phi_at(const KParams<T>& P, const T* phi, int x, int y) {
    return phi[(long long)y * P.nx + x];
}

// phi on an x-wall ghost column (forward value, for the corner derivatives).
template <typename T>
__device__ __forceinline__ T xghost(const KParams<T>& P, const T* phi, int side, int y) {
    return side == 0 ? wet_ghost(P, 0, phi_at(P, phi, 0, y), phi_at(P, phi, 1, y))
                     : wet_ghost(P, 1, phi_at(P, phi, P.nx - 1, y), phi_at(P, phi, P.nx - 2, y));
}

constexpr int EDGE_THREADS = 1024;

template <typename T>
__global__ __launch_bounds__(EDGE_THREADS) void k_adj_edges(KParams<T> P, const char* tape, size_t slot, int j,
                                                            AdjView<T> V) {
    __shared__ T corner[2][2][2];          // [side x][side y][depth]: adjoint added to x-ghost rows
    __shared__ double red[4][EDGE_THREADS];
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    AdjHeader* H = V.hdr();
    if (H->status != 0) return;
    const int tid = threadIdx.x;
    const Copy<T> S = copy_at<T>(const_cast<char*>(tape + TAPE_HDR + (size_t)j * slot), P.plane);
    double th[4] = {0.0, 0.0, 0.0, 0.0};
    for (int lev = 0; lev < (n == 0 ? 1 : 2); lev++) {
        const T* phi = lev ? S.h : V.s(S_PHI);
        // corner ghosts: y-wall ghosts of the x-ghost columns
        if (tid == 0 && P.wall_x && P.wall_y) {
            for (int sx = 0; sx < 2; sx++)
                for (int sy = 0; sy < 2; sy++) {
                    const int X = sx ? P.nx : -1, Y = sy ? P.ny : -1;
                    const int y1 = sy ? P.ny - 1 : 0, y2 = sy ? P.ny - 2 : 1;
                    const T q = ext_adjoint(P, V, lev, X, Y);
                    T d1, d2, dth;
                    wet_ghost_grad(P, 2 + sy, xghost(P, phi, sx, y1), xghost(P, phi, sx, y2), d1, d2, dth);
                    corner[sx][sy][0] = d1 * q;
                    corner[sx][sy][1] = d2 * q;
                    th[2 + sy] += (double)(dth * q);
                }
        }
        __syncthreads();
        if (P.wall_y) {
            for (int X = tid; X < P.nx; X += EDGE_THREADS)
                for (int sy = 0; sy < 2; sy++) {
                    const int Y = sy ? P.ny : -1;
                    const int y1 = sy ? P.ny - 1 : 0, y2 = sy ? P.ny - 2 : 1;
                    const T q = ext_adjoint(P, V, lev, X, Y);
                    T d1, d2, dth;
                    wet_ghost_grad(P, 2 + sy, phi_at(P, phi, X, y1), phi_at(P, phi, X, y2), d1, d2, dth);
                    V.e(lev, 2 + sy, 0)[X] = d1 * q;
                    V.e(lev, 2 + sy, 1)[X] = d2 * q;
                    th[2 + sy] += (double)(dth * q);
                }
        }
        if (P.wall_x) {
            for (int Y = tid; Y < P.ny; Y += EDGE_THREADS)
                for (int sx = 0; sx < 2; sx++) {
                    const int X = sx ? P.nx : -1;
                    T q = ext_adjoint(P, V, lev, X, Y);
                    if (P.wall_y) {
                        if (Y == 0) q += corner[sx][0][0];
                        if (Y == 1) q += corner[sx][0][1];
                        if (Y == P.ny - 1) q += corner[sx][1][0];
                        if (Y == P.ny - 2) q += corner[sx][1][1];
                    }
                    const int x1 = sx ? P.nx - 1 : 0, x2 = sx ? P.nx - 2 : 1;
                    T d1, d2, dth;
                    wet_ghost_grad(P, sx, phi_at(P, phi, x1, Y), phi_at(P, phi, x2, Y), d1, d2, dth);
                    V.e(lev, sx, 0)[Y] = d1 * q;
                    V.e(lev, sx, 1)[Y] = d2 * q;
                    th[sx] += (double)(dth * q);
                }
        }
        __syncthreads();   // corner[] is rewritten by the next level
    }
    for (int k = 0; k < 4; k++) red[k][tid] = th[k];
    __syncthreads();
    for (int w = EDGE_THREADS / 2; w > 0; w >>= 1) {
        if (tid < w)
            for (int k = 0; k < 4; k++) red[k][tid] += red[k][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        double* pth = V.part + 2 * V.ntA;
        for (int k = 0; k < 4; k++) pth[k] += red[k][0];
        H->level = n;
    }
}

// ---------------------------------------------------------------- adjoint step, kernel B
template <typename T>
__global__ void k_adj_gather(KParams<T> P, const char* tape, int j, AdjView<T> V) {
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    if (V.hdr()->status != 0) return;
    const bool first = n == 0;
    const int co = (int)(n & 1);
    const long long nn = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / P.nx), x = (int)(k - (long long)y * P.nx);
        for (int lev = 0; lev < (first ? 1 : 2); lev++) {
            T acc = V.s(lev ? S_PHP : S_PHIC)[k] + ext_adjoint(P, V, lev, x, y);
            if (P.wall_x) {
                if (x == 0) acc += V.e(lev, 0, 0)[y];
                if (x == 1) acc += V.e(lev, 0, 1)[y];
                if (x == P.nx - 1) acc += V.e(lev, 1, 0)[y];
                if (x == P.nx - 2) acc += V.e(lev, 1, 1)[y];
            }
            if (P.wall_y) {
                if (y == 0) acc += V.e(lev, 2, 0)[x];
                if (y == 1) acc += V.e(lev, 2, 1)[x];
                if (y == P.ny - 1) acc += V.e(lev, 3, 0)[x];
                if (y == P.ny - 2) acc += V.e(lev, 3, 1)[x];
            }
            if (lev == 0) {
                for (int i = 0; i < Q; i++) V.plane_of(co, i)[k] += acc;   // phi = sum_i f_i
            } else {
                V.plane_of(co, 18)[k] = acc;
            }
        }
        if (first) V.plane_of(co, 18)[k] = T(0);
    }
}

// ---------------------------------------------------------------- seed, init, parameters
template <typename T>
__global__ void k_adj_seed(KParams<T> P, const char* state, size_t off_stamp, AdjView<T> V, const T* dL) {
    const int64_t N = *reinterpret_cast<const int64_t*>(state + off_stamp);
    const int c = (int)(N & 1);
    const long long nn = (long long)P.nx * P.ny;
    const long long nslot = 2LL * V.ntA + 4;
    const long long lim = nn > nslot ? nn : nslot;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < lim;
         k += (long long)gridDim.x * blockDim.x) {
        if (k < nn) {
            const T d = dL[k];
            for (int i = 0; i < Q; i++) V.plane_of(c, i)[k] = d;
            for (int i = 9; i < ADJ_PLANES; i++) V.plane_of(c, i)[k] = T(0);
        }
        if (k < nslot) V.part[k] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        V.hdr()->level = N;
        V.hdr()->status = 0;
    }
}

template <typename T>
__global__ void k_adj_import(KParams<T> P, AdjView<T> V, const T* fb, const T* gb, const T* hb, int64_t level) {
    const int c = (int)(level & 1);
    const long long nn = (long long)P.nx * P.ny;
    const long long nslot = 2LL * V.ntA + 4;
    const long long lim = nn > nslot ? nn : nslot;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < lim;
         k += (long long)gridDim.x * blockDim.x) {
        if (k < nn) {
            for (int i = 0; i < Q; i++) V.plane_of(c, i)[k] = fb ? fb[i * nn + k] : T(0);
            for (int i = 0; i < Q; i++) V.plane_of(c, 9 + i)[k] = gb ? gb[i * nn + k] : T(0);
            for (int i = 0; i < 3; i++) V.plane_of(c, 18 + i)[k] = hb ? hb[i * nn + k] : T(0);
        }
        if (k < nslot) V.part[k] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        V.hdr()->level = level;
        V.hdr()->status = 0;
    }
}

template <typename T>
__global__ void k_adj_export(KParams<T> P, AdjView<T> V, T* fb, T* gb, T* hb) {
    const int c = (int)(V.hdr()->level & 1);
    const long long nn = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
         k += (long long)gridDim.x * blockDim.x) {
        if (fb)
            for (int i = 0; i < Q; i++) fb[i * nn + k] = V.plane_of(c, i)[k];
        if (gb)
            for (int i = 0; i < Q; i++) gb[i * nn + k] = V.plane_of(c, 9 + i)[k];
        if (hb)
            for (int i = 0; i < 3; i++) hb[i * nn + k] = V.plane_of(c, 18 + i)[k];
    }
}

// dL/dphi0 through the level-0 state of lbm_init with zero velocity:
// f_i^0 = w_i phi0 (the equilibrium of Eq. MfMRAC1 at u = 0), and g^0 does not
// depend on phi0 at u = 0.
template <typename T>
__global__ void k_adj_init(KParams<T> P, AdjView<T> V, T* out) {
    const bool ok = V.hdr()->level == 0 && V.hdr()->status == 0;
    const long long nn = (long long)P.nx * P.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
         k += (long long)gridDim.x * blockDim.x) {
        if (!ok) {
            out[k] = T(NAN);
            continue;
        }
        const T a = V.plane_of(0, 1)[k] + V.plane_of(0, 2)[k] + V.plane_of(0, 3)[k] + V.plane_of(0, 4)[k];
        const T d = V.plane_of(0, 5)[k] + V.plane_of(0, 6)[k] + V.plane_of(0, 7)[k] + V.plane_of(0, 8)[k];
        out[k] = (T(4) / T(9)) * V.plane_of(0, 0)[k] + (T(1) / T(9)) * a + (T(1) / T(36)) * d;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_reduce(AdjView<T> V) {
    __shared__ double red[2][256];
    const int tid = threadIdx.x;
    double sx = 0.0, sy = 0.0;
    for (int b = tid; b < V.ntA; b += 256) {
        sx += V.part[2 * b];
        sy += V.part[2 * b + 1];
    }
    red[0][tid] = sx;
    red[1][tid] = sy;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        AdjHeader* H = V.hdr();
        H->result[0] = red[0][0];
        H->result[1] = red[1][0];
        for (int k = 0; k < 4; k++) H->result[2 + k] = V.part[2 * V.ntA + k];
    }
}

// ---------------------------------------------------------------- host side
static int grid1d(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

template <typename T>
static void launch_tape_steps(const KParams<T>& P, char* tape, size_t slot, int nlevels, int ty, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX;
    dim3 blk(TX, BY);
    const bool small = slot < (size_t(1) << 32);
    for (int j = 0; j + 1 < nlevels; j++) {
        if (ty == 4) {
            const int nty = (P.ny + 3) / 4;
            if (small) k_tape_step<T, 4, uint32_t><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
            else k_tape_step<T, 4, uint64_t><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
        } else if (ty == 8 || sizeof(T) == 8) {
            const int nty = (P.ny + 7) / 8;
            if (small) k_tape_step<T, 8, uint32_t><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
            else k_tape_step<T, 8, uint64_t><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
        } else {
            constexpr int TY16 = sizeof(T) == 8 ? 8 : 16;
            const int nty = (P.ny + TY16 - 1) / TY16;
            if (small) k_tape_step<T, TY16, uint32_t><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
            else k_tape_step<T, TY16, uint64_t><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
        }
    }
}

template <typename T>
static void launch_adj_step(const KParams<T>& P, const char* tape, size_t slot, int j, const AdjView<T>& V,
                            hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + ATY - 1) / ATY;
    k_adj_local<T><<<ntx * nty, dim3(TX, BY), 0, s>>>(P, tape, slot, j, V);
    k_adj_edges<T><<<1, EDGE_THREADS, 0, s>>>(P, tape, slot, j, V);
    k_adj_gather<T><<<grid1d((long long)P.nx * P.ny), 256, 0, s>>>(P, tape, j, V);
}

}  // namespace lbm

using namespace lbm;

extern "C" {

int lbm_tape_size(const lbm_params* p, int32_t nlevels, size_t* nbytes) {
    int rc = validate(p);
    if (rc) return rc;
    if (!nbytes) return LBM_E_NULL;
    if (nlevels < 1) return LBM_E_SIZE;
    *nbytes = TAPE_HDR + (size_t)nlevels * layout_of(p).buf_bytes;
    return LBM_OK;
}

int lbm_tape_record(const lbm_params* p, const void* state, void* tape, int32_t nlevels, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state || !tape) return LBM_E_NULL;
    if (nlevels < 1) return LBM_E_SIZE;
    if ((uintptr_t)tape % 256) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    k_tape_copy<<<grid1d((long long)(L.buf_bytes / 16)), 256, 0, s>>>((const char*)state, L.off_buf[0], L.off_buf[1],
                                                                       L.off_stamp, L.buf_bytes, (char*)tape, nlevels,
                                                                       p->nx, p->ny, p->dtype);
    const int ty = step_tile_rows(p);
    if (p->dtype == LBM_F32) launch_tape_steps<float>(resolve<float>(p, L), (char*)tape, L.buf_bytes, nlevels, ty, s);
    else launch_tape_steps<double>(resolve<double>(p, L), (char*)tape, L.buf_bytes, nlevels, ty, s);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_size(const lbm_params* p, size_t* nbytes) {
    int rc = validate(p);
    if (rc) return rc;
    if (!nbytes) return LBM_E_NULL;
    *nbytes = adj_layout_of(p).total;
    return LBM_OK;
}

int lbm_adjoint_phi(const lbm_params* p, const void* state, void* adj, const void* dL_dphi, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!state || !adj || !dL_dphi) return LBM_E_NULL;
    if ((uintptr_t)adj % 256) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    const long long lim = std::max<long long>((long long)p->nx * p->ny, 2LL * A.ntA + 4);
    if (p->dtype == LBM_F32)
        k_adj_seed<float><<<grid1d(lim), 256, 0, s>>>(resolve<float>(p, L), (const char*)state, L.off_stamp,
                                                       adj_view<float>(adj, A), (const float*)dL_dphi);
    else
        k_adj_seed<double><<<grid1d(lim), 256, 0, s>>>(resolve<double>(p, L), (const char*)state, L.off_stamp,
                                                        adj_view<double>(adj, A), (const double*)dL_dphi);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_step(const lbm_params* p, const void* tape, int32_t j, void* adj, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!tape || !adj) return LBM_E_NULL;
    if (j < 0) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == LBM_F32)
        launch_adj_step<float>(resolve<float>(p, L), (const char*)tape, L.buf_bytes, j, adj_view<float>(adj, A), s);
    else
        launch_adj_step<double>(resolve<double>(p, L), (const char*)tape, L.buf_bytes, j, adj_view<double>(adj, A), s);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_init(const lbm_params* p, const void* adj, void* dL_dphi0, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!adj || !dL_dphi0) return LBM_E_NULL;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    const long long nn = (long long)p->nx * p->ny;
    if (p->dtype == LBM_F32)
        k_adj_init<float><<<grid1d(nn), 256, 0, s>>>(resolve<float>(p, L), adj_view<float>((void*)adj, A),
                                                      (float*)dL_dphi0);
    else
        k_adj_init<double><<<grid1d(nn), 256, 0, s>>>(resolve<double>(p, L), adj_view<double>((void*)adj, A),
                                                       (double*)dL_dphi0);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_params(const lbm_params* p, const void* adj, double* out, int64_t* level, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!adj || !out) return LBM_E_NULL;
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == LBM_F32) k_adj_reduce<float><<<1, 256, 0, s>>>(adj_view<float>((void*)adj, A));
    else k_adj_reduce<double><<<1, 256, 0, s>>>(adj_view<double>((void*)adj, A));
    AdjHeader h;
    hipError_t e = hipMemcpyAsync(&h, adj, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    for (int k = 0; k < 6; k++) out[k] = h.result[k];
    if (level) *level = h.level;
    return h.status ? LBM_E_PARAM : LBM_OK;
}

int lbm_adjoint_export(const lbm_params* p, const void* adj, void* fbar, void* gbar, void* hbar, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!adj) return LBM_E_NULL;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    const long long nn = (long long)p->nx * p->ny;
    if (p->dtype == LBM_F32)
        k_adj_export<float><<<grid1d(nn), 256, 0, s>>>(resolve<float>(p, L), adj_view<float>((void*)adj, A),
                                                        (float*)fbar, (float*)gbar, (float*)hbar);
    else
        k_adj_export<double><<<grid1d(nn), 256, 0, s>>>(resolve<double>(p, L), adj_view<double>((void*)adj, A),
                                                         (double*)fbar, (double*)gbar, (double*)hbar);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_import(const lbm_params* p, void* adj, const void* fbar, const void* gbar, const void* hbar,
                       int64_t level, void* stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!adj) return LBM_E_NULL;
    if (level < 0) return LBM_E_SIZE;
    if ((uintptr_t)adj % 256) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    const long long lim = std::max<long long>((long long)p->nx * p->ny, 2LL * A.ntA + 4);
    if (p->dtype == LBM_F32)
        k_adj_import<float><<<grid1d(lim), 256, 0, s>>>(resolve<float>(p, L), adj_view<float>(adj, A),
                                                         (const float*)fbar, (const float*)gbar, (const float*)hbar,
                                                         level);
    else
        k_adj_import<double><<<grid1d(lim), 256, 0, s>>>(resolve<double>(p, L), adj_view<double>(adj, A),
                                                          (const double*)fbar, (const double*)gbar,
                                                          (const double*)hbar, level);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

}  // extern "C"
