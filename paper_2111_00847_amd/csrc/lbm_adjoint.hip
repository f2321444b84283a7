// lbm_adjoint.hip -- reverse mode of the fused step: tapes of forward levels
// and the adjoint step.
//
// Tape.  A segment of the forward trajectory, levels n0 .. n0 + L - 1, each
// one state copy (the same bytes as a ping-pong copy), recorded by running the
// step bodies of lbm_step from slot j into slot j + 1 (the two-level body from
// slot j into slots j + 1 and j + 2 where lbm_step takes two levels per
// launch), so that its levels are bitwise those of the plain path.
//
// Adjoint.  The adjoint of level n holds dL/df^n and dL/dg^n of the
// post-streaming populations and dL/d(phi, u, v) of the history stored at
// level n (the level n-1 fields).  It lives in one of two copies (n & 1) of an
// adjoint buffer, with dL/df_i^n kept as fd_i + phib: the direct part of each
// population and the common part that reaches all nine through phi = sum f_i.
// One adjoint step n+1 -> n runs three kernels:
//   A (k_adj_local, tiles)  recomputes the forward node update of level n from
//       the tape, reads the adjoint of each post-collision population where the
//       population streams to (the reverse of the pull, with bounce-back), and
//       applies node_vjp.  It writes fd, the adjoints of g and of the previous
//       velocity, and the adjoints of the stencil inputs (gradient, Laplacian,
//       centre) to scratch planes, plus per-tile sums of the gravity
//       derivative.
//   G (k_adj_ghosts, one thread per wall ghost)  the adjoint of each ghost (what
//       its neighbours' stencils took from it; for an x-wall ghost next to a
//       y-wall also what the corner ghost built on it took), routed through
//       Eq. Dwetting to its first and second fluid node (edge arrays), and the
//       contact-angle derivatives.
//   B (k_adj_gather, tiles)  the transposed stencils: phib at a node gathers the
//       stencil adjoints of the nodes whose windows hold it and adds the edge
//       arrays of G; likewise for the previous phi of the history.
// Parameter derivatives accumulate into fixed per-workgroup slots (no atomics;
// deterministic) and are summed by lbm_adjoint_params.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/lbm.h"
#include "lbm_adjoint.hpp"
#include "lbm_fused.hpp"
#include "lbm_kernels.hpp"
#include "lbm_step2.hpp"

namespace lbm {

Layout layout_of(const lbm_params* p);
int validate(const lbm_params* p);
int hip_fail(hipError_t e);
void step_shape(const lbm_params* p, int* ty, int* by);
template <typename T>
KParams<T> resolve(const lbm_params* p, const Layout& L);

// The reverse mode covers the Allen-Cahn step with the stencil gradient (present and
// original models) only.
static int validate_ac(const lbm_params* p) {
    const int rc = validate(p);
    if (rc) return rc;
    return p->phase_eq == LBM_ALLEN_CAHN && p->grad_scheme == LBM_GRAD_STENCIL && p->model != LBM_MODEL_CORRECTED
               ? LBM_OK
               : LBM_E_UNSUPPORTED;
}

constexpr size_t ADJ_HDR = 256;
constexpr size_t TAPE_HDR = 256;
constexpr int ATY = 16;   // tiles of kernel A: 64 x 16, one node per thread of 64 x ABY
constexpr int ABY = 16;
constexpr int BTY = BY;   // tiles of kernel B: 64 x 4, one node per thread

struct TapeHeader {
    int64_t n0;
    int32_t nlevels, nx, ny, dtype;
};

struct AdjHeader {
    int64_t level;     // level of the adjoint currently held
    int32_t status;    // 0 ok; 1 an adjoint step met an adjoint of the wrong level; 2 init not at level 0;
                       // 3 a tape without slot j, or recorded for another lattice or dtype
    int32_t nx, ny, dtype;
    double result[6];  // lbm_adjoint_params output
};

// Scratch planes written by A and read by B (S_PHI: phi of level n, only at
// nodes within two of a wall).
enum { S_PHIC = 0, S_GX, S_GY, S_LAP, S_PHP, S_GXP, S_GYP, S_PHI, S_COUNT };
constexpr int ADJ_PLANES = 22;   // fd (9), g (9), history (3), phib
constexpr int P_PHIB = 21;

struct AdjLayout {
    long long plane;
    size_t esz;
    size_t off_copy[2];
    size_t off_scr;
    size_t off_edge;      // G -> B: [level][wall][depth][position along the wall]
    long long emax;
    size_t off_part;      // doubles: 2 per tile of A (gravity), then 4 per workgroup of G (contact angles)
    int ntA, ntB, nB;
    size_t total;
};

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

static int ghost_blocks(const lbm_params* p);

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
    A.ntB = ((p->nx + TX - 1) / TX) * ((p->ny + BTY - 1) / BTY);
    A.nB = ghost_blocks(p);   // workgroups of kernel G
    A.total = al256(A.off_part + (size_t)(2 * A.ntA + 4 * A.nB) * sizeof(double));
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
    int ntA, ntB, nB;
    __device__ AdjHeader* hdr() const { return reinterpret_cast<AdjHeader*>(base); }
    __device__ T* plane_of(int c, int i) const { return copy[c] + (long long)i * plane; }
    __device__ T* s(int i) const { return scr + (long long)i * plane; }
    // lev 0: phi of level n, 1: previous phi; wall 0..3 (x-, x+, y-, y+); depth 0: first fluid node
    __device__ T* e(int lev, int wall, int depth) const { return edge + ((lev * 4 + wall) * 2 + depth) * emax; }
    __device__ long long nslot() const { return 2LL * ntA + 4LL * nB; }
};

template <typename T>
AdjView<T> adj_view(void* adj, const AdjLayout& A) {
    AdjView<T> V;
    V.base = (char*)adj;
    V.plane = A.plane;
    V.copy[0] = reinterpret_cast<T*>(V.base + A.off_copy[0]);
    V.copy[1] = reinterpret_cast<T*>(V.base + A.off_copy[1]);
    V.scr = reinterpret_cast<T*>(V.base + A.off_scr);
    V.part = reinterpret_cast<double*>(V.base + A.off_part);
    V.ntA = A.ntA;
    V.ntB = A.ntB;
    V.nB = A.nB;
    V.edge = reinterpret_cast<T*>(V.base + A.off_edge);
    V.emax = A.emax;
    return V;
}

// Sum over a workgroup of `nw` 64-lane waves (fixed order: deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------- tape
__global__ void k_tape_copy(const char* state, size_t off0, size_t off1, size_t off_stamp, size_t bytes,
                            char* tape, int nlevels, int nx, int ny, int dtype) {
    const int64_t sv = *reinterpret_cast<const int64_t*>(state + off_stamp), n = stamp_level(sv);
    const uint4* src = reinterpret_cast<const uint4*>(state + (stamp_copy(sv) ? off1 : off0));
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

// Tape slot j as the current level of a state: copy 0, and every level stamp
// set to `sv` (that level in copy 0).
__global__ void k_tape_restore(const char* tape, size_t slot, int j, size_t bytes, char* state, size_t off0,
                               size_t off_stamp, size_t nstamp, int64_t sv) {
    const uint4* src = reinterpret_cast<const uint4*>(tape + TAPE_HDR + (size_t)j * slot);
    uint4* dst = reinterpret_cast<uint4*>(state + off0);
    int64_t* stamps = reinterpret_cast<int64_t*>(state + off_stamp);
    const size_t nv = bytes / sizeof(uint4);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nv; i += (size_t)gridDim.x * blockDim.x) {
        dst[i] = src[i];
        if (i < nstamp) stamps[i] = sv;
    }
}

template <typename T, int TY, typename OFF, int NBY, bool STD, bool NT = true>
__global__ __launch_bounds__(TX* NBY) __attribute__((amdgpu_waves_per_eu(StepWaves<T, TY, NBY>::value)))
void k_tape_step(KParams<T> P, char* tape, size_t slot, int j, int ntx, int nty) {
    __shared__ T sphi[TY + 2][TX + 3];
    __shared__ T sphp[TY + 2][TX + 3];
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    char* src = tape + TAPE_HDR + (size_t)j * slot;
    int xt, yt;
    xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    step_core<T, TY, 0, OFF, NBY, STD, NT>(P, src, src + slot, n, xt, yt, nullptr, nullptr, nullptr, sphi, sphp);
}

// Two tape levels per launch (lbm_step2.hpp): slot j to slot j + 1 (the
// intermediate level, stored non-temporally: the adjoint reads it back later)
// and slot j + 2, on the lattices where lbm_step takes two levels per launch;
// bitwise the levels of two k_tape_step launches.
template <typename T, int TY, int NBY, bool STD, bool NTS>
__global__ __launch_bounds__(TX* NBY) void k_tape_step2(KParams<T> P, char* tape, size_t slot, int j, int ntx,
                                                         int nty) {
    __shared__ Step2Lds<T, TY> L;
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    char* src = tape + TAPE_HDR + (size_t)j * slot;
    int xt, yt;
    xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    step2_mid<T, TY, NBY, STD, NTS>(P, src, src + slot, src + 2 * slot, n, xt, yt, L);
}

// ---------------------------------------------------------------- adjoint step, kernel A
// Adjoint of post-collision population i of node (x, y): the population
// streams to (x, y) + c_i, or back to (x, y) as opp(i) through a wall.
// planes: the adjoint copy of level n + 1; returns fd + phib of the receiver.
// Adjoints of post-collision f_i and g_i of node (x, y), read where they
// stream to (fd + phib of the receiver; phib from the LDS window `sb`, whose
// position (wx, wy) is the node's own).
template <typename T, typename OFF>
__device__ __forceinline__ void push_read(const char* cp, OFF pl, const KParams<T>& P, int i, int x, int y,
                                          const T (*sb)[TX + 3], int wx, int wy, T& fo, T& go) {
    constexpr OFF ES = sizeof(T);
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
    const OFF k = bb ? (OFF)y * (OFF)P.nx + (OFF)x : (OFF)ty * (OFF)P.nx + (OFF)tx;
    const OFF d = (OFF)(bb ? opp(i) : i);
    fo = ld<T>(cp, (d * pl + k) * ES) + (bb ? sb[wy][wx] : sb[wy + cy(i)][wx + cx(i)]);
    go = ld<T>(cp, ((9 + d) * pl + k) * ES);
}

// One 64 x ATY tile per workgroup of 64 x ABY threads, ATY / ABY nodes per
// thread.  Every thread pulls its nodes' populations from the tape slot once
// (their phi goes into the LDS window), spare threads pull the window's ring,
// and the node update is recomputed from the registers.  OFF: byte offsets
// within a tape slot and within the adjoint buffer.
template <typename T, typename OFF>
__global__ __launch_bounds__(TX* ABY) void k_adj_local(KParams<T> P, const char* tape, size_t slot, int j,
                                                      AdjView<T> V) {
    constexpr int R = ATY / ABY;
    constexpr int WX = TX + 2, WY = ATY + 2;
    constexpr OFF ES = sizeof(T);
    __shared__ T sphi[ATY + 2][TX + 3];
    __shared__ T sphp[ATY + 2][TX + 3];
    __shared__ T sphib[ATY + 2][TX + 3];   // phib of level n + 1 on the tile and its ring
    __shared__ double red[2][ABY];
    // The tape must hold slot j and have been recorded for this lattice and
    // dtype; otherwise nothing of the tape beyond its header is read, the
    // status records why, and the later kernel of the step (which exits on a
    // non-zero status) and lbm_adjoint_params report it.
    const TapeHeader* TH = reinterpret_cast<const TapeHeader*>(tape);
    const bool tape_ok = j >= 0 && j < TH->nlevels && TH->nx == P.nx && TH->ny == P.ny &&
                         TH->dtype == (sizeof(T) == 8 ? LBM_F64 : LBM_F32);
    const int64_t n = TH->n0 + j;
    AdjHeader* H = V.hdr();
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (!tape_ok || H->status != 0 || H->level != n + 1) {
        if (blockIdx.x == 0 && tid == 0 && H->status == 0) H->status = tape_ok ? 1 : 3;
        return;
    }
    const bool first = n == 0;
    const char* src = tape + TAPE_HDR + (size_t)j * slot;
    const OFF pl = (OFF)P.plane;
    const OFF bF = pl * ES, bG = bF + 8 * pl * ES, bH = bG + 9 * pl * ES;
    const int ntx = (P.nx + TX - 1) / TX;
    int xt, yt;   // tiles dealt to the XCDs as the step deals them: halo rows stay in one L2
    xcd_tile(blockIdx.x, ntx, V.ntA / ntx, xt, yt);
    const int x0 = xt * TX, y0 = yt * ATY;
    const int lx = threadIdx.x;
    const int x = x0 + lx;
    const int ci = (int)((n + 1) & 1), co = (int)(n & 1);
    const char* cin = reinterpret_cast<const char*>(V.copy[ci]);
    const OFF bPB = (OFF)P_PHIB * pl * ES;

    // own nodes: populations, history, phi into the window
    T f[R][9], g[R][9], up[R], vp[R];
    double phid[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * ABY, y = y0 + ly;
        phid[r] = 0.0;
        up[r] = vp[r] = T(0);
        if (x >= P.nx || y >= P.ny) continue;
        double f0;
        const OFF k = pull_fg_at<T, OFF>(P, src, bF, bG, bH, pl, x, y, f[r], f0, g[r]);
        f[r][0] = (T)f0;
        phid[r] = f0 + moving_sum_d(f[r]);
        const T hp = ld<T>(src, bH + k * ES);
        up[r] = ld<T>(src, bH + (pl + k) * ES);
        vp[r] = ld<T>(src, bH + (2 * pl + k) * ES);
        sphi[ly + 1][lx + 1] = (T)phid[r];
        if (!first) sphp[ly + 1][lx + 1] = hp;
        sphib[ly + 1][lx + 1] = ld<T>(cin, bPB + k * ES);
    }
    // the ring of the window, and positions of a ragged tile beyond the
    // lattice that a periodic axis wraps onto nodes
    auto fill = [&](int wx, int wy) {
        const int gx = region_node(x0 - 1 + wx, P.nx, P.wall_x), gy = region_node(y0 - 1 + wy, P.ny, P.wall_y);
        if (gx < 0 || gy < 0) return;
        T fw[9];
        double fw0;
        const OFF k = pull_f_at<T, OFF>(P, src, bF, bH, pl, gx, gy, fw, fw0);
        sphi[wy][wx] = (T)(fw0 + moving_sum_d(fw));
        if (!first) sphp[wy][wx] = ld<T>(src, bH + k * ES);
        sphib[wy][wx] = ld<T>(cin, bPB + k * ES);
    };
    for (int idx = tid; idx < 2 * WX + 2 * ATY; idx += TX * ABY) {
        if (idx < 2 * WX) fill(idx % WX, idx < WX ? 0 : WY - 1);
        else fill(idx < 2 * WX + ATY ? 0 : WX - 1, 1 + (idx - 2 * WX) % ATY);
    }
    if (x0 + TX > P.nx || y0 + ATY > P.ny)
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int ly = threadIdx.y + r * ABY;
            if (x >= P.nx || y0 + ly >= P.ny) fill(lx + 1, ly + 1);
        }
    __syncthreads();
    wall_ghosts<T, ATY, ABY>(P, !first, x0, y0, sphi, sphp);

    char* cout = reinterpret_cast<char*>(V.copy[co]);
    char* scr = reinterpret_cast<char*>(V.scr);
    double gsum_x = 0.0, gsum_y = 0.0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * ABY, y = y0 + ly;
        if (x >= P.nx || y >= P.ny) continue;
        const OFF k = (OFF)y * (OFF)P.nx + (OFF)x;
        T gx, gy, lap, gxp = T(0), gyp = T(0), lp, php = T(0);
        win_stencil<T, ATY>(sphi, lx + 1, ly + 1, gx, gy, lap);
        if (!first) {
            win_stencil<T, ATY>(sphp, lx + 1, ly + 1, gxp, gyp, lp);
            php = sphp[ly + 1][lx + 1];
        }
        const T upr = first ? T(0) : up[r], vpr = first ? T(0) : vp[r];
        const Macro<T> M = macro(P, g[r], sphi[ly + 1][lx + 1], gx, gy, lap, first, php, gxp, gyp, upr, vpr);
        T fo[9], go[9];
#pragma unroll
        for (int i = 0; i < Q; i++) push_read<T, OFF>(cin, pl, P, i, x, y, sphib, lx + 1, ly + 1, fo[i], go[i]);
        const T hphi = ld<T>(cin, (18 * pl + k) * ES), hu = ld<T>(cin, (19 * pl + k) * ES),
                hv = ld<T>(cin, (20 * pl + k) * ES);
        NodeAdj<T> A;
        node_vjp(P, M, f[r], g[r], gx, gy, lap, first, php, gxp, gyp, upr, vpr, fo, go, hphi, hu, hv, A);
#pragma unroll
        for (int i = 0; i < Q; i++) {
            *reinterpret_cast<T*>(cout + ((OFF)i * pl + k) * ES) = A.f[i];
            *reinterpret_cast<T*>(cout + ((OFF)(9 + i) * pl + k) * ES) = A.g[i];
        }
        *reinterpret_cast<T*>(cout + (19 * pl + k) * ES) = first ? T(0) : A.up;
        *reinterpret_cast<T*>(cout + (20 * pl + k) * ES) = first ? T(0) : A.vp;
        const T sv[7] = {A.phic, A.gx, A.gy, A.lap, A.php, A.gxp, A.gyp};   // S_PHIC .. S_GYP
#pragma unroll
        for (int q = 0; q < 7; q++) *reinterpret_cast<T*>(scr + ((OFF)q * pl + k) * ES) = sv[q];
        const bool near_x = P.wall_x && (x < 2 || x >= P.nx - 2);
        const bool near_y = P.wall_y && (y < 2 || y >= P.ny - 2);
        if (near_x || near_y) *reinterpret_cast<T*>(scr + ((OFF)S_PHI * pl + k) * ES) = M.phi;
        gsum_x += (double)A.grav_x;
        gsum_y += (double)A.grav_y;
    }
    // per-tile sums of the gravity derivative, accumulated over the steps of a pass
    gsum_x = wave_sum(gsum_x);
    gsum_y = wave_sum(gsum_y);
    if (lx == 0) {
        red[0][threadIdx.y] = gsum_x;
        red[1][threadIdx.y] = gsum_y;
    }
    __syncthreads();
    if (tid == 0) {
        double sx = 0.0, sy = 0.0;
        for (int w = 0; w < ABY; w++) {
            sx += red[0][w];
            sy += red[1][w];
        }
        V.part[2 * blockIdx.x] += sx;
        V.part[2 * blockIdx.x + 1] += sy;
    }
}

// ---------------------------------------------------------------- wall-ghost helpers (kernel G)
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
// Element k of a plane through a byte offset of type OFF (uint32_t while the
// adjoint buffer and a tape slot stay below 4 GiB: a uniform base and one
// offset register per load).
template <typename T, typename OFF>
__device__ __forceinline__ T at(const T* plane, OFF k) {
    return ld<T, OFF>(reinterpret_cast<const char*>(plane), k * (OFF)sizeof(T));
}
template <typename T, typename OFF>
__device__ __forceinline__ void put(T* plane, OFF k, T v) {
    st<T, OFF, false>(reinterpret_cast<char*>(plane), k * (OFF)sizeof(T), v);
}

template <typename T, typename OFF>
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
            const OFF k = (OFF)ys * (OFF)P.nx + (OFF)xs;
            acc += wgx<T>(-dx, -dy) * at<T, OFF>(sgx, k) + wgy<T>(-dx, -dy) * at<T, OFF>(sgy, k);
            if (!lev) acc += wlap<T>(-dx, -dy) * at<T, OFF>(slp, k);
        }
    return acc;
}

template <typename T, typename OFF>
__device__ __forceinline__ T phi_at(const KParams<T>& P, const T* phi, int x, int y) {
    return at<T, OFF>(phi, (OFF)y * (OFF)P.nx + (OFF)x);
}

// phi on an x-wall ghost column (forward value, for the corner derivatives).
template <typename T, typename OFF>
__device__ __forceinline__ T xghost(const KParams<T>& P, const T* phi, int side, int y) {
    return side == 0 ? wet_ghost(P, 0, phi_at<T, OFF>(P, phi, 0, y), phi_at<T, OFF>(P, phi, 1, y))
                     : wet_ghost(P, 1, phi_at<T, OFF>(P, phi, P.nx - 1, y), phi_at<T, OFF>(P, phi, P.nx - 2, y));
}

// Adjoint of the x-wall ghost (side 0: x = -1, side 1: x = nx) in row y,
// including what the corner ghosts built on it took from it.
template <typename T, typename OFF>
__device__ T xghost_adjoint(const KParams<T>& P, const AdjView<T>& V, int lev, const T* phi, int side, int y) {
    const int X = side ? P.nx : -1;
    T q = ext_adjoint<T, OFF>(P, V, lev, X, y);
    if (P.wall_y) {
        for (int sy = 0; sy < 2; sy++) {
            const int y1 = sy ? P.ny - 1 : 0, y2 = sy ? P.ny - 2 : 1;
            if (y != y1 && y != y2) continue;
            const T qc = ext_adjoint<T, OFF>(P, V, lev, X, sy ? P.ny : -1);
            T c1, c2, cth;
            wet_ghost_grad(P, 2 + sy, xghost<T, OFF>(P, phi, side, y1), xghost<T, OFF>(P, phi, side, y2), c1, c2,
                           cth);
            if (y == y1) q += c1 * qc;
            if (y == y2) q += c2 * qc;
        }
    }
    return q;
}

// ---------------------------------------------------------------- adjoint step, kernel B
// One 64 x 4 tile per workgroup.  The stencil adjoints of the tile and its
// one-node ring are staged in LDS (periodic axes wrap; positions beyond a wall
// hold no node and contribute nothing); every node gathers the nine
// transposed stencil terms, and wall nodes add what kernel G routed to them
// from the ghosts (edge arrays).
template <typename T, typename OFF>
__global__ __launch_bounds__(TX* BY) void k_adj_gather(KParams<T> P, const char* tape, int j, AdjView<T> V) {
    constexpr int WX = TX + 2, WY = BTY + 2;
    __shared__ T sw[5][WY][WX + 1];   // gx, gy, lap of phi^n; gx, gy of phi^{n-1}
    // the header and status are read with the staging loads (all of valid
    // memory); the status gates the stores
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    const int32_t status = V.hdr()->status;
    const int ntx = (P.nx + TX - 1) / TX;
    int xt, yt;   // tiles dealt to the XCDs as kernel A deals its own
    xcd_tile(blockIdx.x, ntx, V.ntB / ntx, xt, yt);
    const int x0 = xt * TX, y0 = yt * BTY;
    const int tid = threadIdx.y * TX + threadIdx.x;
    const T* src[5] = {V.s(S_GX), V.s(S_GY), V.s(S_LAP), V.s(S_GXP), V.s(S_GYP)};
    for (int idx = tid; idx < WX * WY; idx += TX * BY) {
        const int wy = idx / WX, wx = idx - wy * WX;
        int gx = x0 - 1 + wx, gy = y0 - 1 + wy;
        bool none = gx > P.nx || gy > P.ny;
        if (gx < 0 || gx >= P.nx) {
            if (P.wall_x) none = true;
            else gx = gx < 0 ? gx + P.nx : gx - P.nx;
        }
        if (gy < 0 || gy >= P.ny) {
            if (P.wall_y) none = true;
            else gy = gy < 0 ? gy + P.ny : gy - P.ny;
        }
        const OFF k = (OFF)gy * (OFF)P.nx + (OFF)gx;
#pragma unroll
        for (int q = 0; q < 5; q++) sw[q][wy][wx] = none ? T(0) : at<T, OFF>(src[q], k);
    }
    __syncthreads();
    if (status != 0) return;
    const bool first = n == 0;
    const int co = (int)(n & 1);
    if (blockIdx.x == 0 && tid == 0) V.hdr()->level = n;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) return;
    const OFF k = (OFF)y * (OFF)P.nx + (OFF)x;
    // what the wall ghosts built from this node received (kernel G)
    auto edges = [&](int lev) -> T {
        T a = T(0);
        if (P.wall_x) {
            if (x == 0) a += at<T, OFF>(V.e(lev, 0, 0), (OFF)y);
            if (x == 1) a += at<T, OFF>(V.e(lev, 0, 1), (OFF)y);
            if (x == P.nx - 1) a += at<T, OFF>(V.e(lev, 1, 0), (OFF)y);
            if (x == P.nx - 2) a += at<T, OFF>(V.e(lev, 1, 1), (OFF)y);
        }
        if (P.wall_y) {
            if (y == 0) a += at<T, OFF>(V.e(lev, 2, 0), (OFF)x);
            if (y == 1) a += at<T, OFF>(V.e(lev, 2, 1), (OFF)x);
            if (y == P.ny - 1) a += at<T, OFF>(V.e(lev, 3, 0), (OFF)x);
            if (y == P.ny - 2) a += at<T, OFF>(V.e(lev, 3, 1), (OFF)x);
        }
        return a;
    };
    // node (x - dx, y - dy) holds (x, y) at window offset (dx, dy)
    T acc = at<T, OFF>(V.s(S_PHIC), k) + edges(0), accp = T(0);
#pragma unroll
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
            const int wy = ly + 1 - dy, wx = lx + 1 - dx;
            acc += wgx<T>(dx, dy) * sw[0][wy][wx] + wgy<T>(dx, dy) * sw[1][wy][wx] + wlap<T>(dx, dy) * sw[2][wy][wx];
        }
    put<T, OFF>(V.plane_of(co, P_PHIB), k, acc);
    if (!first) {
        accp = at<T, OFF>(V.s(S_PHP), k) + edges(1);
#pragma unroll
        for (int dy = -1; dy <= 1; dy++)
#pragma unroll
            for (int dx = -1; dx <= 1; dx++) {
                const int wy = ly + 1 - dy, wx = lx + 1 - dx;
                accp += wgx<T>(dx, dy) * sw[3][wy][wx] + wgy<T>(dx, dy) * sw[4][wy][wx];
            }
    }
    put<T, OFF>(V.plane_of(co, 18), k, accp);
}

// ---------------------------------------------------------------- adjoint step, kernel G
// Items, per level (the previous level only when n > 0): y-wall ghosts
// (2 nx, when the y axis has walls), then x-wall ghosts (2 ny, when the x axis
// has walls).
constexpr int GHOST_THREADS = 256;

__host__ __device__ inline long long ghost_items(int nx, int ny, bool wall_x, bool wall_y) {
    return (wall_y ? 2LL * nx : 0LL) + (wall_x ? 2LL * ny : 0LL);
}

// Workgroups of kernel G: the first half takes the items of the current phi,
// the second half those of the previous phi (so that every pointer a
// workgroup reads through is uniform).
static int ghost_blocks(const lbm_params* p) {
    const long long per = ghost_items(p->nx, p->ny, p->bc_x == LBM_WALLS, p->bc_y == LBM_WALLS);
    const long long b = (per + GHOST_THREADS - 1) / GHOST_THREADS;
    return 2 * (int)(b < 1 ? 1 : (b > 512 ? 512 : b));
}

template <typename T, typename OFF>
__global__ __launch_bounds__(GHOST_THREADS) void k_adj_ghosts(KParams<T> P, const char* tape, size_t slot, int j,
                                                             AdjView<T> V) {
    __shared__ double red[4][GHOST_THREADS / 64];
    // A chain of a few dependent loads per item bounds this kernel: the
    // header, the status and the workgroup's parameter slots are read together
    // with the items' first loads (every item of both levels reads valid
    // memory), and the status gates the stores instead of the loads.
    const int64_t n = reinterpret_cast<const TapeHeader*>(tape)->n0 + j;
    const int32_t status = V.hdr()->status;
    double* pth = V.part + 2 * V.ntA + 4 * blockIdx.x;
    double pold[4] = {0.0, 0.0, 0.0, 0.0};
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; q++) pold[q] = pth[q];
    const Copy<T> S = copy_at<T>(const_cast<char*>(tape + TAPE_HDR + (size_t)j * slot), P.plane);
    const long long per = ghost_items(P.nx, P.ny, P.wall_x, P.wall_y);
    const long long ny2 = P.wall_y ? 2LL * P.nx : 0LL;
    double th[4] = {0.0, 0.0, 0.0, 0.0};
    const int half = (int)gridDim.x / 2;
    const int lev = (int)blockIdx.x >= half ? 1 : 0;   // uniform over the workgroup
    const T* phi = lev ? S.h : V.s(S_PHI);
    for (long long it = (blockIdx.x - lev * half) * (long long)blockDim.x + threadIdx.x; it < per;
         it += (long long)half * blockDim.x) {
        // item -> (wall, position) by comparisons: it < 2 nx + 2 ny
        int wall, pos;
        T d1, d2, dth, q, cth = T(0), qc = T(0);
        if (it < ny2) {   // y-wall ghost (x, -1) or (x, ny)
            const int sy = it >= P.nx ? 1 : 0, x = (int)(it - (sy ? P.nx : 0));
            const int y1 = sy ? P.ny - 1 : 0, y2 = sy ? P.ny - 2 : 1;
            q = ext_adjoint<T, OFF>(P, V, lev, x, sy ? P.ny : -1);
            wet_ghost_grad(P, 2 + sy, phi_at<T, OFF>(P, phi, x, y1), phi_at<T, OFF>(P, phi, x, y2), d1, d2, dth);
            if (P.wall_x && (x == 0 || x == P.nx - 1)) {   // the corner ghost beside it
                const int side = x == 0 ? 0 : 1;
                qc = ext_adjoint<T, OFF>(P, V, lev, side ? P.nx : -1, sy ? P.ny : -1);
                T c1, c2;
                wet_ghost_grad(P, 2 + sy, xghost<T, OFF>(P, phi, side, y1), xghost<T, OFF>(P, phi, side, y2), c1, c2,
                               cth);
            }
            wall = 2 + sy;
            pos = x;
        } else {          // x-wall ghost (-1, y) or (nx, y)
            const long long i2 = it - ny2;
            const int sx = i2 >= P.ny ? 1 : 0, y = (int)(i2 - (sx ? P.ny : 0));
            const int x1 = sx ? P.nx - 1 : 0, x2 = sx ? P.nx - 2 : 1;
            q = xghost_adjoint<T, OFF>(P, V, lev, phi, sx, y);
            wet_ghost_grad(P, sx, phi_at<T, OFF>(P, phi, x1, y), phi_at<T, OFF>(P, phi, x2, y), d1, d2, dth);
            wall = sx;
            pos = y;
        }
        if (status == 0 && (lev == 0 || n > 0)) {   // the previous level only when n > 0
            put<T, OFF>(V.e(lev, wall, 0), (OFF)pos, d1 * q);
            put<T, OFF>(V.e(lev, wall, 1), (OFF)pos, d2 * q);
            th[wall] += (double)(dth * q);
            if (wall >= 2) th[wall] += (double)(cth * qc);
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < 4; q++) {
        const double v = wave_sum(th[q]);
        if (lane == 0) red[q][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0 && status == 0)
        for (int q = 0; q < 4; q++) {
            double t = red[q][0];
            for (int w = 1; w < GHOST_THREADS / 64; w++) t += red[q][w];
            pth[q] = pold[q] + t;
        }
}

// ---------------------------------------------------------------- seed, init, parameters
template <typename T>
__global__ void k_adj_seed(KParams<T> P, const char* state, size_t off_stamp, AdjView<T> V, const T* dL) {
    const int64_t N = stamp_level(*reinterpret_cast<const int64_t*>(state + off_stamp));
    const int c = (int)(N & 1);   // the adjoint's own copies alternate with the level
    const long long nn = (long long)P.nx * P.ny;
    const long long nslot = V.nslot();
    const long long lim = nn > nslot ? nn : nslot;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < lim;
         k += (long long)gridDim.x * blockDim.x) {
        if (k < nn) {
            for (int i = 0; i < P_PHIB; i++) V.plane_of(c, i)[k] = T(0);
            V.plane_of(c, P_PHIB)[k] = dL[k];   // reaches every f_i through phi = sum_i f_i
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
    const long long nslot = V.nslot();
    const long long lim = nn > nslot ? nn : nslot;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < lim;
         k += (long long)gridDim.x * blockDim.x) {
        if (k < nn) {
            for (int i = 0; i < Q; i++) V.plane_of(c, i)[k] = fb ? fb[i * nn + k] : T(0);
            for (int i = 0; i < Q; i++) V.plane_of(c, 9 + i)[k] = gb ? gb[i * nn + k] : T(0);
            for (int i = 0; i < 3; i++) V.plane_of(c, 18 + i)[k] = hb ? hb[i * nn + k] : T(0);
            V.plane_of(c, P_PHIB)[k] = T(0);
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
        if (fb) {
            const T pb = V.plane_of(c, P_PHIB)[k];
            for (int i = 0; i < Q; i++) fb[i * nn + k] = V.plane_of(c, i)[k] + pb;
        }
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
        // sum_i w_i (fd_i + phib) with sum_i w_i = 1
        out[k] = (T(4) / T(9)) * V.plane_of(0, 0)[k] + (T(1) / T(9)) * a + (T(1) / T(36)) * d +
                 V.plane_of(0, P_PHIB)[k];
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
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    if (tid < 4)
        for (int b = 0; b < V.nB; b++) t[0] += V.part[2 * V.ntA + 4 * b + tid];
    __syncthreads();
    if (tid < 4) red[0][tid + 8] = t[0];   // slots 8..11 are free after the tree above
    __syncthreads();
    if (tid == 0) {
        AdjHeader* H = V.hdr();
        H->result[0] = red[0][0];
        H->result[1] = red[1][0];
        for (int k = 0; k < 4; k++) H->result[2 + k] = red[0][8 + k];
    }
}

// ---------------------------------------------------------------- host side
static int grid1d(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

template <typename T, int TY, int NBY>
static void tape_step_launch(const KParams<T>& P, char* tape, size_t slot, int j, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    // the same specialisation as lbm_step, so that the tape holds the forward levels bitwise;
    // ordinary stores while a level and the next fit the last-level cache (the
    // next tape step reads the level just written)
    if (2 * slot <= (size_t)LBM_NT_MIN_BYTES) {
        if (P.rates_std)
            k_tape_step<T, TY, uint32_t, NBY, true, false><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, tape, slot, j, ntx,
                                                                                               nty);
        else
            k_tape_step<T, TY, uint32_t, NBY, false, false><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, tape, slot, j, ntx,
                                                                                                nty);
    } else if (slot < (size_t(1) << 32)) {
        if (P.rates_std)
            k_tape_step<T, TY, uint32_t, NBY, true><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, tape, slot, j, ntx, nty);
        else
            k_tape_step<T, TY, uint32_t, NBY, false><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, tape, slot, j, ntx, nty);
    } else {
        if (P.rates_std)
            k_tape_step<T, TY, uint64_t, NBY, true><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, tape, slot, j, ntx, nty);
        else
            k_tape_step<T, TY, uint64_t, NBY, false><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, tape, slot, j, ntx, nty);
    }
}

template <typename T, int TY, int NBY>
static void tape_step2_launch(const KParams<T>& P, char* tape, size_t slot, int j, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    const dim3 blk(TX, NBY);
    // slot j + 2 with ordinary stores while it and the next fit the last-level cache (the next launch reads it)
    if (2 * slot <= (size_t)LBM_NT_MIN_BYTES) {
        if (P.rates_std) k_tape_step2<T, TY, NBY, true, false><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
        else k_tape_step2<T, TY, NBY, false, false><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
    } else {
        if (P.rates_std) k_tape_step2<T, TY, NBY, true, true><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
        else k_tape_step2<T, TY, NBY, false, true><<<ntx * nty, blk, 0, s>>>(P, tape, slot, j, ntx, nty);
    }
}

// The tile rows of the two-level launch of lbm_step (lbm_step2.hip).
template <typename T>
static void tape_step2(const KParams<T>& P, char* tape, size_t slot, int j, hipStream_t s) {
    const long long ntx = (P.nx + TX - 1) / TX;
    const long long t8 = ntx * ((P.ny + 7) / 8), t16 = ntx * ((P.ny + 15) / 16);
    if constexpr (sizeof(T) == 4) {
        if (t16 <= 256 && t8 > 256) tape_step2_launch<T, 16, 16>(P, tape, slot, j, s);
        else tape_step2_launch<T, 8, 8>(P, tape, slot, j, s);
    } else {
        tape_step2_launch<T, 8, 8>(P, tape, slot, j, s);
    }
}

// The launches of lbm_step: two levels per launch where it takes two (`two`),
// then one-level launches of its shapes (step_shape).
template <typename T>
static void launch_tape_steps(const KParams<T>& P, char* tape, size_t slot, int nlevels, bool two, int ty, int by,
                              hipStream_t s) {
    constexpr int T16 = sizeof(T) == 8 ? 8 : 16;
    int j0 = 0;
    if (two)
        for (; j0 + 2 < nlevels; j0 += 2) tape_step2<T>(P, tape, slot, j0, s);
    for (int j = j0; j + 1 < nlevels; j++) {
        if (ty == 4) tape_step_launch<T, 4, 4>(P, tape, slot, j, s);
        else if (ty == 8 || sizeof(T) == 8) {
            if (by == 8) tape_step_launch<T, 8, 8>(P, tape, slot, j, s);
            else tape_step_launch<T, 8, 4>(P, tape, slot, j, s);
        } else {
            if (by == 8) tape_step_launch<T, T16, 8>(P, tape, slot, j, s);
            else tape_step_launch<T, T16, 4>(P, tape, slot, j, s);
        }
    }
}

template <typename T>
static void launch_adj_step(const KParams<T>& P, const char* tape, size_t slot, int j, const AdjView<T>& V,
                            size_t adj_bytes, hipStream_t s) {
    // 32-bit byte offsets while a tape slot and the adjoint buffer stay below 4 GiB
    if (slot < (size_t(1) << 32) && adj_bytes < (size_t(1) << 32)) {
        k_adj_local<T, uint32_t><<<V.ntA, dim3(TX, ABY), 0, s>>>(P, tape, slot, j, V);
        if (P.wall_x || P.wall_y) k_adj_ghosts<T, uint32_t><<<V.nB, GHOST_THREADS, 0, s>>>(P, tape, slot, j, V);
        k_adj_gather<T, uint32_t><<<V.ntB, dim3(TX, BY), 0, s>>>(P, tape, j, V);
    } else {
        k_adj_local<T, uint64_t><<<V.ntA, dim3(TX, ABY), 0, s>>>(P, tape, slot, j, V);
        if (P.wall_x || P.wall_y) k_adj_ghosts<T, uint64_t><<<V.nB, GHOST_THREADS, 0, s>>>(P, tape, slot, j, V);
        k_adj_gather<T, uint64_t><<<V.ntB, dim3(TX, BY), 0, s>>>(P, tape, j, V);
    }
}

}  // namespace lbm

using namespace lbm;

extern "C" {

int lbm_tape_size(const lbm_params* p, int32_t nlevels, size_t* nbytes) {
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!nbytes) return LBM_E_NULL;
    if (nlevels < 1) return LBM_E_SIZE;
    *nbytes = TAPE_HDR + (size_t)nlevels * layout_of(p).buf_bytes;
    return LBM_OK;
}

int lbm_tape_record(const lbm_params* p, const void* state, void* tape, int32_t nlevels, void* stream) {
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!state || !tape) return LBM_E_NULL;
    if (nlevels < 1) return LBM_E_SIZE;
    if ((uintptr_t)tape % 256) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    k_tape_copy<<<grid1d((long long)(L.buf_bytes / 16)), 256, 0, s>>>((const char*)state, L.off_buf[0], L.off_buf[1],
                                                                       L.off_stamp, L.buf_bytes, (char*)tape, nlevels,
                                                                       p->nx, p->ny, p->dtype);
    int ty, by;
    step_shape(p, &ty, &by);
    const bool two = two_level_path(L, p->nx, p->ny, p->phase_eq, p->model, p->grad_scheme);
    if (p->dtype == LBM_F32)
        launch_tape_steps<float>(resolve<float>(p, L), (char*)tape, L.buf_bytes, nlevels, two, ty, by, s);
    else
        launch_tape_steps<double>(resolve<double>(p, L), (char*)tape, L.buf_bytes, nlevels, two, ty, by, s);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_tape_restore(const lbm_params* p, const void* tape, int32_t j, void* state, void* stream) {
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!state || !tape) return LBM_E_NULL;
    if ((uintptr_t)tape % 256) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    TapeHeader h;
    hipError_t e = hipMemcpyAsync(&h, tape, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    if (h.nx != p->nx || h.ny != p->ny || h.dtype != p->dtype) return LBM_E_PARAM;
    if (j < 0 || j >= h.nlevels) return LBM_E_SIZE;
    // nstamp (one per 64-node band of a row) is below the slot's 16-byte words
    k_tape_restore<<<grid1d((long long)(L.buf_bytes / 16)), 256, 0, s>>>((const char*)tape, L.buf_bytes, j,
                                                                         L.buf_bytes, (char*)state, L.off_buf[0],
                                                                         L.off_stamp, L.nstamp,
                                                                         stamp_of(h.n0 + j, 0));
    e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_size(const lbm_params* p, size_t* nbytes) {
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!nbytes) return LBM_E_NULL;
    *nbytes = adj_layout_of(p).total;
    return LBM_OK;
}

int lbm_adjoint_phi(const lbm_params* p, const void* state, void* adj, const void* dL_dphi, void* stream) {
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!state || !adj || !dL_dphi) return LBM_E_NULL;
    if ((uintptr_t)adj % 256) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    const long long lim = std::max<long long>((long long)p->nx * p->ny, 2LL * A.ntA + 4LL * A.nB);
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
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!tape || !adj) return LBM_E_NULL;
    if (j < 0) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == LBM_F32)
        launch_adj_step<float>(resolve<float>(p, L), (const char*)tape, L.buf_bytes, j, adj_view<float>(adj, A),
                               A.total, s);
    else
        launch_adj_step<double>(resolve<double>(p, L), (const char*)tape, L.buf_bytes, j, adj_view<double>(adj, A),
                                A.total, s);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_run(const lbm_params* p, const void* tape, int32_t j_first, int32_t count, void* adj,
                    void* stream) {
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!tape || !adj) return LBM_E_NULL;
    if (count < 0 || j_first - count + 1 < 0) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    for (int32_t j = j_first; j > j_first - count; j--) {
        if (p->dtype == LBM_F32)
            launch_adj_step<float>(resolve<float>(p, L), (const char*)tape, L.buf_bytes, j, adj_view<float>(adj, A),
                                   A.total, s);
        else
            launch_adj_step<double>(resolve<double>(p, L), (const char*)tape, L.buf_bytes, j, adj_view<double>(adj, A),
                                    A.total, s);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_adjoint_init(const lbm_params* p, const void* adj, void* dL_dphi0, void* stream) {
    int rc = validate_ac(p);
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
    int rc = validate_ac(p);
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
    int rc = validate_ac(p);
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
    int rc = validate_ac(p);
    if (rc) return rc;
    if (!adj) return LBM_E_NULL;
    if (level < 0) return LBM_E_SIZE;
    if ((uintptr_t)adj % 256) return LBM_E_SIZE;
    const Layout L = layout_of(p);
    const AdjLayout A = adj_layout_of(p);
    hipStream_t s = (hipStream_t)stream;
    const long long lim = std::max<long long>((long long)p->nx * p->ny, 2LL * A.ntA + 4LL * A.nB);
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
