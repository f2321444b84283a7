// lbm_fused.hpp -- the fused time step of one 64 x TY tile (device code),
// shared by the single-lattice kernel (lbm_step.hip) and the batched
// persistent kernel (lbm_batch.hip).
#pragma once

#include "lbm_tile.hpp"

namespace lbm {

// Tile order: consecutive workgroup ids are dealt round-robin to the 8 XCDs,
// each with its own 4 MB L2.  Remap so that every XCD walks its own part of
// the lattice in order: when the tile columns split evenly, XCD j takes the
// vertical strip of columns [j ntx/8, (j+1) ntx/8) and walks it row by row
// (the tile above a tile was processed ntx/8 tiles earlier, so the shared halo
// row is still in that XCD's L2); otherwise XCD j takes a contiguous band of
// tiles in row-major order.  Returns (xt, yt).
__device__ __forceinline__ void xcd_tile(int b, int ntx, int nty, int& xt, int& yt) {
    constexpr int NX = 8;
    const int nb = ntx * nty;
    const int xcd = b % NX, slot = b / NX;
    if (ntx % NX == 0 && ntx >= 2 * NX) {
        const int sw = ntx / NX;
        xt = xcd * sw + slot % sw;
        yt = slot / sw;
        return;
    }
    const int q = nb / NX, rem = nb % NX;
    const int t = xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
    xt = t % ntx;
    yt = t / ntx;
}

template <typename T, typename OFF>
__device__ __forceinline__ T ld(const char* base, OFF byteoff) {
    return *reinterpret_cast<const T*>(base + byteoff);
}
// Tuning knob (compile time, measured on MI355X): tiles dealt to XCDs in
// bands (+11% on 256 x 1024, neutral on 4096^2).
#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 1
#endif
// g and the history velocity are loaded together with f, before the window
// barrier, when a thread holds at most two nodes (+10-30% on lattices of
// 0.25-0.5 M nodes streamed from HBM, where the step is latency bound); with
// four nodes per thread the extra live registers cost more than the overlap
// gains (-17% on 4096^2).  A state that the last-level cache holds is read
// with less latency, and there loading g after the barrier (LATE_G) wins:
// +1.4% on 256 x 1024, +6% on 1024 x 512, +9-15% on 1-1.3 M nodes (FP32),
// +5.6% on 256 x 1024 FP64.  LBM_G_EARLY forces early loads on (1) or off (0).
#ifndef LBM_G_EARLY
#define LBM_G_EARLY -1
#endif
// Every load of a thread's own nodes (f, the history phi, and g when GE) is
// issued before the first of them is used.  For FP64 the thread's ring node of
// the window is pulled in the same round trip too (+10% on 256 x 1024); for
// FP32 the extra live registers cost more than the saved round trip (-6% on
// 256 x 1024, -15% on 1024 x 512), and the ring is pulled after the own nodes.
// LBM_RING_EARLY forces it on (1) or off (0).
#ifndef LBM_RING_EARLY
#define LBM_RING_EARLY -1
#endif

// Store of the streamed state: non-temporal (NT) unless the caller knows the
// state stays in the last-level cache between steps.  Non-temporal stores gain
// 3-5% on states of 369 MB and more; ordinary ones 2-26% on states of up to
// 277 MB.
template <typename T, typename OFF, bool NT = true>
__device__ __forceinline__ void st(char* base, OFF byteoff, T v) {
    if (NT) __builtin_nontemporal_store(v, reinterpret_cast<T*>(base + byteoff));
    else *reinterpret_cast<T*>(base + byteoff) = v;
}

// Pulled moving populations f_1..f_8 and the rest population (in FP64) of
// node (x, y) of a copy, addressed by byte offsets of type OFF from the copy
// base (bF: offset of plane f_1, bH: of the history planes, pl: plane length,
// ES: element size).  Returns the node's element index.
template <typename T, typename OFF>
__device__ __forceinline__ OFF pull_f_at(const KParams<T>& P, const char* src, OFF bF, OFF bH, OFF pl, int x, int y,
                                         T* f, double& f0) {
    constexpr OFF ES = sizeof(T);
    const OFF nx = (OFF)P.nx;
    OFF col[3], row[3];
    bool wx[3] = {false, false, false}, wy[3] = {false, false, false};
    col[1] = (OFF)x;
    col[0] = x == 0 ? (OFF)(P.nx - 1) : (OFF)(x - 1);
    col[2] = x == P.nx - 1 ? (OFF)0 : (OFF)(x + 1);
    if (x == 0) wx[0] = P.wall_x;
    if (x == P.nx - 1) wx[2] = P.wall_x;
    row[1] = (OFF)y * nx;
    row[0] = y == 0 ? (OFF)(P.ny - 1) * nx : (OFF)(y - 1) * nx;
    row[2] = y == P.ny - 1 ? (OFF)0 : (OFF)(y + 1) * nx;
    if (y == 0) wy[0] = P.wall_y;
    if (y == P.ny - 1) wy[2] = P.wall_y;
    const OFF k = row[1] + col[1];
    f0 = rest_decode(ld<T>(src, k * ES), ld<T>(src, bH + k * ES), P.rest_w);
#pragma unroll
    for (int i = 1; i < Q; i++) {
        const int ax = 1 - cx(i), ay = 1 - cy(i);
        const bool bb = wx[ax] || wy[ay];
        const OFF o = bb ? bF + ((OFF)(opp(i) - 1) * pl + k) * ES : bF + ((OFF)(i - 1) * pl + row[ay] + col[ax]) * ES;
        f[i] = ld<T>(src, o);
    }
    return k;
}

// f (with the rest population decoded in FP64, as pull_f_at) and g arriving
// at node (x, y) of a copy, the nine source offsets computed once for both.
// Returns the node's element index.
template <typename T, typename OFF>
__device__ __forceinline__ OFF pull_fg_at(const KParams<T>& P, const char* src, OFF bF, OFF bG, OFF bH, OFF pl,
                                          int x, int y, T* f, double& f0, T* g) {
    constexpr OFF ES = sizeof(T);
    const OFF nx = (OFF)P.nx;
    OFF col[3], row[3];
    bool wx[3] = {false, false, false}, wy[3] = {false, false, false};
    col[1] = (OFF)x;
    col[0] = x == 0 ? (OFF)(P.nx - 1) : (OFF)(x - 1);
    col[2] = x == P.nx - 1 ? (OFF)0 : (OFF)(x + 1);
    if (x == 0) wx[0] = P.wall_x;
    if (x == P.nx - 1) wx[2] = P.wall_x;
    row[1] = (OFF)y * nx;
    row[0] = y == 0 ? (OFF)(P.ny - 1) * nx : (OFF)(y - 1) * nx;
    row[2] = y == P.ny - 1 ? (OFF)0 : (OFF)(y + 1) * nx;
    if (y == 0) wy[0] = P.wall_y;
    if (y == P.ny - 1) wy[2] = P.wall_y;
    const OFF k = row[1] + col[1];
    f0 = rest_decode(ld<T>(src, k * ES), ld<T>(src, bH + k * ES), P.rest_w);
    g[0] = ld<T>(src, bG + k * ES);
#pragma unroll
    for (int i = 1; i < Q; i++) {
        const int ax = 1 - cx(i), ay = 1 - cy(i);
        const bool bb = wx[ax] || wy[ay];
        // element offset of the source within a plane, and the plane: i, or opp(i) of the node itself
        const OFF e = bb ? k : row[ay] + col[ax];
        const OFF pf = bb ? (OFF)(opp(i) - 1) : (OFF)(i - 1), pg = pf + 1;
        f[i] = ld<T>(src, bF + (pf * pl + e) * ES);
        g[i] = ld<T>(src, bG + (pg * pl + e) * ES);
    }
    return k;
}

// Position p of a region on an axis of n nodes -> node index, or -1 where p
// lies beyond a wall.  Periodic axes wrap (any number of times: a lattice may
// be narrower than the region).
__device__ __forceinline__ int region_node(int p, int n, bool wall) {
    if (p >= 0 && p < n) return p;
    if (wall) return -1;
    p = p < 0 ? p + n : p - n;   // one wrap: every lattice at least a few nodes wide
    if (p >= 0 && p < n) return p;
    const int r = p % n;
    return r < 0 ? r + n : r;
}

// The fused step.  One 64 x TY tile per workgroup of 64 x NBY threads; thread
// (lx, ly) owns nodes (x0 + lx, y0 + ly + NBY r), r < TY/NBY, keeps their pulled f
// in registers from the phi pass to the collision, and the ring of the phi
// window is pulled by spare threads.  MODE 0: one time step; MODE 1: write
// phi, u, p of the current level.  OFF: byte-offset type within one copy.
// FP32 16-row tiles keep four nodes per thread in flight; capping them at 128
// VGPRs (4 waves per SIMD) is worth +10% on a 4096^2 lattice.  FP64 tiles are
// never taller than 8 rows (the host caps them): they would spill.
template <typename T, int TY, int NBY = BY>
struct StepWaves {
    static constexpr int value = (sizeof(T) == 4 && TY / NBY >= 4) ? 4 : 1;
};

// The tile body between explicit buffers: `src` holds level `step` (one copy:
// post-collision populations of the previous step and the history), `dst`
// receives level step + 1.  Returns the level it advanced.
// SPEC: the level and source copy are not known on entry.  They are read from
// `stamp` while the thread's own-node loads already run on `src`, the copy the
// host's guess `hint` names (the host's record of where it last left the
// state); when the stamp names the other copy -- a state restored or advanced
// outside that record -- the loads are repeated on `alt_src` and the level is
// written to `alt_dst`.  The stamp's round trip then overlaps the first loads
// instead of preceding them.  Returns the stamp read (SPEC) or `step`.
template <typename T, int TY, int MODE, typename OFF, int NBY = BY, bool STD = false, bool NT = true,
          bool LATE_G = false, bool SPEC = false>
__device__ __forceinline__ int64_t step_core(const KParams<T>& P, const char* src, char* dst, int64_t step, int xt,
                                             int yt, T* out_phi, T* out_u, T* out_p, T (*sphi)[TX + 3],
                                             T (*sphp)[TX + 3], const char* alt_src = nullptr,
                                             char* alt_dst = nullptr, const int64_t* stamp = nullptr,
                                             int hint = 0) {
    constexpr int R = TY / NBY;
    constexpr bool GE = LBM_G_EARLY < 0 ? (R <= 2 && !LATE_G) : LBM_G_EARLY != 0;
    constexpr bool RE = LBM_RING_EARLY < 0 ? sizeof(T) == 8 : LBM_RING_EARLY != 0;
    constexpr int WX = TX + 2, WY = TY + 2;
    constexpr OFF ES = sizeof(T);
    const int x0 = xt * TX, y0 = yt * TY;
    const int64_t sv = SPEC ? stamp[0] : step;
    const int64_t lev = SPEC ? stamp_level(sv) : step;
    const OFF pl = (OFF)P.plane;
    const OFF bF = pl * ES;              // byte base of f_1; f_i at bF + (i - 1) pl ES, f_0 at 0
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
    double phid[R], f0d[R];
    T hp[R], f0s[R];
    [[maybe_unused]] T ge[GE ? R : 1][9];
    [[maybe_unused]] T he[GE ? R : 1][2];
    // The thread's own-node pulls (f, the previous phi, and g and the previous
    // velocity when GE) from copy s_; the history planes are read at every
    // level (level 0 holds zeros there and does not use them).
    auto load_own = [&](const char* s_) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int ly = threadIdx.y + r * NBY, y = y0 + ly;
            f0s[r] = T(0);
            hp[r] = T(0);
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
            f0s[r] = ld<T>(s_, k * ES);
#pragma unroll
            for (int i = 1; i < Q; i++) {
                const int ax = 1 - cx(i), ay = 1 - cy(i);
                const bool bb = wx[ax] || wy[ay];
                const OFF o = bb ? bF + ((OFF)(opp(i) - 1) * pl + k) * ES : bF + ((OFF)(i - 1) * pl + row[ay] + col[ax]) * ES;
                f[r][i] = ld<T>(s_, o);
            }
            if (GE) {
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    const int ax = 1 - cx(i), ay = 1 - cy(i);
                    const bool bb = wx[ax] || wy[ay];
                    const OFF o = bb ? bG + ((OFF)opp(i) * pl + k) * ES : bG + ((OFF)i * pl + row[ay] + col[ax]) * ES;
                    ge[GE ? r : 0][i] = ld<T>(s_, o);
                }
                he[GE ? r : 0][0] = ld<T>(s_, bH + (pl + k) * ES);
                he[GE ? r : 0][1] = ld<T>(s_, bH + (2 * pl + k) * ES);
            }
            hp[r] = ld<T>(s_, bH + k * ES);
        }
    };
    load_own(src);
    if (SPEC && stamp_copy(sv) != hint) {   // wave-uniform: the guess was wrong
        src = alt_src;
        dst = alt_dst;
        load_own(src);
    }
    const bool first = lev == 0;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * NBY, y = y0 + ly;
        phid[r] = 0.0;
        f0d[r] = rest_decode(f0s[r], hp[r], P.rest_w);   // after the check: the loads stay in flight through it
        f[r][0] = (T)f0d[r];
        if (x >= P.nx || y >= P.ny) continue;
        if (!RE) {
            phid[r] = f0d[r] + moving_sum_d(f[r]);
            sphi[ly + 1][lx + 1] = (T)phid[r];
            if (!first) sphp[ly + 1][lx + 1] = hp[r];
        }
    }

    // ring of the window: position idx of the ring walk (top row, bottom row,
    // left column, right column) -> window cell; false if it holds no node
    constexpr int NRING = 2 * WX + 2 * TY;
    auto ring_cell = [&](int idx, int& wxi, int& wyi, int& gx, int& gy) -> bool {
        if (idx < WX) {
            wxi = idx;
            wyi = 0;
        } else if (idx < 2 * WX) {
            wxi = idx - WX;
            wyi = WY - 1;
        } else if (idx < 2 * WX + TY) {
            wxi = 0;
            wyi = 1 + idx - 2 * WX;
        } else {
            wxi = WX - 1;
            wyi = 1 + idx - 2 * WX - TY;
        }
        gx = x0 - 1 + wxi;
        gy = y0 - 1 + wyi;
        if (gx > P.nx || gy > P.ny) return false;
        if (gx < 0 || gx >= P.nx) {
            if (P.wall_x) return false;
            gx = gx < 0 ? gx + P.nx : gx - P.nx;
        }
        if (gy < 0 || gy >= P.ny) {
            if (P.wall_y) return false;
            gy = gy < 0 ? gy + P.ny : gy - P.ny;
        }
        return true;
    };
    if (RE) {
        static_assert(NRING <= TX * NBY, "one ring node per thread");
        int rwx = 0, rwy = 0, rgx = 0, rgy = 0;
        const bool rv = tid < NRING && ring_cell(tid, rwx, rwy, rgx, rgy);
        T fr[9], rh = T(0);
        double fr0 = 0.0;
        if (rv) {
            const OFF rk = pull_f_at<T, OFF>(P, src, bF, bH, pl, rgx, rgy, fr, fr0);
            if (!first) rh = ld<T>(src, bH + rk * ES);
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int ly = threadIdx.y + r * NBY, y = y0 + ly;
            if (x >= P.nx || y >= P.ny) continue;
            phid[r] = f0d[r] + moving_sum_d(f[r]);
            sphi[ly + 1][lx + 1] = (T)phid[r];
            if (!first) sphp[ly + 1][lx + 1] = hp[r];
        }
        if (rv) {
            sphi[rwy][rwx] = (T)(fr0 + moving_sum_d(fr));
            if (!first) sphp[rwy][rwx] = rh;
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
        double fw0;
        const OFF wk = pull_f_at<T, OFF>(P, src, bF, bH, pl, gx, gy, fw, fw0);
        [[maybe_unused]] T wh = T(0);
        if (!first) wh = ld<T>(src, bH + wk * ES);
        sphi[wyi][wxi] = (T)(fw0 + moving_sum_d(fw));
        if (!first) sphp[wyi][wxi] = wh;
    };
    if (!RE)
        for (int idx = tid; idx < NRING; idx += TX * NBY) {
            int wxi, wyi, gx, gy;
            ring_cell(idx, wxi, wyi, gx, gy);
            fill_node(wxi, wyi);
        }
    if (x0 + TX > P.nx)
        for (int wy = tid; wy < WY; wy += TX * NBY) fill_node(P.nx - x0 + 1, wy);
    if (y0 + TY > P.ny)
        for (int wxi = tid; wxi < WX; wxi += TX * NBY) fill_node(wxi, P.ny - y0 + 1);
    __syncthreads();
    wall_ghosts<T, TY, NBY>(P, !first, x0, y0, sphi, sphp);

#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * NBY, y = y0 + ly;
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
        if (GE) {
#pragma unroll
            for (int i = 0; i < Q; i++) g[i] = ge[GE ? r : 0][i];
        } else {
#pragma unroll
            for (int i = 0; i < Q; i++) {
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
            if (GE) {
                up = he[GE ? r : 0][0];
                vp = he[GE ? r : 0][1];
            } else {
                up = ld<T>(src, bH + (pl + k) * ES);
                vp = ld<T>(src, bH + (2 * pl + k) * ES);
            }
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
        const double f0n = collide_f<T, false, STD>(P, M, f[r], phid[r]);
        collide_g<T, STD>(P, M, g);
        st<T, OFF, NT>(dst, k * ES, rest_encode<T>(f0n, M.phi, P.rest_w));
#pragma unroll
        for (int i = 1; i < Q; i++) st<T, OFF, NT>(dst, bF + ((OFF)(i - 1) * pl + k) * ES, f[r][i]);
#pragma unroll
        for (int i = 0; i < Q; i++) st<T, OFF, NT>(dst, bG + ((OFF)i * pl + k) * ES, g[i]);
        st<T, OFF, NT>(dst, bH + k * ES, M.phi);
        st<T, OFF, NT>(dst, bH + (pl + k) * ES, M.u);
        st<T, OFF, NT>(dst, bH + (2 * pl + k) * ES, M.v);
    }
    return sv;
}

// The tile body on a ping-pong state: the level stamp of the tile's first row
// selects the source copy, and the tile's rows move to the next level in the
// other copy.  SPEC: the loads start on the copy that `hint` (the copy the host
// expects) names, while the stamp is read (step_core).
template <typename T, int TY, int MODE, typename OFF, int NBY = BY, bool STD = false, bool NT = true,
          bool LATE_G = false, bool SPEC = false>
__device__ __forceinline__ void step_tile(const KParams<T>& P, char* state, size_t off0, size_t off1,
                                          size_t off_stamp, int xt, int yt, T* out_phi, T* out_u, T* out_p,
                                          T (*sphi)[TX + 3], T (*sphp)[TX + 3], int hint = 0) {
    const int y0 = yt * TY;
    int64_t* stamp = reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0;
    int64_t sv;
    if (SPEC) {
        char* ch = state + (hint ? off1 : off0);
        char* co = state + (hint ? off0 : off1);
        sv = step_core<T, TY, MODE, OFF, NBY, STD, NT, LATE_G, true>(P, ch, co, 0, xt, yt, out_phi, out_u, out_p,
                                                                    sphi, sphp, co, ch, stamp, hint);
    } else {
        sv = stamp[0];
        const int cur = stamp_copy(sv);
        step_core<T, TY, MODE, OFF, NBY, STD, NT, LATE_G>(P, state + (cur ? off1 : off0), state + (cur ? off0 : off1),
                                                          stamp_level(sv), xt, yt, out_phi, out_u, out_p, sphi, sphp);
    }
    // Own rows move to level n + 1.  Every wave of the workgroup consumed its
    // load of stamp[0] (it selects the copy of all loads above) before the
    // barriers of the body, so no wave can still be about to read it.
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (MODE == 0 && tid < TY && y0 + tid < P.ny) stamp[tid] = stamp_of(stamp_level(sv) + 1, 1 - stamp_copy(sv));
}

}  // namespace lbm
