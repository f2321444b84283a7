// lbm_step2.hpp -- the tile body of two time levels of the Allen-Cahn step
// (stencil gradients) per launch: the plain two-level launch (lbm_step2.hip)
// and the two-level batch launch (lbm_batch.hip) run it.  The scheme and its
// bitwise equality with two one-level steps are described in lbm_step2.hip.
#pragma once

#include "lbm_fused.hpp"

namespace lbm {

// Wall ghosts (Eq. Dwetting) of a window whose position (wx, wy) is node
// (x0 - H + wx, y0 - H + wy): the rule and order of wall_ghosts (x-walls on
// every row that is not beyond a y-wall, then y-walls across all columns up to
// the x-ghosts), on windows of any halo H.  Ends synchronised.
template <typename T, int WW, int WH, int H, int NT, int PITCH>
__device__ __forceinline__ void ghosts_h(const KParams<T>& P, bool need_prev, int x0, int y0, T (*a)[PITCH],
                                         T (*b)[PITCH]) {
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (P.wall_x) {
        const int wl = H - 1 - x0;          // window column of x = -1
        const int wr = P.nx - x0 + H;       // window column of x = nx
        for (int wy = tid; wy < WH; wy += NT) {
            const int gy = y0 - H + wy;
            if (P.wall_y && (gy < 0 || gy >= P.ny)) continue;
            if (wl >= 0 && wl + 2 < WW) {
                a[wy][wl] = wet_ghost(P, 0, a[wy][wl + 1], a[wy][wl + 2]);
                if (need_prev) b[wy][wl] = wet_ghost(P, 0, b[wy][wl + 1], b[wy][wl + 2]);
            }
            if (wr < WW && wr - 2 >= 0) {
                a[wy][wr] = wet_ghost(P, 1, a[wy][wr - 1], a[wy][wr - 2]);
                if (need_prev) b[wy][wr] = wet_ghost(P, 1, b[wy][wr - 1], b[wy][wr - 2]);
            }
        }
        __syncthreads();
    }
    if (P.wall_y) {
        const int wb = H - 1 - y0;
        const int wt = P.ny - y0 + H;
        for (int wx = tid; wx < WW; wx += NT) {
            const int gx = x0 - H + wx;
            if (P.wall_x && (gx < -1 || gx > P.nx)) continue;
            if (wb >= 0 && wb + 2 < WH) {
                a[wb][wx] = wet_ghost(P, 2, a[wb + 1][wx], a[wb + 2][wx]);
                if (need_prev) b[wb][wx] = wet_ghost(P, 2, b[wb + 1][wx], b[wb + 2][wx]);
            }
            if (wt < WH && wt - 2 >= 0) {
                a[wt][wx] = wet_ghost(P, 3, a[wt - 1][wx], a[wt - 2][wx]);
                if (need_prev) b[wt][wx] = wet_ghost(P, 3, b[wt - 1][wx], b[wt - 2][wx]);
            }
        }
        __syncthreads();
    }
}

template <typename T, int TY>
struct Step2Lds {
    static constexpr int AW = TX + 4, AH = TY + 4;   // region of A: the tile and a two-node ring
    static constexpr int WW = TX + 6, WH = TY + 6;   // phi windows of A: a three-node ring
    static constexpr int GW = TX + 2, GH = TY + 2;   // g of A and the phi window of B: a one-node ring
    T pa[WH][WW + 1];       // phi of level n (with wall ghosts); B's history window
    T pp[WH][WW + 1];       // phi of level n-1 (the history of the copy)
    T fa[Q][AW * AH];       // post-collision f of A (f_0 in the stored encoding)
    T ga[Q][GW * GH];       // post-collision g of A
    T pb[TY + 2][TX + 3];   // phi of level n + 1 (with wall ghosts)
    T ua[TY * TX], va[TY * TX];   // velocity of level n on the tile (B's history)
};

// The local gradient scheme (Eq. local) also hands B m^phiC of level n.
template <typename T, int TY>
struct Step2LdsLocal : Step2Lds<T, TY> {
    T mxa[TY * TX], mya[TY * TX];
};

// Two levels of the tile (xt, yt), with the LDS `L` of the workgroup.
// STAMPED: on a ping-pong state (copies at `state` + off0 and + off1), the
// level stamp of the tile's first row selects the source copy, the tile's rows
// move to level n + 2 in the other copy and their stamps follow.  Otherwise
// level lev in the copy at `src` goes to level lev + 2 in the copy at `dst`,
// and MID also stores the tile's level lev + 1 (what a one-level step would
// write) into the copy at `mid`, non-temporally.  NBY thread rows of 64;
// every thread owns TY / NBY nodes of the tile in B and up to S positions of
// A's region.  NTS: non-temporal stores into the destination copy.  A caller
// that reuses `L` for another tile synchronises first.  P is taken by value:
// by reference the compiler spent 1.3% more VALU instructions on the body.
// LOCAL: the Allen-Cahn step with the local gradient scheme (Eq. local; the
// one-level body of lbm_local_step.hpp): grad phi of levels >= 1 from each
// node's own f and g, a history of five planes (phi, u, v and m^phiC of the
// previous level), no window of the previous phi, and the general collision
// (STD false), as the one-level kernel runs it.
template <typename T, int TY, int NBY, bool STD, bool NTS, bool STAMPED, bool MID = false, bool LOCAL = false,
          typename LdsT = Step2Lds<T, TY>>
__device__ __forceinline__ void step2_body(const KParams<T> P, char* state, size_t off0, size_t off1,
                                           size_t off_stamp, const char* src_in, char* mid, char* dst_in,
                                           int64_t lev_in, int xt, int yt, LdsT& L) {
    using Lds = Step2Lds<T, TY>;
    static_assert(!(LOCAL && (MID || STD)), "the local scheme: no tape, general collision");
    constexpr int AW = Lds::AW, AH = Lds::AH, NA = AW * AH;
    constexpr int WW = Lds::WW, WH = Lds::WH, GW = Lds::GW, GH = Lds::GH;
    constexpr int NT = TX * NBY;
    constexpr int S = (NA + NT - 1) / NT;
    constexpr int NRING3 = 2 * WW + 2 * AH;        // window positions of A outside its region
    constexpr int NRING1 = 2 * GW + 2 * TY;        // window positions of B outside the tile
    constexpr int R = TY / NBY;
    static_assert(TY % NBY == 0, "whole thread rows");
    static_assert(NRING3 <= NT, "one window ring position per thread");
    constexpr uint32_t ES = sizeof(T);

    const int x0 = xt * TX, y0 = yt * TY;
    const int tid = threadIdx.y * TX + threadIdx.x;
    int64_t* stamp = STAMPED ? reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0 : nullptr;
    const int64_t sv = STAMPED ? stamp[0] : 0;
    const int64_t lev = STAMPED ? stamp_level(sv) : lev_in;
    const int cur = stamp_copy(sv);
    const char* src = STAMPED ? state + (cur ? off1 : off0) : src_in;
    char* dst = STAMPED ? state + (cur ? off0 : off1) : dst_in;
    const bool first = lev == 0;
    const uint32_t pl = (uint32_t)P.plane;
    const uint32_t bF = pl * ES, bG = bF + 8 * pl * ES, bH = bG + 9 * pl * ES;

    // ---- A: loads of the region (f, g, history) and of the window ring (f, history phi)
    T f[S][9], g[S][9], hp[S], hu[S], hv[S], hmx[S], hmy[S];
    double f0d[S];
    bool ok[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int idx = tid + s * NT;
        const int ay = idx / AW, ax = idx - ay * AW;
        const int nxi = region_node(x0 - 2 + ax, P.nx, P.wall_x);
        const int nyi = region_node(y0 - 2 + ay, P.ny, P.wall_y);
        ok[s] = idx < NA && nxi >= 0 && nyi >= 0;
        hp[s] = hu[s] = hv[s] = hmx[s] = hmy[s] = T(0);
        f0d[s] = 0.0;
        if (ok[s]) {
            const uint32_t k = pull_fg_at<T, uint32_t>(P, src, bF, bG, bH, pl, nxi, nyi, f[s], f0d[s], g[s]);
            hp[s] = ld<T>(src, bH + k * ES);
            hu[s] = ld<T>(src, bH + (pl + k) * ES);
            hv[s] = ld<T>(src, bH + (2 * pl + k) * ES);
            if constexpr (LOCAL) {
                hmx[s] = ld<T>(src, bH + (3 * pl + k) * ES);
                hmy[s] = ld<T>(src, bH + (4 * pl + k) * ES);
            }
        }
    }
    // ring of the windows: top row, bottom row, left column, right column
    int rwx = 0, rwy = 0;
    bool rok = false;
    T fr[9], rh = T(0);
    double fr0 = 0.0;
    if (tid < NRING3) {
        if (tid < WW) {
            rwx = tid;
            rwy = 0;
        } else if (tid < 2 * WW) {
            rwx = tid - WW;
            rwy = WH - 1;
        } else if (tid < 2 * WW + AH) {
            rwx = 0;
            rwy = 1 + tid - 2 * WW;
        } else {
            rwx = WW - 1;
            rwy = 1 + tid - 2 * WW - AH;
        }
        const int nxi = region_node(x0 - 3 + rwx, P.nx, P.wall_x);
        const int nyi = region_node(y0 - 3 + rwy, P.ny, P.wall_y);
        rok = nxi >= 0 && nyi >= 0;
        if (rok) {
            const uint32_t k = pull_f_at<T, uint32_t>(P, src, bF, bH, pl, nxi, nyi, fr, fr0);
            if constexpr (!LOCAL) rh = ld<T>(src, bH + k * ES);
        }
    }
    double phid[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int idx = tid + s * NT;
        const int ay = idx / AW, ax = idx - ay * AW;
        phid[s] = 0.0;
        if (ok[s]) {
            f[s][0] = (T)f0d[s];
            phid[s] = f0d[s] + moving_sum_d(f[s]);
            L.pa[ay + 1][ax + 1] = (T)phid[s];
            if constexpr (!LOCAL) L.pp[ay + 1][ax + 1] = hp[s];
        }
    }
    if (rok) {
        L.pa[rwy][rwx] = (T)(fr0 + moving_sum_d(fr));
        if constexpr (!LOCAL) L.pp[rwy][rwx] = rh;
    }
    __syncthreads();
    ghosts_h<T, WW, WH, 3, NT, WW + 1>(P, !first && !LOCAL, x0, y0, L.pa, L.pp);

    // ---- A: the step of level n on the region
#pragma unroll
    for (int s = 0; s < S; s++) {
        if (!ok[s]) continue;
        const int idx = tid + s * NT;
        const int ay = idx / AW, ax = idx - ay * AW;
        T gx, gy, lap, gxp = T(0), gyp = T(0), lp, php = T(0), up = T(0), vp = T(0);
        win_stencil_at(L.pa, ax + 1, ay + 1, gx, gy, lap);
        const Macro<T> M = [&]() -> Macro<T> {
            if constexpr (LOCAL) {
                const T phi = L.pa[ay + 1][ax + 1];
                T mpx = T(0), mpy = T(0);
                if (!first) {
                    php = hp[s];
                    up = hu[s];
                    vp = hv[s];
                    mpx = hmx[s];
                    mpy = hmy[s];
                    local_grad(P, f[s], g[s], phi, lap, php * up, php * vp, gx, gy);
                }
                return macro<T, false, true>(P, g[s], phi, gx, gy, lap, first, php, T(0), T(0), up, vp, T(0), T(0),
                                             mpx, mpy);
            } else {
                if (!first) {
                    win_stencil_at(L.pp, ax + 1, ay + 1, gxp, gyp, lp);
                    php = L.pp[ay + 1][ax + 1];
                    up = hu[s];
                    vp = hv[s];
                }
                return macro(P, g[s], L.pa[ay + 1][ax + 1], gx, gy, lap, first, php, gxp, gyp, up, vp);
            }
        }();
        const double f0n = collide_f<T, false, STD>(P, M, f[s], phid[s]);
        const T f0e = rest_encode<T>(f0n, M.phi, P.rest_w);
        L.fa[0][idx] = f0e;
#pragma unroll
        for (int i = 1; i < Q; i++) L.fa[i][idx] = f[s][i];
        if (ax >= 1 && ax < AW - 1 && ay >= 1 && ay < AH - 1) {
            collide_g<T, STD>(P, M, g[s]);
            const int gi = (ay - 1) * GW + (ax - 1);
#pragma unroll
            for (int i = 0; i < Q; i++) L.ga[i][gi] = g[s][i];
            if (ax >= 2 && ax < AW - 2 && ay >= 2 && ay < AH - 2) {
                L.ua[(ay - 2) * TX + (ax - 2)] = M.u;
                L.va[(ay - 2) * TX + (ax - 2)] = M.v;
                if constexpr (LOCAL) {
                    L.mxa[(ay - 2) * TX + (ax - 2)] = M.mx;
                    L.mya[(ay - 2) * TX + (ax - 2)] = M.my;
                }
                const int x = x0 + ax - 2, y = y0 + ay - 2;
                if (MID && x < P.nx && y < P.ny) {   // a node of the tile (not a wrapped position)
                    const uint32_t k = (uint32_t)y * (uint32_t)P.nx + (uint32_t)x;
                    st<T, uint32_t, true>(mid, k * ES, f0e);
#pragma unroll
                    for (int i = 1; i < Q; i++) st<T, uint32_t, true>(mid, bF + ((uint32_t)(i - 1) * pl + k) * ES, f[s][i]);
#pragma unroll
                    for (int i = 0; i < Q; i++) st<T, uint32_t, true>(mid, bG + ((uint32_t)i * pl + k) * ES, g[s][i]);
                    st<T, uint32_t, true>(mid, bH + k * ES, M.phi);
                    st<T, uint32_t, true>(mid, bH + (pl + k) * ES, M.u);
                    st<T, uint32_t, true>(mid, bH + (2 * pl + k) * ES, M.v);
                }
            }
        }
    }
    __syncthreads();

    // ---- B: phi of level n + 1 on the tile and its one-node ring, from A's f
    // Wall sides of position (x, y) that a population pulled there would come
    // from beyond (x-, x+, y-, y+; on a wall axis a position is its node).
    struct Beyond {
        bool xl, xh, yl, yh;
        __device__ bool of(int i) const {
            return (cx(i) > 0 ? xl : (cx(i) < 0 ? xh : false)) || (cy(i) > 0 ? yl : (cy(i) < 0 ? yh : false));
        }
    };
    auto beyond = [&](int x, int y) -> Beyond {
        return Beyond{P.wall_x && x == 0, P.wall_x && x == P.nx - 1, P.wall_y && y == 0, P.wall_y && y == P.ny - 1};
    };
    // f_i arriving at region position (ax, ay) of node (x, y): from position
    // (ax, ay) - c_i, or its own opp(i) where (x, y) - c_i lies beyond a wall.
    auto pull_a = [&](int ax, int ay, int x, int y, T* fo) -> double {
        const int c = ay * AW + ax;
        const Beyond w = beyond(x, y);
#pragma unroll
        for (int i = 1; i < Q; i++) fo[i] = w.of(i) ? L.fa[opp(i)][c] : L.fa[i][c - cy(i) * AW - cx(i)];
        const double f0 = rest_decode(L.fa[0][c], L.pa[ay + 1][ax + 1], P.rest_w);
        fo[0] = (T)f0;
        return f0 + moving_sum_d(fo);
    };
    T fb[R][9];
    double phb[R];
    const int lx = threadIdx.x;
    const int x = x0 + lx;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * NBY, y = y0 + ly;
        phb[r] = 0.0;
        // a ragged tile's positions beyond the lattice hold wrapped nodes on a
        // periodic axis (they are the ring of the tile's last nodes)
        const bool pos = (x < P.nx || !P.wall_x) && (y < P.ny || !P.wall_y);
        if (pos) {
            phb[r] = pull_a(lx + 2, ly + 2, x, y, fb[r]);
            L.pb[ly + 1][lx + 1] = (T)phb[r];
        }
    }
    for (int idx = tid; idx < NRING1; idx += NT) {
        int wx, wy;
        if (idx < GW) {
            wx = idx;
            wy = 0;
        } else if (idx < 2 * GW) {
            wx = idx - GW;
            wy = GH - 1;
        } else if (idx < 2 * GW + TY) {
            wx = 0;
            wy = 1 + idx - 2 * GW;
        } else {
            wx = GW - 1;
            wy = 1 + idx - 2 * GW - TY;
        }
        const int px = x0 - 1 + wx, py = y0 - 1 + wy;
        if (region_node(px, P.nx, P.wall_x) < 0 || region_node(py, P.ny, P.wall_y) < 0) continue;
        T fw[9];
        L.pb[wy][wx] = (T)pull_a(wx + 1, wy + 1, px, py, fw);
    }
    __syncthreads();
    wall_ghosts<T, TY, NBY>(P, false, x0, y0, L.pb, L.pb);

    // ---- B: the step of level n + 1 on the tile, stored into the other copy
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * NBY, y = y0 + ly;
        if (x >= P.nx || y >= P.ny) continue;
        const int c1 = (ly + 1) * GW + (lx + 1);
        const Beyond w = beyond(x, y);
        T gb[9];
#pragma unroll
        for (int i = 0; i < Q; i++) gb[i] = w.of(i) ? L.ga[opp(i)][c1] : L.ga[i][c1 - cy(i) * GW - cx(i)];
        T gx, gy, lap, gxp, gyp, lp;
        win_stencil_at(L.pb, lx + 1, ly + 1, gx, gy, lap);
        const Macro<T> M = [&]() -> Macro<T> {
            if constexpr (LOCAL) {
                const T phi = L.pb[ly + 1][lx + 1], php = L.pa[ly + 3][lx + 3];
                const T up = L.ua[ly * TX + lx], vp = L.va[ly * TX + lx];
                local_grad(P, fb[r], gb, phi, lap, php * up, php * vp, gx, gy);
                return macro<T, false, true>(P, gb, phi, gx, gy, lap, false, php, T(0), T(0), up, vp, T(0), T(0),
                                             L.mxa[ly * TX + lx], L.mya[ly * TX + lx]);
            } else {
                win_stencil_at(L.pa, lx + 3, ly + 3, gxp, gyp, lp);
                return macro(P, gb, L.pb[ly + 1][lx + 1], gx, gy, lap, false, L.pa[ly + 3][lx + 3], gxp, gyp,
                             L.ua[ly * TX + lx], L.va[ly * TX + lx]);
            }
        }();
        const double f0n = collide_f<T, false, STD>(P, M, fb[r], phb[r]);
        collide_g<T, STD>(P, M, gb);
        const uint32_t k = (uint32_t)y * (uint32_t)P.nx + (uint32_t)x;
        st<T, uint32_t, NTS>(dst, k * ES, rest_encode<T>(f0n, M.phi, P.rest_w));
#pragma unroll
        for (int i = 1; i < Q; i++) st<T, uint32_t, NTS>(dst, bF + ((uint32_t)(i - 1) * pl + k) * ES, fb[r][i]);
#pragma unroll
        for (int i = 0; i < Q; i++) st<T, uint32_t, NTS>(dst, bG + ((uint32_t)i * pl + k) * ES, gb[i]);
        st<T, uint32_t, NTS>(dst, bH + k * ES, M.phi);
        st<T, uint32_t, NTS>(dst, bH + (pl + k) * ES, M.u);
        st<T, uint32_t, NTS>(dst, bH + (2 * pl + k) * ES, M.v);
        if constexpr (LOCAL) {
            st<T, uint32_t, NTS>(dst, bH + (3 * pl + k) * ES, M.mx);
            st<T, uint32_t, NTS>(dst, bH + (4 * pl + k) * ES, M.my);
        }
    }
    // every wave read stamp[0] before the barriers above
    if (STAMPED && tid < TY && y0 + tid < P.ny) stamp[tid] = stamp_of(lev + 2, 1 - cur);
}

// Two levels of the tile (xt, yt) of a ping-pong state (copies at off0 and
// off1, level stamps at off_stamp).
template <typename T, int TY, int NBY, bool STD, bool NTS>
__device__ __forceinline__ void step2_tile(const KParams<T>& P, char* state, size_t off0, size_t off1,
                                           size_t off_stamp, int xt, int yt, Step2Lds<T, TY>& L) {
    step2_body<T, TY, NBY, STD, NTS, true>(P, state, off0, off1, off_stamp, nullptr, nullptr, nullptr, 0, xt, yt, L);
}

// The same with the local gradient scheme (Eq. local).
template <typename T, int TY, int NBY, bool NTS>
__device__ __forceinline__ void step2_local_tile(const KParams<T>& P, char* state, size_t off0, size_t off1,
                                                 size_t off_stamp, int xt, int yt, Step2LdsLocal<T, TY>& L) {
    step2_body<T, TY, NBY, false, NTS, true, false, true>(P, state, off0, off1, off_stamp, nullptr, nullptr, nullptr,
                                                          0, xt, yt, L);
}

// Level lev in the copy at `src` to level lev + 2 in the copy at `dst`, the
// intermediate level into the copy at `mid` (tapes).
template <typename T, int TY, int NBY, bool STD, bool NTS>
__device__ __forceinline__ void step2_mid(const KParams<T>& P, const char* src, char* mid, char* dst, int64_t lev,
                                          int xt, int yt, Step2Lds<T, TY>& L) {
    step2_body<T, TY, NBY, STD, NTS, false, true>(P, nullptr, 0, 0, 0, src, mid, dst, lev, xt, yt, L);
}

}  // namespace lbm
