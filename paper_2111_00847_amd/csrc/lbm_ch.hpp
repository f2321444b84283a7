// lbm_ch.hpp -- tile body of the Cahn-Hilliard variant (Sec. 2, Eq. CHE; App. C,
// Eq. MfMRCH1), shared by its step, moments and diagnostics kernels.
//
// The flux D(phi) = grad mu_phi needs mu on a one-node ring around the tile,
// and mu = psi'(phi) - k lap phi needs phi on a two-node ring.  A 64 x TY tile
// (256 threads, TY/4 nodes per thread) fills phi (and the previous phi) on the
// two-node window, the first ghost layer of phi at walls (Eq. Dwetting, x-walls
// first), mu on the one-node window, the ghosts of mu at walls by mirroring
// the first fluid node (zero normal derivative: no diffusive flux through the
// wall; x-walls first), and then hands every node's Macro to a functor.
//
// The same body serves the corrected comparison model with the Allen-Cahn phase
// field (ACC): its interface force F_a = (drho/dphi) u div(M D) (App. A, Eq.
// NS2-add) needs D = grad phi - lambda n on the one-node ring, hence phi on the
// two-node ring.  D takes the place of mu (x component in `mu`, y in `mup`);
// a wall mirrors D of the first fluid node with its normal component reversed.
#pragma once

#include "lbm_fused.hpp"

namespace lbm {

template <typename T, int TY>
struct ChWindow {
    static constexpr int PX = TX + 4, PY = TY + 4;   // phi: node (x0 - 2 + wx, y0 - 2 + wy)
    static constexpr int MX = TX + 2, MY = TY + 2;   // mu: node (x0 - 1 + wx, y0 - 1 + wy)
    T phi[PY][PX + 1];
    T php[PY][PX + 1];
    T mu[MY][MX + 1];
    T mup[MY][MX + 1];
};

// Lattice node held by window coordinate (gx, gy): periodic axes wrap; false
// beyond a wall or beyond the window's reach (gx > lim_x, gy > lim_y).
template <typename T>
__device__ __forceinline__ bool ch_node(const KParams<T>& P, int& gx, int& gy, int lim_x, int lim_y) {
    if (gx > lim_x || gy > lim_y) return false;
    if (gx < 0 || gx >= P.nx) {
        if (P.wall_x) return false;
        gx = ((gx % P.nx) + P.nx) % P.nx;
    }
    if (gy < 0 || gy >= P.ny) {
        if (P.wall_y) return false;
        gy = ((gy % P.ny) + P.ny) % P.ny;
    }
    return true;
}

// phi (and the previous phi) of window position (wx, wy), filled from the
// lattice by the ghost-free rule of ch_node; positions beyond a wall are left
// for the wall-ghost passes.  The copy is addressed by byte offsets of type
// OFF from its base `src` (bF, bH: offsets of plane f_1 and of the history).
template <typename T, int TY, typename OFF>
__device__ __forceinline__ void ch_fill(const KParams<T>& P, const char* src, OFF bF, OFF bH, OFF pl, bool first,
                                        int x0, int y0, int wx, int wy, ChWindow<T, TY>& W) {
    int gx = x0 - 2 + wx, gy = y0 - 2 + wy;
    if (!ch_node(P, gx, gy, P.nx + 1, P.ny + 1)) return;
    T fw[9];
    double f0;
    const OFF k = pull_f_at<T, OFF>(P, src, bF, bH, pl, gx, gy, fw, f0);
    W.phi[wy][wx] = (T)(f0 + moving_sum_d(fw));
    if (!first) W.php[wy][wx] = ld<T>(src, bH + k * (OFF)sizeof(T));
}

// per_node(M, f, g, phid, x, y, k): called for every node of the tile with its
// Macro (Cahn-Hilliard closure), pulled populations f, g and FP64 phi.  The
// copy S is read through byte offsets of type OFF from its base (32-bit ones
// while the copy is below 4 GiB: a uniform base and one offset register per
// load, as the Allen-Cahn step reads its copy).
// Thread (lx, ly) of 64 x NBY owns nodes (x0 + lx, y0 + ly + NBY r), r < TY /
// NBY: their f, g and history are pulled first and kept in registers to the
// collision; the two-node ring of the phi window is pulled afterwards by all
// threads.
template <typename T, int TY, bool ACC = false, int NBY = BY, typename OFF = uint64_t, typename F>
__device__ __forceinline__ void ch_tile(const KParams<T>& P, const Copy<T>& S, int64_t step, int x0, int y0,
                                        ChWindow<T, TY>& W, F&& per_node) {
    using Win = ChWindow<T, TY>;
    static_assert(TY % NBY == 0, "whole thread rows");
    constexpr int R = TY / NBY;
    constexpr int NRING = 4 * Win::PX + 4 * TY;   // two rows above and below, two columns left and right
    const bool first = step == 0;
    const int tid = threadIdx.y * TX + threadIdx.x;
    const int lx = threadIdx.x;
    const char* src = reinterpret_cast<const char*>(S.f0);
    constexpr OFF ES = sizeof(T);
    const OFF pl = (OFF)P.plane;
    const OFF bF = pl * ES, bG = 9 * pl * ES, bH = 18 * pl * ES;
    // 1. own nodes (kept), then the ring of the two-node phi window
    T f[R][9], g[R][9], up[R], vp[R];
    double phid[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * NBY;
        const int x = x0 + lx, y = y0 + ly;
        if (x < P.nx && y < P.ny) {
            double f0d;
            const OFF k = pull_fg_at<T, OFF>(P, src, bF, bG, bH, pl, x, y, f[r], f0d, g[r]);
            f[r][0] = (T)f0d;
            phid[r] = f0d + moving_sum_d(f[r]);
            W.phi[ly + 2][lx + 2] = (T)phid[r];
            if (!first) {
                W.php[ly + 2][lx + 2] = ld<T>(src, bH + k * ES);
                up[r] = ld<T>(src, bH + (pl + k) * ES);
                vp[r] = ld<T>(src, bH + (2 * pl + k) * ES);
            }
        } else {
            ch_fill<T, TY, OFF>(P, src, bF, bH, pl, first, x0, y0, lx + 2, ly + 2, W);   // ragged tile: serves as ring
        }
    }
    for (int idx = tid; idx < NRING; idx += TX * NBY) {
        int wx, wy;
        if (idx < 4 * Win::PX) {
            const int band = idx / Win::PX;
            wx = idx - band * Win::PX;
            wy = band < 2 ? band : TY + band;
        } else {
            const int j = idx - 4 * Win::PX, c = j & 3;
            wy = 2 + (j >> 2);
            wx = c < 2 ? c : TX + c;
        }
        ch_fill<T, TY, OFF>(P, src, bF, bH, pl, first, x0, y0, wx, wy, W);
    }
    __syncthreads();
    // 2. first ghost layer of phi: x-walls on rows that hold nodes, then y-walls across all columns
    if (P.wall_x) {
        const int wr = P.nx - x0 + 2;   // window column of x = nx
        for (int wy = tid; wy < Win::PY; wy += TX * NBY) {
            const int gy = y0 - 2 + wy;
            if (gy > P.ny + 1 || (P.wall_y && (gy < 0 || gy >= P.ny))) continue;
            if (x0 == 0) {
                W.phi[wy][1] = wet_ghost(P, 0, W.phi[wy][2], W.phi[wy][3]);
                if (!first) W.php[wy][1] = wet_ghost(P, 0, W.php[wy][2], W.php[wy][3]);
            }
            if (wr <= Win::PX - 1) {
                W.phi[wy][wr] = wet_ghost(P, 1, W.phi[wy][wr - 1], W.phi[wy][wr - 2]);
                if (!first) W.php[wy][wr] = wet_ghost(P, 1, W.php[wy][wr - 1], W.php[wy][wr - 2]);
            }
        }
        __syncthreads();
    }
    if (P.wall_y) {
        const int wt = P.ny - y0 + 2;   // window row of y = ny
        for (int wx = tid; wx < Win::PX; wx += TX * NBY) {
            const int gx = x0 - 2 + wx;
            if (P.wall_x ? (gx < -1 || gx > P.nx) : gx > P.nx + 1) continue;
            if (y0 == 0) {
                W.phi[1][wx] = wet_ghost(P, 2, W.phi[2][wx], W.phi[3][wx]);
                if (!first) W.php[1][wx] = wet_ghost(P, 2, W.php[2][wx], W.php[3][wx]);
            }
            if (wt <= Win::PY - 1) {
                W.phi[wt][wx] = wet_ghost(P, 3, W.phi[wt - 1][wx], W.phi[wt - 2][wx]);
                if (!first) W.php[wt][wx] = wet_ghost(P, 3, W.php[wt - 1][wx], W.php[wt - 2][wx]);
            }
        }
        __syncthreads();
    }
    // 3. mu (ACC: D) on the one-node window (nodes only)
    for (int idx = tid; idx < Win::MX * Win::MY; idx += TX * NBY) {
        const int wy = idx / Win::MX, wx = idx - wy * Win::MX;
        int gx = x0 - 1 + wx, gy = y0 - 1 + wy;
        if (!ch_node(P, gx, gy, P.nx, P.ny)) continue;
        T gxx, gyy, lap;
        win_stencil_at(W.phi, wx + 1, wy + 1, gxx, gyy, lap);
        if (ACC) {
            T lnx, lny, mx, my;
            mass_flux(P, W.phi[wy + 1][wx + 1], gxx, gyy, lnx, lny, mx, my);
            W.mu[wy][wx] = gxx - lnx;
            W.mup[wy][wx] = gyy - lny;
            continue;
        }
        W.mu[wy][wx] = chem_pot(P, W.phi[wy + 1][wx + 1], lap);
        if (!first) {
            win_stencil_at(W.php, wx + 1, wy + 1, gxx, gyy, lap);
            W.mup[wy][wx] = chem_pot(P, W.php[wy + 1][wx + 1], lap);
        }
    }
    __syncthreads();
    // 4. ghosts: mirror of the first fluid node, x-walls first (ACC: D with its
    //    wall-normal component reversed)
    const T sxx = ACC ? T(-1) : T(1);   // x-walls: factor of mu (ACC: of D_x); D_y keeps its sign
    const T syy = ACC ? T(-1) : T(1);   // y-walls: factor of mu (ACC: of D_y); D_x keeps its sign
    const bool second = ACC || !first;  // mup holds D_y (ACC) or the previous mu
    if (P.wall_x) {
        const int wr = P.nx - x0 + 1;   // mu-window column of x = nx
        for (int wy = tid; wy < Win::MY; wy += TX * NBY) {
            const int gy = y0 - 1 + wy;
            if (gy > P.ny || (P.wall_y && (gy < 0 || gy >= P.ny))) continue;
            if (x0 == 0) {
                W.mu[wy][0] = sxx * W.mu[wy][1];
                if (second) W.mup[wy][0] = W.mup[wy][1];
            }
            if (wr <= Win::MX - 1) {
                W.mu[wy][wr] = sxx * W.mu[wy][wr - 1];
                if (second) W.mup[wy][wr] = W.mup[wy][wr - 1];
            }
        }
        __syncthreads();
    }
    if (P.wall_y) {
        const int wt = P.ny - y0 + 1;
        for (int wx = tid; wx < Win::MX; wx += TX * NBY) {
            const int gx = x0 - 1 + wx;
            if (gx > P.nx) continue;
            if (y0 == 0) {
                W.mu[0][wx] = W.mu[1][wx];
                if (second) W.mup[0][wx] = syy * W.mup[1][wx];
            }
            if (wt <= Win::MY - 1) {
                W.mu[wt][wx] = W.mu[wt - 1][wx];
                if (second) W.mup[wt][wx] = syy * W.mup[wt - 1][wx];
            }
        }
        __syncthreads();
    }
    // 5. the nodes of the tile
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * NBY;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= P.nx || y >= P.ny) continue;
        const long long k = (long long)y * P.nx + x;
        T gx, gy, lap, gmx, gmy, lm, gxp = T(0), gyp = T(0), lp, php = T(0), upr = T(0), vpr = T(0);
        T gmxp = T(0), gmyp = T(0), lmp;
        win_stencil_at(W.phi, lx + 2, ly + 2, gx, gy, lap);
        if (ACC) {
            // div D by Eq. central1: d D_x / dx + d D_y / dy
            T ddx, ddy, t0, t1;
            win_stencil_at(W.mu, lx + 1, ly + 1, ddx, t0, t1);
            win_stencil_at(W.mup, lx + 1, ly + 1, t0, ddy, t1);
            if (!first) {
                php = W.php[ly + 2][lx + 2];
                upr = up[r];
                vpr = vp[r];
            }
            const Macro<T> M = macro<T, false, false, true>(P, g[r], W.phi[ly + 2][lx + 2], gx, gy, lap, first, php,
                                                            T(0), T(0), upr, vpr, T(0), T(0), T(0), T(0), ddx + ddy);
            per_node(M, f[r], g[r], phid[r], x, y, k);
            continue;
        }
        win_stencil_at(W.mu, lx + 1, ly + 1, gmx, gmy, lm);
        if (!first) {
            win_stencil_at(W.php, lx + 2, ly + 2, gxp, gyp, lp);
            win_stencil_at(W.mup, lx + 1, ly + 1, gmxp, gmyp, lmp);
            php = W.php[ly + 2][lx + 2];
            upr = up[r];
            vpr = vp[r];
        }
        const Macro<T> M = macro<T, true, false, true>(P, g[r], W.phi[ly + 2][lx + 2], gx, gy, lap, first, php, gxp, gyp, upr,
                                          vpr, gmx, gmy, gmxp, gmyp, lm);
        per_node(M, f[r], g[r], phid[r], x, y, k);
    }
}

}  // namespace lbm
