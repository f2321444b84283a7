// lbm_tile.hpp -- the 64 x TY tile of the step kernels: LDS window of phi
// with wall ghosts, stencils from the window, end-of-step signalling.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

constexpr int TX = 64;
constexpr int BY = 4;

// phi of node (x, y) in FP64: rest population plus the pulled moving ones.
template <typename T>
__device__ __forceinline__ double node_phi(const KParams<T>& P, const Copy<T>& C, int x, int y, T* f) {
    const long long k = (long long)y * P.nx + x;
    const double f0 = rest_decode(C.f0[k], C.h[k], P.rest_w);
    f[0] = (T)f0;
#pragma unroll
    for (int i = 1; i < Q; i++) f[i] = pull(C.f, P, i, x, y);
    return f0 + moving_sum_d(f);
}

// Wall ghosts of the window (Eq. Dwetting): x-walls first, then y-walls
// across the extended rows, which fixes the corners.  Call after the window
// interior and ring are filled and synchronised; ends synchronised.
template <typename T, int TY, int NBY = BY>
__device__ __forceinline__ void wall_ghosts(const KParams<T>& P, bool need_prev, int x0, int y0,
                                            T (*sphi)[TX + 3], T (*sphp)[TX + 3]) {
    constexpr int WX = TX + 2, WY = TY + 2;
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (P.wall_x) {
        const int wxr = P.nx - x0 + 1;  // window column of x = nx
        for (int wy = tid; wy < WY; wy += TX * NBY) {
            // rows beyond a y-wall get their ghosts below; on a periodic y axis
            // the halo rows -1 and ny hold wrapped rows and need x-ghosts too
            const int gy = y0 - 1 + wy;
            if (gy > P.ny || (P.wall_y && (gy < 0 || gy >= P.ny))) continue;
            if (x0 == 0) {
                sphi[wy][0] = wet_ghost(P, 0, sphi[wy][1], sphi[wy][2]);
                if (need_prev) sphp[wy][0] = wet_ghost(P, 0, sphp[wy][1], sphp[wy][2]);
            }
            if (wxr <= WX - 1) {
                sphi[wy][wxr] = wet_ghost(P, 1, sphi[wy][wxr - 1], sphi[wy][wxr - 2]);
                if (need_prev) sphp[wy][wxr] = wet_ghost(P, 1, sphp[wy][wxr - 1], sphp[wy][wxr - 2]);
            }
        }
        __syncthreads();
    }
    if (P.wall_y) {
        const int wyt = P.ny - y0 + 1;  // window row of y = ny
        for (int wx = tid; wx < WX; wx += TX * NBY) {
            int gx = x0 - 1 + wx;
            if (gx > P.nx) continue;
            if (y0 == 0) {
                sphi[0][wx] = wet_ghost(P, 2, sphi[1][wx], sphi[2][wx]);
                if (need_prev) sphp[0][wx] = wet_ghost(P, 2, sphp[1][wx], sphp[2][wx]);
            }
            if (wyt <= WY - 1) {
                sphi[wyt][wx] = wet_ghost(P, 3, sphi[wyt - 1][wx], sphi[wyt - 2][wx]);
                if (need_prev) sphp[wyt][wx] = wet_ghost(P, 3, sphp[wyt - 1][wx], sphp[wyt - 2][wx]);
            }
        }
        __syncthreads();
    }
}

// Fill the LDS window of phi (and of phi_prev when `need_prev`) for the tile
// at (x0, y0).  Window (wx, wy) is node (x0 - 1 + wx, y0 - 1 + wy).  Periodic
// axes wrap; wall ghosts follow Eq. (Dwetting): x-walls first, then y-walls
// across the extended rows, which fixes the corners.
template <typename T, int TY>
__device__ __forceinline__ void fill_window(const KParams<T>& P, const Copy<T>& C, bool need_prev, int x0,
                                            int y0, T (*sphi)[TX + 3], T (*sphp)[TX + 3]) {
    constexpr int WX = TX + 2, WY = TY + 2;
    const int tid = threadIdx.y * TX + threadIdx.x;
    for (int idx = tid; idx < WX * WY; idx += TX * BY) {
        int wy = idx / WX, wx = idx - wy * WX;
        int gx = x0 - 1 + wx, gy = y0 - 1 + wy;
        if (gx > P.nx || gy > P.ny) continue;
        bool ghost = false;
        if (gx < 0 || gx >= P.nx) {
            if (P.wall_x) ghost = true;
            else gx = gx < 0 ? gx + P.nx : gx - P.nx;
        }
        if (gy < 0 || gy >= P.ny) {
            if (P.wall_y) ghost = true;
            else gy = gy < 0 ? gy + P.ny : gy - P.ny;
        }
        if (ghost) continue;
        T fw[9];
        sphi[wy][wx] = (T)node_phi(P, C, gx, gy, fw);
        if (need_prev) sphp[wy][wx] = C.h[(long long)gy * P.nx + gx];
    }
    __syncthreads();
    wall_ghosts<T, TY>(P, need_prev, x0, y0, sphi, sphp);
}

// The same stencils on any 2-D window array, centred at (wx, wy).
template <typename A, typename T>
__device__ __forceinline__ void win_stencil_at(const A& s, int wx, int wy, T& gx, T& gy, T& lap) {
    stencil(s[wy - 1][wx - 1], s[wy - 1][wx], s[wy - 1][wx + 1], s[wy][wx - 1], s[wy][wx], s[wy][wx + 1],
            s[wy + 1][wx - 1], s[wy + 1][wx], s[wy + 1][wx + 1], gx, gy, lap);
}

template <typename T, int TY>
__device__ __forceinline__ void win_stencil(T (*s)[TX + 3], int wx, int wy, T& gx, T& gy, T& lap) {
    stencil(s[wy - 1][wx - 1], s[wy - 1][wx], s[wy - 1][wx + 1], s[wy][wx - 1], s[wy][wx],
            s[wy][wx + 1], s[wy + 1][wx - 1], s[wy + 1][wx], s[wy + 1][wx + 1], gx, gy, lap);
}

}  // namespace lbm
