// lbm_local_step.hpp -- one time step (or the moments) of one 64 x TY tile of
// the Allen-Cahn step with the local gradient scheme of Eq. local, shared by
// the single-lattice kernel (lbm_local.hip) and the batched kernel
// (lbm_batch.hip).  grad phi of levels >= 1 from each node's own f and g
// (local_grad), lap phi from the one-node phi window; the history of a copy
// holds phi, u, v and m^phiC of the previous level (5 planes).
#pragma once

#include "lbm_fused.hpp"

namespace lbm {

// MODE 0: one time step, the tile's rows move to the next level; MODE 1:
// phi, u, p of the current level into out_*.  sphi: the tile's phi window.
// OFF: byte offsets within a copy (uint32_t while the copy is below 4 GiB).
template <typename T, int TY, int MODE, bool NT = true, int NBY = BY, typename OFF = uint64_t>
__device__ __forceinline__ void local_step_tile(const KParams<T>& P, char* state, size_t off0, size_t off1,
                                                size_t off_stamp, int xt, int yt, T* out_phi, T* out_u, T* out_p,
                                                T (*sphi)[TX + 3]) {
    static_assert(TY % NBY == 0, "whole thread rows");
    constexpr int R = TY / NBY;
    const int x0 = xt * TX, y0 = yt * TY;
    int64_t* stamp = reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0;
    const int64_t sv = stamp[0], step = stamp_level(sv);
    const bool first = step == 0;
    const int cur = stamp_copy(sv);
    const char* src = state + (cur ? off1 : off0);
    char* dst = state + (cur ? off0 : off1);
    constexpr OFF ES = sizeof(T);
    const OFF pl = (OFF)P.plane;
    const OFF bF = pl * ES, bG = 9 * pl * ES, bH = 18 * pl * ES;
    const int tid = threadIdx.y * TX + threadIdx.x;
    const int lx = threadIdx.x;
    // phi of window position (wx, wy) = node (x0 - 1 + wx, y0 - 1 + wy): periodic
    // axes wrap; positions beyond a wall are left for wall_ghosts
    auto fill = [&](int wx, int wy) {
        int gx = x0 - 1 + wx, gy = y0 - 1 + wy;
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
        double f0;
        pull_f_at<T, OFF>(P, src, bF, bH, pl, gx, gy, fw, f0);
        sphi[wy][wx] = (T)(f0 + moving_sum_d(fw));
    };
    // 1. own nodes first (f, g and the history kept in registers), then the ring
    T f[R][9], g[R][9], hv[R][5];
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
            if (!first)
#pragma unroll
                for (int j = 0; j < 5; j++) hv[r][j] = ld<T>(src, bH + ((OFF)j * pl + k) * ES);
            sphi[ly + 1][lx + 1] = (T)phid[r];
        } else {
            fill(lx + 1, ly + 1);   // ragged tile: the position serves as ring
        }
    }
    constexpr int WX = TX + 2;
    for (int idx = tid; idx < 2 * WX + 2 * TY; idx += TX * NBY) {
        if (idx < 2 * WX) fill(idx % WX, idx < WX ? 0 : TY + 1);
        else fill(idx < 2 * WX + TY ? 0 : WX - 1, 1 + (idx - 2 * WX) % TY);
    }
    __syncthreads();
    wall_ghosts<T, TY, NBY>(P, false, x0, y0, sphi, sphi);
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ly = threadIdx.y + r * NBY;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= P.nx || y >= P.ny) continue;
        const long long k = (long long)y * P.nx + x;
        T gx, gy, lap;
        win_stencil_at(sphi, lx + 1, ly + 1, gx, gy, lap);
        const T phi = sphi[ly + 1][lx + 1];
        T php = T(0), up = T(0), vp = T(0), mpx = T(0), mpy = T(0);
        if (!first) {
            php = hv[r][0];
            up = hv[r][1];
            vp = hv[r][2];
            mpx = hv[r][3];
            mpy = hv[r][4];
            local_grad(P, f[r], g[r], phi, lap, php * up, php * vp, gx, gy);
        }
        const Macro<T> M =
            macro<T, false, true>(P, g[r], phi, gx, gy, lap, first, php, T(0), T(0), up, vp, T(0), T(0), mpx, mpy);
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
        collide_g(P, M, g[r]);
        const OFF kk = (OFF)k;
        st<T, OFF, NT>(dst, kk * ES, rest_encode<T>(f0n, M.phi, P.rest_w));
#pragma unroll
        for (int i = 1; i < Q; i++) st<T, OFF, NT>(dst, ((OFF)i * pl + kk) * ES, f[r][i]);
#pragma unroll
        for (int i = 0; i < Q; i++) st<T, OFF, NT>(dst, ((OFF)(9 + i) * pl + kk) * ES, g[r][i]);
        const T hout[5] = {M.phi, M.u, M.v, M.mx, M.my};
#pragma unroll
        for (int j = 0; j < 5; j++) st<T, OFF, NT>(dst, ((OFF)(18 + j) * pl + kk) * ES, hout[j]);
    }
    // every wave read stamp[0] before the window barrier
    if (MODE == 0 && tid < TY && y0 + tid < P.ny) stamp[tid] = stamp_of(step + 1, 1 - cur);
}

}  // namespace lbm
