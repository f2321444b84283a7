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
template <typename T, int TY, int MODE>
__device__ __forceinline__ void local_step_tile(const KParams<T>& P, char* state, size_t off0, size_t off1,
                                                size_t off_stamp, int xt, int yt, T* out_phi, T* out_u, T* out_p,
                                                T (*sphi)[TX + 3]) {
    constexpr int R = TY / BY;
    const int x0 = xt * TX, y0 = yt * TY;
    int64_t* stamp = reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0;
    const int64_t step = stamp[0];
    const bool first = step == 0;
    const int cur = (int)(step & 1);
    const Copy<T> S = copy_at<T>(state + (cur ? off1 : off0), P.plane);
    const Copy<T> D = copy_at<T>(state + (cur ? off0 : off1), P.plane);
    fill_window<T, TY>(P, S, false, x0, y0, sphi, sphi);   // no previous-level window is needed
    const long long pl = P.plane;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int lx = threadIdx.x, ly = threadIdx.y + r * BY;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= P.nx || y >= P.ny) continue;
        const long long k = (long long)y * P.nx + x;
        T f[9], g[9];
        const double phid = node_phi(P, S, x, y, f);
#pragma unroll
        for (int i = 0; i < Q; i++) g[i] = pull(S.g, P, i, x, y);
        T gx, gy, lap;
        win_stencil_at(sphi, lx + 1, ly + 1, gx, gy, lap);
        const T phi = sphi[ly + 1][lx + 1];
        T php = T(0), up = T(0), vp = T(0), mpx = T(0), mpy = T(0);
        if (!first) {
            php = S.h[k];
            up = S.h[pl + k];
            vp = S.h[2 * pl + k];
            mpx = S.h[3 * pl + k];
            mpy = S.h[4 * pl + k];
            local_grad(P, f, g, phi, lap, php * up, php * vp, gx, gy);
        }
        const Macro<T> M =
            macro<T, false, true>(P, g, phi, gx, gy, lap, first, php, T(0), T(0), up, vp, T(0), T(0), mpx, mpy);
        if (MODE == 1) {
            if (out_phi) out_phi[k] = M.phi;
            if (out_u) {
                out_u[k] = M.u;
                out_u[(long long)P.nx * P.ny + k] = M.v;
            }
            if (out_p) out_p[k] = M.p;
            continue;
        }
        const double f0n = collide_f(P, M, f, phid);
        collide_g(P, M, g);
        st<double, long long>(reinterpret_cast<char*>(D.f0), 8 * k, f0n);
        for (int i = 1; i < Q; i++) st<T, long long>(reinterpret_cast<char*>(D.f), (long long)sizeof(T) * (i * pl + k), f[i]);
        for (int i = 0; i < Q; i++) st<T, long long>(reinterpret_cast<char*>(D.g), (long long)sizeof(T) * (i * pl + k), g[i]);
        const T hv[5] = {M.phi, M.u, M.v, M.mx, M.my};
        for (int j = 0; j < 5; j++) st<T, long long>(reinterpret_cast<char*>(D.h), (long long)sizeof(T) * (j * pl + k), hv[j]);
    }
    // every wave read stamp[0] before the window barrier
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (MODE == 0 && tid < TY && y0 + tid < P.ny) stamp[tid] = step + 1;
}

}  // namespace lbm
