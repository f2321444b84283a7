// lbm_ch_step.hpp -- one time step (or the moments) of one 64 x TY tile of the
// two-node-window models (the Cahn-Hilliard variant; the corrected comparison
// model with the Allen-Cahn phase field, ACC) on a ping-pong state, shared by
// the single-lattice kernel (lbm_step.hip) and the batched kernel
// (lbm_batch.hip), so that a case advanced in a batch runs the same body.
#pragma once

#include "lbm_ch.hpp"
#include "lbm_fused.hpp"

namespace lbm {

// MODE 0: one time step, the tile's rows move to the next level; MODE 1:
// phi, u, p of the current level into out_*.  W: the tile's LDS windows.
// STD: the paper's default rates compiled in (P.rates_std).
template <typename T, int TY, int MODE, bool ACC, bool STD = false, bool NT = true, int NBY = BY>
__device__ __forceinline__ void ch_step_tile(const KParams<T>& P, char* state, size_t off0, size_t off1,
                                             size_t off_stamp, int xt, int yt, T* out_phi, T* out_u, T* out_p,
                                             ChWindow<T, TY>& W) {
    const int x0 = xt * TX, y0 = yt * TY;
    int64_t* stamp = reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0;
    const int64_t sv = stamp[0], step = stamp_level(sv);
    const int cur = stamp_copy(sv);
    const Copy<T> S = copy_at<T>(state + (cur ? off1 : off0), P.plane);
    const Copy<T> D = copy_at<T>(state + (cur ? off0 : off1), P.plane);
    ch_tile<T, TY, ACC, NBY>(P, S, step, x0, y0, W, [&](const Macro<T>& M, T* f, T* g, double phid, int, int, long long k) {
        if (MODE == 1) {
            if (out_phi) out_phi[k] = M.phi;
            if (out_u) {
                out_u[k] = M.u;
                out_u[(long long)P.nx * P.ny + k] = M.v;
            }
            if (out_p) out_p[k] = M.p;
            return;
        }
        const double f0n = collide_f<T, !ACC, STD>(P, M, f, phid);
        collide_g<T, STD>(P, M, g);
        const long long pl = P.plane;
        st<T, long long, NT>(reinterpret_cast<char*>(D.f0), (long long)sizeof(T) * k, rest_encode<T>(f0n, M.phi, P.rest_w));
        for (int i = 1; i < Q; i++) st<T, long long, NT>(reinterpret_cast<char*>(D.f), (long long)sizeof(T) * (i * pl + k), f[i]);
        for (int i = 0; i < Q; i++) st<T, long long, NT>(reinterpret_cast<char*>(D.g), (long long)sizeof(T) * (i * pl + k), g[i]);
        st<T, long long, NT>(reinterpret_cast<char*>(D.h), (long long)sizeof(T) * k, M.phi);
        st<T, long long, NT>(reinterpret_cast<char*>(D.h), (long long)sizeof(T) * (pl + k), M.u);
        st<T, long long, NT>(reinterpret_cast<char*>(D.h), (long long)sizeof(T) * (2 * pl + k), M.v);
    });
    // every wave read stamp[0] before the barriers of the tile body
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (MODE == 0 && tid < TY && y0 + tid < P.ny) stamp[tid] = stamp_of(step + 1, 1 - cur);
}

}  // namespace lbm
