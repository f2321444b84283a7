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
// STD: the paper's default rates compiled in (P.rates_std).  OFF: byte
// offsets within a copy (uint32_t while the copy is below 4 GiB).
template <typename T, int TY, int MODE, bool ACC, bool STD = false, bool NT = true, int NBY = BY,
          typename OFF = uint64_t>
__device__ __forceinline__ void ch_step_tile(const KParams<T>& P, char* state, size_t off0, size_t off1,
                                             size_t off_stamp, int xt, int yt, T* out_phi, T* out_u, T* out_p,
                                             ChWindow<T, TY>& W) {
    const int x0 = xt * TX, y0 = yt * TY;
    int64_t* stamp = reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0;
    const int64_t sv = stamp[0], step = stamp_level(sv);
    const int cur = stamp_copy(sv);
    const Copy<T> S = copy_at<T>(state + (cur ? off1 : off0), P.plane);
    const Copy<T> D = copy_at<T>(state + (cur ? off0 : off1), P.plane);
    char* dst = reinterpret_cast<char*>(D.f0);
    ch_tile<T, TY, ACC, NBY, OFF>(P, S, step, x0, y0, W, [&](const Macro<T>& M, T* f, T* g, double phid, int, int,
                                                           long long k) {
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
        constexpr OFF ES = sizeof(T);
        const OFF pl = (OFF)P.plane, kk = (OFF)k;
        st<T, OFF, NT>(dst, kk * ES, rest_encode<T>(f0n, M.phi, P.rest_w));
#pragma unroll
        for (int i = 1; i < Q; i++) st<T, OFF, NT>(dst, ((OFF)i * pl + kk) * ES, f[i]);
#pragma unroll
        for (int i = 0; i < Q; i++) st<T, OFF, NT>(dst, ((OFF)(9 + i) * pl + kk) * ES, g[i]);
        st<T, OFF, NT>(dst, (18 * pl + kk) * ES, M.phi);
        st<T, OFF, NT>(dst, (19 * pl + kk) * ES, M.u);
        st<T, OFF, NT>(dst, (20 * pl + kk) * ES, M.v);
    });
    // every wave read stamp[0] before the barriers of the tile body
    const int tid = threadIdx.y * TX + threadIdx.x;
    if (MODE == 0 && tid < TY && y0 + tid < P.ny) stamp[tid] = stamp_of(step + 1, 1 - cur);
}

}  // namespace lbm
