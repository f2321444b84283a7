// lbm_local.hip -- the Allen-Cahn step with grad phi from the local scheme of
// Eq. local (levels >= 1; level 0 and lap phi by the stencils of Eqs. central1
// and central2).  The history of a copy then holds phi, u, v and m^phiC of the
// previous level (5 planes), since m^phiC of that level came from its own
// local gradient.  One 64 x 8 tile per workgroup of 64 x 4 threads, the phi
// window with a one-node ring in LDS (for lap phi), tiles dealt to the XCDs as
// for the stencil step, non-temporal stores.
#include "lbm_fused.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

constexpr int LOC_TY = 8;

template <typename T, int MODE>
__global__ __launch_bounds__(TX* BY) void k_step_local(KParams<T> P, char* state, size_t off0, size_t off1,
                                                      size_t off_stamp, int ntx, int nty, T* out_phi, T* out_u,
                                                      T* out_p) {
    constexpr int R = LOC_TY / BY;
    __shared__ T sphi[LOC_TY + 2][TX + 3];
    int xt, yt;
    if (LBM_XCD_REMAP) {
        xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    } else {
        xt = blockIdx.x % ntx;
        yt = blockIdx.x / ntx;
    }
    const int x0 = xt * TX, y0 = yt * LOC_TY;
    int64_t* stamp = reinterpret_cast<int64_t*>(state + off_stamp) + (size_t)xt * P.ny + y0;
    const int64_t step = stamp[0];
    const bool first = step == 0;
    const int cur = (int)(step & 1);
    const Copy<T> S = copy_at<T>(state + (cur ? off1 : off0), P.plane);
    const Copy<T> D = copy_at<T>(state + (cur ? off0 : off1), P.plane);
    fill_window<T, LOC_TY>(P, S, false, x0, y0, sphi, sphi);   // no previous-level window is needed
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
    if (MODE == 0 && tid < LOC_TY && y0 + tid < P.ny) stamp[tid] = step + 1;
}

template <typename T, int MODE>
void launch_local(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + LOC_TY - 1) / LOC_TY;
    k_step_local<T, MODE><<<ntx * nty, dim3(TX, BY), 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp,
                                                              ntx, nty, phi, u, p);
}

template void launch_local<float, 0>(const KParams<float>&, char*, const Layout&, hipStream_t, float*, float*, float*);
template void launch_local<float, 1>(const KParams<float>&, char*, const Layout&, hipStream_t, float*, float*, float*);
template void launch_local<double, 0>(const KParams<double>&, char*, const Layout&, hipStream_t, double*, double*,
                                      double*);
template void launch_local<double, 1>(const KParams<double>&, char*, const Layout&, hipStream_t, double*, double*,
                                      double*);

}  // namespace lbm
