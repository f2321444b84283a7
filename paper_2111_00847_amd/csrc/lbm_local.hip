// lbm_local.hip -- the Allen-Cahn step with grad phi from the local scheme of
// Eq. local (levels >= 1; level 0 and lap phi by the stencils of Eqs. central1
// and central2).  The history of a copy then holds phi, u, v and m^phiC of the
// previous level (5 planes), since m^phiC of that level came from its own
// local gradient.  One 64 x 8 tile per workgroup of 64 x 8 threads, the phi
// window with a one-node ring in LDS (for lap phi), tiles dealt to the XCDs as
// for the stencil step, the same store policy (non-temporal for states beyond
// the last-level cache).
#include "lbm_kernels.hpp"
#include "lbm_local_step.hpp"

namespace lbm {

// Thread rows: one node per thread (measured on MI355X, FP32 RTI, us per
// step against 64 x 4 threads of two nodes each: 256 x 256 7.65 against 10.0,
// 4096 x 4096 582 against 599, 1024 x 512 20.9 against 20.1 -- a lattice the
// two-level launch takes).  LBM_LOC_NBY=4 restores two nodes per thread.
constexpr int LOC_TY = 8;
#ifndef LBM_LOC_NBY
#define LBM_LOC_NBY 8
#endif
constexpr int LOC_NBY = LBM_LOC_NBY;

template <typename T, int MODE, bool NT = true, typename OFF = uint64_t>
__global__ __launch_bounds__(TX* LOC_NBY) void k_step_local(KParams<T> P, char* state, size_t off0, size_t off1,
                                                      size_t off_stamp, int ntx, int nty, T* out_phi, T* out_u,
                                                      T* out_p) {
    __shared__ T sphi[LOC_TY + 2][TX + 3];
    int xt, yt;
    if (LBM_XCD_REMAP) {
        xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    } else {
        xt = blockIdx.x % ntx;
        yt = blockIdx.x / ntx;
    }
    local_step_tile<T, LOC_TY, MODE, NT, LOC_NBY, OFF>(P, state, off0, off1, off_stamp, xt, yt, out_phi, out_u,
                                                       out_p, sphi);
}

// Steps address a copy below 4 GiB with 32-bit byte offsets from a uniform base
// (measured on MI355X, FP32 RTI, us per step against 64-bit offsets: 256 x 256
// 6.21 against 7.84, 1024 x 512 20.3 against 22.4, 4096 x 4096 582 either way);
// moments and larger copies with 64-bit ones.
template <typename T, int MODE>
void launch_local(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + LOC_TY - 1) / LOC_TY;
    const dim3 grd(ntx * nty), blk(TX, LOC_NBY);
    const bool small = L.buf_bytes < (size_t(1) << 32);
    if (MODE == 0 && cached_state(L))
        k_step_local<T, MODE, false, uint32_t><<<grd, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp,
                                                                  ntx, nty, phi, u, p);
    else if (MODE == 0 && small)
        k_step_local<T, MODE, true, uint32_t><<<grd, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp,
                                                                 ntx, nty, phi, u, p);
    else
        k_step_local<T, MODE><<<grd, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, ntx, nty, phi,
                                                  u, p);
}

template void launch_local<float, 0>(const KParams<float>&, char*, const Layout&, hipStream_t, float*, float*, float*);
template void launch_local<float, 1>(const KParams<float>&, char*, const Layout&, hipStream_t, float*, float*, float*);
template void launch_local<double, 0>(const KParams<double>&, char*, const Layout&, hipStream_t, double*, double*,
                                      double*);
template void launch_local<double, 1>(const KParams<double>&, char*, const Layout&, hipStream_t, double*, double*,
                                      double*);

}  // namespace lbm
