// lbm_step2.hip -- two time levels of the Allen-Cahn step (stencil gradients)
// per launch.
//
// On states that the last-level cache holds, a one-level launch is bound by
// its own latency (the load, window, collide, store chain of every tile, and
// the launch itself) more than by bytes; on larger states it is bound by HBM,
// which it crosses once per level.  A two-level launch pays the chain once and
// crosses HBM once for two levels: a tile of 64 x TY nodes advances from level
// n to n + 2 by
//   A. computing level n + 1 (the step of level n) on the tile and a two-node
//      ring around it: the populations of that region are pulled from the
//      state, phi of level n on a three-node ring is summed into an LDS
//      window (with the phi of level n-1 from the history), and the
//      post-collision f (and g on the one-node ring) are kept in LDS;
//   B. the step of level n + 1 on the tile alone, pulling from LDS, and storing
//      the result into the other copy.
// Every quantity of A is computed from the same inputs with the same device
// functions as the one-level step (lbm_fused.hpp), and B consumes exactly
// what a one-level step would load back from the copy written by A (the FP32
// rest population included: it is kept in the stored encoding), so two levels
// of this launch equal two one-level launches bit for bit.  The ring costs
// recomputation (the region of A is (64 + 4)(TY + 4) nodes) and L2 reads of
// the neighbouring tiles' rows, not HBM traffic beyond those rows: a launch
// reads the state once and writes it once for two levels.  Stores bypass the
// caches (non-temporal) on states larger than the last-level cache.
//
// A launch writes level n + 2 into the other copy (the level stamps carry the
// copy, lbm_common.hpp).
#include "lbm_kernels.hpp"
#include "lbm_step2.hpp"

namespace lbm {

// Two levels of one tile per workgroup, tiles dealt to the XCDs (xcd_tile).
template <typename T, int TY, int NBY, bool STD, bool NTS>
__global__ __launch_bounds__(TX* NBY) void k_step2(KParams<T> P, char* state, size_t off0, size_t off1,
                                                   size_t off_stamp, int ntx, int nty) {
    __shared__ Step2Lds<T, TY> L;
    int xt, yt;
    xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    step2_tile<T, TY, NBY, STD, NTS>(P, state, off0, off1, off_stamp, xt, yt, L);
}

// The same for the local gradient scheme (Eq. local; the general collision,
// as the one-level kernel runs it).
template <typename T, int TY, int NBY, bool NTS>
__global__ __launch_bounds__(TX* NBY) void k_step2_local(KParams<T> P, char* state, size_t off0, size_t off1,
                                                         size_t off_stamp, int ntx, int nty) {
    __shared__ Step2LdsLocal<T, TY> L;
    int xt, yt;
    xcd_tile(blockIdx.x, ntx, nty, xt, yt);
    step2_local_tile<T, TY, NBY, NTS>(P, state, off0, off1, off_stamp, xt, yt, L);
}

template <typename T, int TY, int NBY>
static void launch_step2_local(const KParams<T>& P, char* state, const Layout& L, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    if (cached_state(L))
        k_step2_local<T, TY, NBY, false><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                             L.off_stamp, ntx, nty);
    else
        k_step2_local<T, TY, NBY, true><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                            L.off_stamp, ntx, nty);
}

template <typename T, int TY, int NBY, bool STD>
static void launch_step2_std(const KParams<T>& P, char* state, const Layout& L, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
    // the one-level step's store policy: ordinary stores while both copies fit the cache
    if (cached_state(L))
        k_step2<T, TY, NBY, STD, false><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                            L.off_stamp, ntx, nty);
    else
        k_step2<T, TY, NBY, STD, true><<<ntx * nty, dim3(TX, NBY), 0, s>>>(P, state, L.off_buf[0], L.off_buf[1],
                                                                           L.off_stamp, ntx, nty);
}

template <typename T, int TY, int NBY>
static void launch_step2_ty(const KParams<T>& P, char* state, const Layout& L, hipStream_t s) {
    if (P.grad == 1) launch_step2_local<T, TY, NBY>(P, state, L, s);
    else if (P.rates_std) launch_step2_std<T, TY, NBY, true>(P, state, L, s);
    else launch_step2_std<T, TY, NBY, false>(P, state, L, s);
}

// Tile rows of the two-level launch.  8-row tiles (68 KB of LDS in FP32, 136 KB
// in FP64) run two workgroups of 512 threads per CU (FP32); 16-row FP32 tiles
// (117 KB) one of 1024 threads, with 1.33 region nodes per tile node against
// 1.59.  Measured on MI355X (FP32): 16 rows when they fill the 256 CUs in one
// round and 8 rows would need two workgroups per CU (256 x 1024: 7.77 against
// 8.12 us per level); 8 rows otherwise (1024 x 512: 15.6 against 16.2 us).
// LBM_STEP2_TY forces 4, 8 or 16 (FP32).
#ifndef LBM_STEP2_TY
#define LBM_STEP2_TY 0
#endif

template <typename T>
void launch_step2(const KParams<T>& P, char* state, const Layout& L, hipStream_t s) {
    const long long ntx = (P.nx + TX - 1) / TX;
    const long long t8 = ntx * ((P.ny + 7) / 8), t16 = ntx * ((P.ny + 15) / 16);
    const bool rows16 = LBM_STEP2_TY == 16 || (LBM_STEP2_TY == 0 && t16 <= 256 && t8 > 256);
    if constexpr (LBM_STEP2_TY == 4) launch_step2_ty<T, 4, 4>(P, state, L, s);
    else if constexpr (sizeof(T) == 4) {
        if (rows16) launch_step2_ty<T, 16, 16>(P, state, L, s);
        else launch_step2_ty<T, 8, 8>(P, state, L, s);
    } else {
        launch_step2_ty<T, 8, 8>(P, state, L, s);
    }
}

template void launch_step2<float>(const KParams<float>&, char*, const Layout&, hipStream_t);
template void launch_step2<double>(const KParams<double>&, char*, const Layout&, hipStream_t);

}  // namespace lbm
