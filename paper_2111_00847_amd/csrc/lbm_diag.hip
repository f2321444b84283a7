// lbm_diag.hip -- diagnostics of the current level (Sec. 4.1): sum of phi,
// div u = tr S from the local strain rate (Eq. strainRate), the mass source
// S_m = d_t rho + div m^CC with div m^phiC from the isotropic stencil
// (Eq. central1), max |u| and a non-finite flag.
//
// Pass 1 (tile kernel): per-node quantities; m^phiC and the local part of S_m
// go to scratch planes; per-workgroup partial sums/maxima in FP64.
// Pass 2 (tile kernel): div m^phiC from the scratch planes, S_m^2 partials.
// Pass 3 (one workgroup): fixed-order reduction of the partials.  Every
// reduction has a fixed order, so results are bitwise reproducible.
#include "lbm_ch.hpp"
#include "lbm_kernels.hpp"
#include "lbm_tile.hpp"

namespace lbm {

constexpr int DTY = 8;   // tile rows of the diagnostics kernels

// Block-wide reduction of NV values (sum when is_max[j] == 0, else max) into
// thread 0; fixed tree order.
template <int NV>
__device__ void block_reduce(double* v, const bool* is_max, double (*red)[NV]) {
    const int tid = threadIdx.y * TX + threadIdx.x;
#pragma unroll
    for (int j = 0; j < NV; j++)
        for (int off = 32; off > 0; off >>= 1) {
            double o = __shfl_xor(v[j], off, 64);
            v[j] = is_max[j] ? fmax(v[j], o) : v[j] + o;
        }
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0)
        for (int j = 0; j < NV; j++) red[wave][j] = v[j];
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j < NV; j++) {
            double a = red[0][j];
            for (int w = 1; w < BY; w++) a = is_max[j] ? fmax(a, red[w][j]) : a + red[w][j];
            v[j] = a;
        }
    }
}

// Per-node part of pass 1: div u, the local part of S_m and m^phiC to scratch,
// the running sums/maxima in acc (sum phi, max|div|, sum div^2, max|u|, bad).
template <typename T>
__device__ __forceinline__ void diag_node(const KParams<T>& P, const Macro<T>& M, const T* f, const T* g,
                                          double phid, bool first, T php, long long k, T* scr, double* acc) {
    bool bad = !isfinite(phid);
    for (int i = 0; i < Q; i++) bad = bad || !isfinite(f[i]) || !isfinite(g[i]);
    // g^eq of the current level (Eq. MgMF1 inverted through M1)
    const T u = M.u, v = M.v, rho = M.rho;
    T tr = T(3) * rho * (u * u + v * v) + T(3) * (u * M.mx + v * M.my);
    T meq[9] = {P.rho0, T(-4) * P.rho0 + T(6) * M.p + tr, T(4) * P.rho0 - T(9) * M.p - tr,
                rho * u, -rho * u, rho * v, -rho * v,
                (u * M.mx - v * M.my) + rho * (u * u - v * v),
                T(0.5) * ((u * M.my + v * M.mx) + T(2) * rho * u * v)};
    T geq[9];
    from_moments(meq, geq);
    T s = T(0);
    for (int i = 1; i < Q; i++) s += T(cx(i) * cx(i) + cy(i) * cy(i)) * (g[i] - geq[i]);
    T ugr = u * M.drx + v * M.dry;
    T trM2F = T(2) * (u * M.Fx + v * M.Fy) + (M.d2 + M.d3) + (T(4) / T(3)) * ugr;
    // tr S = -s_2 / (2 rho cs^2) [sum |c|^2 (g - g^eq) + tr M_2F / 2]
    T div = -(T(1.5) * M.snu / rho) * (s + T(0.5) * trM2F);
    T rho_prev = P.drho * (php - P.phiB) + P.rhoB;
    T dtr = first ? T(0) : rho - rho_prev;
    scr[k] = M.mx;
    scr[P.plane + k] = M.my;
    scr[2 * P.plane + k] = dtr + rho * div + ugr;
    acc[0] += phid;
    acc[1] = fmax(acc[1], fabs((double)div));
    acc[2] += (double)div * (double)div;
    acc[3] = fmax(acc[3], sqrt((double)u * (double)u + (double)v * (double)v));
    if (bad) acc[4] = 1.0;
}

template <typename T>
__device__ __forceinline__ void diag_finish(double* acc, double (*red)[5], double* partials) {
    const bool is_max[5] = {false, true, false, true, true};
    block_reduce<5>(acc, is_max, red);
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0 && threadIdx.y == 0)
        for (int j = 0; j < 5; j++) partials[b * 8 + j] = acc[j];
}

template <typename T>
__global__ __launch_bounds__(TX* BY) void k_diag1(KParams<T> P, const char* state, size_t off0,
                                                  size_t off1, size_t off_stamp, T* scr, double* partials) {
    __shared__ T sphi[DTY + 2][TX + 3];
    __shared__ T sphp[DTY + 2][TX + 3];
    __shared__ double red[BY][5];
    const int64_t sv = *reinterpret_cast<const int64_t*>(state + off_stamp), step = stamp_level(sv);
    const bool first = step == 0;
    const int cur = stamp_copy(sv);
    const Copy<T> S = copy_at<T>(const_cast<char*>(state) + (cur ? off1 : off0), P.plane);
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * DTY;
    fill_window<T, DTY>(P, S, true, x0, y0, sphi, sphp);

    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < DTY / BY; r++) {
        const int lx = threadIdx.x, ly = threadIdx.y + r * BY;
        const int x = x0 + lx, y = y0 + ly;
        if (x >= P.nx || y >= P.ny) continue;
        const long long k = (long long)y * P.nx + x;
        T f[9], g[9];
        const double phid = node_phi(P, S, x, y, f);
        for (int i = 0; i < Q; i++) g[i] = pull(S.g, P, i, x, y);
        T gx, gy, lap, gxp = T(0), gyp = T(0), lp, php = sphp[ly + 1][lx + 1], up = T(0), vp = T(0);
        win_stencil<T, DTY>(sphi, lx + 1, ly + 1, gx, gy, lap);
        const T phi = sphi[ly + 1][lx + 1];
        if (!first) {
            up = S.h[P.plane + k];
            vp = S.h[2 * P.plane + k];
        }
        if (P.grad == 1 && !first) {
            // local gradient scheme: grad phi by Eq. local, m^phiC of the previous level stored
            local_grad(P, f, g, phi, lap, php * up, php * vp, gx, gy);
            const Macro<T> M = macro<T, false, true>(P, g, phi, gx, gy, lap, first, php, T(0), T(0), up, vp, T(0),
                                                     T(0), S.h[3 * P.plane + k], S.h[4 * P.plane + k]);
            diag_node(P, M, f, g, phid, first, php, k, scr, acc);
            continue;
        }
        if (!first) win_stencil<T, DTY>(sphp, lx + 1, ly + 1, gxp, gyp, lp);
        const Macro<T> M = macro(P, g, phi, gx, gy, lap, first, php, gxp, gyp, up, vp);
        diag_node(P, M, f, g, phid, first, php, k, scr, acc);
    }
    diag_finish<T>(acc, red, partials);
}

// Pass 1 of the Cahn-Hilliard variant (m^phiC from grad mu) and of the corrected
// Allen-Cahn model (ACC: F_a from div D): the same per-node quantities from the
// two-node-window tile body.
template <typename T, bool ACC>
__global__ __launch_bounds__(TX* BY) void k_diag1_ch(KParams<T> P, const char* state, size_t off0,
                                                     size_t off1, size_t off_stamp, T* scr, double* partials) {
    __shared__ ChWindow<T, DTY> W;
    __shared__ double red[BY][5];
    const int64_t sv = *reinterpret_cast<const int64_t*>(state + off_stamp), step = stamp_level(sv);
    const bool first = step == 0;
    const int cur = stamp_copy(sv);
    const Copy<T> S = copy_at<T>(const_cast<char*>(state) + (cur ? off1 : off0), P.plane);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    ch_tile<T, DTY, ACC>(P, S, step, blockIdx.x * TX, blockIdx.y * DTY, W,
                    [&](const Macro<T>& M, T* f, T* g, double phid, int, int, long long k) {
                        // the previous phi of the node (for d_t rho) is the history plane
                        const T php = first ? M.phi : S.h[k];
                        diag_node(P, M, f, g, phid, first, php, k, scr, acc);
                    });
    diag_finish<T>(acc, red, partials);
}

template <typename T>
__global__ __launch_bounds__(TX* BY) void k_diag2(KParams<T> P, const T* scr, double* partials) {
    __shared__ double red[BY][2];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * DTY;
    double acc[2] = {0.0, 0.0};   // sum S_m^2, count
    for (int r = 0; r < DTY / BY; r++) {
        const int x = x0 + threadIdx.x, y = y0 + threadIdx.y + r * BY;
        if (x >= P.nx || y >= P.ny) continue;
        bool ok = true;
        T dmx = T(0), dmy = T(0);
        for (int i = 1; i < Q; i++) {
            int tx = x + cx(i), ty = y + cy(i);
            if (tx < 0 || tx >= P.nx) {
                if (P.wall_x) ok = false;
                tx = tx < 0 ? tx + P.nx : tx - P.nx;
            }
            if (ty < 0 || ty >= P.ny) {
                if (P.wall_y) ok = false;
                ty = ty < 0 ? ty + P.ny : ty - P.ny;
            }
            if (!ok) break;
            const long long t = (long long)ty * P.nx + tx;
            const T w = i <= 4 ? T(1) / T(9) : T(1) / T(36);
            dmx += w * T(cx(i)) * scr[t];
            dmy += w * T(cy(i)) * scr[P.plane + t];
        }
        if (!ok) continue;
        const long long k = (long long)y * P.nx + x;
        double sm = (double)(scr[2 * P.plane + k] + T(3) * (dmx + dmy));
        acc[0] += sm * sm;
        acc[1] += 1.0;
    }
    const bool is_max[2] = {false, false};
    block_reduce<2>(acc, is_max, red);
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        partials[b * 8 + 5] = acc[0];
        partials[b * 8 + 6] = acc[1];
    }
}

// One workgroup of DIAG3_THREADS: thread t folds the partial records t,
// t + DIAG3_THREADS, ... in that order, then a tree over the threads in a
// fixed pairing (sums: deterministic for a given lattice; maxima: exact).
constexpr int DIAG3_THREADS = 1024;

__global__ __launch_bounds__(DIAG3_THREADS) void k_diag3(const double* partials, int nblocks, long long n,
                                                         double* out) {
    __shared__ double red[7][DIAG3_THREADS];
    const int t = threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};   // sum phi, max div, sum div^2, max |u|, nonfinite, sum S_m^2, count
    for (int b = t; b < nblocks; b += DIAG3_THREADS) {
        const double* r = partials + b * 8;
        v[0] += r[0];
        v[1] = fmax(v[1], r[1]);
        v[2] += r[2];
        v[3] = fmax(v[3], r[3]);
        v[4] = fmax(v[4], r[4]);
        v[5] += r[5];
        v[6] += r[6];
    }
#pragma unroll
    for (int q = 0; q < 7; q++) red[q][t] = v[q];
    __syncthreads();
    for (int w = DIAG3_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] = fmax(red[1][t], red[1][t + w]);
            red[2][t] += red[2][t + w];
            red[3][t] = fmax(red[3][t], red[3][t + w]);
            red[4][t] = fmax(red[4][t], red[4][t + w]);
            red[5][t] += red[5][t + w];
            red[6][t] += red[6][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
        out[2] = sqrt(red[2][0] / (double)n);
        out[3] = red[6][0] > 0 ? sqrt(red[5][0] / red[6][0]) : 0.0;
        out[4] = red[3][0];
        out[5] = red[4][0];
    }
}

template <typename T>
hipError_t launch_diagnostics(const KParams<T>& P, const char* state, const Layout& L, double* host_out,
                              hipStream_t s) {
    dim3 blk(TX, BY);
    dim3 grd((P.nx + TX - 1) / TX, (P.ny + DTY - 1) / DTY);
    T* scr = reinterpret_cast<T*>(const_cast<char*>(state) + L.off_diag);
    double* partials = reinterpret_cast<double*>(const_cast<char*>(state) + L.off_diag + 3 * L.plane * L.esz);
    double* out = partials + L.diag_partials;
    if (P.pf == 1)
        k_diag1_ch<T, false><<<grd, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, scr, partials);
    else if (P.model == 2)
        k_diag1_ch<T, true><<<grd, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, scr, partials);
    else k_diag1<T><<<grd, blk, 0, s>>>(P, state, L.off_buf[0], L.off_buf[1], L.off_stamp, scr, partials);
    k_diag2<T><<<grd, blk, 0, s>>>(P, scr, partials);
    k_diag3<<<1, DIAG3_THREADS, 0, s>>>(partials, (int)(grd.x * grd.y), L.n, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host_out, out, 6 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

template hipError_t launch_diagnostics<float>(const KParams<float>&, const char*, const Layout&, double*,
                                              hipStream_t);
template hipError_t launch_diagnostics<double>(const KParams<double>&, const char*, const Layout&, double*,
                                               hipStream_t);

}  // namespace lbm
