// lbm_common.hpp -- shared definitions of the gfx950 phase-field LBM kernels.
//
// Lattice units (dx = dt = c = 1, cs^2 = 1/3).  D2Q9 velocities in the column
// order of M1 (App. C): c0..c8 = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),
// (-1,-1),(1,-1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 9;
constexpr int HDR_BYTES = 256;     // state header
constexpr uint32_t STATE_MAGIC = 0x4C424D32u;  // "LBM2"

__host__ __device__ constexpr int cx(int i) {
    return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i) {
    return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp axis");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp diag");

// Device-side header at the start of every state buffer.
struct StateHeader {
    uint32_t magic;
    int32_t nx, ny, dtype;
};

// Level stamps.  The time level n of the state and the copy c that holds it
// are kept per (64-wide column band, row): stamp[xt * ny + y] = 2 n + c.  A
// step workgroup reads the stamp of its first row to learn n and its source
// copy, and at its end writes level n + 1 in the other copy into the stamps of
// the rows it owns (a two-level launch: n + 2 in the other copy, so the copy
// is not the parity of the level).  Every (band, row) belongs to exactly one
// workgroup of a launch whatever the tile height, so no two workgroups touch
// the same stamp and no cross-workgroup synchronisation is needed; all stamps
// are equal between launches.
constexpr int STAMP_BAND = 64;
__host__ __device__ constexpr int64_t stamp_of(int64_t level, int copy) { return 2 * level + copy; }
__host__ __device__ constexpr int64_t stamp_level(int64_t s) { return s >> 1; }
__host__ __device__ constexpr int stamp_copy(int64_t s) { return (int)(s & 1); }
// Parameters resolved on the host and passed by value to every kernel.
template <typename T>
struct KParams {
    int nx, ny;
    int wall_x, wall_y;
    int visc_law, model;
    int snu_local;        // s_g^7 = s_g^8 follow nu(phi)
    int pf;               // phase-field equation: 0 Allen-Cahn, 1 Cahn-Hilliard
    int grad;             // grad phi: 0 stencil (Eq. central1), 1 local scheme (Eq. local)
    int rates_std;        // every MRT rate is 1 but s_f^3, s_f^5, s_g^4, s_g^6, s_g^7, s_g^8
                          // (and LBM_STD_RATES allows the compiled-in collision for this dtype)
    long long plane;      // elements between two population planes
    T phiA, phiB, phim;   // phim = (phiA + phiB) / 2
    T beta4, kap;         // 4 beta, k (Sec. 2)
    T lamc;               // sqrt(2 beta / k) = 4 / (W dphi)
    T drho, rhoB;         // drho/dphi, rho_B
    T drhoM;              // drho/dphi * M_phi
    T Mphi, Aloc;         // M_phi; -M_phi - cs^2/2 (the local scheme's A)
    T inv_dphi;
    T muA, muB;           // linear-mu law
    T inv_nuA, inv_nuB;   // inverse-nu law
    T sf[9], sg[9];
    T Gx, Gy, gx, gy, rho_ref;
    T wa[4], wb[4], wc0[4];  // wetting quadratic per wall (x-, x+, y-, y+): a, b, a phiA phiB
    T wda[4];                // d a / d theta per wall
    T rho0, eps2;
    T Hp;                 // H of App. C: (s_g^2 - s_g^0)/(9 s_g^0 s_g^2)
    double rest_w;        // share of phi of the rest population at equilibrium (rest_encode)
};

// The rest population f_0 as a copy stores it.  After each collision it is
// set to phi minus the eight moving populations in double precision, so that
// the total of phi survives the rounding of the stored populations.  FP64
// copies hold it as it is.  FP32 copies hold its offset from w phi_h, phi_h
// being the FP32 history phi the same copy holds for the same node (the phi
// of the collision that produced f_0; zero after initialisation) and w the
// rest population's share of phi at equilibrium (4/9 for the Allen-Cahn
// equilibrium at eta = 1; 1 for the Cahn-Hilliard one, whose rest population
// is phi minus 5/9 of the small chemical potential), and restore it as
// offset + w phi_h in FP64.  The offset is small, so its FP32 rounding costs the
// total of phi about 1e-11 per node and step, where a plain FP32 f_0 of order
// one would round by 3e-8 -- and by the same bias at every step of a steady
// state.
template <typename T>
__host__ __device__ inline double rest_decode(T stored, T hphi, double w) {
    return (double)stored + w * (double)hphi;
}
template <>
__host__ __device__ inline double rest_decode<double>(double stored, double, double) {
    return stored;
}
template <typename T>
__host__ __device__ inline T rest_encode(double f0, T hphi, double w) {
    return (T)(f0 - w * (double)hphi);
}
template <>
__host__ __device__ inline double rest_encode<double>(double f0, double, double) {
    return f0;
}

// One ping-pong copy of the state, every plane of element type T:
// f_0 (stored as rest_encode gives it) | f_1..f_8 | g_0..g_8 | hist phi, u, v
// (previous level) [| m^phiC_x, m^phiC_y of the previous level, local gradient
// scheme].
template <typename T>
struct Copy {
    T* f0;
    T* f;   // f + i * plane is plane i, i = 1..8 (and f + 0 = f0)
    T* g;   // g + i * plane, i = 0..8
    T* h;   // h + j * plane, j = 0..2 (0..4 for the local gradient scheme)
};

template <typename T>
__host__ __device__ inline Copy<T> copy_at(char* base, long long plane) {
    Copy<T> c;
    c.f0 = reinterpret_cast<T*>(base);
    c.f = c.f0;
    c.g = c.f0 + 9 * plane;
    c.h = c.f0 + 18 * plane;
    return c;
}

// Byte layout of a state buffer.
struct Layout {
    long long n;          // nodes
    long long plane;      // padded plane length (elements)
    size_t esz;           // element size
    size_t buf_bytes;     // one ping-pong copy: f[9], g[9], hist[3 or 5] planes
    size_t off_buf[2];
    size_t off_stamp;     // int64 level stamps, ceil(nx / 64) * ny of them
    size_t nstamp;
    size_t off_diag;      // diagnostics scratch: 3 planes (m^phiC, local S_m), partials, result
    size_t diag_partials; // number of double slots for block partials
    size_t total;
};

// nh: history planes (3: phi, u, v; 5 with m^phiC for the local gradient scheme).
inline Layout make_layout(int nx, int ny, size_t esz, size_t diag_blocks, int nh = 3) {
    Layout L;
    L.n = (long long)nx * ny;
    L.plane = (L.n + 63) / 64 * 64;
    L.esz = esz;
    L.buf_bytes = (size_t)(18 + nh) * L.plane * esz;
    L.off_buf[0] = HDR_BYTES;
    L.off_buf[1] = L.off_buf[0] + L.buf_bytes;
    L.off_stamp = L.off_buf[1] + L.buf_bytes;
    L.nstamp = (size_t)((nx + STAMP_BAND - 1) / STAMP_BAND) * ny;
    L.off_diag = L.off_stamp + (L.nstamp * 8 + 255) / 256 * 256;
    L.diag_partials = diag_blocks * 8;
    size_t diag = (size_t)3 * L.plane * esz + L.diag_partials * sizeof(double) + 16 * sizeof(double);
    L.total = L.off_diag + (diag + 255) / 256 * 256;
    return L;
}

// The step kernels store the state with ordinary stores while both copies fit
// in this many bytes, so that the state (or most of it) stays in the 256 MB
// last-level cache from one step to the next, and non-temporally above.
// Measured on MI355X, FP32 (state of both copies): 256 x 1024 (46 MB) +2%,
// 1024 x 512 (92 MB) +7%, 1024 x 1024 (184 MB) +26%, 1024 x 1536 (277 MB) +11%
// with ordinary stores; 2048 x 1024 (369 MB) +3% and 4096^2 (2.9 GB) +5% with
// non-temporal ones (FP64 4096^2 +5%).
#ifndef LBM_NT_MIN_BYTES
#define LBM_NT_MIN_BYTES (320ull << 20)
#endif
inline bool cached_state(const Layout& L) { return 2 * L.buf_bytes <= (size_t)LBM_NT_MIN_BYTES; }
// Both copies within the 256 MB last-level cache itself (the plain step then
// loads g after its window barrier).
inline bool resident_state(const Layout& L) { return 2 * L.buf_bytes <= (size_t(256) << 20); }

}  // namespace lbm
