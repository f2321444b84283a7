// lbm_device.hpp -- per-node device arithmetic of the phase-field LBM step.
//
// Everything here acts on one lattice node; the kernels in lbm_step.hip own the
// memory traffic (pulls from the ping-pong buffers, LDS windows for the
// stencils) and call these helpers.
#pragma once

#include "lbm_common.hpp"

namespace lbm {

// Reciprocal and reciprocal square root of the per-node closure (1/rho, nu,
// s_nu, the normal).  The FP32 path uses the hardware approximations (1 ulp;
// +5% on a 256 x 1024 lattice, where the step is latency bound) instead of the
// correctly rounded division sequences; FP64 always rounds correctly.
// LBM_FAST_RCP=0 restores correct rounding for FP32 too.
#ifndef LBM_FAST_RCP
#define LBM_FAST_RCP 1
#endif
template <typename T>
__device__ __forceinline__ T rcp(T x) {
    return T(1) / x;
}
template <typename T>
__device__ __forceinline__ T rsqrt_(T x) {
    return T(1) / sqrt(x);
}
template <typename T>
__device__ __forceinline__ T div_(T a, T b) {
    return LBM_FAST_RCP && sizeof(T) == 4 ? a * rcp(b) : a / b;
}
#if LBM_FAST_RCP
template <>
__device__ __forceinline__ float rcp<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ float rsqrt_<float>(float x) {
    return __builtin_amdgcn_rsqf(x);
}
#endif

// Population i arriving at node (x, y) by pull streaming: it left x - c_i in
// the previous collision, or -- if x - c_i lies beyond a wall face -- it is the
// opposite population of (x, y) itself, reflected half-way (Sec. 4 preamble).
template <typename T>
__device__ __forceinline__ T pull(const T* __restrict__ src, const KParams<T>& P, int i, int x,
                                  int y) {
    int sx = x - cx(i), sy = y - cy(i);
    bool bb = false;
    if (sx < 0 || sx >= P.nx) {
        if (P.wall_x) bb = true;
        else sx = sx < 0 ? sx + P.nx : sx - P.nx;
    }
    if (sy < 0 || sy >= P.ny) {
        if (P.wall_y) bb = true;
        else sy = sy < 0 ? sy + P.ny : sy - P.ny;
    }
    if (bb) return src[opp(i) * P.plane + (long long)y * P.nx + x];
    return src[i * P.plane + (long long)sy * P.nx + sx];
}

// Wetting ghost value for wall k (0: x-, 1: x+, 2: y-, 3: y+) from the first
// and second fluid nodes of a wall-normal line.  Eq. (Dwetting):
// a phi_w^2 + b phi_w + c = 0, root -2c / (b + sqrt(b^2 - 4ac)) (the paper's
// root in a form finite at a = 0); the ghost node at distance -1/2 from the
// half-way wall lies on the quadratic through (0, phi_w), (1/2, phi1),
// (3/2, phi2).
template <typename T>
__device__ __forceinline__ T wet_ghost(const KParams<T>& P, int k, T phi1, T phi2) {
    const T third = T(1) / T(3);
    T a = P.wa[k], b = P.wb[k];
    T c = P.wc0[k] + phi2 * third - T(3) * phi1;
    T D = b * b - T(4) * a * c;
    D = D > T(0) ? D : T(0);
    T pw = T(-2) * c / (b + sqrt(D));
    return (T(8) * pw - T(6) * phi1 + phi2) * third;
}

// Isotropic gradient and Laplacian (App. C, Eqs. central1, central2) of a 3x3
// neighbourhood: n[j][i] = phi(x + i - 1, y + j - 1).
template <typename T>
__device__ __forceinline__ void stencil(T pSW, T pS, T pSE, T pW, T pC, T pE, T pNW, T pN, T pNE,
                                        T& gx, T& gy, T& lap) {
    const T third = T(1) / T(3), twelfth = T(1) / T(12);
    gx = third * (pE - pW) + twelfth * ((pNE + pSE) - (pNW + pSW));
    gy = third * (pN - pS) + twelfth * ((pNE + pNW) - (pSE + pSW));
    lap = T(2) * third * ((pE + pW) + (pN + pS)) + (T(1) / T(6)) * ((pNE + pNW) + (pSE + pSW)) -
          (T(10) / T(3)) * pC;
}

// m^phiC = -(drho/dphi) M (grad phi - lambda n), n = grad phi / sqrt(|grad phi|^2 + eps^2),
// lambda = sqrt(2 beta / k)(phiA - phi)(phi - phiB)  (Sec. 2).
template <typename T>
__device__ __forceinline__ void mass_flux(const KParams<T>& P, T phi, T gx, T gy, T& lnx, T& lny,
                                          T& mx, T& my) {
    T inv = rsqrt_(gx * gx + gy * gy + P.eps2);
    T lam = P.lamc * (P.phiA - phi) * (phi - P.phiB);
    lnx = lam * gx * inv;
    lny = lam * gy * inv;
    if (P.model != 0) {
        mx = T(0);
        my = T(0);
    } else {
        mx = -P.drhoM * (gx - lnx);
        my = -P.drhoM * (gy - lny);
    }
}

// grad phi of one node by the local scheme of Eq. local (Allen-Cahn, levels >= 1):
// C = sum_i c_i f_i - phi u + d_t(phi u)/2 = A grad phi + B n with A = -M - cs^2/2,
// B = M lambda.  u = u0 + mu_phi grad phi / (2 rho) (Eq. comU, u0 without F_s) and
// d_t(phi u) = phi u - (phi u)^{n-1}, so C0 = sum_i c_i f_i - phi u0/2 - (phi u)^{n-1}/2
// = A' grad phi + B n with A' = A + phi mu_phi/(4 rho): |grad phi| = (|C0| + B)/(-A')
// (clamped at 0) along -C0, the direction regularised as n is: C0 / sqrt(|C0|^2 +
// (A' eps_n)^2).  lap: Eq. central2 of phi; (phu_prev, phv_prev) = (phi u)^{n-1}.
template <typename T>
__device__ __forceinline__ void local_grad(const KParams<T>& P, const T* f, const T* g, T phi, T lap, T phu_prev,
                                           T phv_prev, T& gx, T& gy) {
    const T t = phi - P.phiB;
    const T rho = P.drho * t + P.rhoB;
    const T mu = P.beta4 * (phi - P.phiA) * t * (phi - P.phim) - P.kap * lap;
    const T lam = P.lamc * (P.phiA - phi) * t;
    const T irho = rcp(rho);
    const T jgx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const T jgy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const T u0 = (jgx + T(0.5) * (P.Gx + (rho - P.rho_ref) * P.gx)) * irho;
    const T v0 = (jgy + T(0.5) * (P.Gy + (rho - P.rho_ref) * P.gy)) * irho;
    const T jfx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const T jfy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const T cx = jfx - T(0.5) * phi * u0 - T(0.5) * phu_prev;
    const T cy = jfy - T(0.5) * phi * v0 - T(0.5) * phv_prev;
    const T ap = P.Aloc + T(0.25) * phi * mu * irho;
    const T cn2 = cx * cx + cy * cy;
    const T mag = div_(sqrt(cn2) + P.Mphi * lam, -ap);
    if (mag > T(0)) {
        const T s = mag * rsqrt_(cn2 + ap * ap * P.eps2);
        gx = -s * cx;
        gy = -s * cy;
    } else {
        gx = T(0);
        gy = T(0);
    }
}

// Macroscopic state of one node at the current level (Sec. 3).
template <typename T>
struct Macro {
    T phi, rho, u, v, p;
    T drx, dry;        // grad rho
    T lnx, lny;        // lambda n
    T mx, my;          // m^phiC
    T Fx, Fy;          // total force
    T snu;             // s_g^7 = s_g^8
    T d0, d1, d2, d3, d4;  // explicit-Euler d_t of phi u, phi v, u m_x, v m_y, u m_y + v m_x
    T mu;              // chemical potential mu_phi (Sec. 2)
};

// Chemical potential mu_phi = psi'(phi) - k lap phi (Sec. 2).
template <typename T>
__device__ __forceinline__ T chem_pot(const KParams<T>& P, T phi, T lap) {
    return P.beta4 * (phi - P.phiA) * (phi - P.phiB) * (phi - P.phim) - P.kap * lap;
}

// Cahn-Hilliard mass flux m^phiC = -(drho/dphi) M grad mu_phi (Sec. 2, D = grad mu).
template <typename T>
__device__ __forceinline__ void mass_flux_ch(const KParams<T>& P, T gmx, T gmy, T& mx, T& my) {
    mx = P.model != 0 ? T(0) : -P.drhoM * gmx;
    my = P.model != 0 ? T(0) : -P.drhoM * gmy;
}

// Closure, velocity (Eq. comU), history derivatives and pressure (Eq. computP,
// second way of Remark 1) of one node.  g: pulled populations; (gx, gy, lap):
// stencils of phi; first: level 0 (time derivatives zero); (php, gxp, gyp,
// up, vp): phi, grad phi and u of the previous level.  CH: the Cahn-Hilliard
// flux from grad mu (gmx, gmy) and grad mu of the previous level (gmxp, gmyp).
// Corrected model (model 2): lmu = div D (lap mu for CH), F_a = (drho/dphi) M lmu u.
// LOC (local gradient scheme): (gx, gy) come from local_grad and (gmxp, gmyp)
// carry the stored m^phiC of the previous level.  CORR: the kernel may run the
// corrected model (compiled out of the plain step, whose code then stays that
// of the present and original models).
template <typename T, bool CH = false, bool LOC = false, bool CORR = false>
__device__ __forceinline__ Macro<T> macro(const KParams<T>& P, const T* g, T phi, T gx, T gy, T lap,
                                          bool first, T php, T gxp, T gyp, T up, T vp, T gmx = T(0),
                                          T gmy = T(0), T gmxp = T(0), T gmyp = T(0), T lmu = T(0)) {
    Macro<T> m;
    m.phi = phi;
    T t = phi - P.phiB;
    m.rho = P.drho * t + P.rhoB;
    T mu_phi = P.beta4 * (phi - P.phiA) * t * (phi - P.phim) - P.kap * lap;
    m.mu = mu_phi;
    m.drx = P.drho * gx;
    m.dry = P.drho * gy;
    if (CH) {
        m.lnx = m.lny = T(0);
        mass_flux_ch(P, gmx, gmy, m.mx, m.my);
    } else {
        mass_flux(P, phi, gx, gy, m.lnx, m.lny, m.mx, m.my);
    }
    m.Fx = mu_phi * gx + P.Gx + (m.rho - P.rho_ref) * P.gx;
    m.Fy = mu_phi * gy + P.Gy + (m.rho - P.rho_ref) * P.gy;
    if (P.snu_local) {
        T nu;
        if (P.visc_law == 0) {
            T s = t * P.inv_dphi;
            nu = div_(s * (P.muA - P.muB) + P.muB, m.rho);
        } else {
            T s = t * P.inv_dphi;
            nu = rcp(s * (P.inv_nuA - P.inv_nuB) + P.inv_nuB);
        }
        m.snu = rcp(T(3) * nu + T(0.5));
    } else {
        m.snu = P.sg[7];
    }
    T jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    T jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    if (CORR && P.model == 2) {
        // corrected model: F = F_0 + a u with a = (drho/dphi) M div D (App. A, Eq. NS2-add);
        // Eq. comU solved for u exactly
        const T a = P.drhoM * lmu;
        const T irho = rcp(m.rho - T(0.5) * a);
        m.u = (jx + T(0.5) * m.Fx) * irho;
        m.v = (jy + T(0.5) * m.Fy) * irho;
        m.Fx += a * m.u;
        m.Fy += a * m.v;
    } else {
        const T irho = rcp(m.rho);
        m.u = (jx + T(0.5) * m.Fx) * irho;
        m.v = (jy + T(0.5) * m.Fy) * irho;
    }
    if (first) {
        m.d0 = m.d1 = m.d2 = m.d3 = m.d4 = T(0);
    } else {
        T lpx, lpy, mpx, mpy;
        if (CH) {
            mass_flux_ch(P, gmxp, gmyp, mpx, mpy);
        } else if (LOC) {
            mpx = gmxp;
            mpy = gmyp;
        } else {
            mass_flux(P, php, gxp, gyp, lpx, lpy, mpx, mpy);
        }
        m.d0 = phi * m.u - php * up;
        m.d1 = phi * m.v - php * vp;
        m.d2 = m.u * m.mx - up * mpx;
        m.d3 = m.v * m.my - vp * mpy;
        m.d4 = (m.u * m.my + m.v * m.mx) - (up * mpy + vp * mpx);
    }
    T sum = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
    T ugr = m.u * m.drx + m.v * m.dry;
    T trQ = m.rho * (m.u * m.u + m.v * m.v) + (m.u * m.mx + m.v * m.my);
    T uF = m.u * m.Fx + m.v * m.Fy;
    T dum = m.d2 + m.d3;
    // p = cs^2/(1 - w0) [sum_{i!=0} g_i + (1/2 + H) u.grad rho + s_0(phi,u) + K (2 F.u + d_t(u.m))]
    // with cs^2/(1 - w0) = 3/5, s_0 = -(2/3) tr(rho uu + m u), K = 1/3.
    m.p = T(0.6) * (sum + (T(0.5) + P.Hp) * ugr - (T(2) / T(3)) * trQ + (T(1) / T(3)) * (T(2) * uF + dum));
    return m;
}

// Sum of the eight moving populations, in the one association used everywhere.
template <typename T>
__device__ __forceinline__ T moving_sum(const T* f) {
    return ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
}

// The same sum accumulated in FP64 (exact for FP32 inputs of similar size).
template <typename T>
__device__ __forceinline__ double moving_sum_d(const T* f) {
    return (((double)f[1] + (double)f[2]) + ((double)f[3] + (double)f[4])) +
           (((double)f[5] + (double)f[6]) + ((double)f[7] + (double)f[8]));
}

// Zeroth moment (phi for f).  phi, m_0 and the rest population of
// from_moments all use moving_sum, so that in a uniform region
// (phi - S) + S == phi exactly and FP32 rounding cannot drift the mass.
template <typename T>
__device__ __forceinline__ T mass(const T* f) {
    return f[0] + moving_sum(f);
}

// Raw D2Q9 moments with M1 (App. C).
template <typename T>
__device__ __forceinline__ void to_moments(const T* f, T* m) {
    T a = (f[1] + f[2]) + (f[3] + f[4]);
    T d = (f[5] + f[6]) + (f[7] + f[8]);
    m[0] = mass(f);
    m[1] = T(-4) * f[0] - a + T(2) * d;
    m[2] = T(4) * f[0] - T(2) * a + d;
    T xd = (f[5] + f[8]) - (f[6] + f[7]);
    T yd = (f[5] + f[6]) - (f[7] + f[8]);
    m[3] = (f[1] - f[3]) + xd;
    m[4] = T(-2) * (f[1] - f[3]) + xd;
    m[5] = (f[2] - f[4]) + yd;
    m[6] = T(-2) * (f[2] - f[4]) + yd;
    m[7] = (f[1] + f[3]) - (f[2] + f[4]);
    m[8] = (f[5] + f[7]) - (f[6] + f[8]);
}

// Inverse transform: M1^-1 = M1^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
// The rest population is m0 minus the eight moving ones (identical in exact
// arithmetic): sum_i f_i then reproduces m0 to one rounding, with no bias from
// the rounded constant 1/9 -- in FP32, 9 * fl(1/9) = 1 + 7.5e-9, which would
// otherwise add that much mass to every node on every step.
template <typename T>
__device__ __forceinline__ void from_moments(const T* m, T* f) {
    T a0 = m[0] * (T(1) / T(9));
    T a1 = m[1] * (T(1) / T(36));
    T a2 = m[2] * (T(1) / T(36));
    T a3 = m[3] * (T(1) / T(6));
    T a4 = m[4] * (T(1) / T(12));
    T a5 = m[5] * (T(1) / T(6));
    T a6 = m[6] * (T(1) / T(12));
    T a7 = m[7] * T(0.25);
    T a8 = m[8] * T(0.25);
    T ax = a0 - a1 - T(2) * a2;           // axis directions
    T dg = a0 + T(2) * a1 + a2;           // diagonal directions
    f[1] = ax + (a3 - T(2) * a4) + a7;
    f[3] = ax - (a3 - T(2) * a4) + a7;
    f[2] = ax + (a5 - T(2) * a6) - a7;
    f[4] = ax - (a5 - T(2) * a6) - a7;
    T px = a3 + a4, py = a5 + a6;
    f[5] = dg + px + py + a8;
    f[6] = dg - px + py - a8;
    f[7] = dg - px - py + a8;
    f[8] = dg + px - py - a8;
    f[0] = m[0] - moving_sum(f);
}

// Both collisions are applied in increment form: the moment change
// dm = -S (m - m^eq) + (I - S/2) m_R is mapped back through M1^-1 and added to
// the incoming populations, so each stored population takes one rounding per
// step (in FP32 the forcing of a heavy phase is only tens of ulps of its
// populations).

// Phase-field collision (Eq. evoPF, moment form; Eq. MfMRAC1 with eta = 1).
// phid: phi of the node in FP64 (rest population + moving sum); returns the
// post-collision rest population phid - sum of the moving ones (m_0 is
// collision-invariant: m_0^eq = phi and m_R has no zeroth moment).
// CH: the Cahn-Hilliard moments of Eq. MfMRCH1 (eta mu_phi in rows 1 and 2;
// lambda n is zero in M).
// STD: the rates other than s_f^3, s_f^5 (s_g^4, s_g^6, s_g^7, s_g^8) are 1 (the
// paper's default, P.rates_std) and are compiled in as constants.
template <typename T, bool CH = false, bool STD = false>
__device__ __forceinline__ double collide_f(const KParams<T>& P, const Macro<T>& M, T* f, double phid) {
    T m[9];
    to_moments(f, m);
    const T phi = M.phi;
    T meq[9] = {phi, T(-2) * phi, phi, phi * M.u, -phi * M.u, phi * M.v, -phi * M.v, T(0), T(0)};
    T rx = M.lnx * (T(1) / T(3)) + M.d0;
    T ry = M.lny * (T(1) / T(3)) + M.d1;
    T mR[9] = {T(0), T(0), T(0), rx, -rx, ry, -ry, T(0), T(0)};
    T dm[9], d[9];
    dm[0] = T(0);
#pragma unroll
    for (int k = 1; k < 9; k++) {
        const T sk = (STD && k != 3 && k != 5) ? T(1) : P.sf[k];
        dm[k] = -sk * (m[k] - meq[k]) + (T(1) - T(0.5) * sk) * mR[k];
    }
    if (CH) {
        // Rows 1, 2 of Eq. MfMRCH1 (eta = 1): m^eq = -4 phi + 2 mu, 4 phi - 3 mu.  With
        // f_0 = phi - S (S = axis sum a + diagonal sum d) the phi terms cancel exactly:
        // m_1 - m_1^eq = 3a + 6d - 2 mu and m_2 - m_2^eq = -6a - 3d + 3 mu, both
        // formed from the small moving populations (in the CH bulk phi = +-1 and the
        // moving populations are O(mu, phi |u|): the plain form would lose them to
        // the rounding of f_0 and phi in FP32).
        const T a = (f[1] + f[2]) + (f[3] + f[4]);
        const T dd = (f[5] + f[6]) + (f[7] + f[8]);
        dm[1] = -(STD ? T(1) : P.sf[1]) * ((T(3) * a + T(6) * dd) - T(2) * M.mu);
        dm[2] = -(STD ? T(1) : P.sf[2]) * ((T(-6) * a - T(3) * dd) + T(3) * M.mu);
    }
    from_moments(dm, d);
#pragma unroll
    for (int i = 1; i < 9; i++) f[i] += d[i];
    return phid - moving_sum_d(f);
}

// Hydrodynamic collision (Remark 2, moment form; Eq. MgMF1).
template <typename T, bool STD = false>
__device__ __forceinline__ void collide_g(const KParams<T>& P, const Macro<T>& M, T* g) {
    T m[9];
    to_moments(g, m);
    const T u = M.u, v = M.v, rho = M.rho;
    T uu = u * u + v * v;
    T um = u * M.mx + v * M.my;
    T tr = T(3) * rho * uu + T(3) * um;
    T ugr = u * M.drx + v * M.dry;
    T uF = u * M.Fx + v * M.Fy;
    T dum = M.d2 + M.d3;
    T e1 = T(3) * dum + T(6) * uF;
    T meq[9] = {P.rho0,
                T(-4) * P.rho0 + T(6) * M.p + tr,
                T(4) * P.rho0 - T(9) * M.p - tr,
                rho * u,
                -rho * u,
                rho * v,
                -rho * v,
                (u * M.mx - v * M.my) + rho * (u * u - v * v),
                T(0.5) * ((u * M.my + v * M.mx) + T(2) * rho * u * v)};
    T mF[9] = {ugr,
               e1,
               -ugr - e1,
               M.Fx,
               -M.Fx,
               M.Fy,
               -M.Fy,
               (T(2) / T(3)) * (u * M.drx - v * M.dry) + T(2) * (u * M.Fx - v * M.Fy) + (M.d2 - M.d3),
               (T(1) / T(3)) * (u * M.dry + v * M.drx) + (u * M.Fy + v * M.Fx) + T(0.5) * M.d4};
    T s[9];
#pragma unroll
    for (int k = 0; k < 9; k++) s[k] = (STD && (k <= 3 || k == 5)) ? T(1) : P.sg[k];
    if (P.snu_local) {
        s[7] = M.snu;
        s[8] = M.snu;
    }
    T dm[9], d[9];
#pragma unroll
    for (int k = 0; k < 9; k++) dm[k] = -s[k] * (m[k] - meq[k]) + (T(1) - T(0.5) * s[k]) * mF[k];
    // Momentum rows: rho u = j + F/2 (Eq. comU) makes m_3 - m_3^eq = -F_x / 2 identically,
    // so dm_3 = F_x and dm_5 = F_y for any s_g^3, s_g^5.  Formed as a difference of j and
    // rho u, the FP32 value would lose the force of a heavy phase to cancellation.
    dm[3] = M.Fx;
    dm[4] = -s[4] * (m[4] - meq[4]) - (T(1) - T(0.5) * s[4]) * M.Fx;
    dm[5] = M.Fy;
    from_moments(dm, d);
#pragma unroll
    for (int i = 0; i < 9; i++) g[i] += d[i];
}

}  // namespace lbm
