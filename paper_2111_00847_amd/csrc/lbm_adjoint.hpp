// lbm_adjoint.hpp -- per-node vector-Jacobian product of the fused step.
//
// The step maps, at every node, the pulled populations f, g, the stencils of
// phi (gradient, Laplacian, centre value) and of the previous phi, and the
// previous velocity to the post-collision populations f', g' and the stored
// history (phi, u, v).  Given the adjoints of those outputs, node_vjp returns
// the adjoints of the inputs by running the forward arithmetic of
// lbm_device.hpp (macro, collide_f, collide_g) backwards, term by term.  The
// momentum rows of the flow collision use the identities of the forward
// (dm_3 = F_x, dm_5 = F_y), which hold for all inputs and so have the same
// derivatives as the general formula.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

// Diagonal of M1 M1^T: M1^-1 = M1^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
template <typename T>
__device__ __forceinline__ T mdiag(int k) {
    return k == 0 ? T(1) / T(9)
                  : (k <= 2 ? T(1) / T(36) : (k == 3 || k == 5 ? T(1) / T(6) : (k == 4 || k == 6 ? T(1) / T(12) : T(0.25))));
}

// out = M1^T b (the transpose of to_moments).
template <typename T>
__device__ __forceinline__ void moments_T(const T* b, T* out) {
    const T ax = b[0] - b[1] - T(2) * b[2];
    const T dg = b[0] + T(2) * b[1] + b[2];
    const T qx = b[3] - T(2) * b[4], qy = b[5] - T(2) * b[6];
    const T px = b[3] + b[4], py = b[5] + b[6];
    out[0] = b[0] - T(4) * b[1] + T(4) * b[2];
    out[1] = ax + qx + b[7];
    out[3] = ax - qx + b[7];
    out[2] = ax + qy - b[7];
    out[4] = ax - qy - b[7];
    out[5] = dg + px + py + b[8];
    out[6] = dg - px + py - b[8];
    out[7] = dg - px - py + b[8];
    out[8] = dg + px - py - b[8];
}

// Adjoint of mass_flux: (lnx, lny, mx, my) as functions of (phi, gx, gy).
template <typename T>
__device__ __forceinline__ void mass_flux_vjp(const KParams<T>& P, T phi, T gx, T gy, T lnx_b, T lny_b, T mx_b,
                                              T my_b, T& phi_b, T& gx_b, T& gy_b) {
    const T inv = T(1) / sqrt(gx * gx + gy * gy + P.eps2);
    const T lam = P.lamc * (P.phiA - phi) * (phi - P.phiB);
    if (P.model != 1) {   // m = -(drho/dphi) M (grad phi - lambda n)
        gx_b -= P.drhoM * mx_b;
        gy_b -= P.drhoM * my_b;
        lnx_b += P.drhoM * mx_b;
        lny_b += P.drhoM * my_b;
    }
    const T s = lnx_b * gx + lny_b * gy;   // lambda n = lam grad phi inv
    const T lam_b = s * inv;
    const T inv_b = s * lam;
    gx_b += lnx_b * lam * inv;
    gy_b += lny_b * lam * inv;
    const T inv3 = inv * inv * inv;        // d inv / d g = -g inv^3
    gx_b -= inv_b * gx * inv3;
    gy_b -= inv_b * gy * inv3;
    phi_b += lam_b * P.lamc * ((P.phiA - phi) - (phi - P.phiB));
}

template <typename T>
struct NodeAdj {
    T f[9], g[9];                // pulled populations
    T phic, gx, gy, lap;         // phi of the node (centre) and its stencils
    T php, gxp, gyp, up, vp;     // previous phi (centre), its gradient, previous velocity
    T grav_x, grav_y;            // this node's share of dL/d gravity
};

// fo_b, go_b: adjoints of f', g'; (hphi_b, hu_b, hv_b): adjoints of the stored
// (phi, u, v).  M: the forward Macro of the node (same inputs).
template <typename T>
__device__ __forceinline__ void node_vjp(const KParams<T>& P, const Macro<T>& M, const T* f, const T* g, T gx,
                                         T gy, T lap, bool first, T php, T gxp, T gyp, T up, T vp, const T* fo_b,
                                         const T* go_b, T hphi_b, T hu_b, T hv_b, NodeAdj<T>& A) {
    const T phi = M.phi, u = M.u, v = M.v, rho = M.rho;
    T phi_b = hphi_b, u_b = hu_b, v_b = hv_b, rho_b = T(0), p_b = T(0);
    T mx_b = T(0), my_b = T(0), lnx_b = T(0), lny_b = T(0), Fx_b = T(0), Fy_b = T(0);
    T drx_b = T(0), dry_b = T(0), snu_b = T(0);
    T d_b[5] = {T(0), T(0), T(0), T(0), T(0)};
    T ugr_b = T(0), uF_b = T(0), dum_b = T(0), trQ_b = T(0);
    T gx_b = T(0), gy_b = T(0), lap_b = T(0);

    // ---- phase-field collision: f' = f + M1^-1 dm, dm_0 = 0
    {
        T b[9], mb[9], t[9];
        to_moments(fo_b, b);
        mb[0] = T(0);
#pragma unroll
        for (int k = 1; k < 9; k++) {
            const T dmb = b[k] * mdiag<T>(k);
            mb[k] = -P.sf[k] * dmb;           // d dm_k / d m_k
            b[k] = P.sf[k] * dmb;             // meq_b
            t[k] = (T(1) - T(0.5) * P.sf[k]) * dmb;   // mR_b
        }
        phi_b += T(-2) * b[1] + b[2] + u * (b[3] - b[4]) + v * (b[5] - b[6]);
        u_b += phi * (b[3] - b[4]);
        v_b += phi * (b[5] - b[6]);
        const T rx_b = t[3] - t[4], ry_b = t[5] - t[6];
        lnx_b += rx_b * (T(1) / T(3));
        lny_b += ry_b * (T(1) / T(3));
        d_b[0] += rx_b;
        d_b[1] += ry_b;
        T fb[9];
        moments_T(mb, fb);
#pragma unroll
        for (int i = 0; i < 9; i++) A.f[i] = fo_b[i] + fb[i];
    }

    // ---- flow collision: g' = g + M1^-1 dm
    const T uu = u * u + v * v;
    {
        T b[9], mb[9], eb[9], fb[9];
        to_moments(go_b, b);
        T s[9];
#pragma unroll
        for (int k = 0; k < 9; k++) s[k] = P.sg[k];
        if (P.snu_local) {
            s[7] = M.snu;
            s[8] = M.snu;
        }
        T dmb[9];
#pragma unroll
        for (int k = 0; k < 9; k++) dmb[k] = b[k] * mdiag<T>(k);
        Fx_b += dmb[3];   // dm_3 = F_x
        Fy_b += dmb[5];   // dm_5 = F_y
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const bool mom = (k == 3 || k == 5);
            mb[k] = mom ? T(0) : -s[k] * dmb[k];
            eb[k] = mom ? T(0) : s[k] * dmb[k];
            fb[k] = mom ? T(0) : (T(1) - T(0.5) * s[k]) * dmb[k];
        }
        if (P.snu_local) {
            T m[9];
            to_moments(g, m);
            const T meq7 = (u * M.mx - v * M.my) + rho * (u * u - v * v);
            const T meq8 = T(0.5) * ((u * M.my + v * M.mx) + T(2) * rho * u * v);
            const T mF7 = (T(2) / T(3)) * (u * M.drx - v * M.dry) + T(2) * (u * M.Fx - v * M.Fy) + (M.d2 - M.d3);
            const T mF8 = (T(1) / T(3)) * (u * M.dry + v * M.drx) + (u * M.Fy + v * M.Fx) + T(0.5) * M.d4;
            snu_b += dmb[7] * (-(m[7] - meq7) - T(0.5) * mF7) + dmb[8] * (-(m[8] - meq8) - T(0.5) * mF8);
        }
        // m^eq of the flow (rows 1, 2, 4, 6, 7, 8; row 0 is constant)
        p_b += T(6) * eb[1] - T(9) * eb[2];
        const T tr_b = eb[1] - eb[2];   // tr = 3 rho |u|^2 + 3 u.m
        rho_b += T(3) * uu * tr_b;
        u_b += tr_b * (T(6) * rho * u + T(3) * M.mx);
        v_b += tr_b * (T(6) * rho * v + T(3) * M.my);
        mx_b += T(3) * u * tr_b;
        my_b += T(3) * v * tr_b;
        rho_b -= u * eb[4] + v * eb[6];
        u_b -= rho * eb[4];
        v_b -= rho * eb[6];
        u_b += eb[7] * (M.mx + T(2) * rho * u);
        v_b -= eb[7] * (M.my + T(2) * rho * v);
        mx_b += u * eb[7];
        my_b -= v * eb[7];
        rho_b += (u * u - v * v) * eb[7];
        u_b += eb[8] * (T(0.5) * M.my + rho * v);
        v_b += eb[8] * (T(0.5) * M.mx + rho * u);
        my_b += T(0.5) * u * eb[8];
        mx_b += T(0.5) * v * eb[8];
        rho_b += u * v * eb[8];
        // source moments m_F (rows 0, 1, 2, 4, 6, 7, 8)
        ugr_b += fb[0] - fb[2];
        const T e1_b = fb[1] - fb[2];   // e1 = 3 d_t(u.m) + 6 u.F
        dum_b += T(3) * e1_b;
        uF_b += T(6) * e1_b;
        Fx_b -= fb[4];
        Fy_b -= fb[6];
        u_b += fb[7] * ((T(2) / T(3)) * M.drx + T(2) * M.Fx);
        v_b -= fb[7] * ((T(2) / T(3)) * M.dry + T(2) * M.Fy);
        drx_b += (T(2) / T(3)) * u * fb[7];
        dry_b -= (T(2) / T(3)) * v * fb[7];
        Fx_b += T(2) * u * fb[7];
        Fy_b -= T(2) * v * fb[7];
        d_b[2] += fb[7];
        d_b[3] -= fb[7];
        u_b += fb[8] * (M.dry * (T(1) / T(3)) + M.Fy);
        v_b += fb[8] * (M.drx * (T(1) / T(3)) + M.Fx);
        dry_b += u * fb[8] * (T(1) / T(3));
        drx_b += v * fb[8] * (T(1) / T(3));
        Fy_b += u * fb[8];
        Fx_b += v * fb[8];
        d_b[4] += T(0.5) * fb[8];
        T gb[9];
        moments_T(mb, gb);
#pragma unroll
        for (int i = 0; i < 9; i++) A.g[i] = go_b[i] + gb[i];
    }

    // ---- pressure (Eq. computP): p = 3/5 [sum_{i>0} g_i + (1/2 + H) u.grad rho - 2/3 trQ + 1/3 (2 u.F + d_t(u.m))]
#pragma unroll
    for (int i = 1; i < 9; i++) A.g[i] += T(0.6) * p_b;
    ugr_b += T(0.6) * (T(0.5) + P.Hp) * p_b;
    trQ_b -= T(0.4) * p_b;
    uF_b += T(0.4) * p_b;
    dum_b += T(0.2) * p_b;
    rho_b += uu * trQ_b;   // trQ = rho |u|^2 + u.m
    u_b += trQ_b * (T(2) * rho * u + M.mx);
    v_b += trQ_b * (T(2) * rho * v + M.my);
    mx_b += u * trQ_b;
    my_b += v * trQ_b;
    u_b += ugr_b * M.drx;
    v_b += ugr_b * M.dry;
    drx_b += u * ugr_b;
    dry_b += v * ugr_b;
    u_b += uF_b * M.Fx;
    v_b += uF_b * M.Fy;
    Fx_b += u * uF_b;
    Fy_b += v * uF_b;
    d_b[2] += dum_b;
    d_b[3] += dum_b;

    // ---- explicit-Euler derivatives of the history products
    T php_b = T(0), gxp_b = T(0), gyp_b = T(0), up_b = T(0), vp_b = T(0);
    if (!first) {
        T lpx, lpy, mpx, mpy;
        mass_flux(P, php, gxp, gyp, lpx, lpy, mpx, mpy);
        T mpx_b = T(0), mpy_b = T(0);
        phi_b += d_b[0] * u + d_b[1] * v;
        u_b += d_b[0] * phi + d_b[2] * M.mx + d_b[4] * M.my;
        v_b += d_b[1] * phi + d_b[3] * M.my + d_b[4] * M.mx;
        mx_b += d_b[2] * u + d_b[4] * v;
        my_b += d_b[3] * v + d_b[4] * u;
        php_b -= d_b[0] * up + d_b[1] * vp;
        up_b -= d_b[0] * php + d_b[2] * mpx + d_b[4] * mpy;
        vp_b -= d_b[1] * php + d_b[3] * mpy + d_b[4] * mpx;
        mpx_b -= d_b[2] * up + d_b[4] * vp;
        mpy_b -= d_b[3] * vp + d_b[4] * up;
        mass_flux_vjp(P, php, gxp, gyp, T(0), T(0), mpx_b, mpy_b, php_b, gxp_b, gyp_b);
    }

    // ---- velocity (Eq. comU): u = (j + F/2) / rho
    {
        const T irho = T(1) / rho;
        const T jx_b = u_b * irho, jy_b = v_b * irho;
        Fx_b += T(0.5) * jx_b;
        Fy_b += T(0.5) * jy_b;
        rho_b -= (u_b * u + v_b * v) * irho;
        A.g[1] += jx_b;
        A.g[3] -= jx_b;
        A.g[5] += jx_b + jy_b;
        A.g[6] += jy_b - jx_b;
        A.g[7] -= jx_b + jy_b;
        A.g[8] += jx_b - jy_b;
        A.g[2] += jy_b;
        A.g[4] -= jy_b;
    }

    // ---- closure (Sec. 2)
    const T t = phi - P.phiB;
    T t_b = T(0);
    if (P.snu_local) {   // s_nu = 1 / (3 nu + 1/2)
        const T nu_b = T(-3) * M.snu * M.snu * snu_b;
        const T sl = t * P.inv_dphi;
        if (P.visc_law == 0) {
            const T nu = (sl * (P.muA - P.muB) + P.muB) / rho;
            rho_b -= nu_b * nu / rho;
            t_b += nu_b * (P.muA - P.muB) * P.inv_dphi / rho;
        } else {
            const T nu = T(1) / (sl * (P.inv_nuA - P.inv_nuB) + P.inv_nuB);
            t_b -= nu_b * nu * nu * (P.inv_nuA - P.inv_nuB) * P.inv_dphi;
        }
    }
    const T mu = P.beta4 * (phi - P.phiA) * t * (phi - P.phim) - P.kap * lap;
    const T mu_b = Fx_b * gx + Fy_b * gy;   // F = mu grad phi + G + (rho - rho_ref) g
    gx_b += Fx_b * mu;
    gy_b += Fy_b * mu;
    rho_b += Fx_b * P.gx + Fy_b * P.gy;
    A.grav_x = Fx_b * (rho - P.rho_ref);
    A.grav_y = Fy_b * (rho - P.rho_ref);
    mass_flux_vjp(P, phi, gx, gy, lnx_b, lny_b, mx_b, my_b, phi_b, gx_b, gy_b);
    gx_b += P.drho * drx_b;
    gy_b += P.drho * dry_b;
    lap_b -= P.kap * mu_b;
    {
        const T a = phi - P.phiA, c = phi - P.phim;
        phi_b += mu_b * P.beta4 * (t * c + a * c + a * t);
    }
    t_b += P.drho * rho_b;
    phi_b += t_b;

    A.phic = phi_b;
    A.gx = gx_b;
    A.gy = gy_b;
    A.lap = lap_b;
    A.php = php_b;
    A.gxp = gxp_b;
    A.gyp = gyp_b;
    A.up = up_b;
    A.vp = vp_b;
}

// Derivatives of the wetting ghost (lbm_device.hpp, wet_ghost) with respect to
// phi1, phi2 and theta of wall k.
template <typename T>
__device__ __forceinline__ void wet_ghost_grad(const KParams<T>& P, int k, T phi1, T phi2, T& d1, T& d2, T& dth) {
    const T third = T(1) / T(3);
    const T a = P.wa[k], b = P.wb[k];
    const T c = P.wc0[k] + phi2 * third - T(3) * phi1;
    const T D = b * b - T(4) * a * c;
    const bool pos = D > T(0);
    const T sq = pos ? sqrt(D) : T(0);
    const T den = b + sq;
    // pw = -2 c / den, den = b + sqrt(D), D = b^2 - 4 a c
    const T isq = pos ? T(1) / sq : T(0);
    const T dpw_dc = T(-2) / den + T(2) * c / (den * den) * (T(-2) * a * isq);
    d1 = (T(8) * dpw_dc * T(-3) - T(6)) * third;
    d2 = (T(8) * dpw_dc * third + T(1)) * third;
    // a = 4 cos(theta) / (W dphi); b = 8/3 - a (phiA + phiB); c0 = a phiA phiB
    const T dc_da = P.phiA * P.phiB;
    const T db_da = -(P.phiA + P.phiB);
    const T dD_da = T(2) * b * db_da - T(4) * c - T(4) * a * dc_da;
    const T dden_da = db_da + T(0.5) * isq * dD_da;
    const T dpw_da = T(-2) * dc_da / den + T(2) * c / (den * den) * dden_da;
    dth = T(8) * third * dpw_da * P.wda[k];
}

}  // namespace lbm
