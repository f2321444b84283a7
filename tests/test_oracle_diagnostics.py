"""Pins of the oracle's diagnostics (Sec. 4.1): div u = tr S of the local
strain rate (Eq. strainRate) and the mass source S_m = d_t rho + div m^CC.

tr S.  The paper obtains Eq. strainRate from its first-order expansion of the
non-equilibrium second moment (Sec. 3.1): sum_i c_i c_i g_i^ne =
-(dt/s_2) [d_t(rho uu + m u + p I) + div(cs^2 rho Delta.u) - (1 - s_2/2) M_2F],
valid when the collision relaxes every second moment c_i c_i at the one rate
s_2 (its condition on Lambda; with M1 that is s_g^0 = s_g^1 = s_g^7 = s_g^8),
and then drops d_t p (second way of Remark 1) and the c_s^2 rho (div u) I part
of div(cs^2 rho Delta.u), which vanish for an incompressible flow.  Kept,
those two terms make the trace of Eq. strainRate read 2 div u + d_t p /
(rho cs^2) for a single-phase flow without forces (to O(u^2)).  A compressive
velocity field, which has both, therefore pins the formula's coefficient,
sign, |c_i|^2 weighting and g^eq: against centred differences of u and of p
in time it must hold to a discretisation error that falls with resolution.

S_m.  With d rho / d phi = 0 (equal densities) every term but rho div u
vanishes, so S_m equals rho tr S node by node.  With a density contrast, an
interface carried through the lattice by a uniform velocity while its
Allen-Cahn flux relaxes a too-wide profile has S_m = 0 in the continuum
(d_t rho + u.grad rho = (drho/dphi) div(M D) cancels div m^phiC =
-(drho/dphi) div(M D), and div u = 0): S_m must fall at second order under
diffusive refinement.  A wrong sign on u.grad rho or on div m^phiC leaves a
residual of the size of those terms, which falls at first order only.
"""
import math

import numpy as np

import oracle
import workloads as W

CS2 = 1.0 / 3.0


def _compressive_wave(N, iso=True, nu=0.1, A=1e-3, B=6e-4):
    snu = 1.0 / (nu / CS2 + 0.5)
    sg = [snu, snu] + [0.0] * 7 if iso else [0.0] * 9
    case = W.Case(nx=N, ny=N, rhoA=1.0, rhoB=1.0, nuA=nu, nuB=nu, sigma=0.0, W=4.0, M=0.1, dtype="f64",
                  s_g=tuple(sg))
    X, Y = W.grid(case)
    k = 2 * math.pi / N
    u0 = np.stack([A * np.sin(k * X), B * np.sin(k * Y + 0.7)])
    return case, np.full((N, N), 0.5), u0


def _trace_residual(N, steps):
    case, phi0, u0 = _compressive_wave(N)
    o = oracle.OracleSim(case).init(phi0, u0, None).step(steps - 1)
    p_prev = o.moments()[2]
    o.step(1)
    _, u, _ = o.moments()
    div, sm = o.div_fields()
    o.step(1)
    p_next = o.moments()[2]
    dtp = 0.5 * (p_next - p_prev)
    cd = 0.5 * (np.roll(u[0], -1, 1) - np.roll(u[0], 1, 1)) + 0.5 * (np.roll(u[1], -1, 0) - np.roll(u[1], 1, 0))
    pred = 2.0 * cd + dtp / CS2      # rho = 1
    return np.abs(div - pred).max() / np.abs(div).max(), np.abs(cd).max(), div, sm


def test_strain_rate_trace_against_the_expansion():
    errs = []
    for N in (32, 64, 128):
        e, dmax, div, sm = _trace_residual(N, N // 8)
        errs.append(e)
        assert dmax > 1e-5            # the field is compressive: div u is not round-off
        # single phase: S_m = rho tr S node by node (rho = 1; periodic: every node counts)
        np.testing.assert_array_equal(sm, div)
    print("tr S residual vs 2 div u + d_t p/(rho cs^2):", errs)
    assert errs[-1] < 0.015, errs
    assert errs[0] > errs[1] > errs[2], errs


def test_mass_source_equals_rho_div_u_for_equal_densities():
    """drho/dphi = 0 (rho_A = rho_B = 2.5) with an interface, walls and gravity:
    S_m = rho tr S at every interior node, NaN next to walls."""
    case = W.Case(nx=40, ny=30, wall_y=True, rhoA=2.5, rhoB=2.5, nuA=0.05, nuB=0.2, sigma=0.01, W=4.0, M=0.05,
                  gravity=(0.0, -1e-5), rho_ref=1.0, dtype="f64")
    _, phi0 = W.static_droplet(n=40, R=8.0)
    phi0 = phi0[5:35, :]
    rng = np.random.default_rng(5)
    u0 = 1e-3 * rng.standard_normal((2, 30, 40))
    o = oracle.OracleSim(case).init(phi0, u0, None).step(7)
    div, sm = o.div_fields()
    inner = np.isfinite(sm)
    assert inner[1:-1].all() and not inner[0].any() and not inner[-1].any()
    np.testing.assert_array_equal(sm[inner], 2.5 * div[inner])
    assert np.abs(div).max() > 1e-7


def _moving_interface(scale, U=1e-3, widen=1.5):
    Wd = 4.0 * scale
    ny = int(64 * scale)
    case = W.Case(nx=2, ny=ny, rhoA=10.0, rhoB=1.0, nuA=0.1, nuB=0.1, sigma=0.0, W=Wd, M=0.05 * scale,
                  dtype="f64")
    X, Y = W.grid(case)
    d = np.minimum(Y - ny / 4, 3 * ny / 4 - Y)
    phi0 = W.tanh_profile(d, widen * Wd)
    u0 = np.zeros((2, ny, 2))
    u0[1] = U
    o = oracle.OracleSim(case).init(phi0, u0, None).step(int(40 * scale * scale))
    _, sm = o.div_fields()
    _, u, _ = o.moments()
    gx, gy = o.grad()
    ugr = np.abs(u[1] * 9.0 * gy).max()
    return math.sqrt(np.nanmean(sm ** 2)), ugr


def test_mass_source_of_a_moving_relaxing_interface_is_second_order():
    res = [_moving_interface(s) for s in (1, 2, 4)]
    sm = [r[0] for r in res]
    orders = [math.log2(sm[i] / sm[i + 1]) for i in range(2)]
    print("S_m^rms:", sm, "orders:", orders, "max|u.grad rho|:", [r[1] for r in res])
    assert min(orders) > 1.8, orders
    assert sm[-1] < 0.15 * res[-1][1]
