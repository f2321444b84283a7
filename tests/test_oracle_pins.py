"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test states what pins which part of the oracle.  Cheap tests only; the
long physics runs are in test_oracle_physics.py.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

CX, CY, WT, M, MINV = oracle.lattice()
CS2 = 1.0 / 3.0


def _rand_macros(rng):
    return dict(rho=rng.uniform(1, 10), pr=rng.normal(0, 1e-2), u=rng.normal(0, 0.05),
                v=rng.normal(0, 0.05), mx=rng.normal(0, 0.01), my=rng.normal(0, 0.01),
                Fx=rng.normal(0, 1e-3), Fy=rng.normal(0, 1e-3), drx=rng.normal(0, 0.5),
                dry=rng.normal(0, 0.5), d_umx=rng.normal(0, 1e-4), d_vmy=rng.normal(0, 1e-4),
                d_cross=rng.normal(0, 1e-4))


# ------------------------------------------------------------------ lattice
def test_weights_give_cs2_one_third_and_fourth_order_isotropy():
    """D2Q9 weights (not printed; App. C fixes cs^2 = c^2/3): sum w = 1, sum w c = 0,
    sum w c_a c_b = delta/3, sum w c_a c_b c_c c_d = (dd + dd + dd)/9."""
    c = np.stack([CX, CY], 1).astype(float)
    assert abs(WT.sum() - 1) < 1e-15
    assert np.abs(WT @ c).max() < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", WT, c, c), np.eye(2) / 3, atol=1e-15)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", WT, c, c, c, c)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(T4, iso, atol=1e-15)


def test_M1_orthogonal_and_inverse():
    """App. C calls M1 orthogonal: M M^T is diagonal with the row norms
    9, 36, 36, 6, 12, 6, 12, 4, 4; the oracle's numeric inverse is exact."""
    G = M @ M.T
    np.testing.assert_allclose(G, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]), atol=1e-13)
    np.testing.assert_allclose(M @ MINV, np.eye(9), atol=1e-14)
    np.testing.assert_allclose(MINV, M.T / np.diag(G), atol=1e-15)


def test_velocity_order_matches_M1_rows():
    """Rows 3, 5, 7, 8 of M1 are c_x, c_y, c_x^2 - c_y^2, c_x c_y (App. C)."""
    np.testing.assert_array_equal(M[3], CX)
    np.testing.assert_array_equal(M[5], CY)
    np.testing.assert_array_equal(M[7], CX ** 2 - CY ** 2)
    np.testing.assert_array_equal(M[8], CX * CY)


# ------------------------------------------------------------------ equilibria
def test_phase_field_moments_equal_known_AC_equilibrium():
    """App. C, Eq. (MfMRAC1) (eta = 1) inverted through M1 gives the standard
    conservative-AC equilibrium f^eq_i = w_i phi (1 + c_i.u / cs^2) and source
    R_i = w_i c_i.(d_t(phi u) + cs^2 lambda n) / cs^2."""
    case = W.Case(nx=4, ny=4)
    rng = np.random.default_rng(0)
    for _ in range(20):
        phi, u, v = rng.uniform(0, 1), rng.normal(0, .1), rng.normal(0, .1)
        lnx, lny, dpu, dpv = rng.normal(0, .1, 4)
        meq, mR = oracle.moments_f(case, phi, u, v, lnx, lny, dpu, dpv)
        feq = MINV @ meq
        R = MINV @ mR
        np.testing.assert_allclose(feq, WT * phi * (1 + (CX * u + CY * v) / CS2), atol=1e-15)
        np.testing.assert_allclose(R, WT * (CX * (dpu + CS2 * lnx) + CY * (dpv + CS2 * lny)) / CS2,
                                   atol=1e-15)


def test_hydro_moment_lists_equal_direct_forms():
    """App. C, Eq. (MgMF1) equals M1 applied to the Sec. 3 direct forms: g^eq of
    Eq. (geq) and F_i with M_2F of Eq. (M2F) in the second way of Remark 1.  Two
    independent statements of the paper; a transcription slip in either fails."""
    rng = np.random.default_rng(1)
    for rho0 in (0.0, 1.3):
        case = W.Case(nx=4, ny=4, rho0=rho0)
        for _ in range(20):
            a = _rand_macros(rng)
            meq, mF = oracle.moments_g(case, **a)
            geq, Fi = oracle.direct_g(case, **a)
            np.testing.assert_allclose(M @ geq, meq, atol=1e-14)
            np.testing.assert_allclose(M @ Fi, mF, atol=1e-14)


def test_hydro_moment_conditions():
    """Eq. (conditions): sum g^eq = rho0, sum c g^eq = rho u,
    sum c c g^eq = rho uu + (m u)_sym + p I, sum c c c g^eq = cs^2 rho Delta.u;
    sum F = u.grad rho, sum c F = F, sum c c F = M_2F (second way)."""
    rng = np.random.default_rng(2)
    case = W.Case(nx=4, ny=4, rho0=0.7)
    c = np.stack([CX, CY], 1).astype(float)
    for _ in range(20):
        a = _rand_macros(rng)
        geq, Fi = oracle.direct_g(case, **a)
        meq, mF = oracle.moments_g(case, **a)
        g = MINV @ meq
        F = MINV @ mF
        uv = np.array([a["u"], a["v"]])
        mm = np.array([a["mx"], a["my"]])
        FF = np.array([a["Fx"], a["Fy"]])
        gr = np.array([a["drx"], a["dry"]])
        assert abs(g.sum() - 0.7) < 1e-14
        np.testing.assert_allclose(c.T @ g, a["rho"] * uv, atol=1e-15)
        P2 = np.einsum("i,ia,ib->ab", g, c, c)
        exp = (a["rho"] * np.outer(uv, uv) + 0.5 * (np.outer(mm, uv) + np.outer(uv, mm))
               + a["pr"] * np.eye(2))
        np.testing.assert_allclose(P2, exp, atol=1e-15)
        P3 = np.einsum("i,ia,ib,ic->abc", g, c, c, c)
        d = np.eye(2)
        ru = a["rho"] * uv
        exp3 = CS2 * (np.einsum("ab,c->abc", d, ru) + np.einsum("bc,a->abc", d, ru)
                      + np.einsum("ac,b->abc", d, ru))
        np.testing.assert_allclose(P3, exp3, atol=1e-15)
        assert abs(F.sum() - uv @ gr) < 1e-15
        np.testing.assert_allclose(c.T @ F, FF, atol=1e-16)
        dmu = np.array([[a["d_umx"], 0.5 * a["d_cross"]], [0.5 * a["d_cross"], a["d_vmy"]]])
        M2F = (np.outer(uv, FF) + np.outer(FF, uv) + dmu
               + CS2 * (np.outer(uv, gr) + np.outer(gr, uv)) + CS2 * (uv @ gr) * np.eye(2))
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", F, c, c), M2F, atol=1e-15)


# ------------------------------------------------------------------ stencils
def test_stencil_fourier_symbols_periodic():
    """Eqs. (central1), (central2) on exp(i k x): gradient symbol i sin k and
    Laplacian symbol 2 (cos k - 1) (second-order isotropic central schemes)."""
    n = 32
    case = W.Case(nx=n, ny=8)
    s = oracle.OracleSim(case)
    X, Y = W.grid(case)
    for m in (1, 3, 5):
        k = 2 * np.pi * m / n
        phi = np.sin(k * X) + 0.5 * np.cos(k * Y * n / 8)
        gx, gy, lap = s.stencils(phi)
        ky = 2 * np.pi * m / 8
        np.testing.assert_allclose(gx, np.sin(k) * np.cos(k * X), atol=1e-14)
        np.testing.assert_allclose(gy, -0.5 * np.sin(ky) * np.sin(ky * Y), atol=1e-14)
        exp_lap = 2 * (np.cos(k) - 1) * np.sin(k * X) + 2 * (np.cos(ky) - 1) * 0.5 * np.cos(ky * Y)
        np.testing.assert_allclose(lap, exp_lap, atol=1e-13)


def test_stencils_exact_on_quadratics_inside_walls():
    """Away from the walls the stencils are exact for quadratics; next to a neutral
    wall the ghost mirrors the first node (zero normal derivative at the face)."""
    case = W.Case(nx=12, ny=10, wall_x=True, wall_y=True)
    s = oracle.OracleSim(case)
    X, Y = W.grid(case)
    a, b, c, d, e = 0.3, -0.2, 0.15, 0.7, -0.4
    phi = a * X ** 2 + b * X * Y + c * Y ** 2 + d * X + e * Y
    gx, gy, lap = s.stencils(phi)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(gx[inner], (2 * a * X + b * Y + d)[inner], atol=1e-12)
    np.testing.assert_allclose(gy[inner], (b * X + 2 * c * Y + e)[inner], atol=1e-12)
    np.testing.assert_allclose(lap[inner], 2 * a + 2 * c, atol=1e-12)
    # neutral wall: a field symmetric about the bottom face has zero y-derivative at row 0
    phi2 = np.cos(np.pi * Y / 10) + 0 * X
    gx2, gy2, _ = s.stencils(phi2)
    exp_row0 = (np.cos(np.pi * 1.5 / 10) - np.cos(np.pi * 0.5 / 10)) / 2  # central difference
    np.testing.assert_allclose(gy2[0], exp_row0, atol=1e-14)


# ------------------------------------------------------------------ wetting
@pytest.mark.parametrize("theta_deg", [30, 45, 60, 75, 90, 105, 120, 135, 150])
def test_wetting_root_solves_the_continuous_condition(theta_deg):
    """Eq. (Dwetting) against Eq. (FEwetting): the returned phi_w is the root the
    paper selects, lies in [0, 1], and the quadratic through (0, phi_w), (1/2, phi1),
    (3/2, phi2) has wall derivative -(4/W)(phiA - phi_w)(phi_w - phiB) cos(theta);
    the ghost at -1/2 lies on the same quadratic."""
    case = W.Case(nx=4, ny=4, W=5.0)
    th = math.radians(theta_deg)
    rng = np.random.default_rng(theta_deg)
    for _ in range(50):
        phi1, phi2 = rng.uniform(0, 1, 2)
        pw, pg = oracle.wetting(case, th, phi1, phi2)
        if phi2 / 3 - 3 * phi1 < 0:
            assert pw >= -1e-12
        Acoef, Bcoef = np.polyfit([0.0, 0.5, 1.5], [pw, phi1, phi2], 2)[:2]
        deriv = Bcoef
        rhs = -(4.0 / case.W) * (1 - pw) * pw * math.cos(th)
        assert abs(deriv - rhs) < 1e-12
        quad = np.polyval(np.polyfit([0.0, 0.5, 1.5], [pw, phi1, phi2], 2), -0.5)
        assert abs(quad - pg) < 1e-12
        a = 4 * math.cos(th) / case.W
        if abs(a) > 1e-12:
            b = 8 / 3 - a
            c = phi2 / 3 - 3 * phi1
            assert abs(pw - (-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)) < 1e-10


def test_wetting_neutral_limit():
    """At 90 degrees a = 0: phi_w = (9 phi1 - phi2)/8 and the ghost equals phi1;
    the root is continuous as theta -> 90 degrees (the printed root form is not,
    in floating point, because cos(pi/2) is not exactly zero)."""
    case = W.Case(nx=4, ny=4)
    for phi1, phi2 in [(0.3, 0.1), (0.9, 0.95), (0.5, 0.5)]:
        pw, pg = oracle.wetting(case, math.pi / 2, phi1, phi2)
        assert abs(pw - (9 * phi1 - phi2) / 8) < 1e-15
        assert abs(pg - phi1) < 1e-15
        pw2, _ = oracle.wetting(case, math.pi / 2 + 1e-9, phi1, phi2)
        assert abs(pw2 - pw) < 1e-9


# ------------------------------------------------------------------ macroscopic recovery
def test_velocity_and_pressure_recovered_from_equilibrium_state():
    """Eqs. (comU), (computP): a state initialised at g = g^eq(p0, u0) with no force
    returns u0 and p0.  Uniform phi (grad rho = 0), random u0, p0."""
    case = W.Case(nx=8, ny=6, rhoA=3.0, rhoB=1.0, sigma=0.0)
    rng = np.random.default_rng(3)
    phi0 = np.full((6, 8), 0.37)
    u0 = 0.02 * rng.standard_normal((2, 6, 8))
    p0 = 1e-3 * rng.standard_normal((6, 8))
    s = oracle.OracleSim(case).init(phi0, u0, p0)
    phi, u, p = s.moments()
    np.testing.assert_allclose(phi, phi0, atol=1e-15)
    np.testing.assert_allclose(u, u0, atol=1e-16)
    np.testing.assert_allclose(p, p0, atol=1e-16)


def test_pressure_recovered_with_density_gradient_at_rest():
    """Same with a non-uniform phi (density gradient and m^phiC != 0) at u0 = 0."""
    case = W.Case(nx=16, ny=16, rhoA=10.0, rhoB=1.0, sigma=0.0, M=0.05)
    X, Y = W.grid(case)
    phi0 = W.tanh_profile(5 - np.hypot(X - 8, Y - 8), 4.0)
    p0 = 1e-3 * np.cos(2 * np.pi * X / 16)
    s = oracle.OracleSim(case).init(phi0, None, p0)
    phi, u, p = s.moments()
    np.testing.assert_allclose(u, 0, atol=1e-17)
    np.testing.assert_allclose(p, p0, atol=1e-16)


def test_uniform_body_force_closed_form():
    """Single phase, periodic, uniform force G: with the half-force correction of
    Eq. (comU) and the (I - S/2) m_F term, the momentum grows by exactly G per step,
    so u^n = (n + 1/2) G / rho, for any s_g^3."""
    for s3 in (0.0, 1.4):
        sg = [0.0] * 9
        sg[3] = sg[5] = s3
        case = W.Case(nx=5, ny=3, rhoA=2.0, rhoB=2.0, body_force=(3e-6, -1e-6), s_g=tuple(sg))
        s = oracle.OracleSim(case).init(np.full((3, 5), 0.4))
        for n in range(0, 40):
            _, u, _ = s.moments()
            np.testing.assert_allclose(u[0], (n + 0.5) * 3e-6 / 2.0, rtol=1e-12)
            np.testing.assert_allclose(u[1], -(n + 0.5) * 1e-6 / 2.0, rtol=1e-12)
            s.step(1)


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("geom", ["periodic", "walls", "wetting"])
def test_total_phi_conserved(geom):
    """The collision keeps the zeroth f moment (m_f^eq[0] = phi, m_R[0] = 0) and
    streaming with half-way bounce-back is a permutation: sum phi is constant."""
    if geom == "periodic":
        case, phi0 = W.square_droplet(n=32, side=16)
    elif geom == "walls":
        case, phi0 = W.dam_break(nx=48, ny=24, column=12, dtype="f64", g=1e-5)
    else:
        case, phi0 = W.spreading_case(64, 32, 45.0, dtype="f64", sigma=0.01)
    s = oracle.OracleSim(case).init(phi0)
    m0 = s.diagnostics()["sum_phi"]
    s.step(400)
    d = s.diagnostics()
    assert d["nonfinite"] == 0
    assert abs(d["sum_phi"] - m0) / m0 < 1e-12


def test_d4_symmetry_preserved():
    """A D4-symmetric state (square droplet) stays D4-symmetric: the MRT rates are
    invariant under the lattice symmetries (s^3 = s^5, s^4 = s^6)."""
    case, phi0 = W.square_droplet(n=32, side=16)
    s = oracle.OracleSim(case).init(phi0).step(300)
    phi, u, p = s.moments()
    assert np.abs(phi - phi[:, ::-1]).max() < 1e-13
    assert np.abs(phi - phi.T).max() < 1e-13
    assert np.abs(u[0] + u[0][:, ::-1]).max() < 1e-15
    assert np.abs(p - p.T).max() < 1e-15


def test_rho0_is_a_gauge():
    """rho0 of Eq. (geq) enters only g_0, which never feeds back at s_g^0 = s_g^1 =
    s_g^2 = 1: phi, u, p trajectories do not depend on it."""
    case, phi0 = W.square_droplet(n=32, side=16)
    a = oracle.OracleSim(case).init(phi0).step(200)
    b = oracle.OracleSim(case.replace(rho0=1.0)).init(phi0).step(200)
    for x, y in zip(a.moments(), b.moments()):
        np.testing.assert_allclose(x, y, atol=1e-13)


def test_rejects_unsupported_parameters():
    """eta != 1 is rejected: with eta != 1 the AC model of Eq. (MfMRAC1) recovers
    M (grad phi - lambda n / eta), since m_R carries no eta."""
    case = W.Case(nx=4, ny=4, eta=0.5)
    with pytest.raises(ValueError):
        oracle.OracleSim(case)
    with pytest.raises(ValueError):
        oracle.OracleSim(W.Case(nx=4, ny=4, s_g=(2.0,) + (0.0,) * 8))
