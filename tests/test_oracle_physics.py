"""Physics pins of the FP64 oracle: closed forms the method must reproduce.

These pin the oracle as a whole (flow solver, forcing, pressure, phase-field
closure and walls) against solutions that do not come from the oracle.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _run(case, phi0, steps):
    return oracle.OracleSim(case).init(phi0).step(steps)


# ------------------------------------------------------------------ single phase
@pytest.mark.parametrize("nu,ny,tol", [(0.1, 16, 1.2e-3), (0.1, 32, 3e-4), (0.125, 32, 1e-6)])
def test_single_phase_poiseuille(nu, ny, tol):
    """Consistency of reduction (Sec. 2): rho_A = rho_B, mu_A = mu_B gives plane
    Poiseuille flow u = G (h^2 - y^2) / (2 mu).  Half-way bounce-back makes the error
    second order (ratio ~4 from ny = 16 to 32) and, with s_q = 1, exact up to round-off
    at nu = 1/8, where (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16."""
    G = 1e-6
    case = W.Case(nx=2, ny=ny, wall_y=True, rhoA=1, rhoB=1, nuA=nu, nuB=nu, body_force=(G, 0))
    s = _run(case, np.full((ny, 2), 0.5), int(12 * (ny / 2) ** 2 / nu))
    _, u, _ = s.moments()
    y = np.arange(ny) + 0.5
    h = ny / 2
    ue = G / (2 * nu) * (h * h - (y - h) ** 2)
    err = np.abs(u[0, :, 0] - ue).max() / ue.max()
    assert err < tol
    assert np.abs(u[1]).max() < 1e-5 * ue.max()   # O(dt^2) normal velocity of the scheme


def test_hydrostatic_pressure():
    """Eq. (computP) with the body force (0, -rho g): at rest dp/dy = -rho g."""
    g, ny = 1e-5, 32
    case = W.Case(nx=2, ny=ny, wall_y=True, rhoA=1, rhoB=1, gravity=(0, -g), rho_ref=0.0)
    s = _run(case, np.full((ny, 2), 0.5), 20000)
    _, u, p = s.moments()
    dp = np.diff(p[:, 0])
    np.testing.assert_allclose(dp, -g, rtol=1e-5)
    assert np.abs(u).max() < 1e-9


# ------------------------------------------------------------------ interface
def test_flat_interface_tanh_profile_second_order():
    """The conservative AC equation is at rest on 1/2 + 1/2 tanh(2 d / W) (its flux
    grad phi - lambda n vanishes, Sec. 2): the lattice keeps the profile to
    O((dx/W)^2) -- the deviation drops ~4x per doubling of W."""
    devs = []
    for Wd in (4.0, 8.0):
        case, phi0 = W.flat_interface(nx=2, ny=int(32 * Wd), W=Wd, M=0.05)
        s = _run(case, phi0, int(2000 * (Wd / 4) ** 2))
        phi, _, _ = s.moments()
        devs.append(np.abs(phi - phi0).max())
    assert devs[0] < 8e-3
    order = math.log2(devs[0] / devs[1])
    assert 1.6 < order < 2.4, devs


@pytest.mark.slow
def test_laplace_law_converges():
    """Static droplet: p_in - p_out -> sigma / R.  The surface force mu_phi grad phi on
    a tanh profile integrates to sigma/R (k kappa int phi'^2 = sigma / R); the lattice
    value approaches it at (at least) second order in dx/W: ~0.935 at W = 4, R = 16
    and ~0.990 at W = 8, R = 32 (deficit ratio ~7 with eps_n = 1e-3, ~4.5 with 1e-6)."""
    ratios = []
    for R, n, Wd, steps in [(16.0, 64, 4.0, 12000), (32.0, 128, 8.0, 24000)]:
        case, phi0 = W.static_droplet(n=n, R=R, W=Wd, M=0.02 * Wd / 4)
        s = _run(case, phi0, steps)
        phi, u, p = s.moments()
        X, Y = W.grid(case)
        r = np.hypot(X - n / 2, Y - n / 2)
        dp = p[r < R - 3 * Wd].mean() - p[r > R + 3 * Wd].mean()
        ratios.append(dp / (case.sigma / R))
        assert np.abs(u).max() < 1e-5       # parasitic currents stay small
    assert 0.90 < ratios[0] < 0.97
    assert 0.97 < ratios[1] < 1.01
    deficit_ratio = (1 - ratios[0]) / (1 - ratios[1])
    assert 3.0 < deficit_ratio < 9.0, ratios


# ------------------------------------------------------------------ layered Poiseuille
def _layered(ratio, ny, Wd, steps):
    case, phi0 = W.layered_poiseuille(nx=2, ny=ny, density_ratio=ratio, visc_ratio=ratio,
                                      umax=1e-4, M=0.1, sigma=1e-3, W=Wd, muB=0.1, dtype="f64")
    y = np.arange(ny) + 0.5 - ny / 2
    G = 1e-6 / W.layered_poiseuille_profile(np.array([0.0]), case, 1.0)[0]
    case = case.replace(body_force=(G, 0))
    ue = W.layered_poiseuille_profile(y, case, G)
    s = _run(case, phi0, steps)
    _, u, _ = s.moments()
    return np.abs(u[0, :, 0] - ue).sum() / np.abs(ue).sum()


def test_layered_poiseuille_paper_setup():
    """Sec. 4.2 set-up (100 nodes across, nu_A = nu_B = 0.1, W = 4): Err_u of the same
    order as the paper's Table 2 (6.6e-3 at 100:1; ours 1.27e-2 -- the paper's node
    placement is not stated)."""
    with open(os.path.join(GOLDEN, "paper_table2_layered_poiseuille.json")) as fh:
        ref = json.load(fh)
    err = _layered(100.0, 100, 4.0, 80000)
    paper = ref["Err_u"][ref["density_ratio"].index(100)]
    assert err < 2.5 * paper


@pytest.mark.slow
def test_layered_poiseuille_second_order_in_interface_width():
    """The closed form of Sec. 4.2 is approached at second order in dx/W at fixed
    geometry in units of W: Err_u(W=4, 100 nodes) / Err_u(W=8, 200 nodes) ~ 4."""
    e4 = _layered(10.0, 100, 4.0, 80000)
    e8 = _layered(10.0, 200, 8.0, 320000)
    assert e4 < 1.5e-2
    assert 3.0 < e4 / e8 < 6.0, (e4, e8)


# ------------------------------------------------------------------ contact angle
def _cap_geometry(phi, nx):
    c = nx // 2
    col = 0.5 * (phi[:, c - 1] + phi[:, c])
    j = np.where(col >= 0.5)[0].max()
    H = j + 0.5 + (col[j] - 0.5) / (col[j] - col[j + 1])

    def width(row):
        r = phi[row]
        idx = np.where(r >= 0.5)[0]
        a, b = idx.min(), idx.max()
        xa = a + 0.5 - (r[a] - 0.5) / (r[a] - r[a - 1])
        xb = b + 0.5 + (r[b] - 0.5) / (r[b] - r[b + 1])
        return xb - xa

    L0, L1 = width(0), width(1)
    L = L0 + 0.5 * (L0 - L1)            # extrapolated from y = 1/2, 3/2 to the wall y = 0
    return H, L


@pytest.mark.parametrize("theta_deg", [60.0, 90.0, 120.0])
def test_equilibrium_contact_angle(theta_deg):
    """Sec. 4.3: the wetting condition of Eq. (Dwetting) yields the prescribed angle,
    theta = 2 arctan(2H/L), and the cap geometry H = R(1 - cos th), L = 2 R sin th,
    R = R0 sqrt((pi/2) / (th - sin th cos th)).  The paper's Table 3 is within 0.8 deg;
    a 1.5 deg tolerance here (R0 = 20 instead of 35, equal densities to equilibrate fast
    -- the equilibrium angle is a static property)."""
    with open(os.path.join(GOLDEN, "paper_table3_contact_angle.json")) as fh:
        ref = json.load(fh)
    i = ref["theta_prescribed_deg"].index(int(theta_deg))
    paper_dev = abs(ref["theta_measured_deg"][i] - theta_deg)
    R0 = 20.0
    case, phi0 = W.spreading_case(120, 60, theta_deg, dtype="f64", R0=R0, rho_ratio=1.0,
                                  mu_ratio=1.0, sigma=0.1, W=5.0, M=0.1, nuB=0.1)
    s = _run(case, phi0, 5000)
    phi, _, _ = s.moments()
    H, L = _cap_geometry(phi, case.nx)
    theta = math.degrees(2 * math.atan(2 * H / L))
    assert abs(theta - theta_deg) < max(1.5, 2 * paper_dev)
    th = math.radians(theta_deg)
    R = R0 * math.sqrt((math.pi / 2) / (th - math.sin(th) * math.cos(th)))
    assert abs(H - R * (1 - math.cos(th))) < 0.6
    assert abs(L - 2 * R * math.sin(th)) < 1.2


def _contour_radii(phi, X, Y, cx, cy, level, nang=32):
    """Radius of the phi = level contour along nang rays from (cx, cy) (linear
    interpolation on the nodes within 0.05 rad of each ray)."""
    r = np.hypot(X - cx, Y - cy)
    ang = np.arctan2(Y - cy, X - cx)
    out = []
    for a in np.linspace(-np.pi, np.pi, nang, endpoint=False):
        m = np.abs(np.angle(np.exp(1j * (ang - a)))) < 0.05
        rr, pp = r[m], phi[m]
        o = np.argsort(rr)
        rr, pp = rr[o], pp[o]
        j = np.where(pp < level)[0][0]
        out.append(rr[j - 1] + (pp[j - 1] - level) / (pp[j - 1] - pp[j]) * (rr[j] - rr[j - 1]))
    return np.array(out)


def test_square_droplet_relaxes_to_the_area_preserving_circle():
    """Sec. 4.1: the square of side D relaxes to the circle of radius R with
    pi R^2 + (4 - pi) W^2 / 4 = D^2 (the area of the square with corners rounded
    by W/2).  64^2, D = 32, W = 4: R = 18.024; measured 18.025, round to 0.002."""
    case, phi0 = W.square_droplet(n=64, side=32.0, dtype="f64")
    s = oracle.OracleSim(case).init(phi0).step(10000)
    phi, u, _ = s.moments()
    X, Y = W.grid(case)
    rs = _contour_radii(phi, X, Y, 32.0, 32.0, 0.5)
    R = math.sqrt((32.0 ** 2 - (4 - math.pi) * case.W ** 2 / 4) / math.pi)
    assert abs(rs.mean() - R) < 0.02, (rs.mean(), R)
    assert rs.std() < 0.01
