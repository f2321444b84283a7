"""Pins of the oracle's local gradient scheme for the Allen-Cahn model (Eq. local):
grad phi from the first moment of f instead of the stencil of Eq. central1.
Level 0 (f at equilibrium, no first-moment information) and lap phi keep the
stencils."""
import numpy as np
import pytest

import oracle
import workloads as W


def _flat(Wd):
    case, phi0 = W.flat_interface(nx=2, ny=int(32 * Wd), W=Wd, M=0.05)
    X, Y = W.grid(case)
    ny = case.ny
    lower = Y - ny / 4 < 3 * ny / 4 - Y
    d = np.minimum(Y - ny / 4, 3 * ny / 4 - Y)
    exact = np.where(lower, 1.0, -1.0) / Wd / np.cosh(2 * d / Wd) ** 2     # d/dy of 1/2 + tanh(2d/W)/2
    return case.replace(grad_scheme="local"), phi0, exact


def test_local_gradient_of_the_tanh_interface_is_second_order():
    """Two flat AC interfaces relaxed in the local scheme: grad phi against the
    derivative of the tanh profile.  Measured 1.4e-2 (W = 4) and 3.4e-3 (W = 8) of
    the peak slope; the stencil gradient of the same runs is 8.4e-2 and 2.8e-2."""
    errs = []
    for Wd in (4.0, 8.0):
        case, phi0, exact = _flat(Wd)
        s = oracle.OracleSim(case).init(phi0).step(int(2000 * (Wd / 4) ** 2))
        gx, gy = s.grad()
        assert np.abs(gx).max() < 1e-12
        errs.append(np.abs(gy - exact).max() / np.abs(exact).max())
    assert errs[0] < 2e-2, errs
    assert 3.0 < errs[0] / errs[1] < 6.0, errs


def test_level_zero_uses_the_stencil():
    case, phi0, _ = _flat(4.0)
    s = oracle.OracleSim(case).init(phi0)
    gx, gy = s.grad()
    sx, sy, _ = s.stencils(s.moments()[0])
    np.testing.assert_array_equal(gy, sy)
    np.testing.assert_array_equal(gx, sx)


def test_local_scheme_laplace_law():
    """Static droplet (R = 16, W = 4): p_in - p_out within the same 10% of sigma / R
    as the stencil scheme, parasitic currents small, sum phi conserved."""
    case, phi0 = W.static_droplet(n=64, R=16.0, W=4.0, M=0.02)
    case = case.replace(grad_scheme="local")
    s = oracle.OracleSim(case).init(phi0).step(12000)
    phi, u, p = s.moments()
    X, Y = W.grid(case)
    r = np.hypot(X - 32, Y - 32)
    ratio = (p[r < 16 - 12].mean() - p[r > 16 + 12].mean()) / (case.sigma / 16)
    assert 0.90 < ratio < 1.05, ratio
    assert np.abs(u).max() < 1e-5
    assert abs(phi.sum() - phi0.sum()) < 1e-10 * phi0.sum()


def test_local_scheme_is_allen_cahn_only_and_its_history_needs_the_flux():
    case, phi0, _ = _flat(4.0)
    with pytest.raises(Exception):
        oracle.OracleSim(case.replace(phase_eq="cahn_hilliard", phiB=-1.0)).init(2 * phi0 - 1)
    s = oracle.OracleSim(case).init(phi0)
    st = s.get_state()
    with pytest.raises(AssertionError):
        s.set_state(st["f"], st["g"], 3, phi0, np.zeros((2,) + phi0.shape))


def test_local_scheme_restart_from_the_five_field_history():
    """A run of the local scheme stopped at level n and restarted from f^n, g^n
    and the level n-1 fields phi, u, m^phiC continues bitwise as the
    uninterrupted run (dam break with wetting walls, gravity, 40 x 24)."""
    case, phi0 = W.dam_break(nx=40, ny=24, column=12, dtype="f64", theta_deg=60.0)
    case = case.replace(grad_scheme="local")
    p0 = "hydrostatic"
    a = oracle.OracleSim(case).init(phi0, None, p0).step(29)
    phi_p, u_p, _ = a.moments()
    m_p = a.flux()
    a.step(1)
    st = a.get_state()
    b = oracle.OracleSim(case).set_state(st["f"], st["g"], 30, phi_p, u_p, m_p)
    a.step(7)
    b.step(7)
    sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sa["f"], sb["f"])
    np.testing.assert_array_equal(sa["g"], sb["g"])
    # the stencil closure's m^phiC of the same level is not the history the run used
    m_s = oracle.OracleSim(case.replace(grad_scheme="stencil")).set_state(
        st["f"], st["g"], 30, phi_p, u_p).flux()
    assert np.abs(m_s - m_p).max() > 1e-8
