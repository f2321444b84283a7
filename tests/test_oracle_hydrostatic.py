"""The oracle's hydrostatic initial pressure (the gravity-driven set-ups of
Secs. 4.4 and 4.5 leave the initial pressure unstated; it is read as the fluids
at rest), pinned by what it is for: far from the interface every column
balances dp/dy = (rho - rho_ref) g_y exactly, and a stably stratified
two-phase column started from it stays close to rest, where p = 0 launches a
pressure transient through the whole lattice."""
import math

import numpy as np

import oracle
import workloads as W


def _stratified(ny=96, rho_ratio=3.0, g=1e-5):
    case = W.Case(nx=4, ny=ny, wall_y=True, rhoA=rho_ratio, rhoB=1.0, nuA=0.05, nuB=0.05, sigma=1e-3, W=4.0,
                  M=0.05, gravity=(0.0, -g), rho_ref=0.5, dtype="f64")
    X, Y = W.grid(case)
    return case, W.tanh_profile(ny / 2.0 - Y, case.W)     # heavy phase A below


def test_hydrostatic_pressure_balances_each_bulk_column():
    case, phi0 = _stratified()
    p0 = oracle.hydrostatic_pressure(case, phi0)
    assert abs(p0.mean()) < 1e-15
    dp = np.diff(p0, axis=0)                      # p[j+1] - p[j]
    g = case.gravity[1]
    np.testing.assert_allclose(dp[:25], (case.rhoA - case.rho_ref) * g, rtol=1e-6)    # heavy bulk
    np.testing.assert_allclose(dp[-25:], (case.rhoB - case.rho_ref) * g, rtol=1e-6)   # light bulk
    # across the interface the jump is the integral of the density law over the tanh layer
    total = p0[0, 0] - p0[-1, 0]
    exact = -g * ((case.rhoA + case.rhoB) / 2 - case.rho_ref) * (case.ny - 1)
    assert abs(total - exact) < 1e-6 * abs(exact)
    assert np.all(oracle.hydrostatic_pressure(case.replace(gravity=(0.0, 0.0)), phi0) == 0)


def test_hydrostatic_start_is_close_to_rest():
    case, phi0 = _stratified()
    u_h = np.abs(oracle.OracleSim(case).init(phi0, None, "hydrostatic").step(400).moments()[1]).max()
    u_0 = np.abs(oracle.OracleSim(case).init(phi0, None, None).step(400).moments()[1]).max()
    print(f"max|u| after 400 steps: hydrostatic start {u_h:.2e}, p = 0 start {u_0:.2e}")
    assert u_h < 0.03 * u_0


def test_seeded_spreading_mix_is_reproducible():
    a = W.spreading_batch()
    b = W.spreading_batch()
    assert [(c.nx, c.ny, c.theta) for c, _ in a] == [(c.nx, c.ny, c.theta) for c, _ in b]
    sizes = {(c.nx, c.ny) for c, _ in a}
    assert sizes == set(W.SPREAD_SIZES)
    th = [math.degrees(c.theta[2]) for c, _ in a]
    assert 30.0 <= min(th) and max(th) <= 150.0
