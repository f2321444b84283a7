"""Paper-replica accuracy suite on the GPU (FP64): the set-ups of Sec. 4.2
(Table 2, layered Poiseuille) and Sec. 4.3 (Table 3, droplet spreading) run
through the C ABI and compared with the printed numbers (tests/golden/).

Table 3 is matched within max(1.5 deg, twice the paper's own deviation).
Table 2 runs with the paper's unregularised normal (eps_n = 1e-9 in FP64; the
default 1e-4 is chosen for FP32 conditioning and, at density ratio 1000, its
residual flux in the tanh tails dominates the error at fine resolution).  Our
Err_u is 1.1e-2 .. 1.3e-2 where the paper prints 1.5e-3 .. 8.4e-3; the
difference converges away at second order in dx/W, i.e. it is discretisation
(the paper samples U_x at y = j dx with an unstated wall placement, we use
half-way walls and nodes at half-integers) -- checked here by doubling the
resolution at fixed W/h.  The GPU value equals the oracle's at the paper's
set-up.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _sim():
    from paper_2111_00847_amd.sim import Sim
    return Sim


# ---------------------------------------------------------------- Table 2
def _layered_case(ratio, ny, Wd):
    """Sec. 4.2: nu_A = nu_B = 0.1 (mu ratio = density ratio), M = 0.1, W = 4 dx,
    U_c = 1e-4 in the paper's units, i.e. 1e-6 in lattice units (dx = 1/100,
    c = 100); Err_u does not depend on U_c (Stokes flow)."""
    case, phi0 = W.layered_poiseuille(nx=10, ny=ny, density_ratio=ratio, visc_ratio=ratio, umax=1e-6, M=0.1,
                                      sigma=1e-3, W=Wd, muB=0.1, dtype="f64")
    case = case.replace(eps_n=1e-9)
    y = np.arange(ny) + 0.5 - ny / 2
    ue = W.layered_poiseuille_profile(y, case, case.body_force[0])
    return case, phi0, ue


def _err(u, ue):
    return float(np.abs(u[0, :, 0] - ue).sum() / np.abs(ue).sum())


def _gpu_err(ratio, ny, Wd, steps):
    case, phi0, ue = _layered_case(ratio, ny, Wd)
    s = _sim()(case, stream=torch.cuda.Stream()).init(phi0).step(steps)
    _, u, _ = s.moments_np()
    return _err(u, ue)


@pytest.mark.parametrize("ratio", [10, 100, 150, 1000])
def test_table2_layered_poiseuille(ratio):
    ref = _golden("paper_table2_layered_poiseuille.json")
    paper = ref["Err_u"][ref["density_ratio"].index(ratio)]
    err = _gpu_err(float(ratio), 100, 4.0, 160000)
    print(f"Table 2, density ratio {ratio}: Err_u {err:.3e} (paper {paper:.3e})", flush=True)
    assert err < 1.5e-2 and err < 8.0 * paper


def test_table2_gpu_equals_oracle():
    """At the paper's set-up (density ratio 1000, 80000 steps) the GPU's Err_u is
    the oracle's."""
    case, phi0, ue = _layered_case(1000.0, 100, 4.0)
    g = _sim()(case, stream=torch.cuda.Stream()).init(phi0).step(80000)
    o = oracle.OracleSim(case).init(phi0).step(80000)
    eg, eo = _err(g.moments_np()[1], ue), _err(o.moments()[1], ue)
    print(f"Err_u GPU {eg:.10e} oracle {eo:.10e}", flush=True)
    assert abs(eg - eo) <= 1e-8 * eo


def test_table2_error_is_second_order_discretisation():
    """Density ratio 1000: doubling the resolution at fixed W/h (W 4 -> 8 on 100 ->
    200 nodes) divides Err_u by about 4 (measured 1.10e-2 -> 2.74e-3)."""
    e1 = _gpu_err(1000.0, 100, 4.0, 160000)
    e2 = _gpu_err(1000.0, 200, 8.0, 640000)
    print(f"Err_u {e1:.3e} -> {e2:.3e}: ratio {e1 / e2:.2f}", flush=True)
    assert 3.0 < e1 / e2 < 6.0


# ---------------------------------------------------------------- Table 3
def _cap_geometry(phi, nx):
    """Height H on the centre line and wetted length L (extrapolated from the two
    first rows to the wall) of the phi = 1/2 contour."""
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
    return H, L0 + 0.5 * (L0 - L1)


@pytest.mark.parametrize("theta_deg", [30, 45, 60, 90, 120, 150])
def test_table3_contact_angle(theta_deg):
    """Sec. 4.3 set-up: 200 x 100, R0 = 35, W = 5, density ratio 1000, viscosity
    ratio 100, sigma = 0.2, M = 0.1; theta = 2 arctan(2H/L) after 300000 steps."""
    ref = _golden("paper_table3_contact_angle.json")
    i = ref["theta_prescribed_deg"].index(theta_deg)
    paper = ref["theta_measured_deg"][i]
    case, phi0 = W.spreading_case(200, 100, float(theta_deg), dtype="f64", R0=35.0, rho_ratio=1000.0,
                                  mu_ratio=100.0, sigma=0.2, W=5.0, M=0.1, nuB=0.1)
    s = _sim()(case, stream=torch.cuda.Stream()).init(phi0).step(300000)
    phi, u, _ = s.moments_np()
    H, L = _cap_geometry(phi, case.nx)
    theta = math.degrees(2 * math.atan(2 * H / L))
    print(f"Table 3, {theta_deg} deg: measured {theta:.2f} (paper {paper})", flush=True)
    assert abs(theta - theta_deg) <= max(1.5, 2 * abs(paper - theta_deg))
