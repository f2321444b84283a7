"""Pins of the differentiable CPU reference (oracle/torch_ref.py), the
reference gradient of the GPU adjoint.

Its forward map must equal the C oracle's (a separately written program) on
every boundary kind, and its autograd gradient must equal central finite
differences of the C oracle's loss -- so a wrong term in either the torch
restatement or in the chain rule would show here.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.torch_ref import OPP, TorchRef, as_params, loss_and_grads, moment_matrix

GEOMS = {
    "periodic": dict(),
    "walls_y": dict(wall_y=True, theta=(math.pi / 2, math.pi / 2, math.radians(50), math.radians(120))),
    "walls_x": dict(wall_x=True, theta=(math.radians(60), math.radians(130), math.pi / 2, math.pi / 2)),
    "walls_xy": dict(wall_x=True, wall_y=True,
                     theta=(math.radians(70), math.radians(110), math.radians(40), math.radians(140))),
}


def test_moment_matrix_equals_oracle_table():
    _, _, _, M, Minv = oracle.lattice()
    np.testing.assert_array_equal(moment_matrix().numpy(), M)
    np.testing.assert_allclose(torch.linalg.inv(moment_matrix()).numpy(), Minv, atol=1e-15)
    assert OPP == tuple(int(i) for i in [0, 3, 4, 1, 2, 7, 8, 5, 6])


def _random_state(case, seed):
    phi0, u0, p0 = W.random_state_fields(case, seed=seed)
    st = oracle.OracleSim(case).init(phi0, u0, p0).get_state()
    rng = np.random.default_rng(seed + 1)
    f = st["f"] + 1e-4 * rng.standard_normal(st["f"].shape)
    g = st["g"] + 1e-5 * rng.standard_normal(st["g"].shape)
    php = phi0 + 1e-3 * rng.standard_normal(phi0.shape)
    upr = u0 + 1e-4 * rng.standard_normal(u0.shape)
    return f, g, php, upr


def _case(geom, nx=23, ny=17, **kw):
    base = dict(nx=nx, ny=ny, rhoA=20.0, rhoB=1.0, nuA=0.05, nuB=0.2, sigma=0.01, W=4.0, M=0.05,
                body_force=(1e-6, -2e-6), gravity=(0.0, -1e-5), rho_ref=3.0, dtype="f64")
    return W.Case(**{**base, **GEOMS[geom], **kw})


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("n", [0, 4])
@pytest.mark.parametrize("visc", ["linear_mu", "inverse_nu"])
def test_step_equals_oracle(geom, n, visc):
    case = _case(geom, visc_law=visc)
    f, g, php, upr = _random_state(case, seed=11 + n)
    ref = TorchRef(case)
    grav, theta = as_params(case)
    st = dict(f=torch.tensor(f), g=torch.tensor(g), phi_prev=torch.tensor(php), u_prev=torch.tensor(upr), n=n)
    with torch.no_grad():
        out = ref.run(st, 3, grav, theta)
    o = oracle.OracleSim(case).set_state(f, g, n, php, upr).step(3).get_state()
    assert np.abs(out["f"].numpy() - o["f"]).max() < 1e-13
    assert np.abs(out["g"].numpy() - o["g"]).max() < 1e-13
    np.testing.assert_allclose(out["phi_prev"].numpy(), o["phi_prev"], atol=1e-13)


def test_trajectory_from_init_equals_oracle():
    case, phi0 = W.dam_break(nx=32, ny=16, column=8, dtype="f64", theta_deg=70.0)
    p0 = oracle.hydrostatic_pressure(case, phi0)
    ref = TorchRef(case)
    grav, theta = as_params(case)
    with torch.no_grad():
        st = ref.run(ref.init(torch.tensor(phi0), torch.tensor(p0)), 40, grav, theta)
    o = oracle.OracleSim(case).init(phi0, None, p0).step(40)
    phi_o, u_o, _ = o.moments()
    assert np.abs(ref.phi(st).numpy() - phi_o).max() < 1e-12


# ---------------------------------------------------------------- gradient pins
def _oracle_loss(case, phi0, target, nsteps, p0):
    o = oracle.OracleSim(case).init(phi0, None, p0).step(nsteps)
    phi, _, _ = o.moments()
    return float(np.sum((phi - target) ** 2))


def _grad_case():
    """Walls on all faces with four contact angles, inverse-nu law, gravity; a
    smooth random phi0 that is neither bulk phase at any wall."""
    case = _case("walls_xy", nx=24, ny=14, visc_law="inverse_nu", gravity=(0.0, -2e-4))
    phi0, _, _ = W.random_state_fields(case, seed=4)
    rng = np.random.default_rng(5)
    target = np.clip(phi0 + 0.05 * rng.standard_normal(phi0.shape), 0, 1)
    return case, phi0, target


def test_gradient_equals_oracle_finite_differences():
    """dL/dgravity, dL/dtheta_k and two directional derivatives in phi0 from
    autograd equal central differences of the C oracle (relative 1e-6)."""
    case, phi0, target = _grad_case()
    nsteps = 25
    p0 = np.zeros_like(phi0)
    L, dphi0, dgrav, dth = loss_and_grads(case, phi0, target, nsteps, p0)
    assert abs(L - _oracle_loss(case, phi0, target, nsteps, p0)) < 1e-12 * max(1.0, L)

    def fd(make, h):
        lp = _oracle_loss(*make(+h))
        lm = _oracle_loss(*make(-h))
        return (lp - lm) / (2 * h)

    checks = []
    gy = case.gravity[1]
    checks.append((fd(lambda h: (case.replace(gravity=(0.0, gy + h)), phi0, target, nsteps, p0), 1e-7),
                   dgrav[1], "gravity_y"))
    for k in range(4):
        def mk(h, k=k):
            th = list(case.theta)
            th[k] += h
            return case.replace(theta=tuple(th)), phi0, target, nsteps, p0
        checks.append((fd(mk, 1e-5), dth[k], f"theta{k}"))
    rng = np.random.default_rng(9)
    for j in range(2):
        dirn = rng.standard_normal(phi0.shape)
        checks.append((fd(lambda h: (case, phi0 + h * dirn, target, nsteps, p0), 1e-6),
                       float(np.sum(dphi0 * dirn)), f"phi0 dir {j}"))
    for num, ana, what in checks:
        print(f"{what}: fd={num:.10e} autograd={ana:.10e}")
    for num, ana, what in checks:
        assert abs(num - ana) <= 1e-6 * abs(ana), (what, num, ana)
