"""The Allen-Cahn step with the local gradient scheme (Eq. local) on the GPU
against the oracle, through the C ABI.  Trajectories from lbm_init (the scheme's
history of m^phiC cannot be imported): FP64 within 1e-10, FP32 within
max|dphi| <= 1e-5 and max|du|/Umax <= 1e-4; ragged tiles, all boundary kinds."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(case, phi0, steps, p0=None):
    from paper_2111_00847_amd.sim import Sim
    case = case.replace(grad_scheme="local")
    if p0 is None and any(case.gravity):
        p0 = W.hydrostatic_pressure(case, phi0)
    g = Sim(case).init(phi0, None, p0).step(steps)
    o = oracle.OracleSim(case.replace(dtype="f64")).init(phi0, None, p0).step(steps)
    torch.cuda.synchronize()
    phi_g, u_g, p_g = g.moments_np()
    phi_o, u_o, p_o = o.moments()
    umax = np.abs(u_o).max()
    dphi = np.abs(phi_g - phi_o).max()
    du = np.abs(u_g - u_o).max() / umax
    return dphi, du, umax, np.abs(p_g - p_o).max()


CASES = {
    "square_droplet_70x37": (lambda dt: W.square_droplet(n=64, side=30.0, dtype=dt)[0].replace(nx=70, ny=37),
                             lambda case: W.tanh_profile(15.0 - np.maximum(np.abs(W.grid(case)[0] - 35),
                                                                           np.abs(W.grid(case)[1] - 18.5)), 4.0),
                             1200),
    "dam_break_64x32": (lambda dt: W.dam_break(nx=64, ny=32, column=16, dtype=dt, theta_deg=70.0)[0],
                        lambda case: W.dam_break(nx=64, ny=32, column=16, theta_deg=70.0)[1], 600),
    "rti_64x256": (lambda dt: W.rti(nx=64, ny=256, dtype=dt)[0], lambda case: W.rti(nx=64, ny=256)[1], 1000),
    "spreading_128x64": (lambda dt: W.spreading_case(128, 64, 60.0, dtype=dt)[0],
                         lambda case: W.spreading_case(128, 64, 60.0)[1], 1000),
}


@pytest.mark.parametrize("name", list(CASES))
def test_local_scheme_fp64(name):
    mk, phi_of, steps = CASES[name]
    case = mk("f64")
    dphi, du, umax, dp = _pair(case, phi_of(case), steps)
    print(f"local {name} fp64 {steps} steps: max|dphi|={dphi:.2e} max|du|/Umax={du:.2e} (Umax {umax:.2e})",
          flush=True)
    assert dphi <= 1e-10 and du <= 1e-9


@pytest.mark.parametrize("name", ["square_droplet_70x37", "rti_64x256"])
def test_local_scheme_fp32(name):
    mk, phi_of, steps = CASES[name]
    case = mk("f32")
    dphi, du, umax, dp = _pair(case, phi_of(case), steps)
    print(f"local {name} fp32 {steps} steps: max|dphi|={dphi:.2e} max|du|/Umax={du:.2e} (Umax {umax:.2e})",
          flush=True)
    assert dphi <= 1e-5 and du <= 1e-4


def test_local_scheme_full_size_rti_fp32_prefix():
    """The benchmark's local-scheme workload (RTI 4096 x 4096 is too large for the
    oracle): RTI 1024 x 1024, FP32, 100 steps, in the same launch shape."""
    case, phi0 = W.rti(nx=1024, ny=1024)
    dphi, du, umax, dp = _pair(case, phi0, 100)
    print(f"local rti 1024^2 fp32 100 steps: max|dphi|={dphi:.2e} max|du|/Umax={du:.2e} (Umax {umax:.2e})",
          flush=True)
    assert dphi <= 1e-5 and du <= 1e-4


def test_local_scheme_diagnostics_fp64():
    from paper_2111_00847_amd.sim import Sim
    mk, phi_of, steps = CASES["square_droplet_70x37"]
    case = mk("f64").replace(grad_scheme="local")
    phi0 = phi_of(case)
    dg = Sim(case).init(phi0).step(steps).diagnostics()
    do = oracle.OracleSim(case).init(phi0).step(steps).diagnostics()
    for key in ("sum_phi", "max_div", "Du_rms", "Sm_rms", "umax"):
        print(f"local diagnostics {key}: GPU {dg[key]:.12e} oracle {do[key]:.12e}", flush=True)
        assert abs(dg[key] - do[key]) <= 1e-8 * abs(do[key]) + 1e-16, key


def test_local_scheme_graph_replay_equals_eager():
    """lbm_step on a side stream replays captured graphs of 32 steps of the
    local-scheme kernel; the moments equal those of eager launches bitwise."""
    from paper_2111_00847_amd.sim import Sim
    case, phi0 = W.rti(nx=128, ny=256)
    case = case.replace(grad_scheme="local")
    p0 = W.hydrostatic_pressure(case, phi0)
    a = Sim(case).init(phi0, None, p0).step(101)
    b = Sim(case, stream=torch.cuda.Stream()).init(phi0, None, p0)
    b.step(70)
    b.step(31)
    torch.cuda.synchronize()
    for x, y in zip(a.moments(), b.moments()):
        assert torch.equal(x, y)
