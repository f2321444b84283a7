"""Degenerate lattices on the GPU against the oracle: a single node, one-node
wide or tall strips (every stencil and streaming neighbour across the periodic
axis is the node itself), and walls two nodes apart (both wetting walls act on
the same two nodes).  Every variant of the step, FP64, 30 steps from a random
state; phi within 1e-10 and u within 1e-9 of the oracle's Umax."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TH = (math.radians(70), math.radians(110), math.radians(40), math.radians(140))
SHAPES = {
    "1x1": dict(nx=1, ny=1),
    "1x9": dict(nx=1, ny=9),
    "1x9_walls_y": dict(nx=1, ny=9, wall_y=True),
    "9x1": dict(nx=9, ny=1),
    "9x1_walls_x": dict(nx=9, ny=1, wall_x=True),
    "2x2_walls_xy": dict(nx=2, ny=2, wall_x=True, wall_y=True),
    "2x5_walls_x": dict(nx=2, ny=5, wall_x=True),
    "5x2_walls_y": dict(nx=5, ny=2, wall_y=True),
}
VARIANTS = {
    "present": dict(),
    "local": dict(grad_scheme="local"),
    "corrected": dict(model="corrected"),
    "cahn_hilliard": dict(phase_eq="cahn_hilliard"),
}


def _case(shape, variant, dtype="f64"):
    case = W.Case(rhoA=20.0, rhoB=1.0, nuA=0.05, nuB=0.2, sigma=0.01, W=4.0, M=0.05,
                  body_force=(1e-6, -2e-6), gravity=(0.0, -1e-5), rho_ref=3.0, dtype=dtype, theta=TH,
                  name=f"{shape}_{variant}", **SHAPES[shape])
    phi0, u0, p0 = W.random_state_fields(case, seed=case.nx * 31 + case.ny)
    opts = dict(VARIANTS[variant])
    if opts.pop("phase_eq", None):
        case, phi0 = W.to_cahn_hilliard(case, phi0)
    return case.replace(**opts), phi0, u0, p0


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("shape", list(SHAPES))
def test_degenerate_lattice(shape, variant):
    from paper_2111_00847_amd.sim import Sim
    case, phi0, u0, p0 = _case(shape, variant)
    g = Sim(case).init(phi0, u0, p0).step(30)
    o = oracle.OracleSim(case).init(phi0, u0, p0).step(30)
    phi_g, u_g, p_g = g.moments_np()
    phi_o, u_o, p_o = o.moments()
    umax = np.abs(u_o).max()
    dphi = np.abs(phi_g - phi_o).max()
    du = np.abs(u_g - u_o).max() / umax
    print(f"{shape} {variant}: max|dphi|={dphi:.2e} max|du|/Umax={du:.2e} (Umax {umax:.2e})", flush=True)
    assert np.isfinite(phi_g).all() and np.isfinite(u_g).all()
    assert dphi <= 1e-10 and du <= 1e-9


@pytest.mark.parametrize("mix", ["plain", "all_variants"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_degenerate_lattices_in_one_batch(dtype, mix):
    """The degenerate shapes in one batch (plain: the 8 Allen-Cahn lattices, one
    batch body; all_variants: 32 lattices, every body) against the same lattices
    advanced alone: Allen-Cahn with the stencil bitwise, the other bodies within
    16 units of rounding (another tile height than the lone lattice may run)."""
    from paper_2111_00847_amd.sim import BatchSim, Sim
    variants = ["present"] if mix == "plain" else list(VARIANTS)
    cases = [_case(s, v, dtype) for s in SHAPES for v in variants]
    B = BatchSim([c for c, *_ in cases])
    B.init([phi for _, phi, _, _ in cases], [p0 for *_, p0 in cases])
    B.step(30)
    eps = np.finfo(np.float64 if dtype == "f64" else np.float32).eps
    for c, (case, phi0, _, p0) in enumerate(cases):
        alone = Sim(case).init(phi0, None, p0).step(30)
        sa, sb = B.case(c).export_state(), alone.export_state()
        assert sa["step"] == sb["step"] == 30, case.name
        exact = case.phase_eq == "allen_cahn" and case.model != "corrected" and case.grad_scheme == "stencil"
        for key in ("f", "g", "hist"):
            ta, tb = sa[key].cpu().numpy(), sb[key].cpu().numpy()
            assert np.isfinite(ta).all(), (case.name, key)
            if exact:
                np.testing.assert_array_equal(ta, tb, err_msg=f"{case.name} {key}")
            else:
                err = float(np.abs(ta - tb).max())
                assert err <= 16 * eps * max(1.0, float(np.abs(tb).max())), (case.name, key, err)


def test_zero_steps_is_a_no_op_and_negative_counts_are_refused():
    """lbm_step / lbm_batch_step with nsteps = 0 leave the state untouched; a
    negative count is LBM_E_SIZE and also leaves it untouched."""
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd._lib import LbmError
    from paper_2111_00847_amd.sim import BatchSim, Sim
    case, phi0, u0, p0 = _case("5x2_walls_y", "present")
    s = Sim(case).init(phi0, u0, p0).step(3)
    torch.cuda.synchronize()
    before = s.state.clone()
    s.step(0)
    with pytest.raises(LbmError) as e:
        api.lbm_step(s.p, s.state, -1)
    assert e.value.code == -2
    torch.cuda.synchronize()
    assert torch.equal(before, s.state)
    assert s.export_state()["step"] == 3
    B = BatchSim([case, case.replace(nx=7)])
    B.init([phi0, np.tile(phi0, (1, 2))[:, :7]], [p0, np.tile(p0, (1, 2))[:, :7]])
    B.step(2)
    torch.cuda.synchronize()
    before = B.state.clone()
    B.step(0)
    torch.cuda.synchronize()
    assert torch.equal(before, B.state)
