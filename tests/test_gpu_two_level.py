"""Two levels per launch against two one-level launches.

The Allen-Cahn step (stencil or local gradients, present or original model)
advances two levels per launch; an odd level count ends on a one-level launch.  Advancing one state n levels by one
lbm_step call and a copy of it one level per call therefore runs the two kernels
on the same input.  The two must agree bit for bit on every population and
history value (the two-level launch computes its first level with the
one-level step's device functions and hands the second exactly what the copy
would hold), from level 0 (no history yet) and from an odd level, in FP32 and
FP64, on periodic and walled lattices (wetting walls at four contact angles),
ragged tiles, lattices narrower than the launch's region, and states larger
than the last-level cache (streamed, with non-temporal stores).
"""
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TH = (math.radians(70), math.radians(110), math.radians(40), math.radians(140))


def _random(nx, ny, dtype, **kw):
    case = W.Case(nx=nx, ny=ny, rhoA=20.0, rhoB=1.0, nuA=0.05, nuB=0.2, sigma=0.01, W=4.0, M=0.05,
                  body_force=(1e-6, -2e-6), gravity=(0.0, -1e-5), rho_ref=3.0, dtype=dtype, theta=TH, **kw)
    phi0, u0, p0 = W.random_state_fields(case, seed=nx * 31 + ny)
    return case, phi0, u0, p0


def _cases():
    out = {}
    case, phi0 = W.rti(dtype="f32")
    out["rti_256x1024_f32"] = (case, phi0, None, "hydrostatic")
    case, phi0 = W.dam_break(nx=200, ny=100, dtype="f32")
    out["dam_break_200x100_f32"] = (case, phi0, None, "hydrostatic")
    case, phi0 = W.spreading_case(130, 37, 47.0, dtype="f64")
    out["spreading_130x37_f64"] = (case, phi0, None, None)
    for nx, ny, kw in ((70, 9, {}), (70, 9, dict(wall_x=True, wall_y=True)), (1, 1, {}), (9, 1, dict(wall_x=True)),
                       (1, 9, {}), (2, 2, dict(wall_x=True, wall_y=True)), (5, 2, dict(wall_y=True)),
                       (66, 130, dict(wall_y=True))):
        for dtype in ("f32", "f64"):
            walls = "".join(a for a, k in (("x", "wall_x"), ("y", "wall_y")) if kw.get(k))
            out[f"random_{nx}x{ny}{'_walls_' + walls if walls else ''}_{dtype}"] = _random(nx, ny, dtype, **kw)
    # 16-row tiles of the two-level launch (3 x 80 of them), ragged in x and y
    out["random_190x1270_walls_xy_f32"] = _random(190, 1270, "f32", wall_x=True, wall_y=True)
    # states streamed from HBM (two copies above the 320 MB cache bound: non-temporal stores), ragged tiles
    out["random_2050x1030_walls_y_f32"] = _random(2050, 1030, "f32", wall_y=True)
    out["random_1030x1030_walls_x_f64"] = _random(1030, 1030, "f64", wall_x=True)
    # the local gradient scheme (Eq. local; five history planes, general collision)
    for nx, ny, kw, dtype in ((70, 9, {}, "f32"), (70, 9, dict(wall_x=True, wall_y=True), "f64"),
                              (2, 2, dict(wall_x=True, wall_y=True), "f32"), (66, 130, dict(wall_y=True), "f64"),
                              (190, 1270, dict(wall_x=True, wall_y=True), "f32"), (2050, 1030, dict(wall_y=True), "f32")):
        case, phi0, u0, p0 = _random(nx, ny, dtype, **kw)
        walls = "".join(a for a, k in (("x", "wall_x"), ("y", "wall_y")) if kw.get(k))
        out[f"local_{nx}x{ny}{'_walls_' + walls if walls else ''}_{dtype}"] = (case.replace(grad_scheme="local"), phi0,
                                                                              u0, p0)
    case, phi0, u0, p0 = _random(96, 40, "f32", wall_y=True)
    out["local_96x40_walls_y_original_f32"] = (case.replace(model="original", grad_scheme="local"), phi0, u0, p0)
    case, phi0, u0, p0 = _random(96, 40, "f32", wall_y=True)
    out["random_96x40_walls_y_original_f32"] = (case.replace(model="original"), phi0, u0, p0)
    case, phi0, u0, p0 = _random(96, 40, "f64", wall_x=True)
    out["random_96x40_walls_x_rates_f64"] = (
        case.replace(s_f=(1.0, 1.2, 1.3, 0.0, 1.1, 0.0, 1.4, 1.5, 1.6), s_g=(1.0, 1.1, 1.2, 1.0, 1.3, 1.0, 1.4, 0.0, 0.0)),
        phi0, u0, p0)
    return out


CASES = _cases()


@pytest.fixture(autouse=True)
def _two_level_on_every_size():
    """The size rule would keep the small lattices on one-level launches."""
    os.environ["LBM_TWO_LEVEL"] = "1"
    yield
    os.environ.pop("LBM_TWO_LEVEL", None)


def _state(sim):
    s = sim.export_state()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in s.items()}


@pytest.mark.parametrize("start", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_two_level_launch_is_two_one_level_launches(name, start):
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.sim import Sim
    case, phi0, u0, p0 = CASES[name]
    L = api.make_params(case)
    assert api.lbm_levels_per_launch(L) == 2, name
    n = 6
    a = Sim(case).init(phi0, u0, p0)
    b = Sim(case).init(phi0, u0, p0)
    if start:
        a.step(1)
        b.step(1)
    a.step(n)
    for _ in range(n):
        b.step(1)
    sa, sb = _state(a), _state(b)
    assert sa["step"] == sb["step"] == start + n
    for k in ("f", "g", "hist"):
        d = np.abs(sa[k].astype(np.float64) - sb[k].astype(np.float64)).max()
        print(f"{name} from level {start}: {k} max|two-level - one-level| = {d:.3e}", flush=True)
        assert np.array_equal(sa[k], sb[k]), (name, k, d)
    # and the two states keep stepping alike, whichever copy each is in
    a.step(1)
    b.step(2)
    a.step(1)
    sa, sb = _state(a), _state(b)
    assert sa["step"] == sb["step"] == start + n + 2
    for k in ("f", "g", "hist"):
        assert np.array_equal(sa[k], sb[k]), (name, k)
