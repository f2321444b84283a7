"""The Cahn-Hilliard variant (Sec. 2, Eq. CHE; App. C, Eq. MfMRCH1) on the GPU
against the oracle, through the C ABI; and the paper's Table 1 comparison of
the present and original models at its own square-droplet set-up.

Bars as for the Allen-Cahn path: one-step maps populations <= 1e-14 (FP64);
trajectories 1e-10 (FP64), max|dphi| <= 1e-5 and max|du|/Umax <= 1e-4 (FP32).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GEOMS = {
    "periodic": dict(),
    "walls_y": dict(wall_y=True, theta=(math.pi / 2, math.pi / 2, math.radians(50), math.radians(120))),
    "walls_x": dict(wall_x=True, theta=(math.radians(60), math.radians(130), math.pi / 2, math.pi / 2)),
    "walls_xy": dict(wall_x=True, wall_y=True,
                     theta=(math.radians(70), math.radians(110), math.radians(40), math.radians(140))),
}


def _contour_radii(phi, X, Y, cx, cy, level, nang=32):
    """Radius of the phi = level contour along nang rays from (cx, cy)."""
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


def _sim():
    from paper_2111_00847_amd.sim import Sim
    return Sim


def _ch_case(geom, nx, ny, **kw):
    base = dict(nx=nx, ny=ny, rhoA=20.0, rhoB=1.0, nuA=0.05, nuB=0.2, sigma=0.01, W=4.0, M=0.05,
                body_force=(1e-6, -2e-6), gravity=(3e-6, -1e-5), rho_ref=3.0, dtype="f64",
                phase_eq="cahn_hilliard", phiA=1.0, phiB=-1.0)
    return W.Case(**{**base, **GEOMS[geom], **kw})


def _random_state(case, seed):
    phi01, u0, p0 = W.random_state_fields(case, seed=seed)
    phi0 = 2.0 * phi01 - 1.0
    st = oracle.OracleSim(case).init(phi0, u0, p0).get_state()
    rng = np.random.default_rng(seed + 1)
    f = st["f"] + 1e-4 * rng.standard_normal(st["f"].shape)
    g = st["g"] + 1e-5 * rng.standard_normal(st["g"].shape)
    php = phi0 + 1e-3 * rng.standard_normal(phi0.shape)
    upr = u0 + 1e-4 * rng.standard_normal(u0.shape)
    return f, g, php, upr


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("shape", [(37, 23), (70, 5), (5, 41)])
@pytest.mark.parametrize("step", [0, 5])
def test_ch_one_step_map_fp64(geom, shape, step):
    nx, ny = shape
    case = _ch_case(geom, nx, ny)
    f, g, php, upr = _random_state(case, seed=nx + 3 * ny)
    hist = np.concatenate([php[None], upr], 0)
    gs = _sim()(case).import_state(f, g, hist if step > 0 else None, step).step(1)
    o = oracle.OracleSim(case).set_state(f, g, step, php, upr).step(1)
    so, sg = o.get_state(), gs.export_state()
    df = np.abs(sg["f"].cpu().numpy() - so["f"]).max()
    dg = np.abs(sg["g"].cpu().numpy() - so["g"]).max()
    print(f"CH {geom} {shape} step {step}: max|df|={df:.2e} max|dg|={dg:.2e}", flush=True)
    assert df < 1e-14 and dg < 1e-14
    for a, b in zip(gs.moments_np(), o.moments()):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


@pytest.mark.parametrize("geom", list(GEOMS))
def test_corrected_model_one_step_map_fp64(geom):
    """Corrected model (m = rho u plus F_a; App. A, Eq. NS2-add) against the oracle."""
    case = _ch_case(geom, 37, 23, model="corrected", sigma=0.2, M=0.5)
    f, g, php, upr = _random_state(case, seed=5)
    hist = np.concatenate([php[None], upr], 0)
    gs = _sim()(case).import_state(f, g, hist, 4).step(1)
    o = oracle.OracleSim(case).set_state(f, g, 4, php, upr).step(1)
    so, sg = o.get_state(), gs.export_state()
    df = np.abs(sg["f"].cpu().numpy() - so["f"]).max()
    dg = np.abs(sg["g"].cpu().numpy() - so["g"]).max()
    print(f"CH corrected {geom}: max|df|={df:.2e} max|dg|={dg:.2e}", flush=True)
    assert df < 1e-14 and dg < 1e-14
    for a, b in zip(gs.moments_np(), o.moments()):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


def _pair(case, phi0, steps):
    g = _sim()(case).init(phi0).step(steps)
    o = oracle.OracleSim(case.replace(dtype="f64")).init(phi0).step(steps)
    torch.cuda.synchronize()
    return g, o


def _compare(g, o, tol_phi, tol_u, what):
    phi_g, u_g, _ = g.moments_np()
    phi_o, u_o, _ = o.moments()
    dphi = np.abs(phi_g - phi_o).max()
    umax = np.abs(u_o).max()
    du = np.abs(u_g - u_o).max() / umax
    print(f"{what}: max|dphi|={dphi:.2e} max|du|/Umax={du:.2e} (Umax {umax:.2e})", flush=True)
    assert dphi <= tol_phi and du <= tol_u


def test_ch_square_droplet_fp64_and_diagnostics():
    case, phi0 = W.square_droplet_ch(n=64, R=16.0, sigma=1e-3, rho_ratio=100.0)
    g, o = _pair(case, phi0, 1500)
    _compare(g, o, 1e-10, 1e-9, "CH square droplet fp64")
    dg, do = g.diagnostics(), o.diagnostics()
    for key in ("sum_phi", "max_div", "Du_rms", "Sm_rms", "umax"):
        assert abs(dg[key] - do[key]) <= 1e-8 * abs(do[key]) + 1e-16, (key, dg[key], do[key])


def test_ch_square_droplet_fp32():
    case, phi0 = W.square_droplet_ch(n=64, R=16.0, sigma=1e-3, rho_ratio=100.0, dtype="f32")
    g, o = _pair(case, phi0, 1500)
    _compare(g, o, 1e-5, 1e-4, "CH square droplet fp32")


def test_corrected_model_square_droplet_fp64():
    case, phi0 = W.square_droplet_ch(n=64, R=16.0, sigma=1e-3, rho_ratio=100.0, model="corrected")
    g, o = _pair(case, phi0, 1500)
    _compare(g, o, 1e-10, 1e-9, "CH corrected square droplet fp64")
    dg, do = g.diagnostics(), o.diagnostics()
    for key in ("Du_rms", "Sm_rms"):
        assert abs(dg[key] - do[key]) <= 1e-8 * abs(do[key]), (key, dg[key], do[key])


def test_ch_walls_gravity_fp64():
    """A CH interface under gravity in a box with wetting walls (all four faces)."""
    case = _ch_case("walls_xy", 48, 40, gravity=(0.0, -2e-5), rho_ref=0.0, body_force=(0.0, 0.0))
    X, Y = W.grid(case)
    phi0 = W.tanh_profile(20.0 + 3.0 * np.cos(2 * np.pi * X / 48) - Y, 4.0, 1.0, -1.0)
    g, o = _pair(case, phi0, 800)
    _compare(g, o, 1e-10, 1e-9, "CH walls + gravity fp64")


def test_ch_table1_present_vs_original():
    """Sec. 4.1 set-up (200 x 200, density ratio 1000, CH, nu = M = 0.1, sigma 1e-5
    in lattice units): the present model's mass source S_m^rms falls below the
    original model's and keeps falling relative to it (measured ratios 0.48,
    0.36, 0.29 at 1e5, 3e5, 1e6 steps; the paper's steady value is 0.12), while
    D_u^rms is the same for both models, and the corrected model's S_m^rms is
    the original's -- the pattern of Table 1.  (Table 1's lower D_u^rms of the
    corrected model is not reproduced: F_a as defined moves it by < 0.1% here.)"""
    marks = (100000, 300000, 1000000)
    out = {}
    radius = {}
    for model in ("present", "original", "corrected"):
        case, phi0 = W.square_droplet_ch(model=model)
        s = _sim()(case, stream=torch.cuda.Stream()).init(phi0)
        done = 0
        for m in marks:
            s.step(m - done)
            done = m
            d = s.diagnostics()
            out[model, m] = (d["Sm_rms"], d["Du_rms"])
            print(f"Table 1 set-up, {model}, {m} steps: S_m^rms {d['Sm_rms']:.4e} D_u^rms {d['Du_rms']:.4e}",
                  flush=True)
        phi, _, _ = s.moments_np()
        X, Y = W.grid(case)
        radius[model] = _contour_radii(phi, X, Y, 100.0, 100.0, 0.0)
        print(f"Table 1 set-up, {model}: final radius {radius[model].mean():.3f} +- {radius[model].std():.3f}",
              flush=True)
    # The radius is printed, not asserted: the heavy droplet's viscous relaxation
    # time (mu R / sigma ~ 5e8 steps here) is far beyond the 1e6 steps run (measured
    # 49.26 +- 5.04, still square-ish); the circle of Sec. 4.1 is pinned on a CH
    # droplet that relaxes in reach (tests/test_oracle_ch.py).
    ratios = [out["present", m][0] / out["original", m][0] for m in marks]
    print("S_m^rms present / original:", ", ".join(f"{r:.3f}" for r in ratios), flush=True)
    assert ratios[0] < 0.55 and ratios[1] < ratios[0] and ratios[2] < ratios[1] and ratios[2] < 0.33
    for m in marks:
        assert abs(out["present", m][1] - out["original", m][1]) <= 1e-3 * out["original", m][1]
        # the corrected model shares the original's mass flux rho u: the same S_m^rms (as printed)
        assert abs(out["corrected", m][0] - out["original", m][0]) <= 1e-2 * out["original", m][0]


@pytest.mark.parametrize("geom", ["periodic", "walls_xy"])
def test_ch_one_step_map_fp64_eight_row_tiles(geom):
    """A lattice large enough for the 8-row CH tiles (the benchmark's launch shape),
    ragged in both directions."""
    case = _ch_case(geom, 1000, 530)
    f, g, php, upr = _random_state(case, seed=17)
    hist = np.concatenate([php[None], upr], 0)
    gs = _sim()(case).import_state(f, g, hist, 3).step(1)
    o = oracle.OracleSim(case).set_state(f, g, 3, php, upr).step(1)
    so, sg = o.get_state(), gs.export_state()
    df = np.abs(sg["f"].cpu().numpy() - so["f"]).max()
    dg = np.abs(sg["g"].cpu().numpy() - so["g"]).max()
    print(f"CH {geom} 1000x530: max|df|={df:.2e} max|dg|={dg:.2e}", flush=True)
    assert df < 1e-14 and dg < 1e-14


def test_ch_square_droplet_fp32_eight_row_tiles():
    case, phi0 = W.square_droplet_ch(n=1024, R=256.0, sigma=1e-3, rho_ratio=100.0, dtype="f32")
    g, o = _pair(case, phi0, 150)
    _compare(g, o, 1e-5, 1e-4, "CH square droplet 1024^2 fp32")


def test_ch_graph_replay_equals_eager():
    """lbm_step on a side stream replays captured graphs of 32 CH steps; the state
    equals that of eager launches bitwise."""
    case, phi0 = W.square_droplet_ch(n=96, R=24.0, sigma=1e-3, rho_ratio=100.0, dtype="f32")
    a = _sim()(case).init(phi0).step(101)
    b = _sim()(case, stream=torch.cuda.Stream()).init(phi0)
    b.step(70)
    b.step(31)
    torch.cuda.synchronize()
    sa, sb = a.export_state(), b.export_state()
    assert sa["step"] == sb["step"] == 101
    for key in ("f", "g", "hist"):
        assert torch.equal(sa[key], sb[key]), key


# ---------------------------------------------------------------- corrected model, Allen-Cahn phase field
def _ac_case(geom, nx, ny, **kw):
    base = dict(nx=nx, ny=ny, rhoA=20.0, rhoB=1.0, nuA=0.05, nuB=0.2, sigma=0.05, W=4.0, M=0.2,
                body_force=(1e-6, -2e-6), gravity=(3e-6, -1e-5), rho_ref=3.0, dtype="f64", model="corrected")
    return W.Case(**{**base, **GEOMS[geom], **kw})


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("shape", [(37, 23), (1000, 530)])
def test_corrected_allen_cahn_one_step_map_fp64(geom, shape):
    """Corrected model with the AC phase field (F_a from div D, D = grad phi -
    lambda n) against the oracle: 4-row and 8-row tiles, ragged, four boundary kinds."""
    case = _ac_case(geom, *shape)
    phi0, u0, p0 = W.random_state_fields(case, seed=31)
    st = oracle.OracleSim(case).init(phi0, u0, p0).get_state()
    rng = np.random.default_rng(32)
    f = st["f"] + 1e-4 * rng.standard_normal(st["f"].shape)
    g = st["g"] + 1e-5 * rng.standard_normal(st["g"].shape)
    php = phi0 + 1e-3 * rng.standard_normal(phi0.shape)
    upr = u0 + 1e-4 * rng.standard_normal(u0.shape)
    hist = np.concatenate([php[None], upr], 0)
    gs = _sim()(case).import_state(f, g, hist, 2).step(1)
    o = oracle.OracleSim(case).set_state(f, g, 2, php, upr).step(1)
    so, sg = o.get_state(), gs.export_state()
    df = np.abs(sg["f"].cpu().numpy() - so["f"]).max()
    dg = np.abs(sg["g"].cpu().numpy() - so["g"]).max()
    print(f"AC corrected {geom} {shape}: max|df|={df:.2e} max|dg|={dg:.2e}", flush=True)
    # div D differentiates the regularised normal once more; where |grad phi| is
    # near eps_n it amplifies the rounding of the two sides (measured 1.6e-14 on
    # 1000 x 530 random fields, 4e-16 on 37 x 23)
    assert df < 1e-13 and dg < 1e-13


def test_corrected_allen_cahn_dam_break_fp64_and_diagnostics():
    case, phi0 = W.dam_break(nx=64, ny=32, column=16, dtype="f64", theta_deg=70.0)
    case = case.replace(model="corrected")
    p0 = "hydrostatic"
    g = _sim()(case).init(phi0, None, p0).step(600)
    o = oracle.OracleSim(case).init(phi0, None, p0).step(600)
    _compare(g, o, 1e-10, 1e-9, "AC corrected dam break 64x32 fp64")
    dg, do = g.diagnostics(), o.diagnostics()
    for key in ("sum_phi", "max_div", "Du_rms", "Sm_rms", "umax"):
        assert abs(dg[key] - do[key]) <= 1e-8 * abs(do[key]) + 1e-16, (key, dg[key], do[key])


def test_corrected_allen_cahn_dam_break_fp32():
    case, phi0 = W.dam_break(nx=64, ny=32, column=16, dtype="f32", theta_deg=70.0)
    case = case.replace(model="corrected")
    p0 = "hydrostatic"
    g = _sim()(case).init(phi0, None, p0).step(600)
    o = oracle.OracleSim(case.replace(dtype="f64")).init(phi0, None, p0).step(600)
    _compare(g, o, 1e-5, 1e-4, "AC corrected dam break 64x32 fp32")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ch_rayleigh_taylor(dtype):
    """Sec. 4.4 runs the RTI with the Cahn-Hilliard phase field (phi in [-1, 1]):
    the 64 x 256 copy of the set-up (walls in y, gravity, hydrostatic start),
    1000 steps, against the oracle."""
    case, phi01 = W.rti(nx=64, ny=256, dtype=dtype)
    case, phi0 = W.to_cahn_hilliard(case, phi01)
    p0 = "hydrostatic"
    g = _sim()(case).init(phi0, None, p0).step(1000)
    o = oracle.OracleSim(case.replace(dtype="f64")).init(phi0, None, p0).step(1000)
    if dtype == "f64":
        _compare(g, o, 1e-10, 1e-9, "CH RTI 64x256 fp64")
    else:
        _compare(g, o, 1e-5, 1e-4, "CH RTI 64x256 fp32")
