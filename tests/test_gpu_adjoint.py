"""The hand-written adjoint (lbm_adjoint_step and the autograd Function) against
the differentiable CPU reference (oracle/torch_ref.py) and against central
finite differences of the GPU forward.

FP64 throughout, except the last test: one adjoint step equals the autograd
vector-Jacobian product of one reference step element by element (1e-11 of
the largest entry); whole-trajectory gradients equal the reference's to 1e-9
relative; on the 64 x 32 copy of the dam break the gradients equal central
finite differences to 1e-4 relative.
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
    "walls_x": dict(wall_x=True, theta=(math.radians(60), math.radians(130), math.pi / 2, math.pi / 2)),
    "walls_y": dict(wall_y=True, theta=(math.pi / 2, math.pi / 2, math.radians(50), math.radians(120))),
    "walls_xy": dict(wall_x=True, wall_y=True,
                     theta=(math.radians(70), math.radians(110), math.radians(40), math.radians(140))),
}


def _case(geom, nx=37, ny=23, **kw):
    base = dict(nx=nx, ny=ny, rhoA=20.0, rhoB=1.0, nuA=0.05, nuB=0.2, sigma=0.01, W=4.0, M=0.05,
                body_force=(1e-6, -2e-6), gravity=(3e-6, -1e-5), rho_ref=3.0, dtype="f64")
    return W.Case(**{**base, **GEOMS[geom], **kw})


def _random_state(case, seed):
    phi0, u0, p0 = W.random_state_fields(case, seed=seed)
    st = oracle.OracleSim(case).init(phi0, u0, p0).get_state()
    rng = np.random.default_rng(seed + 1)
    f = st["f"] + 1e-4 * rng.standard_normal(st["f"].shape)
    g = st["g"] + 1e-5 * rng.standard_normal(st["g"].shape)
    php = phi0 + 1e-3 * rng.standard_normal(phi0.shape)
    upr = u0 + 1e-4 * rng.standard_normal(u0.shape)
    return f, g, php, upr


def _api():
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.sim import Sim
    return api, Sim


def _close(a, b, tol, what):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    print(f"{what}: rel err {err:.2e} (scale {scale:.3e})", flush=True)
    assert err <= tol, (what, err)


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("n", [0, 5])
@pytest.mark.parametrize("visc", ["linear_mu", "inverse_nu"])
def test_one_adjoint_step_equals_reference_vjp(geom, n, visc):
    from oracle.torch_ref import TorchRef, as_params
    api, Sim = _api()
    case = _case(geom, visc_law=visc)
    f, g, php, upr = _random_state(case, seed=3 + n)
    hist = np.concatenate([php[None], upr], 0)
    s = Sim(case).import_state(f, g, hist if n > 0 else None, n)
    p = s.p
    tape = api.new_tape(p, 1)
    api.lbm_tape_record(p, s.state, tape, 1)
    rng = np.random.default_rng(100 + n)
    fb1 = rng.standard_normal((9, case.ny, case.nx))
    gb1 = rng.standard_normal((9, case.ny, case.nx))
    hb1 = rng.standard_normal((3, case.ny, case.nx))
    cuda = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    adj = api.new_adjoint(p)
    api.lbm_adjoint_import(p, adj, cuda(fb1), cuda(gb1), cuda(hb1), n + 1)
    api.lbm_adjoint_step(p, tape, 0, adj)
    fb0 = torch.empty((9, case.ny, case.nx), dtype=torch.float64, device="cuda")
    gb0 = torch.empty_like(fb0)
    hb0 = torch.empty((3, case.ny, case.nx), dtype=torch.float64, device="cuda")
    api.lbm_adjoint_export(p, adj, fb0, gb0, hb0)
    prm, level = api.lbm_adjoint_params(p, adj)
    assert level == n

    ref = TorchRef(case)
    grav, theta = as_params(case)
    st = dict(f=torch.tensor(f, requires_grad=True), g=torch.tensor(g, requires_grad=True),
              phi_prev=torch.tensor(php, requires_grad=True), u_prev=torch.tensor(upr, requires_grad=True), n=n)
    out = ref.step(st, grav, theta)
    J = (out["f"] * torch.tensor(fb1)).sum() + (out["g"] * torch.tensor(gb1)).sum() \
        + (out["phi_prev"] * torch.tensor(hb1[0])).sum() + (out["u_prev"] * torch.tensor(hb1[1:])).sum()
    J.backward()
    tag = f"{geom} n={n} {visc}"
    _close(fb0.cpu().numpy(), st["f"].grad.numpy(), 1e-11, tag + " fbar")
    _close(gb0.cpu().numpy(), st["g"].grad.numpy(), 1e-11, tag + " gbar")
    if n > 0:
        _close(hb0[0].cpu().numpy(), st["phi_prev"].grad.numpy(), 1e-11, tag + " phi_prev bar")
        _close(hb0[1:].cpu().numpy(), st["u_prev"].grad.numpy(), 1e-11, tag + " u_prev bar")
    else:
        assert float(hb0.abs().max()) == 0.0
    _close(prm[0:2], grav.grad.numpy(), 1e-10, tag + " dgravity")
    if geom != "periodic":
        _close(prm[2:6], theta.grad.numpy(), 1e-10, tag + " dtheta")
    else:
        assert max(abs(v) for v in prm[2:6]) == 0.0


def _traj_case(kind):
    if kind == "walls_xy_inverse_nu":
        case = _case("walls_xy", nx=24, ny=14, visc_law="inverse_nu", gravity=(0.0, -2e-4))
        phi0, _, _ = W.random_state_fields(case, seed=4)
    else:
        case, phi0 = W.dam_break(nx=32, ny=16, column=8, dtype="f64", theta_deg=75.0, g=5e-5)
        case = case.replace(theta=tuple(math.radians(t) for t in (75.0, 82.0, 68.0, 101.0)))
    rng = np.random.default_rng(5)
    target = np.clip(phi0 + 0.05 * rng.standard_normal(phi0.shape), 0, 1)
    return case, phi0, target


@pytest.mark.parametrize("kind", ["walls_xy_inverse_nu", "dam_break_32x16"])
def test_trajectory_gradient_equals_reference(kind):
    from oracle.torch_ref import loss_and_grads
    from paper_2111_00847_amd.autograd import trajectory_phi
    case, phi0, target = _traj_case(kind)
    nsteps, chk = 25, 7
    L_ref, dphi_ref, dg_ref, dth_ref = loss_and_grads(case, phi0, target, nsteps, None)
    phi0_t = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
    grav = torch.tensor(list(case.gravity), dtype=torch.float64, requires_grad=True)
    theta = torch.tensor(list(case.theta), dtype=torch.float64, requires_grad=True)
    phiN = trajectory_phi(phi0_t, grav, theta, case, nsteps, None, chk)
    L = ((phiN - torch.tensor(target, device="cuda")) ** 2).sum()
    L.backward()
    assert abs(float(L) - L_ref) <= 1e-12 * L_ref
    _close(phi0_t.grad.cpu().numpy(), dphi_ref, 1e-9, f"{kind} dL/dphi0")
    _close(grav.grad.numpy(), dg_ref, 1e-9, f"{kind} dL/dgravity")
    _close(theta.grad.numpy(), dth_ref, 1e-9, f"{kind} dL/dtheta")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["walls_xy_inverse_nu", "dam_break_32x16"])
def test_two_level_tape_equals_one_level_tape(kind, dtype):
    """Tapes recorded two levels per launch (LBM_TWO_LEVEL=1: the two-level body
    stores its intermediate level too) hold the forward levels bitwise, so the
    gradients equal those from one-level tapes (LBM_TWO_LEVEL=0) bit for bit;
    segments of 7 levels end on a one-level launch."""
    import os
    from paper_2111_00847_amd.autograd import trajectory_phi
    case, phi0, target = _traj_case(kind)
    case = case.replace(dtype=dtype)
    nsteps, chk = 25, 7
    out = {}
    for mode in ("1", "0"):
        os.environ["LBM_TWO_LEVEL"] = mode
        try:
            phi0_t = torch.tensor(phi0, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda",
                                  requires_grad=True)
            grav = torch.tensor(list(case.gravity), dtype=torch.float64, requires_grad=True)
            theta = torch.tensor(list(case.theta), dtype=torch.float64, requires_grad=True)
            phiN = trajectory_phi(phi0_t, grav, theta, case, nsteps, None, chk)
            L = ((phiN - torch.tensor(target, dtype=phiN.dtype, device="cuda")) ** 2).sum()
            L.backward()
            torch.cuda.synchronize()
            out[mode] = (phi0_t.grad.cpu().numpy(), grav.grad.numpy(), theta.grad.numpy())
        finally:
            os.environ.pop("LBM_TWO_LEVEL", None)
    for a, b, what in zip(out["1"], out["0"], ("dL/dphi0", "dL/dgravity", "dL/dtheta")):
        assert np.array_equal(a, b), (kind, dtype, what, float(np.abs(a - b).max()))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["walls_xy_inverse_nu", "dam_break_32x16"])
def test_full_tape_equals_checkpointed(kind, dtype):
    """chk = 0 records every forward level on one tape and ends the forward on
    its last slot: phi^N and the gradients equal those of checkpoints every 7
    levels (segments recomputed in backward) bit for bit; 25 levels, so the
    two-level tape launches end on a one-level one."""
    from paper_2111_00847_amd.autograd import trajectory_phi
    case, phi0, target = _traj_case(kind)
    case = case.replace(dtype=dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    nsteps = 25
    out = {}
    for chk in (0, 7):
        phi0_t = torch.tensor(phi0, dtype=tdt, device="cuda", requires_grad=True)
        grav = torch.tensor(list(case.gravity), dtype=torch.float64, requires_grad=True)
        theta = torch.tensor(list(case.theta), dtype=torch.float64, requires_grad=True)
        phiN = trajectory_phi(phi0_t, grav, theta, case, nsteps, None, chk)
        L = ((phiN - torch.tensor(target, dtype=tdt, device="cuda")) ** 2).sum()
        L.backward()
        torch.cuda.synchronize()
        out[chk] = (phiN.detach().cpu().numpy(), phi0_t.grad.cpu().numpy(), grav.grad.numpy(), theta.grad.numpy())
    for a, b, what in zip(out[0], out[7], ("phi^N", "dL/dphi0", "dL/dgravity", "dL/dtheta")):
        assert np.array_equal(a, b), (kind, dtype, what, float(np.abs(a - b).max()))


@pytest.mark.parametrize("nsteps", [0, 1, 2])
def test_full_tape_short_trajectories(nsteps):
    """Zero, one and two levels with the full tape (tapes of 1, 2, 3 slots)
    against checkpoints every level: phi^N and gradients bit for bit; at zero
    levels phi^N is phi0 and dL/dphi0 = 2 (phi0 - target) to rounding."""
    from paper_2111_00847_amd.autograd import trajectory_phi
    case, phi0, target = _traj_case("dam_break_32x16")
    out = {}
    for chk in (0, 1):
        phi0_t = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
        grav = torch.tensor(list(case.gravity), dtype=torch.float64, requires_grad=True)
        theta = torch.tensor(list(case.theta), dtype=torch.float64, requires_grad=True)
        phiN = trajectory_phi(phi0_t, grav, theta, case, nsteps, None, chk)
        L = ((phiN - torch.tensor(target, device="cuda")) ** 2).sum()
        L.backward()
        torch.cuda.synchronize()
        out[chk] = (phiN.detach().cpu().numpy(), phi0_t.grad.cpu().numpy(), grav.grad.numpy(), theta.grad.numpy())
    for a, b, what in zip(out[0], out[1], ("phi^N", "dL/dphi0", "dL/dgravity", "dL/dtheta")):
        assert np.array_equal(a, b), (nsteps, what, float(np.abs(a - b).max()))
    if nsteps == 0:
        assert np.abs(out[0][0] - phi0).max() <= 1e-14
        assert np.abs(out[0][1] - 2.0 * (phi0 - target)).max() <= 1e-13
        assert not out[0][2].any() and not out[0][3].any()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tape_restore_resumes_the_trajectory(dtype):
    """lbm_tape_restore makes a tape slot the current level of a state: slot 3
    of a tape recorded from level 2 is level 5 exactly (populations, history,
    step), and the restored state steps on as the original does, bit for bit.
    A slot the tape does not hold is LBM_E_SIZE, a tape of another lattice
    LBM_E_PARAM (both from the host, before any copy)."""
    from paper_2111_00847_amd._lib import LbmError
    api, Sim = _api()
    case = _case("walls_xy").replace(dtype=dtype)
    phi0, u0, p0 = W.random_state_fields(case, seed=21)
    ref = Sim(case).init(phi0, u0, p0).step(2)
    tape = api.new_tape(ref.p, 4)
    api.lbm_tape_record(ref.p, ref.state, tape, 4)        # levels 2 .. 5
    ref.step(3)
    other = Sim(case).init(phi0)
    api.lbm_tape_restore(other.p, tape, 3, other.state)
    for k in range(2):
        a, b = other.export_state(), ref.export_state()
        assert a["step"] == b["step"] == 5 + 3 * k
        for key in ("f", "g", "hist"):
            assert torch.equal(a[key], b[key]), (dtype, k, key)
        other.step(3)
        ref.step(3)
    with pytest.raises(LbmError) as e:
        api.lbm_tape_restore(other.p, tape, 4, other.state)
    assert e.value.code == -2
    taller = Sim(case.replace(ny=case.ny + 1)).init(np.vstack([phi0, phi0[-1:]]))
    with pytest.raises(LbmError) as e:
        api.lbm_tape_restore(taller.p, tape, 0, taller.state)
    assert e.value.code == -4


# ---------------------------------------------------------------- cfg: differentiable dam break, 64 x 32 copy
def _dam_small(dtype="f64"):
    """64 x 32 copy of the dam break; the target is phi of a run with seeded
    perturbed parameters: g (1 + 0.1 xi), theta ~ U[60, 120] degrees."""
    case, phi0 = W.dam_break(nx=64, ny=32, column=16, dtype=dtype, theta_deg=90.0, g=1e-6)
    rng = np.random.default_rng(W.SEED)
    g_t = 1e-6 * (1.0 + 0.1 * rng.standard_normal())
    th_t = math.radians(rng.uniform(60.0, 120.0))
    return case, phi0, case.replace(gravity=(0.0, -g_t), theta=(th_t,) * 4)


def _gpu_phi(case, phi0, nsteps):
    _, Sim = _api()
    phi, _, _ = Sim(case).init(phi0).step(nsteps).moments_np()
    return phi


@pytest.mark.parametrize("nsteps", [1000, 4000])
def test_dam_break_64x32_gradients_equal_finite_differences(nsteps):
    """dL/dg (gravity (0, -g)), dL/dtheta (one angle on all walls) and eight
    seeded directional derivatives in phi0, adjoint vs central differences of
    the FP64 GPU forward, checkpoints every 200 (4000 steps: the horizon of the
    differentiable dam break)."""
    from paper_2111_00847_amd.autograd import trajectory_phi
    case, phi0, tcase = _dam_small()
    target = _gpu_phi(tcase, phi0, nsteps)
    loss = lambda c, ph: float(np.sum((_gpu_phi(c, ph, nsteps) - target) ** 2))

    phi0_t = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
    gs = torch.tensor(1e-6, dtype=torch.float64, requires_grad=True)
    th = torch.tensor(math.pi / 2, dtype=torch.float64, requires_grad=True)
    grav = torch.stack([torch.zeros((), dtype=torch.float64), -gs])
    theta = th.expand(4)
    phiN = trajectory_phi(phi0_t, grav, theta, case, nsteps, None, 200)
    L = ((phiN - torch.tensor(target, device="cuda")) ** 2).sum()
    L.backward()
    checks = []
    h = 1e-9
    checks.append(((loss(case.replace(gravity=(0.0, -(1e-6 + h))), phi0)
                    - loss(case.replace(gravity=(0.0, -(1e-6 - h))), phi0)) / (2 * h), float(gs.grad), "dL/dg"))
    h = 1e-5
    checks.append(((loss(case.replace(theta=(math.pi / 2 + h,) * 4), phi0)
                    - loss(case.replace(theta=(math.pi / 2 - h,) * 4), phi0)) / (2 * h), float(th.grad), "dL/dtheta"))
    rng = np.random.default_rng(W.SEED + 1)
    gphi = phi0_t.grad.cpu().numpy()
    for k in range(8):
        d = rng.standard_normal(phi0.shape)
        h = 1e-6
        checks.append(((loss(case, phi0 + h * d) - loss(case, phi0 - h * d)) / (2 * h), float(np.sum(gphi * d)),
                       f"dL/dphi0 . d{k}"))
    for fd, ad, what in checks:
        print(f"{nsteps} steps {what}: fd={fd:.8e} adjoint={ad:.8e}", flush=True)
    for fd, ad, what in checks:
        assert abs(fd - ad) <= 1e-4 * abs(ad), (what, fd, ad)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("geom", ["periodic", "walls_xy", "walls_y"])
def test_adjoint_run_equals_single_steps(geom, dtype):
    """Two lbm_adjoint_run calls in a row over one tape equal that many
    lbm_adjoint_step calls bit for bit: adjoint populations, history adjoint,
    parameter sums and dL/dphi0 (ragged tiles, 37 x 23)."""
    api, Sim = _api()
    case = _case(geom).replace(dtype=dtype)
    phi0, u0, p0 = W.random_state_fields(case, seed=11)
    s = Sim(case).init(phi0, u0, p0)
    nl = 9
    tape = api.new_tape(s.p, nl)
    api.lbm_tape_record(s.p, s.state, tape, nl)
    s.step(nl - 1)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(3)
    dL = torch.tensor(rng.standard_normal((case.ny, case.nx)), dtype=tdt, device="cuda")
    out = []
    for mode in ("run", "steps"):
        adj = api.new_adjoint(s.p)
        api.lbm_adjoint_phi(s.p, s.state, adj, dL)
        if mode == "run":                                  # the adjoint of level 8 down to level 0
            api.lbm_adjoint_run(s.p, tape, nl - 2, 5, adj)     # slots 7 .. 3
            api.lbm_adjoint_run(s.p, tape, nl - 7, nl - 6, adj)  # slots 2 .. 0
        else:
            for j in range(nl - 2, -1, -1):
                api.lbm_adjoint_step(s.p, tape, j, adj)
        fb = torch.empty((9, case.ny, case.nx), dtype=tdt, device="cuda")
        gb = torch.empty_like(fb)
        hb = torch.empty((3, case.ny, case.nx), dtype=tdt, device="cuda")
        api.lbm_adjoint_export(s.p, adj, fb, gb, hb)
        d0 = torch.empty((case.ny, case.nx), dtype=tdt, device="cuda")
        api.lbm_adjoint_init(s.p, adj, d0)
        prm, lev = api.lbm_adjoint_params(s.p, adj)
        assert lev == 0
        out.append([t.cpu().numpy() for t in (fb, gb, hb, d0)] + [np.array(prm)])
    for a, b, what in zip(out[0], out[1], ("fbar", "gbar", "hbar", "dL/dphi0", "params")):
        assert np.array_equal(a, b), (geom, dtype, what, float(np.abs(a - b).max()))


def test_level_mismatch_is_reported():
    """An adjoint step whose tape level is not one below the adjoint's level is
    skipped on the device and reported by lbm_adjoint_params."""
    api, Sim = _api()
    case, phi0, _ = _dam_small()
    s = Sim(case).init(phi0).step(3)
    tape = api.new_tape(s.p, 2)
    api.lbm_tape_record(s.p, s.state, tape, 2)            # levels 3, 4
    adj = api.new_adjoint(s.p)
    z = torch.zeros((case.ny, case.nx), dtype=torch.float64, device="cuda")
    api.lbm_adjoint_phi(s.p, s.state, adj, z)             # adjoint at level 3
    api.lbm_adjoint_step(s.p, tape, 1, adj)               # would need level 5
    from paper_2111_00847_amd._lib import LbmError
    with pytest.raises(LbmError):
        api.lbm_adjoint_params(s.p, adj)


def test_tape_slot_and_lattice_are_checked_on_the_device():
    """An adjoint step on a slot the tape does not hold (j = 3 of a 3-level
    tape, with the adjoint at the level that slot would pair with), or on a
    tape recorded for another lattice, reads nothing of the tape beyond its
    header and is reported by lbm_adjoint_params as LBM_E_PARAM."""
    from paper_2111_00847_amd._lib import LbmError
    api, Sim = _api()
    case, phi0, _ = _dam_small()
    s = Sim(case).init(phi0).step(2)
    tape = api.new_tape(s.p, 3)
    api.lbm_tape_record(s.p, s.state, tape, 3)            # levels 2, 3, 4
    s.step(4)                                             # level 6 = 2 + 3 + 1
    adj = api.new_adjoint(s.p)
    z = torch.zeros((case.ny, case.nx), dtype=torch.float64, device="cuda")
    api.lbm_adjoint_phi(s.p, s.state, adj, z)
    api.lbm_adjoint_step(s.p, tape, 3, adj)
    with pytest.raises(LbmError) as e:
        api.lbm_adjoint_params(s.p, adj)
    assert e.value.code == -4
    # a tape of this lattice used with the parameters of a taller one
    other, phi1, _ = _dam_small()
    other = other.replace(ny=other.ny + 1)
    s1 = Sim(other).init(np.vstack([phi1, phi1[-1:]])).step(3)   # the level slot 0 pairs with
    adj1 = api.new_adjoint(s1.p)
    api.lbm_adjoint_phi(s1.p, s1.state, adj1, torch.zeros((other.ny, other.nx), dtype=torch.float64, device="cuda"))
    api.lbm_adjoint_step(s1.p, tape, 0, adj1)
    with pytest.raises(LbmError) as e:
        api.lbm_adjoint_params(s1.p, adj1)
    assert e.value.code == -4


def test_fp32_adjoint_tracks_fp64():
    """The FP32 adjoint of the 64 x 32 dam break (200 steps) agrees with the FP64
    adjoint to 1e-3 relative in every gradient."""
    from paper_2111_00847_amd.autograd import trajectory_phi
    res = {}
    for dt in ("f64", "f32"):
        case, phi0, tcase = _dam_small(dt)
        target = _gpu_phi(tcase.replace(dtype="f64"), phi0, 200)
        tdt = torch.float64 if dt == "f64" else torch.float32
        phi0_t = torch.tensor(phi0, dtype=tdt, device="cuda", requires_grad=True)
        grav = torch.tensor([0.0, -1e-6], dtype=torch.float64, requires_grad=True)
        theta = torch.tensor([math.radians(80.0)] * 4, dtype=torch.float64, requires_grad=True)
        phiN = trajectory_phi(phi0_t, grav, theta, case, 200, None, 64)
        L = ((phiN.double() - torch.tensor(target, device="cuda")) ** 2).sum()
        L.backward()
        res[dt] = (phi0_t.grad.double().cpu().numpy(), grav.grad.numpy(), theta.grad.numpy())
    for k, name in enumerate(("dL/dphi0", "dL/dgravity", "dL/dtheta")):
        _close(res["f32"][k], res["f64"][k], 1e-3, f"fp32 vs fp64 {name}")


def test_contact_angle_recovered_by_gradient_descent():
    """An inverse problem through the autograd function: the bottom-wall contact
    angle of a spreading droplet (Sec. 4.3 set-up, 96 x 48, density ratio 10,
    FP64, 1500 steps) is recovered from the target shape phi_T (made at 70 deg)
    by secant iterations on dL/dtheta, L = sum (phi - phi_T)^2, from 90 deg."""
    from paper_2111_00847_amd.autograd import trajectory_phi
    case, phi0 = W.spreading_case(96, 48, 70.0, dtype="f64", R0=16.0, rho_ratio=10.0, mu_ratio=10.0,
                                  sigma=5e-3, W=4.0, M=0.1)
    dev = "cuda:0"
    phi0_t = torch.tensor(phi0, dtype=torch.float64, device=dev)
    grav = torch.zeros(2, dtype=torch.float64)
    base = torch.tensor(case.theta, dtype=torch.float64)
    target = trajectory_phi(phi0_t, grav, base, case, 1500, chk=300).detach()

    def loss_grad(theta_bottom):
        th = base.clone()
        th[2] = theta_bottom
        th.requires_grad_(True)
        phi = trajectory_phi(phi0_t, grav, th, case, 1500, chk=300)
        loss = ((phi - target) ** 2).sum()
        loss.backward()
        return float(loss), float(th.grad[2])

    t_prev, t = math.radians(90.0), math.radians(85.0)
    _, g_prev = loss_grad(t_prev)
    for it in range(8):
        L, g = loss_grad(t)
        print(f"iteration {it}: theta {math.degrees(t):.4f} deg, L {L:.3e}, dL/dtheta {g:.3e}", flush=True)
        if abs(math.degrees(t) - 70.0) < 1e-3:
            break
        t_prev, t, g_prev = t, t - g * (t - t_prev) / (g - g_prev), g
    assert abs(math.degrees(t) - 70.0) < 0.01, math.degrees(t)
