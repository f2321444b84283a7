"""Large lattices against tiled small ones.  A periodic lattice made of copies
of a small one must stay those copies bitwise, so a code path that only large
states take is held to the small lattice's path, which the oracle checks:
state copies beyond 4 GiB (the plain step's 64-bit offsets, 32-bit below), and
states beyond the last-level cache (non-temporal stores, early g loads) against
cached ones (ordinary stores; late g loads in the plain step)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

STEPS = 40


@pytest.mark.parametrize("dtype,k", [("f32", 200), ("f64", 100)])
def test_lattice_beyond_4gib_per_copy_is_the_tiled_small_lattice(dtype, k):
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.sim import Sim
    case_s, phi_s = W.rti(nx=256, ny=1024, dtype=dtype)
    p_s = Sim(case_s).hydrostatic_pressure(phi_s).cpu().numpy()
    case_b = case_s.replace(nx=256 * k, name=f"rti_tiled_{256 * k}x1024")
    nbytes = api.lbm_state_size(api.make_params(case_b))
    assert nbytes > 2 * (1 << 32), nbytes          # two copies of more than 4 GiB each
    print(f"{dtype}: {case_b.nx} x {case_b.ny}, state {nbytes / 2**30:.2f} GiB", flush=True)

    small = Sim(case_s).init(phi_s, None, p_s).step(STEPS)
    big = Sim(case_b).init(np.tile(phi_s, (1, k)), None, np.tile(p_s, (1, k))).step(STEPS)
    torch.cuda.synchronize()

    ps, us, prs = small.moments()
    pb, ub, prb = big.moments()
    ny = case_s.ny
    for name, a, b in (("phi", ps, pb), ("u", us[0], ub[0]), ("v", us[1], ub[1]), ("p", prs, prb)):
        tiled = a.unsqueeze(1).expand(ny, k, 256)
        d = (b.view(ny, k, 256) - tiled).abs().max().item()
        print(f"{dtype} {name}: max |big - tiled small| = {d:.3e}", flush=True)
        assert torch.equal(b.view(ny, k, 256), tiled), name

    ds, db = small.diagnostics(), big.diagnostics()
    assert db["nonfinite"] == 0
    assert abs(db["sum_phi"] - k * ds["sum_phi"]) <= 1e-12 * k * ds["sum_phi"]
    assert db["umax"] == ds["umax"]
    del big
    torch.cuda.empty_cache()

    # the small run against the oracle
    o = oracle.OracleSim(case_s.replace(dtype="f64")).init(phi_s, None, p_s).step(STEPS)
    phi_o, u_o, _ = o.moments()
    phi_g, u_g, _ = small.moments_np()
    dphi = np.abs(phi_g - phi_o).max()
    du = np.abs(u_g - u_o).max() / np.abs(u_o).max()
    print(f"{dtype} 256 x 1024 vs oracle after {STEPS} steps: max|dphi|={dphi:.2e} max|du|/Umax={du:.2e}",
          flush=True)
    if dtype == "f64":
        assert dphi <= 1e-12 and du <= 1e-10
    else:
        assert dphi <= 1e-5 and du <= 1e-4


def _tiled_pair(small_case, phi_s, p_s, kx, ky):
    big = small_case.replace(nx=small_case.nx * kx, ny=small_case.ny * ky, name=small_case.name + "_tiled")
    tile = lambda a: None if a is None else np.tile(a, (ky, kx))
    return big, tile(phi_s), tile(p_s)


@pytest.mark.parametrize("variant,dtype", [("plain", "f32"), ("plain", "f64"), ("cahn_hilliard", "f32"),
                                           ("local_gradient", "f32")])
def test_streamed_state_path_is_the_tiled_cached_one(variant, dtype):
    """Lattices whose state exceeds the last-level cache take the non-temporal
    store path with early g loads; small ones keep their state in the cache
    (ordinary stores, and for the plain step g loaded late).  A periodic
    lattice of copies of a small one (same tile shapes) must stay those copies
    bitwise: 30 steps, phi, u and p compared."""
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.sim import Sim
    if variant == "cahn_hilliard":
        case_s, phi_s = W.square_droplet_ch(n=512, R=128.0, sigma=1e-3, rho_ratio=100.0, dtype=dtype)
        case_s, phi_s = case_s.replace(nx=1024, ny=512), np.tile(phi_s, (1, 2))
        p_s, kx, ky = None, 2, 2
    else:
        case_s, phi_s = W.rti(nx=256, ny=1024, dtype=dtype)
        if variant == "local_gradient":
            case_s = case_s.replace(grad_scheme="local")
        p_s, kx, ky = Sim(case_s).hydrostatic_pressure(phi_s).cpu().numpy(), 8, 1
    case_b, phi_b, p_b = _tiled_pair(case_s, phi_s, p_s, kx, ky)
    nb = api.lbm_state_size(api.make_params(case_b))
    ns = api.lbm_state_size(api.make_params(case_s))
    assert ns < (192 << 20) and (340 << 20) < nb < (8 << 30), (ns, nb)   # small: cached; big: streamed
    small = Sim(case_s).init(phi_s, None, p_s).step(30)
    big = Sim(case_b).init(phi_b, None, p_b).step(30)
    torch.cuda.synchronize()
    for name, a, b in zip(("phi", "u", "p"), small.moments(), big.moments()):
        ny, nx = a.shape[-2:]
        lead = a.shape[:-2]
        tiled = a.reshape(lead + (1, ny, 1, nx)).expand(lead + (ky, ny, kx, nx)).reshape(b.shape)
        d = (b - tiled).abs().max().item()
        print(f"{variant} {dtype} {name}: max |big - tiled small| = {d:.3e}", flush=True)
        assert torch.equal(b, tiled), (variant, dtype, name)


def test_reverse_mode_on_a_streamed_state_is_the_tiled_cached_one():
    """The reverse mode's tape recompute stores a level non-temporally when a
    level and the next exceed the last-level cache, with ordinary stores
    otherwise.  On a periodic lattice of 8 copies of the 256 x 1024 RTI field
    (tape levels of 185 MB, streamed) the gradient in phi0 is the tiled gradient
    of the small lattice (cached tape) bitwise, and the gradients in gravity and
    the contact angles are 8 times the small ones (FP64 sums in another order)."""
    import math
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.autograd import trajectory_phi
    case_s, phi_s = W.rti(nx=256, ny=1024, dtype="f32")
    case_b, phi_b, _ = _tiled_pair(case_s, phi_s, None, 8, 1)
    ps, pb = api.make_params(case_s), api.make_params(case_b)
    slot_s = api.lbm_state_size(ps) / 2
    slot_b = api.lbm_state_size(pb) / 2
    assert 2 * slot_s < (320 << 20) < 2 * slot_b, (slot_s, slot_b)
    X, Y = W.grid(case_s)
    w_s = np.cos(2 * np.pi * X / 256.0) * np.exp(-((Y - 512.0) / 40.0) ** 2)
    res = {}
    for name, case, phi0, w in (("small", case_s, phi_s, w_s), ("big", case_b, phi_b, np.tile(w_s, (1, 8)))):
        phi0_t = torch.tensor(phi0, dtype=torch.float32, device="cuda", requires_grad=True)
        grav = torch.tensor(list(case.gravity), dtype=torch.float64, requires_grad=True)
        theta = torch.tensor([math.pi / 2] * 4, dtype=torch.float64, requires_grad=True)
        phiN = trajectory_phi(phi0_t, grav, theta, case, 8, None, 4)
        L = (phiN.double() * torch.tensor(w, device="cuda")).sum()
        L.backward()
        res[name] = (phi0_t.grad.detach().clone(), grav.grad.numpy().copy(), theta.grad.numpy().copy())
    gs, gb = res["small"][0], res["big"][0]
    tiled = gs.unsqueeze(1).expand(1024, 8, 256).reshape(1024, 2048)
    print(f"dL/dphi0: max |big - tiled small| = {(gb - tiled).abs().max().item():.3e}", flush=True)
    assert torch.equal(gb, tiled)
    for k, what in ((1, "gravity"), (2, "theta")):
        a, b = res["small"][k], res["big"][k]
        print(f"dL/d{what}: small {a}, big {b}", flush=True)
        # a component that cancels to 1e-9 of the other (dL/dgravity_x) is held to
        # the vector's size: its FP64 sums run in another order over 8x the nodes
        np.testing.assert_allclose(b, 8 * a, rtol=1e-10, atol=1e-12 * np.abs(8 * a).max())


@pytest.mark.parametrize("mix", ["plain", "with_cahn_hilliard"])
def test_streamed_batch_equals_lone_runs(mix):
    """A batch whose state exceeds the last-level cache stores it non-temporally
    (the smaller batches of the other tests keep theirs in the cache): four
    1024 x 512 FP32 lattices (dam breaks at four contact angles, or three and a
    Cahn-Hilliard droplet), 20 steps, each equal to the lattice advanced alone --
    the Allen-Cahn cases bitwise, the Cahn-Hilliard one within 16 ulp."""
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.sim import BatchSim, Sim
    cases = [W.dam_break(nx=1024, ny=512, theta_deg=th) for th in (50.0, 80.0, 110.0, 140.0)]
    if mix == "with_cahn_hilliard":
        case, phi0 = W.square_droplet_ch(n=512, R=128.0, sigma=1e-3, rho_ratio=100.0, dtype="f32")
        cases[3] = (case.replace(nx=1024, ny=512), np.tile(phi0, (1, 2)))
    total = sum(api.lbm_state_size(api.make_params(c)) for c, _ in cases)
    assert total > (340 << 20), total
    p0s = ["hydrostatic" if any(c.gravity) else None for c, _ in cases]
    B = BatchSim([c for c, _ in cases], stream=torch.cuda.Stream())
    B.init([p for _, p in cases], p0s)
    B.step(20)
    eps = np.finfo(np.float32).eps
    for c, ((case, phi0), p0) in enumerate(zip(cases, p0s)):
        alone = Sim(case).init(phi0, None, p0).step(20)
        torch.cuda.synchronize()
        sa, sb = B.case(c).export_state(), alone.export_state()
        assert sa["step"] == sb["step"] == 20
        for key in ("f", "g", "hist"):
            ta, tb = sa[key], sb[key]
            if case.phase_eq == "allen_cahn":
                assert torch.equal(ta, tb), (c, key)
            else:
                err = (ta - tb).abs().max().item()
                assert err <= 16 * eps * max(1.0, tb.abs().max().item()), (c, key, err)
