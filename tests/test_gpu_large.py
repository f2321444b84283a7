"""Lattices whose state copy exceeds 4 GiB: the plain step then addresses its
buffers with 64-bit offsets (32-bit below that).  A lattice of k side-by-side
copies of the 256 x 1024 Rayleigh-Taylor field (periodic in x) must stay k exact
copies of the 256 x 1024 run, which itself matches the oracle; so the
large-offset path is held to the small one bitwise, at a size the oracle could
not follow step by step."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

STEPS = 40


@pytest.mark.parametrize("dtype,k", [("f32", 188), ("f64", 100)])
def test_lattice_beyond_4gib_per_copy_is_the_tiled_small_lattice(dtype, k):
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.sim import Sim
    case_s, phi_s = W.rti(nx=256, ny=1024, dtype=dtype)
    p_s = W.hydrostatic_pressure(case_s, phi_s)
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
