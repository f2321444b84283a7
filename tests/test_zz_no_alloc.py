"""The batch step that allocates nothing (lbm_batch_step_noalloc) against the
planned batch step (lbm_batch_step) through the C ABI: two calls in a row on
the same GPU, the second with a smaller batch, each bitwise equal to the
planned step of the same cases (untuned plan: the same tile shape)."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mixed_cases(dtype, small=False):
    """Uneven lattices of every tile body: plain Allen-Cahn (periodic, walls,
    ragged), Cahn-Hilliard, corrected Allen-Cahn, local gradient."""
    out = []
    out.append(W.square_droplet(n=48 if small else 64, side=24 if small else 32, dtype=dtype))
    out.append(W.dam_break(nx=70 if small else 100, ny=37, column=20, dtype=dtype, theta_deg=65.0, g=1e-5))
    if not small:
        out.append(W.spreading_case(128, 64, 120.0, dtype=dtype))
        out.append(W.rti(nx=64, ny=130, dtype=dtype))
        c, p = W.to_cahn_hilliard(*W.static_droplet(n=40, R=10.0, dtype=dtype))
        out.append((c, p))
        c, p = W.dam_break(nx=48, ny=32, column=12, dtype=dtype, theta_deg=80.0, g=1e-5)
        out.append((c.replace(model="corrected"), p))
    c, p = W.dam_break(nx=40, ny=24, column=10, dtype=dtype, theta_deg=60.0, g=1e-5)
    out.append((c.replace(grad_scheme="local"), p))
    return out


def _run_both(cases, steps):
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd.sim import BatchSim
    phis = [p for _, p in cases]
    p0s = ["hydrostatic"] * len(cases)
    B = BatchSim([c for c, _ in cases], autotune=False).init(phis, p0s)
    torch.cuda.synchronize()
    other = api._buffer(B.state.numel(), B.state.device)
    other.copy_(B.state)
    B.step(steps)
    api.lbm_batch_step_noalloc(B.params, other, steps)
    torch.cuda.synchronize()
    return B, other


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_batch_step_equals_planned_step(dtype):
    for small, steps in ((False, 23), (True, 17)):
        cases = _mixed_cases(dtype, small)
        print(f"noalloc batch {dtype}: {len(cases)} cases, {steps} steps", flush=True)
        B, other = _run_both(cases, steps)
        assert torch.equal(B.state, other), "no-alloc batch step differs from the planned batch step"
        d = B.case(0).diagnostics()
        assert d["nonfinite"] == 0
        del B, other
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_two_level_batch_step_equals_planned_step(dtype):
    """Plain Allen-Cahn batches with two levels per launch forced on (both
    paths read LBM_TWO_LEVEL): odd step counts end on a one-level launch."""
    import os
    os.environ["LBM_TWO_LEVEL"] = "1"
    try:
        for small, steps in ((False, 23), (True, 17)):
            cases = _mixed_cases(dtype, small)[:4 if not small else 2]
            print(f"noalloc two-level batch {dtype}: {len(cases)} cases, {steps} steps", flush=True)
            B, other = _run_both(cases, steps)
            assert B.levels_per_launch() == 2
            assert torch.equal(B.state, other), "no-alloc two-level batch step differs from the planned batch step"
            assert B.case(0).diagnostics()["nonfinite"] == 0
            del B, other
            torch.cuda.empty_cache()
    finally:
        os.environ.pop("LBM_TWO_LEVEL", None)


def test_noalloc_rejects_oversized_batches():
    from paper_2111_00847_amd import api
    from paper_2111_00847_amd._lib import LbmError
    case, _ = W.square_droplet(n=8, side=4)
    params = [api.make_params(case)] * 257
    buf = api._buffer(1 << 20, "cuda")
    with pytest.raises(LbmError) as e:
        api.lbm_batch_step_noalloc(params, buf, 1)
    assert e.value.code == -2
    with pytest.raises(LbmError) as e:
        api.lbm_batch_step_noalloc(params[:1], buf, -1)
    assert e.value.code == -2
    api.lbm_batch_step_noalloc(params[:1], buf, 0)   # zero steps: a no-op
