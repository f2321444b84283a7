"""Batched execution of many uneven lattices (one persistent launch per step)
and the captured-graph path of the plain step, through the C ABI.

A case advanced inside a batch runs the same per-node arithmetic as the case
advanced alone, so the two are compared bitwise; one FP64 batch is also
compared with the oracle directly.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mods():
    from paper_2111_00847_amd.sim import BatchSim, Sim
    return Sim, BatchSim


def _mixed_cases(dtype):
    """Six cases of unequal, partly ragged sizes and both boundary kinds."""
    out = []
    for k, (nx, ny, th) in enumerate([(128, 64, 40.0), (70, 37, 120.0), (256, 128, 95.0),
                                       (33, 90, 60.0), (128, 64, 150.0), (200, 9, 75.0)]):
        case, phi0 = W.spreading_case(nx, ny, th, dtype=dtype, R0=min(nx, 2 * ny) / 6.0)
        out.append((case, phi0))
    dam, phid = W.dam_break(nx=96, ny=40, column=24, dtype=dtype, theta_deg=70.0)
    out.append((dam, phid))
    return out


def _assert_same_state(a, b, what):
    sa, sb = a.export_state(), b.export_state()
    assert sa["step"] == sb["step"], what
    for key in ("f", "g", "hist"):
        ta, tb = sa[key].cpu().numpy(), sb[key].cpu().numpy()
        assert np.array_equal(ta, tb), (what, key, float(np.abs(ta - tb).max()))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["eager_default_stream", "graph_side_stream", "autotuned_graph"])
def test_batch_bitwise_equals_single(dtype, mode):
    Sim, BatchSim = _mods()
    cases = _mixed_cases(dtype)
    p0s = ["hydrostatic"] * len(cases)
    stream = None if mode == "eager_default_stream" else torch.cuda.Stream()
    B = BatchSim([c for c, _ in cases], autotune=(mode == "autotuned_graph"), stream=stream)
    B.init([p for _, p in cases], p0s)
    print(f"batch {dtype} {mode}: tuning {B.tuning()}", flush=True)
    steps = 75                         # two graph replays of 32 plus 11 eager launches
    B.step(steps)
    for c, ((case, phi0), p0) in enumerate(zip(cases, p0s)):
        alone = Sim(case).init(phi0, None, p0).step(steps)
        torch.cuda.synchronize()
        _assert_same_state(B.case(c), alone, f"case {c} {case.name}")
    d = B.case(2).diagnostics()
    assert d["nonfinite"] == 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["eager_default_stream", "graph_side_stream", "autotuned_graph"])
def test_batch_two_level_bitwise_equals_single(dtype, mode):
    """Plain Allen-Cahn batches advance two levels per launch (forced here on a
    batch below the size rule); 75 steps end on a one-level launch.  Every case
    equals its lone run bit for bit, and a batch with a Cahn-Hilliard case
    keeps one level per launch."""
    import os
    Sim, BatchSim = _mods()
    cases = _mixed_cases(dtype)
    p0s = ["hydrostatic"] * len(cases)
    stream = None if mode == "eager_default_stream" else torch.cuda.Stream()
    os.environ["LBM_TWO_LEVEL"] = "1"
    try:
        B = BatchSim([c for c, _ in cases], autotune=(mode == "autotuned_graph"), stream=stream)
        ch, php = W.to_cahn_hilliard(*W.static_droplet(n=40, R=10.0, dtype=dtype))
        mixed = BatchSim([cases[0][0], ch], stream=stream)
    finally:
        os.environ.pop("LBM_TWO_LEVEL", None)
    assert B.levels_per_launch() == 2
    assert mixed.levels_per_launch() == 1
    del mixed
    B.init([p for _, p in cases], p0s)
    steps = 75                         # two graph replays of 32 plus 11 eager levels
    B.step(steps)
    for c, ((case, phi0), p0) in enumerate(zip(cases, p0s)):
        alone = Sim(case).init(phi0, None, p0).step(steps)
        torch.cuda.synchronize()
        _assert_same_state(B.case(c), alone, f"case {c} {case.name}")
    assert B.case(2).diagnostics()["nonfinite"] == 0


def test_batch_spreading_64_two_level_by_size_rule():
    """The 64-case spreading batch (3.3 M nodes) takes two levels per launch by
    the size rule, and stays bitwise equal to lone runs of a few of its cases."""
    Sim, BatchSim = _mods()
    cases = W.spreading_batch()
    B = BatchSim([c for c, _ in cases], stream=torch.cuda.Stream()).init([p for _, p in cases])
    assert B.levels_per_launch() == 2
    steps = 41
    B.step(steps)
    for c in (0, 17, 63):
        case, phi0 = cases[c]
        alone = Sim(case).init(phi0).step(steps)
        torch.cuda.synchronize()
        _assert_same_state(B.case(c), alone, f"spreading case {c}")


def test_batch_fp64_against_oracle():
    Sim, BatchSim = _mods()
    cases = _mixed_cases("f64")[:3]
    B = BatchSim([c for c, _ in cases], stream=torch.cuda.Stream())
    B.init([p for _, p in cases], ["hydrostatic"] * len(cases)).step(120)
    torch.cuda.synchronize()
    for c, (case, phi0) in enumerate(cases):
        o = oracle.OracleSim(case).init(phi0, None, "hydrostatic").step(120)
        for a, b in zip(B.case(c).moments_np(), o.moments()):
            assert np.abs(a - b).max() <= 1e-10 * max(1.0, np.abs(b).max())


def test_batch_autotune_choice_and_reinit():
    """The autotuner returns a valid tuning and leaves every case at step 0 with
    its initial field."""
    Sim, BatchSim = _mods()
    cases = W.spreading_batch(ncases=8, dtype="f32")
    B = BatchSim([c for c, _ in cases], autotune=True)
    B.init([p for _, p in cases])
    t = B.tuning()
    assert t["tile_rows"] in (4, 8, 16) and t["thread_rows"] in (4, 8) and t["thread_rows"] <= t["tile_rows"]
    assert 1 <= t["grid"] <= t["items"]
    for c, (case, phi0) in enumerate(cases):
        s = B.case(c)
        assert s.export_state()["step"] == 0
        phi, _, _ = s.moments_np()
        assert np.abs(phi - phi0).max() < 1e-6


def test_plain_step_graph_equals_eager():
    """lbm_step on a side stream replays a captured graph of 32 steps; the result
    equals the eager launches on the default stream bitwise."""
    Sim, _ = _mods()
    case, phi0 = W.rti(nx=128, ny=256)
    p0 = "hydrostatic"
    a = Sim(case).init(phi0, None, p0).step(101)
    s = torch.cuda.Stream()
    b = Sim(case, stream=s).init(phi0, None, p0)
    b.step(70)
    b.step(31)                         # graph cache hit, then eager remainder
    torch.cuda.synchronize()
    _assert_same_state(a, b, "rti 128x256 graph vs eager")


def test_steps_captured_by_the_caller_replay_like_eager_launches():
    """lbm_step and lbm_batch_step called while the caller captures the stream
    (long enough runs that would otherwise use the library's own graphs) go into
    the caller's graph; each of three replays, with eager work and
    synchronisations between them, advances the state as eager launches do."""
    Sim, BatchSim = _mods()
    case, phi0 = W.rti(nx=128, ny=256)
    p0 = "hydrostatic"
    cases = _mixed_cases("f32")[:3]
    p0s = ["hydrostatic"] * len(cases)
    s = torch.cuda.Stream()
    a = Sim(case, stream=s).init(phi0, None, p0)
    B = BatchSim([c for c, _ in cases], stream=s)
    B.init([p for _, p in cases], p0s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.step(100)
        B.step(40)
    ref = Sim(case).init(phi0, None, p0)
    ref_b = [Sim(c).init(p, None, q) for (c, p), q in zip(cases, p0s)]
    for rep in range(1, 4):
        g.replay()
        torch.cuda.synchronize()
        ref.step(100)
        for r in ref_b:
            r.step(40)
        _ = torch.ones(1000, device="cuda").sum().item()     # eager work between replays
        torch.cuda.synchronize()
        _assert_same_state(a, ref, f"captured lbm_step, replay {rep}")
        for c, r in enumerate(ref_b):
            _assert_same_state(B.case(c), r, f"captured lbm_batch_step case {c}, replay {rep}")


def test_batch_case_view_rejects_bad_index():
    from paper_2111_00847_amd._lib import LbmError
    _, BatchSim = _mods()
    cases = _mixed_cases("f32")[:2]
    B = BatchSim([c for c, _ in cases])
    with pytest.raises(LbmError):
        B.case(2)


def _wide_cases(dtype):
    """A mix with two-node-window cases (Cahn-Hilliard droplets, one ragged with
    walls; a corrected Allen-Cahn dam break), a local-gradient dam break and plain
    Allen-Cahn cases."""
    out = []
    case, phi0 = W.spreading_case(128, 64, 40.0, dtype=dtype, R0=20.0)
    out.append((case, phi0))
    case, phi0 = W.square_droplet_ch(n=64, R=16.0, sigma=1e-3, rho_ratio=100.0, dtype=dtype)
    out.append((case, phi0))
    case = case.replace(nx=70, ny=37, wall_y=True, theta=(1.5708, 1.5708, 1.2, 2.0), name="ch_droplet_70x37_walls")
    X, Y = W.grid(case)
    out.append((case, W.tanh_profile(12.0 - np.hypot(X - 35.0, Y - 18.5), 4.0, 1.0, -1.0)))
    case, phi0 = W.dam_break(nx=96, ny=40, column=24, dtype=dtype, theta_deg=70.0)
    out.append((case.replace(model="corrected"), phi0))
    out.append((case, phi0))
    out.append((case.replace(grad_scheme="local"), phi0))
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["eager_default_stream", "autotuned_graph"])
def test_wide_batch_bitwise_equals_single(dtype, mode):
    """Cahn-Hilliard, corrected Allen-Cahn and local-gradient cases run their own
    bodies inside the batch: plain Allen-Cahn cases equal the case advanced alone
    bitwise; the others to a few units of rounding (the batch may run a body at
    another tile height than the lone lattice, and the compiler contracts the
    arithmetic of the two instantiations into FMAs differently: 1 ulp in FP64
    measured)."""
    Sim, BatchSim = _mods()
    cases = _wide_cases(dtype)
    p0s = ["hydrostatic"] * len(cases)
    stream = None if mode == "eager_default_stream" else torch.cuda.Stream()
    B = BatchSim([c for c, _ in cases], autotune=(mode == "autotuned_graph"), stream=stream)
    B.init([p for _, p in cases], p0s)
    t = B.tuning()
    print(f"wide batch {dtype} {mode}: tuning {t}", flush=True)
    assert t["tile_rows"] in (4, 8) and t["thread_rows"] == t["tile_rows"]   # one node per thread
    steps = 75
    B.step(steps)
    for c, ((case, phi0), p0) in enumerate(zip(cases, p0s)):
        alone = Sim(case).init(phi0, None, p0).step(steps)
        torch.cuda.synchronize()
        what = f"case {c} {case.name} {case.phase_eq} {case.model}"
        if case.phase_eq == "allen_cahn" and case.model != "corrected" and case.grad_scheme == "stencil":
            _assert_same_state(B.case(c), alone, what)
            continue
        eps = np.finfo(np.float64 if dtype == "f64" else np.float32).eps
        sa, sb = B.case(c).export_state(), alone.export_state()
        assert sa["step"] == sb["step"], what
        pairs = ((key, sa[key], sb[key]) for key in ("f", "g", "hist"))
        for key, xa, xb in pairs:
            ta, tb = xa.cpu().numpy(), xb.cpu().numpy()
            err = float(np.abs(ta - tb).max())
            print(f"{what} {key}: max|diff| {err:.2e}", flush=True)
            assert err <= 16 * eps * max(1.0, float(np.abs(tb).max())), (what, key, err)


SHAPES = [(4, 4), (8, 4), (8, 8), (16, 4), (16, 8)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("wide", [False, True])
def test_every_batch_shape_equals_single(dtype, wide):
    """Every tile shape of the one-level batch launch (forced with
    LBM_BATCH_SHAPE, one workgroup per tile and a strided grid of 7
    workgroups) against the cases advanced alone: plain Allen-Cahn cases
    bitwise, the wide bodies' cases to a few units of rounding (as in the
    wide-batch test above).  Two-level launches are off (LBM_TWO_LEVEL=0) so
    that every level runs the forced shape."""
    import os
    from paper_2111_00847_amd._lib import LbmError
    Sim, BatchSim = _mods()
    cases = _wide_cases(dtype) if wide else _mixed_cases(dtype)
    p0s = ["hydrostatic"] * len(cases)
    steps = 13
    alone = [Sim(c).init(phi0, None, p0).step(steps) for (c, phi0), p0 in zip(cases, p0s)]
    torch.cuda.synchronize()
    eps = np.finfo(np.float64 if dtype == "f64" else np.float32).eps
    ran = 0
    for ty, by in SHAPES:
        for grid in (0, 7):
            runnable = not (ty == 16 and dtype == "f64") and not (wide and (by != ty or ty > 8))
            os.environ["LBM_BATCH_SHAPE"] = f"{ty},{by},{grid}"
            os.environ["LBM_TWO_LEVEL"] = "0"
            try:
                if not runnable:
                    with pytest.raises(LbmError) as e:
                        BatchSim([c for c, _ in cases])
                    assert e.value.code == -4
                    continue
                B = BatchSim([c for c, _ in cases], autotune=True)   # the forced shape wins
            finally:
                os.environ.pop("LBM_BATCH_SHAPE", None)
                os.environ.pop("LBM_TWO_LEVEL", None)
            t = B.tuning()
            assert (t["tile_rows"], t["thread_rows"]) == (ty, by), t
            assert t["grid"] == (grid if grid else t["items"]), t
            B.init([p for _, p in cases], p0s)
            B.step(steps)
            torch.cuda.synchronize()
            ran += 1
            for c, (case, _) in enumerate(cases):
                what = f"shape {ty},{by},{grid} case {c} {case.name}"
                exact = case.phase_eq == "allen_cahn" and case.model != "corrected" and case.grad_scheme == "stencil"
                if exact:
                    _assert_same_state(B.case(c), alone[c], what)
                    continue
                sa, sb = B.case(c).export_state(), alone[c].export_state()
                assert sa["step"] == sb["step"], what
                for key in ("f", "g", "hist"):
                    ta, tb = sa[key].cpu().numpy(), sb[key].cpu().numpy()
                    err = float(np.abs(ta - tb).max())
                    assert err <= 16 * eps * max(1.0, float(np.abs(tb).max())), (what, key, err)
            del B
    assert ran == (4 if wide else (6 if dtype == "f64" else 10))
