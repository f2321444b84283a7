#!/usr/bin/env python3
"""Benchmark of the fused phase-field LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the Rayleigh-Taylor set-up of Sec. 4.4 at 256 x 1024 nodes, FP32
(synthetic initial interface, lattice parameters as in workloads.rti).  A step
is one fused time step of the whole lattice (moments, stencils, closure, both
MRT collisions, streaming with walls).  The K steps of lbm_step are captured
as one graph and replayed; each timed region holds exactly K steps with the
state already in device memory, and the value is lattice updates per second
of the median replay.  The 46 MB state of this lattice stays in the 256 MB
last-level cache from step to step, where lbm_step advances two levels per
launch (the two-level kernel: bit for bit two one-level launches); the
`one_level` entry times the same K steps as K one-level launches.  The
point streamed from HBM is `large_grid`.

The JSON line also carries:
  roofline     -- the step kernel against the HBM peak: algorithmic bytes per
                  launch (168 B per lattice update in FP32, times the nodes
                  and the levels one launch advances) / average launch
                  duration (HIP events over the timed region on the launch
                  stream);
                  `traffic` is the measured HBM bytes per launch from the
                  committed rocprofv3 counter summary when it matches the
                  current kernel source, else null; `copy_GBs` is torch's
                  device copy of the same bytes (half read, half written),
                  which stays in the 256 MB cache as the step's 46 MB state
                  does, and `frac_of_copy` the step's rate against it;
  large_grid   -- the same kernels at 4096 x 4096 (state 2.9 GB, far beyond the
                  256 MB Infinity Cache), where a one-level launch is bound by
                  HBM and the two-level launch crosses HBM once per two levels,
                  next to the bandwidth of torch's own device copy and of the
                  streaming probe; large_grid_fp64 the FP64 kernels there,
                  large_grid_2048x8192 the FP32 kernels on a lattice of the
                  same nodes, four times taller than wide;
  batched      -- 64 droplet-spreading cases of uneven sizes (Sec. 4.3 set-up,
                  FP32): one launch per two levels over all cases (the
                  two-level batch kernel; the autotuned one-level launch for an
                  odd tail) replayed from a captured graph, against the same
                  cases advanced one after another with the plain step
                  (graph-captured, and eager); `batched_frac` counts the
                  algorithmic 168 B per update;
  square_droplet -- total-phi drift and max |div u| of the 64 x 64 square
                  droplet after 2000 FP64 steps;
  cahn_hilliard -- the Cahn-Hilliard variant's step kernel on a 4096 x 4096
                  square droplet (Sec. 4.1 set-up scaled up, FP32);
  local_gradient -- the Allen-Cahn step with the local gradient scheme (Eq.
                  local) on the 4096 x 4096 RTI lattice (FP32), two levels per
                  launch (and one-level launches beside it);
  adjoint      -- the differentiable dam break (Sec. 4.5 set-up, 1024 x 512,
                  FP32, 4000 steps, checkpoints every 200): time of the
                  backward pass (tape recompute + adjoint steps) over the time
                  of the plain forward (medians of three passes each);
                  `full_tape` times the same gradients with every level kept
                  on one tape (176 GB, when it fits in 3/4 of the free device
                  memory): the forward records the tape and the backward runs
                  only the adjoint steps;
  cpu_baseline -- the FP64 oracle timed on the host on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ALG_BYTES = {"f32": 168, "f64": 336}   # per lattice update: f, g read+write, (phi, u, v) history read+write
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_step2_rti_256x1024_traffic.json")
# everything the headline's two-level kernel is compiled from (with the build flags)
KERNEL_SOURCES = ["paper_2111_00847_amd/csrc/lbm_step2.hip", "paper_2111_00847_amd/csrc/lbm_step2.hpp",
                  "paper_2111_00847_amd/csrc/lbm_fused.hpp",
                  "paper_2111_00847_amd/csrc/lbm_tile.hpp", "paper_2111_00847_amd/csrc/lbm_device.hpp",
                  "paper_2111_00847_amd/csrc/lbm_common.hpp", "paper_2111_00847_amd/build.py"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_graph(sim, steps, reps, torch, one_level=False):
    """Capture `steps` steps of `sim` as one graph on a side stream (lbm_step's
    launches; `one_level`: one lbm_step call, hence one one-level launch, per
    step), replay it once untimed, then `reps` times between two HIP events on
    that stream, synchronising before and after each replay.  Returns the
    replay times in ms (each replay advances the lattice by `steps` levels)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        if one_level:
            for _ in range(steps):
                sim.step(1)
        else:
            sim.step(steps)
    with torch.cuda.stream(s):
        g.replay()
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            e0.record(s)
            g.replay()
            e1.record(s)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    del g
    return out


def _median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def measured_traffic(nodes):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source and this workload."""
    try:
        with open(PROFILE_TRAFFIC) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("nodes") != nodes:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(budget_s=15.0, budget_1t_s=6.0):
    """The FP64 oracle on the host's cores (all threads, then one thread), on a
    bounded sample of the headline workload."""
    import oracle
    import workloads as W
    case, phi0 = W.rti()
    cores = oracle.num_threads()

    def run(budget):
        s = oracle.OracleSim(case.replace(dtype="f64")).init(phi0, None, "hydrostatic")
        s.step(2)                   # first-touch of the oracle's fields
        steps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            s.step(1)
            steps += 1
        dt = time.perf_counter() - t0
        return case.nodes * steps / dt / 1e6, steps, dt

    mlups, steps, dt = run(budget_s)
    oracle.set_threads(1)
    mlups1, steps1, dt1 = run(budget_1t_s)
    oracle.set_threads(cores)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "single_thread_value": round(mlups1, 3), "cpu_model": cpu, "host_cpus": os.cpu_count(),
            "sample": f"FP64 oracle, rti 256x1024: {steps} steps on {cores} threads ({dt:.1f} s), "
                      f"{steps1} steps on 1 thread ({dt1:.1f} s), each after 2 untimed"}


def measure_main(args, torch, W, Sim):
    """The headline: RTI 256 x 1024, FP32, K steps after W warm-up steps, timed
    as the median of `reps` replays of a captured graph of the K steps."""
    from paper_2111_00847_amd import api
    case, phi0 = W.rti()
    sim = Sim(case, "cuda:0").init(phi0, None, "hydrostatic")
    sim.step(args.warmup)
    torch.cuda.synchronize()
    reps = time_graph(sim, args.steps, args.reps, torch)
    ms = _median(reps)
    levels = api.lbm_levels_per_launch(api.make_params(case))
    launches = args.steps // levels + args.steps % levels
    ms_launch = ms / launches
    nodes = case.nodes
    mlups = nodes * args.steps / (ms * 1e-3) / 1e6
    alg = ALG_BYTES[case.dtype] * nodes * levels
    achieved = alg / (ms_launch * 1e-3) / 1e9
    ms1 = _median(time_graph(sim, args.steps, args.reps, torch, one_level=True))
    ach1 = ALG_BYTES[case.dtype] * nodes / (ms1 / args.steps * 1e-3) / 1e9
    d = sim.diagnostics()
    assert d["nonfinite"] == 0, "non-finite state after the timed steps"
    del sim
    torch.cuda.empty_cache()
    kernel = "k_step2<float> (two levels per launch)" if levels == 2 else "k_step<float>"
    return {
        "metric": "MLUPS (fused FP32 phase-field LBM step, plain single-lattice launches)",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rayleigh_taylor_256x1024", "nx": case.nx, "ny": case.ny,
                   "lattice": "D2Q9 x2 (phase field + flow), MRT", "boundaries": "periodic x, walls y",
                   "timing": f"median of {args.reps} replays of a captured graph of {args.steps} steps",
                   "replay_ms": [round(x, 4) for x in reps]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(nodes),
                     "kernel": kernel, "levels_per_launch": levels, "alg_bytes_per_launch": alg,
                     "avg_launch_ms": round(ms_launch, 5),
                     "state": "46 MB, resident in the 256 MB last-level cache between steps: the launch is "
                              "bound by latency and VALU issue there, not by HBM; the point streamed from HBM is "
                              "large_grid (4096 x 4096)"},
        "one_level": {"kernel": "k_step<float>", "value": round(nodes * args.steps / (ms1 * 1e-3) / 1e6, 2),
                      "unit": "MLUPS", "avg_launch_ms": round(ms1 / args.steps, 5),
                      "achieved_GBs": round(ach1, 1), "frac": round(ach1 / HBM_PEAK_GBS, 4)},
    }


def measure_large(args, torch, W, Sim, dtype="f32", nx=4096, ny=4096):
    """The same kernel on a large lattice, nx x ny (4096 x 4096: state 2.9 GB in
    FP32, 5.6 GB in FP64, far beyond the 256 MB cache), where a one-level launch
    is bound by HBM.
    lbm_step advances two levels per launch there too, crossing HBM once per
    two levels: `achieved_GBs` counts the algorithmic 168 B (FP32) per lattice
    update, `hbm_GBs` the bytes one launch must move (the state read once and
    written once, whatever the levels it advances) over its duration; `one_level`
    times the same steps as one-level launches."""
    from paper_2111_00847_amd import api
    caseL, phiL = W.rti(nx=nx, ny=ny, dtype=dtype)
    simL = Sim(caseL, "cuda:0").init(phiL, None, "hydrostatic")
    simL.step(10)
    steps = args.large_steps if dtype == "f32" else max(args.large_steps // 2, 1)
    levels = api.lbm_levels_per_launch(api.make_params(caseL))
    msL = _median(time_graph(simL, steps, 3, torch))
    ms1 = _median(time_graph(simL, steps, 3, torch, one_level=True))
    assert simL.diagnostics()["nonfinite"] == 0, "non-finite state after the timed large-lattice steps"
    msLl = msL / steps
    alg = ALG_BYTES[dtype] * caseL.nodes
    achL = alg / (msLl * 1e-3) / 1e9
    ach1 = alg / (ms1 / steps * 1e-3) / 1e9
    del simL
    torch.cuda.empty_cache()
    t = "float" if dtype == "f32" else "double"
    return {"workload": f"rayleigh_taylor_{nx}x{ny}", "dtype": dtype, "steps": steps,
            "value": round(caseL.nodes * steps / (msL * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "kernel": f"k_step2<{t}> (two levels per launch)" if levels == 2 else f"k_step<{t}>",
            "levels_per_launch": levels, "achieved_GBs": round(achL, 1),
            "frac": round(achL / HBM_PEAK_GBS, 4), "avg_level_ms": round(msLl, 4),
            "hbm_GBs": round(achL / levels, 1), "hbm_frac": round(achL / levels / HBM_PEAK_GBS, 4),
            "one_level": {"kernel": f"k_step<{t}>", "value": round(caseL.nodes * steps / (ms1 * 1e-3) / 1e6, 1),
                          "achieved_GBs": round(ach1, 1), "frac": round(ach1 / HBM_PEAK_GBS, 4),
                          "avg_launch_ms": round(ms1 / steps, 4)}}


def measure_ch(args, torch, W, Sim, n=4096):
    """The Cahn-Hilliard variant (Sec. 2, Eq. CHE; App. C, Eq. MfMRCH1) on the
    Sec. 4.1 square droplet scaled to n x n (FP32, density ratio 1000): its step
    kernel against the HBM peak at the same 168 B of algorithmic traffic per
    update as the Allen-Cahn step."""
    case, phi0 = W.square_droplet_ch(n=n, R=n / 4.0, dtype="f32")
    sim = Sim(case, "cuda:0").init(phi0)
    sim.step(10)
    ms = _median(time_graph(sim, args.ch_steps, 3, torch))
    ms_launch = ms / args.ch_steps
    alg = ALG_BYTES["f32"] * case.nodes
    ach = alg / (ms_launch * 1e-3) / 1e9
    d = sim.diagnostics()
    assert d["nonfinite"] == 0, "non-finite state after the timed CH steps"
    del sim
    torch.cuda.empty_cache()
    return {"workload": f"square_droplet_cahn_hilliard_{n}x{n}", "dtype": "f32", "steps": args.ch_steps,
            "value": round(case.nodes * args.ch_steps / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "kernel": "k_step_ch<float>", "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
            "avg_launch_ms": round(ms_launch, 4)}


def measure_local(args, torch, W, Sim):
    """The Allen-Cahn step with the local gradient scheme (Eq. local) on the
    4096 x 4096 Rayleigh-Taylor lattice (FP32): two levels per launch, with
    `one_level` the same steps as one-level launches.  Its history also carries
    m^phiC of the previous level: 184 B of algorithmic traffic per update."""
    from paper_2111_00847_amd import api
    case, phi0 = W.rti(nx=4096, ny=4096)
    case = case.replace(grad_scheme="local")
    sim = Sim(case, "cuda:0").init(phi0, None, "hydrostatic")
    sim.step(10)
    steps = args.large_steps
    levels = api.lbm_levels_per_launch(api.make_params(case))
    ms = _median(time_graph(sim, steps, 3, torch))
    ms1 = _median(time_graph(sim, steps, 3, torch, one_level=True))
    alg = 184 * case.nodes
    ach = alg / (ms / steps * 1e-3) / 1e9
    ach1 = alg / (ms1 / steps * 1e-3) / 1e9
    phi, _, _ = sim.moments()
    assert bool(torch.isfinite(phi).all()), "non-finite state after the timed local-scheme steps"
    del sim, phi
    torch.cuda.empty_cache()
    return {"workload": "rayleigh_taylor_4096x4096_local_gradient", "dtype": "f32", "steps": steps,
            "value": round(case.nodes * steps / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "kernel": "k_step2_local<float> (two levels per launch)" if levels == 2 else "k_step_local<float>",
            "levels_per_launch": levels, "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
            "avg_level_ms": round(ms / steps, 4),
            "one_level": {"kernel": "k_step_local<float>", "value": round(case.nodes * steps / (ms1 * 1e-3) / 1e6, 1),
                          "achieved_GBs": round(ach1, 1), "frac": round(ach1 / HBM_PEAK_GBS, 4),
                          "avg_launch_ms": round(ms1 / steps, 4)}}


def measure_square_droplet(torch, W, Sim):
    """The 64 x 64 square droplet (Sec. 4.1 set-up of the AC model, FP64, 2000
    steps): the total-phi drift and max |div u| it is reported by."""
    case, phi0 = W.square_droplet()
    sim = Sim(case, "cuda:0").init(phi0).step(2000)
    d = sim.diagnostics()
    s0 = float(phi0.sum())
    return {"workload": "square_droplet_64x64", "dtype": "f64", "steps": 2000,
            "sum_phi_rel_drift": abs(d["sum_phi"] - s0) / s0, "max_div_u": d["max_div"], "Du_rms": d["Du_rms"],
            "Sm_rms": d["Sm_rms"]}


def measure_copy(torch, mib=1024, reps=20):
    """Bandwidth of torch's device-to-device copy of a `mib` MiB buffer (read + write
    bytes per second): a measured ceiling next to the nominal HBM peak."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = _timed(torch.cuda.current_stream(), torch, lambda: [b.copy_(a) for _ in range(reps)])
    del a, b
    torch.cuda.empty_cache()
    return round(2 * n * 4 * reps / (ms * 1e-3) / 1e9, 1)


def measure_ceiling(torch, mib=1024, reps=5):
    """The device's streaming rates (lbm_bandwidth_probe): read, write and copy
    of a `mib` MiB buffer (beyond the 256 MB last-level cache), swept over grid
    sizes and store policies; each point the median of `reps` launches timed
    with HIP events.  Rates in GB/s (copy: read + written bytes)."""
    from paper_2111_00847_amd import api
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    sweep = []
    for kind, name in ((0, "read"), (1, "write"), (2, "copy")):
        for nt in ((True,) if kind == 0 else (False, True)):
            for blocks in (256, 512, 1024, 2048, 4096, 8192, 16384):
                fn = lambda: api.lbm_bandwidth_probe(kind, dst, src, nbytes, blocks, nt, s)
                fn()
                ts = [_timed(s, torch, fn) for _ in range(reps)]
                ms = _median(ts)
                moved = nbytes * (2 if kind == 2 else 1)
                sweep.append({"kind": name, "nt": nt, "blocks": blocks, "GBs": round(moved / (ms * 1e-3) / 1e9, 1)})
    del src, dst
    torch.cuda.empty_cache()
    best = {k: max(p["GBs"] for p in sweep if p["kind"] == k) for k in ("read", "write", "copy")}
    return {"buffer_MiB": mib, "read_GBs": best["read"], "write_GBs": best["write"], "copy_GBs": best["copy"],
            "sweep": sweep}


def _timed(stream, torch, fn):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def measure_batched(args, torch, W, Sim, BatchSim):
    """64 spreading cases: batched launch vs the plain step case by case."""
    cases = W.spreading_batch()
    phis = [p for _, p in cases]
    nodes = sum(c.nodes for c, _ in cases)
    K = args.batch_steps
    s = torch.cuda.Stream()
    B = BatchSim([c for c, _ in cases], autotune=True, stream=s).init(phis)
    B.step(64)
    ms_b = _timed(s, torch, lambda: B.step(K))
    tun = B.tuning()
    levels = B.levels_per_launch()
    nonfinite = sum(B.case(c).diagnostics()["nonfinite"] for c in range(len(cases)))
    assert nonfinite == 0, "non-finite batched state"
    del B
    sims = [Sim(c, stream=s).init(p) for c, p in cases]
    for sm in sims:
        sm.step(64)                      # captures each case's graph
    ms_g = _timed(s, torch, lambda: [sm.step(K) for sm in sims])
    eager = [Sim(c).init(p) for c, p in cases]   # default stream: one launch per step
    ms_e = _timed(torch.cuda.current_stream(), torch, lambda: [sm.step(K) for sm in eager])
    del sims, eager
    torch.cuda.empty_cache()
    mlups = lambda ms: round(nodes * K / (ms * 1e-3) / 1e6, 1)
    return {"workload": "spreading_batch_64_cases", "cases": len(cases), "nodes": nodes, "steps": K,
            "batched_MLUPS": mlups(ms_b), "sequential_graph_MLUPS": mlups(ms_g),
            "sequential_eager_MLUPS": mlups(ms_e), "speedup_vs_sequential_graph": round(ms_g / ms_b, 3),
            "speedup_vs_sequential_eager": round(ms_e / ms_b, 3),
            "batched_frac": round(ALG_BYTES["f32"] * nodes * K / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "levels_per_launch": levels, "tuning": tun}


def measure_adjoint(args, torch, W, Sim):
    """Backward / forward time ratio of the differentiable dam break."""
    import math
    import numpy as np
    from paper_2111_00847_amd.autograd import LBMFunction
    N, chk = args.adjoint_steps, 200
    case, phi0 = W.dam_break(dtype="f32")
    rng = np.random.default_rng(W.SEED)
    g_t = 1e-6 * (1.0 + 0.1 * rng.standard_normal())
    th_t = math.radians(rng.uniform(60.0, 120.0))
    tgt = Sim(case.replace(gravity=(0.0, -g_t), theta=(th_t,) * 4)).init(phi0).step(N)
    target = tgt.moments()[0]
    del tgt
    stream = torch.cuda.current_stream()
    plain, fw = Sim(case), []
    for _ in range(3):   # the median of three forward passes from phi0
        plain.init(phi0)
        fw.append(_timed(stream, torch, lambda: plain.step(N)))
    ms_fwd = _median(fw)
    del plain
    phi0_t = torch.tensor(phi0, dtype=torch.float32, device="cuda", requires_grad=True)
    grav = torch.tensor([0.0, -1e-6], dtype=torch.float64, requires_grad=True)
    theta = torch.tensor([math.pi / 2] * 4, dtype=torch.float64, requires_grad=True)
    box = {}

    def run(c):
        for t in (phi0_t, grav, theta):
            t.grad = None
        ms_f = _timed(stream, torch, lambda: box.__setitem__("phi", LBMFunction.apply(phi0_t, grav, theta, case, N,
                                                                                       None, c)))
        box["L"] = ((box["phi"] - target) ** 2).sum()
        ms_b = _timed(stream, torch, lambda: box["L"].backward())
        grads = (float(grav.grad[1]), float(theta.grad.sum()))
        ok = bool(torch.isfinite(phi0_t.grad).all()) and all(math.isfinite(v) for v in grads)
        assert ok, "non-finite gradient"
        return ms_f, ms_b, grads

    # the full tape (every level kept, no recomputation) when it fits in 3/4 of
    # the free device memory, else checkpoints only
    from paper_2111_00847_amd import api
    tape_bytes = api.lbm_tape_size(api.make_params(case), N + 1)
    full = tape_bytes <= 0.75 * torch.cuda.mem_get_info()[0]
    modes = ([0] if full else []) + [chk]
    res = {}
    for c in modes:
        run(c)   # untimed: afterwards the snapshots, tape and adjoint buffers come from torch's cache
        rs = [run(c) for _ in range(3)]   # medians of three passes
        res[c] = (_median([r[0] for r in rs]), _median([r[1] for r in rs]), rs[-1][2])
        assert all(r[2] == rs[0][2] for r in rs), "gradients differ from pass to pass"
        box.clear()
        torch.cuda.empty_cache()
    if full:
        assert res[0][2] == res[chk][2], "full-tape and checkpointed gradients differ"
    ck = res[chk]
    out = {"workload": "dam_break_1024x512_fp32", "steps": N, "checkpoint_every": chk,
           "forward_ms": round(ms_fwd, 2), "forward_with_snapshots_ms": round(ck[0], 2),
           "backward_ms": round(ck[1], 2), "backward_over_forward": round(ck[1] / ms_fwd, 3),
           "dL_dg": -ck[2][0], "dL_dtheta": ck[2][1], "full_tape": None}
    if full:
        ft = res[0]
        out["full_tape"] = {"tape_GB": round(tape_bytes / 1e9, 1), "forward_recording_ms": round(ft[0], 2),
                            "backward_ms": round(ft[1], 2), "backward_over_forward": round(ft[1] / ms_fwd, 3)}
    del box, phi0_t
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--reps", type=int, default=5, help="timed graph replays of the headline (median)")
    ap.add_argument("--large-steps", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--adjoint-steps", type=int, default=4000)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--ch-steps", type=int, default=100)
    ap.add_argument("--no-ch", action="store_true")
    ap.add_argument("--no-local", action="store_true")
    ap.add_argument("--only-ch", action="store_true",
                    help="run only the Cahn-Hilliard measurement (profiling runs)")
    ap.add_argument("--only-main", action="store_true",
                    help="run only the headline measurement (profiling runs)")
    ap.add_argument("--large-dtype", choices=["f32", "f64"], default="f32",
                    help="with --only-large: the dtype of the 4096 x 4096 measurement (profiling runs)")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the 4096 x 4096 measurement (profiling runs)")
    ap.add_argument("--only-local", action="store_true",
                    help="run only the local-gradient measurement (profiling runs)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="run only the adjoint measurement (profiling runs)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched measurement (profiling runs)")
    ap.add_argument("--only-ceiling", action="store_true",
                    help="run only the streaming-ceiling sweep (lbm_bandwidth_probe)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark: copy a MIB-sized device buffer 20 times "
                         "(a plain copy kernel of known size, to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "a lattice is not sharded across GPUs here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2111_00847_amd.sim import BatchSim, Sim

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_each_way": n * 4, "launches": 20}))
        return

    out = {}
    if args.only_ch:
        print(json.dumps({"cahn_hilliard": measure_ch(args, torch, W, Sim)}), flush=True)
        return
    if args.only_main:
        print(json.dumps(measure_main(args, torch, W, Sim)), flush=True)
        return
    if args.only_ceiling:
        print(json.dumps({"stream_ceiling": measure_ceiling(torch)}), flush=True)
        return
    if args.only_local:
        print(json.dumps({"local_gradient": measure_local(args, torch, W, Sim)}), flush=True)
        return
    if args.only_adjoint:
        print(json.dumps({"adjoint": measure_adjoint(args, torch, W, Sim)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": measure_batched(args, torch, W, Sim, BatchSim)}), flush=True)
        return
    if not args.only_large:
        out.update(measure_main(args, torch, W, Sim))
        half = out["roofline"]["alg_bytes_per_launch"] // 2
        copy_gbs = measure_copy(torch, mib=max(1, round(half / (1 << 20))), reps=200)
        out["roofline"]["copy_GBs"] = copy_gbs
        out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / copy_gbs, 4)
    if not args.no_large and args.only_large and args.large_dtype == "f64":
        out["large_grid_fp64"] = measure_large(args, torch, W, Sim, "f64")
    elif not args.no_large:
        out["large_grid"] = measure_large(args, torch, W, Sim)
        copy_gbs = measure_copy(torch)
        out["large_grid"]["torch_copy_GBs"] = copy_gbs
        out["large_grid"]["frac_of_copy"] = round(out["large_grid"]["achieved_GBs"] / copy_gbs, 4)
        ceil = measure_ceiling(torch)
        out["large_grid"]["stream_ceiling"] = {k: ceil[k] for k in ("read_GBs", "write_GBs", "copy_GBs")}
        out["large_grid"]["frac_of_stream_copy"] = round(out["large_grid"]["achieved_GBs"] / ceil["copy_GBs"], 4)
        if not args.only_large:
            out["large_grid_fp64"] = measure_large(args, torch, W, Sim, "f64")
            out["large_grid_2048x8192"] = measure_large(args, torch, W, Sim, "f32", nx=2048, ny=8192)
    if not args.only_large:
        out["square_droplet"] = measure_square_droplet(torch, W, Sim)
    if not args.no_ch and not args.only_large:
        out["cahn_hilliard"] = measure_ch(args, torch, W, Sim)
    if not args.no_local and not args.only_large:
        out["local_gradient"] = measure_local(args, torch, W, Sim)
    if not args.no_batched and not args.only_large:
        out["batched"] = measure_batched(args, torch, W, Sim, BatchSim)
    if not args.no_adjoint and not args.only_large:
        out["adjoint"] = measure_adjoint(args, torch, W, Sim)
    if not args.no_cpu_baseline and not args.only_large:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
