"""Write the FP64 oracle trajectories that the long-horizon GPU parity tests
compare against (tests/test_gpu_horizon.py).

    python tests/golden/make_trajectories.py [name ...]

Calls only ``oracle`` (the plain FP64 CPU implementation) and ``workloads``
(the seeded set-ups).  For each workload it runs the oracle from the set-up's
initial state to the stated step count and stores, at a list of snapshot
levels, phi on a fixed sample of nodes (every node with (x + 7 y) % 32 == 0:
nx/32 nodes in every row, ny/32 in every column, tile edges and the walls
included), u and v on the same sample at a few of those levels, and the
full-lattice total of phi and max |u| at every level.  Output:
tests/golden/trajectory_<name>.npz.

The three workloads are the paper's Rayleigh-Taylor instability (Sec. 4.4,
256 x 1024, 20000 steps), the dam break (Sec. 4.5, 1024 x 512, 4000 steps) and
a droplet spreading on a wetting wall (Sec. 4.3 set-up, 512 x 256, contact
angle 47 degrees, 10000 steps).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SAMPLE_STRIDE = 32

WORKLOADS = {
    "rti_256x1024": dict(
        make=lambda: W.rti(dtype="f64"),
        snaps=[250, 500, 1000, 2000, 4000, 6000, 8000, 10000, 12000, 14000, 16000, 18000, 20000],
        vel=[2000, 10000, 20000]),
    "dam_break_1024x512": dict(
        make=lambda: W.dam_break(dtype="f64"),
        snaps=[50, 100, 150, 200, 300, 500, 750, 1000, 1500, 2000, 2500, 3000, 3500, 4000],
        vel=[100, 1000, 4000]),
    "spreading_512x256": dict(
        make=lambda: W.spreading_case(512, 256, 47.0, dtype="f64"),
        snaps=[500, 1000, 2000, 3000, 4000, 5000, 6000, 7000, 8000, 9000, 10000],
        vel=[1000, 5000, 10000]),
}


def sample_index(nx: int, ny: int) -> np.ndarray:
    """Flat indices y * nx + x of the sampled nodes, (x + 7 y) % 32 == 0."""
    y, x = np.mgrid[0:ny, 0:nx]
    return np.flatnonzero(((x + 7 * y) % SAMPLE_STRIDE == 0).ravel())


def path_of(name: str) -> str:
    return os.path.join(HERE, f"trajectory_{name}.npz")


def make(name: str) -> str:
    spec = WORKLOADS[name]
    case, phi0 = spec["make"]()
    idx = sample_index(case.nx, case.ny)
    o = oracle.OracleSim(case).init(phi0, None, "hydrostatic")
    snaps, vel = spec["snaps"], spec["vel"]
    phi_s = np.empty((len(snaps), idx.size))
    u_s = np.empty((len(vel), 2, idx.size))
    sum_phi = np.empty(len(snaps))
    umax = np.empty(len(snaps))
    t0, done = time.time(), 0
    for j, n in enumerate(snaps):
        o.step(n - done)
        done = n
        phi, u, _ = o.moments()
        phi_s[j] = phi.ravel()[idx]
        sum_phi[j] = phi.sum()
        umax[j] = np.sqrt(u[0] ** 2 + u[1] ** 2).max()
        if n in vel:
            u_s[vel.index(n)] = u.reshape(2, -1)[:, idx]
        print(f"{name}: level {n} ({time.time() - t0:.0f} s)", flush=True)
    out = path_of(name)
    np.savez_compressed(out, steps=np.array(snaps), vel_steps=np.array(vel), index=idx, phi=phi_s, u=u_s,
                        sum_phi=sum_phi, umax=umax, sum_phi0=np.sum(phi0), nx=case.nx, ny=case.ny)
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    oracle.set_threads(os.cpu_count() or 1)
    for nm in names:
        print(make(nm), flush=True)
