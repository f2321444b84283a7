"""torch.autograd.Function over a trajectory of the fused step.

``LBMFunction.apply(phi0, gravity, theta, case, nsteps, p0=None, chk=200)``
returns phi of level ``nsteps`` started from ``lbm_init(phi0, u0=None, p0)``.
With ``chk`` > 0, forward keeps a copy of the state every ``chk`` levels;
backward starts the adjoint at level ``nsteps`` and walks the segments newest
first: it records the segment's levels into a tape from its snapshot (bitwise
the forward levels) and runs the library's adjoint step over them.  With
``chk`` = 0 (full tape), forward itself records every level 0 .. nsteps into
one tape (nsteps + 1 copies of the state: 44 MB a level at 1024 x 512 FP32,
so 4000 levels take 176 GB of the device's memory) and ends on its last slot;
backward runs the adjoint steps over that tape with no recomputation.  Both
modes give the same gradients bit for bit (the tape levels are the forward
levels).  Gradients: dL/dphi0 (p0 held fixed), dL/dgravity (2), dL/dtheta
(4 walls: x-, x+, y-, y+).  Every step of both passes runs in the library's
kernels.
"""
from __future__ import annotations

import torch

from . import api


def _params(case, gravity, theta):
    g = [float(v) for v in gravity.detach().cpu().reshape(-1)]
    t = [float(v) for v in theta.detach().cpu().reshape(-1)]
    return api.make_params(case.replace(gravity=(g[0], g[1]), theta=tuple(t)))


class LBMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, gravity, theta, case, nsteps, p0=None, chk=200):
        p = _params(case, gravity, theta)
        dt = api.torch_dtype(p)
        dev = phi0.device
        phi0 = phi0.to(dt).contiguous()
        p0 = None if p0 is None else p0.to(dev, dt).contiguous()
        state = api.new_state(p, dev)
        api.lbm_init(p, state, phi0, None, p0)
        snaps, tape = [], None
        if chk == 0:
            tape = api.new_tape(p, nsteps + 1, dev)
            api.lbm_tape_record(p, state, tape, nsteps + 1)
            api.lbm_tape_restore(p, tape, nsteps, state)
        else:
            if chk < 0:
                raise ValueError("chk must be >= 0")
            done = 0
            while done < nsteps:
                k = min(chk, nsteps - done)
                snaps.append(state.clone())
                api.lbm_step(p, state, k)
                done += k
        phi = torch.empty((p.ny, p.nx), dtype=dt, device=dev)
        api.lbm_moments(p, state, phi, None, None)
        ctx.p, ctx.nsteps, ctx.chk = p, nsteps, chk
        ctx.snaps, ctx.final, ctx.tape = snaps, state, tape
        ctx.dev, ctx.dt = dev, dt
        ctx.param_dtype = (gravity.dtype, gravity.device, theta.dtype, theta.device)
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        p, dev, dt = ctx.p, ctx.dev, ctx.dt
        grad_phi = grad_phi.to(dev, dt).contiguous()
        adj = api.new_adjoint(p, dev)
        api.lbm_adjoint_phi(p, ctx.final, adj, grad_phi)
        if ctx.tape is not None:
            if ctx.nsteps > 0:
                api.lbm_adjoint_run(p, ctx.tape, ctx.nsteps - 1, ctx.nsteps, adj)
        else:
            tape = api.new_tape(p, min(ctx.chk, max(ctx.nsteps, 1)), dev)
            for seg in range(len(ctx.snaps) - 1, -1, -1):
                start = seg * ctx.chk
                L = min(ctx.chk, ctx.nsteps - start)
                api.lbm_tape_record(p, ctx.snaps[seg], tape, L)
                api.lbm_adjoint_run(p, tape, L - 1, L, adj)
        dphi0 = torch.empty((p.ny, p.nx), dtype=dt, device=dev)
        api.lbm_adjoint_init(p, adj, dphi0)
        out, level = api.lbm_adjoint_params(p, adj)
        assert level == 0, level
        gd, gdev, td, tdev = ctx.param_dtype
        dgrav = torch.tensor(out[0:2], dtype=gd, device=gdev)
        dth = torch.tensor(out[2:6], dtype=td, device=tdev)
        ctx.snaps = ctx.final = ctx.tape = None
        return dphi0, dgrav, dth, None, None, None, None


def trajectory_phi(phi0, gravity, theta, case, nsteps, p0=None, chk=200):
    """phi at level nsteps, differentiable in phi0, gravity (2) and theta (4);
    chk = 0 keeps every level on one tape (no recomputation in backward)."""
    return LBMFunction.apply(phi0, gravity, theta, case, nsteps, p0, chk)
