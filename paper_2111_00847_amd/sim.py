"""Convenience wrappers: one lattice (Sim) or a batch of lattices (BatchSim) on one GPU."""
from __future__ import annotations

import numpy as np
import torch

from . import api


class Sim:
    def __init__(self, case, device="cuda:0", state=None, stream=None):
        """`state`: an existing state buffer to view (e.g. one case of a batch);
        `stream`: a torch.cuda.Stream for every call (None = the current stream)."""
        self.case = case
        self.p = api.make_params(case)
        self.device = torch.device(device)
        self.dtype = api.torch_dtype(self.p)
        self.state = api.new_state(self.p, self.device) if state is None else state
        self.stream = stream
        self.shape = (case.ny, case.nx)

    def _t(self, a):
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            return a.to(self.device, self.dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=self.dtype, device=self.device)

    # With a side stream, tensors made on the current stream are handed over
    # (side waits for current) and results handed back (current waits for side).
    def _enter(self):
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self, sync=False):
        if self.stream is not None:
            if sync:                      # inputs freed after return must not be reused early
                self.stream.synchronize()
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def hydrostatic_pressure(self, phi0):
        """The library's hydrostatic initial pressure of phi0 (lbm_hydrostatic_pressure)."""
        phi = self._t(phi0)
        p0 = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        self._enter()
        api.lbm_hydrostatic_pressure(self.p, phi, p0, self.stream)
        self._leave(sync=True)
        return p0

    def init(self, phi0, u0=None, p0=None):
        """p0: a field, None (zero) or "hydrostatic" (lbm_hydrostatic_pressure of phi0)."""
        if isinstance(p0, str):
            assert p0 == "hydrostatic", p0
            p0 = self.hydrostatic_pressure(phi0)
        args = (self._t(phi0), self._t(u0), self._t(p0))
        self._enter()
        api.lbm_init(self.p, self.state, *args, self.stream)
        self._leave(sync=True)
        return self

    def step(self, n=1):
        api.lbm_step(self.p, self.state, n, self.stream)
        return self

    def moments(self):
        phi = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        u = torch.empty((2,) + self.shape, dtype=self.dtype, device=self.device)
        p = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        self._enter()
        api.lbm_moments(self.p, self.state, phi, u, p, self.stream)
        self._leave()
        return phi, u, p

    def moments_np(self):
        return tuple(t.double().cpu().numpy() for t in self.moments())

    def diagnostics(self):
        return api.lbm_diagnostics(self.p, self.state, self.stream)

    def export_state(self):
        f = torch.empty((9,) + self.shape, dtype=self.dtype, device=self.device)
        g = torch.empty_like(f)
        h = torch.empty((api.hist_planes(self.p),) + self.shape, dtype=self.dtype, device=self.device)
        self._enter()
        step = api.lbm_export_state(self.p, self.state, f, g, h, self.stream)
        self._leave()
        return dict(f=f, g=g, hist=h, step=step)

    def import_state(self, f, g, hist, step):
        hist = None if hist is None else self._t(hist)
        f, g = self._t(f), self._t(g)
        self._enter()
        api.lbm_import_state(self.p, self.state, f, g, hist, step, self.stream)
        self._leave(sync=True)
        return self


class BatchSim:
    """Many independent lattices (one dtype) advanced together, one launch per step."""

    def __init__(self, cases, device="cuda:0", autotune=False, stream=None):
        self.cases = list(cases)
        self.params = [api.make_params(c) for c in self.cases]
        self.device = torch.device(device)
        self.dtype = api.torch_dtype(self.params[0])
        self.stream = stream
        self.handle = api.lbm_batch_create(self.params, autotune)
        self.state = api.new_batch_state(self.handle, self.device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            api.lbm_batch_destroy(h)
            self.handle = None

    def _t(self, a):
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            return a.to(self.device, self.dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=self.dtype, device=self.device)

    def init(self, phi0s, p0s=None):
        """p0s: None, "hydrostatic" (every case), or one entry per case (a field,
        None or "hydrostatic")."""
        phis = [self._t(a) for a in phi0s]
        if isinstance(p0s, str):
            p0s = [p0s] * len(phis)
        ps = None
        if p0s is not None:
            ps = []
            for c, a in enumerate(p0s):
                if isinstance(a, str):
                    assert a == "hydrostatic", a
                    ps.append(Sim(self.cases[c], self.device, state=self.state[:0], stream=self.stream)
                              .hydrostatic_pressure(phis[c]))
                else:
                    ps.append(self._t(a))
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
        api.lbm_batch_init(self.handle, self.params, self.state, phis, ps, self.stream)
        if self.stream is not None:
            self.stream.synchronize()
        return self

    def step(self, n=1):
        api.lbm_batch_step(self.handle, self.state, n, self.stream)
        return self

    def tuning(self):
        return api.lbm_batch_tuning(self.handle)

    def levels_per_launch(self):
        return api.lbm_batch_levels_per_launch(self.handle)

    def case(self, c):
        """Sim view of case c (its state lives inside the batch state)."""
        off = api.lbm_batch_case_offset(self.handle, c)
        n = api.lbm_state_size(self.params[c])
        return Sim(self.cases[c], self.device, state=self.state[off:off + n], stream=self.stream)
