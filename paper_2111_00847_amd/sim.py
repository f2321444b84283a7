"""Convenience wrapper: one lattice on one GPU."""
from __future__ import annotations

import numpy as np
import torch

from . import api


class Sim:
    def __init__(self, case, device="cuda:0"):
        self.case = case
        self.p = api.make_params(case)
        self.device = torch.device(device)
        self.dtype = api.torch_dtype(self.p)
        self.state = api.new_state(self.p, self.device)
        self.shape = (case.ny, case.nx)

    def _t(self, a):
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            return a.to(self.device, self.dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=self.dtype, device=self.device)

    def init(self, phi0, u0=None, p0=None):
        api.lbm_init(self.p, self.state, self._t(phi0), self._t(u0), self._t(p0))
        return self

    def step(self, n=1):
        api.lbm_step(self.p, self.state, n)
        return self

    def moments(self):
        phi = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        u = torch.empty((2,) + self.shape, dtype=self.dtype, device=self.device)
        p = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        api.lbm_moments(self.p, self.state, phi, u, p)
        return phi, u, p

    def moments_np(self):
        return tuple(t.double().cpu().numpy() for t in self.moments())

    def diagnostics(self):
        return api.lbm_diagnostics(self.p, self.state)

    def export_state(self):
        f = torch.empty((9,) + self.shape, dtype=self.dtype, device=self.device)
        g = torch.empty_like(f)
        h = torch.empty((3,) + self.shape, dtype=self.dtype, device=self.device)
        step = api.lbm_export_state(self.p, self.state, f, g, h)
        return dict(f=f, g=g, hist=h, step=step)

    def import_state(self, f, g, hist, step):
        hist = None if hist is None else self._t(hist)
        api.lbm_import_state(self.p, self.state, self._t(f), self._t(g), hist, step)
        return self
