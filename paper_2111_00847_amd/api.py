"""Python binding of the C ABI with the same entry-point names (include/lbm.h).

Arguments are torch tensors on the GPU (device memory and streams come from
PyTorch); each function checks shapes and dtypes, passes raw pointers to the
library and raises :class:`LbmError` on a non-zero status.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import torch

from ._lib import (LBM_F32, LBM_F64, LBM_PERIODIC, LBM_WALLS, LbmError, LbmParams, call, lib)

_VISC = {"linear_mu": 0, "inverse_nu": 1}
_MODEL = {"present": 0, "original": 1, "corrected": 2}


def make_params(case) -> LbmParams:
    """lbm_params from a workload case (plain field copy, no derived quantities)."""
    p = LbmParams()
    p.nx, p.ny = int(case.nx), int(case.ny)
    p.dtype = LBM_F64 if case.dtype == "f64" else LBM_F32
    p.bc_x = LBM_WALLS if case.wall_x else LBM_PERIODIC
    p.bc_y = LBM_WALLS if case.wall_y else LBM_PERIODIC
    p.visc_law = _VISC[case.visc_law]
    p.model = _MODEL.get(case.model, 99)
    p.phase_eq = {"allen_cahn": 0, "cahn_hilliard": 1}.get(case.phase_eq, 99)
    p.grad_scheme = {"stencil": 0, "local": 1}.get(getattr(case, "grad_scheme", "stencil"), 99)
    p.phi_A, p.phi_B = case.phiA, case.phiB
    p.rho_A, p.rho_B = case.rhoA, case.rhoB
    p.nu_A, p.nu_B = case.nuA, case.nuB
    p.sigma, p.W, p.M_phi, p.eta = case.sigma, case.W, case.M, case.eta
    for i in range(9):
        p.s_f[i] = case.s_f[i]
        p.s_g[i] = case.s_g[i]
    p.body_force[0], p.body_force[1] = case.body_force
    p.gravity[0], p.gravity[1] = case.gravity
    p.rho_ref = case.rho_ref
    for i in range(4):
        p.theta[i] = case.theta[i]
    p.rho0 = case.rho0
    p.eps_n = case.eps_n
    return p


def torch_dtype(p: LbmParams):
    return torch.float64 if p.dtype == LBM_F64 else torch.float32


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor], p: LbmParams, shape=None, name="array"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != torch_dtype(p):
        raise ValueError(f"{name} has dtype {t.dtype}, expected {torch_dtype(p)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def lbm_state_size(p: LbmParams) -> int:
    n = ctypes.c_size_t()
    call("lbm_state_size", ctypes.byref(p), ctypes.byref(n))
    return n.value


def new_state(p: LbmParams, device="cuda") -> torch.Tensor:
    """A state buffer (uint8 tensor) of lbm_state_size bytes, 256-byte aligned."""
    n = lbm_state_size(p)
    buf = torch.empty(n + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + n]


def _state_ptr(state: torch.Tensor):
    if not state.is_cuda or state.dtype != torch.uint8:
        raise ValueError("state must be a uint8 GPU tensor from new_state()")
    return ctypes.c_void_p(state.data_ptr())


def lbm_init(p, state, phi0, u0=None, p0=None, stream=None):
    shp = (p.ny, p.nx)
    call("lbm_init", ctypes.byref(p), _state_ptr(state), _ptr(phi0, p, shp, "phi0"),
         _ptr(u0, p, (2,) + shp, "u0"), _ptr(p0, p, shp, "p0"), _stream(stream))


def lbm_hydrostatic_pressure(p, phi0, p0, stream=None):
    """Hydrostatic initial pressure of phi0 into p0 (both [ny][nx] GPU tensors)."""
    shp = (p.ny, p.nx)
    call("lbm_hydrostatic_pressure", ctypes.byref(p), _ptr(phi0, p, shp, "phi0"), _ptr(p0, p, shp, "p0"),
         _stream(stream))


def lbm_step(p, state, nsteps=1, stream=None):
    call("lbm_step", ctypes.byref(p), _state_ptr(state), int(nsteps), _stream(stream))


def lbm_bandwidth_probe(kind, dst, src, nbytes, blocks, nt=True, stream=None):
    """One streaming-probe launch (0 read, 1 write, 2 copy) over device tensors."""
    call("lbm_bandwidth_probe", int(kind), dst.data_ptr(), src.data_ptr() if src is not None else None,
         int(nbytes), int(blocks), int(bool(nt)), _stream(stream))


def lbm_levels_per_launch(p) -> int:
    v = ctypes.c_int32()
    call("lbm_levels_per_launch", ctypes.byref(p), ctypes.byref(v))
    return v.value


def lbm_moments(p, state, phi=None, u=None, pr=None, stream=None):
    shp = (p.ny, p.nx)
    call("lbm_moments", ctypes.byref(p), _state_ptr(state), _ptr(phi, p, shp, "phi"),
         _ptr(u, p, (2,) + shp, "u"), _ptr(pr, p, shp, "p"), _stream(stream))


DIAG_NAMES = ("sum_phi", "max_div", "Du_rms", "Sm_rms", "umax", "nonfinite")


def lbm_diagnostics(p, state, stream=None, raise_nonfinite=False):
    out = (ctypes.c_double * 6)()
    code = lib().lbm_diagnostics(ctypes.byref(p), _state_ptr(state), out, _stream(stream))
    if code != 0 and not (code == -7 and not raise_nonfinite):
        raise LbmError("lbm_diagnostics", code)
    return dict(zip(DIAG_NAMES, list(out)))


def hist_planes(p):
    """History planes per node: phi, u, v of the previous level, plus m^phiC for
    the local gradient scheme."""
    return 5 if p.grad_scheme == 1 else 3


def lbm_export_state(p, state, f=None, g=None, hist=None, stream=None):
    shp = (p.ny, p.nx)
    st = ctypes.c_int64()
    call("lbm_export_state", ctypes.byref(p), _state_ptr(state), _ptr(f, p, (9,) + shp, "f"),
         _ptr(g, p, (9,) + shp, "g"), _ptr(hist, p, (hist_planes(p),) + shp, "hist"), ctypes.byref(st),
         _stream(stream))
    return st.value


def lbm_import_state(p, state, f, g, hist, step, stream=None):
    shp = (p.ny, p.nx)
    call("lbm_import_state", ctypes.byref(p), _state_ptr(state), _ptr(f, p, (9,) + shp, "f"),
         _ptr(g, p, (9,) + shp, "g"), _ptr(hist, p, (hist_planes(p),) + shp, "hist"), int(step),
         _stream(stream))


# ---------------------------------------------------------------- reverse mode
def _buffer(nbytes, device):
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def lbm_tape_size(p, nlevels) -> int:
    n = ctypes.c_size_t()
    call("lbm_tape_size", ctypes.byref(p), int(nlevels), ctypes.byref(n))
    return n.value


def new_tape(p, nlevels, device="cuda") -> torch.Tensor:
    return _buffer(lbm_tape_size(p, nlevels), device)


def lbm_tape_record(p, state, tape, nlevels, stream=None):
    call("lbm_tape_record", ctypes.byref(p), _state_ptr(state), _state_ptr(tape), int(nlevels), _stream(stream))


def lbm_tape_restore(p, tape, j, state, stream=None):
    call("lbm_tape_restore", ctypes.byref(p), _state_ptr(tape), int(j), _state_ptr(state), _stream(stream))


def lbm_adjoint_size(p) -> int:
    n = ctypes.c_size_t()
    call("lbm_adjoint_size", ctypes.byref(p), ctypes.byref(n))
    return n.value


def new_adjoint(p, device="cuda") -> torch.Tensor:
    return _buffer(lbm_adjoint_size(p), device)


def lbm_adjoint_phi(p, state, adj, dL_dphi, stream=None):
    call("lbm_adjoint_phi", ctypes.byref(p), _state_ptr(state), _state_ptr(adj),
         _ptr(dL_dphi, p, (p.ny, p.nx), "dL_dphi"), _stream(stream))


def lbm_adjoint_step(p, tape, j, adj, stream=None):
    call("lbm_adjoint_step", ctypes.byref(p), _state_ptr(tape), int(j), _state_ptr(adj), _stream(stream))


def lbm_adjoint_run(p, tape, j_first, count, adj, stream=None):
    call("lbm_adjoint_run", ctypes.byref(p), _state_ptr(tape), int(j_first), int(count), _state_ptr(adj),
         _stream(stream))


def lbm_adjoint_init(p, adj, dL_dphi0, stream=None):
    call("lbm_adjoint_init", ctypes.byref(p), _state_ptr(adj), _ptr(dL_dphi0, p, (p.ny, p.nx), "dL_dphi0"),
         _stream(stream))


ADJ_PARAM_NAMES = ("gravity_x", "gravity_y", "theta_xm", "theta_xp", "theta_ym", "theta_yp")


def lbm_adjoint_params(p, adj, stream=None):
    """Returns (out[6], level): dL/dgravity (2), dL/dtheta (4) and the adjoint's level."""
    out = (ctypes.c_double * 6)()
    lev = ctypes.c_int64()
    call("lbm_adjoint_params", ctypes.byref(p), _state_ptr(adj), out, ctypes.byref(lev), _stream(stream))
    return list(out), lev.value


def lbm_adjoint_export(p, adj, fbar=None, gbar=None, hbar=None, stream=None):
    shp = (p.ny, p.nx)
    call("lbm_adjoint_export", ctypes.byref(p), _state_ptr(adj), _ptr(fbar, p, (9,) + shp, "fbar"),
         _ptr(gbar, p, (9,) + shp, "gbar"), _ptr(hbar, p, (3,) + shp, "hbar"), _stream(stream))


def lbm_adjoint_import(p, adj, fbar, gbar, hbar, level, stream=None):
    shp = (p.ny, p.nx)
    call("lbm_adjoint_import", ctypes.byref(p), _state_ptr(adj), _ptr(fbar, p, (9,) + shp, "fbar"),
         _ptr(gbar, p, (9,) + shp, "gbar"), _ptr(hbar, p, (3,) + shp, "hbar"), int(level), _stream(stream))


# ---------------------------------------------------------------- batches
def lbm_batch_create(params, autotune=False) -> ctypes.c_void_p:
    """Plan a batch of lattices (a list of LbmParams, one dtype); returns the
    opaque handle, to be released with lbm_batch_destroy."""
    arr = (LbmParams * len(params))(*params)
    h = ctypes.c_void_p()
    call("lbm_batch_create", arr, len(params), 1 if autotune else 0, ctypes.byref(h))
    return h


def lbm_batch_state_size(batch) -> int:
    n = ctypes.c_size_t()
    call("lbm_batch_state_size", batch, ctypes.byref(n))
    return n.value


def lbm_batch_case_offset(batch, c: int) -> int:
    n = ctypes.c_size_t()
    call("lbm_batch_case_offset", batch, int(c), ctypes.byref(n))
    return n.value


def new_batch_state(batch, device="cuda") -> torch.Tensor:
    n = lbm_batch_state_size(batch)
    buf = torch.empty(n + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + n]


def lbm_batch_init(batch, params, state, phi0s, p0s=None, stream=None):
    """phi0s / p0s: lists of GPU tensors, one per case (p0s or its entries may be None)."""
    n = len(params)
    if len(phi0s) != n or (p0s is not None and len(p0s) != n):
        raise ValueError("one initial field per case expected")
    phis = (ctypes.c_void_p * n)(*[_ptr(t, params[c], (params[c].ny, params[c].nx), f"phi0[{c}]")
                                    for c, t in enumerate(phi0s)])
    ps = None
    if p0s is not None:
        ps = (ctypes.c_void_p * n)(*[_ptr(t, params[c], (params[c].ny, params[c].nx), f"p0[{c}]")
                                      for c, t in enumerate(p0s)])
    call("lbm_batch_init", batch, _state_ptr(state), phis, ps, _stream(stream))


def lbm_batch_step(batch, state, nsteps=1, stream=None):
    call("lbm_batch_step", batch, _state_ptr(state), int(nsteps), _stream(stream))


def lbm_batch_step_noalloc(params, state, nsteps=1, stream=None):
    """Advance a batch state of the cases `params` (list of LbmParams) without a
    plan and without allocating (the library's fixed device case table)."""
    arr = (LbmParams * len(params))(*params)
    call("lbm_batch_step_noalloc", arr, len(params), _state_ptr(state), int(nsteps), _stream(stream))


def lbm_batch_tuning(batch):
    ty, by, g, items = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    call("lbm_batch_tuning", batch, ctypes.byref(ty), ctypes.byref(by), ctypes.byref(g), ctypes.byref(items))
    return dict(tile_rows=ty.value, thread_rows=by.value, grid=g.value, items=items.value)


def lbm_batch_levels_per_launch(batch):
    v = ctypes.c_int32()
    call("lbm_batch_levels_per_launch", batch, ctypes.byref(v))
    return v.value


def lbm_batch_destroy(batch):
    call("lbm_batch_destroy", batch)
