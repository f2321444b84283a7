"""The C ABI library: loads, exports every declared entry point, validates
parameters on the host (no GPU needed: validation returns before any HIP call)."""
import ctypes
import math
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2111_00847_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    assert "lbm_step" in names and "lbm_init" in names
    for name in names:
        assert hasattr(L, name), name


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirror of lbm_params has the layout the C compiler gives the
    header's struct (size and the offset of every field)."""
    import shutil
    import subprocess
    from paper_2111_00847_amd._lib import LbmParams
    assert ctypes.sizeof(LbmParams) == 10 * 4 + (10 + 18 + 2 + 2 + 1 + 4 + 2) * 8
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    names = [n for n, _ in LbmParams._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"lbm.h\"\nint main(void) {\n"
                   + f'printf("%zu\\n", sizeof(lbm_params));\n'
                   + "".join(f'printf("%zu\\n", offsetof(lbm_params, {n}));\n' for n in names)
                   + "return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(LbmParams)
    for n, off in zip(names, out[1:]):
        assert getattr(LbmParams, n).offset == off, n


def _params(**kw):
    from paper_2111_00847_amd import api
    case, _ = W.square_droplet()
    return api.make_params(case.replace(**kw))


def _size(p):
    from paper_2111_00847_amd._lib import lib
    n = ctypes.c_size_t()
    return lib().lbm_state_size(ctypes.byref(p), ctypes.byref(n)), n.value


def test_state_size_layout():
    from paper_2111_00847_amd._lib import LBM_F64
    rc, n32 = _size(_params(dtype="f32"))
    assert rc == 0
    rc, n64 = _size(_params(dtype="f64"))
    assert rc == 0
    # two copies of 21 planes of 4096 nodes plus header and scratch
    assert n32 >= 256 + 2 * 21 * 4096 * 4
    assert n64 >= 256 + 2 * 21 * 4096 * 8
    assert n32 % 256 == 0 and n64 % 256 == 0


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), -2), (dict(ny=-3), -2), (dict(nx=1, wall_x=True), -2),
    (dict(rhoA=0.0), -4), (dict(nuB=-1.0), -4), (dict(W=0.0), -4), (dict(eta=0.5), -4),
    (dict(phiA=0.0, phiB=1.0), -4), (dict(theta=(0.0, 1.0, 1.0, 1.0)), -4),
    (dict(s_g=(2.0,) + (0.0,) * 8), -5), (dict(s_f=(0.0,) * 3 + (2.5,) + (0.0,) * 5), -5),
    (dict(sigma=float("nan")), -4), (dict(model="other"), -8), (dict(phase_eq="other"), -4),
])
def test_parameter_validation(kw, code):
    rc, _ = _size(_params(**kw))
    assert rc == code


def test_dtype_and_null_checks():
    from paper_2111_00847_amd._lib import lib
    p = _params()
    p.dtype = 7
    assert _size(p)[0] == -3
    p = _params()
    assert lib().lbm_state_size(ctypes.byref(p), None) == -1
    assert lib().lbm_state_size(None, None) == -1
    assert lib().lbm_init(ctypes.byref(p), None, None, None, None, None) == -1
    assert lib().lbm_step(ctypes.byref(p), None, 1, None) == -1
    assert lib().lbm_step(ctypes.byref(p), ctypes.c_void_p(256), -1, None) == -2
    assert lib().lbm_init(ctypes.byref(p), ctypes.c_void_p(300), ctypes.c_void_p(256), None, None,
                          None) == -2   # misaligned state
    assert lib().lbm_import_state(ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(256),
                                  ctypes.c_void_p(256), None, 3, None) == -1   # history required


def test_status_strings():
    from paper_2111_00847_amd._lib import lib
    for c in range(-8, 1):
        assert lib().lbm_status_string(c)


def test_batch_create_validation():
    """lbm_batch_create rejects bad arguments on the host before any HIP call."""
    from paper_2111_00847_amd._lib import LbmParams, lib
    L = lib()
    h = ctypes.c_void_p()
    good = _params(dtype="f32")
    arr1 = (LbmParams * 1)(good)
    assert L.lbm_batch_create(None, 1, 0, ctypes.byref(h)) == -1
    assert L.lbm_batch_create(arr1, 1, 0, None) == -1
    assert L.lbm_batch_create(arr1, 0, 0, ctypes.byref(h)) == -2
    assert L.lbm_batch_create((LbmParams * 2)(good, _params(dtype="f64")), 2, 0, ctypes.byref(h)) == -3
    assert L.lbm_batch_create((LbmParams * 2)(good, _params(W=-1.0)), 2, 0, ctypes.byref(h)) == -4
    # a case whose state copy reaches 4 GiB (the batch kernels address a case with 32-bit offsets)
    big = _params(dtype="f32", nx=51200, ny=1024)
    assert _size(big)[0] == 0
    assert L.lbm_batch_create((LbmParams * 2)(good, big), 2, 0, ctypes.byref(h)) == -2
    assert L.lbm_batch_state_size(None, None) == -1
    assert L.lbm_batch_step(None, None, 1, None) == -1
    assert L.lbm_batch_destroy(None) == -1


def test_cahn_hilliard_rejected_by_reverse_mode():
    """The adjoint runs the Allen-Cahn step only: CH parameters are refused on
    the host (before any HIP call)."""
    from paper_2111_00847_amd._lib import LbmParams, lib
    L = lib()
    p = _params(dtype="f32", phase_eq="cahn_hilliard", phiB=-1.0)
    n = ctypes.c_size_t()
    assert L.lbm_state_size(ctypes.byref(p), ctypes.byref(n)) == 0
    assert L.lbm_tape_record(ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(256), 1, None) == -8
    assert L.lbm_adjoint_run(ctypes.byref(p), ctypes.c_void_p(256), 0, 1, ctypes.c_void_p(256), None) == -8
    assert L.lbm_tape_restore(ctypes.byref(p), ctypes.c_void_p(256), 0, ctypes.c_void_p(256), None) == -8


def test_corrected_model_options():
    """The corrected model runs with either phase field; not with the local
    gradient scheme or in reverse mode."""
    from paper_2111_00847_amd._lib import LbmParams, lib
    L = lib()
    n = ctypes.c_size_t()
    p = _params(dtype="f32", phase_eq="cahn_hilliard", phiB=-1.0, model="corrected")
    assert L.lbm_state_size(ctypes.byref(p), ctypes.byref(n)) == 0
    p = _params(dtype="f32", model="corrected")
    assert L.lbm_state_size(ctypes.byref(p), ctypes.byref(n)) == 0
    q = _params(dtype="f32", model="corrected", grad_scheme="local")
    assert L.lbm_state_size(ctypes.byref(q), ctypes.byref(n)) == -8
    assert L.lbm_tape_record(ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(256), 1, None) == -8


def test_local_gradient_scheme_options():
    """The local gradient scheme (Eq. local) is an Allen-Cahn option with two more
    history planes per copy; the calls it does not cover refuse it on the host."""
    from paper_2111_00847_amd._lib import LbmParams, lib
    L = lib()
    n0, n1 = ctypes.c_size_t(), ctypes.c_size_t()
    p0 = _params(dtype="f32")
    p1 = _params(dtype="f32", grad_scheme="local")
    assert L.lbm_state_size(ctypes.byref(p0), ctypes.byref(n0)) == 0
    assert L.lbm_state_size(ctypes.byref(p1), ctypes.byref(n1)) == 0
    plane = (p0.nx * p0.ny + 63) // 64 * 64
    assert n1.value - n0.value == 2 * 2 * plane * 4          # two copies, two FP32 planes each
    bad = _params(dtype="f32", grad_scheme="other")
    assert L.lbm_state_size(ctypes.byref(bad), ctypes.byref(n0)) == -4
    bad = _params(dtype="f32")
    bad.reserved = 1
    assert L.lbm_state_size(ctypes.byref(bad), ctypes.byref(n0)) == -4
    ch = _params(dtype="f32", grad_scheme="local", phase_eq="cahn_hilliard", phiB=-1.0)
    assert L.lbm_state_size(ctypes.byref(ch), ctypes.byref(n0)) == -8
    assert L.lbm_export_state(ctypes.byref(p1), None, None, None, None, None, None) == -1   # accepted; NULL state
    assert L.lbm_import_state(ctypes.byref(p1), None, None, None, None, 0, None) == -1
    h = ctypes.c_void_p()
    rc = L.lbm_batch_create((LbmParams * 1)(p1), 1, 0, ctypes.byref(h))
    assert rc in (0, -6)      # accepted (the plan's device table needs a GPU: LBM_E_HIP without one)
    if rc == 0:
        assert L.lbm_batch_destroy(h) == 0
    assert L.lbm_tape_record(ctypes.byref(p1), ctypes.c_void_p(256), ctypes.c_void_p(256), 1, None) == -8


def test_noalloc_batch_step_validates_on_the_host():
    """lbm_batch_step_noalloc refuses oversized batches, negative step counts and
    misaligned states before any HIP call; zero steps is a no-op."""
    from paper_2111_00847_amd import _lib
    from paper_2111_00847_amd._lib import LbmParams, lib
    p = _params()
    many = (LbmParams * 257)(*([p] * 257))
    fake = ctypes.c_void_p(1 << 20)          # never dereferenced: every call returns before any HIP call
    assert lib().lbm_batch_step_noalloc(many, 257, fake, 1, None) == -2
    one = (LbmParams * 1)(p)
    assert lib().lbm_batch_step_noalloc(one, 1, fake, -1, None) == -2
    assert lib().lbm_batch_step_noalloc(one, 1, ctypes.c_void_p((1 << 20) + 8), 1, None) == -2
    assert lib().lbm_batch_step_noalloc(one, 0, fake, 1, None) == -2
    assert lib().lbm_batch_step_noalloc(None, 1, fake, 1, None) == -1
    bad = _params(W=-1.0)
    assert lib().lbm_batch_step_noalloc((LbmParams * 1)(bad), 1, fake, 1, None) == -4
    assert lib().lbm_batch_step_noalloc(one, 1, fake, 0, None) == 0
    assert _lib.LBM_OK == 0


def test_levels_per_launch():
    """Two levels per launch exactly for the Allen-Cahn step (stencil or local
    gradients, present or original model) on a lattice whose state copy fits
    32-bit byte offsets (below 4 GiB), of at least 256 tiles of 64 x 8 nodes
    (any size with LBM_TWO_LEVEL=1, none with LBM_TWO_LEVEL=0); one otherwise."""
    from paper_2111_00847_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)

    def levels(**kw):
        v = ctypes.c_int32(-1)
        assert L.lbm_levels_per_launch(ctypes.byref(_params(**kw)), ctypes.byref(v)) == 0
        return v.value

    os.environ.pop("LBM_TWO_LEVEL", None)
    assert levels(nx=256, ny=512, dtype="f32") == 2       # 4 x 64 tiles
    assert levels(nx=256, ny=504, dtype="f32") == 1       # 4 x 63 tiles
    assert levels(nx=64, ny=64, dtype="f32") == 1
    assert levels(nx=4096, ny=4096, dtype="f32") == 2     # streamed from HBM
    os.environ["LBM_TWO_LEVEL"] = "0"
    try:
        assert levels(nx=256, ny=1024, dtype="f32") == 1
        assert levels(nx=4096, ny=4096, dtype="f32") == 1
        os.environ["LBM_TWO_LEVEL"] = "1"
        assert levels(nx=64, ny=64, dtype="f32") == 2
        assert levels(nx=51200, ny=1024, dtype="f32") == 1  # a copy of 4 GiB and more
    finally:
        os.environ["LBM_TWO_LEVEL"] = "1"

    f32 = dict(dtype="f32")
    # the size-independent rules, everything eligible
    assert levels(nx=256, ny=1024, **f32) == 2             # the RTI lattice: 2 x 22 MB
    assert levels(nx=256, ny=1024, dtype="f64") == 2
    assert levels(nx=2, ny=2, wall_x=True, wall_y=True, **f32) == 2
    assert levels(nx=256, ny=1024, model="original", **f32) == 2
    assert levels(nx=256, ny=1024, model="corrected", **f32) == 1
    assert levels(nx=256, ny=1024, grad_scheme="local", **f32) == 2
    assert levels(nx=256, ny=1024, phase_eq="cahn_hilliard", phiA=1.0, phiB=-1.0, **f32) == 1
    assert levels(nx=2048, ny=1024, **f32) == 2            # 2 x 176 MB: streamed from HBM
    assert levels(nx=4096, ny=4096, dtype="f64") == 2      # 2 x 2.8 GB
    assert levels(nx=8192, ny=4096, dtype="f64") == 1      # 2 x 5.6 GB
    os.environ.pop("LBM_TWO_LEVEL", None)
    v = ctypes.c_int32()
    assert L.lbm_levels_per_launch(None, ctypes.byref(v)) == -1
    assert L.lbm_levels_per_launch(ctypes.byref(_params()), None) == -1


def test_bandwidth_probe_validates_on_the_host():
    """Invalid probe requests are refused before any launch."""
    from paper_2111_00847_amd import _lib
    L = _lib.lib()
    p16 = ctypes.c_void_p(16)
    assert L.lbm_bandwidth_probe(3, p16, p16, 1 << 20, 256, 1, None) == -4       # kind
    assert L.lbm_bandwidth_probe(-1, p16, p16, 1 << 20, 256, 1, None) == -4
    assert L.lbm_bandwidth_probe(2, p16, p16, (1 << 20) + 8, 256, 1, None) == -2  # not a multiple of 16
    assert L.lbm_bandwidth_probe(2, p16, p16, 1 << 20, 0, 1, None) == -2          # no workgroups
    assert L.lbm_bandwidth_probe(2, ctypes.c_void_p(24), p16, 1 << 20, 256, 1, None) == -2   # alignment
    assert L.lbm_bandwidth_probe(2, p16, None, 1 << 20, 256, 1, None) == -1       # copy without a source
    assert L.lbm_bandwidth_probe(0, None, p16, 1 << 20, 256, 1, None) == -1


def test_forced_batch_shape_is_validated_on_the_host(monkeypatch):
    """LBM_BATCH_SHAPE must name one of the tuner's shapes that the batch can
    run (16-row tiles in FP32 only; one node per thread for Cahn-Hilliard,
    corrected and local-gradient cases) and a grid >= 0: anything else makes
    lbm_batch_create return LBM_E_PARAM before any HIP call."""
    from paper_2111_00847_amd._lib import LbmParams, lib
    L = lib()
    f32, f64 = _params(dtype="f32"), _params(dtype="f64")
    ch = _params(dtype="f32", phase_eq="cahn_hilliard", phiB=-1.0)
    bad = [("16,8,0", f64), ("3,3,0", f32), ("8,4", f32), ("8,4,-1", f32), ("8,16,0", f32), ("x", f32),
           ("8,4,0", ch), ("16,16,0", ch)]
    for val, p in bad:
        monkeypatch.setenv("LBM_BATCH_SHAPE", val)
        h = ctypes.c_void_p()
        assert L.lbm_batch_create((LbmParams * 1)(p), 1, 1, ctypes.byref(h)) == -4, val
    for val, p in [("16,8,0", f32), ("4,4,7", f64), ("8,8,0", ch)]:
        monkeypatch.setenv("LBM_BATCH_SHAPE", val)
        h = ctypes.c_void_p()
        rc = L.lbm_batch_create((LbmParams * 1)(p), 1, 1, ctypes.byref(h))
        assert rc in (0, -6), val   # accepted (the device table needs a GPU: LBM_E_HIP without one)
        if rc == 0:
            assert L.lbm_batch_destroy(h) == 0
