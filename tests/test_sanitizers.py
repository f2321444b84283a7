"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle: oracle/lbm_oracle.c with oracle/sanitize_check.c, a driver that
  calls every entry point on lattices of every kind the oracle supports (one-
  and two-node-wide lattices, walls, both phase fields, the three models, the
  local gradient scheme, saved and reloaded states), built with gcc and both
  sanitizers, leak detection on.
* The library's host side: every csrc/*.hip compiled with the sanitizers on
  the host pass only (each -fsanitize= behind -Xarch_host; the GPU code, never
  launched here, unoptimised), linked with g++, and tests/sanitize_abi.c
  calling the size queries, parameter validation, null-pointer and alignment
  checks of every entry point -- calls that all return before any HIP call, so
  no GPU is needed.  Leak detection is off there: the HIP runtime keeps allocations
  until exit.

Each build happens in a temporary directory; nothing is written to the tree.
"""
import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    rc, out = _run(["gcc", "-std=c11", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "oracle", "sanitize_check.c"), os.path.join(ROOT, "oracle", "lbm_oracle.c"),
                    "-lm", "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    rc, out = _run([exe], env=env)
    print(out)
    assert rc == 0, out
    assert "ran clean" in out and "runtime error" not in out and "AddressSanitizer" not in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(HIPCC), reason="no host or HIP compiler")
def test_library_host_checks_under_asan_and_ubsan(tmp_path):
    host_san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer"):
        host_san += ["-Xarch_host", flag]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2111_00847_amd", "csrc", "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        # the GPU code is never launched here: built unoptimised, for speed
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
               "-Xarch_host", "-g", *host_san, "-c", src, "-o", obj]
        rc, out = _run(cmd, timeout=900)
        return obj, rc, out

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, srcs))
    for obj, rc, out in results:
        assert rc == 0, out
    lib = str(tmp_path / "liblbm_san.so")
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    rc, out = _run(["g++", "-shared", "-fsanitize=address,undefined", *[o for o, _, _ in results], "-L" + rocm_lib,
                    "-lamdhip64", "-Wl,-rpath," + rocm_lib, "-o", lib])
    assert rc == 0, out
    exe = str(tmp_path / "sanitize_abi")
    rc, out = _run(["gcc", *SAN, os.path.join(ROOT, "tests", "sanitize_abi.c"), "-L" + str(tmp_path), "-llbm_san",
                    "-Wl,-rpath," + str(tmp_path), "-lm", "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LBM_TWO_LEVEL", None)
    rc, out = _run([exe], env=env)
    print(out)
    assert rc == 0, out
    assert "ran clean" in out and "runtime error" not in out and "AddressSanitizer" not in out
