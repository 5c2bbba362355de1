"""Sanitizer builds of the host code (CPU only, no GPU needed).

* The library's host logic (C-ABI validation, workspace sizing, the batch
  schedule planner over random problem sets and every compiled tile, the
  barrier-limit and no-allocation size checks): api.cpp, api_batch.cpp,
  api_surrogate.cpp and stage.hip compiled for the host alone with
  AddressSanitizer + UndefinedBehaviorSanitizer (the kernel launch wrappers
  replaced by stand-ins, tests/sanitize/device_stubs.cpp) and driven by
  tests/sanitize/host_driver.cpp.
* The FP64 oracle (oracle/nlse_oracle.c) built the same way with gcc and
  driven over every entry point, scheme, boundary condition and dimension by
  tests/sanitize/oracle_driver.c.
A sanitizer report or a failed check makes the driver exit non-zero."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1203_1263_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, cwd=None):
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=cwd, env=ENV, timeout=600)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="ROCm toolchain missing")
def test_host_runtime_under_asan_ubsan(tmp_path):
    srcs = [os.path.join(CSRC, f) for f in ("api.cpp", "api_batch.cpp", "api_surrogate.cpp", "stage.hip")]
    srcs += [os.path.join(SAN, "device_stubs.cpp"), os.path.join(SAN, "host_driver.cpp")]
    # host-only compilation; the sanitizers apply to the host pass alone
    flags = ["-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-Xarch_host",
             "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=6) as ex:
        list(ex.map(lambda so: _run([HIPCC] + flags + ["-c", so[0], "-o", so[1]]), zip(srcs, objs)))
    exe = str(tmp_path / "host_driver")
    _run([CLANGXX, "-fsanitize=address,undefined"] + objs + ["-L/opt/rocm/lib", "-lamdhip64",
                                                              "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], cwd=str(tmp_path))
    assert "sanitized host checks passed" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=all", "-ffp-contract=off", os.path.join(ROOT, "oracle", "nlse_oracle.c"),
          os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], cwd=str(tmp_path))
    assert "sanitized oracle checks passed" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
