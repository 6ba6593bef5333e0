"""The library's host code (argument checks, workspace planning, the early
error paths of the entry points) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host side only, and run over a grid of
configurations by a small driver (tests/host_sanitize_driver.cpp).  The
device code of the other sources is linked unchanged from the library's
build folder; nothing here runs on a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_02845_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_2009_02845_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-w", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout[-3000:]}\n{p.stderr[-3000:]}"
    return p


def test_host_code_under_asan_and_ubsan(tmp_path):
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    others = sorted(os.path.join(OBJ, f) for f in os.listdir(OBJ) if f.endswith(".o") and f != "api.o") \
        if os.path.isdir(OBJ) else []
    if not others:
        pytest.skip("library objects not built (run the package build first)")
    api = str(tmp_path / "api.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "drv")
    _run([HIPCC, *FLAGS, *SAN, "-c", os.path.join(CSRC, "api.hip"), "-o", api])
    _run([HIPCC, *FLAGS, *SAN, "-c", os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", drv])
    _run([HIPCC, "--offload-arch=gfx950", *SAN[:4], drv, api, *others, "-o", exe])
    env = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    p = _run([exe], env=env)
    assert "sanitized host checks:" in p.stdout and "runtime error" not in p.stderr, p.stderr[-3000:]
