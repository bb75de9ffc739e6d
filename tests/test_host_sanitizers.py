"""CPU: the host code of both C ABIs under AddressSanitizer and
UndefinedBehaviorSanitizer.

The runtimes are compiled with the sanitizers on the host side only (nothing
here launches a kernel), linked with
tests/sanitize/abi_driver.cpp, and run: every configuration, validation and
sizing path, the FP64 S-parameter combination and the argument checks of the
device entry points.  Any sanitizer report or failed check fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_14176_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_code_under_asan_and_ubsan():
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    os.makedirs(OUT, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-g", "-O1"]
    objs = []
    for src in (os.path.join(CSRC, "yee_runtime.hip"), os.path.join(CSRC, "raymeta.hip"),
                os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp")):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        # device code is compiled as usual (the objects carry it) but never runs here
        cmd = [hipcc, "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-std=c++17", "-fPIC", *san, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = os.path.join(OUT, "abi_driver")
    cmd = [hipcc, *san, *objs, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert "ok: 0 failed checks" in out
