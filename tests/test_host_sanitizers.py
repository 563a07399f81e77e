"""The host side of the C ABI (problem validation, workspace layouts, batch
preparation and tile maps, error paths of every entry point) fuzzed under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.  The harness
(tests/host/fuzz_host.cpp) never reaches a HIP call.  The sanitizers are
applied to host code only; the binary is cached by a hash of its sources."""
import hashlib
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
SOURCES = ["tests/host/fuzz_host.cpp", "paper_2207_05258_amd/csrc/hweno_kernels.hip",
           "paper_2207_05258_amd/csrc/hweno_math.h", "paper_2207_05258_amd/csrc/hweno_adjoint.h",
           "include/hweno.h"]


def _binary():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    h = hashlib.sha256()
    for s in SOURCES:
        with open(os.path.join(ROOT, s), "rb") as fh:
            h.update(fh.read())
    out_dir = os.path.join("/tmp", "hweno_host_fuzz", h.hexdigest()[:16])
    exe = os.path.join(out_dir, "fuzz_host")
    if not os.path.exists(exe):
        os.makedirs(out_dir, exist_ok=True)
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-Xarch_host", "-g",
               "-fno-omit-frame-pointer",
               "-Xarch_host", "-fsanitize=address",
               "-Xarch_host", "-fsanitize=undefined",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-std=c++17", "-I", os.path.join(ROOT, "include"),
               os.path.join(ROOT, SOURCES[0]), os.path.join(ROOT, SOURCES[1]), "-o", exe + ".tmp"]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=1200)
        assert r.returncode == 0, r.stderr[-3000:]
        os.replace(exe + ".tmp", exe)
    return exe


def test_host_code_is_clean_under_asan_and_ubsan():
    exe = _binary()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert " 0 failures" in r.stdout, r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
