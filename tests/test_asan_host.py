"""Host AddressSanitizer + UBSan builds (CPU): the oracle, and the library's
host-side assembly (the operators built at mesh upload and the locality order
of the potential rows), each compiled with its driver under
-fsanitize=address,undefined and run on small Kuhn-split meshes. The run must
finish with status 0 and no sanitizer report (invalid access, leak or
undefined behaviour). Device code is not instrumented: GPU sanitizers are
not available on the target machines."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN = os.path.join(ROOT, "tests", "asan")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd_build, exe):
    r = subprocess.run(cmd_build, capture_output=True, text=True, timeout=600)
    if r.returncode != 0 and ("libasan" in r.stderr or "cannot find" in r.stderr):
        pytest.skip("sanitizer runtime not installed: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_sanitizer(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    out = _run(["gcc", "-std=c11", "-ffp-contract=off"] + SAN + [os.path.join(ASAN, "oracle_driver.c"), "-o", exe,
                                                                 "-lm"], exe)
    assert "minimize rc 0" in out and "curve rc 0" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the HIP headers not found")
def test_host_assembly_under_address_sanitizer(tmp_path):
    exe = str(tmp_path / "assemble_asan")
    csrc = os.path.join(ROOT, "paper_1801_03690_amd", "csrc")
    out = _run(["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", csrc, "-I",
                                              os.path.join(ROOT, "include"), os.path.join(ASAN, "assemble_driver.cpp"),
                                              os.path.join(csrc, "assemble.cpp"), "-o", exe, "-lpthread"], exe)
    assert "order identity" in out and "order tiled" in out
