"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code
(no GPU needed): the oracle with its own driver (tests/san_oracle.c), and the
library's host code -- workspace plan and serving scheduler with an executor
callback -- with tests/san_server.cpp.  The library is compiled for gfx950 as
usual, with the sanitizers on the host side only.  A run passes when the
driver reports ok and the sanitizers stay silent."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1304_1864_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe, what):
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0, out.stdout + out.stderr
    assert f"{what} sanitizer run: ok" in out.stdout
    assert "runtime error" not in out.stderr and "ERROR: AddressSanitizer" not in out.stderr


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "san_oracle")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "oracle.c"),
                           os.path.join(HERE, "san_oracle.c"), "-o", exe, "-lm"])
    env_leaks = dict(ENV, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")  # libgomp's pools
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env_leaks)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "oracle sanitizer run: ok" in out.stdout


@pytest.mark.slow
def test_host_code_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "san_server")
    from paper_1304_1864_amd import build

    srcs = [os.path.join(CSRC, f) for f in build.SOURCES]
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-omit-frame-pointer",
                           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs,
                           os.path.join(HERE, "san_server.cpp"), "-o", exe, *build.LIBS],
                          stderr=subprocess.DEVNULL)
    _run(exe, "host")
