"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The BVH builder (the library's host code that turns triangles into the
  4-wide quantized nodes the trace walks) is compiled with both sanitizers
  beside a checker (tests/native/bvh_check.cpp) that builds seeded scenes,
  degenerate ones included, and checks every node.
- The oracle is compiled with both sanitizers (PV_ORACLE_SANITIZE=1) and its
  pins run against it in a child process with the ASan runtime preloaded.
Any sanitizer report fails the test (errors are not recovered from).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _asan_runtime():
    try:
        path = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no ROCm clang++")
def test_bvh_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "bvh_check")
    subprocess.check_call([CLANG, "-std=c++17", "-O1", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(ROOT, "paper_2103_05875_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "bvh_check.cpp"),
                           os.path.join(ROOT, "paper_2103_05875_amd", "csrc", "bvh.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "every check passed" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None or _asan_runtime() is None, reason="no gcc ASan runtime")
def test_oracle_pins_under_sanitizers():
    env = dict(os.environ, PV_ORACLE_SANITIZE="1", LD_PRELOAD=_asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    subprocess.check_call([sys.executable, "-c", "import oracle; oracle.build()"], cwd=ROOT, env=env)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out
