"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer:
parameter validation, plans and workspace layouts of every admitted size
and of ragged batches, the per-pass twiddle tables of both schedules, and
the tuning cache's reader and writer (round trip, malformed files).  The
checks (tests/host/host_checks.hip) include the runtime's source and run on
the CPU; the sanitizers instrument the host pass only, with libstdc++'s
bounds assertions on."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2508_06678_amd")


def _hipcc():
    c = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return c if os.path.exists(c) else shutil.which("hipcc")


@pytest.mark.skipif(_hipcc() is None, reason="needs hipcc")
def test_host_runtime_under_sanitizers(tmp_path):
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    exe = str(tmp_path / "host_checks")
    cmd = [_hipcc(), "-std=c++17", "-O1", "-g", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-D_GLIBCXX_ASSERTIONS",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "host_checks.hip"),
           "-o", exe, "-L", PKG, "-lqg", "-Wl,-rpath," + PKG,
           "-L", rocm_lib, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + rocm_lib]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host checks ok" in r.stdout
