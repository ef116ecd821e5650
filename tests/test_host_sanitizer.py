"""The C ABI's host-side argument checks and size queries under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: the sanitizers apply to the host pass of hipcc).
mc_abi.cpp and mc_timing.cpp are rebuilt instrumented and linked with the library's other
objects and tests/asan_driver.cpp, which calls every entry point with arguments the checks
reject (no device work) and queries every workspace size over a grid that includes the edges
of each accepted range and sizes whose products overflow int64."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2606_06329_amd")
BUILD = os.path.join(PKG, "_build")
INSTRUMENTED = ("mc_abi.cpp", "mc_timing.cpp")


def test_host_paths_under_asan_and_ubsan(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    if not os.path.isdir(BUILD):
        from paper_2606_06329_amd.build import build
        build()
    objs = [os.path.join(BUILD, f) for f in sorted(os.listdir(BUILD))
            if f.endswith(".o") and f[:-2] not in INSTRUMENTED]
    assert objs, "library objects missing"
    exe = str(tmp_path / "asan_driver")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-x", "hip", *san,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"),
           *[os.path.join(PKG, "csrc", f) for f in INSTRUMENTED],
           os.path.join(ROOT, "tests", "asan_driver.cpp"), "-x", "none", *objs, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "0 failures" in r.stdout
