"""AddressSanitizer and UndefinedBehaviorSanitizer over the C ABI layer, on
the host: the ABI translation unit (api.cpp, pure host code) is compiled with
g++ and both sanitizers (every report fatal) and linked, with a driver
(tests/abi_sanitize.cpp), against the library's other objects as built. The
driver sizes workspaces over a grid of problems and at the documented size
limits (the plan arithmetic must neither overflow nor read out of bounds) and
runs every entry point's argument validation; no device is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1603_00561_amd")
BUILD = os.path.join(PKG, "_build")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def test_abi_layer_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    objs = sorted(os.path.join(BUILD, f) for f in os.listdir(BUILD)
                  if f.endswith(".o") and f != "api.o") if os.path.isdir(BUILD) else []
    if not objs:
        pytest.fail("library objects not built; run python -m paper_1603_00561_amd.build")
    inc = ["-I", os.path.join(ROOT, "include")]
    api = str(tmp_path / "api_san.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "abi_san")
    steps = [
        ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *inc, "-c",
         os.path.join(PKG, "csrc", "api.cpp"), "-o", api],
        ["g++", "-std=c++17", *SAN, *inc, "-c", os.path.join(ROOT, "tests", "abi_sanitize.cpp"),
         "-o", drv],
        ["g++", *SAN, "-static-libasan", drv, api, *objs, "-L/opt/rocm/lib", "-lamdhip64",
         "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert r.returncode == 0, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out
    assert "checks passed" in r.stdout
