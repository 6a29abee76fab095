"""Host sanitizers: the CPU oracle, and the library's host code (planners,
tuning, argument checks, the scratch-cache policy) with the CPU emulator of
the tile programs, built with AddressSanitizer and UndefinedBehaviorSanitizer
(host side only; no device code is instrumented and no GPU is touched) and
run through every host-only entry point.  Any finding aborts the driver."""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "san_oracle")
    _run(["g++", "-O1", "-g", "-std=c++17", "-pthread", *SAN,
          os.path.join(HERE, "sanitize_oracle_driver.cpp"),
          os.path.join(ROOT, "oracle", "bitonic_oracle.cpp"), "-o", exe])
    assert _run([exe], env=ENV).stdout.strip() == "ok"


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    objs = [o for o in glob.glob(os.path.join(ROOT, "_build", "*.o"))
            if os.path.basename(o) != "api.hip.o"]
    if not os.path.exists(hipcc) or not objs:
        pytest.skip("needs hipcc and the library's objects (__graft_entry__.build())")
    inc = os.path.join(ROOT, "include")
    api = str(tmp_path / "api_san.o")
    # sanitizers on the host pass only: each -fsanitize= follows -Xarch_host
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++20", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san,
          "-I", inc, "-c", os.path.join(ROOT, "paper_1506_01446_amd", "csrc", "api.hip"),
          "-o", api])
    emu = str(tmp_path / "emu.o")
    drv = str(tmp_path / "drv.o")
    _run(["g++", "-O1", "-g", "-std=c++20", *SAN, "-I", inc, "-c",
          os.path.join(HERE, "cpu_program_emulator.cpp"), "-o", emu])
    _run(["g++", "-O1", "-g", "-std=c++20", *SAN, "-I", inc, "-c",
          os.path.join(HERE, "sanitize_host_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "san_host")
    _run(["g++", *SAN, drv, emu, api, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    assert _run([exe], env=ENV).stdout.strip() == "ok"
