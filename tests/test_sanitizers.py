"""AddressSanitizer and UndefinedBehaviorSanitizer builds, on the CPU.

- The FP64 oracles (2-D and 3-D) with every entry point, every scheme and
  every boundary kind (tests/sanitize/oracle_driver.c).
- The C ABI's host code (argument checks, workspace arithmetic, the failure
  paths of sts_create) with the kernel launchers replaced by host stand-ins
  (tests/sanitize/abi_driver.c, launch_stubs.hip): the GPU code itself is not
  instrumented (sanitizers are applied to the host side only).
Any invalid access, leak or undefined operation fails the run.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracles_under_sanitizers(tmp_path):
    exe = str(tmp_path / "ora_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fopenmp", "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"),
          "-o", exe, os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "ora.c"),
          os.path.join(ROOT, "oracle", "ora3.c"), "-lm"])
    r = _run([exe], env=ENV, timeout=600)
    assert r.stdout.strip().endswith("OK"), r.stdout[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    assert r.stdout.count("2-D") == 12 and r.stdout.count("3-D") == 8


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None,
                    reason="needs hipcc and g++")
def test_abi_host_code_under_sanitizers(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
    api_o, stub_o = str(tmp_path / "api.o"), str(tmp_path / "stubs.o")
    drv_o, exe = str(tmp_path / "drv.o"), str(tmp_path / "abi_san")
    _run([HIPCC, *common, *san, "-c", os.path.join(ROOT, "paper_1802_04243_amd", "csrc", "sts_api.hip"),
          "-o", api_o])
    _run([HIPCC, *common, *san, "-c", os.path.join(SAN, "launch_stubs.hip"), "-o", stub_o])
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), "-c", os.path.join(SAN, "abi_driver.c"), "-o", drv_o])
    _run(["g++", "-fsanitize=address,undefined", "-o", exe, drv_o, api_o, stub_o,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    r = _run([exe], env=ENV, timeout=300)
    print(r.stdout)
    assert r.stdout.strip().endswith("OK"), r.stdout[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-2000:]
