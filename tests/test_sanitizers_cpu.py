"""Host sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer) of
the oracle and of the C-ABI's argument validation, run on the CPU.

* The oracle's C sources with a driver that calls every entry point on a
  small grid with voids, and a PCG solve to 1e-10.
* The library (host code instrumented; device code is not: the flags are
  given to the host pass only) with a driver that passes invalid arguments
  to every entry point; validation refuses them before any device call, so
  no GPU is needed.
Any sanitizer report ends the driver with a non-zero status."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c99", *SAN, os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "elas3d_oracle.c"),
          os.path.join(ROOT, "oracle", "microstructure_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "ok 1" in r.stdout and "ERROR" not in r.stderr


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_abi_validation_under_address_and_ub_sanitizers(tmp_path):
    from paper_2602_07354_amd import build as B
    objs = []
    for src in B.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        # sanitizers on the host pass only (-Xarch_host before each flag)
        host_san = [f for s in SAN[:3] for f in ("-Xarch_host", s)]
        _run([B.HIPCC, f"--offload-arch={B.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC", *host_san,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", B.CSRC, "-c", os.path.join(B.CSRC, src), "-o", obj])
        objs.append(obj)
    lib = str(tmp_path / "libelas3d_san.so")
    _run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address,undefined",
          "-o", lib, *objs])
    exe = str(tmp_path / "abi_san")
    # the library carries clang's sanitizer runtime references: link the driver with clang too
    clang = os.path.join(os.path.dirname(os.path.realpath(B.HIPCC)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    _run([clang, *SAN, "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "abi_driver.c"), lib,
          "-Wl,-rpath," + str(tmp_path), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "ok (0 failures)" in r.stdout
