"""CPU sanitizer leg: the oracle and the library's host code under
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The oracle (oracle/mg_oracle.c) is rebuilt with gcc -fsanitize=address,
  undefined and the oracle's pin tests run against that build in a child
  pytest (libasan preloaded into the interpreter).
* The library's host code -- argument validation, workspace carving, the
  Kmouflage background solver, the PM-step background lookup -- is rebuilt
  with the sanitizers on the host side only and driven by
  tests/sanitize/abi_host_driver.cpp, whose calls never reach the GPU.
Any sanitizer report aborts the child process and fails the test.
"""
import os
import subprocess
import sys

import pytest

from paper_2110_00566_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtime(name):
    return subprocess.check_output(["gcc", "-print-file-name=" + name], text=True).strip()


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "libmgoracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
                           "-ffp-contract=off", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-shared", "-fPIC", "-o", str(lib),
                           os.path.join(ROOT, "oracle", "mg_oracle.c"), "-lm"])
    env = dict(os.environ, MGORACLE_LIB=str(lib), LD_PRELOAD=_gcc_runtime("libasan.so"),
               OMP_NUM_THREADS="4", **SAN_ENV)
    tests = [os.path.join("tests", t) for t in
             ("test_oracle_transfer.py", "test_oracle_pins.py", "test_oracle_cycles.py",
              "test_oracle_adjoint_pm.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + tests, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1500)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2110_00566_amd", "csrc")
    exe = tmp_path / "abi_host_driver"
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    # sanitizers on the host side only (-Xarch_host before each option);
    # the device code is compiled as in the product build
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize", "abi_host_driver.cpp")] + \
          [os.path.join(csrc, f) for f in build.SOURCES] + ["-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=1200)
    r = subprocess.run([str(exe)], env=dict(os.environ, **SAN_ENV), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "host ABI checks passed" in r.stdout
