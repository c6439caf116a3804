"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

1. The library's host runtime (srmdp_host.cpp, srmdp_rtc.cpp) compiled with
   both sanitizers (host side only; the device units are the normal build's),
   loaded in a process that starts with the sanitizer runtime, must pass the
   ABI host checks: argument validation, sizes, refused combinations and error
   strings, none of which needs a GPU.
2. The oracle compiled with both sanitizers (gcc) must pass its pins: the
   regression, generator, flip-bound, network and problem-plugin tests.

A sanitizer report aborts the child process (halt_on_error), so a clean exit
with every test passed is the check.  The instrumented builds go to a
temporary directory; nothing under paper_2407_21085_amd/ or oracle/ changes.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer"]
ORACLE_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _runtime(cmd):
    path = subprocess.run(cmd, capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"no sanitizer runtime from {' '.join(cmd)}")
    return path


def _pytest(files, env, marker="not gpu"):
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", marker, "-p", "no:cacheprovider"] + files
    res = subprocess.run(cmd, cwd=ROOT, env=dict(os.environ, PYTHONDONTWRITEBYTECODE="1", **ENV, **env),
                         capture_output=True, text=True)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_host_runtime_under_sanitizers(tmp_path):
    import paper_2407_21085_amd.build as B
    rt = _runtime([os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang"),
                   "-print-file-name=libclang_rt.asan-x86_64.so"])
    lib = B.build(extra_flags=HOST_FLAGS, out_path=str(tmp_path / "libsrmdp.so"))
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "the host units are not instrumented"
    out = _pytest(["tests/test_abi_host.py"], {"LD_PRELOAD": rt, "SRMDP_LIBRARY": lib})
    assert " passed" in out


def test_oracle_under_sanitizers(tmp_path):
    import oracle as O
    rt = _runtime(["gcc", "-print-file-name=libasan.so"])
    lib = O.compile_source(O._SRC, str(tmp_path / "libsrmdp_oracle.so"), ORACLE_FLAGS)
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "the oracle is not instrumented"
    out = _pytest(["tests/test_oracle_regression.py", "tests/test_oracle_rng.py", "tests/test_oracle_flip_bound.py",
                   "tests/test_oracle_mlp.py", "tests/test_oracle_model.py"],
                  {"LD_PRELOAD": rt, "SRMDP_ORACLE_LIBRARY": lib})
    assert " passed" in out
