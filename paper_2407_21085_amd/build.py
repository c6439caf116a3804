"""Builds libsrmdp.so (HIP kernels + C ABI host runtime) for gfx950 in-tree.

    python -m paper_2407_21085_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB_NAME = "libsrmdp.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)

SOURCES = ["srmdp_kernels.hip", "srmdp_kernels_gr.hip", "srmdp_kernels_ep.hip", "srmdp_kernels_hd.hip",
           "srmdp_kernels_hd2.hip", "srmdp_kernels_hd3.hip",
           "srmdp_cv.hip", "srmdp_batch.hip", "srmdp_host.cpp"]

# Packed FP32 instructions are kept out of the device code on purpose: some
# of their forms have produced wrong results on this hardware.
HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src: str, obj: str) -> None:
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc()] + HIP_FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def build(verbose: bool = False) -> str:
    """Compiles every source and links libsrmdp.so next to this file."""
    with tempfile.TemporaryDirectory(prefix="srmdp_build_") as tmp:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            list(ex.map(_compile, SOURCES, objs))
        out_tmp = LIB_PATH + ".tmp"
        cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", out_tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("link of libsrmdp.so failed")
        os.replace(out_tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
