"""Builds libsrmdp.so (HIP kernels + C ABI host runtime) for gfx950 in-tree.

    python -m paper_2407_21085_amd.build            # always compiles
    python -m paper_2407_21085_amd.build --if-stale # only when the sources changed
    python -m paper_2407_21085_amd.build --incremental  # reuse unchanged objects

This module imports nothing from the package's binding, so it runs on a tree
where the library has never been built.
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
           "srmdp_cv.hip", "srmdp_batch.hip", "srmdp_noalloc.hip", "srmdp_host.cpp"]

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


OBJ_CACHE = os.path.join(os.path.dirname(HERE), "_build", "objects")


def _unit_hash(src: str) -> str:
    """Hash of one unit: its own text, every header it may include, the flags."""
    import hashlib
    h = hashlib.sha256()
    h.update(" ".join(HIP_FLAGS[:-4]).encode())
    with open(os.path.join(CSRC, src), "rb") as f:
        h.update(f.read())
    for root in (CSRC, INCLUDE):
        for n in sorted(os.listdir(root)):
            if n.endswith((".h", ".hpp")):
                with open(os.path.join(root, n), "rb") as f:
                    h.update(n.encode() + f.read())
    return h.hexdigest()[:24]


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source and links libsrmdp.so next to this file, then
    records the hash of its sources beside it (libsrmdp.so.srchash).

    incremental=True reuses objects under _build/objects whose unit and
    headers are unchanged (a development aid; the default compiles all)."""
    with tempfile.TemporaryDirectory(prefix="srmdp_build_") as tmp:
        if incremental:
            os.makedirs(OBJ_CACHE, exist_ok=True)
            objs = [os.path.join(OBJ_CACHE, f"{s}.{_unit_hash(s)}.o") for s in SOURCES]
        else:
            objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        todo = [(s, o) for s, o in zip(SOURCES, objs) if not os.path.exists(o)]
        if verbose and incremental:
            print(f"compiling {[s for s, _ in todo]}", flush=True)

        def one(so):
            s, o = so
            _compile(s, o + ".part")
            os.replace(o + ".part", o)

        with ThreadPoolExecutor(max_workers=max(1, len(todo))) as ex:
            list(ex.map(one, todo))
        out_tmp = LIB_PATH + ".tmp"
        cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", out_tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("link of libsrmdp.so failed")
        os.replace(out_tmp, LIB_PATH)
    with open(STAMP_PATH + ".tmp", "w") as f:
        f.write(source_hash() + "\n")
    os.replace(STAMP_PATH + ".tmp", STAMP_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


STAMP_PATH = LIB_PATH + ".srchash"


def source_hash() -> str:
    """SHA-256 of every file under csrc/ and include/, this script and the flags.

    Content, not modification times: a copied or extracted tree keeps its
    hash, so a library built from the same sources is recognised as current."""
    import hashlib
    h = hashlib.sha256()
    h.update(" ".join(HIP_FLAGS[:-4]).encode())
    files = [os.path.abspath(__file__)]
    for root in (CSRC, INCLUDE):
        files += [os.path.join(root, n) for n in sorted(os.listdir(root))]
    for path in files:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def is_stale() -> bool:
    """True when libsrmdp.so is missing or was built from other sources."""
    if not os.path.exists(LIB_PATH) or not os.path.exists(STAMP_PATH):
        return True
    with open(STAMP_PATH) as f:
        return f.read().strip() != source_hash()


def ensure_built(verbose: bool = False) -> str:
    """Builds the library only when `is_stale()`; returns its path."""
    if is_stale():
        if verbose:
            print(f"building {LIB_PATH} (missing or built from other sources)", flush=True)
        return build(verbose=verbose)
    return LIB_PATH


if __name__ == "__main__":
    if "--if-stale" in sys.argv:
        ensure_built(verbose=True)
    else:
        build(verbose=True, incremental="--incremental" in sys.argv)
