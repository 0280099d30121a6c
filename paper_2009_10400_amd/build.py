"""Build ``csrc/libtled.so`` for gfx950 with hipcc (in-tree, no JIT cache).

Usage: ``python -m paper_2009_10400_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(CSRC, "libtled.so")
SOURCES = ["setup.cpp", "kernels.hip", "api.hip", "mlp.hip", "copy.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-pthread", "-Wno-unused-command-line-argument"]


# The solver kernels fuse a multiply and an add only inside one source expression
# (-ffp-contract=on), never across statements: every instantiation of a kernel
# (single problem, batch, persistent batch) then rounds the same way, which keeps a
# batch's scenarios equal bit for bit to their single runs.
SOURCE_FLAGS = {"kernels.hip": ["-ffp-contract=on"]}


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "c++"]
        cmd = [HIPCC] + HIP_FLAGS + SOURCE_FLAGS.get(src, []) + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


# Sources of the solver's kernels and of the set-up that lays out their data:
# counter measurements of those kernels stay valid while these are unchanged.
SOLVER_SOURCES = ("device_math.h", "kernels.h", "kernels.hip", "setup.cpp", "tled_internal.h")


def source_digest(names=SOLVER_SOURCES) -> str:
    """Hash of library sources and of the flags they are compiled with (ties counter
    measurements to the kernels that produced them)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(names):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
        h.update(repr((HIP_FLAGS, SOURCE_FLAGS.get(name, []))).encode())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
