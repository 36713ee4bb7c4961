"""Build the gfx950 shared library libnskr.so in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "nskr_lib.hip")
SO = os.path.join(HERE, "libnskr.so")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fused multiply-adds only where one source expression multiplies and
    # adds: every kernel instance (tile size, batched or not) then rounds
    # the same way
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
]


KERNELS = os.path.join(HERE, "csrc", "nskr_kernels.hpp")
# the launch layer: which kernel instance runs, its tile and cache hints
LAUNCH = os.path.join(HERE, "csrc", "nskr_lib.hip")


def _code_only(src: str) -> str:
    """The source without comments, trailing blanks and empty lines (the
    sources hold no string literal that contains a comment marker)."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def kernel_fingerprint() -> str:
    """sha256 over the device-kernel code and the launch layer that picks the
    instances, tiles and cache hints (comments excluded), and the compile
    flags: hardware counters taken for one fingerprint say nothing about
    kernels built or launched from another."""
    h = hashlib.sha256()
    for path in (KERNELS, LAUNCH):
        with open(path, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *FLAGS, "-o", SO + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
