"""Builds the HIP library ``liblbsc.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import hashlib
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lbsc.hip")
KERNEL_SOURCES = ["kernels.h", "kernels1.h", "lattice.h", "lbsc.hip"]
DEPS = [os.path.join(HERE, "csrc", f) for f in KERNEL_SOURCES] + [os.path.join(ROOT, "include", "lbsc.h")]
LIB = os.path.join(HERE, "liblbsc.so")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    # multiply-adds fuse only within one source expression, so every kernel
    # variant that runs the same device functions rounds identically
    "-ffp-contract=on",
]


def kernel_hash() -> str:
    """Hash of the kernel sources' code: comments and whitespace are dropped,
    so edits that change no code keep it (it tags tuning-cache entries and
    counter records)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    """Compile the library (always recompiles); returns its path."""
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", *FLAGS, f'-DLBSC_KERNEL_HASH="{kernel_hash()}"', "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
