"""Build libmpsim.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2511_23438_amd.build  (or call build()).
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpsim.so")
STAMP = LIB + ".srchash"   # hash of the sources and flags the library was built from
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
ARCH = os.environ.get("MPSIM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-pthread",
    # keep hipcc from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def source_hash() -> str:
    """sha256 over every file under csrc/, the public header and the flags."""
    h = hashlib.sha256()
    files = sorted(os.listdir(CSRC))
    for f in files:
        path = os.path.join(CSRC, f)
        if os.path.isfile(path) and f.endswith((".hip", ".cpp", ".h")):
            h.update(f.encode())
            with open(path, "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(HERE, "..", "include", "mpsim.h"), "rb") as fh:
        h.update(fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()


def is_current() -> bool:
    """True when libmpsim.so exists and was built from the current sources."""
    if not (os.path.exists(LIB) and os.path.exists(STAMP)):
        return False
    with open(STAMP) as fh:
        return fh.read().strip() == source_hash()


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = ["hipcc"] + HIPCC_FLAGS + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    with open(STAMP, "w") as fh:
        fh.write(source_hash() + "\n")
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
