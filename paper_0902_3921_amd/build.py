"""Build ``libhlb.so`` (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhlb.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = [os.path.join(CSRC, "hlb_api.hip"), os.path.join(CSRC, "hlb_noalloc.hip"), os.path.join(CSRC, "sur_api.hip")]
HEADERS = [os.path.join(CSRC, h) for h in ("kernels.hpp", "lattice.hpp", "sur_kernels.hpp")] + [
    os.path.join(ROOT, "include", h) for h in ("hlb.h", "sur.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay disabled (hipcc's host pass warns that it
    # does not know the feature; harmless)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    # an undefined symbol fails the link, not the first load of the library
    "-Wl,-z,defs",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def source_hash() -> str:
    """SHA-256 of the library sources (kernels, host code, C header)."""
    import hashlib

    h = hashlib.sha256()
    for path in sorted(SOURCES + HEADERS):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
