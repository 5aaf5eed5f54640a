"""Builds libxdrop.so (gfx950) in-tree.

The HIP sources are compiled with hipcc for gfx950 only and linked against the
HIP runtime that PyTorch ships, so that the library and torch share one
runtime in a process (device pointers and streams from torch are then valid
in the library).
"""
from __future__ import annotations

import os
import subprocess
import sys
import sysconfig

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libxdrop.so")
ARCH = os.environ.get("XD_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 VALU forms anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def torch_lib_dir() -> str:
    """Directory of the HIP runtime bundled with torch (found without importing torch)."""
    purelib = sysconfig.get_paths()["purelib"]
    for base in [purelib] + sys.path:
        cand = os.path.join(base, "torch", "lib")
        if os.path.exists(os.path.join(cand, "libamdhip64.so")):
            return cand
    raise RuntimeError("torch's libamdhip64.so not found")


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith((".hip", ".h"))] + [os.path.join(INCLUDE, "xdrop.h")]


def source_hash() -> str:
    """sha256 over the library's sources and header (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    for path in sources():
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, "xd_lib.o")
    cmd = ["hipcc"] + HIPCC_FLAGS + [f"-I{INCLUDE}", f"-I{CSRC}", "-c",
                                    os.path.join(CSRC, "xd_lib.hip"), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    tl = torch_lib_dir()
    tmp = LIB + ".tmp%d" % os.getpid()
    link = ["g++", "-shared", "-o", tmp, obj, f"-L{tl}", "-l:libamdhip64.so",
            f"-Wl,-rpath,{tl}", "-Wl,--no-undefined"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    build()
