"""Build the HIP library libmhsk.so for gfx950 (in-tree)."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhsk.so")
SOURCES = ["kernels.hip", "engine.cpp", "abi.cpp", "server.cpp", "static_run.cpp"]
ARCH = os.environ.get("MHSK_ARCH", "gfx950")

# Packed FP32 instructions are kept out of every code object.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def source_files():
    """Every file the library is compiled from: the sources, their headers
    and the public header."""
    root = os.path.dirname(HERE)
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    return [os.path.join(CSRC, f) for f in names] + [os.path.join(root, "include", "mhsk.h")]


def source_sha() -> str:
    """First 16 hex digits of the SHA-256 over the source files (name and
    contents, in name order); the build stamps it into mhs_version()."""
    h = hashlib.sha256()
    for path in source_files():
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    sha = source_sha()
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        flags = HIP_FLAGS + [f'-DMHSK_SOURCE_SHA="{sha}"']
        cmd = [hipcc] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip"] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        errs = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
        if verbose and errs.strip():
            print(errs)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.unlink(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
