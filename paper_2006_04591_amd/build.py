"""Builds libshear.so (host C++ + gfx950 device code) in-tree with hipcc.

Each source compiles to an object of its own (in parallel), then one hipcc
link step makes the shared library."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libshear.so")
SOURCES = ["builder.cpp", "shear_api.cpp", "kernels.hip", "shrink.hip"]

FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_command(src: str, obj: str) -> list[str]:
    return [hipcc(), *FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]


def link_command(objs: list[str], out: str = LIB) -> list[str]:
    return [hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", out]


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory(prefix="shear_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        procs = [subprocess.Popen(compile_command(s, o), stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
                 for s, o in zip(SOURCES, objs)]
        failed = False
        for s, p in zip(SOURCES, procs):
            out, _ = p.communicate()
            if verbose or p.returncode != 0:
                sys.stderr.write(out)
            if p.returncode != 0:
                sys.stderr.write(f"hipcc failed compiling {s}\n")
                failed = True
        if failed:
            raise RuntimeError("hipcc failed building libshear.so")
        tmp = LIB + ".tmp"
        res = subprocess.run(link_command(objs, tmp), capture_output=True, text=True)
        if verbose or res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
        if res.returncode != 0:
            raise RuntimeError("hipcc failed linking libshear.so")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
