"""Compile the HIP library in-tree for gfx950: paper_1901_02330_amd/libvem_mi355x.so.

Usage: python -m paper_1901_02330_amd.build  (or __graft_entry__.build()).
Each .hip source is compiled to an object under _build/ (in parallel), then
linked into one shared library exporting the C ABI declared in include/vem.h.
The plain-C test program of that ABI (tests/capi_c/cube_solve) is then built
against it with gcc.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libvem_mi355x.so")
SOURCES = ["mesh.hip", "element_lo.hip", "element_paper.hip", "assemble.hip", "sell.hip", "krylov.hip", "pcg.hip", "schwarz.hip", "capi.hip"]
ARCH = os.environ.get("VEM_OFFLOAD_ARCH", "gfx950")

CFLAGS = [
    "-O3",
    "-fPIC",
    "-std=c++17",
    f"--offload-arch={ARCH}",
    "-mcode-object-version=5",
    # packed FP32 instructions stay off (plain FP32/FP64 code only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [hipcc(), *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l and "(ignoring feature)" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build_c_driver(verbose: bool = True) -> str:
    """Compile tests/capi_c/cube_solve.c, a plain-C test program of the ABI, with gcc against the
    built library (the library is found next to the package through the binary's run path)."""
    src = os.path.join(ROOT, "tests", "capi_c", "cube_solve.c")
    out = os.path.join(ROOT, "tests", "capi_c", "cube_solve")
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", f"-I{INCLUDE}",
           "-I/opt/rocm/include", src, "-o", tmp, f"-L{PKG}", "-l:libvem_mi355x.so", "-L/opt/rocm/lib",
           "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN/../../paper_1901_02330_amd", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed for the C driver:\n" + r.stderr)
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
           "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    build_c_driver(verbose)
    return LIB


if __name__ == "__main__":
    build()
