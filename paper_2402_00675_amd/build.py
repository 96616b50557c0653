"""Builds libmont.so (the HIP library) for gfx950 in-tree.

    python -m paper_2402_00675_amd.build

Every source is compiled with hipcc for gfx950 only, objects go to
``_build/`` at the repository root, and the shared libraries are written next
to this file, where the Python binding loads them: ``libmont.so`` and
``libmont_debug.so`` (the same library with MONT_DEBUG precondition counters).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmont.so")
ARCH = "gfx950"

SOURCES = [
    "mont_k16.hip",
    "mont_k32.hip",
    "mont_k64.hip",
    "mont_ragged.hip",
    "mont_ref.hip",
    "mont_crt.hip",
    "mont_ntt.hip",
    "mont_valu.hip",
    "mont_capi.cpp",
    "mont_setup.cpp",
    "mont_serve.cpp",
    "mont_tunecache.cpp",
    "mont_noalloc.hip",
]

# The MONT_DEBUG library: these sources again with -DMONT_DEBUG (precondition
# counters ahead of every call), the rest shared with the release build.
LIB_DEBUG = os.path.join(PKG, "libmont_debug.so")
DEBUG_SOURCES = ["mont_capi.cpp", "mont_ragged.hip", "mont_crt.hip", "mont_ntt.hip", "mont_serve.cpp",
                 "mont_noalloc.hip", "mont_debug.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # never let the compiler form packed-FP32 instructions (see DESIGN notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src: str, debug: bool = False) -> str:
    obj = os.path.join(BUILD, "debug" if debug else "", os.path.splitext(src)[0] + ".o")
    extra = ["-DMONT_DEBUG"] if debug else []
    cmd = [HIPCC, "-x", "hip", *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def _link(objs: list, lib: str) -> None:
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, lib)


def build(jobs: int | None = None) -> str:
    """Compile every HIP/C++ source, link libmont.so and libmont_debug.so; returns the former's path."""
    os.makedirs(os.path.join(BUILD, "debug"), exist_ok=True)
    jobs = jobs or 8
    units = [(src, False) for src in SOURCES] + [(src, True) for src in DEBUG_SOURCES]
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(*u), units))
    rel = objs[:len(SOURCES)]
    dbg = dict(zip(DEBUG_SOURCES, objs[len(SOURCES):]))
    _link(rel, LIB)
    _link([dbg.get(src, o) for src, o in zip(SOURCES, rel)] + [dbg["mont_debug.hip"]], LIB_DEBUG)
    return LIB


if __name__ == "__main__":
    print(build())
