"""Build libflashrad.so (HIP for gfx950) in-tree.

Compiles every translation unit of the library under csrc/ with hipcc for
gfx950 and links them into paper_2609_19190_amd/libflashrad.so; builds the
peak-measurement library libfrpeaks.so (csrc/peaks.hip, used by the
benchmark's roofline) beside it.  Always rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libflashrad.so")
PEAKS_LIB = os.path.join(HERE, "libfrpeaks.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
         # no packed FP32 instructions in any generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = ["discretise.hip", "map_kernel.hip", "generic_kernel.hip", "api.cpp", "batch.cpp", "server.cpp",
           "scalar.cpp"]
PEAKS_SOURCE = "peaks.hip"
INCLUDE = os.path.join(os.path.dirname(HERE), "include")


def source_hash() -> str:
    """First 16 hex digits of the SHA-256 over the library's sources (every
    csrc/*.hip, *.cpp, *.h and include/*.h, by name): compiled into the
    library, returned by fr_source_hash(), so a caller can tell whether the
    built library matches the tree."""
    import hashlib

    h = hashlib.sha256()
    files = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".cpp", ".h"))]
    files += [os.path.join(INCLUDE, f) for f in sorted(os.listdir(INCLUDE)) if f.endswith(".h")]
    for f in files:
        h.update(os.path.basename(f).encode() + b"\0")
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str, defines=()) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *FLAGS, *defines, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of {os.path.basename(lib)} failed:\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + [PEAKS_SOURCE]
    stamp = [f'-DFR_SOURCE_HASH="{source_hash()}"']
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(lambda f: _compile(f, stamp if f == "api.cpp" else ()), srcs))
    _link(objs[:len(SOURCES)], LIB)
    _link(objs[len(SOURCES):], PEAKS_LIB)
    if verbose:
        print("built", LIB, "and", PEAKS_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
