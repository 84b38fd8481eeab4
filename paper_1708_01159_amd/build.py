"""Builds libgsw.so (HIP for gfx950) and the host graph generators, in-tree.

    python -m paper_1708_01159_amd.build
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsw.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("GSW_OFFLOAD_ARCH", "gfx950")
SOURCES = ["gsw_kernels.hip", "gsw_core.cpp", "gsw_bfs.cpp", "gsw_msbfs.hip", "gsw_noalloc.hip", "gsw_cc.hip"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]
# Device code: gfx950 only, no packed-fp32 instruction selection.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def source_digest() -> str:
    """SHA-256 (first 16 hex digits) of every file libgsw.so is built from:
    the library sources, the internal headers and include/gsw.h.  The build
    stamps it into the library (gsw_source_digest); the binding refuses a
    library whose stamp differs from the sources beside it."""
    h = hashlib.sha256()
    files = sorted(SOURCES + [f for f in os.listdir(CSRC) if f.endswith(".h")])
    for f in files:
        h.update(f.encode() + b"\0")
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "gsw.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src: str, digest: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    lang = ["-x", "hip"] + DEVICE if src.endswith(".hip") else ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    cmd = [HIPCC] + COMMON + lang + ['-DGSW_SOURCE_DIGEST="%s"' % digest, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build_gsw() -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    digest = source_digest()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, digest), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-Wl,-rpath,/opt/rocm/lib", "-L/opt/rocm/lib", "-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


MODEL_LIB = os.path.join(HERE, "libgswmodel.so")


def build_model() -> str:
    """The host library of the benchmark's byte-model counts (g++, OpenMP)."""
    tmp = MODEL_LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", os.path.join(CSRC, "traffic_model.cpp"),
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, MODEL_LIB)
    return MODEL_LIB


def build_all() -> None:
    from . import graphgen

    graphgen.build(force=True)
    build_gsw()
    build_model()


if __name__ == "__main__":
    build_all()
    print("built", LIB, file=sys.stderr)
