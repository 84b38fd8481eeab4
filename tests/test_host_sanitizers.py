"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every source of libgsw is compiled with the sanitizers on its host code only
(device code is built as usual and never runs here), linked into
``tests/sanitize/host_driver.cpp``, and run on the CPU: graph validation on
good and malformed CSRs, graph features of random symmetric and directed
graphs, tree creation, the JSON tree reader on the shipped trees and on every
truncation of a small document, names and option defaults.  Needs no GPU.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_01159_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_HOST = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=undefined"
SAN = "-fsanitize=address,undefined -fno-sanitize-recover=undefined"
BASE = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-I" + os.path.join(ROOT, "include")]
HOSTINC = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(HIPCC)), reason="ROCm toolchain not found")
def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_1708_01159_amd import build

    jobs = []
    for src in build.SOURCES:
        obj = str(tmp_path / (src + ".o"))
        path = os.path.join(CSRC, src)
        if src.endswith(".hip"):
            jobs.append([HIPCC, "-x", "hip"] + DEVICE + BASE + SAN_HOST.split() + ["-c", path, "-o", obj])
        else:
            jobs.append([CLANG, "-x", "c++"] + BASE + HOSTINC + SAN.split() + ["-c", path, "-o", obj])
    drv = str(tmp_path / "driver.o")
    jobs.append([CLANG] + BASE + HOSTINC + SAN.split()
                + ["-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", drv])
    with ThreadPoolExecutor(4) as ex:
        list(ex.map(_run, jobs))
    exe = str(tmp_path / "host_driver")
    objs = [str(tmp_path / (s + ".o")) for s in build.SOURCES] + [drv]
    _run([CLANG] + SAN.split() + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                                         "-fopenmp", "-o", exe])
    trees = os.path.join(ROOT, "paper_1708_01159_amd", "trees")
    env = dict(os.environ, GSW_SAN_TMP=str(tmp_path), HIP_VISIBLE_DEVICES="",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, os.path.join(trees, "seed.json"), os.path.join(trees, "mi355x.json")],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-3000:] + r.stderr[-6000:]
