"""Build libabc_dtn.so in-tree with hipcc for gfx950.

Usage: ``python -m paper_1908_02456_amd.build`` (or ``__graft_entry__.build()``).
Objects go to ``paper_1908_02456_amd/_build``; the library is written next
to this file.  Every call recompiles all sources.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libabc_dtn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["abi.cpp", "setup.cpp", "setup_box.cpp", "kernels_staged.hip", "fused.hip", "adjoint.hip", "h2.hip", "poisson.hip"]

# no packed-FP32 instructions in device code; host pass ignores the feature
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-I" + CSRC,
          "-I" + os.path.join(os.path.dirname(HERE), "include")]


# Host-code check build: the same sources with the host side instrumented by
# AddressSanitizer and UndefinedBehaviorSanitizer (device code as usual).  It
# serves host-only tests (calls that fail or finish before a device is
# touched); load it with the ASan runtime preloaded.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]
HOSTSAN_DIR = os.path.join(BUILD, "hostsan")
HOSTSAN_LIB = os.path.join(HOSTSAN_DIR, "libabc_dtn_hostsan.so")
ASAN_RUNTIME = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


def _compile(src: str, sanitize: bool = False) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(HOSTSAN_DIR if sanitize else BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + (SANITIZE if sanitize else [])
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), res.stderr))
    return obj


def _link(objs, out, sanitize=False):
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC"] + DEVICE_FLAGS + (["-shared-libasan"] + SANITIZE if sanitize else []) + objs + [
        "-o", tmp, "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), res.stderr))
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, host_sanitized: bool = True) -> str:
    """Build libabc_dtn.so and, with host_sanitized, the host-sanitizer
    library HOSTSAN_LIB from the same sources (both compile together)."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(HOSTSAN_DIR, exist_ok=True)
    jobs = [(src, False) for src in SOURCES] + ([(src, True) for src in SOURCES] if host_sanitized else [])
    # the longest compiles first
    jobs.sort(key=lambda j: j[0] != "fused.hip")
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = dict(zip(jobs, ex.map(lambda j: _compile(*j), jobs)))
    _link([objs[(src, False)] for src in SOURCES], LIB)
    if verbose:
        print("built", LIB)
    if host_sanitized:
        _link([objs[(src, True)] for src in SOURCES], HOSTSAN_LIB, sanitize=True)
        if verbose:
            print("built", HOSTSAN_LIB)
    return LIB


def build_host_sanitized() -> str:
    """Build only the host-sanitizer library."""
    os.makedirs(HOSTSAN_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(lambda s: _compile(s, True), SOURCES))
    return _link(objs, HOSTSAN_LIB, sanitize=True)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
