"""Build libhytet.so in-tree with hipcc for gfx950.

Every HIP source is compiled for the MI355X (gfx950) only, with packed FP32
instructions disabled (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
Objects go to ``paper_2308_01792_amd/_build/``; the shared library lands next
to this file so that a copy of the tree carries it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhytet.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["mesh.cpp", "abi.cpp", "kernels.hip", "band.hip", "walk.hip",
           "vcoef.hip", "p2.hip", "p2_host.cpp", "scratch.hip"]
ARCH = os.environ.get("HYTET_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
                 shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    return ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + _flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile all sources and link libhytet.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] \
        + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libhytet.so failed:\n{res.stderr}")
    os.replace(tmp, OUT)
    return OUT


# Host sources: their CPU code (mesh set-up, layouts, stencils, the C ABI's
# argument checks) is what the sanitized variant instruments.
HOST_SOURCES = ["mesh.cpp", "abi.cpp", "p2_host.cpp"]
SANITIZED = os.path.join(BUILD, "san", "libhytet_san.so")


def build_sanitized(verbose: bool = False) -> str:
    """libhytet with AddressSanitizer and UndefinedBehaviorSanitizer on its
    host code (device code is built as usual): the host sources are rebuilt
    instrumented and linked with the regular device objects, which build()
    must have produced.  Load it with clang's ASan runtime preloaded."""
    san_dir = os.path.dirname(SANITIZED)
    os.makedirs(san_dir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in _flags() if f != "-O3"] + ["-O1", "-g"] + san

    def one(src: str) -> str:
        obj = os.path.join(san_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"compiling {src} (sanitized) failed:\n{res.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(one, HOST_SOURCES))
    dev = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o")
           for s in SOURCES if s not in HOST_SOURCES]
    missing = [o for o in dev if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"device objects missing (run build() first): {missing}")
    tmp = SANITIZED + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] \
        + san + ["-shared-libsan"] + objs + dev + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking the sanitized library failed:\n{res.stderr}")
    os.replace(tmp, SANITIZED)
    return SANITIZED


def asan_runtime() -> str:
    """Path of clang's shared ASan runtime (to preload into a host process
    that loads the sanitized library)."""
    res = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    import glob
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not cands:
        raise RuntimeError("clang's ASan runtime not found")
    return cands[-1]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "--sanitized" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
