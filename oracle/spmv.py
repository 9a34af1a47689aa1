"""Loader of the oracle's multi-threaded CSR product (oracle/spmv.cpp) --
test infrastructure only: the benchmark's CPU baseline times it on all host
cores.  build() compiles the shared library with g++; csr_apply() calls it."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spmv.cpp")
LIB = os.path.join(HERE, "libspmv.so")
_lib = None


def build() -> str:
    """Compile oracle/libspmv.so (always recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.run(["g++", "-O3", "-march=x86-64-v2", "-shared", "-fPIC",
                    "-std=c++17", "-pthread", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: run __graft_entry__.build()")
        lib = C.CDLL(LIB)
        lib.oracle_csr_spmv.restype = C.c_int
        lib.oracle_csr_spmv.argtypes = [C.c_int64, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int]
        _lib = lib
    return _lib


def host_threads() -> int:
    """Worker threads for the CPU baseline: the CPUs this process may run
    on, capped by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class CSR:
    """The oracle's matrix in the layout the C product takes."""

    def __init__(self, A):
        A = A.tocsr()
        self.n = A.shape[0]
        self.indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.data = np.ascontiguousarray(A.data, dtype=np.float64)

    def apply(self, x: np.ndarray, y: np.ndarray, threads: int) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert y.dtype == np.float64 and y.flags.c_contiguous and len(y) == self.n
        rc = _load().oracle_csr_spmv(self.n, self.indptr.ctypes.data,
                                     self.indices.ctypes.data, self.data.ctypes.data,
                                     x.ctypes.data, y.ctypes.data, int(threads))
        if rc != 0:
            raise ValueError("oracle_csr_spmv: invalid arguments")
        return y
