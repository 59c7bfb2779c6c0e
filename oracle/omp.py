"""ctypes wrapper of the OpenMP C reference (oracle/cpaa_omp.c).  TEST INFRASTRUCTURE ONLY.

The same FP64 CPAA (Alg. 1, eq. 3.1) and power method (eq. 2.1) as
``oracle.cpaa`` and ``oracle.pagerank_power``, in plain C over all host cores:
the benchmark's multi-core CPU baseline.  Pinned against the numpy oracle in
tests/test_oracle_omp.py.  ``build()`` compiles it with gcc -fopenmp next to
the source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpaa_omp.c")
LIB_PATH = os.path.join(HERE, "libcpaa_ref_omp.so")
_lib = None


def build() -> str:
    tmp = f"{LIB_PATH}.{os.getpid()}.tmp"   # concurrent builds (test workers) do not collide
    subprocess.run(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                    SRC, "-o", tmp, "-lm"], check=True, capture_output=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run oracle.omp.build())")
        L = ctypes.CDLL(LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        L.cpaa_ref_cpaa.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_double, f64p,
                                    ctypes.c_int, f64p, ctypes.c_int]
        L.cpaa_ref_cpaa.restype = ctypes.c_int
        L.cpaa_ref_power.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_double, f64p,
                                     ctypes.c_double, ctypes.c_int, f64p, ctypes.c_int]
        L.cpaa_ref_power.restype = ctypes.c_int
        _lib = L
    return _lib


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    return rp, ci, rp.ctypes.data_as(i32p), ci.ctypes.data_as(i32p)


def cpaa(g, b: np.ndarray, c: float, M: int, threads: int = 0) -> np.ndarray:
    """x_M of eq. 3.1 applied to b (one vector), FP64, on `threads` threads."""
    rp, ci, prp, pci = _csr(g)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(g.n)
    f64p = ctypes.POINTER(ctypes.c_double)
    st = lib().cpaa_ref_cpaa(g.n, prp, pci, c, bb.ctypes.data_as(f64p), M,
                             x.ctypes.data_as(f64p), threads)
    if st != 0:
        raise ValueError("cpaa_ref_cpaa: bad argument")
    return x


def power(g, p: np.ndarray, c: float, tol: float, max_iter: int = 100000,
          threads: int = 0) -> tuple[np.ndarray, int]:
    """The power method from (1-c)p; returns (x, steps)."""
    rp, ci, prp, pci = _csr(g)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    x = np.empty(g.n)
    f64p = ctypes.POINTER(ctypes.c_double)
    it = lib().cpaa_ref_power(g.n, prp, pci, c, pp.ctypes.data_as(f64p), tol, max_iter,
                              x.ctypes.data_as(f64p), threads)
    if it < 0:
        raise ValueError("cpaa_ref_power: bad argument")
    return x, it
