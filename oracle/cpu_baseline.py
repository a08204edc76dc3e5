"""CPU baseline of the benchmark (the all-cores leg) -- TEST INFRASTRUCTURE.

ctypes wrapper of ``cpu_rows_omp.c``: the numeric phase of stiffness + mass
on every host core (OpenMP over the rows), given the oracle's pattern.  Only
bench.py's cpu_baseline leg uses it; it shares no code with the GPU library
and is not the oracle (whose numeric phase is the per-triangle loop of
fem_oracle.c).  ``build()`` compiles it with ``gcc -O2 -fopenmp
-ffp-contract=off``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_rows_omp.c")
LIB = os.path.join(HERE, "libcpu_rows_omp.so")

_lib = None
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build() -> str:
    tmp = LIB + ".tmp"
    from . import sanitize_flags
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c99", "-Wall", "-fPIC",
                    *sanitize_flags(), "-shared", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = C.CDLL(LIB)
    lib.cpu_rows_threads.restype = C.c_int
    lib.cpu_rows_threads.argtypes = []
    lib.cpu_rows_stiff_mass.restype = None
    lib.cpu_rows_stiff_mass.argtypes = [C.c_int32, _f64p, _i32p, _i32p, _i32p, _i32p, _i32p,
                                        _f64p, _f64p]
    _lib = lib
    return lib


def threads() -> int:
    return int(_load().cpu_rows_threads())


def stiff_mass_rows(q, me, P, S, M):
    """S, M [nnz] (overwritten) on the oracle pattern P, every host core."""
    _load().cpu_rows_stiff_mass(P.nq, np.ascontiguousarray(q, np.float64).reshape(-1),
                                np.ascontiguousarray(me, np.int32).reshape(-1), P.row_ptr,
                                P.col_idx, P.inc_ptr, P.inc, S, M)
