"""Large-graph leg of the oracle (test infrastructure only): the plain C
implementation in ``ckpm.c`` of the graph build (Sec. 2.1) and the stochastic
Chebyshev moments (Sec. 3.1) for graphs whose intermediate arrays do not fit
the numpy/scipy version (a billion undirected edges).  Same definitions as
:mod:`oracle.graph` and :mod:`oracle.kpm`, fp64 throughout; it is pinned
against exact moments and against the numpy oracle in the CPU tests.

The shared library is built with gcc next to the source (``build()``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckpm.c")
_LIB = os.path.join(_HERE, "libckpm.so")
_lib = None


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("old_id", ctypes.c_void_p)]


def build(force: bool = False) -> str:
    """Compile ckpm.c into libckpm.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        p, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        lib.ock_build_csr.argtypes = [i64, i64, p, p, ctypes.POINTER(_Graph)]
        lib.ock_build_csr.restype = ctypes.c_int
        lib.ock_free.argtypes = [ctypes.POINTER(_Graph)]
        lib.ock_free.restype = None
        lib.ock_moments.argtypes = [ctypes.POINTER(_Graph), i32, u64, p, i32, p, i64, p, p]
        lib.ock_moments.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class BigGraph:
    """Symmetric simple graph held by the C oracle (freed with the object)."""

    def __init__(self, n_nodes: int, src, dst):
        lib = _load()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape:
            raise ValueError("src/dst length mismatch")
        self._g = _Graph()
        rc = lib.ock_build_csr(int(n_nodes), int(src.size), _ptr(src), _ptr(dst), ctypes.byref(self._g))
        if rc != 0:
            raise (MemoryError if rc == -2 else ValueError)("ock_build_csr failed (%d)" % rc)

    def __del__(self):
        if getattr(self, "_g", None) is not None and _lib is not None:
            _lib.ock_free(ctypes.byref(self._g))
            self._g = None

    @property
    def n(self) -> int:
        return int(self._g.n)

    @property
    def nnz(self) -> int:
        return int(self._g.nnz)

    def _view(self, addr, count, dtype):
        buf = (ctypes.c_char * (count * np.dtype(dtype).itemsize)).from_address(addr)
        return np.frombuffer(buf, dtype=dtype, count=count)

    def row_ptr(self) -> np.ndarray:
        return self._view(self._g.row_ptr, self.n + 1, np.int64).copy()

    def old_id(self) -> np.ndarray:
        return self._view(self._g.old_id, self.n, np.int32).copy()

    def col_view(self) -> np.ndarray:
        """The column array itself (no copy; valid while the graph lives)."""
        return self._view(self._g.col, self.nnz, np.int32)

    def moments(self, k: int, M: int, seed: int = 0, rows=None, unit_nodes=None):
        """(mu_pp [k][M], ldos [len(rows)][M] or None): Rademacher probes from
        `seed`, or unit probes on `unit_nodes` (then k = len(unit_nodes))."""
        lib = _load()
        un = None
        if unit_nodes is not None:
            un = np.ascontiguousarray(unit_nodes, dtype=np.int64)
            k = int(un.size)
        mu_pp = np.zeros((k, M))
        r = np.ascontiguousarray(rows if rows is not None else np.zeros(0), dtype=np.int64)
        ld = np.zeros((r.size, M)) if r.size else None
        rc = lib.ock_moments(ctypes.byref(self._g), int(k), ctypes.c_uint64(seed & (2**64 - 1)), _ptr(un), int(M),
                             _ptr(mu_pp), int(r.size), _ptr(r) if r.size else None, _ptr(ld))
        if rc != 0:
            raise (MemoryError if rc == -2 else ValueError)("ock_moments failed (%d)" % rc)
        return mu_pp, ld
