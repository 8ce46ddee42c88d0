"""CPU oracle for the BFS hot path: plain, slow, obviously correct.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU library
(``paper_2009_07463_amd``) never imports it and shares no code with it.

The arithmetic is in ``oracle.c`` (plain C, single thread); this module only
marshals numpy arrays. What each function computes and which passage of the
paper it follows is stated in ``oracle.c``:

* ``build_csr``      -- undirected simple graph as CSR (Section 5.1.1).
* ``bfs``            -- FIFO-queue BFS: hop-distance levels, first-discoverer
                        parents (the result of Algorithms 1 and 9).
* ``validate``       -- the spanning-tree rules of Section 5.3 (V1-V4).
* ``degree_counts``  -- degree-0 / degree-1 / other counts (Algorithm 8, MH=0).
* ``etvca``          -- Algorithm 8 for any MH.

Pins (tests that tie this oracle to something other than itself) are in
``tests/test_oracle_*.py``. Parent arrays are legitimately non-unique:
parent parity is "unpinned"; parents are checked by ``validate`` only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CORE_INTERNAL, CORE_EDGE, TREE_INTERNAL, TREE_LEAF, VERTEX_ZERO = range(5)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.oracle_csr_count.argtypes = [i64, i64, p, p, p]
        lib.oracle_csr_count.restype = i64
        lib.oracle_csr_fill.argtypes = [i64, i64, p, p, p, p]
        lib.oracle_csr_fill.restype = i64
        lib.oracle_bfs.argtypes = [i64, p, p, i32, p, p]
        lib.oracle_bfs.restype = i64
        lib.oracle_validate.argtypes = [i64, p, p, i32, p, p, p]
        lib.oracle_validate.restype = ctypes.c_int
        lib.oracle_degree_counts.argtypes = [i64, p, p]
        lib.oracle_degree_counts.restype = None
        lib.oracle_reached_degree_sum.argtypes = [i64, p, p]
        lib.oracle_reached_degree_sum.restype = i64
        lib.oracle_etvca.argtypes = [i64, p, p, ctypes.c_int, p]
        lib.oracle_etvca.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class CSR:
    """Undirected simple graph: int64 offsets, int32 sorted rows."""

    def __init__(self, off: np.ndarray, col: np.ndarray):
        self.off = off
        self.col = col

    @property
    def n(self) -> int:
        return self.off.size - 1

    @property
    def nnz(self) -> int:
        return int(self.off[-1])

    def degree(self) -> np.ndarray:
        return np.diff(self.off)


def build_csr(n: int, src, dst) -> CSR:
    lib = _load()
    src = _c(src, np.int32)
    dst = _c(dst, np.int32)
    off = np.zeros(n + 1, np.int64)
    total = lib.oracle_csr_count(n, src.size, src.ctypes.data, dst.ctypes.data, off.ctypes.data)
    if total < 0:
        raise ValueError("edge endpoint outside [0, n)")
    col = np.empty(max(total, 1), np.int32)
    e = lib.oracle_csr_fill(n, src.size, src.ctypes.data, dst.ctypes.data, off.ctypes.data,
                            col.ctypes.data)
    if e < 0:
        raise MemoryError("oracle_csr_fill failed")
    return CSR(off, col[:e])


def bfs(g: CSR, root: int):
    """(parent, level) int32 arrays of a FIFO BFS from root."""
    lib = _load()
    parent = np.empty(g.n, np.int32)
    level = np.empty(g.n, np.int32)
    col = g.col if g.col.size else np.zeros(1, np.int32)
    r = lib.oracle_bfs(g.n, g.off.ctypes.data, col.ctypes.data, int(root), parent.ctypes.data,
                       level.ctypes.data)
    if r < 0:
        raise ValueError("bad root %r" % root)
    return parent, level


def validate(g: CSR, root: int, parent, level):
    """(code, vertex): code 0 = valid, else the first failed rule V1..V4."""
    lib = _load()
    parent = _c(parent, np.int32)
    level = _c(level, np.int32)
    assert parent.size == g.n and level.size == g.n
    bad = ctypes.c_int64(-1)
    col = g.col if g.col.size else np.zeros(1, np.int32)
    code = lib.oracle_validate(g.n, g.off.ctypes.data, col.ctypes.data, int(root),
                               parent.ctypes.data, level.ctypes.data, ctypes.addressof(bad))
    return int(code), int(bad.value)


def degree_counts(g: CSR):
    """(n_deg0, n_deg1, n_deg_ge2)."""
    out = np.zeros(3, np.int64)
    _load().oracle_degree_counts(g.n, g.off.ctypes.data, out.ctypes.data)
    return int(out[0]), int(out[1]), int(out[2])


def reached_edges(g: CSR, level) -> int:
    """Traversed undirected edges: half the degree sum over reached vertices."""
    level = _c(level, np.int32)
    return int(_load().oracle_reached_degree_sum(g.n, g.off.ctypes.data, level.ctypes.data)) // 2


def etvca(g: CSR, height: int) -> np.ndarray:
    """Algorithm 8 vertex types (uint8, see the module constants)."""
    t = np.empty(g.n, np.uint8)
    col = g.col if g.col.size else np.zeros(1, np.int32)
    if _load().oracle_etvca(g.n, g.off.ctypes.data, col.ctypes.data, int(height), t.ctypes.data):
        raise MemoryError
    return t
