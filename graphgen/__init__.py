"""Seeded synthetic graph inputs shared by the oracle, the tests and the benchmark.

This package makes inputs only: Kronecker (R-MAT) edge lists with the Graph500
initiator of the paper's Section 6.1, deterministic root samples, and small
structured graphs (paths, cycles, grids, ...) as edge lists. It contains none
of the traversal method's arithmetic (no CSR build, no degree classes, no BFS).

The R-MAT generator lives in ``kronecker.c`` (built into ``libgraphgen.so``);
see its header for the exact random-number definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

GRAPH500_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP). Returns the library path."""
    src = os.path.join(_HERE, "kronecker.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.gg_kronecker_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, p,
                                           ctypes.c_uint64, ctypes.c_int, p, p]
        lib.gg_kronecker_edges.restype = ctypes.c_int
        lib.gg_sample_roots.argtypes = [ctypes.c_int64, ctypes.c_int64, p, p, ctypes.c_uint64,
                                        ctypes.c_int64, p]
        lib.gg_sample_roots.restype = ctypes.c_int64
        lib.gg_scramble.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64]
        lib.gg_scramble.restype = ctypes.c_int64
        lib.gg_random_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_random_u64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def kronecker_edges(scale: int, edgefactor: int = 16, seed: int = 1, abcd=GRAPH500_ABCD,
                    permute: bool = True, out_src: np.ndarray | None = None,
                    out_dst: np.ndarray | None = None, first: int = 0, count: int | None = None):
    """Edges [first, first+count) of the seeded R-MAT stream as (src, dst) int32 arrays.

    The whole graph has 2**scale vertices and edgefactor * 2**scale edges.
    ``out_src``/``out_dst`` may be given (int32, contiguous, e.g. pinned host
    buffers) to avoid an extra copy.
    """
    lib = _load()
    m = edgefactor * (1 << scale) if count is None else count
    src = np.empty(m, np.int32) if out_src is None else out_src
    dst = np.empty(m, np.int32) if out_dst is None else out_dst
    assert src.dtype == np.int32 and dst.dtype == np.int32 and src.size >= m and dst.size >= m
    prob = (ctypes.c_double * 4)(*abcd)
    rc = lib.gg_kronecker_edges(scale, first, m, ctypes.cast(prob, ctypes.c_void_p).value,
                                seed, 1 if permute else 0, _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError("bad generator arguments")
    return src[:m], dst[:m]


def sample_roots(n: int, src: np.ndarray, dst: np.ndarray, k: int, seed: int = 2) -> np.ndarray:
    """k distinct seeded roots among vertices touching a non-self-loop edge."""
    lib = _load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    out = np.empty(k, np.int32)
    got = lib.gg_sample_roots(n, src.size, _ptr(src), _ptr(dst), seed, k, _ptr(out))
    if got < 0:
        raise MemoryError("gg_sample_roots failed")
    return out[:got]


def scramble(scale: int, seed: int, x: int) -> int:
    return int(_load().gg_scramble(scale, seed, x))


def random_u64(seed: int, stream: int, i: int) -> int:
    return int(_load().gg_random_u64(seed, stream, i))


# ---------------------------------------------------------------------------
# Small structured graphs as undirected edge lists (each edge listed once).
# ---------------------------------------------------------------------------

def _pack(pairs) -> tuple[np.ndarray, np.ndarray]:
    a = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return a[:, 0].astype(np.int32), a[:, 1].astype(np.int32)


def path(n: int):
    return _pack([(i, i + 1) for i in range(n - 1)])


def cycle(n: int):
    return _pack([(i, (i + 1) % n) for i in range(n)])


def star(n: int):
    """Centre 0 joined to 1..n-1."""
    return _pack([(0, i) for i in range(1, n)])


def complete(n: int):
    return _pack([(i, j) for i in range(n) for j in range(i + 1, n)])


def complete_bipartite(a: int, b: int):
    return _pack([(i, a + j) for i in range(a) for j in range(b)])


def grid(rows: int, cols: int):
    e = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                e.append((v, v + 1))
            if r + 1 < rows:
                e.append((v, v + cols))
    return _pack(e)


def hypercube(d: int):
    n = 1 << d
    return _pack([(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < (v ^ (1 << b))])


def binary_tree(n: int):
    """Heap-ordered complete binary tree on n vertices."""
    return _pack([((i - 1) // 2, i) for i in range(1, n)])


def relabel(src: np.ndarray, dst: np.ndarray, perm: np.ndarray):
    """Apply vertex relabelling perm (old id -> new id) to an edge list."""
    return perm[src].astype(np.int32), perm[dst].astype(np.int32)


def random_gnp(n: int, p: float, seed: int, loops: bool = True, dup: bool = True):
    """Erdos-Renyi G(n, p) edge list, optionally with self-loops and repeated edges."""
    rng = np.random.default_rng(seed)
    e = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    if loops:
        e += [(i, i) for i in range(n) if rng.random() < p]
    if dup and e:
        picks = rng.integers(0, len(e), size=max(1, len(e) // 4))
        e += [(e[k][1], e[k][0]) for k in picks]
    if not e:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    return _pack(e)
