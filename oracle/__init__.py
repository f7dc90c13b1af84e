"""CPU oracle for the Atos graph applications (BFS, PageRank, colouring).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU baseline are the only callers.  The product path (the HIP library and
its Python binding) never imports this package, and this package imports
nothing from the product.

The arithmetic lives in ``atos_oracle.c`` (plain C, FP64, sequential unless a
thread count is given); this module compiles it with gcc and marshals numpy
arrays.  Every graph argument is anything with ``n``, ``offsets`` (int64,
n+1) and ``cols`` (int32) attributes: an undirected CSR graph with both
directions of every edge stored.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "atos_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)


def build(src: str = _SRC, out: str = _LIB_PATH, native: bool = False) -> str:
    """Compile the oracle (or another copy of its source) into a shared
    library; by default oracle/_build/liboracle.so.  Always rebuilds.
    `native` adds -march=native: only for a build made and used on the same
    host (the CPU timing), since the default build travels to other hosts."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    arch = ["-march=native"] if native else []
    subprocess.run(["gcc", "-O3", *arch, "-std=c11", "-fopenmp", "-shared", "-fPIC",
                    "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


def _load(path: str | None = None):
    """Load the oracle library; `path` loads another build of the same source
    (the planted-mistake tests) in place of the default one."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    if path is None:
        path = os.environ.get("ATOS_ORACLE_LIB") or _LIB_PATH  # env: a planted-mistake build
        if not os.path.exists(path):
            build()
    lib = ctypes.CDLL(path)
    lib.oracle_bfs.restype = ctypes.c_int64
    lib.oracle_bfs.argtypes = [ctypes.c_int64, _I64P, _I32P, ctypes.c_int64, _I32P]
    lib.oracle_bfs_levelsync.restype = ctypes.c_int64
    lib.oracle_bfs_levelsync.argtypes = [ctypes.c_int64, _I64P, _I32P, ctypes.c_int64, ctypes.c_int,
                                         _I32P]
    lib.oracle_pagerank.restype = ctypes.c_int
    lib.oracle_pagerank.argtypes = [ctypes.c_int64, _I64P, _I32P, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, _F64P, _F64P,
                                    _F64P]
    lib.oracle_ppr.restype = ctypes.c_int
    lib.oracle_ppr.argtypes = [ctypes.c_int64, _I64P, _I32P, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _F64P, _F64P, _F64P]
    lib.oracle_pagerank_push_bsp.restype = ctypes.c_int
    lib.oracle_pagerank_push_bsp.argtypes = [ctypes.c_int64, _I64P, _I32P, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int, _F64P, _F64P, _I64P,
                                             _I64P]
    lib.oracle_greedy_color.restype = ctypes.c_int64
    lib.oracle_greedy_color.argtypes = [ctypes.c_int64, _I64P, _I32P, _I32P]
    lib.oracle_color_fifo.restype = ctypes.c_int64
    lib.oracle_color_fifo.argtypes = [ctypes.c_int64, _I64P, _I32P, ctypes.c_uint64, ctypes.c_int64,
                                      _I32P, _I64P]
    lib.oracle_color_rank_keys.restype = None
    lib.oracle_color_rank_keys.argtypes = [ctypes.c_int64, _I64P, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_uint32)]
    _lib = lib
    return lib


def _csr(g):
    offsets = np.ascontiguousarray(g.offsets, dtype=np.int64)
    cols = np.ascontiguousarray(g.cols, dtype=np.int32)
    n = int(g.n)
    if offsets.shape != (n + 1,) or cols.shape != (int(offsets[-1]),):
        raise ValueError("malformed CSR")
    return n, offsets, cols, offsets.ctypes.data_as(_I64P), cols.ctypes.data_as(_I32P)


def bfs(g, source: int) -> np.ndarray:
    """Minimum hop counts from ``source`` (int32, -1 = unreached)."""
    n, offsets, cols, po, pc = _csr(g)
    depth = np.empty(n, dtype=np.int32)
    r = _load().oracle_bfs(n, po, pc, int(source), depth.ctypes.data_as(_I32P))
    if r < 0:
        raise ValueError("oracle_bfs: bad argument")
    return depth


def bfs_levelsync(g, source: int, threads: int = 0) -> np.ndarray:
    """Level-synchronous BFS over ``threads`` OpenMP threads (CPU timing);
    the same depths as ``bfs``."""
    n, offsets, cols, po, pc = _csr(g)
    depth = np.empty(n, dtype=np.int32)
    r = _load().oracle_bfs_levelsync(n, po, pc, int(source), int(threads),
                                     depth.ctypes.data_as(_I32P))
    if r < 0:
        raise ValueError("oracle_bfs_levelsync: bad argument")
    return depth


def pagerank(g, damping: float = 0.85, tol: float = 1e-12, max_iter: int = 2000,
             threads: int = 0):
    """FP64 fixed point of x = (1-d) + d*A*D^-1*x.

    Returns (x, sweeps, last max|dx|, per-vertex error bound array)."""
    n, offsets, cols, po, pc = _csr(g)
    x = np.empty(n, dtype=np.float64)
    delta = ctypes.c_double()
    wdelta = ctypes.c_double()
    it = _load().oracle_pagerank(n, po, pc, float(damping), float(tol), int(max_iter),
                                 int(threads), x.ctypes.data_as(_F64P), ctypes.byref(delta),
                                 ctypes.byref(wdelta))
    if it < 0:
        raise ValueError("oracle_pagerank: bad argument")
    deg = np.maximum(np.diff(offsets), 1).astype(np.float64)
    bound = deg * damping / (1.0 - damping) * wdelta.value
    return x, it, delta.value, bound


def ppr(g, source: int, damping: float = 0.85, tol: float = 1e-15, max_iter: int = 5000,
        threads: int = 0):
    """FP64 fixed point of x = (1-d)*e_source + d*A*D^-1*x (personalized)."""
    n, offsets, cols, po, pc = _csr(g)
    x = np.empty(n, dtype=np.float64)
    delta = ctypes.c_double()
    wdelta = ctypes.c_double()
    it = _load().oracle_ppr(n, po, pc, int(source), float(damping), float(tol), int(max_iter),
                            int(threads), x.ctypes.data_as(_F64P), ctypes.byref(delta),
                            ctypes.byref(wdelta))
    if it < 0:
        raise ValueError("oracle_ppr: bad argument")
    deg = np.maximum(np.diff(offsets), 1).astype(np.float64)
    bound = deg * damping / (1.0 - damping) * wdelta.value
    return x, it, delta.value, bound


def pagerank_push_bsp(g, damping: float = 0.85, epsilon: float = 1e-7, max_rounds: int = 100000):
    """Sequential FP64 run of the bulk-synchronous push PageRank.

    Returns (rank, residue, rounds, edge_pushes, pops)."""
    n, offsets, cols, po, pc = _csr(g)
    rank = np.empty(n, dtype=np.float64)
    res = np.empty(n, dtype=np.float64)
    pushes = ctypes.c_int64()
    pops = ctypes.c_int64()
    rounds = _load().oracle_pagerank_push_bsp(n, po, pc, float(damping), float(epsilon),
                                              int(max_rounds), rank.ctypes.data_as(_F64P),
                                              res.ctypes.data_as(_F64P), ctypes.byref(pushes),
                                              ctypes.byref(pops))
    if rounds < 0:
        raise ValueError("oracle_pagerank_push_bsp: bad argument")
    return rank, res, rounds, pushes.value, pops.value


def greedy_color(g):
    """First-fit colouring in vertex-ID order; returns (colours int32, count)."""
    n, offsets, cols, po, pc = _csr(g)
    color = np.empty(n, dtype=np.int32)
    k = _load().oracle_greedy_color(n, po, pc, color.ctypes.data_as(_I32P))
    if k < 0:
        raise ValueError("oracle_greedy_color: bad argument")
    return color, int(k)


def color_rank_keys(g, seed: int) -> np.ndarray:
    """32-bit colouring rank keys (degree high, pseudo-random priority low)."""
    n, offsets, cols, po, pc = _csr(g)
    key = np.empty(n, dtype=np.uint32)
    _load().oracle_color_rank_keys(n, po, ctypes.c_uint64(seed),
                                   key.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return key


def color_fifo(g, seed: int, order_degree: int = 0):
    """Speculative colouring run by one worker, one task at a time, FIFO;
    vertices of degree >= order_degree (> 0) form the ordered class.

    Returns (colours int32, colour count, tasks processed)."""
    n, offsets, cols, po, pc = _csr(g)
    color = np.empty(n, dtype=np.int32)
    tasks = ctypes.c_int64()
    k = _load().oracle_color_fifo(n, po, pc, ctypes.c_uint64(seed), int(order_degree),
                                  color.ctypes.data_as(_I32P), ctypes.byref(tasks))
    if k < 0:
        raise ValueError("oracle_color_fifo: bad argument")
    return color, int(k), int(tasks.value)
