"""Seeded synthetic inputs shared by the CPU oracle and the GPU engine.

This package only *generates inputs* (graphs, edge weights, source vertices).
It holds none of the traversal or ranking arithmetic of either side.  The C
implementation lives in ``graphgen.c`` and is compiled with gcc into
``libgraphgen.so`` next to this file.

Graph recipe (the paper evaluates on undirected simple graphs, Sec. 6 and its
Table 1; R-MAT stands in for kron_g500-logn21 and the perturbed lattice for the
mesh-like rgg_n_24 / roadnet_CA):

* R-MAT scale s, edge factor ef, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05),
  no noise and no permutation, symmetrised, self loops and duplicates removed.
* Grid: side x side lattice, each lattice edge dropped with p = 0.03, plus
  0.1 % (of the lattice edge count) uniformly random long edges.
* Bipartite R-MAT (for the bipartite rankings): the same draws, edge (u, v)
  joining left vertex u to right vertex 2^scale + v.
* Weights: uniform integers in [1, maxw], a function of the unordered pair, so
  the weighted graph stays symmetric (the paper draws SSSP weights in 1..64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)
SEED_GRAPH, SEED_WEIGHTS, SEED_SOURCES, SEED_ARRIVALS = 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with gcc (OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        vp, i32, i64, u32, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [i32, i32, f64, f64, f64, u64]
        lib.gg_bipartite_rmat.restype = vp
        lib.gg_bipartite_rmat.argtypes = [i32, i32, f64, f64, f64, u64]
        lib.gg_grid.restype = vp
        lib.gg_grid.argtypes = [i32, f64, i64, u64]
        lib.gg_from_edges.restype = vp
        lib.gg_from_edges.argtypes = [i32, i64, vp, vp]
        lib.gg_graph_n.restype = i32
        lib.gg_graph_n.argtypes = [vp]
        lib.gg_graph_m.restype = i64
        lib.gg_graph_m.argtypes = [vp]
        lib.gg_graph_copy.restype = None
        lib.gg_graph_copy.argtypes = [vp, vp, vp]
        lib.gg_graph_free.restype = None
        lib.gg_graph_free.argtypes = [vp]
        lib.gg_weights.restype = None
        lib.gg_weights.argtypes = [i32, vp, vp, u32, u64, vp]
        lib.gg_sample_sources.restype = i64
        lib.gg_sample_sources.argtypes = [i32, vp, vp, i32, u64, vp]
        lib.gg_hash.restype = u64
        lib.gg_hash.argtypes = [u64, u64, u64]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _take(h):
    if not h:
        raise MemoryError("graphgen: generation failed (bad parameters or out of memory)")
    lib = _L()
    try:
        n = lib.gg_graph_n(h)
        m = lib.gg_graph_m(h)
        row = np.empty(n + 1, dtype=np.int32)
        col = np.empty(max(m, 0), dtype=np.int32)
        lib.gg_graph_copy(h, _ptr(row), _ptr(col) if m > 0 else _ptr(np.empty(1, np.int32)))
    finally:
        lib.gg_graph_free(h)
    return row, col


def rmat(scale: int, edge_factor: int = 16, abcd=RMAT_ABCD, seed: int = SEED_GRAPH):
    """R-MAT graph as symmetric simple CSR ``(row_offsets int32[n+1], col int32[m])``."""
    a, b, c, _d = abcd
    return _take(_L().gg_rmat(scale, edge_factor, a, b, c, seed))


def bipartite_rmat(scale: int, edge_factor: int = 16, abcd=RMAT_ABCD, seed: int = SEED_GRAPH):
    """Bipartite R-MAT: left vertices [0, 2^scale), right [2^scale, 2^(scale+1)); symmetric
    simple CSR whose every edge joins the two sides."""
    a, b, c, _d = abcd
    return _take(_L().gg_bipartite_rmat(scale, edge_factor, a, b, c, seed))


def grid(side: int = 4096, p_drop: float = 0.03, long_frac: float = 0.001,
         seed: int = SEED_GRAPH):
    """Perturbed lattice with random long edges, symmetric simple CSR."""
    n_long = int(round(long_frac * 2 * side * (side - 1)))
    return _take(_L().gg_grid(side, p_drop, n_long, seed))


def from_edges(n: int, eu, ev):
    """Symmetric simple CSR from an undirected edge list (drops loops and duplicates)."""
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    if eu.shape != ev.shape:
        raise ValueError("edge arrays differ in length")
    if eu.size == 0:
        return np.zeros(n + 1, np.int32), np.zeros(0, np.int32)
    return _take(_L().gg_from_edges(n, eu.size, _ptr(eu), _ptr(ev)))


def weights(row: np.ndarray, col: np.ndarray, maxw: int = 64, seed: int = SEED_WEIGHTS):
    """uint32 weights in [1, maxw], symmetric per unordered vertex pair."""
    n = row.size - 1
    w = np.empty(col.size, dtype=np.uint32)
    if col.size:
        _L().gg_weights(n, _ptr(row), _ptr(col), maxw, seed, _ptr(w))
    return w


def sample_sources(row: np.ndarray, col: np.ndarray, k: int, seed: int = SEED_SOURCES):
    """k distinct vertices drawn uniformly from the largest connected component."""
    n = row.size - 1
    out = np.empty(k, dtype=np.int32)
    size = _L().gg_sample_sources(n, _ptr(row), _ptr(col), k, seed, _ptr(out))
    if size < 0:
        raise ValueError("graphgen: fewer than %d vertices in the largest component" % k)
    return out


def hash3(seed: int, a: int, b: int) -> int:
    return int(_L().gg_hash(seed, a, b))


def csr_digest(row: np.ndarray, col: np.ndarray, w: np.ndarray | None = None) -> str:
    """SHA-256 of the CSR arrays (recorded in bench output)."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(row).tobytes())
    h.update(np.ascontiguousarray(col).tobytes())
    if w is not None:
        h.update(np.ascontiguousarray(w).tobytes())
    return h.hexdigest()
